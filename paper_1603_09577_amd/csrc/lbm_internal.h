// Internal types shared by the host API and the kernel translation units of
// liblbm.so.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kBlock = 256;     // threads per workgroup (4 wave64)
constexpr int kMaxP = 9;        // coefficients of B, D, K, R polynomials
constexpr int kMaxC = 16;       // coefficients of the C-bar polynomials
constexpr int kNumXcd = 8;      // accelerator complex dies on MI355X
constexpr int kRedParts = 1024; // most workgroups of the phi reductions (one partial row each)

// n / d for n < 2^31 via one high multiply (Granlund-Montgomery).
struct FastDiv {
    uint32_t d, m, s;
    void set(uint32_t div) {
        d = div;
        if (div <= 1) { m = 0; s = 0; return; }
        uint32_t sh = 0;
        while ((1ull << sh) < div) ++sh;
        s = sh;
        m = (uint32_t)(((1ull << (31 + sh)) / div) + 1);
    }
    __device__ __forceinline__ uint32_t div(uint32_t n) const {
        return d == 1 ? n : (__umulhi(n, m) >> (s - 1));
    }
};

// Grid geometry of one instance.
struct Geom {
    uint32_t nx, ny, nz, N;
    uint64_t plane;       // elements between consecutive direction planes
    FastDiv fx, fxy;      // division by nx and by nx*ny
    uint32_t nblocks;     // 256-node blocks of one sweep
    uint32_t chunk;       // consecutive blocks swept by one workgroup (>= 1)
    int remap;            // XCD-aware block order
};

// Per-instance model constants in the compute type.  Symmetric tensors use
// the order (xx, yy, zz, xy, yz, xz).
template <typename TC>
struct Coefs {
    TC b[3][kMaxP];       // B_a(phi)
    TC bp[3][kMaxP];      // B'_a(phi)
    TC cb[6][kMaxC];      // C-bar = C + d cs^2 D  (Eq. 16 notation)
    TC cbd[6][kMaxC];     // C-bar'(phi)
    TC bpp[3][kMaxP];     // B''(phi)
    TC g0[6];             // 3 K0 / d : A^-1 = g0 k(phi) + I/2   (Eq. 26)
    TC kp[kMaxP];         // k(phi)
    TC kdp[kMaxP];        // k'(phi)
    TC a[6];              // A when k is constant
    TC r[kMaxP];          // R(phi)
    TC rp[kMaxP];         // R'(phi)
    TC ew[2][19];         // anti-bounce-back wall terms 2 (e+_k(phi_w) - w_k phi_ref)
    TC ewp[2][19];        // 2 e+_k(phi_w): the wall terms without the offset
    TC s[19];             // diagonal rates in moment order
    TC phi_ref;
    TC srate;             // common non-flux rate (equal-rate path)
    TC k0scale;           // 3 / d = dG / d(K0 k)
    int nb, ncb, nk, nr;  // used coefficient counts
    // rational flux B_a = (sum b[a] phi^p) / Q(phi) (Remark III only): Q and Q',
    // nq = 0 for a polynomial B
    TC bq[kMaxP];
    TC bqp[kMaxP];
    int nq;
};

struct Dims {
    int q;
    int prec;             // 0 f64, 1 f32, 2 f16
    bool eqr;             // equal non-flux rates: velocity-space collision
    bool src;             // R != 0 (Scheme-A history needed)
    bool kvar;            // k(phi) not constant: A per node
    bool wall;            // walls on the last axis
    bool lowdeg;          // every polynomial of degree <= 3 (C-bar <= 5)
    bool deg3 = false;    // every polynomial of degree <= 2 (C-bar <= 3): 3-term kernels (D2Q9)
    bool o32 = false;     // every indexed array spans < 4 GiB: 32-bit byte offsets (the 3-term and two-step kernels)
    bool nt;              // non-temporal distribution accesses
    bool sb;              // Scheme B (Eq. 33-35): stored fbar, explicit source
    bool rat = false;     // rational B (Remark III): the 9-term kernels evaluate P / Q
};

// Elements between consecutive direction planes.  A plane stride that is a
// multiple of the L2 set span (4 MB, 16 ways, 128-byte lines: 256 KiB) puts
// the same offset of every plane in one cache set and on one memory channel;
// the default pad shifts consecutive planes by about span / q bytes (an odd
// multiple of 256 bytes), which spreads the q concurrent streams.
inline uint64_t plane_stride(uint64_t n, int q, size_t elem, int pad_req) {
    const uint64_t align = 256 / elem;                      // keep planes 256-byte aligned
    uint64_t base = (n + align - 1) / align * align;
    if (pad_req < 0) return base;
    if (pad_req > 0) return base + ((uint64_t)pad_req + align - 1) / align * align;
    const uint64_t span = 256 * 1024;
    uint64_t want = span / (uint64_t)q / 256;               // shift per plane, in 256-byte units
    if ((want & 1) == 0) ++want;
    const uint64_t cur = (base * elem) % span;
    const uint64_t target = want * 256;
    const uint64_t pad_bytes = (target + span - cur) % span;
    return base + pad_bytes / elem;
}

// Kernel launchers, one set per lattice (sweep_d2q9.hip, sweep_d3q19.hip).
#define LBM_LAUNCHERS(SFX)                                                                              \
    hipError_t launch_sweep_##SFX(const Dims &dm, const Geom &g, const void *coefs, const void *fin,   \
                                  void *fout, void *p, int *flag, hipStream_t st);                      \
    hipError_t launch_sweep_gen_##SFX(const Dims &dm, const Geom &g, const void *coefs, const void *fin, \
                                      void *fout, void *p, int *flag, const double *kfield,             \
                                      const double *rfield, bool remark3, hipStream_t st);              \
    hipError_t launch_init_##SFX(const Dims &dm, const Geom &g, const void *coefs, const double *phi0, \
                                 void *f, void *p, const double *rfield, hipStream_t st);               \
    hipError_t launch_phi_##SFX(const Dims &dm, const Geom &g, const void *coefs, const void *f,       \
                                double *phi, const double *rfield, hipStream_t st);                     \
    hipError_t launch_phi_reduce_##SFX(const Dims &dm, const Geom &g, const void *coefs, const void *f,\
                                       const double *ref, const double *rfield, double *part,          \
                                       int nparts, double *out, hipStream_t st);                        \
    hipError_t launch_recenter_##SFX(const Dims &dm, const Geom &g, void *coefs, void *f, void *p,     \
                                     double *part, int nparts, double *shift, hipStream_t st);          \
    hipError_t launch_adjoint_##SFX(const Dims &dm, const Geom &g, const void *coefs, const void *f,   \
                                    const void *p, const void *psi_next, const double *pi_next,         \
                                    void *psi_out, double *pi_out, double *gk_part, hipStream_t st);    \
    hipError_t launch_adjoint_init_##SFX(const Dims &dm, const Geom &g, const void *coefs,             \
                                         const double *phi0, const void *psi0, const double *pi0,       \
                                         double *gphi0, hipStream_t st);                                \
    hipError_t launch_seed_##SFX(const Dims &dm, const Geom &g, const double *gphi, void *psi,         \
                                 double *pi, hipStream_t st);                                           \
    hipError_t launch_set_wall_##SFX(const Dims &dm, void *coefs, const double *ewp, hipStream_t st);
LBM_LAUNCHERS(q9)
LBM_LAUNCHERS(q19)
#undef LBM_LAUNCHERS

hipError_t launch_zero(double *p, uint32_t n, hipStream_t st);
// fold of per-workgroup reduction partials (lbm_reduce.hip)
hipError_t launch_reduce_final(const double *part, int nparts, double *out, hipStream_t st);

// Two time steps per pass, D2Q9 only (sweep_d2q9.hip), with tile shape `shape`.
hipError_t launch_sweep2_q9(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                            const void *pin, void *pout, int *flag, int shape, hipStream_t st);
// tile shape `shape` of two-step passes (rows, waves per workgroup); false past the last
bool two_step_shape_of(int prec, int shape, int *rows, int *waves);
// Two time steps per pass, D3Q19 (sweep_d3q19.hip): columns of 62 x rows nodes,
// chunks of zc planes; its tile shapes
hipError_t launch_sweep2_q19(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                             const void *pin, void *pout, int *flag, int shape, uint32_t zc, hipStream_t st);
// resident workgroups per CU of the D3Q19 two-step kernel this run would launch
hipError_t sweep2_q19_occupancy(const Dims &dm, const Geom &g, int shape, int *blocks_per_cu);
bool two_step3_shape_of(int prec, int shape, int *rows, int *waves);
// Two reversed sweeps per pass (sweep s, then s - 1), D2Q9 only, in tile
// shape `shape` (adjoint2_shape_of); and the resident workgroups per CU of
// that kernel.
hipError_t launch_adjoint2_q9(const Dims &dm, const Geom &g, const void *coefs, const void *f1, const void *p1,
                              const void *f0, const void *p0, const void *psi_next, const double *pi_next,
                              void *psi_out, double *pi_out, double *gk_part, int shape, hipStream_t st);
hipError_t adjoint2_q9_occupancy(const Dims &dm, const Geom &g, int shape, int *blocks_per_cu);
// rows and waves per workgroup of an adjoint tile shape; false past the last
bool adjoint2_shape_of(int shape, int *rows, int *waves);

// Generic FP64 reductions (lbm_reduce.hip).
hipError_t launch_reduce(const double *phi, const double *ref, uint32_t n, double *part,
                         int nparts, double *out, hipStream_t st);
hipError_t launch_copy16(const void *src, void *dst, size_t n16, int grid, hipStream_t st);
hipError_t launch_sum_partials(const double *part, int nparts, int width, double *acc,
                               hipStream_t st);

}  // namespace lbm
