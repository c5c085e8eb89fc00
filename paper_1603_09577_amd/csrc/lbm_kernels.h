// Device code of the fused MRT stream-collide sweep (pull form).
//
// State convention: a distribution buffer holds, at node x and direction k,
// the value that node x + c_k gathers at the next sweep (the post-collision
// population of the previous step).  One sweep gathers g_k(x) = f_k(x - c_k)
// (Eq. 2 left-hand side read backwards: streaming), computes phi = sum g
// (Eq. 10a), relaxes in moment space (Eq. 2, 17-19) or, when every non-flux
// rate is equal, with the equivalent velocity-space form, adds the Scheme-A
// source (Remark II), and stores the result at x.  Walls on the last axis use
// anti-bounce-back: a population that would come from beyond the wall is
// g_k(x) = -f_kbar(x) + 2 e+_k(phi_w), e+ the even part of Eq. 3.
//
// Stored values are offsets h_k = f_k - w_k phi_ref (phi_ref = 0 gives plain
// distributions); the equilibrium and the source are formed directly in
// offset form, so FP32/FP16 storage keeps the small differences.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_internal.h"
#include "lbm_lattice.h"
#include "lbm_reduce.h"   // before the contraction pragma below: the same rounding as lbm_reduce.hip

// Multiply-adds fuse only within one source expression (as the language
// allows), never across statements: the rounding of a node update is then
// the same in every kernel it is inlined into, which is what makes the
// one-sweep, two-sweep and batched kernels agree bit for bit.
#pragma clang fp contract(on)

namespace lbm {

template <typename TS>
struct HistType { using T = float; };
template <>
struct HistType<double> { using T = double; };

// Plain or non-temporal (streaming) accesses of the distribution planes.  The
// streaming form skips cache allocation: a gain when the state is far larger
// than the caches, a loss when it would stay resident in them.
template <typename TC, bool NT = false, typename TS>
__device__ __forceinline__ TC load_s(const TS *p) {
    if (NT) return (TC)__builtin_nontemporal_load(p);
    return (TC)(*p);
}

template <bool NT = false, typename TS, typename TC>
__device__ __forceinline__ void store_s(TS *p, TC v) {
    if (NT) __builtin_nontemporal_store((TS)v, p);
    else *p = (TS)v;
}

// Element idx of an array starting at `base`.  With O32 the host has checked
// that every array the kernel indexes spans less than 4 GiB, so the byte
// offset is formed in 32 bits: an access is then a scalar base plus one
// 32-bit vector offset, with no 64-bit address arithmetic per access.
template <bool O32, typename T>
__device__ __forceinline__ T *at(T *base, uint32_t idx) {
    if constexpr (O32) {
        using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
        return reinterpret_cast<T *>(reinterpret_cast<B *>(base) + idx * (uint32_t)sizeof(T));
    } else {
        return base + idx;
    }
}

// Stores of the q direction planes at one node, with 32-bit offsets (every
// array the kernel indexes spans less than 4 GiB).  The byte offset passes
// through an empty asm before each store, so each store sees its own opaque
// offset and takes the scalar-base form (plane base in scalar registers,
// offset in one vector register).  Without it the compiler forms one 64-bit
// vector address for the node and adds each plane's offset to it with a
// 64-bit vector instruction per store.
template <int Q, bool NT, typename TS, typename TC>
__device__ __forceinline__ void store_planes(TS *__restrict__ base, uint64_t plane, uint32_t n, const TC *out) {
    uint32_t off = n * (uint32_t)sizeof(TS);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        asm("" : "+v"(off));
        store_s<NT>(reinterpret_cast<TS *>(reinterpret_cast<char *>(base + (uint64_t)k * plane) + off), out[k]);
    }
}

// sum_{p < N} c[p] x^p by Horner over a compile-time length: no branches;
// the host picks the short length whenever every polynomial fits in it (the
// coefficients beyond a polynomial's degree are zero).
template <int N, typename T>
__device__ __forceinline__ T poly(const T *c, T x) {
    T acc = c[N - 1];
#pragma unroll
    for (int p = N - 2; p >= 0; --p) acc = acc * x + c[p];
    return acc;
}

// coefficient counts: NP for B, D, K, R and their derivatives, NC for C-bar
// (the host packs exact derivatives, so a derivative of an NP-term polynomial
// has NP - 1 terms)
template <int NP>
struct PolyLen {
    static constexpr int NC = 2 * NP - 2;                // C-bar
    static constexpr int ND = NP > 1 ? NP - 1 : 1;       // B', k', R'
    static constexpr int ND2 = NP > 2 ? NP - 2 : 1;      // B''
    static constexpr int NCD = NC > 1 ? NC - 1 : 1;      // C-bar'
};

// B_a(phi) of Eq. 1 and B'_a(phi).  A rational flux B_a = P_a / Q (Remark III,
// cf->nq > 0) is evaluated only by the 9-term kernels, which the host selects
// for it; the shorter kernels evaluate the polynomial P_a alone.  B' by the
// quotient rule, (P'_a - B_a Q') / Q.
template <int NP, typename TC>
__device__ __forceinline__ TC flux_b(const Coefs<TC> *__restrict__ cf, int a, TC phi) {
    const TC num = poly<NP>(cf->b[a], phi);
    if constexpr (NP == kMaxP) {
        if (cf->nq) return num / poly<NP>(cf->bq, phi);
    }
    return num;
}

template <int NP, typename TC>
__device__ __forceinline__ TC flux_bp(const Coefs<TC> *__restrict__ cf, int a, TC phi) {
    const TC dnum = poly<PolyLen<NP>::ND>(cf->bp[a], phi);
    if constexpr (NP == kMaxP) {
        if (cf->nq) {
            const TC q = poly<NP>(cf->bq, phi);
            const TC b = poly<NP>(cf->b[a], phi) / q;
            return (dnum - b * poly<PolyLen<NP>::ND>(cf->bqp, phi)) / q;
        }
    }
    return dnum;
}

// Workgroup order that gives each XCD one contiguous run of the domain, so
// the neighbouring rows and planes a workgroup reads sit in its own L2.
__device__ __forceinline__ uint32_t block_index(uint32_t b, uint32_t nb, int remap) {
    if (!remap) return b;
    const uint32_t q = nb / kNumXcd, r = nb % kNumXcd;
    const uint32_t xcd = b % kNumXcd, i = b / kNumXcd;
    return xcd * q + (xcd < r ? xcd : r) + i;
}

// 1/x: correctly rounded in FP64; the hardware reciprocal (1 ulp) in FP32,
// whose error is far below the FP32-storage error of the sweep.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Symmetric inverse of G (2x2 or 3x3), symmetric storage (xx, yy, zz, xy, yz, xz).
template <int DIM, typename T>
__device__ __forceinline__ void sym_inverse(const T *G, T *A) {
    if (DIM == 2) {
        const T det = G[0] * G[1] - G[3] * G[3];
        const T id = recip(det);
        A[0] = G[1] * id;
        A[1] = G[0] * id;
        A[3] = -G[3] * id;
        A[2] = T(0); A[4] = T(0); A[5] = T(0);
    } else {
        const T c00 = G[1] * G[2] - G[4] * G[4];
        const T c11 = G[0] * G[2] - G[5] * G[5];
        const T c22 = G[0] * G[1] - G[3] * G[3];
        const T c01 = G[5] * G[4] - G[3] * G[2];
        const T c12 = G[3] * G[5] - G[0] * G[4];
        const T c02 = G[3] * G[4] - G[5] * G[1];
        const T det = G[0] * c00 + G[3] * c01 + G[5] * c02;
        const T id = recip(det);
        A[0] = c00 * id; A[1] = c11 * id; A[2] = c22 * id;
        A[3] = c01 * id; A[4] = c12 * id; A[5] = c02 * id;
    }
}

// Flux block A at phi (Eq. 26): A = (g0 k(phi) + I/2)^-1, or the constant.
template <int DIM, bool KVAR, int NP, typename TC>
__device__ __forceinline__ void ablock(const Coefs<TC> *__restrict__ cf, TC phi, TC *A) {
    if (KVAR) {
        const TC kv = poly<NP>(cf->kp, phi);
        TC G[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) G[i] = cf->g0[i] * kv + (i < 3 ? TC(0.5) : TC(0));
        sym_inverse<DIM>(G, A);
    } else {
#pragma unroll
        for (int i = 0; i < 6; ++i) A[i] = cf->a[i];
    }
}

// A = (g0n k(phi) + I/2)^-1 (Eq. 26) with a per-node g0n = 3 K0(x) / d.
template <int DIM, int NP, typename TC>
__device__ __forceinline__ void ablock_field(const Coefs<TC> *__restrict__ cf, const TC *g0n, TC phi, TC *A) {
    const TC kv = poly<NP>(cf->kp, phi);
    TC G[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) G[i] = g0n[i] * kv + (i < 3 ? TC(0.5) : TC(0));
    sym_inverse<DIM>(G, A);
}

// Per-node 3 K0(x) / d from a field of K0 (2-D: xx, yy, xy; 3-D: xx, yy, zz,
// xy, yz, xz per node, FP64), in the symmetric order (xx, yy, zz, xy, yz, xz).
template <int DIM, typename TC>
__device__ __forceinline__ void g0_of_field(const Coefs<TC> *__restrict__ cf, const double *kfield, uint32_t n,
                                            TC *g0n) {
    constexpr int NK = DIM == 2 ? 3 : 6;
    const double *kf = kfield + (size_t)n * NK;
    const TC sc = cf->k0scale;
    if (DIM == 2) {
        g0n[0] = sc * (TC)kf[0]; g0n[1] = sc * (TC)kf[1]; g0n[3] = sc * (TC)kf[2];
        g0n[2] = g0n[4] = g0n[5] = TC(0);
    } else {
#pragma unroll
        for (int i = 0; i < 6; ++i) g0n[i] = sc * (TC)kf[i];
    }
}

// Equilibrium offsets feq_k - w_k phi_ref (Eq. 3 with c = 1, cs^2 = 1/3):
// w_k [ (phi - phi_ref) + 3 c.B + 9/2 ((Cbar - phi/3 I) : (c c - I/3)) ].
template <int Q, int NP, typename TC>
__device__ __forceinline__ void equilibrium(const Coefs<TC> *__restrict__ cf, TC phi, TC phio,
                                            TC *feq) {
    using L = Lattice<Q>;
    constexpr int D = L::dim;
    TC B[3], E[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) B[a] = (a < D) ? flux_b<NP>(cf, a, phi) : TC(0);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const bool used = (D == 3) || (i == 0 || i == 1 || i == 3);
        E[i] = used ? poly<PolyLen<NP>::NC>(cf->cb[i], phi) : TC(0);
    }
    const TC third = phi * TC(1.0 / 3.0);
    E[0] -= third; E[1] -= third;
    if (D == 3) E[2] -= third;
    const TC trE3 = (E[0] + E[1] + E[2]) * TC(1.0 / 3.0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int x = L::cx(k), y = L::cy(k), z = L::cz(k);
        TC cB = TC(0), ccE = -trE3;
        if (x) cB += x * B[0];
        if (y) cB += y * B[1];
        if (z) cB += z * B[2];
        if (x) ccE += E[0];
        if (y) ccE += E[1];
        if (z) ccE += E[2];
        if (x && y) ccE += TC(2 * x * y) * E[3];
        if (y && z) ccE += TC(2 * y * z) * E[4];
        if (x && z) ccE += TC(2 * x * z) * E[5];
        feq[k] = TC(L::w(k)) * (phio + TC(3) * cB + TC(4.5) * ccE);
    }
}

// Scheme-A source pieces at one time level: R(phi) and Btilde = (I - A/2) B'
// (Eq. 28 with gamma = 0).
template <int DIM, int NP, typename TC>
__device__ __forceinline__ void source_terms(const Coefs<TC> *__restrict__ cf, TC phi, const TC *A,
                                             TC *Bt, TC &R) {
    TC Bp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Bp[a] = (a < DIM) ? flux_bp<NP>(cf, a, phi) : TC(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        TC acc = Bp[a];
#pragma unroll
        for (int b = 0; b < DIM; ++b) acc -= TC(0.5) * A[sym(a, b)] * Bp[b];
        Bt[a] = (a < DIM) ? acc : TC(0);
    }
    R = poly<NP>(cf->r, phi);
}

struct NodeGeo {
    uint32_t n;
    int om[3], op[3];   // index offset of the neighbour at coord - 1 / coord + 1
    bool lo, hi;        // node next to the low / high wall of the last axis
};

template <int Q, bool WALL>
__device__ __forceinline__ NodeGeo node_geometry(const Geom &g, uint32_t n) {
    constexpr int D = Lattice<Q>::dim;
    NodeGeo ng;
    ng.n = n;
    uint32_t x, y, z = 0;
    if (D == 2) {
        y = g.fx.div(n);
        x = n - y * g.nx;
    } else {
        const uint32_t yz = g.fx.div(n);
        x = n - yz * g.nx;
        z = g.fxy.div(n);
        y = yz - z * g.ny;
    }
    const int nx = (int)g.nx, ny = (int)g.ny, nz = (int)g.nz;
    const int sy = nx, sz = nx * ny;
    ng.om[0] = (x == 0) ? (nx - 1) : -1;
    ng.op[0] = ((int)x == nx - 1) ? -(nx - 1) : 1;
    ng.om[1] = (y == 0) ? (ny - 1) * sy : -sy;
    ng.op[1] = ((int)y == ny - 1) ? -(ny - 1) * sy : sy;
    ng.om[2] = (z == 0) ? (nz - 1) * sz : -sz;
    ng.op[2] = ((int)z == nz - 1) ? -(nz - 1) * sz : sz;
    const uint32_t last = (D == 2) ? y : z;
    const uint32_t nlast = (D == 2) ? g.ny : g.nz;
    ng.lo = WALL && last == 0;
    ng.hi = WALL && last == nlast - 1;
    return ng;
}

// Gather g_k(x) (offset form) with periodic wrap and anti-bounce-back walls.
template <int Q, bool WALL, bool NT = false, bool O32 = false, typename TS, typename TC>
__device__ __forceinline__ void gather(const Geom &g, const Coefs<TC> *__restrict__ cf,
                                       const TS *__restrict__ fin, const NodeGeo &ng, TC *h) {
    using L = Lattice<Q>;
    constexpr int D = L::dim;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        int off = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int c = L::c(k, a);
            off += (c == 1) ? ng.om[a] : ((c == -1) ? ng.op[a] : 0);
        }
        const int cl = L::c(k, D - 1);
        if (WALL && ((cl == 1 && ng.lo) || (cl == -1 && ng.hi))) {
            h[k] = -load_s<TC, NT>(at<O32>(fin + (uint64_t)L::opp(k) * g.plane, ng.n)) + cf->ew[cl == 1 ? 0 : 1][k];
        } else {
            h[k] = load_s<TC, NT>(at<O32>(fin + (uint64_t)k * g.plane, (uint32_t)((int)ng.n + off)));
        }
    }
}

// ---------------------------------------------------------------------------
// the sweep
// ---------------------------------------------------------------------------
// Source offsets of a wave that lies within one grid row (2-D, nx a multiple
// of 64, so the 64 consecutive nodes of a wave share their row): the rows
// y - 1, y, y + 1 (periodic) are wave-uniform, their byte offsets scalar; the
// columns x - 1, x, x + 1 are byte offsets per lane.  The gathers below take
// a scalar row base plus one column offset per load, with no per-node
// division or neighbour selects.
struct RowWave {
    uint32_t n;          // this lane's node
    uint32_t rowb[3];    // byte offsets of rows y - 1, y, y + 1
    uint32_t colb[3];    // byte offsets of columns x - 1, x, x + 1
    bool lo, hi;         // the row next to the low / high wall
};

template <typename T, bool WALL>
__device__ __forceinline__ RowWave row_wave(const Geom &g, uint32_t n) {
    RowWave w;
    w.n = n;
    const uint32_t nw = __builtin_amdgcn_readfirstlane(n & ~63u);   // first node of the wave
    const uint32_t y = g.fx.div(nw), x = n - y * g.nx;
    const uint32_t nx = g.nx, ny = g.ny, rb = nx * (uint32_t)sizeof(T);
    w.rowb[0] = (y == 0 ? ny - 1 : y - 1) * rb;
    w.rowb[1] = y * rb;
    w.rowb[2] = (y == ny - 1 ? 0 : y + 1) * rb;
    w.colb[0] = (x == 0 ? nx - 1 : x - 1) * (uint32_t)sizeof(T);
    w.colb[1] = x * (uint32_t)sizeof(T);
    w.colb[2] = (x == nx - 1 ? 0 : x + 1) * (uint32_t)sizeof(T);
    w.lo = WALL && y == 0;
    w.hi = WALL && y == ny - 1;
    return w;
}

// Element at row offset rb and column offset c of plane base p; the column
// offset passes through an empty asm so that each load keeps the
// scalar-base form.
template <typename T>
__device__ __forceinline__ const T *row_elem(const T *p, uint32_t rb, uint32_t &c) {
    asm("" : "+v"(c));
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + rb + c);
}

// gather (pull: row y - c_y, column x - c_x) for a row wave, D2Q9.
template <bool WALL, bool NT, typename TS, typename TC>
__device__ __forceinline__ void gather_rw(const Geom &g, const Coefs<TC> *__restrict__ cf,
                                          const TS *__restrict__ fin, RowWave &w, TC *h) {
    using L = Lattice<9>;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = L::cx(k), cy = L::cy(k);
        if (WALL && ((cy == 1 && w.lo) || (cy == -1 && w.hi)))
            h[k] = -load_s<TC, NT>(at<true>(fin + (uint64_t)L::opp(k) * g.plane, w.n)) + cf->ew[cy == 1 ? 0 : 1][k];
        else
            h[k] = load_s<TC, NT>(row_elem(fin + (uint64_t)k * g.plane, w.rowb[1 - cy], w.colb[1 - cx]));
    }
}

// Scheme B, Eq. 35: phi = sum_k fbar_k + R(phi) / 2, for x = phi - phi_ref
// given x0 = sum_k fbar_k - phi_ref (the sum of the stored offsets) and the
// external source rext at the node.  R = r0 + r1 phi + r2 phi^2 + rext (the
// host admits degree <= 2 in Scheme B).  A source that does not depend on phi
// makes Eq. 35 explicit: x = x0 + R / 2.  Otherwise, expanded about phi_ref,
// Eq. 35 is the quadratic  a x^2 + b x + c = 0  with a = r2 / 2,
// b = R'(phi_ref) / 2 - 1, c = x0 + R(phi_ref) / 2, and the root that tends to
// x0 + R / 2 as R -> 0 is x = 2 c / (sqrt(b^2 - 4 a c) - b): with b close to
// -1 the denominator is close to 2, so no digits cancel.  Sets *R = R at that
// root and returns x0 + R / 2 (Eq. 35 itself, equal to the root up to
// rounding): the sweep then writes exactly the stored mass plus R, whereas the
// root's own rounding error, biased in FP32, would add to the mass every step.
template <typename T, typename TC>
__device__ __forceinline__ T phi_scheme_b(const Coefs<TC> *__restrict__ cf, T x0, T rext, T *R) {
    if (cf->nr <= 1) {
        *R = (T)cf->r[0] + rext;
        return x0 + T(0.5) * *R;
    }
    const T pr = (T)cf->phi_ref, r0 = (T)cf->r[0] + rext, r1 = (T)cf->r[1], r2 = (T)cf->r[2];
    const T a = T(0.5) * r2;
    const T b = T(0.5) * (r1 + T(2) * r2 * pr) - T(1);
    const T c = x0 + T(0.5) * (r0 + pr * (r1 + pr * r2));
    const T x = T(2) * c / (sqrt(b * b - T(4) * a * c) - b);
    const T phi = pr + x;
    *R = r0 + phi * (r1 + phi * r2);
    return x0 + T(0.5) * *R;
}

// The Scheme-A source terms of one time level at a node: R and Btilde of
// Eq. 28 (gamma = 0), from which Eq. 9 builds R_k.
template <typename TC>
struct SrcLevel {
    TC R;
    TC Bt[3];
};

// Hands this level's terms (R, Bt) to cur and takes the previous level's
// (Rp, Btp) from prev, or rebuilds them at phi(t - 1) = phi_ref + pp_off.
template <int D, bool KVAR, int NP, typename TC>
__device__ __forceinline__ void src_levels(const Coefs<TC> *__restrict__ cf, bool kfon, const TC *g0n, TC pp_off,
                                           TC R, const TC *Bt, SrcLevel<TC> *cur, const SrcLevel<TC> *prev,
                                           TC &Rp, TC *Btp) {
    if (cur) {
        cur->R = R;
#pragma unroll
        for (int a = 0; a < 3; ++a) cur->Bt[a] = Bt[a];
    }
    if (prev) {
        Rp = prev->R;
#pragma unroll
        for (int a = 0; a < 3; ++a) Btp[a] = prev->Bt[a];
        return;
    }
    TC Ap[6];
    const TC pp = cf->phi_ref + pp_off;
    if (kfon) ablock_field<D, NP>(cf, g0n, pp, Ap);
    else ablock<D, KVAR, NP>(cf, pp, Ap);
    source_terms<D, NP>(cf, pp, Ap, Btp, Rp);
}

// One node of the sweep (shared by the single-instance and batched kernels).
//
// SB: Scheme B (Eq. 33-35): the stored variable is fbar = f - R_k / 2, phi =
// sum fbar + R / 2 with R = R(phi) + an external field R(x, t) (Eq. 35,
// solved by phi_scheme_b), Btilde = B', and the source enters as
// M^-1 (I - S/2) M R_k (Eq. 34).  SRC
// then stays false (it is the Scheme-A source with its phi history).
// KF: K0 per node from `kfield` (A per node by Eq. 26).
// rem3 (uniform across a launch): Remark III, Eq. 36-38.  The equilibrium has
// C = 0 (the host leaves C out of C-bar) and the source
// G_k = w_k c_k . (I - A/2) dB/dt / cs^2 (Eq. 37) is added, with dB/dt the
// difference B(phi(t)) - B(phi(t - 1)) over the last step from the phi history.
// The per-node collision of one sweep on gathered populations h (offset
// form), with the phi history pp_off = phi(t - 1) - phi_ref: writes the
// post-collision populations to out and returns phio = phi - phi_ref, which
// the caller stores as the history when SRC or rem3 (see sweep_node).
// Scheme A only: cur (if given) receives this level's source terms; prev (if
// given) supplies the previous level's instead of rebuilding them from
// pp_off.  A caller that passes the terms of the same node one step later
// gets the values the rebuild would give (the same function of the same phi)
// without its arithmetic.
template <int Q, typename TC, bool EQR, bool SRC, bool KVAR, int NP, bool SB = false, bool KF = false>
__device__ __forceinline__ TC collide_node(const Coefs<TC> *__restrict__ cf, const TC *h, TC pp_off, uint32_t n,
                                           const double *kfield, const double *rfield, bool rem3, TC *out,
                                           SrcLevel<TC> *cur = nullptr, const SrcLevel<TC> *prev = nullptr) {
    using L = Lattice<Q>;
    constexpr int D = L::dim;
    TC g0n[6];
    const bool kfon = KF && kfield != nullptr;   // uniform across the launch
    if (kfon) g0_of_field<D>(cf, kfield, n, g0n);
    TC phio = TC(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) phio += h[k];
    // Scheme B: phi from Eq. 35 and R at this node and time
    TC Rx = TC(0);
    if (SB) phio = phi_scheme_b<TC>(cf, phio, rfield ? (TC)rfield[n] : TC(0), &Rx);
    const TC phi = cf->phi_ref + phio;

    TC A[6];
    if (kfon) ablock_field<D, NP>(cf, g0n, phi, A);
    else ablock<D, KVAR, NP>(cf, phi, A);

    // mass the source adds this step: Scheme A 3/2 R(t) - 1/2 R(t-1); Scheme B
    // R / 2 on top of phi - phi_ref (the stored sum is phi - R/2 before, phi + R/2 after)
    TC Se = TC(0);
    if (EQR) {
        // All non-flux rates equal s.  With orthogonal rows and the flux rows
        // equal to c_a, (M^-1 S M)(g - feq) = s (g - feq) + c_k . v with
        // v = (A - s I)(j - B) / |c_a|^2 (the density row drops out in Scheme A
        // since sum g = sum feq = phi).  Adding s feq_k and the Scheme-A source
        // and splitting every term into its part even and odd under
        // c_k -> -c_k gives
        //   out_k = (1 - s) g_k + w_k (s phio + Se + 9/2 s (E : c_k c_k - tr E / 3))
        //           + c_k . (w_k (3 s B + Vo) - v),
        // E = Cbar - phi/3 I, Se = 3/2 R(t) - 1/2 R(t-1) and
        // Vo = 3 (3/2 R(t) Btilde(t) - 1/2 R(t-1) Btilde(t-1)).  Opposite
        // directions share the even part and negate the odd one.
        const TC s = cf->srate;
        TC B[3], E[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) B[a] = (a < D) ? flux_b<NP>(cf, a, phi) : TC(0);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const bool used = (D == 3) || (i == 0 || i == 1 || i == 3);
            E[i] = used ? poly<PolyLen<NP>::NC>(cf->cb[i], phi) : TC(0);
        }
        const TC third = phi * TC(1.0 / 3.0);
        E[0] -= third; E[1] -= third;
        if (D == 3) E[2] -= third;
        const TC trE3 = (E[0] + E[1] + E[2]) * TC(1.0 / 3.0);
        TC Vo[3] = {TC(0), TC(0), TC(0)};
        TC jsh[3] = {TC(0), TC(0), TC(0)};   // Scheme B: R B' / 2, the part of j the shift removed
        if (SRC) {
            TC Bt[3], R, Btp[3], Rp;
            source_terms<D, NP>(cf, phi, A, Bt, R);
            src_levels<D, KVAR, NP>(cf, kfon, g0n, pp_off, R, Bt, cur, prev, Rp, Btp);
            Se = TC(1.5) * R - TC(0.5) * Rp;
#pragma unroll
            for (int a = 0; a < D; ++a) Vo[a] = TC(4.5) * R * Bt[a] - TC(1.5) * Rp * Btp[a];
        }
        if (SB) {
            // (1 - s/2) R_k = w_k (1 - s/2) R + c_k . 3 w_k (1 - s/2) R B'
            const TC hs = (TC(1) - TC(0.5) * s) * Rx;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const TC bp = flux_bp<NP>(cf, a, phi);
                Vo[a] = TC(3) * hs * bp;
                jsh[a] = TC(0.5) * Rx * bp;
            }
        }
        if (rem3) {
            // Remark III: c_k . 3 w_k (I - A/2) (B(phi) - B(phi(t - 1)))
            const TC pp = cf->phi_ref + pp_off;
            TC dB[3] = {TC(0), TC(0), TC(0)};
#pragma unroll
            for (int a = 0; a < D; ++a) dB[a] = flux_b<NP>(cf, a, phi) - flux_b<NP>(cf, a, pp);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                TC acc = dB[a];
#pragma unroll
                for (int b = 0; b < D; ++b) acc -= TC(0.5) * A[sym(a, b)] * dB[b];
                Vo[a] += TC(3) * acc;
            }
        }
        // j - B, with j the first moment of the gathered populations (Scheme B:
        // of f = fbar + R_k / 2, i.e. plus R B' / 2)
        TC jd[3], v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            TC acc = TC(0);
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const int c = L::c(k, a);
                if (c == 1) acc += h[k];
                else if (c == -1) acc -= h[k];
            }
            jd[a] = (a < D) ? acc + jsh[a] - B[a] : TC(0);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            TC acc = TC(0);
#pragma unroll
            for (int b = 0; b < D; ++b) acc += (A[sym(a, b)] - (a == b ? s : TC(0))) * jd[b];
            v[a] = acc * TC(1.0 / L::jnorm);
        }
        // even source part: Scheme A Se; Scheme B (1 - s/2) R.  Mass target
        // below: Scheme A phio + Se; Scheme B phio + R/2 (sum of the gathered
        // fbar is phio - R/2, the collision returns phio + R/2).
        const TC base = s * phio + (SB ? (TC(1) - TC(0.5) * s) * Rx : Se);
        if (SB) Se = TC(0.5) * Rx;
        const TC s45 = TC(4.5) * s;
        const TC oms = TC(1) - s;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const int kb = L::opp(k);
            if (kb < k) continue;
            const int x = L::cx(k), y = L::cy(k), z = L::cz(k);
            TC ccE = -trE3;
            if (x) ccE += E[0];
            if (y) ccE += E[1];
            if (z) ccE += E[2];
            if (x && y) ccE += TC(2 * x * y) * E[3];
            if (y && z) ccE += TC(2 * y * z) * E[4];
            if (x && z) ccE += TC(2 * x * z) * E[5];
            const TC w = TC(L::w(k));
            const TC even = w * (base + s45 * ccE);
            if (kb == k) {
                out[k] = oms * h[k] + even;
                continue;
            }
            TC odd = TC(0);
            if (x) odd += TC(x) * (w * (TC(3) * s * B[0] + Vo[0]) - v[0]);
            if (y) odd += TC(y) * (w * (TC(3) * s * B[1] + Vo[1]) - v[1]);
            if (z) odd += TC(z) * (w * (TC(3) * s * B[2] + Vo[2]) - v[2]);
            out[k] = oms * h[k] + even + odd;
            out[kb] = oms * h[kb] + even - odd;
        }
    } else {
        // m = M (g - feq); relax with S (diagonal rates, block A on the flux
        // rows, Eq. 17); back with M^-1 = M^T N^-1 (orthogonal rows).
        TC feq[Q];
        equilibrium<Q, NP>(cf, phi, phio, feq);
        TC dlt[Q], m[Q], r[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) dlt[k] = h[k] - feq[k];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            TC acc = TC(0);
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const int mm = L::M(i, k);
                if (mm == 1) acc += dlt[k];
                else if (mm == -1) acc -= dlt[k];
                else if (mm) acc += TC(mm) * dlt[k];
            }
            m[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) r[i] = cf->s[i] * m[i];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            TC acc = TC(0);
#pragma unroll
            for (int b = 0; b < D; ++b) acc += A[sym(a, b)] * m[L::jrow[b]];
            r[L::jrow[a]] = acc;
        }
        if (SB) {
            // r -= (I - S/2) M R_k, R_k = w_k R (1 + 3 c_k . B') (Eq. 9, Btilde = B')
            TC Bp[3] = {TC(0), TC(0), TC(0)};
#pragma unroll
            for (int a = 0; a < D; ++a) Bp[a] = flux_bp<NP>(cf, a, phi);
            TC Rk[Q], mR[Q], sR[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                TC cb = TC(0);
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    const int c = L::c(k, a);
                    if (c) cb += TC(c) * Bp[a];
                }
                Rk[k] = TC(L::w(k)) * Rx * (TC(1) + TC(3) * cb);
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                TC acc = TC(0);
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    const int mm = L::M(i, k);
                    if (mm == 1) acc += Rk[k];
                    else if (mm == -1) acc -= Rk[k];
                    else if (mm) acc += TC(mm) * Rk[k];
                }
                mR[i] = acc;
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) sR[i] = cf->s[i] * mR[i];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                TC acc = TC(0);
#pragma unroll
                for (int b = 0; b < D; ++b) acc += A[sym(a, b)] * mR[L::jrow[b]];
                sR[L::jrow[a]] = acc;
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) r[i] -= mR[i] - TC(0.5) * sR[i];
            Se = TC(0.5) * Rx;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) r[i] *= TC(1.0 / L::N(i));
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            TC acc = TC(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int mm = L::M(i, k);
                if (mm == 1) acc += r[i];
                else if (mm == -1) acc -= r[i];
                else if (mm) acc += TC(mm) * r[i];
            }
            out[k] = h[k] - acc;
        }
    }

    if (SRC && !EQR) {
        // Scheme A: + 3/2 R_k(t) - 1/2 R_k(t - 1), R_k = w_k (1 + 3 c.Btilde) R (Eq. 9)
        TC Bt[3], R, Btp[3], Rp;
        source_terms<D, NP>(cf, phi, A, Bt, R);
        src_levels<D, KVAR, NP>(cf, kfon, g0n, pp_off, R, Bt, cur, prev, Rp, Btp);
        const TC r1 = TC(1.5) * R, r0 = TC(0.5) * Rp;
        Se = r1 - r0;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            TC cb1 = TC(0), cb0 = TC(0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int c = L::c(k, a);
                if (c) { cb1 += TC(c) * Bt[a]; cb0 += TC(c) * Btp[a]; }
            }
            out[k] += TC(L::w(k)) * (r1 * (TC(1) + TC(3) * cb1) - r0 * (TC(1) + TC(3) * cb0));
        }
    }

    if (rem3 && !EQR) {
        // Remark III: + G_k = 3 w_k c_k . (I - A/2) (B(phi) - B(phi(t - 1)))
        const TC pp = cf->phi_ref + pp_off;
        TC dB[3] = {TC(0), TC(0), TC(0)}, gq[3] = {TC(0), TC(0), TC(0)};
#pragma unroll
        for (int a = 0; a < D; ++a) dB[a] = flux_b<NP>(cf, a, phi) - flux_b<NP>(cf, a, pp);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            TC acc = dB[a];
#pragma unroll
            for (int b = 0; b < D; ++b) acc -= TC(0.5) * A[sym(a, b)] * dB[b];
            gq[a] = TC(3) * acc;
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            TC cg = TC(0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int c = L::c(k, a);
                if (c) cg += TC(c) * gq[a];
            }
            out[k] += TC(L::w(k)) * cg;
        }
    }

    // Mass balance.  Collision conserves sum_k g_k and the Scheme-A source adds
    // exactly Se to it (Eq. 9 sums to R over k), so the rest population takes
    // the remainder.  The map is unchanged in exact arithmetic; in FP32 it
    // stops the drift that rounded weights (sum_k w_k = 1 + O(1e-8)) would
    // otherwise add to the mass at every step.
    {
        TC moving = TC(0);
#pragma unroll
        for (int k = 1; k < Q; ++k) moving += out[k];
        out[0] = (phio + Se) - moving;
    }

    return phio;
}

template <int Q, typename TS, typename TC, bool EQR, bool SRC, bool KVAR, bool WALL, int NP, bool NT = false,
          bool SB = false, bool KF = false, bool O32 = false, bool RW = false>
__device__ __forceinline__ void sweep_node(const Geom &g, const Coefs<TC> *__restrict__ cf,
                                           const TS *__restrict__ fin, TS *__restrict__ fout,
                                           typename HistType<TS>::T *p, int *flag, uint32_t n,
                                           const double *kfield = nullptr, const double *rfield = nullptr,
                                           bool rem3 = false) {
    TC h[Q];
    if constexpr (RW) {
        static_assert(Q == 9 && O32, "row waves: D2Q9 with 32-bit offsets");
        RowWave w = row_wave<TS, WALL>(g, n);
        gather_rw<WALL, NT>(g, cf, fin, w, h);
    } else {
        const NodeGeo ng = node_geometry<Q, WALL>(g, n);
        gather<Q, WALL, NT, O32>(g, cf, fin, ng, h);
    }
    // history read issued together with the gathers, so its latency overlaps theirs
    const TC pp_off = (SRC || rem3) ? (TC)*at<O32>(p, n) : TC(0);
    TC out[Q];
    const TC phio = collide_node<Q, TC, EQR, SRC, KVAR, NP, SB, KF>(cf, h, pp_off, n, kfield, rfield, rem3, out);
    if (SRC || rem3) *at<O32>(p, n) = (typename HistType<TS>::T)phio;

    if constexpr (O32) {
        store_planes<Q, NT>(fout, g.plane, n, out);
    } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) store_s<NT>(fout + (uint64_t)k * g.plane + n, out[k]);
    }

    if (!__builtin_isfinite(phio)) *flag = 1;
}

// RW: every wave lies within one grid row (D2Q9 with nx a multiple of 64;
// the host checks), and the gathers take the row-wave form.
// SB: Scheme B with R(phi) and no fields (the fields take k_sweep_gen).
template <int Q, typename TS, typename TC, bool EQR, bool SRC, bool KVAR, bool WALL, int NP, bool NT, bool O32 = false,
          bool RW = false, bool SB = false>
__global__ void __launch_bounds__(kBlock)
k_sweep(const Geom g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ fin,
        TS *__restrict__ fout, typename HistType<TS>::T *p, int *flag) {
    // each workgroup sweeps `chunk` consecutive blocks; with the XCD-aware
    // order every XCD covers one contiguous slab of the domain
    const uint32_t first = block_index(blockIdx.x, gridDim.x, g.remap) * g.chunk;
    for (uint32_t i = 0; i < g.chunk; ++i) {
        const uint32_t n = (first + i) * kBlock + threadIdx.x;
        if (n >= g.N) return;
        sweep_node<Q, TS, TC, EQR, SRC, KVAR, WALL, NP, NT, SB, false, O32, RW>(g, cf, fin, fout, p, flag, n);
    }
}

// ---------------------------------------------------------------------------
// Two time steps per pass (D2Q9; periodic or walls on y, equal or unequal
// non-flux rates: the template parameters below).  A workgroup owns a tile of
// 62 x TH nodes.  Phase 1 runs step t on the tile
// plus a one-node halo (64 x (TH + 2) nodes) from the stored state, and keeps
// the post-collision populations and the new phi history in LDS, rounded to
// the storage and history types exactly as a store would round them.  Phase 2
// runs step t + 1 on the tile, gathering from LDS, and stores only its result.
// Every node update is the single-sweep arithmetic on the same inputs, so the
// result equals two single sweeps bit for bit; the state is read and written
// once per two steps.  The phi history is read at halo nodes, which another
// tile may already have advanced, so it is read from `pin` and written to
// `pout` (two history buffers, alternating).  NW waves per workgroup share
// the TH + 2 rows of phase 1 (more waves: fewer rows and registers per wave).
// ---------------------------------------------------------------------------
// Periodic image of a tile coordinate v >= -1 on an axis of n >= 1 nodes
// (v exceeds n by at most the tile span, so the loop runs a bounded number of
// times; once at most when n is at least the tile span).
__device__ __forceinline__ int wrap_coord(int v, int n) {
    if (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// One tile of a two-step pass (tile (tx, ty) of 62 x TH nodes of the grid g;
// NW waves of the workgroup).  Grids narrower or lower than a tile are fine:
// halo lanes and rows then repeat nodes (computed identically) and only the
// tile's own nodes inside the grid are stored.  SB: Scheme B with R(phi) (no
// history; phi from Eq. 35 at every node of both phases).  WALL:
// anti-bounce-back walls at both ends of y (x periodic).  Rows beyond a wall
// are not computed; a population that comes from beyond the wall is the
// node's own post-collision opposite, negated, plus the wall term, read from
// the state in phase 1 and from LDS in phase 2 (the one-sweep gather's form).
// EQ: the equal-rate collision; otherwise the moment-space one (unequal
// non-flux rates, Eq. 2 with S of Eq. 17).
template <typename TS, typename TC, bool SRC, bool KVAR, int NP, int TH, int NW, bool SB = false, bool WALL = false,
          bool EQ = true>
__device__ __forceinline__ void sweep2_tile(const Geom &g, const Coefs<TC> *__restrict__ cf,
                                            const TS *__restrict__ fin, TS *__restrict__ fout,
                                            const typename HistType<TS>::T *__restrict__ pin,
                                            typename HistType<TS>::T *__restrict__ pout, uint32_t tx, uint32_t ty,
                                            int *flag) {
    using L = Lattice<9>;
    using TP = typename HistType<TS>::T;
    constexpr int TX = 64, TR = TH + 2, NR = TR / NW;
    static_assert(TR % NW == 0, "tile rows must split evenly over the waves");
    // Scheme A: phase 2 takes each node's previous-level source terms from
    // the registers of the wave that formed them in phase 1 (the same node,
    // one step earlier) instead of rebuilding them from the phi history; the
    // history type equals the compute type, so the rebuild would see the same
    // phi and give the same values
    constexpr bool HAND = SRC && !SB && std::is_same<TP, TC>::value;
    __shared__ TS lf[9][TR][TX];
    __shared__ TP lp[HAND ? 1 : TR][TX];
    SrcLevel<TC> lev[HAND ? NR : 1];
    const int x0 = (int)(tx * (TX - 2)), y0 = (int)(ty * TH);
    const int lane = threadIdx.x & 63;
    // the wave index is the same in every lane; taken into a scalar register,
    // it makes the row arithmetic of both phases scalar
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nx = (int)g.nx, ny = (int)g.ny;
    bool bad = false;
    // phase 1: the tile and its halo, coordinates x0 - 1 + lane and y0 - 1 + r.
    // A population with velocity c comes from column x - c_x of row y - c_y
    // (periodic).  The three source columns are byte offsets fixed per lane;
    // the source rows are wave-uniform, so every load is a scalar row base
    // plus one of the three offsets (each passed through an empty asm so that
    // the load keeps that form instead of a 64-bit vector address per load).
    const int xg = wrap_coord(x0 - 1 + lane, nx);
    uint32_t cb[3] = {(uint32_t)(xg == 0 ? nx - 1 : xg - 1) * (uint32_t)sizeof(TS),   // c_x = 1
                      (uint32_t)xg * (uint32_t)sizeof(TS),                              // c_x = 0
                      (uint32_t)(xg == nx - 1 ? 0 : xg + 1) * (uint32_t)sizeof(TS)};   // c_x = -1
    const uint32_t row_bytes = g.nx * (uint32_t)sizeof(TS);
    if constexpr (sizeof(TS) == 8) {
        // FP64: all of a wave's phase-1 loads are issued before its first
        // collision, so the latency of its later rows overlaps the arithmetic
        // of the first (measured +1% with 6 x 8 tiles, +8% with 6 x 4; the
        // FP32 shapes gained nothing that way)
        TS hs[NR][9];
        TS ps[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int yl = y0 - 1 + wv + i * NW;
            if (WALL && (yl < 0 || yl >= ny)) continue;   // beyond a wall
            const int yg = WALL ? yl : wrap_coord(yl, ny);
            const int ym = yg == 0 ? ny - 1 : yg - 1, yp = yg == ny - 1 ? 0 : yg + 1;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int cy = L::cy(k);
                const bool wl = WALL && ((cy == 1 && yg == 0) || (cy == -1 && yg == ny - 1));
                const uint32_t row = (uint32_t)(wl ? yg : (cy == 1 ? ym : (cy == -1 ? yp : yg)));
                const char *rb = reinterpret_cast<const char *>(fin + (uint64_t)(wl ? L::opp(k) : k) * g.plane) +
                                 row * row_bytes;
                uint32_t &c = cb[wl ? 1 : 1 - L::cx(k)];
                asm("" : "+v"(c));
                hs[i][k] = *reinterpret_cast<const TS *>(rb + c);
            }
            ps[i] = SRC ? *at<true>(pin, (uint32_t)yg * g.nx + (uint32_t)xg) : TS(0);
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int r = wv + i * NW;
            const int yl = y0 - 1 + r;
            if (WALL && (yl < 0 || yl >= ny)) continue;
            TC h[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int cy = L::cy(k);
                const bool wl = WALL && ((cy == 1 && yl == 0) || (cy == -1 && yl == ny - 1));
                h[k] = wl ? -(TC)hs[i][k] + cf->ew[cy == 1 ? 0 : 1][k] : (TC)hs[i][k];
            }
            TC out[9];
            const TC phio = collide_node<9, TC, EQ, SRC, KVAR, NP, SB>(cf, h, ps[i], 0u, nullptr, nullptr, false, out,
                                                                        HAND ? &lev[HAND ? i : 0] : nullptr);
#pragma unroll
            for (int k = 0; k < 9; ++k) lf[k][r][lane] = (TS)out[k];
            if (!HAND) lp[HAND ? 0 : r][lane] = (TP)phio;
            bad |= !__builtin_isfinite(phio);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int r = wv + i * NW;
            const int yl = y0 - 1 + r;
            if (WALL && (yl < 0 || yl >= ny)) continue;   // beyond a wall
            const int yg = WALL ? yl : wrap_coord(yl, ny);
            const int ym = yg == 0 ? ny - 1 : yg - 1, yp = yg == ny - 1 ? 0 : yg + 1;
            const uint32_t n = (uint32_t)yg * g.nx + (uint32_t)xg;
            TC h[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int cy = L::cy(k);
                const bool wl = WALL && ((cy == 1 && yg == 0) || (cy == -1 && yg == ny - 1));
                const uint32_t row = (uint32_t)(wl ? yg : (cy == 1 ? ym : (cy == -1 ? yp : yg)));
                const char *rb = reinterpret_cast<const char *>(fin + (uint64_t)(wl ? L::opp(k) : k) * g.plane) +
                                 row * row_bytes;
                uint32_t &c = cb[wl ? 1 : 1 - L::cx(k)];
                asm("" : "+v"(c));
                const TC v = (TC)*reinterpret_cast<const TS *>(rb + c);
                h[k] = wl ? -v + cf->ew[cy == 1 ? 0 : 1][k] : v;
            }
            const TC pp_off = SRC ? (TC)*at<true>(pin, n) : TC(0);
            TC out[9];
            const TC phio = collide_node<9, TC, EQ, SRC, KVAR, NP, SB>(cf, h, pp_off, n, nullptr, nullptr, false, out,
                                                                        HAND ? &lev[HAND ? i : 0] : nullptr);
#pragma unroll
            for (int k = 0; k < 9; ++k) lf[k][r][lane] = (TS)out[k];
            if (!HAND) lp[HAND ? 0 : r][lane] = (TP)phio;
            bad |= !__builtin_isfinite(phio);
        }
    }
    __syncthreads();
    // phase 2: interior lanes 1..62, rows 1..TH (no rows beyond a wall)
    if (lane >= 1 && lane <= TX - 2) {
        const int x = x0 + lane - 1;
        auto row2 = [&](int r, const SrcLevel<TC> *prev) {
            const int y = y0 + r - 1;
            TC h[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int cy = L::cy(k);
                const bool wl = WALL && ((cy == 1 && y == 0) || (cy == -1 && y == ny - 1));
                h[k] = wl ? -(TC)lf[L::opp(k)][r][lane] + cf->ew[cy == 1 ? 0 : 1][k]
                          : (TC)lf[k][r - cy][lane - L::cx(k)];
            }
            const TC pp_off = (SRC && !HAND) ? (TC)lp[HAND ? 0 : r][lane] : TC(0);
            TC out[9];
            const TC phio = collide_node<9, TC, EQ, SRC, KVAR, NP, SB>(cf, h, pp_off, 0u, nullptr, nullptr, false, out,
                                                                        nullptr, prev);
            bad |= !__builtin_isfinite(phio);
            if (x < nx && y < ny) {
                const uint32_t m = (uint32_t)y * g.nx + (uint32_t)x;
                store_planes<9, false>(fout, g.plane, m, out);
                if (SRC) *at<true>(pout, m) = (TP)phio;
            }
        };
        if constexpr (HAND) {
            // the rows this wave ran in phase 1, halo rows excepted
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int r = wv + i * NW;
                if (r < 1 || r > TH || (WALL && y0 + r - 1 >= ny)) continue;
                row2(r, &lev[i]);
            }
        } else {
            for (int r = 1 + wv; r <= TH; r += NW) {
                if (WALL && y0 + r - 1 >= ny) break;
                row2(r, nullptr);
            }
        }
    }
    if (bad) *flag = 1;
}

template <typename TS, typename TC, bool SRC, bool KVAR, int NP, int TH, int NW = kBlock / 64, bool SB = false,
          bool WALL = false, bool EQ = true>
__global__ void __launch_bounds__(64 * NW)
k_sweep2(const Geom g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ fin, TS *__restrict__ fout,
         const typename HistType<TS>::T *__restrict__ pin, typename HistType<TS>::T *__restrict__ pout,
         uint32_t tiles_x, int *flag) {
    const uint32_t tile = block_index(blockIdx.x, gridDim.x, g.remap);
    const uint32_t ty = tile / tiles_x, tx = tile - ty * tiles_x;
    sweep2_tile<TS, TC, SRC, KVAR, NP, TH, NW, SB, WALL, EQ>(g, cf, fin, fout, pin, pout, tx, ty, flag);
}

// The general sweep: Scheme B and/or per-node fields.  Polynomials of any
// length, K(phi) evaluated per node, Scheme-A history kept when SB is off.
// ---------------------------------------------------------------------------
// Two time steps per pass for D3Q19 (3-term polynomials; walls on z or
// periodic).  A workgroup owns a column of 62 x TY nodes in x and y and a
// chunk of zc planes in z, and marches up the chunk.  At logical plane i
// (z = z0 - 1 + i) phase 1 runs step t on the column plus a one-node halo in
// x and y and keeps the post-collision populations in LDS, rounded to the
// storage type as a store would round them; phase 2 then runs step t + 1 on
// plane i - 1 of the column's own nodes, gathering from LDS, and stores only
// that result.  The ring is split by the z component of the velocity:
// c_z = +1 populations are read one plane up (two slots by plane parity,
// written after phase 2 since slot i & 1 still holds plane i - 2 then),
// c_z = 0 on their own plane (two slots) and c_z = -1 one plane down (two
// slots: at the low wall a node also reads its own c_z = -1 populations).
// Every node update is the one-sweep arithmetic on the same inputs, so the
// result equals two single sweeps bit for bit; the state crosses HBM once
// per two steps.  Planes beyond a wall are not computed: the gather there is
// the anti-bounce-back form, -f*_opp(k) of the node itself plus the wall term.
// ---------------------------------------------------------------------------
struct Zc3 {
    // the populations of Eq. 6 by the z component of their velocity
    static constexpr int p[5] = {5, 11, 13, 15, 18};                 // c_z = +1
    static constexpr int z[9] = {0, 1, 2, 3, 4, 7, 8, 9, 10};        // c_z = 0
    static constexpr int m[5] = {6, 12, 14, 16, 17};                 // c_z = -1
    // position of population k within its class
    static constexpr int pos(int k) {
        for (int i = 0; i < 5; ++i) if (p[i] == k || m[i] == k) return i;
        for (int i = 0; i < 9; ++i) if (z[i] == k) return i;
        return -1;
    }
};

// Phase 1 reads each population from a wave-uniform source row (plane
// z - c_z and row y - c_y, periodic, a 32-bit byte offset) plus one of three
// per-lane column offsets (x - c_x, periodic), and the loads of the next
// plane are issued before the current plane's arithmetic, so that their
// latency overlaps phase 1, phase 2 and both barriers.
// SRC: a Scheme-A source.  Phase 1 reads the phi history of its nodes from
// pin (phi(t - 1), the node itself) and keeps phi(t), rounded to the history
// type as a store would round it, and the source terms of phi(t) for phase 2
// of the next plane (in registers when the history type is the compute type,
// else phi(t) in a two-slot ring); phase 2 writes phi(t + 1) to pout, which
// must not be pin (neighbouring columns still read pin at their halo).
// EQ: the equal-rate collision; otherwise the moment-space one (unequal
// non-flux rates).
template <typename TS, typename TC, bool KVAR, bool WALL, int NP, int TY, int NW, bool SB = false, bool SRC = false,
          bool EQ = true>
__global__ void __launch_bounds__(64 * NW)
k_sweep2_3d(const Geom g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ fin, TS *__restrict__ fout,
            const typename HistType<TS>::T *__restrict__ pin, typename HistType<TS>::T *__restrict__ pout,
            uint32_t tiles_x, uint32_t tiles_y, uint32_t zc, int *flag) {
    using L = Lattice<19>;
    using TP = typename HistType<TS>::T;
    constexpr int TX = 64, TR = TY + 2;
    constexpr int PR = (TR + NW - 1) / NW;          // phase-1 rows per wave
    __shared__ TS rp[2][5][TR][TX];
    __shared__ TS r0[2][9][TR][TX];
    __shared__ TS rm[2][5][TR][TX];
    // Scheme A: phase 2 runs the rows the wave ran in phase 1 one plane
    // earlier, so that phi(t) and the source terms of phi(t) of its nodes come
    // from the wave's registers (the history type equals the compute type:
    // they are the values the rebuild from the history would give)
    constexpr bool HAND = SRC && !SB && std::is_same<TP, TC>::value;
    __shared__ TP lp[(SRC && !HAND) ? 2 : 1][(SRC && !HAND) ? TR : 1][TX];
    SrcLevel<TC> lev1[HAND ? PR : 1], lev0[HAND ? PR : 1];   // planes i - 1 and i
    TP ph1[HAND ? PR : 1];                                    // phi - phi_ref of plane i - 1
    const uint32_t blk = block_index(blockIdx.x, gridDim.x, g.remap);
    const uint32_t per_z = tiles_x * tiles_y;
    const uint32_t tz = blk / per_z, rem = blk - tz * per_z;
    const uint32_t tyi = rem / tiles_x, txi = rem - tyi * tiles_x;
    const int nx = (int)g.nx, ny = (int)g.ny, nz = (int)g.nz;
    const int x0 = (int)(txi * (TX - 2)), y0 = (int)(tyi * TY), z0 = (int)(tz * zc);
    const int zend = min(z0 + (int)zc, nz);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int xg = wrap_coord(x0 - 1 + lane, nx);
    // byte offsets of the source columns x - c_x for c_x = 1, 0, -1
    uint32_t cb[3] = {(uint32_t)(xg == 0 ? nx - 1 : xg - 1) * (uint32_t)sizeof(TS),
                      (uint32_t)xg * (uint32_t)sizeof(TS),
                      (uint32_t)(xg == nx - 1 ? 0 : xg + 1) * (uint32_t)sizeof(TS)};
    const uint32_t row_bytes = g.nx * (uint32_t)sizeof(TS);
    uint32_t pcb = (uint32_t)xg * (uint32_t)sizeof(TP);   // the history of the node itself
    bool bad = false;
    const int nplanes = zend - z0 + 2;
    // raw values of the phase-1 gathers of logical plane i (this wave's rows):
    // population k from the source node, or at a wall the own node's opposite
    auto load = [&](int i, TS (&dst)[PR][19], TP (&pdst)[PR]) {
        const int zl = z0 - 1 + i;
        if (WALL && (zl < 0 || zl >= nz)) return;
        const int zg = WALL ? zl : wrap_coord(zl, nz);
        const int zs[3] = {zg == nz - 1 ? 0 : zg + 1, zg, zg == 0 ? nz - 1 : zg - 1};   // z - c_z, c_z = -1, 0, 1
#pragma unroll
        for (int j = 0; j < PR; ++j) {
            const int r = wv + j * NW;
            if (r < TR) {
                const int yg = wrap_coord(y0 - 1 + r, ny);
                const int ys[3] = {yg == ny - 1 ? 0 : yg + 1, yg, yg == 0 ? ny - 1 : yg - 1};   // y - c_y
#pragma unroll
                for (int k = 0; k < 19; ++k) {
                    const int cx = L::cx(k), cy = L::cy(k), cz = L::cz(k);
                    const bool wl = WALL && ((cz == 1 && zg == 0) || (cz == -1 && zg == nz - 1));
                    const uint32_t rb = wl ? ((uint32_t)zg * g.ny + (uint32_t)yg) * row_bytes
                                           : ((uint32_t)zs[1 + cz] * g.ny + (uint32_t)ys[1 + cy]) * row_bytes;
                    dst[j][k] = wl ? *row_elem(fin + (uint64_t)L::opp(k) * g.plane, rb, cb[1])
                                   : *row_elem(fin + (uint64_t)k * g.plane, rb, cb[1 - cx]);
                }
                if (SRC) pdst[j] = *row_elem(pin, ((uint32_t)zg * g.ny + (uint32_t)yg) * g.nx * (uint32_t)sizeof(TP),
                                             pcb);
            }
        }
    };
    TS hn[PR][19];
    TP pn[PR];
    load(0, hn, pn);
    for (int i = 0; i < nplanes; ++i) {
        const int zl = z0 - 1 + i;
        const int s1 = i & 1, s0 = s1 ^ 1;          // slots of plane i and of plane i - 1
        const bool p1 = WALL ? (zl >= 0 && zl < nz) : true;
        const int zg = WALL ? zl : wrap_coord(zl, nz);
        TS hc[PR][19];
        TP pc[PR];
#pragma unroll
        for (int j = 0; j < PR; ++j) {
            pc[j] = pn[j];
#pragma unroll
            for (int k = 0; k < 19; ++k) hc[j][k] = hn[j][k];
        }
        if (i + 1 < nplanes) load(i + 1, hn, pn);
        // phase 1: plane zl (skipped beyond a wall)
        TS keep[PR][5];
        TP ph0[HAND ? PR : 1];
        if (p1) {
#pragma unroll
            for (int j = 0; j < PR; ++j) {
                const int r = wv + j * NW;
                if (r < TR) {
                    TC h[19];
#pragma unroll
                    for (int k = 0; k < 19; ++k) {
                        const int cz = L::cz(k);
                        const bool wl = WALL && ((cz == 1 && zg == 0) || (cz == -1 && zg == nz - 1));
                        h[k] = wl ? -(TC)hc[j][k] + cf->ew[cz == 1 ? 0 : 1][k] : (TC)hc[j][k];
                    }
                    TC out[19];
                    const TC phio = collide_node<19, TC, EQ, SRC, KVAR, NP, SB>(
                        cf, h, SRC ? (TC)pc[j] : TC(0), 0u, nullptr, nullptr, false, out,
                        HAND ? &lev0[HAND ? j : 0] : nullptr);
                    bad |= !__builtin_isfinite(phio);
                    if (SRC && !HAND) lp[s1 & 1][(SRC && !HAND) ? r : 0][lane] = (TP)phio;
                    if (HAND) ph0[HAND ? j : 0] = (TP)phio;
#pragma unroll
                    for (int c = 0; c < 9; ++c) r0[s1][c][r][lane] = (TS)out[Zc3::z[c]];
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        rm[s1][c][r][lane] = (TS)out[Zc3::m[c]];
                        keep[j][c] = (TS)out[Zc3::p[c]];
                    }
                }
            }
        }
        __syncthreads();
        // phase 2: plane zl - 1 of the column's own nodes
        if (i >= 2 && lane >= 1 && lane <= TX - 2) {
            const int zc2 = zl - 1;
            const bool lo = WALL && zc2 == 0, hi = WALL && zc2 == nz - 1;
            const int x = x0 + lane - 1;
            auto row2 = [&](int r, TC pp_off, const SrcLevel<TC> *prev) {
                const int y = y0 + r - 1;
                TC h[19];
#pragma unroll
                for (int k = 0; k < 19; ++k) {
                    const int cx = L::cx(k), cy = L::cy(k), cz = L::cz(k);
                    if (WALL && cz == 1 && lo) {
                        h[k] = -(TC)rm[s0][Zc3::pos(L::opp(k))][r][lane] + cf->ew[0][k];
                    } else if (WALL && cz == -1 && hi) {
                        h[k] = -(TC)rp[s0][Zc3::pos(L::opp(k))][r][lane] + cf->ew[1][k];
                    } else if (cz == 1) {
                        h[k] = (TC)rp[s1][Zc3::pos(k)][r - cy][lane - cx];
                    } else if (cz == -1) {
                        h[k] = (TC)rm[s1][Zc3::pos(k)][r - cy][lane - cx];
                    } else {
                        h[k] = (TC)r0[s0][Zc3::pos(k)][r - cy][lane - cx];
                    }
                }
                TC out[19];
                const TC phio = collide_node<19, TC, EQ, SRC, KVAR, NP, SB>(cf, h, pp_off, 0u, nullptr, nullptr,
                                                                             false, out, nullptr, prev);
                bad |= !__builtin_isfinite(phio);
                if (x < nx && y < ny) {
                    const uint32_t m = ((uint32_t)zc2 * g.ny + (uint32_t)y) * g.nx + (uint32_t)x;
                    store_planes<19, false>(fout, g.plane, m, out);
                    if (SRC) *at<true>(pout, m) = (TP)phio;
                }
            };
            if constexpr (HAND) {
#pragma unroll
                for (int j = 0; j < PR; ++j) {
                    const int r = wv + j * NW;
                    if (r >= 1 && r <= TY) row2(r, (TC)ph1[j], &lev1[j]);
                }
            } else {
                for (int r = 1 + wv; r <= TY; r += NW)
                    row2(r, SRC ? (TC)lp[s0 & 1][(SRC && !HAND) ? r : 0][lane] : TC(0), nullptr);
            }
        }
        if constexpr (HAND) {
#pragma unroll
            for (int j = 0; j < PR; ++j) {
                lev1[j] = lev0[j];
                ph1[j] = ph0[j];
            }
        }
        __syncthreads();
        // the c_z = +1 populations of plane i, now that plane i - 2's are read
        if (p1) {
#pragma unroll
            for (int j = 0; j < PR; ++j) {
                const int r = wv + j * NW;
                if (r < TR) {
#pragma unroll
                    for (int c = 0; c < 5; ++c) rp[s1][c][r][lane] = keep[j][c];
                }
            }
        }
    }
    if (bad) *flag = 1;
}

template <int Q, typename TS, typename TC, bool EQR, bool WALL, bool SB>
__global__ void __launch_bounds__(kBlock)
k_sweep_gen(const Geom g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ fin,
            TS *__restrict__ fout, typename HistType<TS>::T *p, int *flag, const double *kfield,
            const double *rfield, int remark3) {
    const uint32_t n = block_index(blockIdx.x, gridDim.x, g.remap) * kBlock + threadIdx.x;
    if (n >= g.N) return;
    sweep_node<Q, TS, TC, EQR, !SB, true, WALL, 9, false, SB, true>(g, cf, fin, fout, p, flag, n, kfield, rfield,
                                                                   remark3 != 0);
}

// ---------------------------------------------------------------------------
// initialisation (Eq. 40) in the gather convention
// ---------------------------------------------------------------------------
template <int Q, int NP, typename TC>
__device__ __forceinline__ TC feq_one(const Coefs<TC> *__restrict__ cf, TC phi, int kk) {
    TC feq[Q];
    equilibrium<Q, NP>(cf, phi, phi - cf->phi_ref, feq);
    TC v = feq[0];
#pragma unroll
    for (int k = 1; k < Q; ++k)
        if (k == kk) v = feq[k];
    return v;
}

// Scheme B: R_k / 2 at a node (Eq. 9 with Btilde = B', R explicit in phi).
template <int Q, int NP, typename TC>
__device__ __forceinline__ TC half_source_one(const Coefs<TC> *__restrict__ cf, TC phi, TC R, int kk) {
    using L = Lattice<Q>;
    TC cb = TC(0);
#pragma unroll
    for (int a = 0; a < L::dim; ++a) {
        const int c = L::c(kk, a);
        if (c) cb += TC(c) * flux_bp<NP>(cf, a, phi);
    }
    return TC(0.5) * TC(L::w(kk)) * R * (TC(1) + TC(3) * cb);
}

template <int Q, typename TS, typename TC, bool WALL, int NP, bool SB = false>
__global__ void __launch_bounds__(kBlock)
k_init(const Geom g, const Coefs<TC> *__restrict__ cf, const double *__restrict__ phi0,
       TS *__restrict__ f, typename HistType<TS>::T *p, const double *rfield = nullptr) {
    using L = Lattice<Q>;
    constexpr int D = L::dim;
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const NodeGeo ng = node_geometry<Q, WALL>(g, n);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        // slot k at x is read by x + c_k, unless that lies beyond a wall;
        // then it is read back by x itself for the opposite direction.
        const int cl = L::c(k, D - 1);
        TC v;
        if (WALL && ((cl == 1 && ng.hi) || (cl == -1 && ng.lo))) {
            const TC ph = (TC)phi0[n];
            TC e = feq_one<Q, NP>(cf, ph, L::opp(k));
            // Scheme B stores fbar = feq - R_k / 2 (Eq. 33)
            if (SB) e -= half_source_one<Q, NP>(cf, ph, poly<NP>(cf->r, ph) + (rfield ? (TC)rfield[n] : TC(0)), L::opp(k));
            v = cf->ew[cl == 1 ? 1 : 0][k] - e;
        } else {
            int off = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int c = L::c(k, a);
                off += (c == 1) ? ng.op[a] : ((c == -1) ? ng.om[a] : 0);
            }
            const uint32_t src = (uint32_t)((int)n + off);
            const TC ph = (TC)phi0[src];
            v = feq_one<Q, NP>(cf, ph, k);
            if (SB) v -= half_source_one<Q, NP>(cf, ph, poly<NP>(cf->r, ph) + (rfield ? (TC)rfield[src] : TC(0)), k);
        }
        store_s(f + (uint64_t)k * g.plane + n, v);
    }
    if (p) p[n] = (typename HistType<TS>::T)((TC)phi0[n] - cf->phi_ref);
}

// phi = phi_ref + sum_k g_k (Scheme B: + R / 2, Eq. 35), accumulated in FP64.
// phi at node n of a state (Eq. 10a; Scheme B Eq. 35), in FP64.
template <int Q, typename TS, typename TC, bool WALL, bool SB>
__device__ __forceinline__ double phi_at(const Geom &g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ f,
                                         uint32_t n, const double *rfield) {
    const NodeGeo ng = node_geometry<Q, WALL>(g, n);
    TC h[Q];
    gather<Q, WALL>(g, cf, f, ng, h);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) acc += (double)h[k];
    if (SB) {
        double R;
        acc = phi_scheme_b<double>(cf, acc, rfield ? rfield[n] : 0.0, &R);
    }
    return (double)cf->phi_ref + acc;
}

template <int Q, typename TS, typename TC, bool WALL, bool SB>
__global__ void __launch_bounds__(kBlock)
k_phi(const Geom g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ f,
      double *__restrict__ phi, const double *rfield = nullptr) {
    const uint32_t n = block_index(blockIdx.x, gridDim.x, g.remap) * kBlock + threadIdx.x;
    if (n >= g.N) return;
    phi[n] = phi_at<Q, TS, TC, WALL, SB>(g, cf, f, n, rfield);
}

// The FP64 reductions of lbm_reduce over phi formed from the state on the
// fly (no phi field written or read): per-workgroup partials in the same
// per-thread order as the reduction over a stored phi field.
template <int Q, typename TS, typename TC, bool WALL, bool SB>
__global__ void __launch_bounds__(kBlock)
k_phi_reduce(const Geom g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ f,
             const double *__restrict__ ref, const double *rfield, double *__restrict__ part) {
    double acc[kRed];
    red_init(acc);
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < g.N; i += gridDim.x * kBlock)
        red_add(acc, phi_at<Q, TS, TC, WALL, SB>(g, cf, f, i, rfield), ref ? ref[i] : 0.0);
    red_block_fold(acc, part + (size_t)blockIdx.x * kRed);
}

// ---------------------------------------------------------------------------
// Anti-bounce-back wall terms rewritten on the device (time-dependent wall
// values): 2 e+_k(phi_w) for both walls arrive as a kernel argument, and the
// stored offset form 2 e+_k - 2 w_k phi_ref uses the phi_ref on the device.
// ---------------------------------------------------------------------------
struct WallTerms {
    double ewp[2][19];
};

template <int Q, typename TC>
__global__ void __launch_bounds__(64) k_set_wall(Coefs<TC> *cf, WallTerms w) {
    using L = Lattice<Q>;
    const int t = threadIdx.x;
    if (t < 2 * Q) {
        const int side = t / Q, k = t % Q;
        cf->ewp[side][k] = (TC)w.ewp[side][k];
        cf->ew[side][k] = (TC)(w.ewp[side][k] - 2.0 * L::w(k) * (double)cf->phi_ref);
    }
}

// ---------------------------------------------------------------------------
// Sum of an FP64 value over the 64 lanes of a wave (every lane must be
// active), returned in every lane.  Inside each row of 16 lanes the DPP quad
// swaps (lane ^ 1, lane ^ 2) and the half-row and row mirrors pair every
// quad, then every half-row, with its partner, leaving the row sum in all 16
// lanes; the four row sums are then read from lanes 0, 16, 32 and 48.  No
// LDS traffic and a fixed order (deterministic).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float lane_f32(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// DPP move restricted to the rows in ROWS; lanes of the other rows read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}

// Sum over the 64 lanes of a wave, the same in every lane.  The four row
// sums r0..r3 are combined with the row broadcasts of the DPP unit: rows 1
// and 3 add lane 15 of the row before (r1 + r0, r3 + r2), then row 3 adds
// lane 31 ((r3 + r2) + (r1 + r0)); one read of lane 63.  IEEE addition is
// commutative, so this equals (r0 + r1) + (r2 + r3), the order of the FP64
// form below, bit for bit.
__device__ __forceinline__ float wave_total(float v) {
    v += dpp_f32<0xB1>(v);                 // quad_perm (1, 0, 3, 2)
    v += dpp_f32<0x4E>(v);                 // quad_perm (2, 3, 0, 1)
    v += dpp_f32<0x141>(v);                // row_half_mirror
    v += dpp_f32<0x140>(v);                // row_mirror: every lane holds its row's sum
    v += dpp_rows_f32<0x142, 0xA>(v);      // row_bcast:15 into rows 1 and 3
    v += dpp_rows_f32<0x143, 0xC>(v);      // row_bcast:31 into rows 2 and 3
    return lane_f32(v, 63);
}

__device__ __forceinline__ double wave_total(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm (1, 0, 3, 2)
    v += dpp_f64<0x4E>(v);   // quad_perm (2, 3, 0, 1)
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// ---------------------------------------------------------------------------
// Re-centring of the stored offsets h_k = f_k - w_k phi_ref.  Moving phi_ref
// to the current mean of phi keeps the stored magnitudes at the size of the
// fluctuations of phi, which is what bounds the rounding of short storage
// formats when phi drifts (source terms, walls).  In exact arithmetic nothing
// the method computes changes: with delta = old - new,
//   h_k += w_k delta,  P += delta,  wall terms 2 e+_k(phi_w) - 2 w_k new,
// so every gathered population, phi, and the Scheme-A history are the same.
// ---------------------------------------------------------------------------

// Per-workgroup FP64 sums of the offset mass: the history P (one value per
// node, phi of the previous step less phi_ref) when the run keeps one, else
// the sum over the stored populations.
template <int Q, typename TS>
__global__ void __launch_bounds__(kBlock)
k_offset_sum(const Geom g, const TS *__restrict__ f, const typename HistType<TS>::T *__restrict__ p,
             int use_hist, double *__restrict__ part) {
    double acc = 0.0;
    for (uint32_t n = blockIdx.x * kBlock + threadIdx.x; n < g.N; n += gridDim.x * kBlock) {
        if (use_hist) {
            acc += (double)p[n];
        } else {
#pragma unroll
            for (int k = 0; k < Q; ++k) acc += (double)f[(uint64_t)k * g.plane + n];
        }
    }
    __shared__ double sh[kBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
        part[blockIdx.x] = t;
    }
}

// One workgroup: fold the partial sums in a fixed order, move phi_ref to the
// mean and rewrite the wall terms; the shift old - new goes to shift[0].
template <int Q, typename TC>
__global__ void __launch_bounds__(kBlock)
k_recenter_fold(Coefs<TC> *cf, const double *__restrict__ part, int nparts, uint32_t N,
                double *__restrict__ shift) {
    using L = Lattice<Q>;
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) acc += part[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double old = (double)cf->phi_ref;
    const TC nref = (TC)(old + sh[0] / (double)N);
    __syncthreads();  // every lane has read phi_ref before it is rewritten
    if (threadIdx.x < 2 * Q) {
        const int side = threadIdx.x / Q, k = threadIdx.x % Q;
        cf->ew[side][k] = (TC)((double)cf->ewp[side][k] - 2.0 * L::w(k) * (double)nref);
    }
    if (threadIdx.x == 0) {
        cf->phi_ref = nref;
        shift[0] = old - (double)nref;
    }
}

template <int Q, typename TS, typename TC>
__global__ void __launch_bounds__(kBlock)
k_shift(const Geom g, const double *__restrict__ shift, TS *__restrict__ f,
        typename HistType<TS>::T *__restrict__ p) {
    using L = Lattice<Q>;
    using TP = typename HistType<TS>::T;
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const double d = shift[0];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        TS *q = f + (uint64_t)k * g.plane + n;
        *q = (TS)((TC)*q + (TC)(L::w(k) * d));
    }
    p[n] = (TP)((double)p[n] + d);
}

}  // namespace lbm
