// Many independent D2Q9 instances of uneven size advanced by one launch per
// time step.
//
// All instances' distribution planes live in two arenas (ping-pong) and one
// phi-history arena owned by the caller.  A device work list holds one entry
// per tile (instance, first node); a tile is WG * NPT consecutive nodes of
// one instance.  Workgroups walk contiguous chunks of the list (persistent
// when the grid is smaller than the tile count); the chunk order is
// XCD-aware so that each XCD sweeps a contiguous run of instances.  Runs of
// sweeps are replayed from captured HIP graphs.  An autotuner times the
// candidate (WG, NPT, grid) shapes on the real batch and keeps the fastest;
// results are cached in a small text file.  Batches without a source whose
// polynomials have degree <= 2 may instead advance two time steps per launch:
// a second work list holds one entry per (instance, 62 x TH tile), and each
// workgroup runs the two-step tile of the single-instance pass on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include <cerrno>
#include <sys/stat.h>
#include <sys/types.h>

#include "../../include/lbm.h"
#include "lbm_kernels.h"

namespace lbm {

struct BatchInst {
    Geom g;
    uint64_t f_off;    // element offset of plane 0 in the distribution arenas
    uint64_t p_off;    // element offset in the history arena and the phi arena
};

struct TileShape {
    int wg, npt;
};

constexpr TileShape kShapes[] = {{256, 1}, {256, 2}, {128, 1}, {512, 1}};
constexpr int kNumShapes = 4;

// two-step shapes (tile rows, waves per workgroup), batch shape indices
// kNumShapes + i: 4- and 2-byte storage, and FP64
struct TwoShape {
    int rows, waves;
};
constexpr TwoShape kTwo4[] = {{14, 8}, {6, 4}};
constexpr TwoShape kTwo8[] = {{6, 8}};
constexpr int kMaxTwo = 2;

template <typename TS, typename TC, bool SRC, bool KVAR, int WG, int NPT, int NP>
__global__ void __launch_bounds__(WG)
k_batch_sweep(const BatchInst *__restrict__ inst, const Coefs<TC> *__restrict__ coefs,
              const uint2 *__restrict__ tiles, uint32_t ntiles, uint32_t chunk, int remap,
              const TS *__restrict__ fin, TS *__restrict__ fout, typename HistType<TS>::T *p, int *flag) {
    const uint32_t b = block_index(blockIdx.x, gridDim.x, remap);
    const uint32_t t0 = b * chunk;
    const uint32_t t1 = min(t0 + chunk, ntiles);
    for (uint32_t t = t0; t < t1; ++t) {
        const uint2 e = tiles[t];
        const BatchInst &I = inst[e.x];
        const Geom g = I.g;
        const Coefs<TC> *cf = coefs + e.x;
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const uint32_t n = e.y + j * WG + threadIdx.x;
            if (n < g.N)
                sweep_node<9, TS, TC, true, SRC, KVAR, false, NP>(g, cf, fin + I.f_off, fout + I.f_off,
                                                               p + I.p_off, flag, n);
        }
    }
}

// Two time steps per launch (no source, so no phi history): one workgroup per
// entry (instance, tx | ty << 16) of the two-step work list.
template <typename TS, typename TC, bool KVAR, int TH, int NW>
__global__ void __launch_bounds__(64 * NW)
k_batch_sweep2(const BatchInst *__restrict__ inst, const Coefs<TC> *__restrict__ coefs,
               const uint2 *__restrict__ tiles, int remap, const TS *__restrict__ fin, TS *__restrict__ fout,
               int *flag) {
    const uint2 e = tiles[block_index(blockIdx.x, gridDim.x, remap)];
    const BatchInst &I = inst[e.x];
    const Geom g = I.g;
    sweep2_tile<TS, TC, false, KVAR, 3, TH, NW>(g, coefs + e.x, fin + I.f_off, fout + I.f_off, nullptr, nullptr,
                                               e.y & 0xffffu, e.y >> 16, flag);
}

template <typename TS, typename TC, int NP>
__global__ void __launch_bounds__(256)
k_batch_init(const BatchInst *__restrict__ inst, const Coefs<TC> *__restrict__ coefs,
             const uint2 *__restrict__ tiles, uint32_t ntiles, int tile_nodes, const double *__restrict__ phi0,
             TS *__restrict__ f, typename HistType<TS>::T *p) {
    using L = Lattice<9>;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint2 e = tiles[t];
        const BatchInst &I = inst[e.x];
        const Geom g = I.g;
        const Coefs<TC> *cf = coefs + e.x;
        for (int j = threadIdx.x; j < tile_nodes; j += 256) {
            const uint32_t n = e.y + j;
            if (n >= g.N) continue;
            const NodeGeo ng = node_geometry<9, false>(g, n);
            const double *ph0 = phi0 + I.p_off;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                int off = 0;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int c = L::c(k, a);
                    off += (c == 1) ? ng.op[a] : ((c == -1) ? ng.om[a] : 0);
                }
                const TC ph = (TC)ph0[(uint32_t)((int)n + off)];
                store_s(f + I.f_off + (uint64_t)k * g.plane + n, feq_one<9, NP>(cf, ph, k));
            }
            p[I.p_off + n] = (typename HistType<TS>::T)((TC)ph0[n] - cf->phi_ref);
        }
    }
}

template <typename TS, typename TC>
__global__ void __launch_bounds__(256)
k_batch_phi(const BatchInst *__restrict__ inst, const Coefs<TC> *__restrict__ coefs,
            const uint2 *__restrict__ tiles, uint32_t ntiles, int tile_nodes, const TS *__restrict__ f,
            double *__restrict__ phi) {
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint2 e = tiles[t];
        const BatchInst &I = inst[e.x];
        const Geom g = I.g;
        const Coefs<TC> *cf = coefs + e.x;
        for (int j = threadIdx.x; j < tile_nodes; j += 256) {
            const uint32_t n = e.y + j;
            if (n >= g.N) continue;
            const NodeGeo ng = node_geometry<9, false>(g, n);
            TC h[9];
            gather<9, false>(g, cf, f + I.f_off, ng, h);
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 9; ++k) acc += (double)h[k];
            phi[I.p_off + n] = (double)cf->phi_ref + acc;
        }
    }
}

}  // namespace lbm

using namespace lbm;

namespace lbm {
// coefficient derivation shared with the single-instance API (lbm_api.hip)
int derive_coefs(const lbm_desc *d, int *prec, bool *eqr, bool *src, bool *kvar, bool *lowdeg, bool *deg3,
                 void *coefs_out, size_t *coef_bytes);
const char *api_error_message();
int api_fail(int code, const char *msg);
}  // namespace lbm

struct lbm_batch {
    int count = 0;
    int prec = 0;
    bool src = false, kvar = false, lowdeg = true, deg3 = true;
    size_t coef_stride = 0;
    std::vector<BatchInst> inst;
    std::vector<int> nx, ny;
    uint64_t total_nodes = 0;
    BatchInst *d_inst = nullptr;
    void *d_coefs = nullptr;
    // one tile list per shape (tile size differs)
    uint2 *d_tiles[kNumShapes] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t ntiles[kNumShapes] = {0, 0, 0, 0};
    // two-step work lists, one per two-step shape (tile rows differ)
    uint2 *d_tiles2[kMaxTwo] = {nullptr, nullptr};
    uint32_t ntiles2[kMaxTwo] = {0, 0};
    int ntwo = 0;           // two-step shapes available (0: no source-free 3-term batch)
    int *d_flag = nullptr;
    int shape = 0;          // index into kShapes, or kNumShapes + a two-step shape
    uint32_t grid = 0;      // workgroups per sweep (0 = one per tile)
    int remap = 1;
    void *f[2] = {nullptr, nullptr};
    void *p = nullptr;
    const double *phi0 = nullptr;
    int cur = 0;
    long long t = 0;
    bool bound = false;
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::string key;
};

namespace {

constexpr int kBatchGraphSteps = 32;

size_t ssize(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }
size_t hsize(int prec) { return prec == 0 ? 8 : 4; }
size_t r256(size_t v) { return (v + 255) & ~size_t(255); }

TwoShape two_shape(const lbm_batch *b, int i) { return b->prec == 0 ? kTwo8[i] : kTwo4[i]; }

bool is_two(const lbm_batch *b) { return b->shape >= kNumShapes; }

// one sweep; single-sweep shape `shape` (a two-step batch uses shape 0 for
// an odd remaining step)
hipError_t batch_sweep_launch(lbm_batch *b, const void *fin, void *fout, hipStream_t st, int shape) {
    const TileShape sh = kShapes[shape];
    const uint32_t nt = b->ntiles[shape];
    const uint32_t grid = (shape != b->shape || b->grid == 0 || b->grid > nt) ? nt : b->grid;
    const uint32_t chunk = (nt + grid - 1) / grid;
    const uint32_t nblk = (nt + chunk - 1) / chunk;
    const uint2 *tl = b->d_tiles[shape];
#define LBM_BL(TS, TC, S, K, WG, NPT)                                                                   \
    if (b->lowdeg) LBM_BL_NP(TS, TC, S, K, WG, NPT, 4) else LBM_BL_NP(TS, TC, S, K, WG, NPT, 9)
#define LBM_BL_NP(TS, TC, S, K, WG, NPT, NP)                                                            \
    hipLaunchKernelGGL((k_batch_sweep<TS, TC, S, K, WG, NPT, NP>), dim3(nblk), dim3(WG), 0, st,         \
                       b->d_inst, (const Coefs<TC> *)b->d_coefs, tl, nt, chunk, b->remap,               \
                       (const TS *)fin, (TS *)fout, (typename HistType<TS>::T *)b->p, b->d_flag);
#define LBM_BL_SHAPE(TS, TC, S, K)                                                                      \
    switch (shape) {                                                                                    \
        case 0: LBM_BL(TS, TC, S, K, 256, 1); break;                                                    \
        case 1: LBM_BL(TS, TC, S, K, 256, 2); break;                                                    \
        case 2: LBM_BL(TS, TC, S, K, 128, 1); break;                                                    \
        default: LBM_BL(TS, TC, S, K, 512, 1); break;                                                   \
    }
#define LBM_BL_FLAGS(TS, TC)                                                                            \
    if (b->src && b->kvar) { LBM_BL_SHAPE(TS, TC, true, true) }                                         \
    else if (b->src) { LBM_BL_SHAPE(TS, TC, true, false) }                                              \
    else if (b->kvar) { LBM_BL_SHAPE(TS, TC, false, true) }                                             \
    else { LBM_BL_SHAPE(TS, TC, false, false) }
    (void)sh;
    if (b->prec == 0) { LBM_BL_FLAGS(double, double) }
    else if (b->prec == 1) { LBM_BL_FLAGS(float, float) }
    else { LBM_BL_FLAGS(_Float16, float) }
#undef LBM_BL_FLAGS
#undef LBM_BL_SHAPE
#undef LBM_BL
#undef LBM_BL_NP
    return hipGetLastError();
}

// two time steps, two-step shape b->shape - kNumShapes
hipError_t batch_sweep2_launch(lbm_batch *b, const void *fin, void *fout, hipStream_t st) {
    const int i = b->shape - kNumShapes;
    const TwoShape sh = two_shape(b, i);
    const dim3 grid(b->ntiles2[i]);
    const uint2 *tl = b->d_tiles2[i];
#define LBM_B2(TS, TC, K, TH, NW)                                                                       \
    hipLaunchKernelGGL((k_batch_sweep2<TS, TC, K, TH, NW>), grid, dim3(64 * NW), 0, st, b->d_inst,      \
                       (const Coefs<TC> *)b->d_coefs, tl, b->remap, (const TS *)fin, (TS *)fout, b->d_flag)
#define LBM_B2_SHAPE(TS, TC, K)                                                                         \
    if (sh.rows == 14) LBM_B2(TS, TC, K, 14, 8);                                                        \
    else LBM_B2(TS, TC, K, 6, 4);
    if (b->prec == 0) {
        if (b->kvar) LBM_B2(double, double, true, 6, 8);
        else LBM_B2(double, double, false, 6, 8);
    } else if (b->prec == 1) {
        if (b->kvar) { LBM_B2_SHAPE(float, float, true) }
        else { LBM_B2_SHAPE(float, float, false) }
    } else {
        if (b->kvar) { LBM_B2_SHAPE(_Float16, float, true) }
        else { LBM_B2_SHAPE(_Float16, float, false) }
    }
#undef LBM_B2_SHAPE
#undef LBM_B2
    return hipGetLastError();
}

// `steps` time steps from f[start]: pairs in two-step launches (the odd step,
// if any, a single sweep); the state ends in f[start ^ (launches & 1)]
hipError_t batch_advance(lbm_batch *b, int start, int steps, hipStream_t st, int *end) {
    hipError_t e = hipSuccess;
    int cur = start;
    if (is_two(b)) {
        for (int i = 0; i + 1 < steps && e == hipSuccess; i += 2) {
            e = batch_sweep2_launch(b, b->f[cur], b->f[cur ^ 1], st);
            cur ^= 1;
        }
        if ((steps & 1) && e == hipSuccess) {
            e = batch_sweep_launch(b, b->f[cur], b->f[cur ^ 1], st, 0);
            cur ^= 1;
        }
    } else {
        for (int i = 0; i < steps && e == hipSuccess; ++i) {
            e = batch_sweep_launch(b, b->f[cur], b->f[cur ^ 1], st, b->shape);
            cur ^= 1;
        }
    }
    *end = cur;
    return e;
}

void drop_graphs(lbm_batch *b) {
    for (int i = 0; i < 2; ++i)
        if (b->gexec[i]) { (void)hipGraphExecDestroy(b->gexec[i]); b->gexec[i] = nullptr; }
}

hipError_t make_graph(lbm_batch *b, int start) {
    hipError_t e = hipSuccess;
    if (!b->cap) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    int end = start;
    const hipError_t le = batch_advance(b, start, kBatchGraphSteps, b->cap, &end);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->cap, &graph);
    if (le != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return le; }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->gexec[start], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return e;
}

#define LBM_INIT_NP(KERNEL, ...)                                                      \
    do {                                                                              \
        if (b->lowdeg) {                                                              \
            constexpr int NPV = 4;                                                    \
            hipLaunchKernelGGL(KERNEL, __VA_ARGS__);                                  \
        } else {                                                                      \
            constexpr int NPV = 9;                                                    \
            hipLaunchKernelGGL(KERNEL, __VA_ARGS__);                                  \
        }                                                                             \
    } while (0)

hipError_t batch_init_launch(lbm_batch *b, hipStream_t st) {
    const uint32_t nt = b->ntiles[0];
    const int tn = kShapes[0].wg * kShapes[0].npt;
    const uint32_t grid = std::min<uint32_t>(nt, 8192);
    if (b->prec == 0)
        LBM_INIT_NP((k_batch_init<double, double, NPV>), dim3(grid), dim3(256), 0, st, b->d_inst,
                           (const Coefs<double> *)b->d_coefs, b->d_tiles[0], nt, tn, b->phi0, (double *)b->f[0],
                           (double *)b->p);
    else if (b->prec == 1)
        LBM_INIT_NP((k_batch_init<float, float, NPV>), dim3(grid), dim3(256), 0, st, b->d_inst,
                           (const Coefs<float> *)b->d_coefs, b->d_tiles[0], nt, tn, b->phi0, (float *)b->f[0],
                           (float *)b->p);
    else
        LBM_INIT_NP((k_batch_init<_Float16, float, NPV>), dim3(grid), dim3(256), 0, st, b->d_inst,
                           (const Coefs<float> *)b->d_coefs, b->d_tiles[0], nt, tn, b->phi0, (_Float16 *)b->f[0],
                           (float *)b->p);
    return hipGetLastError();
}

std::string cache_path() {
    const char *env = std::getenv("LBM_TUNE_CACHE");
    if (env && *env) return env;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/lbm_batch_tune.txt";
}

bool cache_lookup(const std::string &key, int &shape, uint32_t &grid, int &remap) {
    std::ifstream in(cache_path());
    std::string k;
    int s, r;
    unsigned g;
    while (in >> k >> s >> g >> r)
        if (k == key && s >= 0 && s < kNumShapes + kMaxTwo) { shape = s; grid = g; remap = r; return true; }
    return false;
}

// create every missing directory of `dir` (no shell involved)
bool make_dirs(const std::string &dir) {
    for (size_t i = 1; i <= dir.size(); ++i) {
        if (i < dir.size() && dir[i] != '/') continue;
        const std::string part = dir.substr(0, i);
        struct stat st;
        if (stat(part.c_str(), &st) == 0) {
            if (!S_ISDIR(st.st_mode)) return false;
        } else if (mkdir(part.c_str(), 0755) != 0 && errno != EEXIST) {
            return false;
        }
    }
    return true;
}

void cache_store(const std::string &key, int shape, uint32_t grid, int remap) {
    const std::string path = cache_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos && slash > 0 && !make_dirs(path.substr(0, slash))) return;
    std::ofstream out(path, std::ios::app);
    if (out) out << key << " " << shape << " " << grid << " " << remap << "\n";
}

}  // namespace

extern "C" {

int lbm_batch_create(const lbm_desc *descs, int count, lbm_batch **out) {
    if (!descs || !out || count < 1) return api_fail(LBM_E_INVALID, "null descriptions or count < 1");
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return api_fail(LBM_E_INVALID, "out of host memory");
    b->count = count;
    std::vector<unsigned char> coefs;
    std::ostringstream key;
    uint64_t foff = 0, poff = 0;
    for (int i = 0; i < count; ++i) {
        const lbm_desc &d = descs[i];
        if (d.lattice != LBM_D2Q9) { delete b; return api_fail(LBM_E_UNSUPPORTED, "batches are D2Q9 only"); }
        if (d.bc[0] != LBM_BC_PERIODIC || d.bc[1] != LBM_BC_PERIODIC) {
            delete b;
            return api_fail(LBM_E_UNSUPPORTED, "batched instances must be periodic");
        }
        int prec = 0;
        bool eqr = false, src = false, kvar = false, low = false, d3 = false;
        size_t cb = 0;
        std::vector<unsigned char> tmp(sizeof(Coefs<double>));
        const int rc = derive_coefs(&d, &prec, &eqr, &src, &kvar, &low, &d3, tmp.data(), &cb);
        if (rc != LBM_OK) { delete b; return rc; }
        if (!eqr) { delete b; return api_fail(LBM_E_UNSUPPORTED, "batched instances need equal non-flux rates"); }
        if (d.flags & LBM_FLAG_REMARK3) {
            delete b;
            return api_fail(LBM_E_UNSUPPORTED, "batched instances use the equilibrium of Eq. 3 (no Remark III)");
        }
        if (d.scheme == LBM_SCHEME_B && src) {
            delete b;
            return api_fail(LBM_E_UNSUPPORTED, "batched instances run Scheme A (Scheme B only without a source)");
        }
        if (i == 0) { b->prec = prec; b->coef_stride = cb; }
        else if (prec != b->prec) { delete b; return api_fail(LBM_E_INVALID, "all instances need the same precision"); }
        b->src = b->src || src;
        b->kvar = b->kvar || kvar;
        b->lowdeg = b->lowdeg && low;
        b->deg3 = b->deg3 && d3;
        coefs.insert(coefs.end(), tmp.begin(), tmp.begin() + cb);
        BatchInst I;
        std::memset(&I, 0, sizeof(I));
        I.g.nx = d.nx; I.g.ny = d.ny; I.g.nz = 1;
        I.g.N = (uint32_t)((size_t)d.nx * d.ny);
        I.g.plane = plane_stride(I.g.N, 9, ssize(prec), d.plane_pad);
        I.g.fx.set(I.g.nx);
        I.g.fxy.set(I.g.N);
        I.g.nblocks = 0;
        I.g.remap = 0;
        I.f_off = foff;
        I.p_off = poff;
        foff += 9ull * I.g.plane;      // plane strides keep every plane 256-byte aligned
        poff += I.g.N;
        b->inst.push_back(I);
        b->nx.push_back(d.nx);
        b->ny.push_back(d.ny);
        b->total_nodes += I.g.N;
        key << d.nx << "x" << d.ny << ",";
    }
    if (b->total_nodes >= (1ull << 31) || foff >= (1ull << 40)) {
        delete b;
        return api_fail(LBM_E_INVALID, "batch too large");
    }
    {
        // short key: precision, flags, FNV-1a of the size list
        std::string s = key.str();
        uint64_t h = 1469598103934665603ull;
        for (char c : s) { h ^= (unsigned char)c; h *= 1099511628211ull; }
        char buf[64];
        std::snprintf(buf, sizeof(buf), "p%d_s%d_k%d_n%d_%016llx", b->prec, (int)b->src, (int)b->kvar, count,
                      (unsigned long long)h);
        b->key = buf;
    }
    hipError_t e = hipMalloc((void **)&b->d_inst, sizeof(BatchInst) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_coefs, coefs.size());
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_flag, 256);
    if (e == hipSuccess) e = hipMemcpy(b->d_inst, b->inst.data(), sizeof(BatchInst) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_coefs, coefs.data(), coefs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_flag, 0, 256);
    for (int s = 0; s < kNumShapes && e == hipSuccess; ++s) {
        const uint32_t tn = (uint32_t)(kShapes[s].wg * kShapes[s].npt);
        std::vector<uint2> tl;
        for (int i = 0; i < count; ++i)
            for (uint32_t n = 0; n < b->inst[i].g.N; n += tn) tl.push_back(make_uint2((unsigned)i, n));
        b->ntiles[s] = (uint32_t)tl.size();
        e = hipMalloc((void **)&b->d_tiles[s], sizeof(uint2) * tl.size());
        if (e == hipSuccess) e = hipMemcpy(b->d_tiles[s], tl.data(), sizeof(uint2) * tl.size(), hipMemcpyHostToDevice);
    }
    // two-step work lists: source-free batches with 3-term polynomials, every
    // instance below 65536 tiles per axis (16-bit tile coordinates) and with
    // planes below 4 GiB (32-bit byte offsets)
    bool fits = true;
    for (int i = 0; i < count; ++i)
        fits = fits && (b->inst[i].g.nx + 61) / 62 < 65536u && b->inst[i].g.ny < 65536u * 6u &&
               (uint64_t)b->inst[i].g.plane * 8u < (1ull << 32);
    b->ntwo = (!b->src && b->deg3 && fits) ? (b->prec == 0 ? 1 : 2) : 0;
    for (int s = 0; s < b->ntwo && e == hipSuccess; ++s) {
        const uint32_t th = (uint32_t)two_shape(b, s).rows;
        std::vector<uint2> tl;
        for (int i = 0; i < count; ++i) {
            const uint32_t tx = (b->inst[i].g.nx + 61) / 62, ty = (b->inst[i].g.ny + th - 1) / th;
            for (uint32_t y = 0; y < ty; ++y)
                for (uint32_t x = 0; x < tx; ++x) tl.push_back(make_uint2((unsigned)i, x | (y << 16)));
        }
        b->ntiles2[s] = (uint32_t)tl.size();
        e = hipMalloc((void **)&b->d_tiles2[s], sizeof(uint2) * tl.size());
        if (e == hipSuccess) e = hipMemcpy(b->d_tiles2[s], tl.data(), sizeof(uint2) * tl.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        lbm_batch_destroy(b);
        std::string m = std::string("batch setup: ") + hipGetErrorString(e);
        return api_fail(LBM_E_HIP, m.c_str());
    }
    *out = b;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b) {
    if (!b) return;
    drop_graphs(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_coefs) (void)hipFree(b->d_coefs);
    if (b->d_flag) (void)hipFree(b->d_flag);
    for (int s = 0; s < kNumShapes; ++s)
        if (b->d_tiles[s]) (void)hipFree(b->d_tiles[s]);
    for (int s = 0; s < kMaxTwo; ++s)
        if (b->d_tiles2[s]) (void)hipFree(b->d_tiles2[s]);
    delete b;
}

int lbm_batch_layout(const lbm_batch *b, size_t *f_bytes, size_t *p_bytes, long long *total_nodes) {
    if (!b) return api_fail(LBM_E_INVALID, "null batch");
    const BatchInst &last = b->inst.back();
    const uint64_t fel = last.f_off + 9ull * last.g.plane;
    if (f_bytes) *f_bytes = r256(fel * ssize(b->prec));
    if (p_bytes) *p_bytes = r256(b->total_nodes * hsize(b->prec));
    if (total_nodes) *total_nodes = (long long)b->total_nodes;
    return LBM_OK;
}

int lbm_batch_instance(const lbm_batch *b, int i, long long *node_offset, int *nx, int *ny) {
    if (!b || i < 0 || i >= b->count) return api_fail(LBM_E_INVALID, "bad instance index");
    if (node_offset) *node_offset = (long long)b->inst[i].p_off;
    if (nx) *nx = b->nx[i];
    if (ny) *ny = b->ny[i];
    return LBM_OK;
}

int lbm_batch_init(lbm_batch *b, const double *phi0, void *f_a, void *f_b, void *p, void *stream) {
    if (!b || !phi0 || !f_a || !f_b || !p) return api_fail(LBM_E_INVALID, "null argument");
    if (f_a == f_b) return api_fail(LBM_E_INVALID, "the two distribution buffers must differ");
    if (((uintptr_t)f_a | (uintptr_t)f_b | (uintptr_t)p) & 255) return api_fail(LBM_E_INVALID, "buffers must be 256-byte aligned");
    if (b->f[0] != f_a || b->f[1] != f_b || b->p != p) drop_graphs(b);
    b->f[0] = f_a; b->f[1] = f_b; b->p = p; b->phi0 = phi0;
    b->cur = 0; b->t = 0; b->bound = true;
    hipError_t e = batch_init_launch(b, (hipStream_t)stream);
    if (e != hipSuccess) return api_fail(LBM_E_HIP, hipGetErrorString(e));
    return LBM_OK;
}

int lbm_batch_set_shape(lbm_batch *b, int shape, unsigned grid, int remap) {
    if (!b || shape < 0 || shape >= kNumShapes + (b ? b->ntwo : 0))
        return api_fail(LBM_E_INVALID, "bad shape index");
    b->shape = shape;
    b->grid = grid;
    b->remap = remap ? 1 : 0;
    drop_graphs(b);
    return LBM_OK;
}

int lbm_batch_get_shape(const lbm_batch *b, int *shape, unsigned *grid, int *remap, int *wg, int *npt) {
    if (!b) return api_fail(LBM_E_INVALID, "null batch");
    if (shape) *shape = b->shape;
    if (grid) *grid = b->grid;
    if (remap) *remap = b->remap;
    if (is_two(b)) {
        const TwoShape t = two_shape(b, b->shape - kNumShapes);
        if (wg) *wg = 64 * t.waves;
        if (npt) *npt = -t.rows;    // minus the tile rows: two steps per launch
    } else {
        if (wg) *wg = kShapes[b->shape].wg;
        if (npt) *npt = kShapes[b->shape].npt;
    }
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int nsteps, void *stream) {
    if (!b) return api_fail(LBM_E_INVALID, "null batch");
    if (!b->bound) return api_fail(LBM_E_STATE, "lbm_batch_init has not been called");
    if (nsteps < 0) return api_fail(LBM_E_INVALID, "negative step count");
    hipStream_t st = (hipStream_t)stream;
    while (nsteps >= kBatchGraphSteps) {
        if (!b->gexec[b->cur]) {
            hipError_t e = make_graph(b, b->cur);
            if (e != hipSuccess) return api_fail(LBM_E_HIP, hipGetErrorString(e));
        }
        hipError_t e = hipGraphLaunch(b->gexec[b->cur], st);
        if (e != hipSuccess) return api_fail(LBM_E_HIP, hipGetErrorString(e));
        // 32 single sweeps or 16 two-step launches: an even number of buffer swaps
        b->t += kBatchGraphSteps;
        nsteps -= kBatchGraphSteps;
    }
    if (nsteps > 0) {
        int end = b->cur;
        hipError_t e = batch_advance(b, b->cur, nsteps, st, &end);
        if (e != hipSuccess) return api_fail(LBM_E_HIP, hipGetErrorString(e));
        b->cur = end;
        b->t += nsteps;
    }
    return LBM_OK;
}

int lbm_batch_get_phi(lbm_batch *b, double *phi, void *stream) {
    if (!b || !phi) return api_fail(LBM_E_INVALID, "null argument");
    if (!b->bound) return api_fail(LBM_E_STATE, "lbm_batch_init has not been called");
    const uint32_t nt = b->ntiles[0];
    const int tn = kShapes[0].wg * kShapes[0].npt;
    const uint32_t grid = std::min<uint32_t>(nt, 8192);
    hipStream_t st = (hipStream_t)stream;
    if (b->prec == 0)
        hipLaunchKernelGGL((k_batch_phi<double, double>), dim3(grid), dim3(256), 0, st, b->d_inst,
                           (const Coefs<double> *)b->d_coefs, b->d_tiles[0], nt, tn, (const double *)b->f[b->cur], phi);
    else if (b->prec == 1)
        hipLaunchKernelGGL((k_batch_phi<float, float>), dim3(grid), dim3(256), 0, st, b->d_inst,
                           (const Coefs<float> *)b->d_coefs, b->d_tiles[0], nt, tn, (const float *)b->f[b->cur], phi);
    else
        hipLaunchKernelGGL((k_batch_phi<_Float16, float>), dim3(grid), dim3(256), 0, st, b->d_inst,
                           (const Coefs<float> *)b->d_coefs, b->d_tiles[0], nt, tn, (const _Float16 *)b->f[b->cur], phi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return api_fail(LBM_E_HIP, hipGetErrorString(e));
    return LBM_OK;
}

int lbm_batch_tune(lbm_batch *b, int reps, int use_cache, void *stream, char *report, size_t report_len) {
    if (!b) return api_fail(LBM_E_INVALID, "null batch");
    if (!b->bound) return api_fail(LBM_E_STATE, "lbm_batch_init has not been called");
    if (reps < 1) reps = 1;
    hipStream_t st = (hipStream_t)stream;
    std::ostringstream rep;
    int shape = 0, remap = 1;
    uint32_t grid = 0;
    if (use_cache && cache_lookup(b->key, shape, grid, remap) && shape < kNumShapes + b->ntwo) {
        lbm_batch_set_shape(b, shape, grid, remap);
        rep << "cached " << b->key << " shape " << shape << " grid " << grid << " remap " << remap;
    } else {
        int cus = 256;
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t pr;
            if (hipGetDeviceProperties(&pr, dev) == hipSuccess) cus = pr.multiProcessorCount;
        }
        const uint32_t grids[] = {0u, (uint32_t)cus * 4, (uint32_t)cus * 8, (uint32_t)cus * 16};
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return api_fail(LBM_E_HIP, "hipEventCreate");
        float best = 1e30f;
        for (int s = 0; s < kNumShapes; ++s)
            for (uint32_t gr : grids)
                for (int rm = 0; rm < 2; ++rm) {
                    b->shape = s; b->grid = gr; b->remap = rm;
                    // sweeps read the current state and write the other buffer only
                    hipError_t e = batch_sweep_launch(b, b->f[b->cur], b->f[b->cur ^ 1], st, s);
                    if (e == hipSuccess) e = hipEventRecord(e0, st);
                    for (int r = 0; r < reps && e == hipSuccess; ++r)
                        e = batch_sweep_launch(b, b->f[b->cur], b->f[b->cur ^ 1], st, s);
                    if (e == hipSuccess) e = hipEventRecord(e1, st);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) {
                        (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
                        return api_fail(LBM_E_HIP, hipGetErrorString(e));
                    }
                    ms /= reps;
                    rep << "wg " << kShapes[s].wg << " npt " << kShapes[s].npt << " grid " << gr << " remap " << rm
                        << ": " << ms << " ms\n";
                    if (ms < best) { best = ms; shape = s; grid = gr; remap = rm; }
                }
        // two steps per launch: time per step
        for (int i = 0; i < b->ntwo; ++i)
            for (int rm = 0; rm < 2; ++rm) {
                b->shape = kNumShapes + i; b->grid = 0; b->remap = rm;
                hipError_t e = batch_sweep2_launch(b, b->f[b->cur], b->f[b->cur ^ 1], st);
                if (e == hipSuccess) e = hipEventRecord(e0, st);
                for (int r = 0; r < reps && e == hipSuccess; ++r)
                    e = batch_sweep2_launch(b, b->f[b->cur], b->f[b->cur ^ 1], st);
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
                    return api_fail(LBM_E_HIP, hipGetErrorString(e));
                }
                ms /= 2 * reps;
                const TwoShape t = two_shape(b, i);
                rep << "two steps per launch rows " << t.rows << " waves " << t.waves << " remap " << rm << ": "
                    << ms << " ms per step\n";
                if (ms < best) { best = ms; shape = kNumShapes + i; grid = 0; remap = rm; }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        lbm_batch_set_shape(b, shape, grid, remap);
        if (use_cache) cache_store(b->key, shape, grid, remap);
        rep << "chosen shape " << shape << " grid " << grid << " remap " << remap << " (" << best << " ms)";
        // the history buffer was overwritten by the trial sweeps: restore the state
        hipError_t e = batch_init_launch(b, st);
        if (e != hipSuccess) return api_fail(LBM_E_HIP, hipGetErrorString(e));
        b->t = 0;
        b->cur = 0;
    }
    if (report && report_len) {
        std::string s = rep.str();
        std::snprintf(report, report_len, "%s", s.c_str());
    }
    return LBM_OK;
}

}  // extern "C"
