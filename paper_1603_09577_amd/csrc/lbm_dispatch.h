// Template dispatch of the kernels of one lattice; included by exactly one
// translation unit per lattice (sweep_d2q9.hip, sweep_d3q19.hip) with
// LBM_Q defined.
#pragma once

#include "lbm_kernels.h"
#include "lbm_adjoint.h"

namespace lbm {

template <int Q, typename TS, typename TC>
hipError_t sweep_typed(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                       void *p, int *flag, hipStream_t st) {
    using TP = typename HistType<TS>::T;
    const auto *cf = (const Coefs<TC> *)coefs;
    const auto *fi = (const TS *)fin;
    auto *fo = (TS *)fout;
    auto *pp = (TP *)p;
    const dim3 grid((g.nblocks + g.chunk - 1) / g.chunk), block(kBlock);
    // Scheme B with a source (dm.sb) keeps no history: the Scheme-A flag is off
    const bool sa = dm.src && !dm.sb;
    // every polynomial of degree <= 2: 3-term kernels (32-bit offsets)
    {
        if (dm.eqr && dm.deg3 && dm.o32) {
            if (dm.sb) {
                // Scheme B with R(phi): 3-term kernels only (no row-wave variant)
                const int cb = (dm.kvar ? 2 : 0) | (dm.wall ? 1 : 0) | (dm.nt ? 8 : 0);
#define LBM_SWEEP3B(K, W, NT)                                                                         \
    case (NT * 8 + K * 2 + W):                                                                        \
        hipLaunchKernelGGL((k_sweep<Q, TS, TC, true, false, K, W, 3, NT, true, false, true>), grid, block, 0, st, g, \
                           cf, fi, fo, pp, flag);                                                     \
        break;
                switch (cb) {
                    LBM_SWEEP3B(0, 0, 0) LBM_SWEEP3B(0, 1, 0) LBM_SWEEP3B(1, 0, 0) LBM_SWEEP3B(1, 1, 0)
                    LBM_SWEEP3B(0, 0, 1) LBM_SWEEP3B(0, 1, 1) LBM_SWEEP3B(1, 0, 1) LBM_SWEEP3B(1, 1, 1)
                    default: return hipErrorInvalidValue;
                }
#undef LBM_SWEEP3B
                return hipGetLastError();
            }
            const int c3 = (sa ? 4 : 0) | (dm.kvar ? 2 : 0) | (dm.wall ? 1 : 0) | (dm.nt ? 8 : 0);
            if constexpr (Q == 9) {
                if (dm.wall && g.nx % 64 == 0) {
                    // every wave within one row: the row-wave gathers (k_sweep
                    // RW).  With walls only: there they measured 2.9% faster on
                    // 1024^2 FP32; on periodic grids 1.8% slower
#define LBM_SWEEP3R(S, K, NT)                                                                         \
    case (NT * 8 + S * 4 + K * 2 + 1):                                                                \
        hipLaunchKernelGGL((k_sweep<Q, TS, TC, true, S, K, true, 3, NT, true, true>), grid, block, 0, st, g, cf, fi, fo, \
                           pp, flag);                                                                 \
        break;
                    switch (c3) {
                        LBM_SWEEP3R(0, 0, 0) LBM_SWEEP3R(0, 1, 0) LBM_SWEEP3R(1, 0, 0) LBM_SWEEP3R(1, 1, 0)
                        LBM_SWEEP3R(0, 0, 1) LBM_SWEEP3R(0, 1, 1) LBM_SWEEP3R(1, 0, 1) LBM_SWEEP3R(1, 1, 1)
                        default: return hipErrorInvalidValue;
                    }
#undef LBM_SWEEP3R
                    return hipGetLastError();
                }
            }
#define LBM_SWEEP3(S, K, W, NT)                                                                       \
    case (NT * 8 + S * 4 + K * 2 + W):                                                                \
        hipLaunchKernelGGL((k_sweep<Q, TS, TC, true, S, K, W, 3, NT, true>), grid, block, 0, st, g, cf, fi, fo, pp, flag); \
        break;
            switch (c3) {
                LBM_SWEEP3(0, 0, 0, 0) LBM_SWEEP3(0, 0, 1, 0) LBM_SWEEP3(0, 1, 0, 0) LBM_SWEEP3(0, 1, 1, 0)
                LBM_SWEEP3(1, 0, 0, 0) LBM_SWEEP3(1, 0, 1, 0) LBM_SWEEP3(1, 1, 0, 0) LBM_SWEEP3(1, 1, 1, 0)
                LBM_SWEEP3(0, 0, 0, 1) LBM_SWEEP3(0, 0, 1, 1) LBM_SWEEP3(0, 1, 0, 1) LBM_SWEEP3(0, 1, 1, 1)
                LBM_SWEEP3(1, 0, 0, 1) LBM_SWEEP3(1, 0, 1, 1) LBM_SWEEP3(1, 1, 0, 1) LBM_SWEEP3(1, 1, 1, 1)
                default: return hipErrorInvalidValue;
            }
#undef LBM_SWEEP3
            return hipGetLastError();
        }
    }
    // Scheme B sources elsewhere run k_sweep_gen (the host routes them there)
    if (dm.sb) return hipErrorInvalidValue;
    // short polynomials (all degrees <= 3) get the branch-free 4-term kernels
    // non-temporal accesses: equal-rate short-polynomial kernels only
    const int code = (dm.eqr ? 8 : 0) | (dm.src ? 4 : 0) | (dm.kvar ? 2 : 0) | (dm.wall ? 1 : 0) |
                     ((dm.eqr && dm.lowdeg) ? 16 : 0) | ((dm.eqr && dm.lowdeg && dm.nt) ? 32 : 0);
#define LBM_SWEEP_X(E, S, K, W, NP, NT, TAG)                                                          \
    case (TAG + E * 8 + S * 4 + K * 2 + W):                                                           \
        hipLaunchKernelGGL((k_sweep<Q, TS, TC, E, S, K, W, NP, NT>), grid, block, 0, st, g, cf, fi, fo, pp, flag); \
        break;
#define LBM_SWEEP_NP(E, S, K, W, NP, TAG) LBM_SWEEP_X(E, S, K, W, NP, false, TAG)
#define LBM_SWEEP(E, S, K, W) LBM_SWEEP_NP(E, S, K, W, 9, 0)
    switch (code) {
        LBM_SWEEP_X(1, 0, 0, 0, 4, true, 48) LBM_SWEEP_X(1, 0, 0, 1, 4, true, 48)
        LBM_SWEEP_X(1, 0, 1, 0, 4, true, 48) LBM_SWEEP_X(1, 0, 1, 1, 4, true, 48)
        LBM_SWEEP_X(1, 1, 0, 0, 4, true, 48) LBM_SWEEP_X(1, 1, 0, 1, 4, true, 48)
        LBM_SWEEP_X(1, 1, 1, 0, 4, true, 48) LBM_SWEEP_X(1, 1, 1, 1, 4, true, 48)
        LBM_SWEEP_NP(1, 0, 0, 0, 4, 16) LBM_SWEEP_NP(1, 0, 0, 1, 4, 16)
        LBM_SWEEP_NP(1, 0, 1, 0, 4, 16) LBM_SWEEP_NP(1, 0, 1, 1, 4, 16)
        LBM_SWEEP_NP(1, 1, 0, 0, 4, 16) LBM_SWEEP_NP(1, 1, 0, 1, 4, 16)
        LBM_SWEEP_NP(1, 1, 1, 0, 4, 16) LBM_SWEEP_NP(1, 1, 1, 1, 4, 16)
        LBM_SWEEP(0, 0, 0, 0) LBM_SWEEP(0, 0, 0, 1) LBM_SWEEP(0, 0, 1, 0) LBM_SWEEP(0, 0, 1, 1)
        LBM_SWEEP(0, 1, 0, 0) LBM_SWEEP(0, 1, 0, 1) LBM_SWEEP(0, 1, 1, 0) LBM_SWEEP(0, 1, 1, 1)
        LBM_SWEEP(1, 0, 0, 0) LBM_SWEEP(1, 0, 0, 1) LBM_SWEEP(1, 0, 1, 0) LBM_SWEEP(1, 0, 1, 1)
        LBM_SWEEP(1, 1, 0, 0) LBM_SWEEP(1, 1, 0, 1) LBM_SWEEP(1, 1, 1, 0) LBM_SWEEP(1, 1, 1, 1)
        default: return hipErrorInvalidValue;
    }
#undef LBM_SWEEP
#undef LBM_SWEEP_NP
#undef LBM_SWEEP_X
    return hipGetLastError();
}

// Default tile height of a two-step pass by storage size (the LDS tile is
// 9 x (TH + 2) x 64 values; 40 KB with 4-byte and 8-byte storage).
template <typename TS>
constexpr int two_step_rows() { return sizeof(TS) == 8 ? 6 : 14; }

template <typename TS, typename TC, int TH, int NW>
hipError_t sweep2_shape(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                        const void *pin, void *pout, int *flag, hipStream_t st) {
    using TP = typename HistType<TS>::T;
    const auto *cf = (const Coefs<TC> *)coefs;
    const uint32_t tiles_x = (g.nx + 61) / 62, tiles_y = (g.ny + TH - 1) / TH;
    const dim3 grid(tiles_x * tiles_y), block(64 * NW);
    const TS *fi = (const TS *)fin;
    TS *fo = (TS *)fout;
    const TP *pi = (const TP *)pin;
    TP *po = (TP *)pout;
    if (!dm.eqr) {
        // unequal non-flux rates (moment-space collision): 3-term polynomials,
        // the default tile shape; any source, periodic or walls on y
        if constexpr (TH == two_step_rows<TS>() && NW == kBlock / 64) {
            if (!dm.deg3) return hipErrorInvalidValue;
            const int cm = (dm.sb ? 8 : (dm.src ? 4 : 0)) | (dm.kvar ? 2 : 0) | (dm.wall ? 1 : 0);
#define LBM_SW2M(S, B, K, W)                                                                         \
    case ((B ? 8 : S * 4) + K * 2 + W):                                                              \
        hipLaunchKernelGGL((k_sweep2<TS, TC, S, K, 3, TH, NW, B, W, false>), grid, block, 0, st, g, cf, fi, fo, pi, \
                           po, tiles_x, flag);                                                       \
        break;
            switch (cm) {
                LBM_SW2M(false, false, false, false) LBM_SW2M(false, false, false, true)
                LBM_SW2M(false, false, true, false) LBM_SW2M(false, false, true, true)
                LBM_SW2M(true, false, false, false) LBM_SW2M(true, false, false, true)
                LBM_SW2M(true, false, true, false) LBM_SW2M(true, false, true, true)
                LBM_SW2M(false, true, false, false) LBM_SW2M(false, true, false, true)
                LBM_SW2M(false, true, true, false) LBM_SW2M(false, true, true, true)
                default: return hipErrorInvalidValue;
            }
#undef LBM_SW2M
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (dm.wall) {
        // anti-bounce-back walls on y: 3-term kernels; no source, Scheme A
        // (history) or Scheme B
        if (!dm.deg3) return hipErrorInvalidValue;
        const int cw = (dm.sb ? 4 : (dm.src ? 2 : 0)) | (dm.kvar ? 1 : 0);
#define LBM_SW2W(S, K, B)                                                                            \
    case ((B ? 4 : S * 2) + K):                                                                      \
        hipLaunchKernelGGL((k_sweep2<TS, TC, S, K, 3, TH, NW, B, true>), grid, block, 0, st, g, cf, fi, fo, pi, \
                           po, tiles_x, flag);                                                       \
        break;
        switch (cw) {
            LBM_SW2W(false, false, false) LBM_SW2W(false, true, false) LBM_SW2W(true, false, false)
            LBM_SW2W(true, true, false) LBM_SW2W(false, false, true) LBM_SW2W(false, true, true)
            default: return hipErrorInvalidValue;
        }
#undef LBM_SW2W
        return hipGetLastError();
    }
    if (dm.sb) {
        // Scheme B with R(phi), 3-term polynomials: no history
        if (!dm.deg3) return hipErrorInvalidValue;
        if (dm.kvar)
            hipLaunchKernelGGL((k_sweep2<TS, TC, false, true, 3, TH, NW, true>), grid, block, 0, st, g, cf, fi, fo,
                               pi, po, tiles_x, flag);
        else
            hipLaunchKernelGGL((k_sweep2<TS, TC, false, false, 3, TH, NW, true>), grid, block, 0, st, g, cf, fi, fo,
                               pi, po, tiles_x, flag);
        return hipGetLastError();
    }
    const int code = (dm.src ? 4 : 0) | (dm.kvar ? 2 : 0) | (dm.deg3 ? 8 : (dm.lowdeg ? 1 : 0));
#define LBM_SW2(S, K, NP, TAG)                                                                       \
    case (S * 4 + K * 2 + TAG):                                                                      \
        hipLaunchKernelGGL((k_sweep2<TS, TC, S, K, NP, TH, NW>), grid, block, 0, st, g, cf, fi, fo, pi, po, \
                           tiles_x, flag);                                                           \
        break;
    if constexpr (TH == two_step_rows<TS>() && NW == kBlock / 64) {
        switch (code) {
            LBM_SW2(0, 0, 9, 0) LBM_SW2(0, 1, 9, 0) LBM_SW2(1, 0, 9, 0) LBM_SW2(1, 1, 9, 0)
            LBM_SW2(0, 0, 4, 1) LBM_SW2(0, 1, 4, 1) LBM_SW2(1, 0, 4, 1) LBM_SW2(1, 1, 4, 1)
            LBM_SW2(0, 0, 3, 8) LBM_SW2(0, 1, 3, 8) LBM_SW2(1, 0, 3, 8) LBM_SW2(1, 1, 3, 8)
            default: return hipErrorInvalidValue;
        }
    } else {
        // the other tile shapes: 3-term kernels only
        switch (code) {
            LBM_SW2(0, 0, 3, 8) LBM_SW2(0, 1, 3, 8) LBM_SW2(1, 0, 3, 8) LBM_SW2(1, 1, 3, 8)
            default: return hipErrorInvalidValue;
        }
    }
#undef LBM_SW2
    return hipGetLastError();
}

// Tile shapes of a two-step pass, (rows, waves per workgroup).  Shape 0 is the
// default for the storage size; the others (3-term polynomials only) trade
// halo work against waves per CU: phase 1 gives each wave (rows + 2) / waves
// rows, and fewer rows per wave need fewer registers.
template <typename TS>
constexpr int two_step_shape_count() { return sizeof(TS) == 8 ? 3 : 4; }

template <typename TS>
constexpr bool two_step_shape(int id, int &rows, int &waves) {
    constexpr int r8[3][2] = {{6, 4}, {6, 8}, {14, 16}};
    constexpr int r4[4][2] = {{14, 4}, {14, 8}, {10, 6}, {6, 4}};
    if (id < 0 || id >= two_step_shape_count<TS>()) return false;
    rows = sizeof(TS) == 8 ? r8[id][0] : r4[id][0];
    waves = sizeof(TS) == 8 ? r8[id][1] : r4[id][1];
    return true;
}

template <int Q, typename TS, typename TC>
hipError_t sweep2_typed(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                        const void *pin, void *pout, int *flag, int shape, hipStream_t st) {
    if (Q != 9 || ((dm.wall || !dm.eqr) && !dm.deg3)) return hipErrorNotSupported;
    if (!dm.eqr && shape != 0) return hipErrorInvalidValue;   // moment-space collision: the default shape
    if (shape < 0 || shape >= two_step_shape_count<TS>() || (shape > 0 && !dm.deg3)) return hipErrorInvalidValue;
    if constexpr (sizeof(TS) == 8) {
        if (shape == 1) return sweep2_shape<TS, TC, 6, 8>(dm, g, coefs, fin, fout, pin, pout, flag, st);
        if (shape == 2) return sweep2_shape<TS, TC, 14, 16>(dm, g, coefs, fin, fout, pin, pout, flag, st);
        return sweep2_shape<TS, TC, 6, 4>(dm, g, coefs, fin, fout, pin, pout, flag, st);
    } else {
        if (shape == 1) return sweep2_shape<TS, TC, 14, 8>(dm, g, coefs, fin, fout, pin, pout, flag, st);
        if (shape == 2) return sweep2_shape<TS, TC, 10, 6>(dm, g, coefs, fin, fout, pin, pout, flag, st);
        if (shape == 3) return sweep2_shape<TS, TC, 6, 4>(dm, g, coefs, fin, fout, pin, pout, flag, st);
        return sweep2_shape<TS, TC, 14, 4>(dm, g, coefs, fin, fout, pin, pout, flag, st);
    }
}

// Tile shapes of the D3Q19 two-step pass, (rows TY, waves per workgroup), one
// phase-1 row per wave.  The LDS ring holds 38 planes of 64 x (TY + 2)
// values: FP32 156 KB at TY = 14 (one workgroup of 16 waves per CU), 78 KB at
// TY = 6 (two of 8 waves), 39 KB at TY = 2; FP64 156 KB at TY = 6, 78 KB at
// TY = 2.  Shape 0 measured fastest on 256^3 with walls.
template <typename TS>
constexpr int two_step3_shape_count() { return sizeof(TS) == 8 ? 2 : 3; }

template <typename TS>
constexpr bool two_step3_shape(int id, int &rows, int &waves) {
    constexpr int r8[2][2] = {{6, 8}, {2, 4}};
    constexpr int r4[3][2] = {{14, 16}, {6, 8}, {2, 4}};
    if (id < 0 || id >= two_step3_shape_count<TS>()) return false;
    rows = sizeof(TS) == 8 ? r8[id][0] : r4[id][0];
    waves = sizeof(TS) == 8 ? r8[id][1] : r4[id][1];
    return true;
}

// occ != nullptr: launch nothing and report the kernel's resident workgroups
// per CU instead (the z-chunk choice needs it).
template <typename TS, typename TC, int TY, int NW>
hipError_t sweep2_3d_shape(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                           const void *pin, void *pout, int *flag, uint32_t zc, hipStream_t st, int *occ) {
    using TP = typename HistType<TS>::T;
    const auto *cf = (const Coefs<TC> *)coefs;
    const uint32_t tiles_x = (g.nx + 61) / 62, tiles_y = (g.ny + TY - 1) / TY, tiles_z = (g.nz + zc - 1) / zc;
    const dim3 grid(tiles_x * tiles_y * tiles_z), block(64 * NW);
    const TS *fi = (const TS *)fin;
    TS *fo = (TS *)fout;
    const TP *pi = (const TP *)pin;
    TP *po = (TP *)pout;
    // source: none, Scheme B (no history) or Scheme A (history pin -> pout)
    const int sc = dm.sb ? 1 : (dm.src ? 2 : 0);
    const int code = sc * 4 + (dm.kvar ? 2 : 0) + (dm.wall ? 1 : 0);
    if (!dm.eqr) {
        // unequal non-flux rates (moment-space collision): the default shape
        if constexpr ((sizeof(TS) == 8 && TY == 6 && NW == 8) || (sizeof(TS) != 8 && TY == 14 && NW == 16)) {
#define LBM_SW3M(S, K, W)                                                                            \
    case (S * 4 + K * 2 + W):                                                                        \
        if (occ)                                                                                     \
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(                                     \
                occ, k_sweep2_3d<TS, TC, K, W, 3, TY, NW, S == 1, S == 2, false>, 64 * NW, 0);       \
        hipLaunchKernelGGL((k_sweep2_3d<TS, TC, K, W, 3, TY, NW, S == 1, S == 2, false>), grid, block, 0, st, g, cf, \
                           fi, fo, pi, po, tiles_x, tiles_y, zc, flag);                              \
        break;
            switch (code) {
                LBM_SW3M(0, 0, 0) LBM_SW3M(0, 0, 1) LBM_SW3M(0, 1, 0) LBM_SW3M(0, 1, 1)
                LBM_SW3M(1, 0, 0) LBM_SW3M(1, 0, 1) LBM_SW3M(1, 1, 0) LBM_SW3M(1, 1, 1)
                LBM_SW3M(2, 0, 0) LBM_SW3M(2, 0, 1) LBM_SW3M(2, 1, 0) LBM_SW3M(2, 1, 1)
                default: return hipErrorInvalidValue;
            }
#undef LBM_SW3M
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
#define LBM_SW3(S, K, W)                                                                             \
    case (S * 4 + K * 2 + W):                                                                        \
        if (occ)                                                                                     \
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(                                     \
                occ, k_sweep2_3d<TS, TC, K, W, 3, TY, NW, S == 1, S == 2>, 64 * NW, 0);              \
        hipLaunchKernelGGL((k_sweep2_3d<TS, TC, K, W, 3, TY, NW, S == 1, S == 2>), grid, block, 0, st, g, cf, fi, \
                           fo, pi, po, tiles_x, tiles_y, zc, flag);                                  \
        break;
    switch (code) {
        LBM_SW3(0, 0, 0) LBM_SW3(0, 0, 1) LBM_SW3(0, 1, 0) LBM_SW3(0, 1, 1)
        LBM_SW3(1, 0, 0) LBM_SW3(1, 0, 1) LBM_SW3(1, 1, 0) LBM_SW3(1, 1, 1)
        LBM_SW3(2, 0, 0) LBM_SW3(2, 0, 1) LBM_SW3(2, 1, 0) LBM_SW3(2, 1, 1)
        default: return hipErrorInvalidValue;
    }
#undef LBM_SW3
    return hipGetLastError();
}

// D3Q19 two steps per pass: equal non-flux rates, 3-term polynomials, no source
// (no phi history), walls on z or periodic; chunks of zc planes.
template <int Q, typename TS, typename TC>
hipError_t sweep2_3d_typed(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                           const void *pin, void *pout, int *flag, int shape, uint32_t zc, hipStream_t st,
                           int *occ) {
    if constexpr (Q == 19) {
        if (!dm.deg3 || !dm.o32 || zc < 1) return hipErrorNotSupported;
        if (!dm.eqr && shape != 0) return hipErrorInvalidValue;   // moment-space collision: the default shape
        // a Scheme-A source reads the history pin and writes pout (distinct)
        if (!occ && dm.src && !dm.sb && (!pin || !pout || pin == pout)) return hipErrorInvalidValue;
        if constexpr (sizeof(TS) == 8) {
            if (shape == 0) return sweep2_3d_shape<TS, TC, 6, 8>(dm, g, coefs, fin, fout, pin, pout, flag, zc, st, occ);
            if (shape == 1) return sweep2_3d_shape<TS, TC, 2, 4>(dm, g, coefs, fin, fout, pin, pout, flag, zc, st, occ);
        } else {
            if (shape == 0) return sweep2_3d_shape<TS, TC, 14, 16>(dm, g, coefs, fin, fout, pin, pout, flag, zc, st, occ);
            if (shape == 1) return sweep2_3d_shape<TS, TC, 6, 8>(dm, g, coefs, fin, fout, pin, pout, flag, zc, st, occ);
            if (shape == 2) return sweep2_3d_shape<TS, TC, 2, 4>(dm, g, coefs, fin, fout, pin, pout, flag, zc, st, occ);
        }
        return hipErrorInvalidValue;
    } else {
        return hipErrorNotSupported;
    }
}

// Scheme B and/or per-node fields: the general kernel (any polynomial length).
template <int Q, typename TS, typename TC>
hipError_t sweep_gen_typed(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                           void *p, int *flag, const double *kfield, const double *rfield, bool remark3,
                           hipStream_t st) {
    using TP = typename HistType<TS>::T;
    const auto *cf = (const Coefs<TC> *)coefs;
    const auto *fi = (const TS *)fin;
    auto *fo = (TS *)fout;
    auto *pp = (TP *)p;
    const dim3 grid(g.nblocks), block(kBlock);
    const int code = (dm.eqr ? 4 : 0) | (dm.wall ? 2 : 0) | (dm.sb ? 1 : 0);
#define LBM_GEN(E, W, B)                                                                            \
    case (E * 4 + W * 2 + B):                                                                       \
        hipLaunchKernelGGL((k_sweep_gen<Q, TS, TC, E, W, B>), grid, block, 0, st, g, cf, fi, fo, pp, flag, \
                           kfield, rfield, remark3 ? 1 : 0);                                        \
        break;
    switch (code) {
        LBM_GEN(0, 0, 0) LBM_GEN(0, 0, 1) LBM_GEN(0, 1, 0) LBM_GEN(0, 1, 1)
        LBM_GEN(1, 0, 0) LBM_GEN(1, 0, 1) LBM_GEN(1, 1, 0) LBM_GEN(1, 1, 1)
        default: return hipErrorInvalidValue;
    }
#undef LBM_GEN
    return hipGetLastError();
}

template <int Q, typename TS, typename TC>
hipError_t init_typed(const Dims &dm, const Geom &g, const void *coefs, const double *phi0, void *f,
                      void *p, const double *rfield, hipStream_t st) {
    using TP = typename HistType<TS>::T;
    const auto *cf = (const Coefs<TC> *)coefs;
    const dim3 grid(g.nblocks), block(kBlock);
    const bool low = dm.lowdeg && !dm.sb;
#define LBM_INIT(W, NP, B) \
    hipLaunchKernelGGL((k_init<Q, TS, TC, W, NP, B>), grid, block, 0, st, g, cf, phi0, (TS *)f, (TP *)p, rfield)
    if (dm.sb) {
        if (dm.wall) LBM_INIT(true, 9, true);
        else LBM_INIT(false, 9, true);
    } else if (dm.wall && low) LBM_INIT(true, 4, false);
    else if (dm.wall) LBM_INIT(true, 9, false);
    else if (low) LBM_INIT(false, 4, false);
    else LBM_INIT(false, 9, false);
#undef LBM_INIT
    return hipGetLastError();
}

template <int Q, typename TS, typename TC>
hipError_t phi_typed(const Dims &dm, const Geom &g, const void *coefs, const void *f, double *phi,
                     const double *rfield, hipStream_t st) {
    const auto *cf = (const Coefs<TC> *)coefs;
    const dim3 grid(g.nblocks), block(kBlock);
    const TS *fs = (const TS *)f;
    if (dm.wall && dm.sb)
        hipLaunchKernelGGL((k_phi<Q, TS, TC, true, true>), grid, block, 0, st, g, cf, fs, phi, rfield);
    else if (dm.wall)
        hipLaunchKernelGGL((k_phi<Q, TS, TC, true, false>), grid, block, 0, st, g, cf, fs, phi, rfield);
    else if (dm.sb)
        hipLaunchKernelGGL((k_phi<Q, TS, TC, false, true>), grid, block, 0, st, g, cf, fs, phi, rfield);
    else
        hipLaunchKernelGGL((k_phi<Q, TS, TC, false, false>), grid, block, 0, st, g, cf, fs, phi, rfield);
    return hipGetLastError();
}

// Reductions over phi formed from the state (k_phi_reduce), then the fold.
template <int Q, typename TS, typename TC>
hipError_t phi_reduce_typed(const Dims &dm, const Geom &g, const void *coefs, const void *f, const double *ref,
                            const double *rfield, double *part, int nparts, double *out, hipStream_t st) {
    const auto *cf = (const Coefs<TC> *)coefs;
    const dim3 grid(nparts), block(kBlock);
    const TS *fs = (const TS *)f;
    if (dm.wall && dm.sb)
        hipLaunchKernelGGL((k_phi_reduce<Q, TS, TC, true, true>), grid, block, 0, st, g, cf, fs, ref, rfield, part);
    else if (dm.wall)
        hipLaunchKernelGGL((k_phi_reduce<Q, TS, TC, true, false>), grid, block, 0, st, g, cf, fs, ref, rfield, part);
    else if (dm.sb)
        hipLaunchKernelGGL((k_phi_reduce<Q, TS, TC, false, true>), grid, block, 0, st, g, cf, fs, ref, rfield, part);
    else
        hipLaunchKernelGGL((k_phi_reduce<Q, TS, TC, false, false>), grid, block, 0, st, g, cf, fs, ref, rfield, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_final(part, nparts, out, st);
}

template <int Q, typename TS, typename TC>
hipError_t adjoint_typed(const Dims &dm, const Geom &g, const void *coefs, const void *f, const void *p,
                         const void *psi_next, const double *pi_next, void *psi_out, double *pi_out,
                         double *gk_part, hipStream_t st) {
    using TP = typename HistType<TS>::T;
    const auto *cf = (const Coefs<TC> *)coefs;
    const auto *fs = (const TS *)f;
    const auto *ps = (const TP *)p;
    const auto *pn = (const TC *)psi_next;
    auto *po = (TC *)psi_out;
    const dim3 grid(g.nblocks), block(kBlock);
    {
        if (dm.eqr && dm.deg3 && dm.o32) {
            // streaming accesses when the state exceeds the Infinity Cache (dm.nt)
            const int c3 = (dm.nt ? 8 : 0) | (dm.src ? 4 : 0) | (dm.kvar ? 2 : 0) | (dm.wall ? 1 : 0);
#define LBM_ADJ3(S, K, W, NT)                                                                           \
    case (NT * 8 + S * 4 + K * 2 + W):                                                                  \
        hipLaunchKernelGGL((k_adjoint<Q, TS, TC, true, S, K, W, 3, true, NT>), grid, block, 0, st, g, cf, fs, ps, \
                           pn, pi_next, po, pi_out, gk_part);                                           \
        break;
            if constexpr (Q == 9) {
                if (sizeof(TS) == 8 && !dm.nt && g.nx % 64 == 0) {
                    // every wave within one row: the row-wave loads (k_adjoint
                    // RW).  FP64 only: in FP32 they measured slower on the
                    // 512^2 grid (6.35 against 6.27 us per sweep), in FP64
                    // faster (10.3 against 10.4-10.8)
#define LBM_ADJ3R(S, K, W)                                                                              \
    case (S * 4 + K * 2 + W):                                                                           \
        hipLaunchKernelGGL((k_adjoint<Q, TS, TC, true, S, K, W, 3, true, false, true>), grid, block, 0, st, g, cf, \
                           fs, ps, pn, pi_next, po, pi_out, gk_part);                                   \
        break;
                    switch (c3) {
                        LBM_ADJ3R(0, 0, 0) LBM_ADJ3R(0, 0, 1) LBM_ADJ3R(0, 1, 0) LBM_ADJ3R(0, 1, 1)
                        LBM_ADJ3R(1, 0, 0) LBM_ADJ3R(1, 0, 1) LBM_ADJ3R(1, 1, 0) LBM_ADJ3R(1, 1, 1)
                        default: return hipErrorInvalidValue;
                    }
#undef LBM_ADJ3R
                    return hipGetLastError();
                }
            }
            switch (c3) {
                LBM_ADJ3(0, 0, 0, 0) LBM_ADJ3(0, 0, 1, 0) LBM_ADJ3(0, 1, 0, 0) LBM_ADJ3(0, 1, 1, 0)
                LBM_ADJ3(1, 0, 0, 0) LBM_ADJ3(1, 0, 1, 0) LBM_ADJ3(1, 1, 0, 0) LBM_ADJ3(1, 1, 1, 0)
                LBM_ADJ3(0, 0, 0, 1) LBM_ADJ3(0, 0, 1, 1) LBM_ADJ3(0, 1, 0, 1) LBM_ADJ3(0, 1, 1, 1)
                LBM_ADJ3(1, 0, 0, 1) LBM_ADJ3(1, 0, 1, 1) LBM_ADJ3(1, 1, 0, 1) LBM_ADJ3(1, 1, 1, 1)
                default: return hipErrorInvalidValue;
            }
#undef LBM_ADJ3
            return hipGetLastError();
        }
    }
    const int code = (dm.eqr ? 8 : 0) | (dm.src ? 4 : 0) | (dm.kvar ? 2 : 0) | (dm.wall ? 1 : 0) |
                     ((dm.eqr && dm.lowdeg) ? 16 : 0);
#define LBM_ADJ_NP(E, S, K, W, NP, TAG)                                                                 \
    case (TAG + E * 8 + S * 4 + K * 2 + W):                                                             \
        hipLaunchKernelGGL((k_adjoint<Q, TS, TC, E, S, K, W, NP>), grid, block, 0, st, g, cf, fs, ps, pn, \
                           pi_next, po, pi_out, gk_part);                                               \
        break;
#define LBM_ADJ(E, S, K, W) LBM_ADJ_NP(E, S, K, W, 9, 0)
    switch (code) {
        LBM_ADJ_NP(1, 0, 0, 0, 4, 16) LBM_ADJ_NP(1, 0, 0, 1, 4, 16)
        LBM_ADJ_NP(1, 0, 1, 0, 4, 16) LBM_ADJ_NP(1, 0, 1, 1, 4, 16)
        LBM_ADJ_NP(1, 1, 0, 0, 4, 16) LBM_ADJ_NP(1, 1, 0, 1, 4, 16)
        LBM_ADJ_NP(1, 1, 1, 0, 4, 16) LBM_ADJ_NP(1, 1, 1, 1, 4, 16)
        LBM_ADJ(0, 0, 0, 0) LBM_ADJ(0, 0, 0, 1) LBM_ADJ(0, 0, 1, 0) LBM_ADJ(0, 0, 1, 1)
        LBM_ADJ(0, 1, 0, 0) LBM_ADJ(0, 1, 0, 1) LBM_ADJ(0, 1, 1, 0) LBM_ADJ(0, 1, 1, 1)
        LBM_ADJ(1, 0, 0, 0) LBM_ADJ(1, 0, 0, 1) LBM_ADJ(1, 0, 1, 0) LBM_ADJ(1, 0, 1, 1)
        LBM_ADJ(1, 1, 0, 0) LBM_ADJ(1, 1, 0, 1) LBM_ADJ(1, 1, 1, 0) LBM_ADJ(1, 1, 1, 1)
        default: return hipErrorInvalidValue;
    }
#undef LBM_ADJ
#undef LBM_ADJ_NP
    return hipGetLastError();
}

// Two reversed sweeps per pass (D2Q9, periodic, equal rates): sweep s with
// (f1, p1), then sweep s - 1 with (f0, p0); TH tile rows.
// occ != nullptr: launch nothing and report the kernel's resident workgroups
// per CU instead.
template <typename TS, typename TC, int TH, int NW>
hipError_t adjoint2_rows(const Dims &dm, const Geom &g, const void *coefs, const void *f1, const void *p1,
                         const void *f0, const void *p0, const void *psi_next, const double *pi_next,
                         void *psi_out, double *pi_out, double *gk_part, hipStream_t st, int *occ) {
    using TP = typename HistType<TS>::T;
    const auto *cf = (const Coefs<TC> *)coefs;
    const uint32_t tiles_x = (g.nx + 61) / 62, tiles_y = (g.ny + TH - 1) / TH;
    const dim3 grid(tiles_x * tiles_y), block(NW * 64);
    const auto *a1 = (const TS *)f1, *a0 = (const TS *)f0;
    const auto *q1 = (const TP *)p1, *q0 = (const TP *)p0;
    const auto *pn = (const TC *)psi_next;
    auto *po = (TC *)psi_out;
    const int code = (dm.src ? 4 : 0) | (dm.kvar ? 2 : 0) | (dm.deg3 ? 8 : (dm.lowdeg ? 1 : 0));
#define LBM_ADJ2(S, K, NP, TAG)                                                                      \
    case (S * 4 + K * 2 + TAG):                                                                      \
        if (occ)                                                                                     \
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_adjoint2<TS, TC, S, K, NP, TH, NW>, \
                                                                NW * 64, 0);                         \
        hipLaunchKernelGGL((k_adjoint2<TS, TC, S, K, NP, TH, NW>), grid, block, 0, st, g, cf, a1, q1, a0, q0, pn, \
                           pi_next, po, pi_out, gk_part, tiles_x);                                   \
        break;
    switch (code) {
        LBM_ADJ2(0, 0, 9, 0) LBM_ADJ2(0, 1, 9, 0) LBM_ADJ2(1, 0, 9, 0) LBM_ADJ2(1, 1, 9, 0)
        LBM_ADJ2(0, 0, 4, 1) LBM_ADJ2(0, 1, 4, 1) LBM_ADJ2(1, 0, 4, 1) LBM_ADJ2(1, 1, 4, 1)
        LBM_ADJ2(0, 0, 3, 8) LBM_ADJ2(0, 1, 3, 8) LBM_ADJ2(1, 0, 3, 8) LBM_ADJ2(1, 1, 3, 8)
        default: return hipErrorInvalidValue;
    }
#undef LBM_ADJ2
    return hipGetLastError();
}

// Tile shapes of the two-sweep adjoint, (rows, waves per workgroup): 6 x 4,
// 10 x 4 and 10 x 12 (the host picks one per context, lbm_api.hip).
constexpr int kAdjShapes = 3;
constexpr int kAdjShape[kAdjShapes][2] = {{6, 4}, {10, 4}, {10, 12}};

template <int Q, typename TS, typename TC>
hipError_t adjoint2_typed(const Dims &dm, const Geom &g, const void *coefs, const void *f1, const void *p1,
                          const void *f0, const void *p0, const void *psi_next, const double *pi_next,
                          void *psi_out, double *pi_out, double *gk_part, hipStream_t st, int shape, int *occ) {
    static_assert(Q == 9, "two reversed sweeps per pass are D2Q9 only");
    if (dm.wall || !dm.eqr) return hipErrorNotSupported;   // periodic, equal-rate tiles only
#define LBM_ADJ2S(ID, TH, NW)                                                                        \
    if (shape == ID)                                                                                 \
        return adjoint2_rows<TS, TC, TH, NW>(dm, g, coefs, f1, p1, f0, p0, psi_next, pi_next, psi_out, pi_out, \
                                             gk_part, st, occ);
    LBM_ADJ2S(0, 6, 4) LBM_ADJ2S(1, 10, 4) LBM_ADJ2S(2, 10, 12)
#undef LBM_ADJ2S
    return hipErrorInvalidValue;
}

template <int Q, typename TS, typename TC>
hipError_t adjoint_init_typed(const Dims &dm, const Geom &g, const void *coefs, const double *phi0,
                              const void *psi0, const double *pi0, double *out, hipStream_t st) {
    if (dm.lowdeg)
        hipLaunchKernelGGL((k_adjoint_init<Q, TC, 4>), dim3(g.nblocks), dim3(kBlock), 0, st, g,
                           (const Coefs<TC> *)coefs, phi0, (const TC *)psi0, pi0, out);
    else
        hipLaunchKernelGGL((k_adjoint_init<Q, TC, 9>), dim3(g.nblocks), dim3(kBlock), 0, st, g,
                           (const Coefs<TC> *)coefs, phi0, (const TC *)psi0, pi0, out);
    return hipGetLastError();
}

template <int Q, typename TS, typename TC>
hipError_t seed_typed(const Dims &, const Geom &g, const double *gphi, void *psi, double *pi, hipStream_t st) {
    hipLaunchKernelGGL((k_seed<Q, TC>), dim3(g.nblocks), dim3(kBlock), 0, st, g, gphi, (TC *)psi, pi);
    return hipGetLastError();
}

template <int Q, typename TS, typename TC>
hipError_t recenter_typed(const Dims &dm, const Geom &g, void *coefs, void *f, void *p, double *part, int nparts,
                          double *shift, hipStream_t st) {
    using TP = typename HistType<TS>::T;
    hipLaunchKernelGGL((k_offset_sum<Q, TS>), dim3(nparts), dim3(kBlock), 0, st, g, (const TS *)f,
                       (const TP *)p, (dm.src && !dm.sb) ? 1 : 0, part);
    hipLaunchKernelGGL((k_recenter_fold<Q, TC>), dim3(1), dim3(kBlock), 0, st, (Coefs<TC> *)coefs, part, nparts,
                       g.N, shift);
    hipLaunchKernelGGL((k_shift<Q, TS, TC>), dim3(g.nblocks), dim3(kBlock), 0, st, g, (const double *)shift,
                       (TS *)f, (TP *)p);
    return hipGetLastError();
}

template <int Q, typename TS, typename TC>
hipError_t set_wall_typed(const Dims &, void *coefs, const double *ewp, hipStream_t st) {
    WallTerms w;
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < 19; ++k) w.ewp[s][k] = ewp[s * 19 + k];
    hipLaunchKernelGGL((k_set_wall<Q, TC>), dim3(1), dim3(64), 0, st, (Coefs<TC> *)coefs, w);
    return hipGetLastError();
}

inline hipError_t zero_doubles(double *p, uint32_t n, hipStream_t st) {
    const uint32_t grid = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_zero, dim3(grid < 1024 ? grid : 1024), dim3(kBlock), 0, st, p, n);
    return hipGetLastError();
}

// FP64 and FP32 storage only (no adjoint for FP16 storage)
#define LBM_BY_PREC_ADJ(fn, ...)                                                   \
    switch (dm.prec) {                                                             \
        case 0: return fn<LBM_Q, double, double>(__VA_ARGS__);                     \
        case 1: return fn<LBM_Q, float, float>(__VA_ARGS__);                       \
        default: return hipErrorNotSupported;                                      \
    }

#define LBM_BY_PREC(fn, ...)                                                       \
    switch (dm.prec) {                                                             \
        case 0: return fn<LBM_Q, double, double>(__VA_ARGS__);                     \
        case 1: return fn<LBM_Q, float, float>(__VA_ARGS__);                        \
        case 2: return fn<LBM_Q, _Float16, float>(__VA_ARGS__);                     \
        default: return hipErrorInvalidValue;                                      \
    }

}  // namespace lbm
