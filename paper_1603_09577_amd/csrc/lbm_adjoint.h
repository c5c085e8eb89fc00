// Reversed (discrete adjoint) sweep of the D2Q9 stream-collide step.
//
// Forward sweep s at node x: g = gather(f_s) (offset form h), phi = phi_ref
// + sum h, then (equal-rate or moment-space relaxation, Eq. 2/17/19) plus the
// Scheme-A source 3/2 R_k(phi) - 1/2 R_k(p) with R_k = w_k (1 + 3 c.Btilde) R
// and Btilde = (I - A/2) B' (Eq. 9, 28 with gamma = 0); the result is stored
// at x and p(x) <- phi - phi_ref.
//
// Reverse: lambda_k(x) = dL/df_{s+1,k}(x) is psi_{s+1} read at the node that
// gathers it, x + c_k (or, across a wall, -psi_{s+1,kbar}(x): the
// anti-bounce-back read has coefficient -1).  The node map is then
// differentiated by hand in reverse order: relaxation -> A block -> Btilde,
// R -> equilibrium -> phi.  A depends on phi through K(phi) = K0 k(phi):
// A = G^-1 with G = (3/d) K0 k(phi) + I/2, so the adjoint of G is
// Gbar = -A Abar A, which also gives dL/dK0.
#pragma once

#include "lbm_kernels.h"

namespace lbm {

template <int Q, int NP, typename TC>
__device__ __forceinline__ void eq_derivative(const Coefs<TC> *__restrict__ cf, TC phi, TC *dfeq) {
    // d feq_k / d phi = w_k [1 + 3 c.B' + 9/2 (E' : c c - tr E' / 3)],
    // E' = C-bar'(phi) - I/3
    using L = Lattice<Q>;
    constexpr int D = L::dim;
    TC Bp[3], E[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) Bp[a] = (a < D) ? poly<PolyLen<NP>::ND>(cf->bp[a], phi) : TC(0);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const bool used = (D == 3) || (i == 0 || i == 1 || i == 3);
        E[i] = used ? poly<PolyLen<NP>::NCD>(cf->cbd[i], phi) : TC(0);
    }
    E[0] -= TC(1.0 / 3.0); E[1] -= TC(1.0 / 3.0);
    if (D == 3) E[2] -= TC(1.0 / 3.0);
    const TC trE3 = (E[0] + E[1] + E[2]) * TC(1.0 / 3.0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int x = L::cx(k), y = L::cy(k), z = L::cz(k);
        TC cB = TC(0), ccE = -trE3;
        if (x) { cB += x * Bp[0]; ccE += E[0]; }
        if (y) { cB += y * Bp[1]; ccE += E[1]; }
        if (z) { cB += z * Bp[2]; ccE += E[2]; }
        if (x && y) ccE += TC(2 * x * y) * E[3];
        if (y && z) ccE += TC(2 * y * z) * E[4];
        if (x && z) ccE += TC(2 * x * z) * E[5];
        dfeq[k] = TC(L::w(k)) * (TC(1) + TC(3) * cB + TC(4.5) * ccE);
    }
}

// Adjoint of A = G^-1 for a symmetric Abar (full storage Ab[a][b]):
// Gbar = -A Abar A (symmetric), returned in symmetric slots.
template <int DIM, typename TC>
__device__ __forceinline__ void gbar_of(const TC *A, const TC Ab[3][3], TC *Gb) {
    TC T[3][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            TC acc = TC(0);
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc += A[sym(a, c)] * TC(0.5) * (Ab[c][b] + Ab[b][c]);
            T[a][b] = acc;
        }
#pragma unroll
    for (int i = 0; i < 6; ++i) Gb[i] = TC(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = a; b < DIM; ++b) {
            TC acc = TC(0);
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc += T[a][c] * A[sym(c, b)];
            Gb[sym(a, b)] = -acc;
        }
}

// Contribution of Gbar at a phi value to dL/dphi (when k varies) and to the
// per-node K0 accumulator (symmetric parametrisation: off-diagonal entries
// count twice).
template <int DIM, bool KVAR, int NP, typename TC>
__device__ __forceinline__ TC gbar_scatter(const Coefs<TC> *__restrict__ cf, TC phi, const TC *Gb, TC *gk) {
    const TC kv = KVAR ? poly<NP>(cf->kp, phi) : cf->kp[0];
    // g0 = 3 K0 / d, so dG/dK0_ab = (3/d) k(phi); g0 / K0 = 3 / d is folded on the host
#pragma unroll
    for (int i = 0; i < 6; ++i) gk[i] += Gb[i] * kv * (i < 3 ? TC(1) : TC(2));
    if (!KVAR) return TC(0);
    const TC kd = poly<PolyLen<NP>::ND>(cf->kdp, phi);
    TC acc = TC(0);
#pragma unroll
    for (int i = 0; i < 6; ++i) acc += Gb[i] * cf->g0[i] * (i < 3 ? TC(1) : TC(2));
    return acc * kd;
}

// lambda_k(x) = psi_{s+1,k}(x + c_k): the transposed streaming of the pull
// gather (across a wall, -psi_{s+1,kbar}(x), the transposed anti-bounce-back).
// NT: streaming (non-temporal) loads, for states far larger than the caches.
template <int Q, bool WALL, bool O32 = false, bool NT = false, typename TC>
__device__ __forceinline__ void gather_adjoint(const Geom &g, const TC *__restrict__ psi_next, const NodeGeo &ng,
                                               TC *lam) {
    using L = Lattice<Q>;
    constexpr int D = L::dim;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        int off = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int c = L::c(k, a);
            off += (c == 1) ? ng.op[a] : ((c == -1) ? ng.om[a] : 0);
        }
        const int cl = L::c(k, D - 1);
        if (WALL && ((cl == 1 && ng.hi) || (cl == -1 && ng.lo)))
            lam[k] = -load_s<TC, NT>(at<O32>(psi_next + (uint64_t)L::opp(k) * g.plane, ng.n));
        else
            lam[k] = load_s<TC, NT>(at<O32>(psi_next + (uint64_t)k * g.plane, (uint32_t)((int)ng.n + off)));
    }
}

// gather_adjoint (row y + c_y, column x + c_x) for a row wave (RowWave), D2Q9.
template <bool WALL, bool NT, typename TC>
__device__ __forceinline__ void gather_adjoint_rw(const Geom &g, const TC *__restrict__ psi_next, RowWave &w,
                                                  TC *lam) {
    using L = Lattice<9>;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = L::cx(k), cy = L::cy(k);
        if (WALL && ((cy == 1 && w.hi) || (cy == -1 && w.lo)))
            lam[k] = -load_s<TC, NT>(at<true>(psi_next + (uint64_t)L::opp(k) * g.plane, w.n));
        else
            lam[k] = load_s<TC, NT>(row_elem(psi_next + (uint64_t)k * g.plane, w.rowb[1 + cy], w.colb[1 + cx]));
    }
}

// The reversed map at one node, shared by the one-sweep and two-sweep
// kernels: from the gathered forward populations h (offset form), the history
// pp_off = p_s(x), lam_k = psi_{s+1,k}(x + c_k) and pin = pi_{s+1}(x), writes
// psi_s(x) to out and returns pi_s(x); adds this node's K0 terms to gk.
template <int Q, typename TC, bool EQR, bool SRC, bool KVAR, int NP>
__device__ __forceinline__ TC adjoint_node(const Coefs<TC> *__restrict__ cf, const TC *h, TC pp_off,
                                           const TC *lam, TC pin, TC *out, TC *gk) {
    using L = Lattice<Q>;
    constexpr int D = L::dim;
    TC phio = TC(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) phio += h[k];
    const TC phi = cf->phi_ref + phio;
    TC A[6];
    ablock<D, KVAR, NP>(cf, phi, A);

    TC Ab[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Ab[a][b] = TC(0);
    TC phib = TC(0), pb = TC(0);
    TC hb[Q];

    if (EQR) {
        // Forward (see sweep_node):
        //   out_k = (1 - s) g_k + w_k (s phio + Se + 9/2 s (E : c_k c_k - tr E / 3))
        //           + c_k . (w_k (3 s B + Vo) - v),  v = (A - s I)(j - B) / |c_a|^2,
        //   Se = 3/2 R - 1/2 Rp, Vo = 9/2 R Bt - 3/2 Rp Btp, Bt = (I - A/2) B'.
        // Its adjoint needs only moments of lambda:
        //   L0w = sum w lam, L1 = sum c lam, L1w = sum w c lam, L2w = sum w c c lam.
        const TC s = cf->srate;
        constexpr TC inv_nc = TC(1.0 / L::jnorm);
        TC L0w = TC(0), L1[3] = {TC(0), TC(0), TC(0)}, L1w[3] = {TC(0), TC(0), TC(0)};
        TC L2w[6] = {TC(0), TC(0), TC(0), TC(0), TC(0), TC(0)};
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const TC wl = TC(L::w(k)) * lam[k];
            L0w += wl;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int c = L::c(k, a);
                if (c) { L1[a] += TC(c) * lam[k]; L1w[a] += TC(c) * wl; }
            }
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a; b < D; ++b) {
                    const int cc = L::c(k, a) * L::c(k, b);
                    if (cc) L2w[sym(a, b)] += TC(cc) * wl;
                }
        }
        // forward pieces at phi
        TC B[3], Bp[3], Bpp[3], jd[3];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            B[a] = poly<NP>(cf->b[a], phi);
            Bp[a] = poly<PolyLen<NP>::ND>(cf->bp[a], phi);
            Bpp[a] = poly<PolyLen<NP>::ND2>(cf->bpp[a], phi);
            TC acc = TC(0);
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const int c = L::c(k, a);
                if (c == 1) acc += h[k];
                else if (c == -1) acc -= h[k];
            }
            jd[a] = acc - B[a];
        }
        // u = (A - s I) L1 / |c|^2: adjoint of j (with a minus) and of B
        TC u[3];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            TC acc = TC(0);
#pragma unroll
            for (int b = 0; b < D; ++b) acc += (A[sym(a, b)] - (a == b ? s : TC(0))) * L1[b];
            u[a] = acc * inv_nc;
        }
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) Ab[a][b] -= L1[a] * jd[b] * inv_nc;
        // phio, B, E
        phib = s * L0w;
#pragma unroll
        for (int a = 0; a < D; ++a) phib += (TC(3) * s * L1w[a] + u[a]) * Bp[a];
        {
            const TC s45 = TC(4.5) * s;
            TC tr = TC(0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                // dE_aa/dphi = Cbar'_aa - 1/3, weight 9/2 s (L2w_aa - L0w / 3)
                const TC cbd = poly<PolyLen<NP>::NCD>(cf->cbd[a], phi) - TC(1.0 / 3.0);
                tr += s45 * (L2w[a] - L0w * TC(1.0 / 3.0)) * cbd;
            }
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a + 1; b < D; ++b)
                    tr += s45 * TC(2) * L2w[sym(a, b)] * poly<PolyLen<NP>::NCD>(cf->cbd[sym(a, b)], phi);
            phib += tr;
        }
        if (SRC) {
            TC Bt[3], R, Btp[3], Rp, Ap[6];
            source_terms<D, NP>(cf, phi, A, Bt, R);
            const TC pp = cf->phi_ref + pp_off;
            ablock<D, KVAR, NP>(cf, pp, Ap);
            source_terms<D, NP>(cf, pp, Ap, Btp, Rp);
            TC t1 = TC(0), t1p = TC(0);
#pragma unroll
            for (int a = 0; a < D; ++a) { t1 += L1w[a] * Bt[a]; t1p += L1w[a] * Btp[a]; }
            const TC Rb = TC(1.5) * L0w + TC(4.5) * t1;
            const TC Rpb = TC(-0.5) * L0w - TC(1.5) * t1p;
            phib += Rb * poly<PolyLen<NP>::ND>(cf->rp, phi);
            pb += Rpb * poly<PolyLen<NP>::ND>(cf->rp, pp);
            TC Btb[3], Btpb[3], Bpq[3], Bppq[3];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                Btb[a] = TC(4.5) * R * L1w[a];
                Btpb[a] = TC(-1.5) * Rp * L1w[a];
                Bpq[a] = poly<PolyLen<NP>::ND>(cf->bp[a], pp);
                Bppq[a] = poly<PolyLen<NP>::ND2>(cf->bpp[a], pp);
            }
            TC Apb[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) Apb[a][b] = TC(0);
#pragma unroll
            for (int b = 0; b < D; ++b) {
                TC acc = Btb[b], accp = Btpb[b];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    acc -= TC(0.5) * A[sym(a, b)] * Btb[a];
                    accp -= TC(0.5) * Ap[sym(a, b)] * Btpb[a];
                }
                phib += acc * Bpp[b];
                pb += accp * Bppq[b];
            }
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    Ab[a][b] -= TC(0.5) * Btb[a] * Bp[b];
                    Apb[a][b] -= TC(0.5) * Btpb[a] * Bpq[b];
                }
            TC Gbp[6];
            gbar_of<D>(Ap, Apb, Gbp);
            pb += gbar_scatter<D, KVAR, NP>(cf, pp, Gbp, gk);
        }
        const TC oms = TC(1) - s;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            TC cu = TC(0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int c = L::c(k, a);
                if (c) cu += TC(c) * u[a];
            }
            hb[k] = oms * lam[k] - cu;
        }
    } else {
        TC feq[Q], dlt[Q];
        equilibrium<Q, NP>(cf, phi, phio, feq);
#pragma unroll
        for (int k = 0; k < Q; ++k) dlt[k] = h[k] - feq[k];
        // out = h - M^T N^-1 S M dlt: u = N^-1 M lambda, rbar = -u,
        // mbar = S^T rbar, dbar = M^T mbar, Abar_ab += rbar_ja m_jb
        TC m[Q], u[Q], db[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            TC acc = TC(0), accl = TC(0);
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const int mm = L::M(i, k);
                if (mm) { acc += TC(mm) * dlt[k]; accl += TC(mm) * lam[k]; }
            }
            m[i] = acc;
            u[i] = accl * TC(1.0 / L::N(i));
        }
        TC mb[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) mb[i] = -cf->s[i] * u[i];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            TC acc = TC(0);
#pragma unroll
            for (int b = 0; b < D; ++b) acc -= A[sym(b, a)] * u[L::jrow[b]];
            mb[L::jrow[a]] = acc;
        }
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) Ab[a][b] -= u[L::jrow[a]] * m[L::jrow[b]];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            TC acc = TC(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int mm = L::M(i, k);
                if (mm) acc += TC(mm) * mb[i];
            }
            db[k] = acc;
        }
        // h enters directly (out = h - ...) and through dlt; feq through
        // dlt with a minus sign, and feq depends on phi only
#pragma unroll
        for (int k = 0; k < Q; ++k) hb[k] = lam[k] + db[k];
        {
            TC dfe[Q];
            eq_derivative<Q, NP>(cf, phi, dfe);
#pragma unroll
            for (int k = 0; k < Q; ++k) phib -= db[k] * dfe[k];
        }
        if (SRC) {
            TC Bt[3], R, Btp[3], Rp, Ap[6];
            source_terms<D, NP>(cf, phi, A, Bt, R);
            const TC pp = cf->phi_ref + pp_off;
            ablock<D, KVAR, NP>(cf, pp, Ap);
            source_terms<D, NP>(cf, pp, Ap, Btp, Rp);
            TC S1 = TC(0), T1[3] = {TC(0), TC(0), TC(0)};
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const TC wl = TC(L::w(k)) * lam[k];
                S1 += wl;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    const int c = L::c(k, a);
                    if (c) T1[a] += TC(c) * wl;
                }
            }
            // time level t: + 3/2 R (S1 + 3 T1.Bt);  level t-1: - 1/2 Rp (S1 + 3 T1.Btp)
            TC tb = TC(0), tbp = TC(0);
#pragma unroll
            for (int a = 0; a < D; ++a) { tb += T1[a] * Bt[a]; tbp += T1[a] * Btp[a]; }
            const TC Rb = TC(1.5) * (S1 + TC(3) * tb);
            const TC Rpb = TC(-0.5) * (S1 + TC(3) * tbp);
            TC Btb[3], Btpb[3];
#pragma unroll
            for (int a = 0; a < D; ++a) { Btb[a] = TC(4.5) * R * T1[a]; Btpb[a] = TC(-1.5) * Rp * T1[a]; }
            phib += Rb * poly<PolyLen<NP>::ND>(cf->rp, phi);
            pb += Rpb * poly<PolyLen<NP>::ND>(cf->rp, pp);
            TC Bp[3], Bpp[3], Bpq[3], Bppq[3];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                Bp[a] = poly<PolyLen<NP>::ND>(cf->bp[a], phi);
                Bpp[a] = poly<PolyLen<NP>::ND2>(cf->bpp[a], phi);
                Bpq[a] = poly<PolyLen<NP>::ND>(cf->bp[a], pp);
                Bppq[a] = poly<PolyLen<NP>::ND2>(cf->bpp[a], pp);
            }
            TC Apb[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) Apb[a][b] = TC(0);
#pragma unroll
            for (int b = 0; b < D; ++b) {
                TC acc = Btb[b], accp = Btpb[b];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    acc -= TC(0.5) * A[sym(a, b)] * Btb[a];
                    accp -= TC(0.5) * Ap[sym(a, b)] * Btpb[a];
                }
                phib += acc * Bpp[b];
                pb += accp * Bppq[b];
            }
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    Ab[a][b] -= TC(0.5) * Btb[a] * Bp[b];
                    Apb[a][b] -= TC(0.5) * Btpb[a] * Bpq[b];
                }
            TC Gbp[6];
            gbar_of<D>(Ap, Apb, Gbp);
            pb += gbar_scatter<D, KVAR, NP>(cf, pp, Gbp, gk);
        }
    }
    {
        TC Gb[6];
        gbar_of<D>(A, Ab, Gb);
        phib += gbar_scatter<D, KVAR, NP>(cf, phi, Gb, gk);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) out[k] = hb[k] + phib + pin;
    return pb;
}

// K0 partials of one workgroup: the per-thread terms are summed over the wave
// in the compute type (FP32 terms carry FP32 rounding already), then over the
// waves in FP64 with (3/d) applied; the workgroup owns `slot` and adds to it
// over the reversed sweeps (folded once when the gradient is read).  In 2-D
// only xx, yy and xy (slots 0, 1, 3) can be non-zero.  Called by every thread
// of the workgroup; sh is workgroup memory for 6 x NW doubles (NW waves per
// workgroup) that no thread still reads.
template <int D, int NW = kBlock / 64, typename TC>
__device__ __forceinline__ void k0_partials(const Coefs<TC> *__restrict__ cf, const TC *gk,
                                            double *__restrict__ gk_part, uint32_t slot,
                                            double (*sh)[NW]) {
    constexpr int NK = D == 2 ? 3 : 6;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int i = (D == 2 && j == 2) ? 3 : j;
        const double v = (double)wave_total(gk[i]) * (double)cf->k0scale;
        if (lane == 0) sh[j][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < NK) {
        const int j = threadIdx.x;
        const int i = (D == 2 && j == 2) ? 3 : j;
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) v += sh[j][w];
        // An atomic add without return instead of a load, an add and a
        // store: the workgroup's last wave no longer waits for a global load
        // before it can finish.  The slot belongs to this workgroup and the
        // sweeps that add to it are successive launches, so no two adds to
        // it are ever in flight together: the sum is formed in the same
        // order, one FP64 addition per sweep, as before.
        unsafeAtomicAdd(gk_part + (size_t)slot * 6 + i, v);
    }
}

// Occupancy: D2Q9 is held at 4 waves per SIMD (it fits 128 registers without
// spills); D3Q19 keeps 19 populations, their adjoints and the outputs live and
// is allowed down to 2.
// RW: every wave lies within one grid row (D2Q9 with nx a multiple of 64;
// the host checks), and the loads take the row-wave form above.
template <int Q, typename TS, typename TC, bool EQR, bool SRC, bool KVAR, bool WALL, int NP, bool O32 = false,
          bool NT = false, bool RW = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Q == 9 ? 4 : 2, 8)))
k_adjoint(const Geom g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ fs,
          const typename HistType<TS>::T *__restrict__ ps, const TC *__restrict__ psi_next,
          const double *pi_next, TC *__restrict__ psi_out, double *pi_out, double *__restrict__ gk_part) {
    using L = Lattice<Q>;
    constexpr int D = L::dim;
    const uint32_t n = block_index(blockIdx.x, gridDim.x, g.remap) * kBlock + threadIdx.x;
    TC gk[6] = {TC(0), TC(0), TC(0), TC(0), TC(0), TC(0)};
    if (n < g.N) {
        TC h[Q], lam[Q];
        TC pp_off, pin;
        if constexpr (RW) {
            static_assert(Q == 9 && O32, "row waves: D2Q9 with 32-bit offsets");
            RowWave w = row_wave<TS, WALL>(g, n);
            // ---- forward recomputation ----
            gather_rw<WALL, NT>(g, cf, fs, w, h);
            pp_off = SRC ? (TC)*at<true>(ps, n) : TC(0);
            pin = (TC)*at<true>(pi_next, n);   // p_{s+1} = phi - phi_ref
            // ---- lambda = dL/d(out) by transposed streaming ----
            gather_adjoint_rw<WALL, NT>(g, psi_next, w, lam);
        } else {
            const NodeGeo ng = node_geometry<Q, WALL>(g, n);
            gather<Q, WALL, NT, O32>(g, cf, fs, ng, h);
            pp_off = SRC ? (TC)*at<O32>(ps, n) : TC(0);
            pin = (TC)*at<O32>(pi_next, n);
            gather_adjoint<Q, WALL, O32, NT>(g, psi_next, ng, lam);
        }

        TC out[Q];
        const TC pb = adjoint_node<Q, TC, EQR, SRC, KVAR, NP>(cf, h, pp_off, lam, pin, out, gk);
        if constexpr (O32) {
            store_planes<Q, NT>(psi_out, g.plane, n, out);
        } else {
#pragma unroll
            for (int k = 0; k < Q; ++k) store_s<NT>(psi_out + (uint64_t)k * g.plane + n, out[k]);
        }
        *at<O32>(pi_out, n) = (double)pb;
    }
    __shared__ double sh[6][kBlock / 64];
    k0_partials<D>(cf, gk, gk_part, blockIdx.x, sh);
}

// Row (halo included) that row slot j of a tile of TR rows takes when NW
// waves split the rows, slot j = wave + pass * NW.  With several rows per
// wave, the first pass takes the four rows the tile shares with the tiles
// above and below (0, 1, TR - 2, TR - 1), so that both tiles read them at
// about the same time and the second read finds them in L2 (FP64 512^2:
// fetched bytes 1.10 -> 1.03 x the algorithmic reads); the inner rows
// follow.  A permutation of 0 .. TR - 1 for every TR >= 4.
template <int TR, int NW>
__device__ __forceinline__ constexpr int shared_rows_first(int j) {
    return (TR / NW == 1 || j < 2) ? j : (j < 4 ? TR - 4 + j : j - 2);
}

// Two reversed sweeps in one pass (D2Q9, periodic, equal rates): sweep s,
// then sweep s - 1, on a tile of 62 x TH nodes.  Phase 1 runs the reversed
// map of sweep s on the tile and a one-node halo around it (64 x (TH + 2)
// nodes), reading (f_s, p_s), psi_{s+1} and pi_{s+1}, and keeps psi_s and
// pi_s in workgroup memory in the compute type, exactly as a store and a
// reload would leave them.  Phase 2 runs sweep s - 1 on the tile's own nodes,
// reading (f_{s-1}, p_{s-1}) and psi_s at x + c_k from workgroup memory, and
// stores psi_{s-1} and pi_{s-1}.  Both phases call adjoint_node, so psi and
// pi are bit-identical to two one-sweep launches; the K0 terms of phase 1
// count only the tile's own nodes (the halo belongs to the neighbours).
// pi_out must differ from pi_next: neighbouring tiles still read pi_{s+1} at
// their halo.
// A workgroup has NW waves; the TH + 2 rows of phase 1 split evenly over
// them, and phase 2 gives the TH own rows to the waves in turn.
// FP64 6-row tiles with short polynomials are held to 3 waves per SIMD (168
// registers), what their workgroup memory allows anyway (3 workgroups of 4
// waves per CU); with 9-term polynomials that limit would spill.  10-row
// tiles fit 2 workgroups per CU, and take no register limit.
template <typename TS, typename TC, bool SRC, bool KVAR, int NP, int TH, int NW>
__global__ void __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu(sizeof(TC) == 8 && NP <= 4 && TH == 6 ? 3 : 1, 8)))
k_adjoint2(const Geom g, const Coefs<TC> *__restrict__ cf, const TS *__restrict__ f1,
           const typename HistType<TS>::T *__restrict__ p1, const TS *__restrict__ f0,
           const typename HistType<TS>::T *__restrict__ p0, const TC *__restrict__ psi_next,
           const double *__restrict__ pi_next, TC *__restrict__ psi_out, double *__restrict__ pi_out,
           double *__restrict__ gk_part, uint32_t tiles_x) {
    using L = Lattice<9>;
    constexpr int TX = 64, TR = TH + 2;
    static_assert(TR % NW == 0, "tile rows must split evenly over the waves");
    static_assert(sizeof(TC) * 9 * TR * TX >= sizeof(double) * 6 * NW, "reduction scratch");
    __shared__ alignas(16) TC lpsi[9][TR][TX];
    __shared__ TC lpi[TR][TX];
    const uint32_t tile = block_index(blockIdx.x, gridDim.x, g.remap);
    const uint32_t ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int x0 = (int)(tx * (TX - 2)), y0 = (int)(ty * TH);
    const int lane = threadIdx.x & 63;
    // wave index in a scalar register: the rows of both phases are wave-uniform
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nx = (int)g.nx, ny = (int)g.ny;
    TC gk[6] = {TC(0), TC(0), TC(0), TC(0), TC(0), TC(0)};
    // a lane owns column x0 + lane - 1 when it is an interior lane inside the grid
    const bool xown = lane >= 1 && lane <= TX - 2 && x0 + lane - 1 < nx;
    // phase 1: the tile and its halo (coordinates wrapped periodically; narrow
    // or low grids repeat nodes in the halo, which only the owner counts)
    const int xg = wrap_coord(x0 - 1 + lane, nx);
    // byte offsets of the columns x - 1, x, x + 1 (periodic), fixed per lane;
    // rows are wave-uniform, so every load is a scalar row base plus one of
    // them (the same for an owner's node in phase 2, where x = xg)
    static_assert(sizeof(TS) == sizeof(TC), "adjoint state and psi share the element size");
    RowWave w;
    w.colb[0] = (uint32_t)(xg == 0 ? nx - 1 : xg - 1) * (uint32_t)sizeof(TS);
    w.colb[1] = (uint32_t)xg * (uint32_t)sizeof(TS);
    w.colb[2] = (uint32_t)(xg == nx - 1 ? 0 : xg + 1) * (uint32_t)sizeof(TS);
    w.lo = w.hi = false;
    const uint32_t rowb = g.nx * (uint32_t)sizeof(TS);
    // FP32 unrolls the rows (all loads in flight); FP64 takes them one by one
    // (about 165 registers per lane as it is: 3 waves per SIMD)
    constexpr int kUnroll = sizeof(TC) == 4 ? TR / NW : 1;
#pragma unroll kUnroll
    for (int i = 0; i < TR / NW; ++i) {
        const int r = shared_rows_first<TR, NW>(wv + i * NW);
        const int yg = wrap_coord(y0 - 1 + r, ny);
        const uint32_t n = (uint32_t)yg * g.nx + (uint32_t)xg;
        w.n = n;
        w.rowb[0] = (uint32_t)(yg == 0 ? ny - 1 : yg - 1) * rowb;
        w.rowb[1] = (uint32_t)yg * rowb;
        w.rowb[2] = (uint32_t)(yg == ny - 1 ? 0 : yg + 1) * rowb;
        TC h[9], lam[9], out[9];
        gather_rw<false, false>(g, cf, f1, w, h);
        gather_adjoint_rw<false, false>(g, psi_next, w, lam);
        const TC pp_off = SRC ? (TC)*at<true>(p1, n) : TC(0);
        const TC pin = (TC)*at<true>(pi_next, n);
        TC gkn[6] = {TC(0), TC(0), TC(0), TC(0), TC(0), TC(0)};
        const TC pb = adjoint_node<9, TC, true, SRC, KVAR, NP>(cf, h, pp_off, lam, pin, out, gkn);
        if (xown && r >= 1 && r <= TH && y0 + r - 1 < ny) {
#pragma unroll
            for (int j = 0; j < 6; ++j) gk[j] += gkn[j];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) lpsi[k][r][lane] = out[k];
        lpi[r][lane] = pb;
    }
    __syncthreads();
    // phase 2: the tile's own nodes, psi_s gathered from x + c_k in the tile
    if (xown) {
        const uint32_t x = (uint32_t)(x0 + lane - 1);
        for (int r = 1 + wv; r <= TH && y0 + r - 1 < ny; r += NW) {
            const int y = y0 + r - 1;
            const uint32_t n = (uint32_t)y * g.nx + x;
            w.n = n;
            w.rowb[0] = (uint32_t)(y == 0 ? ny - 1 : y - 1) * rowb;
            w.rowb[1] = (uint32_t)y * rowb;
            w.rowb[2] = (uint32_t)(y == ny - 1 ? 0 : y + 1) * rowb;
            TC h[9], lam[9], out[9];
            gather_rw<false, false>(g, cf, f0, w, h);
#pragma unroll
            for (int k = 0; k < 9; ++k) lam[k] = lpsi[k][r + L::cy(k)][lane + L::cx(k)];
            const TC pp_off = SRC ? (TC)*at<true>(p0, n) : TC(0);
            const TC pb = adjoint_node<9, TC, true, SRC, KVAR, NP>(cf, h, pp_off, lam, lpi[r][lane], out, gk);
            store_planes<9, false>(psi_out, g.plane, n, out);
            *at<true>(pi_out, n) = (double)pb;
        }
    }
    __syncthreads();   // the tile buffer becomes the reduction scratch
    k0_partials<2, NW>(cf, gk, gk_part, blockIdx.x, reinterpret_cast<double(*)[NW]>(&lpsi[0][0][0]));
}

// zero the per-workgroup K0 slots (a kernel, so that the adjoint can be
// captured in a graph without memset nodes)
static __global__ void __launch_bounds__(kBlock)
k_zero(double *__restrict__ p, uint32_t n) {
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = 0.0;
}

// dL/dphi0 = sum_k psi_0,k dfeq_k/dphi(phi0) + pi_0   (adjoint of Eq. 40)
template <int Q, typename TC, int NP>
__global__ void __launch_bounds__(kBlock)
k_adjoint_init(const Geom g, const Coefs<TC> *__restrict__ cf, const double *__restrict__ phi0,
               const TC *__restrict__ psi0, const double *__restrict__ pi0, double *__restrict__ out) {
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    TC dfe[Q];
    eq_derivative<Q, NP>(cf, (TC)phi0[n], dfe);
    double acc = pi0[n];
#pragma unroll
    for (int k = 0; k < Q; ++k) acc += (double)(psi0[(uint64_t)k * g.plane + n] * dfe[k]);
    out[n] = acc;
}

template <int Q, typename TC>
__global__ void __launch_bounds__(kBlock)
k_seed(const Geom g, const double *__restrict__ gphi, TC *__restrict__ psi, double *__restrict__ pi) {
    // psi_T,k = dL/dphi(T) for every k (phi = sum_k g_k), pi_T = 0
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const TC v = (TC)gphi[n];
#pragma unroll
    for (int k = 0; k < Q; ++k) psi[(uint64_t)k * g.plane + n] = v;
    pi[n] = 0.0;
}

}  // namespace lbm
