// Host side of the C ABI declared in include/lbm.h: validation, derivation
// of the model constants, context state and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/lbm.h"
#include "lbm_internal.h"
#include "lbm_lattice.h"


using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return LBM_E_HIP;
}

constexpr int kAdjWidth = 6;          // K0 gradient entries per adjoint partial
constexpr int kMaxAdjParts = 65536;   // workgroups covered by the adjoint partials
constexpr int kGraphSteps = 32;       // sweeps per captured graph (even: ends on the start buffer)
constexpr int kRecenterF16 = 256;     // default re-centring interval, FP16 storage with a source (steps)

}  // namespace

struct lbm_ctx {
    lbm_desc desc;
    Dims dm;
    Geom g;
    size_t coef_bytes;
    unsigned char host_coefs[sizeof(Coefs<double>)];
    void *d_coefs = nullptr;
    // device scratch: [flag int (256 B)] [reduce partials] [reduce out 8] [adj partials] [k0 acc 8]
    // [offset shift 8]
    void *d_scratch = nullptr;
    int *d_flag = nullptr;
    double *d_red_part = nullptr, *d_red_out = nullptr, *d_adj_part = nullptr, *d_k0acc = nullptr;
    double *d_shift = nullptr;
    void *f[2] = {nullptr, nullptr};
    void *p = nullptr;
    const double *phi0 = nullptr;
    int cur = 0;
    long long t = 0;
    int check_every = 0;
    int recenter_every = 0;   // steps between re-centrings of the stored offsets (0: never)
    bool recentered = false;  // phi_ref on the device differs from the description's
    // per-node fields (caller-owned, FP64): K0(x) and the external source R(x, t)
    const double *kfield = nullptr, *rfield = nullptr;
    // two time steps per pass: the caller's second phi history buffer (needed
    // only when the run keeps a history), and whether the path is on
    void *p2 = nullptr;
    bool two_ok = false, two = false;
    // lbm_step replays captured graphs of kGraphSteps sweeps (lbm_tune may
    // find direct launches faster)
    bool use_graphs = true;
    // D3Q19 passes: resident workgroups per CU of each tile shape's kernel
    // (0: not asked yet) and the device's CU count, for the z-chunk choice
    int occ3[4] = {0, 0, 0, 0};
    int ncu = 0;
    int two_shape = 0;        // tile shape of two-step passes (two_step_shape_of; 0: the default)
    int adj_shape = 0;        // tile shape of the two-sweep adjoint (adjoint2_shape_of)
    int adj_shape_auto = 0;   // the shape pick_adj_shape chose
    uint32_t adj_slots = 0;   // K0 partial slots: workgroups of the one- and two-sweep adjoints
    bool bound = false;
    // graphs of kGraphSteps sweeps starting from buffer 0 / 1, captured on an
    // internal stream and launched on the caller's stream
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
};

namespace {

size_t storage_size(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }
size_t hist_size(int prec) { return prec == 0 ? 8 : 4; }
size_t round256(size_t v) { return (v + 255) & ~size_t(255); }

int top_count(const double *c, int n) {
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (c[i] != 0.0) m = i + 1;
    return m;
}

bool spd(const double K[3][3], int dim) {
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b)
            if (std::fabs(K[a][b] - K[b][a]) > 1e-14 * (std::fabs(K[a][b]) + std::fabs(K[b][a])) + 0.0)
                return false;
    const double m1 = K[0][0];
    const double m2 = K[0][0] * K[1][1] - K[0][1] * K[1][0];
    if (!(m1 > 0.0) || !(m2 > 0.0)) return false;
    if (dim == 3) {
        const double m3 = K[0][0] * (K[1][1] * K[2][2] - K[1][2] * K[2][1]) -
                          K[0][1] * (K[1][0] * K[2][2] - K[1][2] * K[2][0]) +
                          K[0][2] * (K[1][0] * K[2][1] - K[1][1] * K[2][0]);
        if (!(m3 > 0.0)) return false;
    }
    return true;
}

// symmetric 2x2 / 3x3 inverse in FP64 (storage xx, yy, zz, xy, yz, xz)
void sym_inv_host(const double *G, double *A, int dim) {
    if (dim == 2) {
        const double det = G[0] * G[1] - G[3] * G[3];
        A[0] = G[1] / det; A[1] = G[0] / det; A[3] = -G[3] / det;
        A[2] = A[4] = A[5] = 0.0;
    } else {
        const double c00 = G[1] * G[2] - G[4] * G[4], c11 = G[0] * G[2] - G[5] * G[5];
        const double c22 = G[0] * G[1] - G[3] * G[3], c01 = G[5] * G[4] - G[3] * G[2];
        const double c12 = G[3] * G[5] - G[0] * G[4], c02 = G[3] * G[4] - G[5] * G[1];
        const double det = G[0] * c00 + G[3] * c01 + G[5] * c02;
        A[0] = c00 / det; A[1] = c11 / det; A[2] = c22 / det;
        A[3] = c01 / det; A[4] = c12 / det; A[5] = c02 / det;
    }
}

struct HostModel {
    double b[3][kMaxP], bp[3][kMaxP], bpp[3][kMaxP], cb[6][kMaxC], cbd[6][kMaxC], g0[6], kp[kMaxP],
        kdp[kMaxP], a[6], r[kMaxP], rp[kMaxP], ew[2][19], ewp[2][19], s[19], phi_ref, srate, k0scale,
        bq[kMaxP], bqp[kMaxP];
    int nb, ncb, nk, nr, nq;
};

// A rational B: a denominator other than 0 (unset) or the constant 1.
bool rational_flux(const lbm_desc &d) {
    if (d.bden[0] != 0.0 && d.bden[0] != 1.0) return true;
    for (int p = 1; p < LBM_MAXP; ++p)
        if (d.bden[p] != 0.0) return true;
    return false;
}

double polyval(const double *c, int n, double x) {
    double acc = 0.0;
    for (int p = n - 1; p >= 0; --p) acc = acc * x + c[p];
    return acc;
}

// e+_k(pw): the even part of Eq. 3 at a wall value, from the C-bar
// polynomials already in m (so Remark III's C = 0 carries over).
double wall_even(const HostModel &m, const Dims &dm, double pw, int k) {
    const int dim = dm.q == 9 ? 2 : 3;
    double E[6];
    for (int i = 0; i < 6; ++i) E[i] = polyval(m.cb[i], kMaxC, pw) - (i < dim ? pw / 3.0 : 0.0);
    if (dim == 2) E[2] = 0.0;
    const double tr3 = (E[0] + E[1] + E[2]) / 3.0;
    int c[3];
    double w;
    if (dm.q == 9) { c[0] = Lattice<9>::cx(k); c[1] = Lattice<9>::cy(k); c[2] = 0; w = Lattice<9>::w(k); }
    else { c[0] = Lattice<19>::cx(k); c[1] = Lattice<19>::cy(k); c[2] = Lattice<19>::cz(k); w = Lattice<19>::w(k); }
    double cc = -tr3;
    for (int a = 0; a < 3; ++a) cc += c[a] * c[a] * E[a];
    cc += 2.0 * (c[0] * c[1] * E[3] + c[1] * c[2] * E[4] + c[0] * c[2] * E[5]);
    return w * (pw + 4.5 * cc);
}

// All derived constants of a description (FP64).
void derive(const lbm_desc &d, const Dims &dm, HostModel &m) {
    std::memset(&m, 0, sizeof(m));
    const int dim = dm.q == 9 ? 2 : 3;
    static const int pa[6] = {0, 1, 2, 0, 1, 0}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p < kMaxP; ++p) m.b[a][p] = (a < dim) ? d.b[a][p] : 0.0;
    m.nb = 1;
    for (int a = 0; a < dim; ++a) m.nb = std::max(m.nb, top_count(d.b[a], kMaxP));
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p + 1 < kMaxP; ++p) m.bp[a][p] = (p + 1) * m.b[a][p + 1];
    // Eq. 7 integrated term by term from C(0) = 0:
    //   C_ab = sum_{p,r>=1} p r b_ap b_br / (p + r - 1) phi^(p + r - 1),
    // plus d cs^2 D_ab(phi) to form C-bar (Eq. 16 notation).
    // Remark III (Eq. 38): C = 0, C-bar = d cs^2 D only
    const bool with_c = !(d.flags & LBM_FLAG_REMARK3);
    for (int i = 0; i < 6; ++i) {
        const int a = pa[i], b = pb[i];
        if (a >= dim || b >= dim) continue;
        for (int p = 1; p < kMaxP && with_c; ++p)
            for (int r = 1; r < kMaxP; ++r) {
                const double v = m.b[a][p] * m.b[b][r];
                if (v != 0.0) m.cb[i][p + r - 1] += p * r * v / (p + r - 1);
            }
        for (int p = 0; p < kMaxP; ++p) m.cb[i][p] += d.d / 3.0 * d.dten[a][b] * d.dpoly[p];
    }
    m.ncb = 1;
    for (int i = 0; i < 6; ++i) m.ncb = std::max(m.ncb, top_count(m.cb[i], kMaxC));
    for (int i = 0; i < 6; ++i)
        for (int p = 0; p + 1 < kMaxC; ++p) m.cbd[i][p] = (p + 1) * m.cb[i][p + 1];
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p + 1 < kMaxP; ++p) m.bpp[a][p] = (p + 1) * m.bp[a][p + 1];
    m.k0scale = 3.0 / d.d;
    // Eq. 26 with dt = 1, cs^2 = 1/3:  A^-1 = 3 K / d + I/2
    for (int i = 0; i < 6; ++i) m.g0[i] = (pa[i] < dim && pb[i] < dim) ? 3.0 * d.k0[pa[i]][pb[i]] / d.d : 0.0;
    for (int p = 0; p < kMaxP; ++p) m.kp[p] = d.kpoly[p];
    for (int p = 0; p + 1 < kMaxP; ++p) m.kdp[p] = (p + 1) * d.kpoly[p + 1];
    m.nk = std::max(1, top_count(d.kpoly, kMaxP));
    {
        double G[6];
        for (int i = 0; i < 6; ++i) G[i] = m.g0[i] * d.kpoly[0] + (i < dim ? 0.5 : 0.0);
        if (dim == 2) G[2] = 1.0;
        sym_inv_host(G, m.a, dim);
        if (dim == 2) m.a[2] = 0.0;
    }
    for (int p = 0; p < kMaxP; ++p) m.r[p] = d.rpoly[p];
    for (int p = 0; p + 1 < kMaxP; ++p) m.rp[p] = (p + 1) * d.rpoly[p + 1];
    m.nr = std::max(1, top_count(d.rpoly, kMaxP));
    // anti-bounce-back constants: 2 (e+_k(phi_w) - w_k phi_ref), e+ the even
    // part of Eq. 3 at the wall value
    const int la = dim - 1;
    for (int side = 0; side < 2; ++side)
        for (int k = 0; k < dm.q; ++k) {
            const double w = dm.q == 9 ? Lattice<9>::w(k) : Lattice<19>::w(k);
            const double ep = wall_even(m, dm, d.phi_wall[la][side], k);
            m.ewp[side][k] = 2.0 * ep;
            m.ew[side][k] = 2.0 * (ep - w * d.phi_ref);
        }
    for (int i = 0; i < 19; ++i) m.s[i] = (i < dm.q) ? d.s[i] : 0.0;
    m.srate = d.s[1];
    m.phi_ref = d.phi_ref;
    // rational flux (Remark III): the denominator and its derivative
    m.nq = 0;
    if (rational_flux(d)) {
        for (int p = 0; p < kMaxP; ++p) m.bq[p] = d.bden[p];
        for (int p = 0; p + 1 < kMaxP; ++p) m.bqp[p] = (p + 1) * d.bden[p + 1];
        m.nq = std::max(1, top_count(d.bden, kMaxP));
    }
}

template <typename TC>
void pack(const HostModel &m, Coefs<TC> &c) {
    std::memset(&c, 0, sizeof(c));
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p < kMaxP; ++p) {
            c.b[a][p] = (TC)m.b[a][p]; c.bp[a][p] = (TC)m.bp[a][p]; c.bpp[a][p] = (TC)m.bpp[a][p];
        }
    for (int i = 0; i < 6; ++i)
        for (int p = 0; p < kMaxC; ++p) { c.cb[i][p] = (TC)m.cb[i][p]; c.cbd[i][p] = (TC)m.cbd[i][p]; }
    for (int i = 0; i < 6; ++i) { c.g0[i] = (TC)m.g0[i]; c.a[i] = (TC)m.a[i]; }
    for (int p = 0; p < kMaxP; ++p) {
        c.kp[p] = (TC)m.kp[p]; c.kdp[p] = (TC)m.kdp[p]; c.r[p] = (TC)m.r[p]; c.rp[p] = (TC)m.rp[p];
    }
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < 19; ++k) { c.ew[s][k] = (TC)m.ew[s][k]; c.ewp[s][k] = (TC)m.ewp[s][k]; }
    for (int i = 0; i < 19; ++i) c.s[i] = (TC)m.s[i];
    c.phi_ref = (TC)m.phi_ref;
    c.srate = (TC)m.srate;
    c.k0scale = (TC)m.k0scale;
    c.nb = m.nb; c.ncb = m.ncb; c.nk = m.nk; c.nr = m.nr;
    for (int p = 0; p < kMaxP; ++p) { c.bq[p] = (TC)m.bq[p]; c.bqp[p] = (TC)m.bqp[p]; }
    c.nq = m.nq;
}

int validate(const lbm_desc *d, Dims &dm) {
    if (!d) return fail(LBM_E_INVALID, "null description");
    if (d->lattice != LBM_D2Q9 && d->lattice != LBM_D3Q19) return fail(LBM_E_INVALID, "lattice must be 9 or 19");
    const int dim = d->lattice == LBM_D2Q9 ? 2 : 3;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(LBM_E_INVALID, "grid sizes must be >= 1");
    if (dim == 2 && d->nz != 1) return fail(LBM_E_INVALID, "D2Q9 needs nz = 1");
    const double nn = (double)d->nx * d->ny * d->nz;
    if (nn >= 2147483648.0) return fail(LBM_E_INVALID, "more than 2^31 nodes");
    if (d->precision < LBM_F64 || d->precision > LBM_F16) return fail(LBM_E_INVALID, "unknown precision");
    if (!(d->d > 0.0) || !std::isfinite(d->d)) return fail(LBM_E_INVALID, "d must be positive");
    if (d->scheme != LBM_SCHEME_A && d->scheme != LBM_SCHEME_B) return fail(LBM_E_INVALID, "unknown scheme");
    for (int a = 0; a < 3; ++a)
        if (d->bc[a] != LBM_BC_PERIODIC && d->bc[a] != LBM_BC_ABB) return fail(LBM_E_INVALID, "unknown boundary");
    for (int a = 0; a < dim - 1; ++a)
        if (d->bc[a] != LBM_BC_PERIODIC) return fail(LBM_E_UNSUPPORTED, "walls are supported on the last axis only");
    const bool wall = d->bc[dim - 1] == LBM_BC_ABB;
    if (!spd(d->k0, dim)) return fail(LBM_E_INVALID, "k0 must be symmetric positive definite");
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b)
            if (d->dten[a][b] != d->dten[b][a]) return fail(LBM_E_INVALID, "dten must be symmetric");
    const int q = d->lattice;
    const int j0 = 3, j1 = 5, j2 = (q == 19) ? 7 : -1;
    bool eq = true;
    double s_common = -1.0;
    for (int i = 1; i < q; ++i) {
        if (i == j0 || i == j1 || i == j2) continue;
        if (!(d->s[i] > 0.0 && d->s[i] < 2.0)) return fail(LBM_E_INVALID, "relaxation rates must lie in (0, 2)");
        if (s_common < 0.0) s_common = d->s[i];
        else if (d->s[i] != s_common) eq = false;
    }
    if (!(d->s[0] >= 0.0 && d->s[0] < 2.0)) return fail(LBM_E_INVALID, "s0 must lie in [0, 2)");
    bool src = false, kvar = false;
    for (int p = 0; p < LBM_MAXP; ++p) {
        if (!std::isfinite(d->rpoly[p]) || !std::isfinite(d->kpoly[p]) || !std::isfinite(d->dpoly[p]))
            return fail(LBM_E_INVALID, "non-finite polynomial coefficient");
        if (d->rpoly[p] != 0.0) src = true;
        if (p > 0 && d->kpoly[p] != 0.0) kvar = true;
    }
    if (!(d->kpoly[0] > 0.0)) return fail(LBM_E_INVALID, "kpoly[0] must be positive (K(0) positive definite)");
    if (d->scheme == LBM_SCHEME_B)
        for (int p = 3; p < LBM_MAXP; ++p)
            if (d->rpoly[p] != 0.0)
                return fail(LBM_E_UNSUPPORTED,
                            "Scheme B solves Eq. 35 in closed form for R of degree <= 2 in phi");
    for (int p = 0; p < LBM_MAXP; ++p)
        if (!std::isfinite(d->bden[p])) return fail(LBM_E_INVALID, "non-finite polynomial coefficient");
    const bool rat = rational_flux(*d);
    if (rat && !(d->flags & LBM_FLAG_REMARK3))
        return fail(LBM_E_UNSUPPORTED, "a rational B needs LBM_FLAG_REMARK3 (its C of Eq. 7 is not integrated)");
    {
        int nb = 0;
        for (int a = 0; a < dim; ++a) nb = std::max(nb, top_count(d->b[a], LBM_MAXP));
        // C-bar = C + d/3 D: degree 2 (nb - 1) - 1 and the degree of dpoly
        const int ncb = std::max(nb > 1 ? 2 * nb - 2 : 1, top_count(d->dpoly, LBM_MAXP));
        dm.lowdeg = nb <= 4 && ncb <= 6 && top_count(d->kpoly, LBM_MAXP) <= 4 &&
                    top_count(d->rpoly, LBM_MAXP) <= 4;
        dm.deg3 = nb <= 3 && ncb <= 4 && top_count(d->kpoly, LBM_MAXP) <= 3 &&
                  top_count(d->rpoly, LBM_MAXP) <= 3;
        // a rational B is evaluated by the 9-term kernels only
        if (rat) dm.lowdeg = dm.deg3 = false;
    }
    dm.rat = rat;
    dm.nt = false;
    dm.q = q;
    dm.prec = d->precision;
    dm.eqr = eq && !(d->flags & LBM_FLAG_MOMENT_PATH);
    dm.src = src;
    dm.kvar = kvar;
    dm.wall = wall;
    dm.sb = d->scheme == LBM_SCHEME_B;
    return LBM_OK;
}

// Derive and pack the constants of c->desc into c->host_coefs (no upload).
void pack_host(lbm_ctx *c, HostModel &m) {
    derive(c->desc, c->dm, m);
    if (c->dm.prec == 0) {
        Coefs<double> cf;
        pack(m, cf);
        std::memcpy(c->host_coefs, &cf, sizeof(cf));
        c->coef_bytes = sizeof(cf);
    } else {
        Coefs<float> cf;
        pack(m, cf);
        std::memcpy(c->host_coefs, &cf, sizeof(cf));
        c->coef_bytes = sizeof(cf);
    }
}

int upload_coefs(lbm_ctx *c) {
    HostModel m;
    derive(c->desc, c->dm, m);
    if (c->dm.prec == 0) {
        Coefs<double> cf;
        pack(m, cf);
        std::memcpy(c->host_coefs, &cf, sizeof(cf));
        c->coef_bytes = sizeof(cf);
    } else {
        Coefs<float> cf;
        pack(m, cf);
        std::memcpy(c->host_coefs, &cf, sizeof(cf));
        c->coef_bytes = sizeof(cf);
    }
    hipError_t e = hipMemcpy(c->d_coefs, c->host_coefs, c->coef_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(coefficients)");
    return LBM_OK;
}

// Launch dimensions: Scheme B matters only with a source (with R = 0 it is
// Scheme A exactly).
Dims eff_dims(const lbm_ctx *c) {
    Dims d = c->dm;
    d.sb = c->dm.sb && (c->dm.src || c->rfield);
    return d;
}

bool remark3(const lbm_ctx *c) { return (c->desc.flags & LBM_FLAG_REMARK3) != 0; }

// The sweep needs the general kernel: per-node fields, Remark III, or Scheme B
// with a source outside the 3-term equal-rate kernels.
bool general_path(const lbm_ctx *c) {
    if (c->kfield || c->rfield || remark3(c)) return true;
    return eff_dims(c).sb && !(c->dm.eqr && c->dm.deg3 && c->dm.o32);
}

// The sweep reads and writes the phi history: a Scheme-A source (Remark III
// takes the general kernel and never runs two-step passes).
bool keeps_history(const lbm_ctx *c) { return c->dm.src && !c->dm.sb; }

// Calls the adjoint does not cover: Scheme B sources, fields, Remark III.
bool adjoint_refused(const lbm_ctx *c) { return eff_dims(c).sb || c->kfield || c->rfield || remark3(c); }

// Two-step passes can run: the run qualifies (Scheme B sources with 3-term
// polynomials) and, when it keeps a phi history, the caller bound the second
// history buffer.
bool two_ready(const lbm_ctx *c) {
    return c->two_ok && (!eff_dims(c).sb || c->dm.deg3) && (!keeps_history(c) || c->p2 != nullptr);
}

bool two_active(const lbm_ctx *c) { return c->two && two_ready(c) && !general_path(c); }

// Bytes of the second history buffer (0 when two-step passes never read one).
size_t hist2_bytes(const lbm_ctx *c) {
    return (c->two_ok && keeps_history(c)) ? round256((size_t)c->g.N * hist_size(c->dm.prec)) : 0;
}

// Four steps as two passes of two steps each: f[start] -> f[start ^ 1] with the
// history p -> p2, then back; state and history end where four single sweeps
// would leave them.
void query_cus(lbm_ctx *c) {
    if (c->ncu) return;
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
        c->ncu = n;
}

// Resident workgroups per CU of the D3Q19 pass in the current tile shape and
// the CU count, asked of the runtime once per shape (outside graph capture:
// lbm_init, lbm_set_two_step and lbm_tune call this before any pass).
void prepare_zchunk(lbm_ctx *c) {
    if (c->dm.q != 19 || !c->two_ok || c->two_shape < 0 || c->two_shape > 3) return;
    query_cus(c);
    if (!c->occ3[c->two_shape]) {
        int occ = 0;
        if (sweep2_q19_occupancy(eff_dims(c), c->g, c->two_shape, &occ) == hipSuccess && occ > 0)
            c->occ3[c->two_shape] = occ;
    }
}

// Tile shape of the two-sweep adjoint: 6 x 4, 10 x 4 or 10 x 12 (rows x
// waves).  Its workgroups run in rounds of (resident workgroups per CU) x
// CUs, and a partial last round costs a whole one.  10-row tiles recompute
// fewer halo rows but fit fewer workgroups per CU; they win where they need
// fewer rounds than 6-row tiles (512^2 FP64: 9.3 against 10.9 us per reversed
// sweep; 768^2 FP32: 9.5 against 10.0), and 6-row tiles win at equal rounds
// (1024^2 FP64: 34.7 against 36.8).  An FP32 launch too small to give every
// SIMD several waves (at most 6 waves per SIMD with 12 per 10-row tile) runs
// 10-row tiles with one row per wave when that at least halves the tiles
// per CU (512^2: 2 against 4; 5.3 against 6.1 us); with as many tiles per CU
// the 6-row tiles' smaller work per tile wins (384^2: 4.8 against 4.3 us).
// FP64, held to 2 or 3 waves per SIMD by its registers, gains nothing from
// the extra waves (512^2: 10.3 against 9.3).
void pick_adj_shape(lbm_ctx *c) {
    query_cus(c);
    c->adj_shape = 0;
    int occ6 = 0, occ10 = 0;
    if (c->ncu <= 0 || adjoint2_q9_occupancy(c->dm, c->g, 0, &occ6) != hipSuccess ||
        adjoint2_q9_occupancy(c->dm, c->g, 1, &occ10) != hipSuccess || occ6 <= 0 || occ10 <= 0) {
        c->adj_shape_auto = c->adj_shape;
        return;
    }
    auto tiles = [&](uint32_t th) { return (uint64_t)((c->g.nx + 61) / 62) * ((c->g.ny + th - 1) / th); };
    auto rounds = [&](uint32_t th, int occ) {
        const uint64_t slots = (uint64_t)occ * (uint64_t)c->ncu;
        return (tiles(th) + slots - 1) / slots;
    };
    if (rounds(10, occ10) < rounds(6, occ6)) c->adj_shape = 1;
    const uint64_t ncu = (uint64_t)c->ncu;
    const uint64_t per_cu6 = (tiles(6) + ncu - 1) / ncu, per_cu10 = (tiles(10) + ncu - 1) / ncu;
    if (c->dm.prec == 1 && tiles(10) * 12 <= 6 * 4 * ncu && 2 * per_cu10 <= per_cu6) c->adj_shape = 2;
    c->adj_shape_auto = c->adj_shape;
}

// z planes per column of the D3Q19 pass.  Each workgroup lives for its chunk
// of zc planes plus two, and one workgroup slot per CU (or a few) runs them
// in rounds, so the pass takes about ceil(workgroups / slots) * (zc + 2)
// plane-times: the chunk that minimises this fills the last round (256^3,
// FP32 14 x 16, one slot per CU: zc = 32 gives 760 workgroups in 2.97
// rounds, 52 GLUPS; zc = 24 gave 1045 in 4.08, i.e. five rounds, 44.5).
// Without the occupancy figures: about 1024 workgroups.
uint32_t zchunk(const lbm_ctx *c) {
    int rows = 0, waves = 0;
    if (!two_step3_shape_of(c->dm.prec, c->two_shape, &rows, &waves)) return c->g.nz;
    const uint64_t tiles_xy = (uint64_t)((c->g.nx + 61) / 62) * ((c->g.ny + (uint32_t)rows - 1) / (uint32_t)rows);
    const uint32_t nz = c->g.nz;
    const int occ = (c->two_shape >= 0 && c->two_shape < 4) ? c->occ3[c->two_shape] : 0;
    if (occ > 0 && c->ncu > 0) {
        const uint64_t slots = (uint64_t)occ * (uint64_t)c->ncu;
        uint32_t best_zc = nz;
        uint64_t best = ~0ull;
        for (uint32_t zc = 1; zc <= nz; ++zc) {
            const uint64_t tz = (nz + zc - 1) / zc;
            if (zc > 1 && (nz + zc - 2) / (zc - 1) == tz) continue;   // same chunk count as zc - 1
            const uint64_t rounds = (tiles_xy * tz + slots - 1) / slots;
            const uint64_t cost = rounds * (zc + 2);
            if (cost < best) { best = cost; best_zc = zc; }
        }
        return best_zc;
    }
    uint64_t tiles_z = (1024 + tiles_xy - 1) / tiles_xy;
    if (tiles_z > nz) tiles_z = nz;
    if (tiles_z < 1) tiles_z = 1;
    return (uint32_t)((nz + tiles_z - 1) / tiles_z);
}

// Without a source the kernels touch no history, and p stands in for p2.
hipError_t sweep_pair(lbm_ctx *c, int start, hipStream_t st) {
    void *p2 = keeps_history(c) ? c->p2 : c->p;
    if (c->dm.q == 19) {
        const uint32_t zc = zchunk(c);
        const Dims d = eff_dims(c);
        hipError_t e = launch_sweep2_q19(d, c->g, c->d_coefs, c->f[start], c->f[start ^ 1], c->p, p2, c->d_flag,
                                         c->two_shape, zc, st);
        if (e == hipSuccess)
            e = launch_sweep2_q19(d, c->g, c->d_coefs, c->f[start ^ 1], c->f[start], p2, c->p, c->d_flag,
                                  c->two_shape, zc, st);
        return e;
    }
    const Dims d = eff_dims(c);
    hipError_t e = launch_sweep2_q9(d, c->g, c->d_coefs, c->f[start], c->f[start ^ 1], c->p, p2, c->d_flag,
                                    c->two_shape, st);
    if (e == hipSuccess)
        e = launch_sweep2_q9(d, c->g, c->d_coefs, c->f[start ^ 1], c->f[start], p2, c->p, c->d_flag,
                             c->two_shape, st);
    return e;
}

hipError_t sweep(lbm_ctx *c, const void *fin, void *fout, void *p, hipStream_t st) {
    const Dims d = eff_dims(c);
    if (general_path(c))
        return c->dm.q == 9 ? launch_sweep_gen_q9(d, c->g, c->d_coefs, fin, fout, p, c->d_flag, c->kfield, c->rfield,
                                                  remark3(c), st)
                            : launch_sweep_gen_q19(d, c->g, c->d_coefs, fin, fout, p, c->d_flag, c->kfield, c->rfield,
                                                   remark3(c), st);
    return c->dm.q == 9 ? launch_sweep_q9(d, c->g, c->d_coefs, fin, fout, p, c->d_flag, st)
                        : launch_sweep_q19(d, c->g, c->d_coefs, fin, fout, p, c->d_flag, st);
}

void drop_graphs(lbm_ctx *c) {
    for (int i = 0; i < 2; ++i)
        if (c->gexec[i]) { (void)hipGraphExecDestroy(c->gexec[i]); c->gexec[i] = nullptr; }
}

// kGraphSteps sweeps starting from buffer `start`, as one executable graph.
hipError_t make_graph(lbm_ctx *c, int start) {
    hipError_t e = hipSuccess;
    if (!c->cap) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    int cur = start;
    hipError_t le = hipSuccess;
    if (two_active(c)) {
        for (int i = 0; i < kGraphSteps / 4 && le == hipSuccess; ++i) le = sweep_pair(c, start, c->cap);
    } else {
        for (int i = 0; i < kGraphSteps && le == hipSuccess; ++i) {
            le = sweep(c, c->f[cur], c->f[cur ^ 1], c->p, c->cap);
            cur ^= 1;
        }
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(c->cap, &graph);
    if (le != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return le; }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&c->gexec[start], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return e;
}

// Re-centre the stored offsets of the current state on the mean of phi
// (device-side: no host synchronisation, so it may sit between graph launches).
hipError_t recenter(lbm_ctx *c, hipStream_t st) {
    int parts = (int)std::min<uint32_t>(kRedParts, c->g.nblocks);
    if (parts < 1) parts = 1;
    const Dims d = eff_dims(c);
    hipError_t e = c->dm.q == 9
                       ? launch_recenter_q9(d, c->g, c->d_coefs, c->f[c->cur], c->p, c->d_red_part, parts,
                                            c->d_shift, st)
                       : launch_recenter_q19(d, c->g, c->d_coefs, c->f[c->cur], c->p, c->d_red_part, parts,
                                             c->d_shift, st);
    if (e == hipSuccess) c->recentered = true;
    return e;
}

// Reads the divergence flag (a host wait): LBM_E_DIVERGED once any sweep has
// met a non-finite phi.
int check_flag(lbm_ctx *c, hipStream_t st) {
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "divergence check");
    if (flag) {
        char buf[96];
        std::snprintf(buf, sizeof(buf), "non-finite phi by step %lld", c->t);
        return fail(LBM_E_DIVERGED, buf);
    }
    return LBM_OK;
}

// n sweeps from the current buffer: whole graphs of kGraphSteps sweeps, then
// pairs of two-step passes where they apply, then single launches.  With the
// divergence check (every k steps) the steps run in chunks that end on the
// multiples of k, passes and single sweeps within a chunk, and the flag is
// read at the end of each chunk that reaches a multiple.
int advance(lbm_ctx *c, int nsteps, hipStream_t st) {
    if (c->check_every > 0) {
        while (nsteps > 0) {
            int chunk = c->check_every - (int)(c->t % c->check_every);
            if (chunk > nsteps) chunk = nsteps;
            nsteps -= chunk;
            while (two_active(c) && chunk >= 4) {
                hipError_t e = sweep_pair(c, c->cur, st);
                if (e != hipSuccess) return hip_fail(e, "two-step sweep kernel");
                c->t += 4;
                chunk -= 4;
            }
            for (; chunk > 0; --chunk) {
                hipError_t e = sweep(c, c->f[c->cur], c->f[c->cur ^ 1], c->p, st);
                if (e != hipSuccess) return hip_fail(e, "sweep kernel");
                c->cur ^= 1;
                ++c->t;
            }
            if (c->t % c->check_every == 0) {
                const int rc = check_flag(c, st);
                if (rc != LBM_OK) return rc;
            }
        }
        return LBM_OK;
    }
    const bool graphs = !(c->desc.flags & LBM_FLAG_NO_GRAPH) && c->use_graphs;
    while (graphs && nsteps >= kGraphSteps) {
        if (!c->gexec[c->cur]) {
            hipError_t e = make_graph(c, c->cur);
            if (e != hipSuccess) return hip_fail(e, "graph capture");
        }
        hipError_t e = hipGraphLaunch(c->gexec[c->cur], st);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        c->t += kGraphSteps;
        nsteps -= kGraphSteps;
    }
    while (two_active(c) && nsteps >= 4) {
        hipError_t e = sweep_pair(c, c->cur, st);
        if (e != hipSuccess) return hip_fail(e, "two-step sweep kernel");
        c->t += 4;
        nsteps -= 4;
    }
    for (int i = 0; i < nsteps; ++i) {
        hipError_t e = sweep(c, c->f[c->cur], c->f[c->cur ^ 1], c->p, st);
        if (e != hipSuccess) return hip_fail(e, "sweep kernel");
        c->cur ^= 1;
        ++c->t;
    }
    return LBM_OK;
}

}  // namespace

namespace lbm {

// Validation and packed constants of one description (used by the batch API).
int derive_coefs(const lbm_desc *d, int *prec, bool *eqr, bool *src, bool *kvar, bool *lowdeg, bool *deg3,
                 void *coefs_out, size_t *coef_bytes) {
    Dims dm;
    const int rc = validate(d, dm);
    if (rc != LBM_OK) return rc;
    HostModel m;
    derive(*d, dm, m);
    if (dm.prec == 0) {
        Coefs<double> cf;
        pack(m, cf);
        std::memcpy(coefs_out, &cf, sizeof(cf));
        *coef_bytes = sizeof(cf);
    } else {
        Coefs<float> cf;
        pack(m, cf);
        std::memcpy(coefs_out, &cf, sizeof(cf));
        *coef_bytes = sizeof(cf);
    }
    *prec = dm.prec;
    *eqr = dm.eqr;
    *src = dm.src;
    *kvar = dm.kvar;
    *lowdeg = dm.lowdeg;
    *deg3 = dm.deg3;
    return LBM_OK;
}

int api_fail(int code, const char *msg) { return fail(code, msg); }

}  // namespace lbm

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

int lbm_create(const lbm_desc *desc, lbm_ctx **out) {
    if (!out) return fail(LBM_E_INVALID, "null output pointer");
    Dims dm;
    int rc = validate(desc, dm);
    if (rc != LBM_OK) return rc;
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_E_INVALID, "out of host memory");
    c->desc = *desc;
    c->dm = dm;
    Geom &g = c->g;
    g.nx = desc->nx; g.ny = desc->ny; g.nz = desc->nz;
    g.N = (uint32_t)((size_t)desc->nx * desc->ny * desc->nz);
    g.plane = plane_stride(g.N, dm.q, storage_size(dm.prec), desc->plane_pad);
    g.fx.set(g.nx);
    g.fxy.set(g.nx * g.ny);
    g.nblocks = (g.N + kBlock - 1) / kBlock;
    g.chunk = 1;
    g.remap = (desc->flags & LBM_FLAG_NO_XCD_REMAP) ? 0 : 1;
    {
        // When the two distribution buffers and the history exceed the 256 MB
        // Infinity Cache: streaming (non-temporal) accesses, and the hardware's
        // round-robin workgroup order, which spreads HBM traffic better than
        // one slab per XCD (D3Q19 256^3 FP32: 5.73 against 5.33 TB/s).  A
        // cache-resident state keeps the slab order, whose neighbour rows stay
        // in one XCD's L2 (1024^2 FP32: 5.88 against 5.55 TB/s).
        const double bytes = 2.0 * dm.q * (double)g.plane * storage_size(dm.prec) + (double)g.N * hist_size(dm.prec);
        c->dm.nt = bytes > 256.0 * 1024 * 1024;
        if (c->dm.nt) g.remap = 0;
    }
    // every array a kernel indexes (planes of f and psi, p, pi: at most 8-byte
    // elements, at most `plane` of them) spans < 4 GiB: 32-bit byte offsets
    c->dm.o32 = (uint64_t)g.plane * 8u < (1ull << 32);
    // two steps per pass: D2Q9 runs (with walls on y or unequal non-flux
    // rates: 3-term polynomials); D3Q19 runs with 3-term polynomials (walls
    // on z allowed)
    c->two_ok = (dm.q == 9 && ((dm.eqr && !dm.wall) || dm.deg3) && c->dm.o32) ||
                (dm.q == 19 && dm.deg3 && c->dm.o32);
    c->two = c->two_ok;   // on by default where it applies (bit-identical; lbm_tune re-decides)
    {
        // the two-sweep adjoint: periodic D2Q9 only; its partial slots cover
        // the 6-row tiling, the finer of the two
        const uint32_t tiles = ((g.nx + 61) / 62) * ((g.ny + 5) / 6);
        c->adj_slots = dm.q == 9 && !dm.wall && dm.eqr && c->two_ok && tiles > g.nblocks ? tiles : g.nblocks;
        if (dm.q == 9 && !dm.wall && dm.eqr && c->two_ok && dm.prec != 2) pick_adj_shape(c);
    }
    hipError_t e = hipMalloc(&c->d_coefs, sizeof(Coefs<double>));
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipMalloc(coefficients)"); }
    const size_t scratch = 256 + sizeof(double) * (size_t)(kRedParts * 8 + 8 + kMaxAdjParts * kAdjWidth + 16);
    e = hipMalloc(&c->d_scratch, scratch);
    if (e != hipSuccess) { (void)hipFree(c->d_coefs); delete c; return hip_fail(e, "hipMalloc(scratch)"); }
    char *base = (char *)c->d_scratch;
    c->d_flag = (int *)base;
    c->d_red_part = (double *)(base + 256);
    c->d_red_out = c->d_red_part + kRedParts * 8;
    c->d_adj_part = c->d_red_out + 8;
    c->d_k0acc = c->d_adj_part + (size_t)kMaxAdjParts * kAdjWidth;
    c->d_shift = c->d_k0acc + 8;
    // a source moves the whole field away from phi_ref; without one the mean
    // drifts only through walls and centring on it can enlarge the stored values
    c->recenter_every = (dm.prec == 2 && dm.src) ? kRecenterF16 : 0;
    e = hipMemset(c->d_scratch, 0, scratch);
    if (e != hipSuccess) { lbm_destroy(c); return hip_fail(e, "hipMemset(scratch)"); }
    rc = upload_coefs(c);
    if (rc != LBM_OK) { lbm_destroy(c); return rc; }
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->d_coefs) (void)hipFree(c->d_coefs);
    if (c->d_scratch) (void)hipFree(c->d_scratch);
    delete c;
}

int lbm_state_bytes(const lbm_ctx *c, size_t *f_bytes, size_t *p_bytes, size_t *p2_bytes) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (f_bytes) *f_bytes = round256((size_t)c->dm.q * c->g.plane * storage_size(c->dm.prec));
    if (p_bytes) *p_bytes = round256((size_t)c->g.N * hist_size(c->dm.prec));
    if (p2_bytes) *p2_bytes = hist2_bytes(c);
    return LBM_OK;
}

int lbm_adjoint_bytes(const lbm_ctx *c, size_t *psi_bytes) {
    if (!c || !psi_bytes) return fail(LBM_E_INVALID, "null argument");
    *psi_bytes = round256((size_t)c->dm.q * c->g.plane * (c->dm.prec == 0 ? 8 : 4));
    return LBM_OK;
}

int lbm_init(lbm_ctx *c, const double *phi0, void *f_a, void *f_b, void *p, void *p2, void *stream) {
    if (!c || !phi0 || !f_a || !f_b || !p) return fail(LBM_E_INVALID, "null argument");
    if (f_a == f_b) return fail(LBM_E_INVALID, "the two distribution buffers must differ");
    if (((uintptr_t)f_a | (uintptr_t)f_b | (uintptr_t)p | (uintptr_t)p2) & 255)
        return fail(LBM_E_INVALID, "buffers must be 256-byte aligned");
    if (p2 && (p2 == p || p2 == f_a || p2 == f_b))
        return fail(LBM_E_INVALID, "the second history buffer must differ from the other buffers");
    if (hist2_bytes(c) == 0) p2 = nullptr;   // never read: keep no pointer to it
    if (c->f[0] != f_a || c->f[1] != f_b || c->p != p || c->p2 != p2) drop_graphs(c);
    c->f[0] = f_a; c->f[1] = f_b; c->p = p; c->p2 = p2; c->phi0 = phi0;
    c->cur = 0; c->t = 0; c->bound = true;
    hipStream_t st = (hipStream_t)stream;
    if (c->recentered) {
        // back to the description's phi_ref (the host copy was never changed)
        hipError_t e = hipMemcpyAsync(c->d_coefs, c->host_coefs, c->coef_bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(coefficients)");
        c->recentered = false;
    }
    const Dims d = eff_dims(c);
    hipError_t e = (c->dm.q == 9) ? launch_init_q9(d, c->g, c->d_coefs, phi0, f_a, p, c->rfield, st)
                                  : launch_init_q19(d, c->g, c->d_coefs, phi0, f_a, p, c->rfield, st);
    if (e != hipSuccess) return hip_fail(e, "init kernel");
    // a fill kernel, not a memset node, in case the caller captures this call
    e = launch_zero((double *)c->d_flag, 1, st);
    if (e != hipSuccess) return hip_fail(e, "flag reset");
    prepare_zchunk(c);
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int nsteps, void *stream) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (!c->bound) return fail(LBM_E_STATE, "lbm_init has not been called");
    if (nsteps < 0) return fail(LBM_E_INVALID, "negative step count");
    hipStream_t st = (hipStream_t)stream;
    while (nsteps > 0) {
        int n = nsteps;
        const int K = c->recenter_every;
        if (K > 0) {
            const long long left = K - (c->t % K);
            if (left < n) n = (int)left;
        }
        const int rc = advance(c, n, st);
        if (rc != LBM_OK) return rc;
        nsteps -= n;
        if (K > 0 && c->t % K == 0) {
            hipError_t e = recenter(c, st);
            if (e != hipSuccess) return hip_fail(e, "re-centring kernels");
        }
    }
    return LBM_OK;
}

int lbm_recenter(lbm_ctx *c, void *stream) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (!c->bound) return fail(LBM_E_STATE, "lbm_init has not been called");
    hipError_t e = recenter(c, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "re-centring kernels");
    return LBM_OK;
}

// a tile shape usable here: in the table, 3-term polynomials for the
// non-default shapes (tiles wrap periodically, so any grid size will do)
static bool shape_of(const lbm_ctx *c, int shape, int *rows, int *waves) {
    return c->dm.q == 9 ? two_step_shape_of(c->dm.prec, shape, rows, waves)
                        : two_step3_shape_of(c->dm.prec, shape, rows, waves);
}

static bool two_shape_usable(const lbm_ctx *c, int shape) {
    int rows = 0, waves = 0;
    if (!shape_of(c, shape, &rows, &waves)) return false;
    // the moment-space collision (unequal rates) has the default shape only
    return shape == 0 || (c->dm.deg3 && c->dm.eqr);
}

int lbm_two_step_shape(const lbm_ctx *c, int shape, int *rows, int *waves) {
    if (!c || !rows || !waves) return fail(LBM_E_INVALID, "null argument");
    if (!shape_of(c, shape, rows, waves)) return fail(LBM_E_INVALID, "no such tile shape");
    return LBM_OK;
}

int lbm_set_two_step(lbm_ctx *c, int mode) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (mode < 0) return fail(LBM_E_INVALID, "mode must be 0 (off) or 1 + a tile shape");
    if (mode && !c->two_ok)
        return fail(LBM_E_UNSUPPORTED,
                    "two steps per pass need 32-bit offsets and, on D3Q19 and with walls or unequal rates on "
                    "D2Q9, polynomials of degree <= 2");
    if (mode && eff_dims(c).sb && !c->dm.deg3)
        return fail(LBM_E_UNSUPPORTED, "two steps per pass with a Scheme-B source need polynomials of degree <= 2");
    if (mode && c->bound && keeps_history(c) && !c->p2)
        return fail(LBM_E_STATE, "two steps per pass with a source need the second history buffer (lbm_init p2)");
    const int shape = mode > 0 ? mode - 1 : 0;
    if (mode && !two_shape_usable(c, shape))
        return fail(LBM_E_INVALID, "tile shape not available for this storage type or polynomial length");
    drop_graphs(c);
    c->two = mode != 0;
    c->two_shape = shape;
    prepare_zchunk(c);
    return LBM_OK;
}

int lbm_set_recenter(lbm_ctx *c, int every) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (every < 0) return fail(LBM_E_INVALID, "negative re-centring interval");
    c->recenter_every = every;
    return LBM_OK;
}

int lbm_set_phi_wall(lbm_ctx *c, double phi_lo, double phi_hi, void *stream) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (!c->dm.wall) return fail(LBM_E_INVALID, "the description has no walls");
    if (!std::isfinite(phi_lo) || !std::isfinite(phi_hi)) return fail(LBM_E_INVALID, "non-finite wall value");
    const int la = (c->dm.q == 9 ? 2 : 3) - 1;
    c->desc.phi_wall[la][0] = phi_lo;
    c->desc.phi_wall[la][1] = phi_hi;
    HostModel m;
    pack_host(c, m);   // the host copy (restored by lbm_init) carries the new values too
    double ewp[2 * 19];
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < 19; ++k) ewp[s * 19 + k] = m.ewp[s][k];
    hipError_t e = c->dm.q == 9 ? launch_set_wall_q9(c->dm, c->d_coefs, ewp, (hipStream_t)stream)
                                : launch_set_wall_q19(c->dm, c->d_coefs, ewp, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "wall kernel");
    return LBM_OK;
}

int lbm_set_fields(lbm_ctx *c, const double *k0_field, const double *r_field) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (((uintptr_t)k0_field | (uintptr_t)r_field) & 7) return fail(LBM_E_INVALID, "fields must be 8-byte aligned");
    if (r_field && !c->dm.sb)
        return fail(LBM_E_UNSUPPORTED, "an external source field needs Scheme B (Scheme A would also need R(t - 1))");
    if (k0_field != c->kfield || r_field != c->rfield) drop_graphs(c);
    c->kfield = k0_field;
    c->rfield = r_field;
    return LBM_OK;
}

int lbm_sweep(lbm_ctx *c, const void *f_in, void *f_out, void *p, void *stream) {
    if (!c || !f_in || !f_out || !p) return fail(LBM_E_INVALID, "null argument");
    if (f_in == f_out) return fail(LBM_E_INVALID, "f_in and f_out must differ");
    hipError_t e = sweep(c, f_in, f_out, p, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sweep kernel");
    return LBM_OK;
}

int lbm_phi_of(lbm_ctx *c, const void *f, double *phi, void *stream) {
    if (!c || !f || !phi) return fail(LBM_E_INVALID, "null argument");
    const Dims d = eff_dims(c);
    hipError_t e = (c->dm.q == 9) ? launch_phi_q9(d, c->g, c->d_coefs, f, phi, c->rfield, (hipStream_t)stream)
                                  : launch_phi_q19(d, c->g, c->d_coefs, f, phi, c->rfield, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "phi kernel");
    return LBM_OK;
}

int lbm_get_phi(lbm_ctx *c, double *phi, void *stream) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (!c->bound) return fail(LBM_E_STATE, "lbm_init has not been called");
    return lbm_phi_of(c, c->f[c->cur], phi, stream);
}

int lbm_current(const lbm_ctx *c, void **f, void **p, long long *t) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (!c->bound) return fail(LBM_E_STATE, "lbm_init has not been called");
    if (f) *f = c->f[c->cur];
    if (p) *p = c->p;
    if (t) *t = c->t;
    return LBM_OK;
}

int lbm_set_current(lbm_ctx *c, int which, long long t) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (!c->bound) return fail(LBM_E_STATE, "lbm_init has not been called");
    if (which != 0 && which != 1) return fail(LBM_E_INVALID, "which must be 0 or 1");
    c->cur = which;
    c->t = t;
    return LBM_OK;
}

int lbm_set_check(lbm_ctx *c, int every) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (every < 0) return fail(LBM_E_INVALID, "negative check interval");
    c->check_every = every;
    return LBM_OK;
}

int lbm_set_k0(lbm_ctx *c, const double k0[9]) {
    if (!c || !k0) return fail(LBM_E_INVALID, "null argument");
    if (c->recentered) return fail(LBM_E_STATE, "offsets were re-centred: call lbm_init before lbm_set_k0");
    lbm_desc d = c->desc;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) d.k0[a][b] = k0[a * 3 + b];
    Dims dm;
    int rc = validate(&d, dm);
    if (rc != LBM_OK) return rc;
    c->desc = d;
    return upload_coefs(c);
}

int lbm_reduce(lbm_ctx *c, const double *phi, const double *ref, double out[8], void *stream) {
    if (!c || !phi || !out) return fail(LBM_E_INVALID, "null argument");
    hipStream_t st = (hipStream_t)stream;
    int parts = (int)std::min<uint32_t>(kRedParts, (c->g.N + kBlock - 1) / kBlock);
    if (parts < 1) parts = 1;
    hipError_t e = launch_reduce(phi, ref, c->g.N, c->d_red_part, parts, c->d_red_out, st);
    if (e == hipSuccess) e = hipMemcpyAsync(out, c->d_red_out, 8 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reduction");
    return LBM_OK;
}

int lbm_reduce_async(lbm_ctx *c, const double *phi, const double *ref, double *out_dev, void *stream) {
    if (!c || !phi || !out_dev) return fail(LBM_E_INVALID, "null argument");
    int parts = (int)std::min<uint32_t>(kRedParts, (c->g.N + kBlock - 1) / kBlock);
    if (parts < 1) parts = 1;
    const hipError_t e = launch_reduce(phi, ref, c->g.N, c->d_red_part, parts, out_dev, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "reduction");
    return LBM_OK;
}

int lbm_reduce_state(lbm_ctx *c, const double *ref, double *out_dev, void *stream) {
    if (!c || !out_dev) return fail(LBM_E_INVALID, "null argument");
    if (!c->bound) return fail(LBM_E_STATE, "lbm_init has not been called");
    int parts = (int)std::min<uint32_t>(kRedParts, (c->g.N + kBlock - 1) / kBlock);
    if (parts < 1) parts = 1;
    const Dims d = eff_dims(c);
    const hipStream_t st = (hipStream_t)stream;
    const hipError_t e =
        c->dm.q == 9
            ? launch_phi_reduce_q9(d, c->g, c->d_coefs, c->f[c->cur], ref, c->rfield, c->d_red_part, parts, out_dev, st)
            : launch_phi_reduce_q19(d, c->g, c->d_coefs, c->f[c->cur], ref, c->rfield, c->d_red_part, parts, out_dev,
                                    st);
    if (e != hipSuccess) return hip_fail(e, "state reduction");
    return LBM_OK;
}

int lbm_adjoint_seed(lbm_ctx *c, const double *gphi, void *psi, double *pi, void *stream) {
    if (!c || !gphi || !psi || !pi) return fail(LBM_E_INVALID, "null argument");
    if (c->dm.prec == 2) return fail(LBM_E_UNSUPPORTED, "no adjoint for FP16 storage");
    if (adjoint_refused(c)) return fail(LBM_E_UNSUPPORTED, "no adjoint for Scheme B sources, per-node fields or Remark III");
    if (c->recentered)
        return fail(LBM_E_STATE, "offsets were re-centred during the forward run; the adjoint needs a fixed phi_ref");
    hipStream_t st = (hipStream_t)stream;
    if (c->adj_slots > (uint32_t)kMaxAdjParts) return fail(LBM_E_UNSUPPORTED, "grid too large for the adjoint partials");
    hipError_t e = c->dm.q == 9 ? launch_seed_q9(c->dm, c->g, gphi, psi, pi, st)
                                : launch_seed_q19(c->dm, c->g, gphi, psi, pi, st);
    if (e == hipSuccess) e = launch_zero(c->d_adj_part, c->adj_slots * kAdjWidth, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint seed");
    return LBM_OK;
}

int lbm_adjoint_step(lbm_ctx *c, const void *f_s, const void *p_s, const void *psi_next,
                     const double *pi_next, void *psi_out, double *pi_out, void *stream) {
    if (!c || !f_s || !p_s || !psi_next || !pi_next || !psi_out || !pi_out)
        return fail(LBM_E_INVALID, "null argument");
    if (psi_next == psi_out) return fail(LBM_E_INVALID, "psi_next and psi_out must differ");
    if (c->dm.prec == 2) return fail(LBM_E_UNSUPPORTED, "no adjoint for FP16 storage");
    if (adjoint_refused(c)) return fail(LBM_E_UNSUPPORTED, "no adjoint for Scheme B sources, per-node fields or Remark III");
    if (c->recentered)
        return fail(LBM_E_STATE, "offsets were re-centred during the forward run; the adjoint needs a fixed phi_ref");
    if (c->adj_slots > (uint32_t)kMaxAdjParts) return fail(LBM_E_UNSUPPORTED, "grid too large for the adjoint partials");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = c->dm.q == 9 ? launch_adjoint_q9(c->dm, c->g, c->d_coefs, f_s, p_s, psi_next, pi_next, psi_out,
                                                    pi_out, c->d_adj_part, st)
                                : launch_adjoint_q19(c->dm, c->g, c->d_coefs, f_s, p_s, psi_next, pi_next, psi_out,
                                                     pi_out, c->d_adj_part, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel");
    return LBM_OK;
}

// Two reversed sweeps per launch: the forward pass's tile conditions.
static bool adjoint_pair_applies(const lbm_ctx *c) {
    return c->dm.q == 9 && !c->dm.wall && c->dm.eqr && c->two_ok && c->dm.prec != 2 &&
           c->adj_slots <= (uint32_t)kMaxAdjParts;
}

int lbm_adjoint_pair_ok(const lbm_ctx *c, int *ok) {
    if (!c || !ok) return fail(LBM_E_INVALID, "null argument");
    *ok = adjoint_pair_applies(c) && !adjoint_refused(c) ? 1 : 0;
    return LBM_OK;
}

int lbm_adjoint_tile_shape(const lbm_ctx *c, int shape, int *rows, int *waves) {
    if (!c || !rows || !waves) return fail(LBM_E_INVALID, "null argument");
    if (!adjoint2_shape_of(shape, rows, waves)) return fail(LBM_E_INVALID, "no such adjoint tile shape");
    return LBM_OK;
}

int lbm_set_adjoint_tile(lbm_ctx *c, int mode) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    int rows = 0, waves = 0;
    if (mode < 0 || (mode > 0 && !adjoint2_shape_of(mode - 1, &rows, &waves)))
        return fail(LBM_E_INVALID, "mode must be 0 (the pick) or 1 + an adjoint tile shape");
    c->adj_shape = mode == 0 ? c->adj_shape_auto : mode - 1;
    return LBM_OK;
}

int lbm_adjoint_tile(const lbm_ctx *c, int *shape) {
    if (!c || !shape) return fail(LBM_E_INVALID, "null argument");
    *shape = c->adj_shape;
    return LBM_OK;
}

int lbm_adjoint_step2(lbm_ctx *c, const void *f_s, const void *p_s, const void *f_sm1, const void *p_sm1,
                      const void *psi_next, const double *pi_next, void *psi_out, double *pi_out, void *stream) {
    if (!c || !f_s || !p_s || !f_sm1 || !p_sm1 || !psi_next || !pi_next || !psi_out || !pi_out)
        return fail(LBM_E_INVALID, "null argument");
    if (psi_next == psi_out) return fail(LBM_E_INVALID, "psi_next and psi_out must differ");
    if ((const void *)pi_next == (const void *)pi_out)
        return fail(LBM_E_INVALID, "pi_next and pi_out must differ for two sweeps per launch");
    if (c->dm.prec == 2) return fail(LBM_E_UNSUPPORTED, "no adjoint for FP16 storage");
    if (adjoint_refused(c)) return fail(LBM_E_UNSUPPORTED, "no adjoint for Scheme B sources, per-node fields or Remark III");
    if (c->recentered)
        return fail(LBM_E_STATE, "offsets were re-centred during the forward run; the adjoint needs a fixed phi_ref");
    if (!adjoint_pair_applies(c))
        return fail(LBM_E_UNSUPPORTED,
                    "two reversed sweeps per launch need D2Q9, periodic axes and equal rates");
    hipError_t e = launch_adjoint2_q9(c->dm, c->g, c->d_coefs, f_s, p_s, f_sm1, p_sm1, psi_next, pi_next, psi_out,
                                      pi_out, c->d_adj_part, c->adj_shape, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint pair kernel");
    return LBM_OK;
}

int lbm_adjoint_init(lbm_ctx *c, const double *phi0, const void *psi0, const double *pi0, double *gphi0,
                     void *stream) {
    if (!c || !phi0 || !psi0 || !pi0 || !gphi0) return fail(LBM_E_INVALID, "null argument");
    if (c->dm.prec == 2) return fail(LBM_E_UNSUPPORTED, "no adjoint for FP16 storage");
    if (adjoint_refused(c)) return fail(LBM_E_UNSUPPORTED, "no adjoint for Scheme B sources, per-node fields or Remark III");
    if (c->recentered)
        return fail(LBM_E_STATE, "offsets were re-centred during the forward run; the adjoint needs a fixed phi_ref");
    hipError_t e = c->dm.q == 9
                       ? launch_adjoint_init_q9(c->dm, c->g, c->d_coefs, phi0, psi0, pi0, gphi0, (hipStream_t)stream)
                       : launch_adjoint_init_q19(c->dm, c->g, c->d_coefs, phi0, psi0, pi0, gphi0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint init kernel");
    return LBM_OK;
}

int lbm_adjoint_grad_k0(lbm_ctx *c, double out[6], void *stream) {
    if (!c || !out) return fail(LBM_E_INVALID, "null argument");
    hipStream_t st = (hipStream_t)stream;
    double acc[6];
    // fold the per-workgroup slots (fixed order: deterministic)
    hipError_t e = launch_zero(c->d_k0acc, 8, st);
    if (e == hipSuccess) e = launch_sum_partials(c->d_adj_part, (int)c->adj_slots, kAdjWidth, c->d_k0acc, st);
    if (e == hipSuccess) e = hipMemcpyAsync(acc, c->d_k0acc, 6 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "adjoint gradient copy");
    // kernel order (xx, yy, zz, xy, yz, xz) -> ABI order (xx, xy, yy, xz, yz, zz)
    out[0] = acc[0]; out[1] = acc[3]; out[2] = acc[1]; out[3] = acc[5]; out[4] = acc[4]; out[5] = acc[2];
    return LBM_OK;
}

int lbm_set_nontemporal(lbm_ctx *c, int on) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    c->dm.nt = on != 0;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_set_remap(lbm_ctx *c, int on) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    c->g.remap = on ? 1u : 0u;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_set_chunk(lbm_ctx *c, int chunk) {
    if (!c || chunk < 1) return fail(LBM_E_INVALID, "chunk must be >= 1");
    c->g.chunk = (uint32_t)chunk;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_tune(lbm_ctx *c, int reps, void *stream, char *report, size_t report_len) {
    if (!c) return fail(LBM_E_INVALID, "null context");
    if (!c->bound || !c->phi0) return fail(LBM_E_STATE, "lbm_init has not been called");
    if (reps < 1) reps = 1;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(LBM_E_HIP, "hipEventCreate");
    static const int cands[] = {1, 2, 4, 8, 16};
    float best = 1e30f;
    int best_chunk = 1;
    bool best_nt = c->dm.nt;
    uint32_t best_remap = c->g.remap;
    std::string rep;
    const int nts = (c->dm.eqr && c->dm.lowdeg) ? 2 : 1;
    // XCD order: contiguous slab per XCD, or the hardware's round-robin order
    // (LBM_FLAG_NO_XCD_REMAP pins the latter)
    const int remaps = (c->desc.flags & LBM_FLAG_NO_XCD_REMAP) ? 1 : 2;
    for (int ci = 0; ci < 5 * nts * remaps; ++ci) {
        const int ch = cands[ci % 5];
        if ((uint32_t)ch > c->g.nblocks) continue;
        c->g.chunk = (uint32_t)ch;
        c->dm.nt = ((ci / 5) % nts) == 1;
        c->g.remap = (remaps == 2 && ci / (5 * nts) == 0) ? 1u : 0u;
        // trial sweeps read the current state and write the other buffer
        hipError_t e = sweep(c, c->f[c->cur], c->f[c->cur ^ 1], c->p, st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = sweep(c, c->f[c->cur], c->f[c->cur ^ 1], c->p, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
            return hip_fail(e, "tuning sweep");
        }
        ms /= reps;
        char line[96];
        std::snprintf(line, sizeof(line), "chunk %d nt %d remap %u: %.4f ms\n", ch, (int)c->dm.nt, c->g.remap, ms);
        rep += line;
        if (ms < best) { best = ms; best_chunk = ch; best_nt = c->dm.nt; best_remap = c->g.remap; }
    }
    // two steps per pass: time pairs of passes (four steps), per step
    bool best_two = false;
    int best_shape = 0;
    c->g.chunk = (uint32_t)best_chunk;
    c->dm.nt = best_nt;
    if (two_ready(c) && !general_path(c)) {
        // four steps per pair; twice the steps of a single-sweep trial, as the
        // shapes differ by a few per cent
        const int pair_reps = std::max(2, reps / 2);
        // shapes in order of preference (FP32 1024^2: 14 x 8 and 6 x 4 within 1%,
        // 14 x 4 4% and 10 x 6 5% slower; FP64: 6 x 4 and 6 x 8 within 3%); a
        // later shape must be 2% faster to replace an earlier one, so
        // near-ties resolve the same way in every run.  Every candidate is
        // timed twice, in two passes over the list, and keeps its better time.
        // FP64 14 x 16 (lbm_set_two_step shape 2) is left out: it won short
        // trials on some boxes and then ran 12% slower than 6 x 4 over 5000
        // steps (61.5 against 70 GLUPS on 1024^2).
        static const int order4[4] = {1, 3, 0, 2}, order8[2] = {0, 1}, order3[3] = {0, 1, 2};
        const int *order = c->dm.q == 19 ? order3 : (c->dm.prec == 0 ? order8 : order4);
        const int nshape = c->dm.q == 19 ? (c->dm.prec == 0 ? 2 : 3) : (c->dm.prec == 0 ? 2 : 4);
        float tms[4][2];
        for (int ri = 0; ri < remaps * nshape; ++ri) tms[ri / remaps][ri % remaps] = -1.f;
        for (int pass = 0; pass < 2; ++pass) {
            for (int ri = 0; ri < remaps * nshape; ++ri) {
                const int shape = order[ri / remaps];
                if (!two_shape_usable(c, shape)) continue;
                c->two_shape = shape;
                prepare_zchunk(c);
                c->g.remap = (remaps == 2 && ri % remaps == 0) ? 1u : 0u;
                hipError_t e = sweep_pair(c, c->cur, st);
                if (e == hipSuccess) e = hipEventRecord(e0, st);
                for (int r = 0; r < pair_reps && e == hipSuccess; ++r) e = sweep_pair(c, c->cur, st);
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
                    return hip_fail(e, "tuning two-step sweep");
                }
                ms /= 4 * pair_reps;
                float &t = tms[ri / remaps][ri % remaps];
                if (t < 0.f || ms < t) t = ms;
            }
        }
        float best_two_ms = 1e30f;
        for (int ri = 0; ri < remaps * nshape; ++ri) {
            const int shape = order[ri / remaps];
            const float ms = tms[ri / remaps][ri % remaps];
            if (ms < 0.f) continue;
            const uint32_t remap = (remaps == 2 && ri % remaps == 0) ? 1u : 0u;
            int rows = 0, waves = 0;
            shape_of(c, shape, &rows, &waves);
            char line[112];
            std::snprintf(line, sizeof(line), "two steps per pass rows %d waves %d remap %u: %.4f ms per step\n",
                          rows, waves, remap, ms);
            rep += line;
            // any later candidate (another shape, or the other block order of
            // the same shape) must be 2% faster: a short trial once took the
            // round-robin order for FP64 1024^2 passes, 58 against 67 GLUPS
            // over 1000 steps
            if (ms < 0.98f * best_two_ms) {
                best_two_ms = ms;
                best_shape = shape;
                if (ms < best) { best = ms; best_two = true; best_remap = remap; }
            }
        }
    }
    c->g.remap = best_remap;
    c->two = best_two;
    c->two_shape = best_shape;
    prepare_zchunk(c);
    drop_graphs(c);
    // runs of kGraphSteps sweeps: graph replays against direct launches of the
    // same kernels, alternately, three times each (direct launches measured
    // 0.5-3% faster from 128^2 to 1024^2 and level on 256^3, where a launch
    // takes 0.3 ms; the trial is there for grids so small that the host's
    // launch rate would fall behind the kernels, which graphs avoid).  Direct
    // launches are kept unless graphs are at least 1% faster.
    float graph_ms = -1.f, direct_ms = -1.f;
    c->use_graphs = true;
    if (!(c->desc.flags & LBM_FLAG_NO_GRAPH) && c->check_every == 0) {
        for (int trial = 0; trial < 6; ++trial) {
            c->use_graphs = (trial & 1) == 0;
            int rc = advance(c, kGraphSteps, st);   // warm-up (and the graph capture)
            hipError_t e = rc == LBM_OK ? hipEventRecord(e0, st) : hipErrorUnknown;
            if (e == hipSuccess) rc = advance(c, 4 * kGraphSteps, st);
            if (e == hipSuccess && rc == LBM_OK) e = hipEventRecord(e1, st);
            if (e == hipSuccess && rc == LBM_OK) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess && rc == LBM_OK) e = hipEventElapsedTime(&ms, e0, e1);
            if (rc != LBM_OK || e != hipSuccess) {
                (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
                return rc != LBM_OK ? rc : hip_fail(e, "tuning graph launches");
            }
            ms /= 4 * kGraphSteps;
            float &t = c->use_graphs ? graph_ms : direct_ms;
            if (t < 0.f || ms < t) t = ms;
        }
        c->use_graphs = graph_ms < 0.99f * direct_ms;
        char gl[112];
        std::snprintf(gl, sizeof(gl), "graph replays: %.4f ms per step, direct launches: %.4f ms per step\n", graph_ms,
                      direct_ms);
        rep += gl;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int brows = 0, bwaves = 0;
    if (best_two) shape_of(c, best_shape, &brows, &bwaves);
    char line[176];
    std::snprintf(line, sizeof(line), "chosen chunk %d nt %d remap %u two %d rows %d waves %d graphs %d (%.4f ms)",
                  best_chunk, (int)best_nt, best_remap, (int)best_two, brows, bwaves, (int)c->use_graphs, best);
    rep += line;
    if (report && report_len) std::snprintf(report, report_len, "%s", rep.c_str());
    // the history buffer was overwritten by the trial sweeps: restart from phi0
    return lbm_init(c, c->phi0, c->f[0], c->f[1], c->p, c->p2, stream);
}

int lbm_probe_copy(const void *src, void *dst, size_t bytes, int grid, void *stream) {
    if (!src || !dst) return fail(LBM_E_INVALID, "null argument");
    if (((uintptr_t)src | (uintptr_t)dst | bytes) & 15) return fail(LBM_E_INVALID, "16-byte alignment required");
    const size_t n16 = bytes / 16;
    if (n16 == 0) return LBM_OK;
    const size_t chunks = (n16 + 4 * 256 - 1) / (4 * 256);
    if (grid <= 0 || (size_t)grid > chunks) grid = (int)std::min<size_t>(chunks, 1u << 30);
    hipError_t e = launch_copy16(src, dst, n16, grid, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "copy kernel");
    return LBM_OK;
}

}  // extern "C"
