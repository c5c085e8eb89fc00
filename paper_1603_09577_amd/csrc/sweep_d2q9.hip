// Kernel instantiations for the D2Q9 lattice.
#define LBM_Q 9
#include "lbm_dispatch.h"

namespace lbm {

hipError_t launch_sweep_q9(const Dims &dm, const Geom &g, const void *coefs, const void *fin,
                            void *fout, void *p, int *flag, hipStream_t st) {
    LBM_BY_PREC(sweep_typed, dm, g, coefs, fin, fout, p, flag, st)
}

hipError_t launch_init_q9(const Dims &dm, const Geom &g, const void *coefs, const double *phi0,
                           void *f, void *p, const double *rfield, hipStream_t st) {
    LBM_BY_PREC(init_typed, dm, g, coefs, phi0, f, p, rfield, st)
}

hipError_t launch_phi_q9(const Dims &dm, const Geom &g, const void *coefs, const void *f,
                          double *phi, const double *rfield, hipStream_t st) {
    LBM_BY_PREC(phi_typed, dm, g, coefs, f, phi, rfield, st)
}

hipError_t launch_phi_reduce_q9(const Dims &dm, const Geom &g, const void *coefs, const void *f, const double *ref,
                               const double *rfield, double *part, int nparts, double *out, hipStream_t st) {
    LBM_BY_PREC(phi_reduce_typed, dm, g, coefs, f, ref, rfield, part, nparts, out, st)
}

hipError_t launch_sweep_gen_q9(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                               void *p, int *flag, const double *kfield, const double *rfield, bool remark3,
                               hipStream_t st) {
    LBM_BY_PREC(sweep_gen_typed, dm, g, coefs, fin, fout, p, flag, kfield, rfield, remark3, st)
}

hipError_t launch_recenter_q9(const Dims &dm, const Geom &g, void *coefs, void *f, void *p, double *part,
                              int nparts, double *shift, hipStream_t st) {
    LBM_BY_PREC(recenter_typed, dm, g, coefs, f, p, part, nparts, shift, st)
}

}  // namespace lbm

namespace lbm {

hipError_t launch_adjoint_q9(const Dims &dm, const Geom &g, const void *coefs, const void *f, const void *p,
                             const void *psi_next, const double *pi_next, void *psi_out, double *pi_out,
                             double *gk_part, hipStream_t st) {
    LBM_BY_PREC_ADJ(adjoint_typed, dm, g, coefs, f, p, psi_next, pi_next, psi_out, pi_out, gk_part, st)
}

hipError_t launch_adjoint_init_q9(const Dims &dm, const Geom &g, const void *coefs, const double *phi0,
                                  const void *psi0, const double *pi0, double *out, hipStream_t st) {
    LBM_BY_PREC_ADJ(adjoint_init_typed, dm, g, coefs, phi0, psi0, pi0, out, st)
}

hipError_t launch_seed_q9(const Dims &dm, const Geom &g, const double *gphi, void *psi, double *pi,
                          hipStream_t st) {
    LBM_BY_PREC_ADJ(seed_typed, dm, g, gphi, psi, pi, st)
}

hipError_t launch_zero(double *p, uint32_t n, hipStream_t st) { return zero_doubles(p, n, st); }


hipError_t launch_set_wall_q9(const Dims &dm, void *coefs, const double *ewp, hipStream_t st) {
    LBM_BY_PREC(set_wall_typed, dm, coefs, ewp, st)
}


hipError_t launch_sweep2_q9(const Dims &dm, const Geom &g, const void *coefs, const void *fin, void *fout,
                            const void *pin, void *pout, int *flag, int shape, hipStream_t st) {
    LBM_BY_PREC(sweep2_typed, dm, g, coefs, fin, fout, pin, pout, flag, shape, st)
}

bool two_step_shape_of(int prec, int shape, int *rows, int *waves) {
    int r = 0, w = 0;
    const bool ok = prec == 0 ? two_step_shape<double>(shape, r, w) : two_step_shape<float>(shape, r, w);
    if (ok) { *rows = r; *waves = w; }
    return ok;
}

hipError_t launch_adjoint2_q9(const Dims &dm, const Geom &g, const void *coefs, const void *f1, const void *p1,
                              const void *f0, const void *p0, const void *psi_next, const double *pi_next,
                              void *psi_out, double *pi_out, double *gk_part, int shape, hipStream_t st) {
    if (!dm.eqr || dm.wall) return hipErrorInvalidValue;
    LBM_BY_PREC_ADJ(adjoint2_typed, dm, g, coefs, f1, p1, f0, p0, psi_next, pi_next, psi_out, pi_out, gk_part, st,
                    shape, nullptr)
}

hipError_t adjoint2_q9_occupancy(const Dims &dm, const Geom &g, int shape, int *blocks_per_cu) {
    if (!dm.eqr || dm.wall) return hipErrorInvalidValue;
    LBM_BY_PREC_ADJ(adjoint2_typed, dm, g, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                    nullptr, nullptr, nullptr, shape, blocks_per_cu)
}

bool adjoint2_shape_of(int shape, int *rows, int *waves) {
    if (shape < 0 || shape >= kAdjShapes) return false;
    *rows = kAdjShape[shape][0];
    *waves = kAdjShape[shape][1];
    return true;
}


}  // namespace lbm
