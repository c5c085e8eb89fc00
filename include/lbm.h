/*
 * lbm.h - C ABI of the MI355X (gfx950) MRT lattice Boltzmann sweep for the
 * nonlinear anisotropic convection-diffusion equation with a source term
 *
 *     d_t phi + div B(phi) = div[K . (div D(phi))] + R            (Eq. 1)
 *
 * following the general multiple-relaxation-time model of Chai, Shi & Guo
 * (Sec. 2.2, Eq. 2-10, 14-28; Remark II for the source schemes).
 *
 * Conventions
 *  - Lattice units: c = dx = dt = 1, cs^2 = 1/3 (Eq. 5/6 and the text after
 *    them).  A problem stated with other dx, dt is rewritten by the caller
 *    (B dt/dx, K dt/dx^2, R dt).
 *  - Every buffer that grows with the grid is owned by the caller: both
 *    distribution buffers, the phi history and, for two steps per pass with a
 *    source, a second history (sizes from lbm_state_bytes).  The library
 *    never allocates or frees caller buffers.  A context owns only its
 *    parameter table and a fixed device scratch area (divergence flag,
 *    reduction partials, adjoint K0 partials: about 3.1 MiB whatever the
 *    grid size); a batch owns its per-instance tables and tile work lists.
 *  - Calls are asynchronous on the caller's HIP stream (a hipStream_t passed
 *    as void*, NULL = the default stream) unless stated otherwise.
 *  - Every call returns LBM_OK (0) or a negative error code; lbm_last_error()
 *    returns a thread-local message.  No exception crosses the ABI.
 *  - Field layout seen by the caller (phi0, phi, targets, gradients): FP64,
 *    C order [nz][ny][nx].  Distribution buffers are opaque (size from
 *    lbm_state_bytes); internally they are structure-of-arrays planes, one
 *    plane of nx*ny*nz values per lattice direction, in the storage type,
 *    consecutive planes padded apart (plane_pad).
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define LBM_OK 0
#define LBM_E_INVALID -1      /* bad argument or parameter set               */
#define LBM_E_UNSUPPORTED -2  /* valid for the method, not built on the GPU  */
#define LBM_E_HIP -3          /* a HIP runtime call failed                   */
#define LBM_E_DIVERGED -4     /* a non-finite phi was produced               */
#define LBM_E_STATE -5        /* call out of order (e.g. step before init)   */

/* ---- enumerations ------------------------------------------------------- */
#define LBM_D2Q9 9            /* Eq. 5 */
#define LBM_D3Q19 19          /* Eq. 6 */

#define LBM_BC_PERIODIC 0
#define LBM_BC_ABB 1          /* anti-bounce-back Dirichlet wall half a link
                                 beyond the first / last node (Sec. 3.6)    */

#define LBM_F64 0             /* distributions stored in FP64, FP64 math     */
#define LBM_F32 1             /* stored as FP32 offsets f_k - w_k phi_ref,
                                 FP32 math                                    */
#define LBM_F16 2             /* stored as FP16 offsets, FP32 math            */

#define LBM_SCHEME_A 0        /* Remark II, gamma = 0: explicit time difference
                                 of the source, needs phi of the last step   */
#define LBM_SCHEME_B 1        /* Remark II, gamma = 1: Btilde = B', stored
                                 fbar = f - R_k/2 (Eq. 33), Eq. 34, phi from
                                 Eq. 35.  R = rpoly(phi) of degree <= 2 plus
                                 an optional field (lbm_set_fields); when R
                                 depends on phi, Eq. 35 is a quadratic in phi
                                 solved in closed form at every node (the
                                 root that tends to sum fbar + R/2 as R -> 0) */

#define LBM_FLAG_MOMENT_PATH 1 /* always use the moment-space collision even
                                  when all non-flux rates are equal          */
#define LBM_FLAG_NO_XCD_REMAP 2 /* launch blocks in the hardware's round-robin
                                  XCD order (default: one contiguous slab per
                                  XCD while the state fits the 256 MB Infinity
                                  Cache, round-robin beyond; lbm_tune times both) */
#define LBM_FLAG_NO_GRAPH 4   /* lbm_step launches every sweep directly
                                 instead of replaying captured graphs       */
#define LBM_FLAG_REMARK3 8    /* Remark III (Eq. 36-38): equilibrium with C = 0
                                 (Eq. 38) plus the source G_k of Eq. 37, dB/dt
                                 as the difference over the last step (from
                                 the phi history); for a B whose C of Eq. 7 is
                                 not wanted or has no closed form, such as a
                                 rational B (lbm_desc.bden).  General kernel;
                                 no adjoint, no batches                       */

#define LBM_MAXP 9            /* polynomial coefficients per function        */

/* Problem and model description (Eq. 1 coefficients, Eq. 3, Eq. 17).
 *  B_a(phi)  = sum_p b[a][p] phi^p                       (convection, Eq. 1)
 *  D(phi)    = (sum_p dpoly[p] phi^p) * dten             (Eq. 1)
 *  K(phi)    = k0 * (sum_p kpoly[p] phi^p)               (diffusion tensor)
 *  R(phi)    = sum_p rpoly[p] phi^p                      (source)
 *  C(phi)    = integral_0^phi B' B'^T                    (Eq. 7, C(0) = 0)
 *  Flux relaxation block A = (K / (d cs^2) + I/2)^-1      (Eq. 26), per node
 *  when kpoly is not constant.  s[] holds the remaining diagonal rates in the
 *  moment order of Eq. 15 (D2Q9: rho, e, eps, jx, qx, jy, qy, pxx, pxy) or of
 *  the d'Humieres polynomial basis (D3Q19); entries of the flux rows are
 *  ignored.  Only the upper-left 2x2 of k0/dten is used for D2Q9. */
typedef struct lbm_desc {
    int lattice;              /* LBM_D2Q9 or LBM_D3Q19                        */
    int nx, ny, nz;           /* nodes per axis (nz = 1 for D2Q9)             */
    int bc[3];                /* per axis; walls only on the last axis
                                 (y for D2Q9, z for D3Q19)                    */
    double phi_wall[3][2];    /* Dirichlet phi at the low / high wall          */
    int precision;            /* LBM_F64 / LBM_F32 / LBM_F16                  */
    double phi_ref;           /* offset reference of the stored distributions */
    int scheme;               /* LBM_SCHEME_A / LBM_SCHEME_B                  */
    double d;                 /* positive parameter of Eq. 3                  */
    double s[19];             /* diagonal relaxation rates (Eq. 17)           */
    double b[3][LBM_MAXP];
    double dpoly[LBM_MAXP];
    double dten[3][3];
    double k0[3][3];
    double kpoly[LBM_MAXP];
    double rpoly[LBM_MAXP];
    int flags;                /* LBM_FLAG_*                                    */
    int plane_pad;            /* elements added after each direction plane:
                                 0 = library choice (spreads the planes over
                                 the L2 sets and memory channels), > 0 exact,
                                 < 0 none                                      */
    double bden[LBM_MAXP];    /* denominator Q(phi) of a rational flux
                                 B_a = (sum_p b[a][p] phi^p) / Q(phi), e.g. the
                                 Buckley-Leverett flux of Sec. 3.3 (Eq. 54),
                                 whose C of Eq. 7 has no polynomial form; all
                                 zero (or Q = 1) for a polynomial B.  A rational
                                 B needs LBM_FLAG_REMARK3 (C = 0, Eq. 38) and
                                 Q(phi) != 0 on the range phi takes          */
} lbm_desc;

typedef struct lbm_ctx lbm_ctx;

/* Validate a description and derive the model constants.  Rejects
 * (LBM_E_INVALID): unknown lattice, sizes < 1 or 2^31 nodes or more,
 * d <= 0, a used rate outside (0, 2), k0 not symmetric positive definite,
 * dten not symmetric.  LBM_E_UNSUPPORTED: walls on an axis other than the
 * last, Scheme B with rpoly of degree > 2, a rational B (bden) without
 * LBM_FLAG_REMARK3.  Allocates the context's coefficient table and
 * its fixed scratch (about 3.1 MiB, independent of the grid) on the current
 * device, nothing that scales with the grid.  *out is set only on success. */
int lbm_create(const lbm_desc *desc, lbm_ctx **out);

/* Bytes of the buffers the caller provides, each a multiple of 256 (any
 * output pointer may be NULL):
 *  f_bytes  one distribution buffer (two are needed);
 *  p_bytes  the phi-history buffer (phi of the last step: Scheme A's
 *           R_k(t - 1), Remark II);
 *  p2_bytes a second history buffer, used only by two time steps per pass on
 *           runs that keep a history (a Scheme-A source, on runs where the
 *           passes apply: lbm_set_two_step); 0 when no pass would read it.
 *           Without it such a run uses one sweep per step. */
int lbm_state_bytes(const lbm_ctx *ctx, size_t *f_bytes, size_t *p_bytes, size_t *p2_bytes);

/* Bytes of one adjoint-variable buffer psi (same plane layout as the
 * distribution buffers, in the compute type: FP64 or FP32). */
int lbm_adjoint_bytes(const lbm_ctx *ctx, size_t *psi_bytes);

/* Bind two distribution buffers, the phi-history buffer and the optional
 * second history p2, and initialise with the equilibrium of phi0 (Eq. 40; the
 * history is set to phi0, the reading of the first Scheme-A step).  phi0_dev:
 * FP64 [nz][ny][nx] on the device, kept by pointer for lbm_tune.  Buffers
 * must be 256-byte aligned and of lbm_state_bytes sizes.  p2 may be NULL: it
 * is ignored when lbm_state_bytes reports p2_bytes = 0, and otherwise its
 * absence turns two steps per pass off for this binding.  p2 must differ from
 * the other buffers (LBM_E_INVALID). */
int lbm_init(lbm_ctx *ctx, const double *phi0_dev, void *f_a, void *f_b, void *p, void *p2,
             void *stream);

/* Advance nsteps time steps (Eq. 2 with the Scheme-A source, anti-bounce-back
 * walls), one fused stream-collide sweep per step.  Runs of 32 sweeps are
 * replayed from a HIP graph captured on first use (an internal stream; the
 * graph is launched on the caller's stream) unless LBM_FLAG_NO_GRAPH is set,
 * a divergence check is enabled or lbm_tune found direct launches faster.  Asynchronous unless a divergence check is
 * due (lbm_set_check), in which case it synchronises the stream and returns
 * LBM_E_DIVERGED when a non-finite phi appeared. */
int lbm_step(lbm_ctx *ctx, int nsteps, void *stream);

/* One sweep between explicit buffers: f_out <- sweep(f_in), p updated in
 * place (Scheme A history).  f_in and f_out must differ.  Does not touch the
 * bound buffers or the step counter. */
int lbm_sweep(lbm_ctx *ctx, const void *f_in, void *f_out, void *p, void *stream);

/* phi of the current state (Eq. 10a), FP64 [nz][ny][nx] into phi_dev. */
int lbm_get_phi(lbm_ctx *ctx, double *phi_dev, void *stream);

/* phi of an explicit distribution buffer (same layout as the bound ones). */
int lbm_phi_of(lbm_ctx *ctx, const void *f, double *phi_dev, void *stream);

/* The buffers that hold the current state and the number of steps taken. */
int lbm_current(const lbm_ctx *ctx, void **f, void **p, long long *t);

/* Exchange the roles of the two bound distribution buffers and set the step
 * counter (used after the caller restored a state into the other buffer). */
int lbm_set_current(lbm_ctx *ctx, int which, long long t);

/* Launch shape: each workgroup sweeps `chunk` consecutive 256-node blocks
 * (1 = one block per workgroup, the default). */
int lbm_set_chunk(lbm_ctx *ctx, int chunk);

/* Workgroup order: on = one contiguous run of the domain per XCD (the
 * default unless the state exceeds the Infinity Cache or
 * LBM_FLAG_NO_XCD_REMAP is set), off = the hardware's round-robin order.
 * lbm_tune sets it too. */
int lbm_set_remap(lbm_ctx *ctx, int on);

/* Non-temporal (streaming) loads and stores of the distributions in the
 * equal-rate sweep (default: on when the state exceeds 256 MB, the size of
 * the Infinity Cache, where they raise HBM throughput; off otherwise, where
 * they would keep a cache-resident state out of the cache). */
int lbm_set_nontemporal(lbm_ctx *ctx, int on);

/* Autotuner (synchronous): times the sweep on the bound buffers for chunk =
 * 1, 2, 4, 8, 16 workgroup blocks, with and without non-temporal accesses,
 * and with the XCD-aware block order (one contiguous slab per XCD) or the
 * hardware's round-robin order (unless LBM_FLAG_NO_XCD_REMAP pins the
 * latter), and, where allowed, two time steps per pass (lbm_set_two_step);
 * keeps the fastest; then, unless LBM_FLAG_NO_GRAPH is set or a divergence
 * check is enabled, times lbm_step's graph replays against direct launches of
 * the same kernels and keeps direct launches unless graphs are at least 1%
 * faster (results are identical either way); writes the timings into
 * `report` (may be NULL) and
 * re-initialises the state from the phi0 given to lbm_init (step counter
 * back to 0; phi0 must still be valid). */
int lbm_tune(lbm_ctx *ctx, int reps, void *stream, char *report, size_t report_len);

/* Two time steps per pass inside lbm_step.  Every node update is the
 * single-sweep arithmetic on the same inputs (post-collision values kept in
 * LDS are rounded to the storage type as a store would round them), so
 * results equal single sweeps bit for bit, while the state crosses HBM once
 * per two steps.
 *  - D2Q9, periodic axes (any grid size: tiles wrap periodically) with equal
 *    non-flux rates, or, with polynomials of degree <= 2, also walls on y
 *    and unequal rates (the latter in the default tile shape only): a
 *    workgroup runs step t on a 62 x rows tile with a one-node halo and step
 *    t + 1 on the tile.  Passes run in pairs (four
 *    steps); with a Scheme-A source they alternate the history between p and
 *    the caller's p2 (lbm_init).  Scheme-B sources need polynomials of
 *    degree <= 2.
 *  - D3Q19, polynomials of degree <= 2 (unequal non-flux rates in the
 *    default tile shape only), walls on z or periodic: a workgroup owns a column of 62 x rows nodes and a chunk of z
 *    planes and marches up it, phase 1 (step t, with a one-node halo in x
 *    and y) feeding a ring of three planes in LDS that phase 2 (step t + 1)
 *    reads one plane behind.  Passes run in pairs; with a Scheme-A source
 *    they alternate the history between p and p2 as in 2-D.
 * Remaining steps use single sweeps.  On by default where it applies (with a
 * Scheme-A source: where p2 is bound); lbm_tune times it against single
 * sweeps.  Not used with per-node fields or Remark III.
 * mode: 0 off; k >= 1 on with tile shape k - 1 (lbm_two_step_shape; shape 0
 * is the default).  The non-default D2Q9 shapes need every polynomial of
 * degree <= 2.
 * Errors: LBM_E_UNSUPPORTED when the run does not qualify; LBM_E_STATE when a
 * run with a Scheme-A source was bound without p2; LBM_E_INVALID for a shape
 * that is not available here. */
int lbm_set_two_step(lbm_ctx *ctx, int mode);

/* Tile shape `shape` of two-step passes for this context's lattice and
 * storage type: tile rows (the tile is 62 x rows nodes, phase 1 covers
 * 64 x (rows + 2)) and waves per workgroup.  D2Q9, 4- and 2-byte storage:
 * 14 x 4, 14 x 8, 10 x 6, 6 x 4; FP64: 6 x 4, 6 x 8, 14 x 16.  D3Q19 (one
 * phase-1 row per wave): 4- and 2-byte storage 14 x 16, 6 x 8, 2 x 4; FP64
 * 6 x 8, 2 x 4.  More waves per workgroup (fewer rows each) fit more waves per
 * CU; fewer rows per tile cost more halo work.  LBM_E_INVALID past the last
 * shape. */
int lbm_two_step_shape(const lbm_ctx *ctx, int shape, int *rows, int *waves);

/* Divergence check every `every` steps inside lbm_step (0 = off): lbm_step
 * then waits on the host at every multiple of `every` (counted from lbm_init)
 * and returns LBM_E_DIVERGED once a sweep has met a non-finite phi.  Steps
 * between two checks still run as two-step passes where those apply; the
 * per-step graphs are not used. */
int lbm_set_check(lbm_ctx *ctx, int every);

/* Re-centre the stored offsets of the current state (asynchronous, on the
 * device): phi_ref moves to the mean of phi (from the phi history when the run
 * keeps one, else from the stored populations), every stored value gains
 * w_k (old - new) and the history old - new, and the wall terms are rewritten.
 * The distributions f_k themselves are unchanged in exact arithmetic, so every
 * result of Eq. 2 is the same; what changes is the size of the stored numbers,
 * which bounds the rounding of FP16 (and FP32) storage when phi drifts far
 * from phi_ref under a source or through walls.  Afterwards the adjoint calls
 * and lbm_set_k0 return LBM_E_STATE until the next lbm_init, which restores
 * the description's phi_ref.  Errors: LBM_E_STATE before lbm_init. */
int lbm_recenter(lbm_ctx *ctx, void *stream);

/* Re-centre automatically inside lbm_step every `every` steps, counted from
 * lbm_init (0 = never).  Default: 256 for LBM_F16 storage with a source term
 * (R != 0: the whole field moves away from phi_ref), 0 otherwise (the mean is
 * then fixed, or moves only through walls, and a field that is mostly at one
 * level with structure elsewhere is stored best against that level, not
 * against its mean). */
int lbm_set_recenter(lbm_ctx *ctx, int every);

/* New Dirichlet values of the two walls (anti-bounce-back, half a link beyond
 * the first and last node of the wall axis; Sec. 3.6), for time-dependent
 * walls.  Asynchronous on `stream` (one small kernel rewrites the wall terms
 * in the device constants, so it may sit between captured graphs).
 * Timing: the state after the sweep from t to t + 1 holds the post-collision
 * values of step t, and the next gather (the next sweep, or lbm_get_phi)
 * streams them with the wall values set at that moment.  So a schedule
 * phi_w(t) used in the streaming of step t is followed by setting phi_w(t)
 * right after the sweep of step t.  The first gather after lbm_init only
 * undoes the initial layout and must see the wall values lbm_init saw.
 * Errors: LBM_E_INVALID (no walls, non-finite values). */
int lbm_set_phi_wall(lbm_ctx *ctx, double phi_lo, double phi_hi, void *stream);

/* Per-node fields, read by lbm_init, lbm_step, lbm_sweep and lbm_get_phi
 * (device pointers owned by the caller; NULL unbinds):
 *  - k0_field: FP64, per node (2-D) xx, yy, xy or (3-D) xx, yy, zz, xy, yz, xz,
 *    [nz][ny][nx][3 or 6].  K(x, phi) = K0(x) kpoly(phi) replaces the
 *    description's k0; A is formed per node by Eq. 26 (the variable diffusion
 *    tensor of Sec. 3.5).  Each K0(x) must be symmetric positive definite; it
 *    is not checked (a non-finite phi shows in lbm_set_check).
 *  - r_field: FP64 [nz][ny][nx], an external source added to R: R(x, t) =
 *    rpoly(phi) + r_field(x) (Eq. 1; Scheme B only).  Its contents are R at
 *    the current time: a sweep from t to
 *    t + 1 reads R(x, t), and lbm_get_phi reads it as R(x, t) of the state it
 *    converts, so a time-dependent source is rewritten between steps (on the
 *    same stream).
 * Scheme B with a source, or a K0 field, runs the general kernel (any
 * polynomial length, no streaming hints).  The adjoint calls refuse them.
 * Errors: LBM_E_INVALID (misaligned), LBM_E_UNSUPPORTED (r_field with
 * Scheme A). */
int lbm_set_fields(lbm_ctx *ctx, const double *k0_field, const double *r_field);

/* Replace K0 (keeps every other parameter); same validation as lbm_create. */
int lbm_set_k0(lbm_ctx *ctx, const double k0[9]);

/* FP64 reductions over a phi field (synchronous), the quantities the method
 * is checked with: the total of phi, whose change over a step is the source
 * total because phi = sum_k f_k (Eq. 10a) and streaming permutes the
 * populations; and the error norms against a reference field, out[7] /
 * sum |ref| being the global relative error of Eq. 39 and
 * sqrt(out[2] / out[3]) the relative L2 error.  The field is N FP64 values
 * (the node count of the context), ref_dev N values or NULL (then ref = 0).
 *   out[0] = sum phi,  out[1] = sum phi^2,  out[2] = sum (phi - ref)^2,
 *   out[3] = sum ref^2,  out[4] = min phi,  out[5] = max phi,
 *   out[6] = number of non-finite values (left out of every other entry),
 *   out[7] = sum |phi - ref|.
 * Partials are folded in a fixed order, so results do not vary between runs.
 * Errors: LBM_E_INVALID (null argument), LBM_E_HIP. */
int lbm_reduce(lbm_ctx *ctx, const double *phi_dev, const double *ref_dev, double out[8],
               void *stream);

/* The same reductions without waiting: the 8 values of lbm_reduce are
 * written, in the same order and bit for bit the same, to out_dev (8 doubles
 * of caller device memory) on the stream; nothing returns to the host.  Calls
 * on one context share its partial-sum scratch, so two reductions of the
 * same context (this call or lbm_reduce) must not run on different streams
 * at the same time.  Errors: LBM_E_INVALID (null argument), LBM_E_HIP. */
int lbm_reduce_async(lbm_ctx *ctx, const double *phi_dev, const double *ref_dev, double *out_dev, void *stream);

/* The reductions of lbm_reduce over the phi of the current state (the one
 * lbm_get_phi would write), formed on the fly from the stored populations in
 * one pass: no phi field is written or read.  The 8 values, bit for bit those
 * of lbm_reduce over lbm_get_phi's field, go to out_dev (8 doubles of caller
 * device memory) on the stream, without waiting.  Shares the context's
 * partial-sum scratch like lbm_reduce_async.  Errors: LBM_E_INVALID (null
 * argument), LBM_E_STATE (before lbm_init), LBM_E_HIP. */
int lbm_reduce_state(lbm_ctx *ctx, const double *ref_dev, double *out_dev, void *stream);

/* The reductions of lbm_reduce_async over any FP64 field of n values, with no
 * context and no allocation: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The per-workgroup partial sums live in a fixed device array of
 * the library (64 KiB: 1024 rows of 8 FP64 values), one copy per GPU, held
 * until the process ends; its address is resolved on the first call on each
 * device, with that device current.  The call launches two kernels and makes
 * no allocating call (no hipMalloc, hipFree or library allocation) and no
 * memset: every partial row the fold reads is written by the same call first,
 * so nothing needs clearing between calls.  Results equal, bit for bit,
 * those of lbm_reduce_async on a context of n nodes over the same fields
 * (same partial rows, same fixed folding order).
 *   phi_dev  n FP64 values on the current device;
 *   ref_dev  n FP64 values or NULL (ref = 0);
 *   out_dev  8 FP64 values of caller device memory, the order of lbm_reduce
 *            (n = 0 gives 0, 0, 0, 0, +inf, -inf, 0, 0).
 * Asynchronous on `stream`, which must belong to the current device.  All
 * calls on one GPU share its array: calls that overlap in time on one GPU
 * (different streams, or host threads) race and must be serialised by the
 * caller.  Errors: LBM_E_INVALID (null phi or out, n above
 * LBM_NOALLOC_MAX_NODES), LBM_E_HIP. */
#define LBM_NOALLOC_MAX_NODES 2147483647
int lbm_reduce_noalloc(const double *phi_dev, const double *ref_dev, size_t n, double *out_dev, void *stream);

/* ---- discrete adjoint (D2Q9 and D3Q19, F64 and F32) ---------------------- *
 * Sweep s maps the state X_s = (f_s, p_s) to X_{s+1}: it gathers g_s from f_s,
 * collides with history p_s and stores f_{s+1}; p_{s+1} = sum_k g_s,k.
 * With L a function of phi(T) = sum_k g_T,k, the adjoint variables are
 *   psi_s = dL/dg_s  (q values per node, same layout and size as f buffers,
 *                      stored in the compute type: FP64 or FP32),
 *   pi_s  = dL/dp_s  (FP64 [nz][ny][nx]).
 * psi_s equals the gradient with respect to the pre-collision distributions
 * of step s.  Gradients with respect to K0 accumulate into a per-context FP64
 * accumulator (lbm_adjoint_grad_k0).  Not defined for FP16 storage, Scheme B
 * sources, per-node fields or Remark III (LBM_E_UNSUPPORTED), nor after the
 * offsets were re-centred (LBM_E_STATE). */

/* psi_T from dL/dphi(T) (FP64 field): psi_T,k = gphi for every k, pi_T = 0;
 * clears the K0 accumulator.  Seed, step and init launch kernels only (no
 * memset or allocation), so a caller may capture them in a HIP graph. */
int lbm_adjoint_seed(lbm_ctx *ctx, const double *gphi_dev, void *psi, double *pi_out,
                     void *stream);

/* One reversed sweep: from the forward state (f_s, p_s) and (psi_{s+1},
 * pi_{s+1}) compute (psi_s, pi_s) and add dL/dK0 of this sweep.  psi_next and
 * psi_out must differ; pi may be updated in place (pi_out == pi_next). */
int lbm_adjoint_step(lbm_ctx *ctx, const void *f_s, const void *p_s, const void *psi_next,
                     const double *pi_next, void *psi_out, double *pi_out, void *stream);

/* Two reversed sweeps in one launch: sweep s from (f_s, p_s) and (psi_{s+1},
 * pi_{s+1}), then sweep s - 1 from (f_sm1, p_sm1) = (f_{s-1}, p_{s-1}),
 * giving (psi_{s-1}, pi_{s-1}) in (psi_out, pi_out) and adding dL/dK0 of both
 * sweeps.  psi and pi equal those of two lbm_adjoint_step calls bit for bit;
 * the K0 sums agree up to the order of FP64 additions.  The intermediate
 * (psi_s, pi_s) lives in workgroup memory only.  Applies to D2Q9 with
 * periodic axes and equal non-flux rates (lbm_adjoint_pair_ok tells in
 * advance; elsewhere LBM_E_UNSUPPORTED).
 * psi_out must differ from psi_next and pi_out from pi_next (LBM_E_INVALID):
 * neighbouring tiles read pi_{s+1} during the launch. */
int lbm_adjoint_step2(lbm_ctx *ctx, const void *f_s, const void *p_s, const void *f_sm1, const void *p_sm1,
                      const void *psi_next, const double *pi_next, void *psi_out, double *pi_out,
                      void *stream);

/* *ok = 1 if lbm_adjoint_step2 applies to this context, else 0. */
int lbm_adjoint_pair_ok(const lbm_ctx *ctx, int *ok);

/* Tile shapes of lbm_adjoint_step2, 62 columns wide: shape 0 = 6 rows x 4
 * waves per workgroup, 1 = 10 x 4, 2 = 10 x 12 (one row per wave).
 * lbm_adjoint_tile_shape reports a shape's rows and waves (LBM_E_INVALID past
 * the last).  lbm_create picks one for the grid and device: the 6- or 10-row
 * tiling that runs the launch in fewer rounds of resident workgroups (6 at
 * equal rounds), and 10 x 12 for FP32 launches with at most 6 waves per SIMD
 * in all where it at least halves the tiles per CU.  lbm_set_adjoint_tile forces shape mode - 1, or restores the pick
 * with mode 0 (LBM_E_INVALID otherwise); lbm_adjoint_tile reports the shape
 * in use.  Every shape gives the same psi and pi bit for bit; the K0 sums
 * differ in the order of FP64 additions. */
int lbm_adjoint_tile_shape(const lbm_ctx *ctx, int shape, int *rows, int *waves);
int lbm_set_adjoint_tile(lbm_ctx *ctx, int mode);
int lbm_adjoint_tile(const lbm_ctx *ctx, int *shape);

/* Adjoint of the initialisation (Eq. 40): dL/dphi0 = sum_k psi_0,k dfeq_k/dphi
 * + pi_0, into gphi0_dev (FP64). */
int lbm_adjoint_init(lbm_ctx *ctx, const double *phi0_dev, const void *psi0, const double *pi0,
                     double *gphi0_dev, void *stream);

/* Accumulated dL/dK0 (synchronous): out = (xx, xy, yy, xz, yz, zz), the
 * symmetric entries each treated as one parameter (D2Q9: the z entries are 0). */
int lbm_adjoint_grad_k0(lbm_ctx *ctx, double out[6], void *stream);

void lbm_destroy(lbm_ctx *ctx);
const char *lbm_last_error(void);

/* Measurement aid: plain device copy of `bytes` (multiple of 16, 16-byte
 * aligned pointers) in chunks of 16 KiB, each copied by one workgroup of 256
 * lanes (four coalesced 16-byte loads per lane, then the stores); `grid`
 * workgroups loop over the chunks (<= 0 or more than the chunks: one
 * workgroup per chunk).  Gives the practical bandwidth of a read-once /
 * write-once stream and calibrates the traffic counters. */
int lbm_probe_copy(const void *src, void *dst, size_t bytes, int grid, void *stream);

/* ---- batches of independent D2Q9 instances ------------------------------- *
 * Many periodic D2Q9 instances of uneven size, each with its own description
 * (sizes, K0, B, ... ; same precision, equal non-flux rates), advanced by one
 * launch per time step over a device work list of tiles, replayed from
 * captured HIP graphs.  The caller owns three arenas: two distribution arenas
 * and one history arena (sizes from lbm_batch_layout); phi fields of all
 * instances are concatenated in one FP64 arena, instance i at node offset
 * lbm_batch_instance(i) in [ny][nx] order. */
typedef struct lbm_batch lbm_batch;

/* Validate every description (as lbm_create; LBM_E_UNSUPPORTED for walls,
 * D3Q19 or unequal non-flux rates) and build the work lists.  Allocates the
 * per-instance tables and work lists on the current device. */
int lbm_batch_create(const lbm_desc *descs, int count, lbm_batch **out);
int lbm_batch_layout(const lbm_batch *b, size_t *f_bytes, size_t *p_bytes, long long *total_nodes);
int lbm_batch_instance(const lbm_batch *b, int i, long long *node_offset, int *nx, int *ny);

/* Bind the arenas and initialise every instance at equilibrium (Eq. 40) from
 * the concatenated phi0 arena (kept by pointer until the next init: the
 * autotuner re-initialises from it). */
int lbm_batch_init(lbm_batch *b, const double *phi0_arena, void *f_a, void *f_b, void *p, void *stream);

/* Advance every instance nsteps steps. */
int lbm_batch_step(lbm_batch *b, int nsteps, void *stream);

/* phi of every instance into the FP64 arena. */
int lbm_batch_get_phi(lbm_batch *b, double *phi_arena, void *stream);

/* Autotuner (synchronous): times each candidate launch shape (workgroup size
 * and nodes per thread, persistent grid size, XCD-aware order) over `reps`
 * sweeps of the bound batch, keeps the fastest, then re-initialises the
 * state from the phi0 arena given to lbm_batch_init (step counter back to 0).
 * With use_cache, a previous decision for the same batch signature is read
 * from (and new ones appended to) the text file named by $LBM_TUNE_CACHE,
 * default ~/.cache/lbm_batch_tune.txt.  A report of the timings is written
 * into `report` (may be NULL). */
int lbm_batch_tune(lbm_batch *b, int reps, int use_cache, void *stream, char *report, size_t report_len);

/* Force / read the launch shape: shape index 0..3 = (256 threads, 1 node per
 * thread), (256, 2), (128, 1), (512, 1); grid 0 = one workgroup per tile,
 * otherwise persistent workgroups over contiguous chunks of the list.
 * Batches without a source whose polynomials all have degree <= 2 also offer
 * two time steps per launch (the two-step pass of lbm_set_two_step, one
 * workgroup per 62 x rows tile of an instance, bit-identical to single
 * sweeps): shape 4 = 14 rows x 8 waves and shape 5 = 6 rows x 4 waves for 4-
 * and 2-byte storage, shape 4 = 6 rows x 8 waves for FP64; the grid argument
 * is ignored for them, an odd remaining step runs shape 0, and get_shape
 * reports wg = 64 x waves and npt = -rows.  lbm_batch_tune times them with the
 * others.  LBM_E_INVALID for a shape the batch does not offer. */
int lbm_batch_set_shape(lbm_batch *b, int shape, unsigned grid, int remap);
int lbm_batch_get_shape(const lbm_batch *b, int *shape, unsigned *grid, int *remap, int *wg, int *npt);

void lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif
