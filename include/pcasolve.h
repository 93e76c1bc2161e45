/*
 * pcasolve -- per-projection PCA lung-motion solve on MI355X (gfx950).
 *
 * Method: Li et al., "3D tumor localization through real-time volumetric
 * x-ray imaging for lung cancer radiotherapy".  Given one cone-beam x-ray
 * projection y at a known gantry angle, find the PCA coefficients w that
 * minimise (Eq. 2)
 *
 *     J(w, a, b) = || P f(x, f0) - a y - b 1 ||^2,   x = xbar + U w   (Eq. 1)
 *
 * where f is the reference image f0 pulled back through the deformation
 * field x by trilinear interpolation (Eqs. A.3, A.5) and P is the cone-beam
 * projection at that angle; then locate the tumour by inverting the solved
 * pull-back field at one point.
 *
 * C ABI: plain pointers and sizes only.
 *   - "device" arrays live in GPU memory owned by the caller; the library
 *     never frees them and never keeps a pointer past the call.
 *   - "host" arrays are ordinary CPU memory owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Unless stated otherwise an entry point only enqueues work on `stream`
 *     and returns; outputs are valid once the stream reaches that point.
 *   - `dtype` selects the element type of every floating-point device array
 *     of the call (all of them share it): PCAS_F32 (float) or PCAS_F64
 *     (double).  Reductions always accumulate in double.
 *   - Every argument is validated on the host before the first HIP call
 *     (a volume must be smaller than 2 GiB: kernels use 32-bit offsets);
 *     an invalid call returns a negative status and touches no memory.
 *
 * Layouts (0-based versions of the Appendix's 1-based (i, j, k)):
 *   volume       f[i + n1*(j + n2*k)]            i = lateral, fastest
 *   vector field x[c*N + v], c = 0 lateral, 1 AP, 2 SI, in mm, N = n1*n2*n3
 *   modes        U[(k*3 + c)*N + v], k = 0..K-1 (mm per unit coefficient)
 *   detector     p[iu + nu*iv]                   u (tangential) fastest
 *
 * Geometry (the paper fixes only that P depends on the gantry angle):
 *   voxel (i,j,k) centre = origin + (i,j,k) * spacing  (mm)
 *   source = (SAD sin t, -SAD cos t, 0); flat detector at distance SID from
 *   the source with axes e_u = (cos t, sin t, 0), e_v = (0, 0, 1); pixel
 *   (iu, iv) centre at u = (iu - (nu-1)/2) pitch_u + offset_u (same for v).
 *   One ray per pixel centre.  P integrates the trilinear interpolant of the
 *   volume along the chord through the box spanned by the first and last
 *   voxel centres with the midpoint rule: n = ceil(L / step) samples of
 *   width dt = L / n.  Outside the grid every volume reads as zero.
 */
#ifndef PCASOLVE_H
#define PCASOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCAS_ABI_VERSION 8
#define PCAS_MAX_K 8

typedef enum { PCAS_F32 = 0, PCAS_F64 = 1 } pcas_dtype;

/* status codes (return values) */
enum {
    PCAS_OK = 0,
    PCAS_EINVAL = -1,      /* null pointer, dimension < 2, K outside [1, 8], bad dtype, bad option */
    PCAS_EGEOM = -2,       /* SAD <= 0, SID <= SAD, pitch <= 0, step <= 0, source inside the volume */
    PCAS_ESINGULAR = -3,   /* Y^T Y of Eq. A.1 singular (constant measured projection) */
    PCAS_ENONFINITE = -4,  /* NaN or Inf in y, w0 or an objective value */
    PCAS_EWORKSPACE = -5,  /* workspace missing, too small or misaligned */
    PCAS_EHIP = -6         /* a HIP runtime call failed; see pcas_last_error() */
};

/* solve_projection termination reasons (pcas_report.status, >= 0) */
enum { PCAS_STOP_CONVERGED = 0, PCAS_STOP_MAXITER = 1, PCAS_STOP_LINESEARCH = 2 };

typedef struct {
    int32_t n[3];          /* n1, n2, n3 (each >= 2) */
    double spacing[3];     /* mm, > 0 */
    double origin[3];      /* mm, centre of voxel (0, 0, 0) */
} pcas_vol;

typedef struct {
    double angle;          /* gantry angle t (radians) */
    double sad, sid;       /* source-axis and source-detector distances (mm) */
    int32_t nu, nv;        /* detector pixels (>= 1) */
    double pitch_u, pitch_v;   /* pixel pitch at the detector (mm) */
    double offset_u, offset_v; /* detector shift (mm), 0 for a centred full fan */
    double step;           /* ray-march sample spacing (mm) */
} pcas_proj;

typedef struct {
    int32_t method;        /* 0: Appendix algorithm (Eq. A.1 + Eq. A.2 + Armijo); 1: PR+ CG
                              whose line searches start at the minimiser along d of a
                              quadratic model (curvature d.B d, B built from the accepted
                              steps by direct BFGS updates; mu0 / ||d|| before it exists);
                              2: BFGS (dense K x K inverse-Hessian estimate); 1 and 2 work on
                              the reduced objective min_{a,b} J and share one line search */
    int32_t max_iter;      /* accepted iterations */
    int32_t fit_intensity; /* 1: (a, b) from Eq. A.1; 0: a = 1, b = 0 */
    int32_t max_backtracks;/* line-search trials per iteration (methods 1, 2) */
    double mu0;            /* first step length (in units of w) */
    double alpha, beta;    /* Armijo sufficient-decrease and shrink factors */
    double mu_min;         /* method 0: stop once the step falls below it */
    double gtol_rel;       /* methods 1, 2: stop when ||g|| <= gtol_rel ||g0|| */
    double beta_lo;        /* methods 1, 2: lower safeguard of the interpolated shrink */
    double xtol;           /* methods 1, 2: a trial step shorter than xtol fails the search */
    int32_t locate;        /* 1: also run tumour_position at c0_mm after the solve */
    int32_t locate_max_iter;
    double locate_tol;     /* mm */
    double c0_mm[3];       /* tumour centre in the reference image (mm) */
    int32_t profile;       /* kernel classes to time with HIP events (report.kernel_ms): bit c
                              for class c of the PCAS_K_* list below, PCAS_PROFILE_ALL for every
                              class, 0 for none.  Each timed launch adds two event records to
                              the stream, a few microseconds each, so a caller timing one kernel
                              sets that kernel's bit alone */
    int32_t grad_mode;     /* how dJ/dw is formed (the same quantity either way, by the
                              adjoint identity <P^T r, J_k> = <r, P J_k>):
                              1: back-project r, then g = 2 U^T (df/dx) P^T r (the Appendix's
                                 route, the default); the solver runs drr_adjoint's kernel
                                 with grad_w's chain applied to each brick as it completes,
                                 so P^T r never goes to device memory
                              0: project the K Jacobian volumes J_k = U_k^T (df/dx) and take
                                 g_k = 2 <r, P J_k> (gathers only, no back-projection)
                              2: fused evaluation: every evaluation forms f and the J_k in
                                 one voxel pass and projects all K + 1 volumes together,
                                 keeping per pixel r0 = p - a0 y - b0 (a0, b0 a reference
                                 fit) and q_k = (P J_k); the sums of r0, r0 y, r0^2, q_k r0,
                                 q_k y and q_k give J, the fit and g_k = 2 <r, P J_k> at
                                 the fit found, so a gradient costs no launch of its own */
    double ftol_rel;       /* methods 1, 2: the noise band of J (relative): a rejected trial
                              with |J_t - J| <= ftol_rel J ends the solve as converged, and
                              either method also ends, converged, when its model predicts a
                              decrease <= ftol_rel J for the next first trial (method 2:
                              g.H g / 2; method 1: (g.d)^2 / (2 d.B d)) while trusting its
                              model (the last step's decrease was also <= ftol_rel J, or
                              within a factor 2 of the model's prediction for that step, when
                              it was accepted at its first trial).  < 0 (default): a rounding
                              model per point, 6 u sqrt(sum p^2 / (M J)) with u = 2^-24 for
                              PCAS_F32 and 2^-53 for PCAS_F64 (three times the spread of J
                              that rounding each p_i by u |p_i| produces) */
    double ls_extrap;      /* methods 1, 2: when the first trial of a line search passes Armijo
                              and the quadratic through J(0), J'(0), J(t) has its minimiser
                              t_q > 2t, one more trial at min(t_q, ls_extrap t) follows and the
                              lower point is kept; 0 turns this off (>= 0, finite) */
    int32_t polish;        /* methods 1, 2: 1 = when the solve stops at the noise band (noise
                              or decrement stop, failed search), try one step w - H g with
                              the inverse-Hessian estimate (method 2's own; method 1 keeps
                              one from its steps) and keep it if ||g|| drops; costs one
                              evaluation and one gradient.  The gradient resolves the
                              minimiser below the noise of J: without it an FP32 solve stops
                              where FP32 values of J stop resolving decreases, about 1.5e-4
                              from the minimiser in w at the clinical size.  Default 1 */
    int32_t speculate;     /* methods 1, 2 with grad_mode 1: 1 = launch the
                              gradient right behind each evaluation after which the solve may
                              ask for it (its start and polish points, line-search trials),
                              gated on the GPU by the solve's own rule (Armijo acceptance,
                              the extrapolation test) applied to the evaluated J, so that an
                              accepted trial costs one host round trip instead of two.  A
                              launch whose gate is shut exits at once (report class
                              PCAS_K_SPEC_SKIP).  Results are bit-identical with 0.
                              Default 1 */
    int32_t precond;       /* method 1 with grad_mode 2: 1 = precondition CG by the
                              Gauss-Newton matrix of the reduced objective at each point,
                              H = 2 (Q^T Q - Q^T Y (Y^T Y)^-1 Y^T Q) with Q = dp/dw (the
                              projected Jacobian volumes, columns q_k) and Y = [y, 1]
                              (2 Q^T Q when the fit is fixed), which the fused evaluation's
                              sums give: directions -H^-1 g + beta d (PR+ with
                              preconditioned inner products), first trials and the stop
                              from the model g.d + d.H d / 2, and the polish step the
                              Gauss-Newton step.  Default 0 */
} pcas_opts;

/* kernel classes of pcas_report.kernel_ms / kernel_launches (in a solve,
   PCAS_K_ADJOINT is the back-projection fused with the Jacobian chain,
   PCAS_K_SPEC_SKIP a speculative launch of it (opts.speculate) whose gate
   was shut, so that it exited at once, and PCAS_K_WARP_JAC /
   PCAS_K_DRR_EVAL the two launches of a fused evaluation (grad_mode 2)) */
enum {
    PCAS_K_RAYS = 0, PCAS_K_WARP = 1, PCAS_K_DRR = 2, PCAS_K_RESIDUAL = 3,
    PCAS_K_ADJOINT = 4, PCAS_K_GRAD = 5, PCAS_K_LOCATE = 6, PCAS_K_YSUMS = 7,
    PCAS_K_JACOBIAN = 8, PCAS_K_DRR_DOT = 9, PCAS_K_SPEC_SKIP = 10, PCAS_K_WARP_JAC = 11,
    PCAS_K_DRR_EVAL = 12, PCAS_K_CLASSES = 13
};
#define PCAS_PROFILE_ALL ((1 << PCAS_K_CLASSES) - 1)

typedef struct {
    int32_t status;        /* PCAS_STOP_* */
    int32_t iters;         /* accepted iterations */
    int32_t n_fevals;      /* forward evaluations (warp + projection) */
    int32_t n_grads;       /* gradient evaluations (see opts.grad_mode) */
    double J0, J;          /* objective at w0 and at the returned w */
    double a, b;           /* intensity fit at the returned w */
    double gnorm0, gnorm;  /* ||dJ/dw|| at w0 and at the returned w */
    double tumour_mm[3];   /* located tumour position (if opts.locate) */
    int32_t locate_iters;  /* fixed-point iterations, -1 if not converged */
    int32_t spec_grads;    /* of n_grads, how many a speculative launch supplied */
    double kernel_ms[PCAS_K_CLASSES];   /* with opts.profile: summed kernel time per class (ms) */
    int32_t kernel_launches[PCAS_K_CLASSES];
    double host_ms;        /* wall time of the solve_projection call on the host (ms) */
    double wait_ms;        /* of host_ms, the time spent waiting for the GPU's read-backs; the
                              rest is host work (checks, the state machine, launch calls) */
} pcas_report;

/* ---- utilities --------------------------------------------------------- */

int pcas_abi_version(void);
const char *pcas_status_string(int status);
/* Text of the last PCAS_EHIP failure on the calling thread ("" if none). */
const char *pcas_last_error(void);
/* Defaults: method 1 (CG), 30 iterations, fit on, 12 backtracks, mu0 = 1,
 * alpha = 0.1, beta = 0.5 (the Appendix's Armijo constants), mu_min = 0.01,
 * gtol_rel = 1e-9, beta_lo = 0.1, xtol = 1e-10, no localisation, 100
 * localisation iterations, 1e-9 mm tolerance, grad_mode 1 (back-projection),
 * ftol_rel by dtype, ls_extrap = 10, polish = 1. */
void pcas_default_opts(pcas_opts *opts);
/* Appendix algorithm: method 0, 10 iterations, mu0 = 0.2, alpha = 0.1,
 * beta = 0.5, stop below mu_min = 0.01 (the paper's 2 and 0.1 rescaled from
 * its coefficient standard deviation of 10 to ours of 1). */
void pcas_paper_opts(pcas_opts *opts);

/* ---- a1: ray table (Sec. II.A: P depends on the gantry angle) ----------
 * One record per detector pixel: entry point and per-sample step in voxel
 * index units, sample width dt (mm) and sample count n, computed in double
 * from the geometry above and stored in `dtype`.  Every projection and
 * back-projection call of one geometry reads the same table, which is what
 * makes drr_adjoint the exact transpose of drr_forward.
 * rays: device, pcas_ray_table_bytes() bytes, 16-byte aligned. */
size_t pcas_ray_table_bytes(pcas_dtype dtype, const pcas_proj *proj);
int ray_table(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, void *rays,
              void *stream);

/* ---- a2: Eq. 1, x = xbar + sum_k w_k u_k ---------------------------------
 * mean: device [3][N] or NULL (zero mean); U: device [K][3][N];
 * w: host double[K]; dvf_out: device [3][N] (mm). */
int pca_dvf(pcas_dtype dtype, int64_t nvox, int32_t K, const void *mean, const void *U,
            const double *w, void *dvf_out, void *stream);

/* ---- a3: Eqs. A.3 / A.5, f(i,j,k) = f0 at (i,j,k) + x/spacing ------------
 * Trilinear pull-back with zero extension outside the grid.
 * f0: device [N]; dvf: device [3][N] (mm); f_out: device [N] (no aliasing). */
int warp_trilinear(pcas_dtype dtype, const pcas_vol *vol, const void *f0, const void *dvf,
                   void *f_out, void *stream);

/* ---- a2 + a3 fused: the field of Eq. 1 is formed per voxel in registers
 * and never stored.  Arguments as pca_dvf / warp_trilinear. */
int warp_pca(pcas_dtype dtype, const pcas_vol *vol, int32_t K, const void *f0, const void *mean,
             const void *U, const double *w, void *f_out, void *stream);

/* ---- a4: forward projection p = P f (Eq. 2) ------------------------------
 * rays: device table from ray_table() for the same (dtype, vol, proj);
 * f: device [N]; p_out: device [nv][nu].  Pixels whose ray misses the box
 * get 0. */
int drr_forward(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *rays,
                const void *f, void *p_out, void *stream);

/* ---- exact-path projection (Siddon's method; Sec. II.B simulates the
 * digital projections with it) -------------------------------------------
 * The volume read as constant over voxel cells [centre - s/2, centre + s/2];
 * each pixel gets the sum over cells of (length of the source-to-pixel ray
 * inside the cell) x (cell value).  A second operator beside drr_forward's
 * trilinear ray march, e.g. to make measurements that the solve's own P did
 * not produce.  Geometry and sums in double.  f: device [N]; p_out: device
 * [nv][nu]. */
int drr_siddon(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *f,
               void *p_out, void *stream);

/* ---- a6: back-projection bp = P^T r (Appendix, gradient of J) -----------
 * The exact transpose of drr_forward for the same ray table: every sample
 * of every ray adds dt * r * (its trilinear weight) to its eight voxels
 * (the same cell and fractions as drr_forward computes for it).
 * Accumulated per 32 x 16 x 8 voxel brick in on-chip memory in 64-bit fixed
 * point with no global atomics; bit-for-bit reproducible.  The brick's
 * power-of-two scale comes from its largest |r| and the weight bound of
 * pcas_backprojection_bound taken over the brick's neighbourhood, so no
 * partial sum can overflow.  r: device [nv][nu]; bp_out: device [N], fully
 * overwritten. */
int drr_adjoint(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *rays,
                const void *r, void *bp_out, void *stream);

/* The same back-projection with 32-bit fixed-point accumulators (PCAS_F32
 * only; PCAS_EINVAL otherwise): the accumulation the solver's FP32 gradient
 * uses.  Half the on-chip bytes per add, so faster; each contribution is
 * rounded to nearest, to about 2^-19 (clinical geometry) of the largest
 * contribution the brick's bound allows, against the float products' own
 * 2^-24.  Same arguments, layout and reproducibility as drr_adjoint. */
int drr_adjoint32(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *rays,
                  const void *r, void *bp_out, void *stream);

/* Bound B on the summed trilinear weight that all rays of a projection give
 * one voxel: (P^T 1)(v) <= step * B for every voxel v (the pixel centres
 * whose rays can meet a voxel's cube of index half-width 1, from the
 * worst-case magnification over the grid box, times what one ray can give
 * it).  Host-only, no device memory.  Returns a negative value for an
 * invalid volume or projection. */
double pcas_backprojection_bound(const pcas_vol *vol, const pcas_proj *proj);

/* The same bound over one back-projection brick (brick order: see
 * backprojection_brick_count): (P^T 1)(v) <= step * B_brick for every voxel v of the brick and of
 * its one-voxel halo.  This is what sizes the brick's fixed-point
 * accumulators in drr_adjoint, drr_adjoint32 and the solver's gradient.
 * Host-only; negative for an invalid volume, projection or brick index. */
double pcas_backprojection_brick_bound(const pcas_vol *vol, const pcas_proj *proj,
                                       int32_t brick);

/* Number of back-projection bricks: the volume is cut into 32 x 16 x 8
 * voxel bricks (brick x fastest, then y, then z), the brick index of
 * pcas_backprojection_brick_bound.  Host-only; -1 for an invalid volume. */
int32_t backprojection_brick_count(const pcas_vol *vol);

/* Voxels of the bricks a projection can read: a brick is live unless the
 * image of its box with a one-voxel halo (which holds every sample whose
 * cell touches a voxel of the brick) misses the detector by more than a
 * pixel.  Inside solve_projection and the serving loop the warp writes only
 * these voxels.  Host-only; -1 for an invalid volume or projection. */
int64_t pcas_live_voxels(const pcas_vol *vol, const pcas_proj *proj);

/* ---- a5: intensity fit (Eq. A.1) and residual ----------------------------
 * stats_out: device double[8] =
 *   { J, a, b, sum p, sum p*y, sum p*p, sum y, sum y*y }
 * with (a, b) from Eq. A.1 (or (1, 0) if fit_intensity == 0), J = ||r||^2;
 * r_out: device [M] = p - a y - b (may be NULL; may alias p).
 * If Y^T Y is singular a, b and J are NaN (checked by the caller).
 * workspace: device, residual_fit_workspace_bytes() bytes. */
size_t residual_fit_workspace_bytes(int64_t npix);
int residual_fit(pcas_dtype dtype, int64_t npix, const void *p, const void *y, int32_t fit_intensity,
                 void *r_out, double *stats_out, void *workspace, size_t workspace_bytes,
                 void *stream);

/* ---- a7: Jacobian chain and K-reduction ----------------------------------
 * g = 2 U^T (df/dx) bp with df/dx the diagonal Jacobian of Eq. A.8 (and its
 * two analogues) at x = xbar + U w, per mm; the right-side derivative at
 * integer positions.  bp is normally P^T r, making g = dJ/dw at fixed (a, b).
 * f0, bp: device [N]; mean: device [3][N] or NULL; U: device [K][3][N];
 * w: host double[K]; g_out: device double[K].  Deterministic (fixed-order
 * reduction).  workspace: device, grad_w_workspace_bytes() bytes. */
size_t grad_w_workspace_bytes(pcas_dtype dtype, const pcas_vol *vol, int32_t K);
int grad_w(pcas_dtype dtype, const pcas_vol *vol, int32_t K, const void *f0, const void *mean,
           const void *U, const double *w, const void *bp, double *g_out, void *workspace,
           size_t workspace_bytes, void *stream);

/* ---- grad_w for callers that cannot allocate ----------------------------
 * For code that must not call hipMalloc or take a caller workspace: work
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Computes exactly what grad_w computes (same kernels, same
 * fixed-order reduction, bit-identical g_out) but keeps the reduction's
 * block partials and counter in a file-scope device array of the library,
 * grad_w_noalloc_scratch_bytes() bytes (about 128 KiB), one per GPU, held
 * until the process ends.  Every volume that grad_w accepts fits (its grid
 * is capped at 2048 blocks); a larger need would return PCAS_EWORKSPACE.
 * The array is shared by all calls on a GPU and keeps the last call's
 * contents: each call first zeroes the counter on `stream`, and calls that
 * overlap on one GPU (other streams or threads) race on it.  Asynchronous on
 * `stream`; allocates nothing.  Arguments as grad_w without the workspace. */
size_t grad_w_noalloc_scratch_bytes(void);
int grad_w_noalloc(pcas_dtype dtype, const pcas_vol *vol, int32_t K, const void *f0,
                   const void *mean, const void *U, const double *w, const void *bp,
                   double *g_out, void *stream);

/* ---- a9: tumour position (Sec. II.A, pull-back inversion at one point) --
 * Fixed point y <- c0 - x(y) from y = c0, with x the trilinear value of the
 * field of Eq. 1 at y (zero outside the grid); stops when a step is shorter
 * than tol (mm) or after max_iter iterations.
 * out: device double[4] = { y1, y2, y3 (mm), iterations or -1 }. */
int tumour_position(pcas_dtype dtype, const pcas_vol *vol, int32_t K, const void *mean,
                    const void *U, const double *w, const double c0_mm[3], double tol,
                    int32_t max_iter, double *out, void *stream);

/* ---- a5 + a6 + a7: objective and gradient at one point ------------------
 * J(w) of Eq. 2 with (a, b) from Eq. A.1 (fit_intensity = 1) or a = 1, b = 0,
 * and dJ/dw at that (a, b), exactly as solve_projection forms them, the
 * gradient by the route grad_mode selects (see pcas_opts.grad_mode).
 * Arguments as solve_projection; w: host double[K];
 * out: host double[3 + K] = { J, a, b, g_0 .. g_{K-1} }, and for grad_mode 2
 * double[3 + K + K * K] with the Gauss-Newton matrix of the reduced
 * objective at w after g (row-major; see pcas_opts.precond).  Synchronous. */
int objective_gradient(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, int32_t K,
                       const void *f0, const void *mean, const void *U, const void *y,
                       const double *w, int32_t fit_intensity, int32_t grad_mode,
                       void *workspace, size_t workspace_bytes, double *out, void *stream);

/* ---- a1-a9: the per-projection solve -------------------------------------
 * Minimise Eq. 2 over w from w0 with the method in opts (Appendix algorithm,
 * CG or BFGS; see pcas_opts), then optionally locate the tumour.
 * f0: device [N]; mean: device [3][N] or NULL; U: device [K][3][N];
 * y: device [nv][nu]; w0: host double[K]; w_out: host double[K];
 * report: host.  workspace: device, solve_projection_workspace() bytes,
 * 256-byte aligned, used exclusively by this call until it returns.
 * Synchronous: returns after the result has been copied to the host.  Each
 * of the solve's read-backs waits by spinning the calling thread on a word
 * in mapped host memory that a one-wave kernel on `stream` sets after
 * copying the values; the stream may still be retiring that kernel when the
 * call returns, and work enqueued on it later runs after it.
 * Returns PCAS_OK (with the stop reason in report->status) or an error. */
size_t solve_projection_workspace(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj,
                                  int32_t K);
int solve_projection(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, int32_t K,
                     const void *f0, const void *mean, const void *U, const void *y,
                     const double *w0, const pcas_opts *opts, void *workspace,
                     size_t workspace_bytes, double *w_out, pcas_report *report, void *stream);

/* ---- Eq. 3: initial coefficients of the next projection ----------------
 * Sec. II.A, Eq. 3: each coefficient is predicted separately as a linear
 * combination of its last L optimised values, w_k0(t) = sum_{l=1..L} c_kl
 * w*_k(t - l) (the paper uses L = 2).  Host-only, no device memory.
 * coeffs: host double[K][L] with coeffs[k*L + l-1] = c_kl; history: host
 * double[n_hist][K], the most recent solution last (n_hist >= L);
 * w_out: host double[K].  PCAS_EINVAL for K outside [1, 8], L outside
 * [1, 8] or n_hist < L; PCAS_ENONFINITE for NaN or Inf in the inputs. */
int pcas_predict(int32_t K, int32_t L, const double *coeffs, const double *history,
                 int32_t n_hist, double *w_out);
/* The c_kl of Eq. 3 by least squares on a training sequence, separately for
 * every coefficient (Sec. II.A fits them on resampled training coefficients;
 * any sequence of solutions serves): minimises sum_{t=L}^{T-1} (w[t][k] -
 * sum_l c_kl w[t-l][k])^2 by a QR factorisation of the lagged values.
 * w_train: host double[T][K] (T > L); coeffs_out: host double[K][L].
 * PCAS_ESINGULAR when a coefficient's lagged values are (numerically)
 * linearly dependent, e.g. a constant sequence with L = 2. */
int pcas_fit_predictor(int32_t T, int32_t K, int32_t L, const double *w_train,
                       double *coeffs_out);

/* ---- serving: many solves in flight, batched into shared launches -------
 * A server solves requests (one projection of one registered model each)
 * concurrently.  Its device memory is one caller-owned arena (256-byte
 * aligned): pcas_server_reserved_bytes() for its launch tables, the rest
 * carved per request (pcas_server_request_bytes(): ray table, warped
 * volume, projection, reduction scratch).  A submitted request waits until
 * its footprint fits in the free arena and one of max_active slots is free;
 * requests behind it that fit may go first.  Registered models (f0, mean, U)
 * stay resident in the caller's memory; a request's y (device) must stay
 * valid until its result has been polled.
 * Each pcas_server_step() admits what fits, runs one operation of every
 * admitted request's solve (an evaluation of Eq. 2, a residual, a gradient
 * by back-projection with the chain fused; the admission work; or the
 * tumour localisation), batching each kind of operation for all requests
 * of one dtype and K (or slab axis) into one launch, reads back all their
 * scalars in one transfer and returns the number of requests completed.
 * A grad_mode 2 request's evaluation is the fused one and its gradients
 * follow from the evaluation's sums on the host, without a step of their own.
 * A batched block runs what the request's own launch would run, so every
 * result equals solve_projection's for the same request, bit for bit.
 * Requests run the solve of their opts (method, fit, tolerances, locate,
 * grad_mode 1 or 2).  report.kernel_ms is not filled.
 * The server keeps pinned host staging for its tables and read-backs.
 * Synchronous steps on `stream`; one thread at a time per server. */
typedef struct pcas_server pcas_server;
size_t pcas_server_reserved_bytes(int32_t max_active);
int pcas_server_create(void *arena, size_t arena_bytes, int32_t max_active, void *stream,
                       pcas_server **out);
int pcas_server_destroy(pcas_server *server);
/* model_id: 0, 1, ... in registration order. */
int pcas_server_add_model(pcas_server *server, pcas_dtype dtype, const pcas_vol *vol, int32_t K,
                          const void *f0, const void *mean, const void *U, int32_t *model_id);
/* Arena bytes a request of this model and geometry occupies while admitted
 * with these options (opts may be NULL: the defaults); a grad_mode 2
 * request also holds the warped image with its K Jacobian volumes.  0 for
 * an invalid model or geometry. */
size_t pcas_server_request_bytes(pcas_server *server, int32_t model_id, const pcas_proj *proj,
                                 const pcas_opts *opts);
/* w0: host double[K]; request_id: unique, increasing.  PCAS_EWORKSPACE if
 * the request could never fit in the arena. */
int pcas_server_submit(pcas_server *server, int32_t model_id, const pcas_proj *proj,
                       const void *y, const double *w0, const pcas_opts *opts,
                       int64_t *request_id);
/* One step: admits what fits, runs one operation of every admitted request
 * (a main pass), then extra passes for the cheap requests, those whose
 * operation costs at most a quarter of the most expensive admitted one's
 * (estimated as N + M * volume diagonal / step), while the extra passes'
 * summed cost stays within substep_share (default 0.25) of the main pass's.
 * A request's result does not depend on the passes it ran in. */
int pcas_server_step(pcas_server *server, int32_t *n_completed);
/* share in [0, 16]; 0 gives one pass per step. */
int pcas_server_set_substep_share(pcas_server *server, double share);
/* *done = 1 and the request's status (PCAS_OK or the error that ended it)
 * once it has completed, with w_out (host double[K], may be NULL) and
 * report (may be NULL) filled; the request is then forgotten.  *done = 0
 * while it is pending or running. */
int pcas_server_poll(pcas_server *server, int64_t request_id, double *w_out, pcas_report *report,
                     int32_t *done);
int pcas_server_stats(pcas_server *server, int32_t *n_pending, int32_t *n_active,
                      size_t *arena_used);

#ifdef __cplusplus
}
#endif

#endif /* PCASOLVE_H */
