// Internal declarations shared by the HIP translation units of libpcasolve.
// Kernels are written for gfx950 (CDNA4): wave64, LDS-staged reductions,
// double accumulation for every reduction, no global atomics on data.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pcasolve.h"
#include "solver.h"

namespace pcas {

// Launch-time volume description (index space).  inv_s is 1/spacing.
struct VolDims {
    int n0, n1, n2;       // n1, n2, n3 of the API (i fastest)
    double inv_s[3];
    double spacing[3];
    double origin[3];
};

// Cone-beam frame of one projection, precomputed on the host in double.
struct Frame {
    double src[3];        // source position (mm)
    double det[3];        // detector centre (mm)
    double eu[3], ev[3];  // detector axes
    double en[3];         // unit vector source -> detector centre
    double sid;
    double pitch_u, pitch_v, offset_u, offset_v, step;
    int nu, nv;
};

// Per-ray record: entry point and per-sample step in voxel-index units,
// sample width dt (mm), sample count n.  Sample s sits at e + (s + 1/2) d.
template <typename T> struct RayRec;
template <> struct alignas(16) RayRec<float> {
    float e[3];
    float d[3];
    float dt;
    int32_t n;
};
template <> struct alignas(16) RayRec<double> {
    double e[3];
    double d[3];
    double dt;
    int32_t n;
    int32_t pad_;
};
static_assert(sizeof(RayRec<float>) == 32, "RayRec<float> layout");
static_assert(sizeof(RayRec<double>) == 64, "RayRec<double> layout");

// Back-projection brick (the voxels one workgroup accumulates in LDS).
constexpr int BRICK_X = 32, BRICK_Y = 16, BRICK_Z = 8;
// Waves sharing one brick, each with its own ray queue.  8 (with 16 x 16 x 8
// bricks): 32 waves per CU, the VGPR limit, in 4 bricks, against 28 in 7
// bricks with 4 waves; the fused gradient kernel measured 410 against
// 431 us, 2 waves 582 us.  FWD_THREADS: a forward-projection block.
constexpr int ADJ_WAVES = 8;
constexpr int ADJ_THREADS = 64 * ADJ_WAVES;
constexpr int FWD_THREADS = 256;
// Forward projection, tile shape ts: fwd_split(ts) lanes march one ray
// (interleaved samples), a wave covers fwd_wu(ts) x fwd_wv(ts) neighbouring
// rays, a 256-thread block 2 x 2 such wave tiles (a bundle of tile_u(ts) x
// tile_v(ts) rays).  The bundle stages its footprint in the volume slab by
// slab in an LDS box of FWD_LDS_BYTES per volume (two for several volumes).
// Shape 0: 4 lanes a ray, 8 x 8 rays.  Shape 1: one lane a ray, 16 x 16 rays,
// whose larger box serves four times the rays (the plan takes it for FP32
// projections of three or more volumes whenever its boxes fit some slabs).
constexpr int fwd_split(int ts) { return ts == 0 ? 4 : 1; }
constexpr int fwd_wu(int ts) { return ts == 0 ? 4 : 8; }
constexpr int fwd_wv(int ts) { return 64 / fwd_split(ts) / fwd_wu(ts); }
constexpr int tile_u(int ts) { return 2 * fwd_wu(ts); }
constexpr int tile_v(int ts) { return 2 * fwd_wv(ts); }
constexpr int FWD_LDS_BYTES = 16384;
constexpr int FWD_MAX_SLABS = 128;
static_assert(fwd_wu(0) * fwd_wv(0) * fwd_split(0) == 64, "forward wave tile");
static_assert(fwd_wu(1) * fwd_wv(1) * fwd_split(1) == 64, "forward wave tile");
static_assert(tile_u(1) * tile_v(1) >= tile_u(0) * tile_v(0), "shape 0 has the most blocks");
// Values one scalar read-back can return (the mapped mailbox's size).
constexpr int MAILBOX_VALUES = 80;
// Sums the fused evaluation's projection reduces for K modes (see
// launch_drr_forward_eval): 6 + 3K + K(K + 1) / 2, at most 66.
constexpr int eval_sums(int K) { return 6 + 3 * K + K * (K + 1) / 2; }
// Reductions: partial-sum slots per block; a reduction of more than
// RED_SLOTS values (the fused evaluation's sums) takes up to RED_SLOTS_WIDE.
constexpr int RED_SLOTS = 8;
constexpr int RED_SLOTS_WIDE = 72;
static_assert(eval_sums(PCAS_MAX_K) <= RED_SLOTS_WIDE && eval_sums(PCAS_MAX_K) <= MAILBOX_VALUES,
              "fused evaluation sums");
// Threads that finish the fused evaluation's deferred sums (the solve's
// read-back and the serving gather use the same width, hence the same
// summation order): wide, since the pass reads every block's partials.
constexpr int EVAL_SUM_WIDTH = 512;
// Where block bid's total of value j goes: a reduction of at most RED_SLOTS
// values keeps each block's totals together; a wider one keeps value j of
// all nblocks blocks together, so that the finishing pass reads them
// coalesced (it reads every value of every block either way).
__host__ __device__ constexpr int64_t red_slot(int ns, int j, int bid, int nblocks) {
    return ns <= RED_SLOTS ? (int64_t)bid * RED_SLOTS + j : (int64_t)j * nblocks + bid;
}
constexpr int GRAD_BLOCKS_MAX = 2048;

// Coefficients passed by value to kernels.
struct WVec {
    double w[PCAS_MAX_K];
};

// Spread consecutive workgroup ids (dispatched round-robin over the 8 XCDs)
// so that each XCD works on a contiguous range of tiles and its L2 sees a
// compact footprint.  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
    const int per = nblocks >> 3;
    const int full = per << 3;
    if (bid >= full) return bid;
    return (bid & 7) * per + (bid >> 3);
}

// Intensity-fit mode of the residual pass (see launch_residual) and of the
// forward pass's objective (FIT_NONE: moments only).
enum { FIT_COEF = 0, FIT_REFIT = 1, FIT_FIXED = 2, FIT_NONE = 3 };
// (a, b): the fixed fit; sy, syy, m: sum y, sum y^2 and the pixel count;
// (a0, b0): the reference fit of the forward pass's moments, which are sums
// of r0 = p - a0 y - b0, r0 y and r0^2 (a0 = b0 = 0: sums of p, p y, p^2).
struct FitArgs {
    int mode;
    double a, b, sy, syy, m;
    double a0 = 0.0, b0 = 0.0;
};
// Above this cancellation factor sum(r0^2) / J the J formed from the
// forward pass's moments is recomputed by the two-pass residual at the fit
// found.
constexpr double MOMENT_KAPPA_MAX = 1e4;

// The objective of Eq. 2 at a fit (a, b) from moments mo = (sum r0,
// sum r0 y, sum r0^2) about a reference fit (a0, b0).  With r0 = p - a0 y -
// b0 and d = (a - a0, b - b0) the residual is r = r0 - d_a y - d_b, so
//   J = S(r0^2) - 2 (d_a S(r0 y) + d_b S(r0)) + d_a^2 S(y^2) + 2 d_a d_b S(y) + M d_b^2,
// and the refit of Eq. A.1 solves [S(y^2) S(y); S(y) M] d = [S(r0 y); S(r0)].
// With the reference near the fit S(r0^2) is close to J and the sum does not
// cancel; kappa = S(r0^2) / J says how far that holds (infinite if J <= 0).
// A singular refit gives NaN a and b.  fit.mode is FIT_REFIT or FIT_FIXED.
// Compiled for host and device without contraction, so both sides get the
// same bits from the same moments.
__host__ __device__ inline void objective_from_moments(const double *mo, const FitArgs &fit,
                                                       double *J, double *a, double *b,
                                                       double *kappa) {
#pragma clang fp contract(off)
    double A, B;
    if (fit.mode == FIT_REFIT) {
        const double det = fit.syy * fit.m - fit.sy * fit.sy;
        if (fabs(det) > 1e-12 * fit.syy * fit.m) {
            A = fit.a0 + (fit.m * mo[1] - fit.sy * mo[0]) / det;
            B = fit.b0 + (fit.syy * mo[0] - fit.sy * mo[1]) / det;
        } else {
            A = B = NAN;
        }
    } else {
        A = fit.a;
        B = fit.b;
    }
    const double da = A - fit.a0, db = B - fit.b0;
    const double j = mo[2] - 2.0 * (da * mo[1] + db * mo[0]) + da * da * fit.syy +
                     2.0 * da * db * fit.sy + fit.m * db * db;
    *J = j;
    *a = A;
    *b = B;
    *kappa = j > 0.0 ? mo[2] / j : INFINITY;
}

// The device's reading of a GradRule (solver.h): true when the machine,
// fed J, asks next for the gradient at the evaluated point.  The quadratic's
// minimiser is computed as the machine computes it, without contraction; a
// disagreement at a boundary costs a gradient, never a wrong one, since the
// driver uses a speculative gradient only when the machine asks for exactly
// that point, fit and slot.
__host__ __device__ inline bool grad_follows(const GradRule &r, double J) {
#pragma clang fp contract(off)
    if (!(J == J)) return false;   // NaN
    switch (r.mode) {
    case GRAD_ALWAYS:
        return true;
    case GRAD_IF_ARMIJO: {
        if (!(J <= r.thr)) return false;
        if (!r.extrap) return true;
        const double tq = -r.gd * r.t * r.t / (2.0 * (J - r.phi - r.gd * r.t));
        return !(tq > 2.0 * r.t);
    }
    case GRAD_IF_BELOW:
        return J < r.thr;
    default:
        return false;
    }
}

// ---- batched launches: one launch serves several requests ----------------
// A job holds one request's arguments and the range [block0, block0 +
// nblocks) of the launch's blocks it owns; block blockIdx.x - block0 of a
// job runs exactly what block of that index runs in the request's own
// launch (same tiles, same reduction slots and order), so a request's
// results do not depend on what it is batched with.  Jobs are sorted by
// block0 and live in device memory.
struct WarpJob {
    VolDims vd;
    const void *f0, *mean, *U;
    WVec w;
    void *f;
    int block0, nblocks;
    const uint8_t *live = nullptr;   // brick liveness (launch_brick_live), or every voxel
};
struct FwdJob {                 // projection with the fit sums (FWD_SUMS)
    VolDims vd;
    Frame fr;
    int tiles_u, slab;
    const void *rays, *f;
    void *p;
    const void *y;
    FitArgs fit;                // reference (a0, b0) and, unless FIT_NONE, the objective's fit
    double *partials;
    uint32_t *counter;
    double *out;
    int block0, nblocks;
};
struct ResJob {
    int64_t M;
    const void *p, *y;
    FitArgs fa;
    const double *src;
    double *partials;
    uint32_t *counter;
    double *out;
    int block0, nblocks;
};
struct AdjJob {                 // back-projection of the residual + Jacobian chain
    VolDims vd;
    Frame fr;
    int nbx, nby;
    double hb;   // one ray's summed weight bound for one voxel
    const void *rays, *p, *y;
    double a, b;
    const void *f0, *mean, *U;
    WVec w;
    double *partials;
    uint32_t *counter;
    double *g_out;
    int block0, nblocks;
    int split;   // blocks per brick (adjoint_chain_split)
    const double *gate = nullptr;   // speculative: (a, b, go) in place of a, b; go = 0 exits
};

// ---- launchers (return the HIP error of the launch) ----------------------
hipError_t launch_fill_u32(uint32_t *p, int count, uint32_t value, hipStream_t s);
// Copies count <= 64 doubles to mapped host memory, then releases seq to *flag_host.
// The deferred end of a reduction whose blocks left partials only: one
// block of the producer's width (threads) sums the nblocks partials in
// grid_reduce's order, so the totals carry the same bits, stores
// scale * total to out[0..ns) and then publishes them like launch_publish.
hipError_t launch_publish_sum(const double *partials, int nblocks, int threads, int ns,
                              double scale, double *out, double *dst_host, uint32_t *flag_host,
                              uint32_t seq, hipStream_t s);
hipError_t launch_publish(const double *src, double *dst_host, int count, uint32_t *flag_host,
                          uint32_t seq, hipStream_t s);
// A gradient started behind its evaluation: launch_spec_decide (FP32
// one-pass evaluations) finishes the evaluation's moment sums (as
// launch_publish_sum with ns = 3, scale 1, does) into mo[0..2] and writes
// gate = (a, b, go) from them; the adjoint chain given the gate exits at
// once when go = 0 and otherwise takes (a, b) from it; launch_publish_spec
// then publishes (mo[0..2], a, b, go, g[0..ns)) with g summed from the
// chain's partials as launch_publish_sum does (zeros when go = 0).
hipError_t launch_spec_decide(const double *partials, int nblocks, int threads,
                              const FitArgs &fit, const GradRule &rule, double *mo, double *gate,
                              hipStream_t s);
// Scalar slot of a solve's speculative gate (a, b, go), inside the scalars
// the serving loop reads back per request.
constexpr int SCAL_GATE = 28;
// Scalars of a solve's workspace, and the slot of the fused evaluation's
// sums (eval_sums(K) values: see launch_drr_forward_eval).
constexpr int SCAL_COUNT = 160;
constexpr int SCAL_EVAL = 64;
static_assert(SCAL_EVAL + eval_sums(PCAS_MAX_K) <= SCAL_COUNT, "solve scalars");
// Several requests' gates in one launch (one FWD_THREADS-wide block each):
// from the moment partials of an FP32 evaluation (partials != null, summed
// as launch_spec_decide does, written to mo) or from an FP64 evaluation's
// (J, a, b) at jab.
struct SpecJob {
    const double *partials = nullptr;
    const double *jab = nullptr;
    int nblocks = 0;
    FitArgs fit{};
    GradRule rule{};
    double *mo = nullptr;
    double *gate = nullptr;
};
hipError_t launch_spec_decide_batch(const SpecJob *jobs, int njobs, hipStream_t s);
// gate from (J, a, b) already on the device (the two-pass residual's).
hipError_t launch_spec_decide_jab(const double *jab, const GradRule &rule, double *gate,
                                  hipStream_t s);
hipError_t launch_publish_spec(const double *partials, int nblocks, int threads, int ns,
                               double scale, const double *mo, const double *gate, double *g_out,
                               double *dst_host, uint32_t *flag_host, uint32_t seq,
                               hipStream_t s);

hipError_t launch_ray_table(pcas_dtype dt, const VolDims &v, const Frame &fr, void *rays,
                            hipStream_t s);

hipError_t launch_pca_dvf(pcas_dtype dt, int64_t N, int K, const void *mean, const void *U,
                          const double *w, void *dvf, hipStream_t s);
hipError_t launch_warp_trilinear(pcas_dtype dt, const VolDims &v, const void *f0, const void *dvf,
                                 void *f, hipStream_t s);
// With live (launch_brick_live's flags), only the voxels of live bricks are
// written: the projection of that geometry reads no other.
hipError_t launch_warp_pca(pcas_dtype dt, const VolDims &v, int K, const void *f0,
                           const void *mean, const void *U, const double *w, void *f,
                           hipStream_t s, const uint8_t *live = nullptr);
// live[brick] = 1 unless the projection of the brick's box with its one-voxel
// halo (back-projection bricks, x fastest) misses the detector by more than
// a pixel: no ray of the projection reaches a voxel of, or a sample cell
// touching, a dead brick.
hipError_t launch_brick_live(const VolDims &v, const Frame &fr, uint8_t *live, hipStream_t s);
// Voxels of the live bricks (the same test, on the host).
int64_t live_voxels(const VolDims &v, const Frame &fr);

// Forward projection.  If sums != nullptr also reduces, with r0 = p - a0 y -
// b0 for fit->a0, fit->b0 (zero when fit is null), (sum r0, sum r0*y,
// sum r0*r0) into sums[0..2] (double) via per-block partials and a
// last-block pass; partials needs drr_forward_blocks() * RED_SLOTS doubles,
// counter one zeroed uint32 (left zeroed on exit).  With counter == nullptr
// the launch leaves the block partials only (256-thread blocks), for
// launch_publish_sum to finish.  The same holds for the dot and chain
// launches below (the chain's blocks have ADJ_THREADS threads).
// The geometry-only launch plan (slab axis and thickness) is computed once
// per projection on the host.
// Blocks of a forward launch in tile shape ts; shape 0, the default, gives
// the most (workspaces are sized with it).
int drr_forward_blocks(int nu, int nv, int ts = 0);
struct ForwardPlan {
    int axis = 0, slab = 0, tile = 0;
};
ForwardPlan plan_drr_forward(pcas_dtype dt, const VolDims &v, const Frame &fr, int nvol);
hipError_t launch_drr_forward(pcas_dtype dt, const VolDims &v, const Frame &fr,
                              const ForwardPlan &plan, const void *rays, const void *f, void *p,
                              const void *y, const FitArgs *fit, double *partials,
                              uint32_t *counter, double *sums, hipStream_t s);
// Projections of the K volumes J[k][voxel] (plan for nvol = K) against the
// residual of the stored projection p: g_out[k] = 2 sum_rays (p - a y - b)
// (P J_k); partials needs drr_forward_blocks() * RED_SLOTS doubles, counter
// one zeroed uint32 (left zeroed on exit).
hipError_t launch_drr_forward_dot(pcas_dtype dt, const VolDims &v, const Frame &fr,
                                  const ForwardPlan &plan, int K, const void *rays, const void *J,
                                  const void *p, const void *y, double a, double b,
                                  double *partials, uint32_t *counter, double *g_out,
                                  hipStream_t s);
// The fused evaluation's projection (plan for nvol = K + 1): vols holds the
// warped image f and then its K Jacobian volumes J_k, each N values.  It
// stores p = P f and reduces eval_sums(K) sums with r0 = p - fit.a0 y -
// fit.b0 and q_k = P J_k (unrounded ray sums):
//   sums[0..2]          = (sum r0, sum r0 y, sum r0^2)   (the objective's moments)
//   sums[3..5]          = 0                              (room for J, a, b)
//   sums[6 + 3k .. +2]  = (sum q_k r0, sum q_k y, sum q_k)
//   then sum q_i q_j for i <= j, row by row (the Gauss-Newton matrix's part)
// so that for any fit (a, b), sum_rays (p - a y - b) q_k = sums[6+3k]
// - (a - a0) sums[7+3k] - (b - b0) sums[8+3k] (gradient_from_moments).
// counter == nullptr leaves block partials (RED_SLOTS_WIDE apart) for
// launch_publish_sum; otherwise the last block writes sums.
hipError_t launch_drr_forward_eval(pcas_dtype dt, const VolDims &v, const Frame &fr,
                                   const ForwardPlan &plan, int K, const void *rays,
                                   const void *vols, void *p, const void *y, const FitArgs &fit,
                                   double *partials, uint32_t *counter, double *sums,
                                   hipStream_t s);
// The warped image and its K Jacobian volumes in one voxel pass: out[0..N)
// = f (the quantity launch_warp_pca computes), out[(1 + k) N ..) = J_k (the
// quantity launch_jacobian computes), from one read of each voxel's f0
// neighbours.  With live (launch_brick_live), voxels of bricks no ray
// reaches are skipped (left as they were).
// Voxels per thread of the fused warp, and its block count for N voxels.
constexpr int WJ_VOX = 2;
int warp_jac_blocks(int64_t N);
hipError_t launch_warp_jac(pcas_dtype dt, const VolDims &v, int K, const void *f0,
                           const void *mean, const void *U, const double *w, void *out,
                           hipStream_t s, const uint8_t *live = nullptr);

// dJ/dw_k = 2 sum_rays (p - a y - b) q_k from the fused evaluation's sums
// taken about the reference fit (a0, b0) (see launch_drr_forward_eval).
// Compiled without contraction so that host and device agree.
__host__ __device__ inline void gradient_from_moments(const double *sums, int K, double a,
                                                      double b, double a0, double b0, double *g) {
#pragma clang fp contract(off)
    const double da = a - a0, db = b - b0;
    for (int k = 0; k < K; ++k) {
        const double *m = sums + 6 + 3 * k;
        g[k] = 2.0 * (m[0] - da * m[1] - db * m[2]);
    }
}

// The Gauss-Newton matrix of the reduced objective phi(w) = min_(a,b) J at
// the evaluated point, from the same sums: with the Jacobian of the
// projection dp/dw = Q = [q_1 .. q_K] (pixels x K) and Y = [y, 1],
//   fit refitted (Eq. A.1):  H = 2 (Q^T Q - Q^T Y (Y^T Y)^-1 Y^T Q)
//   fit fixed:               H = 2 Q^T Q
// (r's dependence on w through the refitted (a, b) is projected out; the
// residual's curvature term is dropped).  sy, syy, m: sum y, sum y^2 and the
// pixel count.  H: K x K, row-major.
__host__ __device__ inline void gn_matrix_from_moments(const double *sums, int K, bool refit,
                                                       double sy, double syy, double m,
                                                       double *H) {
#pragma clang fp contract(off)
    const double *qq = sums + 6 + 3 * K;
    const double det = syy * m - sy * sy;
    for (int i = 0, t = 0; i < K; ++i)
        for (int j = i; j < K; ++j, ++t) {
            double h = qq[t];
            if (refit) {
                // (Y^T Y)^-1 = [[m, -sy], [-sy, syy]] / det
                const double ui = sums[7 + 3 * i], vi = sums[8 + 3 * i];
                const double uj = sums[7 + 3 * j], vj = sums[8 + 3 * j];
                h -= (ui * (m * uj - sy * vj) + vi * (syy * vj - sy * uj)) / det;
            }
            H[i * K + j] = H[j * K + i] = 2.0 * h;
        }
}

// Back-projection.  If y != nullptr the residual r = p - a*y - b is formed
// on the fly from p (passed as r_or_p); otherwise r_or_p is r.  acc32
// (FP32 only): 32-bit fixed-point accumulators, else 64-bit.
hipError_t launch_drr_adjoint(pcas_dtype dt, const VolDims &v, const Frame &fr, const void *rays,
                              const void *r_or_p, const void *y, double a, double b, void *bp,
                              bool acc32, hipStream_t s);
// Back-projection of the residual r = p - a y - b fused with the Jacobian
// chain: g_out[k] = 2 sum_v (P^T r)(v) sum_c U_kc df/dx_c (bp stays on
// chip); partials needs drr_adjoint_chain_blocks() * RED_SLOTS doubles, counter
// one zeroed uint32 (left zeroed on exit).  FP32 accumulates in 32-bit
// fixed point, FP64 in 64-bit.
int drr_adjoint_blocks(const VolDims &v);
// The fused gradient (back-projection + chain) runs adjoint_chain_split(v)
// blocks per brick on small grids: drr_adjoint_chain_blocks(v) blocks, each
// leaving one block partial.
int adjoint_chain_split(const VolDims &v);
int drr_adjoint_chain_blocks(const VolDims &v);
// Bound on sum over rays and samples of the trilinear weight one voxel gets:
// over the whole grid, and over the voxels of one back-projection brick and
// its one-voxel halo.
double backprojection_weight_bound(const VolDims &v, const Frame &fr);
double brick_weight_bound_host(const VolDims &v, const Frame &fr, int brick);
hipError_t launch_drr_adjoint_chain(pcas_dtype dt, const VolDims &v, const Frame &fr, int K,
                                    const void *rays, const void *p, const void *y, double a,
                                    double b, const void *f0, const void *mean, const void *U,
                                    const double *w, double *partials, uint32_t *counter,
                                    double *g_out, hipStream_t s, const double *gate = nullptr);

// J[k][v] = sum_c U_kc(v) df/dx_c(v) at w (Eq. A.8 chain per voxel).
hipError_t launch_jacobian(pcas_dtype dt, const VolDims &v, int K, const void *f0,
                           const void *mean, const void *U, const double *w, void *J,
                           hipStream_t s);

int grad_w_blocks(int64_t N);
hipError_t launch_grad_w(pcas_dtype dt, const VolDims &v, int K, const void *f0, const void *mean,
                         const void *U, const double *w, const void *bp, double *partials,
                         uint32_t *counter, double *g_out, hipStream_t s);

// Sums over two length-M arrays: (sum a, sum a*b, sum a*a, sum b, sum b*b)
// into out[0..4]; partials needs sums_blocks(M) * RED_SLOTS doubles.
int sums_blocks(int64_t M);
hipError_t launch_pair_sums(pcas_dtype dt, int64_t M, const void *a, const void *b,
                            double *partials, uint32_t *counter, double *out, hipStream_t s);
// How the residual pass obtains (a, b):
//   FIT_COEF:  read a = src[0], b = src[1] (device)
//   FIT_REFIT: Eq. A.1 from sum p = src[0], sum p*y = src[1] (device) and the
//              host-known sum y, sum y^2 and pixel count (NaN if singular)
//   FIT_FIXED: the values a, b given here
// r = p - a*y - b; out[0] = J = sum r^2, out[1] = a, out[2] = b.
// r may be nullptr or alias p.
hipError_t launch_residual(pcas_dtype dt, int64_t M, const void *p, const void *y,
                           const FitArgs &fa, const double *src, void *r, double *partials,
                           uint32_t *counter, double *out, hipStream_t s);
// Intensity fit (Eq. A.1) from the sums produced by launch_pair_sums(p, y):
// writes stats[0..1] = (a, b) (NaN if singular) -- one thread.
hipError_t launch_fit_from_sums(int64_t M, int fit, const double *sums, double *stats,
                                hipStream_t s);

// Exact-path (Siddon) projection of the voxel-constant volume f into p.
hipError_t launch_siddon(pcas_dtype dt, const VolDims &v, const Frame &fr, const void *f, void *p,
                         hipStream_t s);

hipError_t launch_locate(pcas_dtype dt, const VolDims &v, int K, const void *mean, const void *U,
                         const double *w, const double c0[3], double tol, int max_iter,
                         double *out, hipStream_t s);

// Batched forms (jobs: device array sorted by block0; total_blocks = sum of
// the jobs' nblocks).  A job is filled like the corresponding single launch;
// the make_* helpers give its arguments and block count (block0 = 0).
int warp_blocks(int64_t N);
hipError_t launch_warp_pca_batch(pcas_dtype dt, int K, const WarpJob *jobs, int njobs,
                                 int total_blocks, hipStream_t s);
FwdJob make_fwd_job(const VolDims &v, const Frame &fr, const ForwardPlan &plan, const void *rays,
                    const void *f, void *p, const void *y, const FitArgs &fit, double *partials,
                    uint32_t *counter, double *sums);
hipError_t launch_drr_forward_sums_batch(pcas_dtype dt, int axis, const FwdJob *jobs, int njobs,
                                         int total_blocks, hipStream_t s);
// Several requests' fused-evaluation projections (launch_drr_forward_eval;
// J.f holds the K + 1 volumes, J.fit the reference fit) of one dtype, K,
// slab axis and tile shape in one launch.
hipError_t launch_drr_forward_eval_batch(pcas_dtype dt, int K, int axis, int tile,
                                         const FwdJob *jobs, int njobs, int total_blocks,
                                         hipStream_t s);
// Several requests' warps with their Jacobian volumes (launch_warp_jac; J.f
// receives the K + 1 volumes) of one dtype and K in one launch.
hipError_t launch_warp_jac_batch(pcas_dtype dt, int K, const WarpJob *jobs, int njobs,
                                 int total_blocks, hipStream_t s);
hipError_t launch_residual_batch(pcas_dtype dt, const ResJob *jobs, int njobs, int total_blocks,
                                 hipStream_t s);
AdjJob make_adj_job(const VolDims &v, const Frame &fr, int K, const void *rays, const void *p,
                    const void *y, double a, double b, const void *f0, const void *mean,
                    const void *U, const double *w, double *partials, uint32_t *counter,
                    double *g_out);
hipError_t launch_drr_adjoint_chain_batch(pcas_dtype dt, int K, const AdjJob *jobs, int njobs,
                                          int total_blocks, hipStream_t s);
// dst[i * count + t] = src[i][t] for i < n (src: device array of pointers).
// The deferred sum of one request's reduction in a serving pass: the
// partials of nblocks blocks of `width` threads (ns totals, 0 for none),
// stored as scale * total to out and to gathered slots [offset, offset + ns).
struct SumJob {
    const double *partials = nullptr;
    double *out = nullptr;
    double scale = 1.0;
    int nblocks = 0, width = 0, ns = 0, offset = 0;
    const double *gate = nullptr;   // a speculative gradient's (a, b, go): no sum when go = 0
};
// dst[b * count + t] = src[b][t] for n requests (one 512-thread block each),
// after finishing sums[b] when sums is given and sums[b].ns > 0.
hipError_t launch_gather_scalars(const double *const *src, double *dst, int n, int count,
                                 const SumJob *sums, hipStream_t s);

}  // namespace pcas
