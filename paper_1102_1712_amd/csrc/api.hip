// C ABI of libpcasolve: argument validation (before any HIP call),
// workspace carving, and the per-projection solve driven from the host.
#include <math.h>
#include <string.h>

#include <chrono>
#include <string>
#include <vector>

#include "host.h"
#include "internal.h"
#include "solver.h"

using namespace pcas;

using namespace pcas::host;


// =========================================================================
extern "C" {

int pcas_abi_version(void) { return PCAS_ABI_VERSION; }

const char *pcas_status_string(int status) {
    switch (status) {
    case PCAS_OK: return "ok";
    case PCAS_EINVAL: return "invalid argument";
    case PCAS_EGEOM: return "invalid geometry";
    case PCAS_ESINGULAR: return "singular intensity fit (constant measured projection)";
    case PCAS_ENONFINITE: return "non-finite input or objective";
    case PCAS_EWORKSPACE: return "workspace missing, too small or misaligned";
    case PCAS_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char *pcas_last_error(void) { return g_last_error.c_str(); }

void pcas_default_opts(pcas_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->method = 1;
    o->max_iter = 30;
    o->fit_intensity = 1;
    o->max_backtracks = 12;
    o->mu0 = 1.0;
    o->alpha = 0.1;
    o->beta = 0.5;
    o->mu_min = 0.01;
    o->gtol_rel = 1e-9;
    o->beta_lo = 0.1;
    o->xtol = 1e-10;
    o->locate = 0;
    o->locate_max_iter = 100;
    o->locate_tol = 1e-9;
    o->ftol_rel = -1.0;
    o->grad_mode = 1;
    o->ls_extrap = 10.0;
    o->polish = 1;
    o->speculate = 1;
    o->precond = 0;
}

void pcas_paper_opts(pcas_opts *o) {
    pcas_default_opts(o);
    if (!o) return;
    o->method = 0;
    o->max_iter = 10;
    o->mu0 = 0.2;
    o->mu_min = 0.01;
}

size_t pcas_ray_table_bytes(pcas_dtype dtype, const pcas_proj *proj) {
    if (!dtype_ok(dtype) || !proj || proj->nu < 1 || proj->nv < 1) return 0;
    return (size_t)npix_of(proj) * rec_size(dtype);
}

int ray_table(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, void *rays,
              void *stream) {
    if (!dtype_ok(dtype)) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if ((st = check_proj(proj, vol))) return st;
    if (!rays || !aligned(rays, 16)) return PCAS_EINVAL;
    HIPCHK(launch_ray_table(dtype, make_dims(vol), make_frame(proj), rays, (hipStream_t)stream));
    return PCAS_OK;
}

int pca_dvf(pcas_dtype dtype, int64_t nvox, int32_t K, const void *mean, const void *U,
            const double *w, void *dvf_out, void *stream) {
    if (!dtype_ok(dtype) || nvox < 1 || nvox > (int64_t)INT32_MAX || K < 1 || K > PCAS_MAX_K)
        return PCAS_EINVAL;
    if (!U || !w || !dvf_out) return PCAS_EINVAL;
    if (!finite_vec(w, K)) return PCAS_ENONFINITE;
    HIPCHK(launch_pca_dvf(dtype, nvox, K, mean, U, w, dvf_out, (hipStream_t)stream));
    return PCAS_OK;
}

int warp_trilinear(pcas_dtype dtype, const pcas_vol *vol, const void *f0, const void *dvf,
                   void *f_out, void *stream) {
    if (!dtype_ok(dtype)) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if (!f0 || !dvf || !f_out || f_out == f0) return PCAS_EINVAL;
    HIPCHK(launch_warp_trilinear(dtype, make_dims(vol), f0, dvf, f_out, (hipStream_t)stream));
    return PCAS_OK;
}

int warp_pca(pcas_dtype dtype, const pcas_vol *vol, int32_t K, const void *f0, const void *mean,
             const void *U, const double *w, void *f_out, void *stream) {
    if (!dtype_ok(dtype) || K < 1 || K > PCAS_MAX_K) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if (!f0 || !U || !w || !f_out || f_out == f0) return PCAS_EINVAL;
    if (!finite_vec(w, K)) return PCAS_ENONFINITE;
    HIPCHK(launch_warp_pca(dtype, make_dims(vol), K, f0, mean, U, w, f_out, (hipStream_t)stream));
    return PCAS_OK;
}

int drr_forward(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *rays,
                const void *f, void *p_out, void *stream) {
    if (!dtype_ok(dtype)) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if ((st = check_proj(proj, vol))) return st;
    if (!rays || !aligned(rays, 16) || !f || !p_out) return PCAS_EINVAL;
    const VolDims vd = make_dims(vol);
    const Frame fr = make_frame(proj);
    HIPCHK(launch_drr_forward(dtype, vd, fr, plan_drr_forward(dtype, vd, fr, 1), rays, f, p_out,
                              nullptr, nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream));
    return PCAS_OK;
}

int drr_siddon(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *f,
               void *p_out, void *stream) {
    if (!dtype_ok(dtype)) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if ((st = check_proj(proj, vol))) return st;
    if (!f || !p_out) return PCAS_EINVAL;
    HIPCHK(launch_siddon(dtype, make_dims(vol), make_frame(proj), f, p_out, (hipStream_t)stream));
    return PCAS_OK;
}

static int adjoint_call(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj,
                        const void *rays, const void *r, void *bp_out, bool acc32, void *stream) {
    if (!dtype_ok(dtype)) return PCAS_EINVAL;
    if (acc32 && dtype != PCAS_F32) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if ((st = check_proj(proj, vol))) return st;
    if (!rays || !aligned(rays, 16) || !r || !bp_out) return PCAS_EINVAL;
    HIPCHK(launch_drr_adjoint(dtype, make_dims(vol), make_frame(proj), rays, r, nullptr, 0.0, 0.0,
                              bp_out, acc32, (hipStream_t)stream));
    return PCAS_OK;
}

int drr_adjoint(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *rays,
                const void *r, void *bp_out, void *stream) {
    return adjoint_call(dtype, vol, proj, rays, r, bp_out, false, stream);
}

int drr_adjoint32(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *rays,
                  const void *r, void *bp_out, void *stream) {
    return adjoint_call(dtype, vol, proj, rays, r, bp_out, true, stream);
}

double pcas_backprojection_bound(const pcas_vol *vol, const pcas_proj *proj) {
    if (check_vol(vol) || check_proj(proj, vol)) return -1.0;
    return backprojection_weight_bound(make_dims(vol), make_frame(proj));
}

double pcas_backprojection_brick_bound(const pcas_vol *vol, const pcas_proj *proj, int32_t brick) {
    if (check_vol(vol) || check_proj(proj, vol)) return -1.0;
    const VolDims v = make_dims(vol);
    if (brick < 0 || brick >= drr_adjoint_blocks(v)) return -1.0;
    return brick_weight_bound_host(v, make_frame(proj), brick);
}

int64_t pcas_live_voxels(const pcas_vol *vol, const pcas_proj *proj) {
    if (check_vol(vol) || check_proj(proj, vol)) return -1;
    return live_voxels(make_dims(vol), make_frame(proj));
}

int32_t backprojection_brick_count(const pcas_vol *vol) {
    if (check_vol(vol)) return -1;
    return drr_adjoint_blocks(make_dims(vol));
}

size_t residual_fit_workspace_bytes(int64_t npix) {
    if (npix < 1) return 0;
    return align256((size_t)sums_blocks(npix) * RED_SLOTS * sizeof(double)) + 512;
}

int residual_fit(pcas_dtype dtype, int64_t npix, const void *p, const void *y, int32_t fit_intensity,
                 void *r_out, double *stats_out, void *workspace, size_t workspace_bytes,
                 void *stream) {
    if (!dtype_ok(dtype) || npix < 1 || npix > (int64_t)INT32_MAX) return PCAS_EINVAL;
    if (!p || !y || !stats_out) return PCAS_EINVAL;
    if (!workspace || !aligned(workspace, 256) || workspace_bytes < residual_fit_workspace_bytes(npix))
        return PCAS_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)workspace;
    double *partials = (double *)base;
    base += align256((size_t)sums_blocks(npix) * RED_SLOTS * sizeof(double));
    uint32_t *counters = (uint32_t *)base;
    double *coef = (double *)(base + 256);
    HIPCHK(launch_fill_u32(counters, 2, 0u, s));
    HIPCHK(launch_pair_sums(dtype, npix, p, y, partials, &counters[0], stats_out + 3, s));
    HIPCHK(launch_fit_from_sums(npix, fit_intensity ? 1 : 0, stats_out + 3, coef, s));
    FitArgs fa{FIT_COEF, 0.0, 0.0, 0.0, 0.0, 0.0};
    HIPCHK(launch_residual(dtype, npix, p, y, fa, coef, r_out, partials, &counters[1], stats_out, s));
    return PCAS_OK;
}

size_t grad_w_workspace_bytes(pcas_dtype dtype, const pcas_vol *vol, int32_t K) {
    (void)K;
    if (!dtype_ok(dtype) || check_vol(vol) != PCAS_OK) return 0;
    return align256((size_t)grad_w_blocks(nvox_of(vol)) * RED_SLOTS * sizeof(double)) + 256;
}

int grad_w(pcas_dtype dtype, const pcas_vol *vol, int32_t K, const void *f0, const void *mean,
           const void *U, const double *w, const void *bp, double *g_out, void *workspace,
           size_t workspace_bytes, void *stream) {
    if (!dtype_ok(dtype) || K < 1 || K > PCAS_MAX_K) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if (!f0 || !U || !w || !bp || !g_out) return PCAS_EINVAL;
    if (!finite_vec(w, K)) return PCAS_ENONFINITE;
    if (!workspace || !aligned(workspace, 256) ||
        workspace_bytes < grad_w_workspace_bytes(dtype, vol, K))
        return PCAS_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    double *partials = (double *)workspace;
    uint32_t *counter = (uint32_t *)((char *)workspace +
                                     align256((size_t)grad_w_blocks(nvox_of(vol)) * RED_SLOTS *
                                              sizeof(double)));
    HIPCHK(launch_fill_u32(counter, 1, 0u, s));
    HIPCHK(launch_grad_w(dtype, make_dims(vol), K, f0, mean, U, w, bp, partials, counter, g_out, s));
    return PCAS_OK;
}

int tumour_position(pcas_dtype dtype, const pcas_vol *vol, int32_t K, const void *mean,
                    const void *U, const double *w, const double c0_mm[3], double tol,
                    int32_t max_iter, double *out, void *stream) {
    if (!dtype_ok(dtype) || K < 1 || K > PCAS_MAX_K) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if (!U || !w || !c0_mm || !out || !(tol > 0.0) || max_iter < 1) return PCAS_EINVAL;
    if (!finite_vec(w, K) || !finite_vec(c0_mm, 3)) return PCAS_ENONFINITE;
    HIPCHK(launch_locate(dtype, make_dims(vol), K, mean, U, w, c0_mm, tol, max_iter, out,
                         (hipStream_t)stream));
    return PCAS_OK;
}

size_t solve_projection_workspace(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj,
                                  int32_t K) {
    if (!dtype_ok(dtype) || K < 1 || K > PCAS_MAX_K || check_vol(vol) != PCAS_OK ||
        check_proj(proj, vol) != PCAS_OK)
        return 0;
    return solve_layout(dtype, vol, proj, K).total;
}

}  // extern "C"

// =========================================================================
// The solve.
namespace {

// Optional per-kernel timing: a pair of HIP events around each launch of
// the selected classes on the solve's stream, read once the solve has
// ended (reading them between a read-back and the next launch would put the
// runtime's event bookkeeping on the solve's critical path).
// A thread that exits destroys its events (see Mailbox).
struct EventPool : std::vector<hipEvent_t> {
    ~EventPool() {
        if (on_main_thread()) return;
        for (hipEvent_t e : *this) (void)hipEventDestroy(e);
    }
};
thread_local EventPool t_events;

struct Profile {
    unsigned mask = 0;   // bit c: time class c
    double ms[PCAS_K_CLASSES] = {0};
    int n[PCAS_K_CLASSES] = {0};
    struct Pending {
        int cls;
        size_t a, b;
    };
    std::vector<Pending> pending;
    size_t next = 0;

    hipError_t event(size_t i, hipEvent_t *e) {
        while (t_events.size() <= i) {
            hipEvent_t ev;
            hipError_t err = hipEventCreate(&ev);
            if (err != hipSuccess) return err;
            t_events.push_back(ev);
        }
        *e = t_events[i];
        return hipSuccess;
    }
    // Call after a read-back: every event recorded so far precedes the
    // publishing kernel on the stream, but the runtime may not have marked
    // the last ones complete yet, so those are waited for.  Event slots are
    // reused after a collect.
    hipError_t collect() {
        for (const Pending &p : pending) {
            float t = 0.f;
            hipError_t err = hipEventElapsedTime(&t, t_events[p.a], t_events[p.b]);
            if (err == hipErrorNotReady) {
                if ((err = hipEventSynchronize(t_events[p.b])) != hipSuccess) return err;
                err = hipEventElapsedTime(&t, t_events[p.a], t_events[p.b]);
            }
            if (err != hipSuccess) return err;
            ms[p.cls] += t;
            n[p.cls] += 1;
        }
        pending.clear();
        next = 0;
        return hipSuccess;
    }
};

struct Solver {
    pcas_dtype dt;
    VolDims vd;
    Frame fr;
    ForwardPlan fplan, fplan_k, fplan_e;   // projection of f; of the K Jacobian volumes; of both
    int K;
    int grad_mode = 0;
    int64_t M;
    const void *f0, *mean, *U, *y;
    char *ws;
    SolveWs L;
    hipStream_t s;
    int fit;
    double sy = 0.0, syy = 0.0;
    int n_fevals = 0, n_grads = 0;
    // Reference fit of the next refitted FP32 evaluation's moments (the last
    // fit found), and the slot and reference of the moments in scal()[0..2].
    double ref_a = 1.0, ref_b = 0.0;
    int mom_slot = -1;
    double mom_a0 = 0.0, mom_b0 = 0.0;
    double *mom_src = nullptr;   // where those moments are (scal() or the fused sums)
    Profile prof;
    // Speculative gradients (opts.speculate; FP32 one-pass evaluations with
    // the fused back-projection): the gradient at the last evaluated point,
    // launched behind the evaluation and gated on the GPU by the machine's
    // rule.  Valid until consumed or until the next evaluation; used only
    // when the machine asks for exactly that point, fit and slot.
    bool speculate = false;
    int spec_grads = 0;
    struct {
        bool valid = false;
        int slot = 0;
        double w[PCAS_MAX_K] = {0}, a = 0.0, b = 0.0, g[PCAS_MAX_K] = {0};
    } spec;

    // The fused evaluation (grad_mode 2): per line-search slot, the point
    // and the sums its projection left (launch_drr_forward_eval), from which
    // the gradient at any fit follows without another launch.
    struct Fused {
        bool valid = false;
        double w[PCAS_MAX_K] = {0};
        double a0 = 0.0, b0 = 0.0;
        double m[eval_sums(PCAS_MAX_K)] = {0};
    } fused[2];

    double *scal() const { return (double *)(ws + L.scalars); }
    uint32_t *counters() const { return (uint32_t *)(ws + L.counters); }

    template <class F> hipError_t timed(int cls, F &&launch) {
        const hipStream_t st = s;
        if (!(prof.mask >> cls & 1u)) return launch();
        hipEvent_t a, b;
        hipError_t e;
        const size_t ia = prof.next++, ib = prof.next++;
        if ((e = prof.event(ia, &a)) != hipSuccess || (e = prof.event(ib, &b)) != hipSuccess) return e;
        if ((e = hipEventRecord(a, st)) != hipSuccess) return e;
        if ((e = launch()) != hipSuccess) return e;
        if ((e = hipEventRecord(b, st)) != hipSuccess) return e;
        prof.pending.push_back({cls, ia, ib});
        return hipSuccess;
    }

    // Host time spent waiting in read-backs (report.wait_ms).
    double wait_ms = 0.0;
    template <class F> int waited(F &&read) {
        const auto t0 = std::chrono::steady_clock::now();
        const int st = read();
        wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                       .count();
        return st;
    }

    int sync_read(double *host, const double *dev, int count) {
        return waited([&] { return readback(host, dev, count, s); });
    }

    // The same for a reduction whose launch left block partials only (no
    // counter): the read-back kernel finishes the sum into dev[0..count).
    int sync_read_sum(double *host, int nblocks, int threads, double scale, double *dev,
                      int count) {
        return waited([&] {
            return readback_sum(host, (const double *)(ws + L.partials), nblocks, threads, scale,
                                dev, count, s);
        });
    }

    FitArgs fit_args(const double *ab_fixed) const {
        FitArgs fa{FIT_FIXED, 1.0, 0.0, sy, syy, (double)M};
        if (ab_fixed) {
            fa.a = ab_fixed[0];
            fa.b = ab_fixed[1];
        } else if (fit) {
            fa.mode = FIT_REFIT;
        }
        return fa;
    }

    // Projection buffer of a line-search slot (0 or 1).
    char *proj_slot(int slot) const { return ws + (slot ? L.p2 : L.p); }

    // J = ||p - a y - b||^2 for the projection in the slot, summed directly
    // over the residual; (a, b) refitted by Eq. A.1 unless fixed.
    // With a gradient rule and the point w of the slot's projection (an FP64
    // evaluation), the gradient at w comes back with J in one read-back.
    // The moments come from mom_src (the slot's evaluation left them there);
    // J, a, b go to jab_dst, and with `tail` the `ntail` values after them
    // come back in the same read-back.
    int residual(const double *ab_fixed, int slot, double *J, double *a, double *b,
                 const GradRule *rule = nullptr, const double *w = nullptr,
                 double *tail = nullptr, int ntail = 0) {
        FitArgs fa = fit_args(ab_fixed);
        if (fa.mode == FIT_REFIT) {   // the refit reads the moments of this slot's projection
            if (slot != mom_slot) return hip_fail(hipErrorInvalidValue, "refit without moments");
            fa.a0 = mom_a0;
            fa.b0 = mom_b0;
        }
        double *jab = mom_src + 3;
        HIPCHK(timed(PCAS_K_RESIDUAL, [&] {
            return launch_residual(dt, M, proj_slot(slot), y, fa, mom_src, nullptr,
                                   (double *)(ws + L.partials), &counters()[3], jab, s);
        }));
        double out[eval_sums(PCAS_MAX_K)];
        int st;
        if (speculate && rule && w && rule->mode != GRAD_NEVER) {
            HIPCHK(launch_spec_decide_jab(jab, *rule, scal() + SCAL_GATE, s));
            st = gated_gradient(w, slot, jab, out);
        } else {
            st = sync_read(out, jab, 3 + ntail);
        }
        if (st) return st;
        for (int j = 0; j < ntail; ++j) tail[j] = out[3 + j];
        *J = out[0];
        *a = out[1];
        *b = out[2];
        if (!isfinite(*a) || !isfinite(*b)) return PCAS_ESINGULAR;
        if (!isfinite(*J)) return PCAS_ENONFINITE;
        ref_a = *a;
        ref_b = *b;
        return PCAS_OK;
    }

    // Warp + projection at w into a slot, then J at the fit (one read-back).
    // FP32: the projection reduces moments about a reference fit (the fixed
    // one, else the last fit found), J and the fit follow from them on the
    // host, and the two-pass residual runs only if that sum would cancel.
    // FP64: moments of p itself and the two-pass residual.
    // With a gradient rule (the machine's, for this evaluation) and
    // speculation on, the gradient at w is started behind the projection and
    // comes back with the moments in the same read-back.
    int evaluate(const double *w, const double *ab_fixed, int slot, double *J, double *a,
                 double *b, const GradRule *rule = nullptr) {
        spec.valid = false;
        if (grad_mode == 2) return evaluate_fused(w, ab_fixed, slot, J, a, b);
        HIPCHK(timed(PCAS_K_WARP, [&] {
            return launch_warp_pca(dt, vd, K, f0, mean, U, w, ws + L.f, s,
                                   (const uint8_t *)(ws + L.live));
        }));
        const bool one_pass = dt == PCAS_F32;
        FitArgs ff = fit_args(ab_fixed);
        if (one_pass) {
            ff.a0 = ff.mode == FIT_FIXED ? ff.a : ref_a;
            ff.b0 = ff.mode == FIT_FIXED ? ff.b : ref_b;
        } else {
            ff.mode = FIT_NONE;
        }
        HIPCHK(timed(PCAS_K_DRR, [&] {
            return launch_drr_forward(dt, vd, fr, fplan, ws + L.rays, ws + L.f, proj_slot(slot), y,
                                      &ff, (double *)(ws + L.partials),
                                      one_pass ? nullptr : &counters()[0], scal(), s);
        }));
        ++n_fevals;
        mom_slot = slot;
        mom_a0 = ff.a0;
        mom_b0 = ff.b0;
        mom_src = scal();
        if (!one_pass) return residual(ab_fixed, slot, J, a, b, rule, w);
        double mo[3], kappa;
        const int nbf = drr_forward_blocks(fr.nu, fr.nv, fplan.tile);
        int st;
        if (speculate && rule && rule->mode != GRAD_NEVER) {
            HIPCHK(launch_spec_decide((const double *)(ws + L.partials), nbf, FWD_THREADS, ff, *rule,
                                      scal(), scal() + SCAL_GATE, s));
            st = gated_gradient(w, slot, scal(), mo);
        } else
            st = sync_read_sum(mo, nbf, FWD_THREADS, 1.0, scal(), 3);
        if (st) return st;
        objective_from_moments(mo, ff, J, a, b, &kappa);
        if (!isfinite(*a) || !isfinite(*b)) return PCAS_ESINGULAR;
        if (!(kappa <= MOMENT_KAPPA_MAX)) {   // cancellation: the two-pass sum at this fit
            const double ab[2] = {*a, *b};
            return residual(ab, slot, J, a, b);
        }
        if (!isfinite(*J)) return PCAS_ENONFINITE;
        ref_a = *a;
        ref_b = *b;
        return PCAS_OK;
    }

    // grad_mode 2: the warp and the K Jacobian volumes in one voxel pass,
    // then one projection of all K + 1 volumes that leaves the objective's
    // moments and the gradient's sums (launch_drr_forward_eval), read back
    // together.  FP32 forms J and the fit from the moments as evaluate()
    // does; FP64 takes them from the two-pass residual (moments of p
    // itself, a0 = b0 = 0), whose J, a, b land in front of the gradient's
    // sums so that one read-back returns both.
    int evaluate_fused(const double *w, const double *ab_fixed, int slot, double *J, double *a,
                       double *b) {
        Fused &F = fused[slot];
        F.valid = false;
        char *vols = ws + L.vol2;
        HIPCHK(timed(PCAS_K_WARP_JAC, [&] {
            return launch_warp_jac(dt, vd, K, f0, mean, U, w, vols, s,
                                   (const uint8_t *)(ws + L.live));
        }));
        const bool one_pass = dt == PCAS_F32;
        FitArgs ff = fit_args(ab_fixed);
        if (one_pass) {
            ff.a0 = ff.mode == FIT_FIXED ? ff.a : ref_a;
            ff.b0 = ff.mode == FIT_FIXED ? ff.b : ref_b;
        }
        double *sums = scal() + SCAL_EVAL;
        HIPCHK(timed(PCAS_K_DRR_EVAL, [&] {
            return launch_drr_forward_eval(dt, vd, fr, fplan_e, K, ws + L.rays, vols,
                                           proj_slot(slot), y, ff, (double *)(ws + L.partials),
                                           one_pass ? nullptr : &counters()[0], sums, s);
        }));
        ++n_fevals;
        mom_slot = slot;
        mom_a0 = ff.a0;
        mom_b0 = ff.b0;
        mom_src = sums;
        const int ns = eval_sums(K);
        int st;
        if (!one_pass) {
            if ((st = residual(ab_fixed, slot, J, a, b, nullptr, nullptr, F.m + 6, ns - 6)))
                return st;
        } else {
            const int nbf = drr_forward_blocks(fr.nu, fr.nv, fplan_e.tile);
            if ((st = sync_read_sum(F.m, nbf, EVAL_SUM_WIDTH, 1.0, sums, ns))) return st;
            double kappa;
            objective_from_moments(F.m, ff, J, a, b, &kappa);
            if (!isfinite(*a) || !isfinite(*b)) return PCAS_ESINGULAR;
            if (!(kappa <= MOMENT_KAPPA_MAX)) {   // cancellation: the two-pass sum at this fit
                const double ab[2] = {*a, *b};
                if ((st = residual(ab, slot, J, a, b))) return st;
            } else {
                if (!isfinite(*J)) return PCAS_ENONFINITE;
                ref_a = *a;
                ref_b = *b;
            }
        }
        F.valid = true;
        F.a0 = ff.a0;
        F.b0 = ff.b0;
        for (int k = 0; k < K; ++k) F.w[k] = w[k];
        return PCAS_OK;
    }

    // Behind an evaluation whose gate (a, b, go) is at scal()[32..34]: the
    // fused back-projection and chain at w in the slot, which exits at once
    // when the gate is shut (profile class PCAS_K_SPEC_SKIP), then one
    // read-back of the evaluation's three values at src (moments, or J, a, b)
    // into head[0..2] with the decision and the gradient.  An open gate
    // leaves the gradient at (w, a, b of the gate) for gradient() to take.
    int gated_gradient(const double *w, int slot, const double *src, double *head) {
        double *partials = (double *)(ws + L.partials);
        double *gate = scal() + SCAL_GATE;
        const unsigned both = (1u << PCAS_K_ADJOINT) | (1u << PCAS_K_SPEC_SKIP);
        const size_t mark = prof.pending.size();
        HIPCHK(timed(prof.mask >> PCAS_K_ADJOINT & 1u ? PCAS_K_ADJOINT : PCAS_K_SPEC_SKIP, [&] {
            return launch_drr_adjoint_chain(dt, vd, fr, K, ws + L.rays, proj_slot(slot), y, 0.0, 0.0,
                                            f0, mean, U, w, partials, nullptr, scal() + 8, s, gate);
        }));
        double out[6 + PCAS_MAX_K];
        const int nba = drr_adjoint_chain_blocks(vd);
        int st = waited([&] {
            return readback_with(out, 6 + K, s, [&](double *vals, uint32_t *flag, uint32_t seq) {
                return launch_publish_spec(partials, nba, ADJ_THREADS, K, 2.0, src, gate,
                                           scal() + 8, vals, flag, seq, s);
            });
        });
        if (st) return st;
        const bool go = out[5] != 0.0;
        if ((prof.mask & both) && prof.pending.size() > mark) {
            const int cls = go ? PCAS_K_ADJOINT : PCAS_K_SPEC_SKIP;
            if (prof.mask >> cls & 1u)
                prof.pending[mark].cls = cls;
            else
                prof.pending.erase(prof.pending.begin() + (long)mark);
        }
        for (int j = 0; j < 3; ++j) head[j] = out[j];
        if (go) {
            spec.valid = true;
            spec.slot = slot;
            for (int k = 0; k < K; ++k) {
                spec.w[k] = w[k];
                spec.g[k] = out[6 + k];
            }
            spec.a = out[3];
            spec.b = out[4];
        }
        return PCAS_OK;
    }

    // Gradient at the w whose projection is in the slot, at (a, b); with H,
    // also the Gauss-Newton matrix there when the fused evaluation gives it
    // (*h_ok says whether it did).
    int gradient(const double *w, double a, double b, int slot, double *g, double *H = nullptr,
                 bool *h_ok = nullptr) {
        if (h_ok) *h_ok = false;
        if (grad_mode == 2 && fused[slot].valid && !memcmp(fused[slot].w, w, K * sizeof(double))) {
            const Fused &F = fused[slot];
            gradient_from_moments(F.m, K, a, b, F.a0, F.b0, g);
            if (H) {
                gn_matrix_from_moments(F.m, K, fit != 0, sy, syy, (double)M, H);
                *h_ok = true;
            }
            ++n_grads;
            for (int k = 0; k < K; ++k)
                if (!isfinite(g[k])) return PCAS_ENONFINITE;
            return PCAS_OK;
        }
        if (spec.valid) {
            spec.valid = false;
            if (spec.slot == slot && !memcmp(spec.w, w, K * sizeof(double)) &&
                !memcmp(&spec.a, &a, sizeof(a)) && !memcmp(&spec.b, &b, sizeof(b))) {
                ++n_grads;
                ++spec_grads;
                for (int k = 0; k < K; ++k) {
                    g[k] = spec.g[k];
                    if (!isfinite(g[k])) return PCAS_ENONFINITE;
                }
                return PCAS_OK;
            }
        }
        if (grad_mode == 0) {
            HIPCHK(timed(PCAS_K_JACOBIAN, [&] {
                return launch_jacobian(dt, vd, K, f0, mean, U, w, ws + L.vol2, s);
            }));
            HIPCHK(timed(PCAS_K_DRR_DOT, [&] {
                return launch_drr_forward_dot(dt, vd, fr, fplan_k, K, ws + L.rays, ws + L.vol2,
                                              proj_slot(slot), y, a, b, (double *)(ws + L.partials),
                                              nullptr, scal() + 8, s);
            }));
        } else {
            // back-projection and Jacobian chain in one pass (bp stays on chip)
            HIPCHK(timed(PCAS_K_ADJOINT, [&] {
                return launch_drr_adjoint_chain(dt, vd, fr, K, ws + L.rays, proj_slot(slot), y, a, b, f0,
                                                mean, U, w, (double *)(ws + L.partials), nullptr,
                                                scal() + 8, s);
            }));
        }
        ++n_grads;
        const int nb = grad_mode == 0 ? drr_forward_blocks(fr.nu, fr.nv, fplan_k.tile)
                                      : drr_adjoint_chain_blocks(vd);
        int st = sync_read_sum(g, nb, grad_mode == 0 ? FWD_THREADS : ADJ_THREADS, 2.0, scal() + 8, K);
        if (st) return st;
        for (int k = 0; k < K; ++k)
            if (!isfinite(g[k])) return PCAS_ENONFINITE;
        return PCAS_OK;
    }

    // Everything a solve needs before its first evaluation: the ray table,
    // the measured image's sums and the fit's solvability.
    int prepare(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, int32_t K_,
                const void *f0_, const void *mean_, const void *U_, const void *y_, int fit_,
                int grad_mode_, unsigned profile, void *workspace, void *stream,
                int speculate_ = 0) {
        dt = dtype;
        vd = make_dims(vol);
        fr = make_frame(proj);
        K = K_;
        grad_mode = grad_mode_;
        speculate = speculate_ && grad_mode_ == 1;
        fplan = plan_drr_forward(dtype, vd, fr, 1);
        fplan_k = plan_drr_forward(dtype, vd, fr, K_);
        fplan_e = plan_drr_forward(dtype, vd, fr, K_ + 1);
        fused[0].valid = fused[1].valid = false;
        M = npix_of(proj);
        f0 = f0_;
        mean = mean_;
        U = U_;
        y = y_;
        ws = (char *)workspace;
        L = solve_layout(dtype, vol, proj, K_);
        mom_src = scal();
        s = (hipStream_t)stream;
        fit = fit_ ? 1 : 0;
        prof.mask = profile;
        HIPCHK(launch_fill_u32(counters(), 64, 0u, s));
        HIPCHK(timed(PCAS_K_RAYS, [&] { return launch_ray_table(dt, vd, fr, ws + L.rays, s); }));
        HIPCHK(launch_brick_live(vd, fr, (uint8_t *)(ws + L.live), s));
        // sums of the measured image: (sum y, sum y^2, ., ., .)
        HIPCHK(timed(PCAS_K_YSUMS, [&] {
            return launch_pair_sums(dt, M, y, y, (double *)(ws + L.partials), &counters()[2],
                                    scal() + 16, s);
        }));
        double ys[5];
        int st = sync_read(ys, scal() + 16, 5);
        if (st) return st;
        if (!isfinite(ys[0]) || !isfinite(ys[2])) return PCAS_ENONFINITE;
        sy = ys[0];
        syy = ys[2];
        if (fit) {
            const double m = (double)M, det = syy * m - sy * sy;
            if (!(fabs(det) > 1e-12 * syy * m)) return PCAS_ESINGULAR;
        }
        return PCAS_OK;
    }
};

// Runs the solve's state machine against this solver's operations.
int drive(Solver &S, SolveMachine &m) {
    while (!m.done()) {
        const SolveOp &op = m.op();
        double J, a, b;
        int st;
        switch (op.kind) {
        case OP_EVAL:
            if ((st = S.evaluate(op.w, op.fixed_ab ? op.ab : nullptr, op.slot, &J, &a, &b,
                                 &op.next_grad)))
                return st;
            m.eval_result(J, a, b);
            break;
        case OP_RESID:
            if ((st = S.residual(nullptr, op.slot, &J, &a, &b))) return st;
            m.eval_result(J, a, b);
            break;
        case OP_GRAD: {
            double g[PCAS_MAX_K], H[PCAS_MAX_K * PCAS_MAX_K];
            bool h_ok = false;
            if ((st = S.gradient(op.w, op.ab[0], op.ab[1], op.slot, g, H, &h_ok))) return st;
            m.grad_result(g, h_ok ? H : nullptr);
            break;
        }
        case OP_DONE:
            break;
        }
    }
    return PCAS_OK;
}

}  // namespace

extern "C" int solve_projection(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj,
                                int32_t K, const void *f0, const void *mean, const void *U,
                                const void *y, const double *w0, const pcas_opts *opts,
                                void *workspace, size_t workspace_bytes, double *w_out,
                                pcas_report *report, void *stream) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!dtype_ok(dtype) || K < 1 || K > PCAS_MAX_K) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if ((st = check_proj(proj, vol))) return st;
    if (!f0 || !U || !y || !w0 || !w_out || !report) return PCAS_EINVAL;
    if ((st = check_opts(opts))) return st;
    if (!finite_vec(w0, K)) return PCAS_ENONFINITE;
    const SolveWs L = solve_layout(dtype, vol, proj, K);
    if (!workspace || !aligned(workspace, 256) || workspace_bytes < L.total) return PCAS_EWORKSPACE;

    memset(report, 0, sizeof(*report));
    report->locate_iters = -1;
    Solver S;
    if ((st = S.prepare(dtype, vol, proj, K, f0, mean, U, y, opts->fit_intensity, opts->grad_mode,
                        (unsigned)opts->profile, workspace, stream, opts->speculate)))
        return st;

    SolveMachine m;
    m.start(*opts, K, noise_model(dtype, *opts, S.M, S.sy, S.syy), w0);
    st = drive(S, m);
    *report = m.report();
    report->spec_grads = S.spec_grads;
    if (st) return st;
    double w[PCAS_MAX_K];
    for (int k = 0; k < K; ++k) w_out[k] = w[k] = m.w()[k];

    if (opts->locate) {
        HIPCHK(S.timed(PCAS_K_LOCATE, [&] {
            return launch_locate(dtype, S.vd, K, mean, U, w, opts->c0_mm, opts->locate_tol,
                                 opts->locate_max_iter, S.scal() + 24, S.s);
        }));
        double loc[4];
        if ((st = S.sync_read(loc, S.scal() + 24, 4))) return st;
        for (int c = 0; c < 3; ++c) report->tumour_mm[c] = loc[c];
        report->locate_iters = (int32_t)loc[3];
    }
    if (S.prof.mask) HIPCHK(S.prof.collect());
    for (int c = 0; c < PCAS_K_CLASSES; ++c) {
        report->kernel_ms[c] = S.prof.ms[c];
        report->kernel_launches[c] = S.prof.n[c];
    }
    report->host_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    report->wait_ms = S.wait_ms;
    return PCAS_OK;
}

extern "C" int objective_gradient(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj,
                                  int32_t K, const void *f0, const void *mean, const void *U,
                                  const void *y, const double *w, int32_t fit_intensity,
                                  int32_t grad_mode, void *workspace, size_t workspace_bytes,
                                  double *out, void *stream) {
    if (!dtype_ok(dtype) || K < 1 || K > PCAS_MAX_K) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if ((st = check_proj(proj, vol))) return st;
    if (!f0 || !U || !y || !w || !out) return PCAS_EINVAL;
    if (grad_mode < 0 || grad_mode > 2) return PCAS_EINVAL;
    if (!finite_vec(w, K)) return PCAS_ENONFINITE;
    const SolveWs L = solve_layout(dtype, vol, proj, K);
    if (!workspace || !aligned(workspace, 256) || workspace_bytes < L.total) return PCAS_EWORKSPACE;
    Solver S;
    if ((st = S.prepare(dtype, vol, proj, K, f0, mean, U, y, fit_intensity, grad_mode, 0u,
                        workspace, stream)))
        return st;
    double J, a, b;
    if ((st = S.evaluate(w, nullptr, 0, &J, &a, &b))) return st;
    bool h_ok = false;
    if ((st = S.gradient(w, a, b, 0, out + 3, grad_mode == 2 ? out + 3 + K : nullptr, &h_ok)))
        return st;
    if (grad_mode == 2 && !h_ok) return hip_fail(hipErrorInvalidValue, "no Gauss-Newton matrix");
    out[0] = J;
    out[1] = a;
    out[2] = b;
    return PCAS_OK;
}
