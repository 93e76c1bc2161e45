// C ABI of libpcasolve: argument validation (before any HIP call),
// workspace carving, and the per-projection solve driven from the host.
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "internal.h"

using namespace pcas;

namespace {

thread_local std::string g_last_error;

int hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return PCAS_EHIP;
}

#define HIPCHK(expr)                                        \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
    } while (0)

bool dtype_ok(int dt) { return dt == PCAS_F32 || dt == PCAS_F64; }
size_t esize(pcas_dtype dt) { return dt == PCAS_F32 ? 4 : 8; }
size_t rec_size(pcas_dtype dt) { return dt == PCAS_F32 ? sizeof(RayRec<float>) : sizeof(RayRec<double>); }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_vol(const pcas_vol *v) {
    if (!v) return PCAS_EINVAL;
    int64_t N = 1;
    for (int c = 0; c < 3; ++c) {
        if (v->n[c] < 2) return PCAS_EINVAL;
        if (!(v->spacing[c] > 0.0) || !isfinite(v->spacing[c]) || !isfinite(v->origin[c]))
            return PCAS_EINVAL;
        N *= v->n[c];
    }
    if (N > (int64_t)INT32_MAX) return PCAS_EINVAL;
    return PCAS_OK;
}

int64_t nvox_of(const pcas_vol *v) { return (int64_t)v->n[0] * v->n[1] * v->n[2]; }

// Kernels address a volume with 32-bit byte offsets: it must stay below 2 GiB.
int check_vol_bytes(const pcas_vol *v, pcas_dtype dt) {
    return nvox_of(v) * (int64_t)esize(dt) < ((int64_t)1 << 31) ? PCAS_OK : PCAS_EINVAL;
}
int64_t npix_of(const pcas_proj *p) { return (int64_t)p->nu * p->nv; }

int check_proj(const pcas_proj *p, const pcas_vol *v) {
    if (!p) return PCAS_EINVAL;
    if (p->nu < 1 || p->nv < 1 || npix_of(p) > (int64_t)INT32_MAX) return PCAS_EINVAL;
    const double vals[] = {p->angle, p->sad, p->sid, p->pitch_u, p->pitch_v,
                           p->offset_u, p->offset_v, p->step};
    for (double x : vals)
        if (!isfinite(x)) return PCAS_EGEOM;
    if (!(p->sad > 0.0) || !(p->sid > p->sad) || !(p->pitch_u > 0.0) || !(p->pitch_v > 0.0) ||
        !(p->step > 0.0))
        return PCAS_EGEOM;
    // The source circles the SI axis at radius SAD; it must stay outside the
    // volume box grown by one voxel (the back-projection footprints project
    // that box through the source).
    double diag2 = 0.0;
    for (int xs = 0; xs < 2; ++xs)
        for (int ys = 0; ys < 2; ++ys) {
            const double x = xs ? v->origin[0] + v->n[0] * v->spacing[0] : v->origin[0] - v->spacing[0];
            const double y = ys ? v->origin[1] + v->n[1] * v->spacing[1] : v->origin[1] - v->spacing[1];
            if (sqrt(x * x + y * y) >= p->sad * (1.0 - 1e-9)) return PCAS_EGEOM;
        }
    for (int c = 0; c < 3; ++c) {
        const double e = (v->n[c] - 1) * v->spacing[c];
        diag2 += e * e;
    }
    if (sqrt(diag2) / p->step > 1.0e8) return PCAS_EGEOM;   // samples per ray must fit int32
    return PCAS_OK;
}

VolDims make_dims(const pcas_vol *v) {
    VolDims d;
    d.n0 = v->n[0];
    d.n1 = v->n[1];
    d.n2 = v->n[2];
    for (int c = 0; c < 3; ++c) {
        d.spacing[c] = v->spacing[c];
        d.inv_s[c] = 1.0 / v->spacing[c];
        d.origin[c] = v->origin[c];
    }
    return d;
}

Frame make_frame(const pcas_proj *p) {
    Frame f;
    const double st = sin(p->angle), ct = cos(p->angle);
    f.src[0] = p->sad * st;
    f.src[1] = -p->sad * ct;
    f.src[2] = 0.0;
    const double mag = (p->sid - p->sad) / p->sad;
    f.det[0] = -mag * f.src[0];
    f.det[1] = -mag * f.src[1];
    f.det[2] = 0.0;
    f.eu[0] = ct; f.eu[1] = st; f.eu[2] = 0.0;
    f.ev[0] = 0.0; f.ev[1] = 0.0; f.ev[2] = 1.0;
    f.en[0] = -st; f.en[1] = ct; f.en[2] = 0.0;
    f.sid = p->sid;
    f.pitch_u = p->pitch_u;
    f.pitch_v = p->pitch_v;
    f.offset_u = p->offset_u;
    f.offset_v = p->offset_v;
    f.step = p->step;
    f.nu = p->nu;
    f.nv = p->nv;
    return f;
}

bool finite_vec(const double *w, int K) {
    for (int k = 0; k < K; ++k)
        if (!isfinite(w[k])) return false;
    return true;
}

// Small pinned host buffer per thread for scalar read-backs.
double *host_scalars() {
    thread_local double *buf = nullptr;
    if (!buf) {
        if (hipHostMalloc((void **)&buf, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
            buf = nullptr;
    }
    return buf;
}

int readback(double *host, const double *dev, int count, hipStream_t s) {
    double *hb = host_scalars();
    if (!hb) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc(scalars)");
    HIPCHK(hipMemcpyAsync(hb, dev, count * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    memcpy(host, hb, count * sizeof(double));
    return PCAS_OK;
}

// ---- workspace layouts ---------------------------------------------------

struct SolveWs {
    size_t rays, f, p, vol2, partials, counters, scalars, total;   // vol2: bp, or the J_k
};

int red_blocks_max(const pcas_vol *v, const pcas_proj *p) {
    int m = drr_forward_blocks(p->nu, p->nv);
    const int nbr = drr_adjoint_blocks(make_dims(v));
    m = m > nbr ? m : nbr;
    m = m > grad_w_blocks(nvox_of(v)) ? m : grad_w_blocks(nvox_of(v));
    m = m > sums_blocks(npix_of(p)) ? m : sums_blocks(npix_of(p));
    return m;
}

SolveWs solve_layout(pcas_dtype dt, const pcas_vol *v, const pcas_proj *p, int K) {
    SolveWs L;
    const size_t M = (size_t)npix_of(p), N = (size_t)nvox_of(v), es = esize(dt);
    size_t off = 0;
    L.rays = off; off += align256(M * rec_size(dt));
    L.f = off; off += align256(N * es);
    L.p = off; off += align256(M * es);
    L.vol2 = off; off += align256((size_t)(K > 1 ? K : 1) * N * es);
    L.partials = off; off += align256((size_t)red_blocks_max(v, p) * RED_SLOTS * sizeof(double));
    L.counters = off; off += 256;
    L.scalars = off; off += align256(64 * sizeof(double));
    L.total = off;
    return L;
}

int check_opts(const pcas_opts *o) {
    if (!o) return PCAS_EINVAL;
    if (o->method != 0 && o->method != 1) return PCAS_EINVAL;
    if (o->grad_mode != 0 && o->grad_mode != 1) return PCAS_EINVAL;
    if (o->max_iter < 0 || o->max_backtracks < 1 || o->locate_max_iter < 1) return PCAS_EINVAL;
    if (!(o->mu0 > 0.0) || !(o->alpha > 0.0 && o->alpha < 1.0) || !(o->beta > 0.0 && o->beta < 1.0))
        return PCAS_EINVAL;
    if (!(o->mu_min >= 0.0) || !(o->gtol_rel >= 0.0) || !(o->xtol >= 0.0) || !(o->locate_tol > 0.0))
        return PCAS_EINVAL;
    if (!(o->beta_lo > 0.0 && o->beta_lo <= o->beta)) return PCAS_EINVAL;
    if (o->locate && !finite_vec(o->c0_mm, 3)) return PCAS_EINVAL;
    return PCAS_OK;
}

}  // namespace

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
                              nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream));
    return PCAS_OK;
}

int drr_adjoint(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, const void *rays,
                const void *r, void *bp_out, void *stream) {
    if (!dtype_ok(dtype)) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if ((st = check_proj(proj, vol))) return st;
    if (!rays || !aligned(rays, 16) || !r || !bp_out) return PCAS_EINVAL;
    HIPCHK(launch_drr_adjoint(dtype, make_dims(vol), make_frame(proj), rays, r, nullptr, 0.0, 0.0,
                              bp_out, (hipStream_t)stream));
    return PCAS_OK;
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

// Optional per-kernel timing: a pair of HIP events around each launch on
// the solve's stream, read after the next synchronisation.
thread_local std::vector<hipEvent_t> t_events;

struct Profile {
    bool on = false;
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
    // Call after the stream has been synchronised.
    hipError_t collect() {
        for (const Pending &p : pending) {
            float t = 0.f;
            hipError_t err = hipEventElapsedTime(&t, t_events[p.a], t_events[p.b]);
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
    ForwardPlan fplan, fplan_k;   // projection of f; of the K Jacobian volumes
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
    Profile prof;

    double *scal() const { return (double *)(ws + L.scalars); }
    uint32_t *counters() const { return (uint32_t *)(ws + L.counters); }

    template <class F> hipError_t timed(int cls, F &&launch) {
        if (!prof.on) return launch();
        hipEvent_t a, b;
        hipError_t e;
        const size_t ia = prof.next++, ib = prof.next++;
        if ((e = prof.event(ia, &a)) != hipSuccess || (e = prof.event(ib, &b)) != hipSuccess) return e;
        if ((e = hipEventRecord(a, s)) != hipSuccess) return e;
        if ((e = launch()) != hipSuccess) return e;
        if ((e = hipEventRecord(b, s)) != hipSuccess) return e;
        prof.pending.push_back({cls, ia, ib});
        return hipSuccess;
    }

    int sync_read(double *host, const double *dev, int count) {
        int st = readback(host, dev, count, s);
        if (st) return st;
        if (prof.on) HIPCHK(prof.collect());
        return PCAS_OK;
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

    // J = ||p - a y - b||^2 for the projection in the p buffer, summed
    // directly over the residual; (a, b) refitted by Eq. A.1 unless fixed.
    int residual(const double *ab_fixed, double *J, double *a, double *b) {
        const FitArgs fa = fit_args(ab_fixed);
        HIPCHK(timed(PCAS_K_RESIDUAL, [&] {
            return launch_residual(dt, M, ws + L.p, y, fa, scal(), nullptr,
                                   (double *)(ws + L.partials), &counters()[3], scal() + 3, s);
        }));
        double out[3];
        int st = sync_read(out, scal() + 3, 3);
        if (st) return st;
        *J = out[0];
        *a = out[1];
        *b = out[2];
        if (!isfinite(*a) || !isfinite(*b)) return PCAS_ESINGULAR;
        if (!isfinite(*J)) return PCAS_ENONFINITE;
        return PCAS_OK;
    }

    // Warp + projection at w, then the residual pass (one read-back).
    int evaluate(const double *w, const double *ab_fixed, double *J, double *a, double *b) {
        HIPCHK(timed(PCAS_K_WARP, [&] {
            return launch_warp_pca(dt, vd, K, f0, mean, U, w, ws + L.f, s);
        }));
        HIPCHK(timed(PCAS_K_DRR, [&] {
            return launch_drr_forward(dt, vd, fr, fplan, ws + L.rays, ws + L.f, ws + L.p, y,
                                      (double *)(ws + L.partials), &counters()[0], scal(), s);
        }));
        ++n_fevals;
        return residual(ab_fixed, J, a, b);
    }

    // Gradient at the w whose projection is in the p buffer, at (a, b).
    int gradient(const double *w, double a, double b, double *g) {
        if (grad_mode == 0) {
            HIPCHK(timed(PCAS_K_JACOBIAN, [&] {
                return launch_jacobian(dt, vd, K, f0, mean, U, w, ws + L.vol2, s);
            }));
            HIPCHK(timed(PCAS_K_DRR_DOT, [&] {
                return launch_drr_forward_dot(dt, vd, fr, fplan_k, K, ws + L.rays, ws + L.vol2,
                                              ws + L.p, y, a, b, (double *)(ws + L.partials),
                                              &counters()[1], scal() + 8, s);
            }));
        } else {
            // back-projection and Jacobian chain in one pass (bp stays on chip)
            HIPCHK(timed(PCAS_K_ADJOINT, [&] {
                return launch_drr_adjoint_chain(dt, vd, fr, K, ws + L.rays, ws + L.p, y, a, b, f0,
                                                mean, U, w, (double *)(ws + L.partials),
                                                &counters()[1], scal() + 8, s);
            }));
        }
        ++n_grads;
        int st = sync_read(g, scal() + 8, K);
        if (st) return st;
        for (int k = 0; k < K; ++k)
            if (!isfinite(g[k])) return PCAS_ENONFINITE;
        return PCAS_OK;
    }

    // Everything a solve needs before its first evaluation: the ray table,
    // the measured image's sums and the fit's solvability.
    int prepare(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj, int32_t K_,
                const void *f0_, const void *mean_, const void *U_, const void *y_, int fit_,
                int grad_mode_, bool profile, void *workspace, void *stream) {
        dt = dtype;
        vd = make_dims(vol);
        fr = make_frame(proj);
        K = K_;
        grad_mode = grad_mode_;
        fplan = plan_drr_forward(dtype, vd, fr, 1);
        fplan_k = plan_drr_forward(dtype, vd, fr, K_);
        M = npix_of(proj);
        f0 = f0_;
        mean = mean_;
        U = U_;
        y = y_;
        ws = (char *)workspace;
        L = solve_layout(dtype, vol, proj, K_);
        s = (hipStream_t)stream;
        fit = fit_ ? 1 : 0;
        prof.on = profile;
        HIPCHK(launch_fill_u32(counters(), 64, 0u, s));
        HIPCHK(timed(PCAS_K_RAYS, [&] { return launch_ray_table(dt, vd, fr, ws + L.rays, s); }));
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

double dot(const double *a, const double *b, int K) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += a[k] * b[k];
    return s;
}

// Appendix algorithm: alternate Eq. A.1 with the normalised gradient step of
// Eq. A.2, the step from Armijo backtracking with (a, b) held fixed.
int run_paper(Solver &S, const pcas_opts &o, double *w, pcas_report *rep) {
    const int K = S.K;
    double a, b, J, g[PCAS_MAX_K], d[PCAS_MAX_K], wt[PCAS_MAX_K];
    int st = S.evaluate(w, nullptr, &J, &a, &b);       // step 1 at w0
    if (st) return st;
    rep->J0 = J;
    rep->status = PCAS_STOP_MAXITER;
    for (int it = 0; it < o.max_iter; ++it) {
        if (it > 0 && (st = S.residual(nullptr, &J, &a, &b))) return st;   // step 1
        rep->J = J;
        rep->a = a;
        rep->b = b;
        if ((st = S.gradient(w, a, b, g))) return st;
        const double gn = sqrt(dot(g, g, K));
        if (it == 0) rep->gnorm0 = gn;
        rep->gnorm = gn;
        if (gn == 0.0 || J == 0.0) {
            rep->status = PCAS_STOP_CONVERGED;
            return PCAS_OK;
        }
        for (int k = 0; k < K; ++k) d[k] = g[k] / gn;                   // step 2
        double mu = o.mu0;
        const double ab[2] = {a, b};
        for (;;) {
            for (int k = 0; k < K; ++k) wt[k] = w[k] - mu * d[k];
            double Jt, at, bt;
            if ((st = S.evaluate(wt, ab, &Jt, &at, &bt))) return st;
            if (Jt <= J - o.alpha * mu * gn) break;
            mu *= o.beta;
            if (mu < o.mu_min) {
                rep->status = PCAS_STOP_CONVERGED;
                return PCAS_OK;
            }
        }
        for (int k = 0; k < K; ++k) w[k] = wt[k];
        rep->iters = it + 1;
    }
    if (o.max_iter > 0 && (st = S.residual(nullptr, &J, &a, &b))) return st;
    rep->a = a;
    rep->b = b;
    rep->J = J;
    return PCAS_OK;
}

// PR+ nonlinear CG on the reduced objective phi(w) = min_{a,b} J(w, a, b).
int run_cg(Solver &S, const pcas_opts &o, double *w, pcas_report *rep) {
    const int K = S.K;
    const double ftol = o.ftol_rel >= 0.0 ? o.ftol_rel : (S.dt == PCAS_F32 ? 1e-8 : 0.0);
    double phi, a, b, g[PCAS_MAX_K], d[PCAS_MAX_K], wt[PCAS_MAX_K], gnew[PCAS_MAX_K];
    int st = S.evaluate(w, nullptr, &phi, &a, &b);
    if (st) return st;
    if ((st = S.gradient(w, a, b, g))) return st;
    rep->J0 = phi;
    const double g0 = sqrt(dot(g, g, K));
    rep->gnorm0 = g0;
    for (int k = 0; k < K; ++k) d[k] = -g[k];
    bool restart = true, first = true;
    double t_prev = 0.0, gd_prev = 0.0;
    int it = 0;
    rep->status = PCAS_STOP_MAXITER;
    while (it < o.max_iter) {
        const double gn = sqrt(dot(g, g, K));
        if (gn <= o.gtol_rel * g0 || phi == 0.0) {
            rep->status = PCAS_STOP_CONVERGED;
            break;
        }
        double gd = dot(g, d, K);
        if (gd >= 0.0) {
            for (int k = 0; k < K; ++k) d[k] = -g[k];
            gd = -gn * gn;
            restart = true;
        }
        const double dn = sqrt(dot(d, d, K));
        double t = first ? o.mu0 / dn : t_prev * gd_prev / gd;
        bool accepted = false, at_noise = false;
        double phi_t = 0.0, a_t = 0.0, b_t = 0.0;
        for (int bt = 0; bt < o.max_backtracks; ++bt) {
            if (t * dn < o.xtol) break;
            for (int k = 0; k < K; ++k) wt[k] = w[k] + t * d[k];
            if ((st = S.evaluate(wt, nullptr, &phi_t, &a_t, &b_t))) return st;
            if (phi_t <= phi + o.alpha * t * gd) {
                accepted = true;
                break;
            }
            if (fabs(phi_t - phi) <= ftol * phi) {   // below the objective's noise
                at_noise = true;
                break;
            }
            const double tq = -gd * t * t / (2.0 * (phi_t - phi - gd * t));
            const double lo = o.beta_lo * t, hi = o.beta * t;
            t = tq < lo ? lo : (tq > hi ? hi : tq);
        }
        if (at_noise) {
            rep->status = PCAS_STOP_CONVERGED;
            break;
        }
        if (!accepted) {
            if (restart) {
                rep->status = PCAS_STOP_LINESEARCH;
                break;
            }
            for (int k = 0; k < K; ++k) d[k] = -g[k];
            restart = true;
            continue;
        }
        for (int k = 0; k < K; ++k) w[k] = wt[k];
        phi = phi_t;
        a = a_t;
        b = b_t;
        if ((st = S.gradient(w, a, b, gnew))) return st;
        double num = 0.0;
        for (int k = 0; k < K; ++k) num += gnew[k] * (gnew[k] - g[k]);
        double beta_pr = num / dot(g, g, K);
        beta_pr = beta_pr > 0.0 ? beta_pr : 0.0;
        for (int k = 0; k < K; ++k) {
            d[k] = -gnew[k] + beta_pr * d[k];
            g[k] = gnew[k];
        }
        t_prev = t;
        gd_prev = gd;
        restart = false;
        first = false;
        ++it;
    }
    rep->iters = it;
    rep->J = phi;
    rep->a = a;
    rep->b = b;
    rep->gnorm = sqrt(dot(g, g, K));
    return PCAS_OK;
}

}  // namespace

extern "C" int solve_projection(pcas_dtype dtype, const pcas_vol *vol, const pcas_proj *proj,
                                int32_t K, const void *f0, const void *mean, const void *U,
                                const void *y, const double *w0, const pcas_opts *opts,
                                void *workspace, size_t workspace_bytes, double *w_out,
                                pcas_report *report, void *stream) {
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
                        opts->profile != 0, workspace, stream)))
        return st;

    double w[PCAS_MAX_K];
    for (int k = 0; k < K; ++k) w[k] = w0[k];
    st = opts->method == 0 ? run_paper(S, *opts, w, report) : run_cg(S, *opts, w, report);
    report->n_fevals = S.n_fevals;
    report->n_grads = S.n_grads;
    if (st) return st;
    for (int k = 0; k < K; ++k) w_out[k] = w[k];

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
    for (int c = 0; c < PCAS_K_CLASSES; ++c) {
        report->kernel_ms[c] = S.prof.ms[c];
        report->kernel_launches[c] = S.prof.n[c];
    }
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
    if (grad_mode != 0 && grad_mode != 1) return PCAS_EINVAL;
    if (!finite_vec(w, K)) return PCAS_ENONFINITE;
    const SolveWs L = solve_layout(dtype, vol, proj, K);
    if (!workspace || !aligned(workspace, 256) || workspace_bytes < L.total) return PCAS_EWORKSPACE;
    Solver S;
    if ((st = S.prepare(dtype, vol, proj, K, f0, mean, U, y, fit_intensity, grad_mode, false,
                        workspace, stream)))
        return st;
    double J, a, b;
    if ((st = S.evaluate(w, nullptr, &J, &a, &b))) return st;
    if ((st = S.gradient(w, a, b, out + 3))) return st;
    out[0] = J;
    out[1] = a;
    out[2] = b;
    return PCAS_OK;
}
