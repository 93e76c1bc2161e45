// Host-side helpers shared by the C ABI and the serving loop: argument
// validation, launch-time descriptions, workspace layout, scalar read-back
// and error text.
#pragma once

#include <math.h>
#include <string.h>
#include <sys/syscall.h>
#include <unistd.h>

#include <string>

#include "internal.h"
#include "solver.h"

namespace pcas {
namespace host {

inline thread_local std::string g_last_error;

inline int hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return PCAS_EHIP;
}

#define HIPCHK(expr)                                        \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
    } while (0)

inline bool dtype_ok(int dt) { return dt == PCAS_F32 || dt == PCAS_F64; }
inline size_t esize(pcas_dtype dt) { return dt == PCAS_F32 ? 4 : 8; }
inline size_t rec_size(pcas_dtype dt) {
    return dt == PCAS_F32 ? sizeof(RayRec<float>) : sizeof(RayRec<double>);
}
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

inline int check_vol(const pcas_vol *v) {
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

inline int64_t nvox_of(const pcas_vol *v) { return (int64_t)v->n[0] * v->n[1] * v->n[2]; }

// Kernels address a volume with 32-bit byte offsets: it must stay below 2 GiB.
inline int check_vol_bytes(const pcas_vol *v, pcas_dtype dt) {
    return nvox_of(v) * (int64_t)esize(dt) < ((int64_t)1 << 31) ? PCAS_OK : PCAS_EINVAL;
}
inline int64_t npix_of(const pcas_proj *p) { return (int64_t)p->nu * p->nv; }

inline int check_proj(const pcas_proj *p, const pcas_vol *v) {
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

inline VolDims make_dims(const pcas_vol *v) {
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

inline Frame make_frame(const pcas_proj *p) {
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

inline bool finite_vec(const double *w, int K) {
    for (int k = 0; k < K; ++k)
        if (!isfinite(w[k])) return false;
    return true;
}

// True on the process's initial thread.
inline bool on_main_thread() { return (pid_t)syscall(SYS_gettid) == getpid(); }

// Scalar read-back through a per-thread mailbox in coherent, mapped host
// memory: MAILBOX_VALUES values and a flag word.  A one-wave kernel on the stream copies
// the values there and then publishes a sequence number in the flag; the
// host spins until it reads that number.  Every few thousand polls it
// queries the stream, so an error on the stream ends the wait with that
// error.  Against a copy and a stream synchronisation this saves, on each of
// a solve's round trips, the copy's dispatch and the synchronisation's
// wake-up.  The stream may still be retiring the publishing kernel when
// readback returns; work enqueued next runs after it.
struct Mailbox {
    double *vals = nullptr;
    uint32_t *flag = nullptr;
    uint32_t seq = 0;
    // A thread that exits returns its mailbox; the main thread's exit ends
    // the process, whose teardown releases it after the runtime's own.
    ~Mailbox() {
        if (vals && !on_main_thread()) (void)hipHostFree(vals);
    }
};

inline Mailbox *host_mailbox() {
    thread_local Mailbox mb;
    if (!mb.vals) {
        void *p = nullptr;
        if (hipHostMalloc(&p, MAILBOX_VALUES * sizeof(double) + 256,
                          hipHostMallocCoherent | hipHostMallocMapped) !=
            hipSuccess)
            return nullptr;
        mb.vals = (double *)p;
        mb.flag = (uint32_t *)((char *)p + MAILBOX_VALUES * sizeof(double));
        __atomic_store_n(mb.flag, 0u, __ATOMIC_RELEASE);
    }
    return &mb;
}

// Publishes count values with `launch(vals, flag, seq)` and waits for them.
template <class Launch>
inline int readback_with(double *host, int count, hipStream_t s, Launch launch) {
    if (count < 0 || count > MAILBOX_VALUES)
        return hip_fail(hipErrorInvalidValue, "scalar read-back size");
    Mailbox *mb = host_mailbox();
    if (!mb) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc(scalar mailbox)");
    if (++mb->seq == 0) mb->seq = 1;   // 0 is the flag's initial value
    const uint32_t seq = mb->seq;
    HIPCHK(launch(mb->vals, mb->flag, seq));
    for (uint32_t n = 1; __atomic_load_n(mb->flag, __ATOMIC_ACQUIRE) != seq; ++n) {
        __builtin_ia32_pause();
        if ((n & 4095u) == 0) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {   // the stream has drained, so the flag store is visible
                if (__atomic_load_n(mb->flag, __ATOMIC_ACQUIRE) == seq) break;
                return hip_fail(hipErrorUnknown, "scalar read-back: value not published");
            }
            if (q != hipErrorNotReady) return hip_fail(q, "hipStreamQuery");
        }
    }
    memcpy(host, mb->vals, count * sizeof(double));
    return PCAS_OK;
}

inline int readback(double *host, const double *dev, int count, hipStream_t s) {
    return readback_with(host, count, s, [&](double *vals, uint32_t *flag, uint32_t seq) {
        return launch_publish(dev, vals, count, flag, seq, s);
    });
}

// Finishes a deferred reduction (blocks of `threads` threads left nblocks
// partials) into dev[0..count) and reads the totals back.
inline int readback_sum(double *host, const double *partials, int nblocks, int threads,
                        double scale, double *dev, int count, hipStream_t s) {
    if (count < 1 || count > RED_SLOTS_WIDE) return hip_fail(hipErrorInvalidValue, "reduction width");
    return readback_with(host, count, s, [&](double *vals, uint32_t *flag, uint32_t seq) {
        return launch_publish_sum(partials, nblocks, threads, count, scale, dev, vals, flag, seq, s);
    });
}

// ---- workspace layouts ---------------------------------------------------

struct SolveWs {
    size_t rays, f, p, p2, vol2, partials, counters, scalars, live, total;   // vol2: bp, or the J_k
};

inline int red_blocks_max(const pcas_vol *v, const pcas_proj *p) {
    int m = drr_forward_blocks(p->nu, p->nv);
    const int nbr = drr_adjoint_chain_blocks(make_dims(v));
    m = m > nbr ? m : nbr;
    m = m > grad_w_blocks(nvox_of(v)) ? m : grad_w_blocks(nvox_of(v));
    m = m > sums_blocks(npix_of(p)) ? m : sums_blocks(npix_of(p));
    return m;
}

// vol2 holds bp, the K Jacobian volumes, or the warped image and its K
// Jacobian volumes (the fused evaluation); with_vol2 = false drops it (the
// fused back-projection + chain needs none of them).  The partials hold the
// widest reduction: the fused evaluation's forward blocks at RED_SLOTS_WIDE.
inline SolveWs solve_layout(pcas_dtype dt, const pcas_vol *v, const pcas_proj *p, int K,
                            bool with_vol2 = true) {
    SolveWs L;
    const size_t M = (size_t)npix_of(p), N = (size_t)nvox_of(v), es = esize(dt);
    size_t off = 0;
    L.rays = off; off += align256(M * rec_size(dt));
    L.f = off; off += align256(N * es);
    L.p = off; off += align256(M * es);
    L.p2 = off; off += align256(M * es);   // second projection slot of the line search
    L.vol2 = off; off += with_vol2 ? align256((size_t)(K + 1) * N * es) : 0;
    const size_t narrow = (size_t)red_blocks_max(v, p) * RED_SLOTS;
    const size_t wide = with_vol2 ? (size_t)drr_forward_blocks(p->nu, p->nv) * RED_SLOTS_WIDE : 0;
    L.partials = off; off += align256((narrow > wide ? narrow : wide) * sizeof(double));
    L.counters = off; off += 256;
    L.scalars = off; off += align256(SCAL_COUNT * sizeof(double));
    L.live = off; off += align256((size_t)drr_adjoint_blocks(make_dims(v)));   // brick liveness
    L.total = off;
    return L;
}

inline int check_opts(const pcas_opts *o) {
    if (!o) return PCAS_EINVAL;
    if (o->method < 0 || o->method > 2) return PCAS_EINVAL;
    if (o->grad_mode < 0 || o->grad_mode > 2) return PCAS_EINVAL;
    if (o->max_iter < 0 || o->max_backtracks < 1 || o->locate_max_iter < 1) return PCAS_EINVAL;
    if (!(o->mu0 > 0.0) || !(o->alpha > 0.0 && o->alpha < 1.0) || !(o->beta > 0.0 && o->beta < 1.0))
        return PCAS_EINVAL;
    if (!(o->mu_min >= 0.0) || !(o->gtol_rel >= 0.0) || !(o->xtol >= 0.0) || !(o->locate_tol > 0.0))
        return PCAS_EINVAL;
    if (!(o->beta_lo > 0.0 && o->beta_lo <= o->beta)) return PCAS_EINVAL;
    if (!(o->ls_extrap >= 0.0) || !isfinite(o->ls_extrap) || isnan(o->ftol_rel)) return PCAS_EINVAL;
    if (o->polish != 0 && o->polish != 1) return PCAS_EINVAL;
    if (o->speculate != 0 && o->speculate != 1) return PCAS_EINVAL;
    // the preconditioner is the fused evaluation's Gauss-Newton matrix, for CG
    if (o->precond != 0 && o->precond != 1) return PCAS_EINVAL;
    if (o->precond && (o->method != 1 || o->grad_mode != 2)) return PCAS_EINVAL;
    if (o->profile < 0 || o->profile > PCAS_PROFILE_ALL) return PCAS_EINVAL;
    if (o->locate && !finite_vec(o->c0_mm, 3)) return PCAS_EINVAL;
    return PCAS_OK;
}

// The solver's noise band of J: opts.ftol_rel when >= 0, else the rounding
// model at the evaluation type's unit roundoff with the measured image's
// sums (sum y, sum y^2) and pixel count.
inline NoiseModel noise_model(pcas_dtype dt, const pcas_opts &o, int64_t M, double sy,
                              double syy) {
    NoiseModel n;
    n.fixed = o.ftol_rel;
    n.u = dt == PCAS_F32 ? 5.9604644775390625e-08 : 1.1102230246251565e-16;   // 2^-24, 2^-53
    n.M = (double)M;
    n.sy = sy;
    n.syy = syy;
    return n;
}

}  // namespace host
}  // namespace pcas
