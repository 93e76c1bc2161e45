// a1: per-projection ray table, plus a small fill kernel.
#include "device_util.h"

namespace pcas {

__global__ void k_fill_u32(uint32_t *p, int count, uint32_t value) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

hipError_t launch_fill_u32(uint32_t *p, int count, uint32_t value, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

// Scalar read-back.  One wave copies up to MAILBOX_VALUES values into host
// memory that the GPU writes through (coherent, mapped), waits for those
// stores, and then stores `seq` to the flag word with a system-scope
// release: a host thread that loads `seq` there (acquire) also sees the
// values.
__global__ __launch_bounds__(64) void k_publish(const double *__restrict__ src, double *dst, int count,
                                                uint32_t *flag, uint32_t seq) {
    const int i = threadIdx.x;
    for (int t = i; t < count; t += 64) dst[t] = src[t];
    __threadfence_system();
    if (i == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_publish(const double *src, double *dst_host, int count, uint32_t *flag_host,
                          uint32_t seq, hipStream_t s) {
    if (count < 0 || count > MAILBOX_VALUES) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, src, dst_host, count, flag_host, seq);
    return hipGetLastError();
}

// The deferred end of a reduction (launch_publish_sum): one block of the
// producer's width finishes the sum with the same code as grid_reduce's last
// block, stores the totals on the device and publishes them as k_publish
// does.  The producing kernel has ended, so plain loads see its partials.
template <int NS>
__global__ __launch_bounds__(1024) void k_publish_sum(const double *__restrict__ partials,
                                                      int nblocks, double scale,
                                                      double *__restrict__ out, double *dst,
                                                      uint32_t *flag, uint32_t seq) {
    double tot[NS];
    __shared__ double tot_s[NS];
    sum_partials<NS, false>(partials, nblocks, scale, (int)blockDim.x, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NS; ++j) tot_s[j] = tot[j];
    }
    __syncthreads();
    // the first wave stores the totals, one per lane, then publishes
    if (threadIdx.x < 64) {
        for (int j = threadIdx.x; j < NS; j += 64) {
            out[j] = tot_s[j];
            dst[j] = tot_s[j];
        }
        __threadfence_system();
        if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

hipError_t launch_publish_sum(const double *partials, int nblocks, int threads, int ns,
                              double scale, double *out, double *dst_host, uint32_t *flag_host,
                              uint32_t seq, hipStream_t s) {
    if (nblocks < 1 || threads < 64 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
    switch (ns) {
#define PCAS_PUBLISH_SUM(N)                                                                        \
    case N:                                                                                        \
        hipLaunchKernelGGL(k_publish_sum<N>, dim3(1), dim3(threads), 0, s, partials, nblocks,      \
                           scale, out, dst_host, flag_host, seq);                                  \
        break;
        PCAS_PUBLISH_SUM(1)
        PCAS_PUBLISH_SUM(2)
        PCAS_PUBLISH_SUM(3)
        PCAS_PUBLISH_SUM(4)
        PCAS_PUBLISH_SUM(5)
        PCAS_PUBLISH_SUM(6)
        PCAS_PUBLISH_SUM(7)
        PCAS_PUBLISH_SUM(8)
        // the fused evaluation's sums, eval_sums(1..8)
        PCAS_PUBLISH_SUM(10)
        PCAS_PUBLISH_SUM(15)
        PCAS_PUBLISH_SUM(21)
        PCAS_PUBLISH_SUM(28)
        PCAS_PUBLISH_SUM(36)
        PCAS_PUBLISH_SUM(45)
        PCAS_PUBLISH_SUM(55)
        PCAS_PUBLISH_SUM(66)
#undef PCAS_PUBLISH_SUM
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Speculative gradient, first half: finishes the projection's moment sums
// exactly as k_publish_sum<3> does (same block width, same order), stores
// them at mo[0..2], and from them the fit and J as the host does
// (objective_from_moments).  gate = (a, b, go): go = 1 when the fit is
// regular, the one-pass sum does not cancel (kappa <= MOMENT_KAPPA_MAX, else
// the host recomputes J by two passes) and the machine's rule says a
// gradient at this point follows.
__global__ __launch_bounds__(1024) void k_spec_decide(const double *__restrict__ partials,
                                                      int nblocks, FitArgs fit, GradRule rule,
                                                      double *__restrict__ mo,
                                                      double *__restrict__ gate) {
    double tot[3];
    sum_partials<3, false>(partials, nblocks, 1.0, (int)blockDim.x, tot);
    if (threadIdx.x == 0) {
        double J, a, b, kappa;
        objective_from_moments(tot, fit, &J, &a, &b, &kappa);
        const bool go = isfinite(a) && isfinite(b) && kappa <= MOMENT_KAPPA_MAX && isfinite(J) &&
                        grad_follows(rule, J);
        for (int j = 0; j < 3; ++j) mo[j] = tot[j];
        gate[0] = a;
        gate[1] = b;
        gate[2] = go ? 1.0 : 0.0;
    }
}

// The same decision from an objective already summed on the device:
// jab = (J, a, b) of the two-pass residual (the FP64 evaluation).
__global__ void k_spec_decide_jab(const double *__restrict__ jab, GradRule rule,
                                  double *__restrict__ gate) {
    if (threadIdx.x != 0) return;
    const double J = jab[0], a = jab[1], b = jab[2];
    const bool go = isfinite(a) && isfinite(b) && isfinite(J) && grad_follows(rule, J);
    gate[0] = a;
    gate[1] = b;
    gate[2] = go ? 1.0 : 0.0;
}

hipError_t launch_spec_decide_jab(const double *jab, const GradRule &rule, double *gate,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_spec_decide_jab, dim3(1), dim3(64), 0, s, jab, rule, gate);
    return hipGetLastError();
}

// The serving loop's gates, one block per request (see SpecJob).
__global__ __launch_bounds__(FWD_THREADS) void k_spec_decide_batch(const SpecJob *__restrict__ jobs) {
    const SpecJob J = jobs[blockIdx.x];
    double tot[3] = {0.0, 0.0, 0.0};
    if (J.partials) sum_partials<3, false>(J.partials, J.nblocks, 1.0, FWD_THREADS, tot);
    if (threadIdx.x != 0) return;
    double Jv, a, b, kappa = 0.0;
    if (J.partials) {
        objective_from_moments(tot, J.fit, &Jv, &a, &b, &kappa);
        for (int j = 0; j < 3; ++j) J.mo[j] = tot[j];
    } else {
        Jv = J.jab[0];
        a = J.jab[1];
        b = J.jab[2];
    }
    const bool go = isfinite(a) && isfinite(b) && isfinite(Jv) && kappa <= MOMENT_KAPPA_MAX &&
                    grad_follows(J.rule, Jv);
    J.gate[0] = a;
    J.gate[1] = b;
    J.gate[2] = go ? 1.0 : 0.0;
}

hipError_t launch_spec_decide_batch(const SpecJob *jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spec_decide_batch, dim3(njobs), dim3(FWD_THREADS), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_spec_decide(const double *partials, int nblocks, int threads,
                              const FitArgs &fit, const GradRule &rule, double *mo, double *gate,
                              hipStream_t s) {
    if (nblocks < 1 || threads < 64 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_spec_decide, dim3(1), dim3(threads), 0, s, partials, nblocks, fit, rule,
                       mo, gate);
    return hipGetLastError();
}

// Speculative gradient, second half: publishes (mo[0..2], a, b, go, g) in
// one read-back, g = scale * the gradient kernel's partials summed as
// k_publish_sum<NS> does (zeros when go = 0: the gradient kernel exited at
// once and left no partials).
template <int NS>
__global__ __launch_bounds__(1024) void k_publish_spec(const double *__restrict__ partials,
                                                       int nblocks, double scale,
                                                       const double *__restrict__ mo,
                                                       const double *__restrict__ gate,
                                                       double *__restrict__ g_out, double *dst,
                                                       uint32_t *flag, uint32_t seq) {
    const bool go = gate[2] != 0.0;   // uniform over the block
    double tot[NS];
    if (go) {
        sum_partials<NS, false>(partials, nblocks, scale, (int)blockDim.x, tot);
    } else {
#pragma unroll
        for (int j = 0; j < NS; ++j) tot[j] = 0.0;
    }
    if (threadIdx.x == 0) {
        for (int j = 0; j < 3; ++j) dst[j] = mo[j];
        for (int j = 0; j < 3; ++j) dst[3 + j] = gate[j];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            g_out[j] = tot[j];
            dst[6 + j] = tot[j];
        }
        __threadfence_system();
        __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

hipError_t launch_publish_spec(const double *partials, int nblocks, int threads, int ns,
                               double scale, const double *mo, const double *gate, double *g_out,
                               double *dst_host, uint32_t *flag_host, uint32_t seq,
                               hipStream_t s) {
    if (nblocks < 1 || threads < 64 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
    switch (ns) {
#define PCAS_PUBLISH_SPEC(N)                                                                       \
    case N:                                                                                        \
        hipLaunchKernelGGL(k_publish_spec<N>, dim3(1), dim3(threads), 0, s, partials, nblocks,     \
                           scale, mo, gate, g_out, dst_host, flag_host, seq);                      \
        break;
        PCAS_PUBLISH_SPEC(1)
        PCAS_PUBLISH_SPEC(2)
        PCAS_PUBLISH_SPEC(3)
        PCAS_PUBLISH_SPEC(4)
        PCAS_PUBLISH_SPEC(5)
        PCAS_PUBLISH_SPEC(6)
        PCAS_PUBLISH_SPEC(7)
        PCAS_PUBLISH_SPEC(8)
#undef PCAS_PUBLISH_SPEC
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One thread per detector pixel, all geometry in double with contraction
// off, so the record is the correctly rounded evaluation of: pixel centre,
// unit direction from the source, slab intersection with the box of voxel
// centres, n = ceil(L / step), dt = L / n; stored as the entry point and the
// per-sample step in voxel-index units.
template <typename T>
__global__ __launch_bounds__(256) void k_ray_table(VolDims v, Frame fr, RayRec<T> *__restrict__ rays) {
#pragma clang fp contract(off)
    const int M = fr.nu * fr.nv;
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= M) return;
    const int iu = pix % fr.nu, iv = pix / fr.nu;
    const double u = (iu - 0.5 * (fr.nu - 1)) * fr.pitch_u + fr.offset_u;
    const double w = (iv - 0.5 * (fr.nv - 1)) * fr.pitch_v + fr.offset_v;
    double dir[3], len2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double P = fr.det[c] + u * fr.eu[c] + w * fr.ev[c];
        dir[c] = P - fr.src[c];
        len2 += dir[c] * dir[c];
    }
    const double len = sqrt(len2);
    for (int c = 0; c < 3; ++c) dir[c] = dir[c] / len;
    const int nn[3] = {v.n0, v.n1, v.n2};
    double t0 = -INFINITY, t1 = INFINITY;
    bool missed = false;
    for (int c = 0; c < 3; ++c) {
        const double lo = v.origin[c];
        const double hi = v.origin[c] + (nn[c] - 1) * v.spacing[c];
        if (dir[c] == 0.0) {
            if (fr.src[c] < lo || fr.src[c] > hi) missed = true;
            continue;
        }
        double ta = (lo - fr.src[c]) / dir[c];
        double tb = (hi - fr.src[c]) / dir[c];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        t0 = ta > t0 ? ta : t0;
        t1 = tb < t1 ? tb : t1;
    }
    const double L = t1 - t0;
    RayRec<T> r;
    if (missed || !(L > 0.0)) {
        for (int c = 0; c < 3; ++c) { r.e[c] = (T)0; r.d[c] = (T)0; }
        r.dt = (T)0;
        r.n = 0;
    } else {
        const double nd = ceil(L / fr.step);
        const double dt = L / nd;
        for (int c = 0; c < 3; ++c) {
            const double X0 = fr.src[c] + t0 * dir[c];
            r.e[c] = (T)((X0 - v.origin[c]) / v.spacing[c]);
            r.d[c] = (T)(dt * dir[c] / v.spacing[c]);
        }
        r.dt = (T)dt;
        r.n = (int32_t)nd;
    }
    if constexpr (sizeof(T) == 8) r.pad_ = 0;
    rays[pix] = r;
}

hipError_t launch_ray_table(pcas_dtype dt, const VolDims &v, const Frame &fr, void *rays,
                            hipStream_t s) {
    const int M = fr.nu * fr.nv;
    dim3 grid((M + 255) / 256), block(256);
    if (dt == PCAS_F32)
        hipLaunchKernelGGL(k_ray_table<float>, grid, block, 0, s, v, fr, (RayRec<float> *)rays);
    else
        hipLaunchKernelGGL(k_ray_table<double>, grid, block, 0, s, v, fr, (RayRec<double> *)rays);
    return hipGetLastError();
}

}  // namespace pcas
