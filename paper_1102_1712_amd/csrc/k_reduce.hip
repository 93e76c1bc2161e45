// a5: sums for the intensity fit of Eq. A.1 and the objective of Eq. 2.
// Grid-stride streams over the detector with double accumulation and the
// fixed-order last-block reduction.
#include "device_util.h"

namespace pcas {

constexpr int SUMS_BLOCKS_MAX = 512;

int sums_blocks(int64_t M) {
    int64_t b = (M + 255) / 256;
    return (int)(b < SUMS_BLOCKS_MAX ? (b > 0 ? b : 1) : SUMS_BLOCKS_MAX);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pair_sums(int64_t M, const T *__restrict__ a,
                                                   const T *__restrict__ b,
                                                   double *__restrict__ partials,
                                                   uint32_t *counter, double *__restrict__ out) {
    const int nb = gridDim.x;
    const int bid = blockIdx.x;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)bid * 256 + threadIdx.x; t < M; t += (int64_t)nb * 256) {
        const double av = (double)a[t], bv = (double)b[t];
        s[0] += av;
        s[1] += av * bv;
        s[2] += av * av;
        s[3] += bv;
        s[4] += bv * bv;
    }
    grid_reduce<5>(s, partials, counter, out, bid, nb, 1.0);
}

// (a, b) of Eq. A.1 by the 2 x 2 normal equations (Y^T Y)(a, b)^T = Y^T p
// with Y = [y, 1]; NaN when Y^T Y is singular.
__device__ __forceinline__ void fit_normal_equations(double sp, double spy, double sy, double syy,
                                                     double m, double *a, double *b) {
    const double det = syy * m - sy * sy;
    if (!(fabs(det) > 1e-12 * syy * m)) {
        *a = *b = NAN;
        return;
    }
    *a = (m * spy - sy * sp) / det;
    *b = (syy * sp - sy * spy) / det;
}

template <typename T>
__device__ __forceinline__ void residual_block(int64_t M, const T *__restrict__ p,
                                               const T *__restrict__ y, const FitArgs &fa,
                                               const double *__restrict__ src, T *r,
                                               double *__restrict__ partials, uint32_t *counter,
                                               double *__restrict__ out, int bid, int nb) {
    double A = fa.a, B = fa.b;
    if (fa.mode == FIT_COEF) {
        A = src[0];
        B = src[1];
    } else if (fa.mode == FIT_REFIT) {
        // src holds the forward pass's moments about the reference (a0, b0):
        // sum p = sum r0 + a0 sum y + M b0, sum p y = sum r0 y + a0 sum y^2 + b0 sum y
        const double sp = src[0] + fa.a0 * fa.sy + fa.m * fa.b0;
        const double spy = src[1] + fa.a0 * fa.syy + fa.b0 * fa.sy;
        fit_normal_equations(sp, spy, fa.sy, fa.syy, fa.m, &A, &B);
    }
    if (bid == 0 && threadIdx.x == 0) {
        out[1] = A;
        out[2] = B;
    }
    double s[1] = {0.0};
    for (int64_t t = (int64_t)bid * 256 + threadIdx.x; t < M; t += (int64_t)nb * 256) {
        const double rv = (double)p[t] - A * (double)y[t] - B;
        if (r) r[t] = (T)rv;
        s[0] += rv * rv;
    }
    grid_reduce<1>(s, partials, counter, out, bid, nb, 1.0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_residual(int64_t M, const T *__restrict__ p,
                                                  const T *__restrict__ y, FitArgs fa,
                                                  const double *__restrict__ src, T *r,
                                                  double *__restrict__ partials, uint32_t *counter,
                                                  double *__restrict__ out) {
    residual_block<T>(M, p, y, fa, src, r, partials, counter, out, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_residual_batch(const ResJob *__restrict__ jobs,
                                                        int njobs) {
    const int j = job_of(jobs, njobs);
    const ResJob &J = jobs[j];
    residual_block<T>(J.M, (const T *)J.p, (const T *)J.y, J.fa, J.src, (T *)nullptr, J.partials,
                      J.counter, J.out, blockIdx.x - J.block0, J.nblocks);
}

hipError_t launch_residual_batch(pcas_dtype dt, const ResJob *jobs, int njobs, int total_blocks,
                                 hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (dt == PCAS_F32)
        hipLaunchKernelGGL(k_residual_batch<float>, dim3(total_blocks), dim3(256), 0, s, jobs,
                           njobs);
    else
        hipLaunchKernelGGL(k_residual_batch<double>, dim3(total_blocks), dim3(256), 0, s, jobs,
                           njobs);
    return hipGetLastError();
}

// (a, b) of Eq. A.1 from (sum p, sum p y, sum p p, sum y, sum y y).
__global__ void k_fit_from_sums(int64_t M, int fit, const double *__restrict__ sums,
                                double *__restrict__ stats) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 1.0, b = 0.0;
    if (fit) fit_normal_equations(sums[0], sums[1], sums[3], sums[4], (double)M, &a, &b);
    stats[0] = a;
    stats[1] = b;
}

hipError_t launch_pair_sums(pcas_dtype dt, int64_t M, const void *a, const void *b,
                            double *partials, uint32_t *counter, double *out, hipStream_t s) {
    const int nb = sums_blocks(M);
    if (dt == PCAS_F32)
        hipLaunchKernelGGL(k_pair_sums<float>, dim3(nb), dim3(256), 0, s, M, (const float *)a,
                           (const float *)b, partials, counter, out);
    else
        hipLaunchKernelGGL(k_pair_sums<double>, dim3(nb), dim3(256), 0, s, M, (const double *)a,
                           (const double *)b, partials, counter, out);
    return hipGetLastError();
}

hipError_t launch_residual(pcas_dtype dt, int64_t M, const void *p, const void *y,
                           const FitArgs &fa, const double *src, void *r, double *partials,
                           uint32_t *counter, double *out, hipStream_t s) {
    const int nb = sums_blocks(M);
    if (dt == PCAS_F32)
        hipLaunchKernelGGL(k_residual<float>, dim3(nb), dim3(256), 0, s, M, (const float *)p,
                           (const float *)y, fa, src, (float *)r, partials, counter, out);
    else
        hipLaunchKernelGGL(k_residual<double>, dim3(nb), dim3(256), 0, s, M, (const double *)p,
                           (const double *)y, fa, src, (double *)r, partials, counter, out);
    return hipGetLastError();
}

hipError_t launch_fit_from_sums(int64_t M, int fit, const double *sums, double *stats,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_fit_from_sums, dim3(1), dim3(64), 0, s, M, fit, sums, stats);
    return hipGetLastError();
}

// Copies count doubles from each of n device locations into dst (n x count),
// so a batch's scalars come back in one transfer.
template <int NS>
__device__ void finish_sum(const SumJob &J, double *tot_s) {
    double tot[NS];
    sum_partials<NS, false>(J.partials, J.nblocks, J.scale, J.width, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            J.out[j] = tot[j];
            tot_s[j] = tot[j];
        }
    }
}

constexpr int GATHER_THREADS = 512;
static_assert(ADJ_THREADS <= GATHER_THREADS && FWD_THREADS <= GATHER_THREADS &&
                  EVAL_SUM_WIDTH <= GATHER_THREADS,
              "gather width");

__global__ __launch_bounds__(GATHER_THREADS) void k_gather_scalars(const double *const *__restrict__ src,
                                                                   double *__restrict__ dst, int count,
                                                                   const SumJob *__restrict__ sums) {
    __shared__ double tot_s[RED_SLOTS_WIDE];
    const int b = blockIdx.x;
    int lo = 0, hi = 0;
    if (sums && sums[b].ns > 0 && (!sums[b].gate || sums[b].gate[2] != 0.0)) {   // uniform
        const SumJob J = sums[b];
        switch (J.ns) {
        case 1: finish_sum<1>(J, tot_s); break;
        case 2: finish_sum<2>(J, tot_s); break;
        case 3: finish_sum<3>(J, tot_s); break;
        case 4: finish_sum<4>(J, tot_s); break;
        case 5: finish_sum<5>(J, tot_s); break;
        case 6: finish_sum<6>(J, tot_s); break;
        case 7: finish_sum<7>(J, tot_s); break;
        case 8: finish_sum<8>(J, tot_s); break;
        // the fused evaluation's sums, eval_sums(1..8)
        case 10: finish_sum<10>(J, tot_s); break;
        case 15: finish_sum<15>(J, tot_s); break;
        case 21: finish_sum<21>(J, tot_s); break;
        case 28: finish_sum<28>(J, tot_s); break;
        case 36: finish_sum<36>(J, tot_s); break;
        case 45: finish_sum<45>(J, tot_s); break;
        case 55: finish_sum<55>(J, tot_s); break;
        default: finish_sum<66>(J, tot_s); break;
        }
        __syncthreads();
        lo = J.offset;
        hi = J.offset + J.ns;
    }
    for (int t = threadIdx.x; t < count; t += blockDim.x)
        dst[b * count + t] = (t >= lo && t < hi) ? tot_s[t - lo] : src[b][t];
}

hipError_t launch_gather_scalars(const double *const *src, double *dst, int n, int count,
                                 const SumJob *sums, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_scalars, dim3(n), dim3(GATHER_THREADS), 0, s, src, dst, count, sums);
    return hipGetLastError();
}

}  // namespace pcas
