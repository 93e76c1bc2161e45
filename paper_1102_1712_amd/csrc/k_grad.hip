// a7: the Jacobian chain of the Appendix, g = 2 U^T (df/dx) bp, and the
// Jacobian volumes J_k = U_k^T (df/dx) whose projections give the same
// gradient as g_k = 2 <r, P J_k> (the adjoint identity).
//
// A voxel stream: each block owns a contiguous run of voxels (lanes step by
// 256 inside it, so every load is coalesced), recomputes x = xbar + U w and
// the diagonal Jacobian of Eq. A.8 from the eight f0 neighbours of the
// pulled-back position, and accumulates bp * sum_c U_kc * df/dx_c in double.
// Voxels with bp = 0 contribute nothing and are skipped without touching
// the mode streams.  Block partials are reduced in block order by the last
// block to finish, so g is bit-for-bit reproducible.
#include "jacobian.h"

namespace pcas {

template <typename T, int K>
__global__ __launch_bounds__(256) void k_grad_w(VolDims vd, const T *__restrict__ f0,
                                                const T *__restrict__ mean,
                                                const T *__restrict__ U, WVec w,
                                                const T *__restrict__ bp,
                                                double *__restrict__ partials, uint32_t *counter,
                                                double *__restrict__ g_out) {
    const int n0 = vd.n0, n1 = vd.n1, n2 = vd.n2;
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int nb = gridDim.x;
    // round-robin over the XCDs: voxels outside the x-ray cone (bp = 0) are
    // skipped, so the work per block is uneven along z
    const int bid = blockIdx.x;
    int64_t per = (N + nb - 1) / nb;
    per = (per + 255) & ~(int64_t)255;
    const int64_t v_begin = (int64_t)bid * per;
    const int64_t v_end = min(N, v_begin + per);
    const int64_t s2 = (int64_t)n0 * n1;
    T wk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) wk[k] = (T)w.w[k];
    const T is0 = (T)vd.inv_s[0], is1 = (T)vd.inv_s[1], is2 = (T)vd.inv_s[2];
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;

    for (int64_t v = v_begin + threadIdx.x; v < v_end; v += 256) {
        const T bpv = bp[v];
        if (bpv == (T)0) continue;
        const int i = (int)(v % n0);
        const int j = (int)((v / n0) % n1);
        const int k = (int)(v / s2);
        T u[K][3], x[3], jac[3];
        voxel_field<T, K, true>(mean, U, wk, N, v, u, x);
        if (!voxel_jacobian(f0, n0, n1, n2, i, j, k, x, is0, is1, is2, jac)) continue;
        const T j0 = jac[0] * bpv, j1 = jac[1] * bpv, j2 = jac[2] * bpv;
#pragma unroll
        for (int kk = 0; kk < K; ++kk)
            acc[kk] += (double)fma_t(u[kk][0], j0, fma_t(u[kk][1], j1, u[kk][2] * j2));
    }
    grid_reduce<K>(acc, partials, counter, g_out, bid, nb, 2.0);
}

// The K Jacobian volumes J_k = sum_c U_kc df/dx_c of the warp at w (the
// chain of Eq. A.8 without the back-projection), J[k][v].
template <typename T, int K>
__global__ __launch_bounds__(256) void k_jacobian(VolDims vd, const T *__restrict__ f0,
                                                  const T *__restrict__ mean,
                                                  const T *__restrict__ U, WVec w,
                                                  T *__restrict__ J) {
    const int n0 = vd.n0, n1 = vd.n1, n2 = vd.n2;
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t v = b * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int i = (int)(v % n0);
    const int j = (int)((v / n0) % n1);
    const int k = (int)(v / ((int64_t)n0 * n1));
    T wk[K];
#pragma unroll
    for (int kk = 0; kk < K; ++kk) wk[kk] = (T)w.w[kk];
    T u[K][3], x[3], jac[3];
    voxel_field<T, K, true>(mean, U, wk, N, v, u, x);
    if (!voxel_jacobian(f0, n0, n1, n2, i, j, k, x, (T)vd.inv_s[0], (T)vd.inv_s[1],
                        (T)vd.inv_s[2], jac)) {
        jac[0] = jac[1] = jac[2] = (T)0;
    }
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
        J[kk * N + v] = fma_t(u[kk][0], jac[0], fma_t(u[kk][1], jac[1], u[kk][2] * jac[2]));
}

int grad_w_blocks(int64_t N) {
    int64_t b = (N + 255) / 256;
    return (int)(b < GRAD_BLOCKS_MAX ? b : GRAD_BLOCKS_MAX);
}

namespace {
template <typename T, int K>
hipError_t grad_k(const VolDims &v, const void *f0, const void *mean, const void *U,
                  const WVec &w, const void *bp, double *partials, uint32_t *counter,
                  double *g_out, hipStream_t s) {
    const int64_t N = (int64_t)v.n0 * v.n1 * v.n2;
    hipLaunchKernelGGL((k_grad_w<T, K>), dim3(grad_w_blocks(N)), dim3(256), 0, s, v,
                       (const T *)f0, (const T *)mean, (const T *)U, w, (const T *)bp, partials,
                       counter, g_out);
    return hipGetLastError();
}
}  // namespace

namespace {
template <typename T, int K>
hipError_t jacobian_k(const VolDims &v, const void *f0, const void *mean, const void *U,
                      const WVec &w, void *J, hipStream_t s) {
    const int64_t N = (int64_t)v.n0 * v.n1 * v.n2;
    hipLaunchKernelGGL((k_jacobian<T, K>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, v,
                       (const T *)f0, (const T *)mean, (const T *)U, w, (T *)J);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_jacobian(pcas_dtype dt, const VolDims &v, int K, const void *f0,
                           const void *mean, const void *U, const double *w, void *J,
                           hipStream_t s) {
    WVec wv{};
    for (int k = 0; k < K; ++k) wv.w[k] = w[k];
#define G(TT, KK) \
    case KK: return jacobian_k<TT, KK>(v, f0, mean, U, wv, J, s)
    if (dt == PCAS_F32) {
        switch (K) { G(float, 1); G(float, 2); G(float, 3); G(float, 4);
                     G(float, 5); G(float, 6); G(float, 7); G(float, 8);
                     default: return hipErrorInvalidValue; }
    }
    switch (K) { G(double, 1); G(double, 2); G(double, 3); G(double, 4);
                 G(double, 5); G(double, 6); G(double, 7); G(double, 8);
                 default: return hipErrorInvalidValue; }
#undef G
}

hipError_t launch_grad_w(pcas_dtype dt, const VolDims &v, int K, const void *f0, const void *mean,
                         const void *U, const double *w, const void *bp, double *partials,
                         uint32_t *counter, double *g_out, hipStream_t s) {
    WVec wv{};
    for (int k = 0; k < K; ++k) wv.w[k] = w[k];
#define G(TT, KK) \
    case KK: return grad_k<TT, KK>(v, f0, mean, U, wv, bp, partials, counter, g_out, s)
    if (dt == PCAS_F32) {
        switch (K) { G(float, 1); G(float, 2); G(float, 3); G(float, 4);
                     G(float, 5); G(float, 6); G(float, 7); G(float, 8);
                     default: return hipErrorInvalidValue; }
    }
    switch (K) { G(double, 1); G(double, 2); G(double, 3); G(double, 4);
                 G(double, 5); G(double, 6); G(double, 7); G(double, 8);
                 default: return hipErrorInvalidValue; }
#undef G
}

}  // namespace pcas
