// a2 + a3: deformation field of Eq. 1 and the trilinear pull-back warp of
// Eqs. A.3 / A.5.  One lane per voxel, i fastest, so the mean / mode /
// output streams are fully coalesced; the eight f0 neighbours of a voxel lie
// within a few voxels of it and are served by L2.
#include "device_util.h"
#include "jacobian.h"

namespace pcas {

// Gather the trilinear value of vol at voxel (i, j, k) displaced by the
// field value (x0, x1, x2) mm, zero outside the grid.  The displacement is
// split into whole voxels + fraction before the voxel index is added, which
// keeps the fraction as accurate as the (small) displacement itself.
template <typename T>
__device__ __forceinline__ T warp_gather(const T *__restrict__ f0, int n0, int n1, int n2, int i,
                                         int j, int k, T x0, T x1, T x2, T is0, T is1, T is2) {
    int o0, o1, o2;
    T z0, z1, z2;
    split_disp(x0, is0, o0, z0);
    split_disp(x1, is1, o1, z1);
    split_disp(x2, is2, o2, z2);
    const int l0 = i + o0, l1 = j + o1, l2 = k + o2;
    // per-axis weights, zeroed for neighbours outside the grid
    const T a0 = (l0 >= 0 && l0 < n0) ? (T)1 - z0 : (T)0;
    const T b0 = (l0 + 1 >= 0 && l0 + 1 < n0) ? z0 : (T)0;
    const T a1 = (l1 >= 0 && l1 < n1) ? (T)1 - z1 : (T)0;
    const T b1 = (l1 + 1 >= 0 && l1 + 1 < n1) ? z1 : (T)0;
    const T a2 = (l2 >= 0 && l2 < n2) ? (T)1 - z2 : (T)0;
    const T b2 = (l2 + 1 >= 0 && l2 + 1 < n2) ? z2 : (T)0;
    if ((a0 == (T)0 && b0 == (T)0) || (a1 == (T)0 && b1 == (T)0) || (a2 == (T)0 && b2 == (T)0))
        return (T)0;
    // clamped indices (a clamped neighbour always carries weight 0)
    const int c0a = min(max(l0, 0), n0 - 1), c0b = min(max(l0 + 1, 0), n0 - 1);
    const int c1a = min(max(l1, 0), n1 - 1), c1b = min(max(l1 + 1, 0), n1 - 1);
    const int c2a = min(max(l2, 0), n2 - 1), c2b = min(max(l2 + 1, 0), n2 - 1);
    const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
    const T *pa = f0 + c2a * s2, *pb = f0 + c2b * s2;
    const T v000 = pa[c1a * s1 + c0a], v100 = pa[c1a * s1 + c0b];
    const T v010 = pa[c1b * s1 + c0a], v110 = pa[c1b * s1 + c0b];
    const T v001 = pb[c1a * s1 + c0a], v101 = pb[c1a * s1 + c0b];
    const T v011 = pb[c1b * s1 + c0a], v111 = pb[c1b * s1 + c0b];
    const T x00 = a0 * v000 + b0 * v100, x10 = a0 * v010 + b0 * v110;
    const T x01 = a0 * v001 + b0 * v101, x11 = a0 * v011 + b0 * v111;
    const T y0 = a1 * x00 + b1 * x10, y1 = a1 * x01 + b1 * x11;
    return a2 * y0 + b2 * y1;
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_pca_dvf(int64_t N, const T *__restrict__ mean,
                                                 const T *__restrict__ U, WVec w,
                                                 T *__restrict__ dvf) {
    const int64_t nb = gridDim.x;
    const int64_t b = xcd_remap(blockIdx.x, (int)nb);
    const int64_t v = b * blockDim.x + threadIdx.x;
    if (v >= N) return;
    T wk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) wk[k] = (T)w.w[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T x = mean ? mean[c * N + v] : (T)0;
#pragma unroll
        for (int k = 0; k < K; ++k) x = fma_t(wk[k], U[(int64_t)(k * 3 + c) * N + v], x);
        dvf[c * N + v] = x;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_warp_trilinear(VolDims vd, const T *__restrict__ f0,
                                                        const T *__restrict__ dvf,
                                                        T *__restrict__ f) {
    const int64_t N = (int64_t)vd.n0 * vd.n1 * vd.n2;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t v = b * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int i = (int)(v % vd.n0);
    const int j = (int)((v / vd.n0) % vd.n1);
    const int k = (int)(v / ((int64_t)vd.n0 * vd.n1));
    f[v] = warp_gather(f0, vd.n0, vd.n1, vd.n2, i, j, k, dvf[v], dvf[N + v], dvf[2 * N + v],
                       (T)vd.inv_s[0], (T)vd.inv_s[1], (T)vd.inv_s[2]);
}

// Block lb of nb blocks of one warp (the single and the batched launch both
// run this).
template <typename T, int K>
__device__ __forceinline__ void warp_pca_block(const VolDims &vd, const T *__restrict__ f0,
                                               const T *__restrict__ mean,
                                               const T *__restrict__ U, const WVec &w,
                                               T *__restrict__ f, int lb, int nb,
                                               const uint8_t *__restrict__ live) {
    // 32-bit index arithmetic (volumes are limited to 2^31 voxels); mean and
    // U are read once, so their loads are non-temporal and leave the caches
    // to the f0 neighbourhoods that neighbouring lanes share
    const int64_t N = (int64_t)vd.n0 * vd.n1 * vd.n2;
    const int b = xcd_remap(lb, nb);
    const int v32 = b * (int)blockDim.x + (int)threadIdx.x;
    if (v32 >= (int)N) return;
    const int64_t v = v32;
    const unsigned q = (unsigned)v32 / (unsigned)vd.n0;
    const int i = v32 - (int)q * vd.n0;
    const int k = (int)(q / (unsigned)vd.n1);
    const int j = (int)q - k * vd.n1;
    if (live) {   // voxels of bricks no ray reaches are never projected
        const int nbx = (vd.n0 + BRICK_X - 1) / BRICK_X, nby = (vd.n1 + BRICK_Y - 1) / BRICK_Y;
        if (!live[(k / BRICK_Z * nby + j / BRICK_Y) * nbx + i / BRICK_X]) return;
    }
    T x[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = mean ? __builtin_nontemporal_load(&mean[c * N + v]) : (T)0;
#pragma unroll
        for (int kk = 0; kk < K; ++kk)
            x[c] = fma_t((T)w.w[kk], __builtin_nontemporal_load(&U[(int64_t)(kk * 3 + c) * N + v]), x[c]);
    }
    f[v] = warp_gather(f0, vd.n0, vd.n1, vd.n2, i, j, k, x[0], x[1], x[2], (T)vd.inv_s[0],
                       (T)vd.inv_s[1], (T)vd.inv_s[2]);
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_warp_pca(VolDims vd, const T *__restrict__ f0,
                                                  const T *__restrict__ mean,
                                                  const T *__restrict__ U, WVec w,
                                                  T *__restrict__ f,
                                                  const uint8_t *__restrict__ live) {
    warp_pca_block<T, K>(vd, f0, mean, U, w, f, blockIdx.x, gridDim.x, live);
}

// Value (Eqs. A.3 / A.5) and diagonal Jacobian (Eq. A.8 and its analogues,
// per mm) of the pulled-back image at voxel (i, j, k) displaced by x (mm),
// from one read of the eight f0 neighbours, each taken as zero outside the
// grid.  Offsets are 32-bit (volumes hold fewer than 2^31 voxels).
template <typename T>
__device__ __forceinline__ T warp_value_jac(const T *__restrict__ f0, int n0, int n1, int n2,
                                            int i, int j, int k, const T (&x)[3], T is0, T is1,
                                            T is2, T (&jac)[3]) {
    int o0, o1, o2;
    T z1, z2, z3;   // the Appendix's z_1..z_3
    split_disp(x[0], is0, o0, z1);
    split_disp(x[1], is1, o1, z2);
    split_disp(x[2], is2, o2, z3);
    const int l = i + o0, m = j + o1, n = k + o2;
    const bool vl = (unsigned)l < (unsigned)n0, vl1 = (unsigned)(l + 1) < (unsigned)n0;
    const bool vm = (unsigned)m < (unsigned)n1, vm1 = (unsigned)(m + 1) < (unsigned)n1;
    const bool vn = (unsigned)n < (unsigned)n2, vn1 = (unsigned)(n + 1) < (unsigned)n2;
    jac[0] = jac[1] = jac[2] = (T)0;
    if (!((vl || vl1) && (vm || vm1) && (vn || vn1))) return (T)0;
    const int cl = min(max(l, 0), n0 - 1), cl1 = min(max(l + 1, 0), n0 - 1);
    const int rm = min(max(m, 0), n1 - 1) * n0, rm1 = min(max(m + 1, 0), n1 - 1) * n0;
    const int pn = min(max(n, 0), n2 - 1) * (n0 * n1), pn1 = min(max(n + 1, 0), n2 - 1) * (n0 * n1);
    auto F = [&](int c, int r, int p, bool ok) -> T { return ok ? f0[p + r + c] : (T)0; };
    const T f000 = F(cl, rm, pn, vl && vm && vn), f100 = F(cl1, rm, pn, vl1 && vm && vn);
    const T f010 = F(cl, rm1, pn, vl && vm1 && vn), f110 = F(cl1, rm1, pn, vl1 && vm1 && vn);
    const T f001 = F(cl, rm, pn1, vl && vm && vn1), f101 = F(cl1, rm, pn1, vl1 && vm && vn1);
    const T f011 = F(cl, rm1, pn1, vl && vm1 && vn1), f111 = F(cl1, rm1, pn1, vl1 && vm1 && vn1);
    const T w1 = (T)1 - z1, w2 = (T)1 - z2, w3 = (T)1 - z3;
    // value: the tent-weighted sum along x, then y, then z
    const T x00 = w1 * f000 + z1 * f100, x10 = w1 * f010 + z1 * f110;
    const T x01 = w1 * f001 + z1 * f101, x11 = w1 * f011 + z1 * f111;
    const T y0 = w2 * x00 + z2 * x10, y1 = w2 * x01 + z2 * x11;
    // Eq. A.8 and its analogues for the other axes (index units), then per mm
    const T g1 = ((f100 - f000) * w2 + (f110 - f010) * z2) * w3 +
                 ((f101 - f001) * w2 + (f111 - f011) * z2) * z3;
    const T g2 = ((f010 - f000) * w1 + (f110 - f100) * z1) * w3 +
                 ((f011 - f001) * w1 + (f111 - f101) * z1) * z3;
    const T g3 = ((f001 - f000) * w1 + (f101 - f100) * z1) * w2 +
                 ((f011 - f010) * w1 + (f111 - f110) * z1) * z2;
    jac[0] = g1 * is0;
    jac[1] = g2 * is1;
    jac[2] = g3 * is2;
    return w3 * y0 + z3 * y1;
}

// The warped image and its K Jacobian volumes J_k = sum_c U_kc df/dx_c
// (Eq. A.8 per mm, through the modes) in one voxel pass, for the fused
// evaluation that projects all K + 1 volumes together.  The field is formed
// as k_warp_pca forms it; the value and the three derivatives share one
// read of the eight f0 neighbours.
// A block covers WJ_VOX * 256 consecutive voxels, each thread WJ_VOX of
// them 256 apart: the streams of mean and U for all of them are in flight
// before the neighbour gathers that depend on them.
template <typename T, int K>
__device__ __forceinline__ void warp_jac_block(const VolDims &vd, const T *__restrict__ f0,
                                               const T *__restrict__ mean,
                                               const T *__restrict__ U, const WVec &w,
                                               T *__restrict__ out, int lb, int nb,
                                               const uint8_t *__restrict__ live) {
    const int64_t N = (int64_t)vd.n0 * vd.n1 * vd.n2;
    const int b = xcd_remap(lb, nb);
    const int nbx = (vd.n0 + BRICK_X - 1) / BRICK_X, nby = (vd.n1 + BRICK_Y - 1) / BRICK_Y;
    T wk[K];
#pragma unroll
    for (int kk = 0; kk < K; ++kk) wk[kk] = (T)w.w[kk];
    bool on[WJ_VOX];
    int vi[WJ_VOX], ii[WJ_VOX], jj[WJ_VOX], kx[WJ_VOX];
    T u[WJ_VOX][K][3], x[WJ_VOX][3];
#pragma unroll
    for (int e = 0; e < WJ_VOX; ++e) {
        const int v32 = (b * WJ_VOX + e) * (int)blockDim.x + (int)threadIdx.x;
        on[e] = v32 < (int)N;
        const int vc = on[e] ? v32 : 0;
        const unsigned q = (unsigned)vc / (unsigned)vd.n0;
        ii[e] = vc - (int)q * vd.n0;
        kx[e] = (int)(q / (unsigned)vd.n1);
        jj[e] = (int)q - kx[e] * vd.n1;
        vi[e] = vc;
        // voxels of bricks no ray reaches are never projected
        if (on[e] && live)
            on[e] = live[(kx[e] / BRICK_Z * nby + jj[e] / BRICK_Y) * nbx + ii[e] / BRICK_X] != 0;
        if (on[e]) voxel_field<T, K, true>(mean, U, wk, N, vc, u[e], x[e]);
    }
#pragma unroll
    for (int e = 0; e < WJ_VOX; ++e) {
        if (!on[e]) continue;
        const int64_t v = vi[e];
        T jac[3];
        out[v] = warp_value_jac(f0, vd.n0, vd.n1, vd.n2, ii[e], jj[e], kx[e], x[e],
                                (T)vd.inv_s[0], (T)vd.inv_s[1], (T)vd.inv_s[2], jac);
#pragma unroll
        for (int kk = 0; kk < K; ++kk)
            out[(int64_t)(kk + 1) * N + v] =
                fma_t(u[e][kk][0], jac[0], fma_t(u[e][kk][1], jac[1], u[e][kk][2] * jac[2]));
    }
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_warp_jac(VolDims vd, const T *__restrict__ f0,
                                                  const T *__restrict__ mean,
                                                  const T *__restrict__ U, WVec w,
                                                  T *__restrict__ out,
                                                  const uint8_t *__restrict__ live) {
    warp_jac_block<T, K>(vd, f0, mean, U, w, out, blockIdx.x, gridDim.x, live);
}

// Several requests' warps with their Jacobian volumes in one launch.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_warp_jac_batch(const WarpJob *__restrict__ jobs,
                                                        int njobs) {
    const int j = job_of(jobs, njobs);
    const WarpJob &J = jobs[j];
    warp_jac_block<T, K>(J.vd, (const T *)J.f0, (const T *)J.mean, (const T *)J.U, J.w, (T *)J.f,
                         blockIdx.x - J.block0, J.nblocks, J.live);
}

// Several requests' warps in one launch (jobs sorted by block0).
template <typename T, int K>
__global__ __launch_bounds__(256) void k_warp_pca_batch(const WarpJob *__restrict__ jobs,
                                                        int njobs) {
    const int j = job_of(jobs, njobs);
    const WarpJob &J = jobs[j];
    warp_pca_block<T, K>(J.vd, (const T *)J.f0, (const T *)J.mean, (const T *)J.U, J.w, (T *)J.f,
                         blockIdx.x - J.block0, J.nblocks, J.live);
}

namespace {
template <typename T, int K>
hipError_t pca_dvf_k(int64_t N, const void *mean, const void *U, const WVec &w, void *dvf,
                     hipStream_t s) {
    dim3 grid((unsigned)((N + 255) / 256)), block(256);
    hipLaunchKernelGGL((k_pca_dvf<T, K>), grid, block, 0, s, N, (const T *)mean, (const T *)U, w,
                       (T *)dvf);
    return hipGetLastError();
}
template <typename T, int K>
hipError_t warp_pca_k(const VolDims &v, const void *f0, const void *mean, const void *U,
                      const WVec &w, void *f, hipStream_t s, const uint8_t *live) {
    const int64_t N = (int64_t)v.n0 * v.n1 * v.n2;
    dim3 grid((unsigned)((N + 255) / 256)), block(256);
    hipLaunchKernelGGL((k_warp_pca<T, K>), grid, block, 0, s, v, (const T *)f0, (const T *)mean,
                       (const T *)U, w, (T *)f, live);
    return hipGetLastError();
}
template <typename T, int K>
hipError_t warp_jac_k(const VolDims &v, const void *f0, const void *mean, const void *U,
                      const WVec &w, void *out, hipStream_t s, const uint8_t *live) {
    const int64_t N = (int64_t)v.n0 * v.n1 * v.n2;
    dim3 grid((unsigned)warp_jac_blocks(N)), block(256);
    hipLaunchKernelGGL((k_warp_jac<T, K>), grid, block, 0, s, v, (const T *)f0, (const T *)mean,
                       (const T *)U, w, (T *)out, live);
    return hipGetLastError();
}
WVec make_w(const double *w, int K) {
    WVec r{};
    for (int k = 0; k < K; ++k) r.w[k] = w[k];
    return r;
}
}  // namespace

#define PCAS_K_SWITCH(K, CALL)         \
    switch (K) {                       \
    case 1: return CALL(1);            \
    case 2: return CALL(2);            \
    case 3: return CALL(3);            \
    case 4: return CALL(4);            \
    case 5: return CALL(5);            \
    case 6: return CALL(6);            \
    case 7: return CALL(7);            \
    case 8: return CALL(8);            \
    default: return hipErrorInvalidValue; \
    }

hipError_t launch_pca_dvf(pcas_dtype dt, int64_t N, int K, const void *mean, const void *U,
                          const double *w, void *dvf, hipStream_t s) {
    const WVec wv = make_w(w, K);
    if (dt == PCAS_F32) {
#define CALL(KK) pca_dvf_k<float, KK>(N, mean, U, wv, dvf, s)
        PCAS_K_SWITCH(K, CALL)
#undef CALL
    }
#define CALL(KK) pca_dvf_k<double, KK>(N, mean, U, wv, dvf, s)
    PCAS_K_SWITCH(K, CALL)
#undef CALL
}

int warp_blocks(int64_t N) { return (int)((N + 255) / 256); }
int warp_jac_blocks(int64_t N) { return (int)((N + 256 * WJ_VOX - 1) / (256 * WJ_VOX)); }

namespace {
template <typename T, int K>
hipError_t warp_batch_k(const WarpJob *jobs, int njobs, int total_blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_warp_pca_batch<T, K>), dim3(total_blocks), dim3(256), 0, s, jobs, njobs);
    return hipGetLastError();
}
template <typename T, int K>
hipError_t warp_jac_batch_k(const WarpJob *jobs, int njobs, int total_blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_warp_jac_batch<T, K>), dim3(total_blocks), dim3(256), 0, s, jobs, njobs);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_warp_pca_batch(pcas_dtype dt, int K, const WarpJob *jobs, int njobs,
                                 int total_blocks, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (dt == PCAS_F32) {
#define CALL(KK) warp_batch_k<float, KK>(jobs, njobs, total_blocks, s)
        PCAS_K_SWITCH(K, CALL)
#undef CALL
    }
#define CALL(KK) warp_batch_k<double, KK>(jobs, njobs, total_blocks, s)
    PCAS_K_SWITCH(K, CALL)
#undef CALL
}

hipError_t launch_warp_trilinear(pcas_dtype dt, const VolDims &v, const void *f0, const void *dvf,
                                 void *f, hipStream_t s) {
    const int64_t N = (int64_t)v.n0 * v.n1 * v.n2;
    dim3 grid((unsigned)((N + 255) / 256)), block(256);
    if (dt == PCAS_F32)
        hipLaunchKernelGGL(k_warp_trilinear<float>, grid, block, 0, s, v, (const float *)f0,
                           (const float *)dvf, (float *)f);
    else
        hipLaunchKernelGGL(k_warp_trilinear<double>, grid, block, 0, s, v, (const double *)f0,
                           (const double *)dvf, (double *)f);
    return hipGetLastError();
}

hipError_t launch_warp_pca(pcas_dtype dt, const VolDims &v, int K, const void *f0,
                           const void *mean, const void *U, const double *w, void *f,
                           hipStream_t s, const uint8_t *live) {
    const WVec wv = make_w(w, K);
    if (dt == PCAS_F32) {
#define CALL(KK) warp_pca_k<float, KK>(v, f0, mean, U, wv, f, s, live)
        PCAS_K_SWITCH(K, CALL)
#undef CALL
    }
#define CALL(KK) warp_pca_k<double, KK>(v, f0, mean, U, wv, f, s, live)
    PCAS_K_SWITCH(K, CALL)
#undef CALL
}

hipError_t launch_warp_jac(pcas_dtype dt, const VolDims &v, int K, const void *f0,
                           const void *mean, const void *U, const double *w, void *out,
                           hipStream_t s, const uint8_t *live) {
    const WVec wv = make_w(w, K);
    if (dt == PCAS_F32) {
#define CALL(KK) warp_jac_k<float, KK>(v, f0, mean, U, wv, out, s, live)
        PCAS_K_SWITCH(K, CALL)
#undef CALL
    }
#define CALL(KK) warp_jac_k<double, KK>(v, f0, mean, U, wv, out, s, live)
    PCAS_K_SWITCH(K, CALL)
#undef CALL
}

hipError_t launch_warp_jac_batch(pcas_dtype dt, int K, const WarpJob *jobs, int njobs,
                                 int total_blocks, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (dt == PCAS_F32) {
#define CALL(KK) warp_jac_batch_k<float, KK>(jobs, njobs, total_blocks, s)
        PCAS_K_SWITCH(K, CALL)
#undef CALL
    }
#define CALL(KK) warp_jac_batch_k<double, KK>(jobs, njobs, total_blocks, s)
    PCAS_K_SWITCH(K, CALL)
#undef CALL
}

}  // namespace pcas
