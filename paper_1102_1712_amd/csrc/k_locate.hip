// a9: tumour position -- fixed-point inversion of the pull-back field at one
// point.  One wavefront; lanes 0..7 evaluate the field of Eq. 1 at the eight
// grid neighbours of the current point and a butterfly sums their weighted
// values in a fixed order.
#include "device_util.h"

namespace pcas {

template <typename T, int K>
__global__ __launch_bounds__(64) void k_locate(VolDims vd, const T *__restrict__ mean,
                                               const T *__restrict__ U, WVec w, double c00,
                                               double c01, double c02, double tol, int max_iter,
                                               double *__restrict__ out) {
    const int lane = threadIdx.x;
    const int64_t N = (int64_t)vd.n0 * vd.n1 * vd.n2;
    const int nn[3] = {vd.n0, vd.n1, vd.n2};
    const double c0[3] = {c00, c01, c02};
    double y[3] = {c00, c01, c02};
    int iters = -1;
    for (int it = 1; it <= max_iter; ++it) {
        double xv[3] = {0.0, 0.0, 0.0};
        if (lane < 8) {
            int idx[3];
            double wgt = 1.0;
            bool inside = true;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int fl;
                double z;
                split_disp(y[c] - vd.origin[c], vd.inv_s[c], fl, z);
                const int bit = (lane >> c) & 1;
                idx[c] = fl + bit;
                wgt *= bit ? z : 1.0 - z;
                inside = inside && idx[c] >= 0 && idx[c] < nn[c];
            }
            if (inside) {
                const int64_t v = idx[0] + (int64_t)nn[0] * (idx[1] + (int64_t)nn[1] * idx[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double x = mean ? (double)mean[c * N + v] : 0.0;
#pragma unroll
                    for (int k = 0; k < K; ++k) x += (double)U[(int64_t)(k * 3 + c) * N + v] * w.w[k];
                    xv[c] = wgt * x;
                }
            }
        }
        double step2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double xs = wave_sum(xv[c]);
            const double yn = c0[c] - xs;
            step2 += (yn - y[c]) * (yn - y[c]);
            y[c] = yn;
        }
        if (sqrt(step2) < tol) {
            iters = it;
            break;
        }
    }
    if (lane == 0) {
        out[0] = y[0];
        out[1] = y[1];
        out[2] = y[2];
        out[3] = (double)iters;
    }
}

namespace {
template <typename T, int K>
hipError_t loc_k(const VolDims &v, const void *mean, const void *U, const WVec &w,
                 const double c0[3], double tol, int max_iter, double *out, hipStream_t s) {
    hipLaunchKernelGGL((k_locate<T, K>), dim3(1), dim3(64), 0, s, v, (const T *)mean,
                       (const T *)U, w, c0[0], c0[1], c0[2], tol, max_iter, out);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_locate(pcas_dtype dt, const VolDims &v, int K, const void *mean, const void *U,
                         const double *w, const double c0[3], double tol, int max_iter,
                         double *out, hipStream_t s) {
    WVec wv{};
    for (int k = 0; k < K; ++k) wv.w[k] = w[k];
#define L(TT, KK) \
    case KK: return loc_k<TT, KK>(v, mean, U, wv, c0, tol, max_iter, out, s)
    if (dt == PCAS_F32) {
        switch (K) { L(float, 1); L(float, 2); L(float, 3); L(float, 4);
                     L(float, 5); L(float, 6); L(float, 7); L(float, 8);
                     default: return hipErrorInvalidValue; }
    }
    switch (K) { L(double, 1); L(double, 2); L(double, 3); L(double, 4);
                 L(double, 5); L(double, 6); L(double, 7); L(double, 8);
                 default: return hipErrorInvalidValue; }
#undef L
}

}  // namespace pcas
