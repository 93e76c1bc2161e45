// Exact-path projection of the voxel-constant volume (Siddon's method, the
// paper's simulator for its digital projections, Sec. II.B): each cell
// [centre - s/2, centre + s/2] contributes (length of the ray inside it) x
// (its value), the ray running from the source to the pixel centre.
//
// One lane per ray walks the cells incrementally: per axis it keeps the
// parameter of the next cell-plane crossing (recomputed exactly from the
// plane index, so nothing drifts), advances to the nearest one, and takes
// the cell of each interval from the interval's midpoint, which is robust to
// ties and rounding.  All geometry and the sum are in double.
#include "device_util.h"

namespace pcas {

template <typename T>
__global__ __launch_bounds__(256) void k_siddon(VolDims v, Frame fr, const T *__restrict__ f,
                                                T *__restrict__ p) {
    const int M = fr.nu * fr.nv;
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= M) return;
    const int iu = pix % fr.nu, iv = pix / fr.nu;
    const double u = (iu - 0.5 * (fr.nu - 1)) * fr.pitch_u + fr.offset_u;
    const double w = (iv - 0.5 * (fr.nv - 1)) * fr.pitch_v + fr.offset_v;
    const int nn[3] = {v.n0, v.n1, v.n2};
    double S[3], d[3], b0[3], len2 = 0.0;
    double amin = 0.0, amax = 1.0;
    bool miss = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        S[c] = fr.src[c];
        d[c] = fr.det[c] + u * fr.eu[c] + w * fr.ev[c] - S[c];
        len2 += d[c] * d[c];
        b0[c] = v.origin[c] - 0.5 * v.spacing[c];
        const double bn = v.origin[c] + (nn[c] - 0.5) * v.spacing[c];
        if (d[c] == 0.0) {
            if (S[c] <= b0[c] || S[c] >= bn) miss = true;
            continue;
        }
        double a0 = (b0[c] - S[c]) / d[c], a1 = (bn - S[c]) / d[c];
        if (a0 > a1) {
            const double t = a0;
            a0 = a1;
            a1 = t;
        }
        amin = fmax(amin, a0);
        amax = fmin(amax, a1);
    }
    if (miss || !(amin < amax)) {
        p[pix] = (T)0;
        return;
    }
    // next crossing after amin per axis
    double anext[3], inv[3];
    int k[3], sg[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0) {
            anext[c] = INFINITY;
            inv[c] = 0.0;
            k[c] = 0;
            sg[c] = 0;
            continue;
        }
        inv[c] = 1.0 / d[c];
        sg[c] = d[c] > 0.0 ? 1 : -1;
        const double q = (S[c] + amin * d[c] - b0[c]) / v.spacing[c];
        k[c] = sg[c] > 0 ? (int)floor(q) + 1 : (int)ceil(q) - 1;
        anext[c] = (b0[c] + k[c] * v.spacing[c] - S[c]) * inv[c];
        if (anext[c] <= amin) {
            k[c] += sg[c];
            anext[c] = (b0[c] + k[c] * v.spacing[c] - S[c]) * inv[c];
        }
    }
    const int64_t s1 = v.n0, s2 = (int64_t)v.n0 * v.n1;
    double acc = 0.0, a = amin;
    while (a < amax) {
        const double an = fmin(fmin(anext[0], anext[1]), fmin(anext[2], amax));
        if (an > a) {
            const double mid = 0.5 * (a + an);
            int64_t idx = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int i = (int)floor((S[c] + mid * d[c] - b0[c]) / v.spacing[c]);
                i = min(max(i, 0), nn[c] - 1);
                idx += (c == 0 ? 1 : (c == 1 ? s1 : s2)) * (int64_t)i;
            }
            acc += (an - a) * (double)f[idx];
        }
        a = an;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (anext[c] <= a) {
                k[c] += sg[c];
                anext[c] = (b0[c] + k[c] * v.spacing[c] - S[c]) * inv[c];
            }
    }
    p[pix] = (T)(acc * sqrt(len2));
}

hipError_t launch_siddon(pcas_dtype dt, const VolDims &v, const Frame &fr, const void *f, void *p,
                         hipStream_t s) {
    const int M = fr.nu * fr.nv;
    const dim3 grid((M + 255) / 256), block(256);
    if (dt == PCAS_F32)
        hipLaunchKernelGGL(k_siddon<float>, grid, block, 0, s, v, fr, (const float *)f, (float *)p);
    else
        hipLaunchKernelGGL(k_siddon<double>, grid, block, 0, s, v, fr, (const double *)f,
                           (double *)p);
    return hipGetLastError();
}

}  // namespace pcas
