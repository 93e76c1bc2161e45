// Per-voxel chain of the Appendix shared by the Jacobian-chain kernels:
// the field of Eq. 1 at a voxel and the diagonal Jacobian of Eq. A.8.
#pragma once

#include "device_util.h"

namespace pcas {

// Diagonal Jacobian of the warped image at voxel (i, j, k) pulled back by
// x (mm): Eq. A.8 and its analogues for the other two axes from the eight
// f0 neighbours of the pulled-back position (zero outside the grid), per mm.
// Returns false when no neighbour is inside the grid (all derivatives 0).
template <typename T>
__device__ __forceinline__ bool voxel_jacobian(const T *__restrict__ f0, int n0, int n1, int n2,
                                               int i, int j, int k, const T (&x)[3], T is0, T is1,
                                               T is2, T (&jac)[3]) {
    const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
    int o0, o1, o2;
    T z1, z2, z3;                                           // the Appendix's z_1..z_3
    split_disp(x[0], is0, o0, z1);
    split_disp(x[1], is1, o1, z2);
    split_disp(x[2], is2, o2, z3);
    const int l = i + o0, m = j + o1, n = k + o2;
    // neighbour values with zero extension
    const bool vl = l >= 0 && l < n0, vl1 = l + 1 >= 0 && l + 1 < n0;
    const bool vm = m >= 0 && m < n1, vm1 = m + 1 >= 0 && m + 1 < n1;
    const bool vn = n >= 0 && n < n2, vn1 = n + 1 >= 0 && n + 1 < n2;
    if (!((vl || vl1) && (vm || vm1) && (vn || vn1))) return false;
    const int cl = min(max(l, 0), n0 - 1), cl1 = min(max(l + 1, 0), n0 - 1);
    const int cm = min(max(m, 0), n1 - 1), cm1 = min(max(m + 1, 0), n1 - 1);
    const int cn = min(max(n, 0), n2 - 1), cn1 = min(max(n + 1, 0), n2 - 1);
    auto F = [&](int ii, int jj, int kk, bool ok) -> T {
        return ok ? f0[ii + s1 * jj + s2 * kk] : (T)0;
    };
    const T f000 = F(cl, cm, cn, vl && vm && vn), f100 = F(cl1, cm, cn, vl1 && vm && vn);
    const T f010 = F(cl, cm1, cn, vl && vm1 && vn), f110 = F(cl1, cm1, cn, vl1 && vm1 && vn);
    const T f001 = F(cl, cm, cn1, vl && vm && vn1), f101 = F(cl1, cm, cn1, vl1 && vm && vn1);
    const T f011 = F(cl, cm1, cn1, vl && vm1 && vn1), f111 = F(cl1, cm1, cn1, vl1 && vm1 && vn1);
    // Eq. A.8 and its analogues (index units), then per mm
    const T g1 = ((f100 - f000) * ((T)1 - z2) + (f110 - f010) * z2) * ((T)1 - z3) +
                 ((f101 - f001) * ((T)1 - z2) + (f111 - f011) * z2) * z3;
    const T g2 = ((f010 - f000) * ((T)1 - z1) + (f110 - f100) * z1) * ((T)1 - z3) +
                 ((f011 - f001) * ((T)1 - z1) + (f111 - f101) * z1) * z3;
    const T g3 = ((f001 - f000) * ((T)1 - z1) + (f101 - f100) * z1) * ((T)1 - z2) +
                 ((f011 - f010) * ((T)1 - z1) + (f111 - f110) * z1) * z2;
    jac[0] = g1 * is0;
    jac[1] = g2 * is1;
    jac[2] = g3 * is2;
    return true;
}

template <bool NT, typename T> __device__ __forceinline__ T load_once(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// x = xbar + U w at voxel v and the modes' three components there.  NT: the
// loads are non-temporal, for voxel-stream kernels whose lanes read whole
// cache lines of mean and U exactly once.  A brick's write-out reads half
// lines whose other halves a neighbouring brick reads later, so it keeps
// ordinary loads (non-temporal ones measured 3% slower there).
template <typename T, int K, bool NT>
__device__ __forceinline__ void voxel_field(const T *__restrict__ mean, const T *__restrict__ U,
                                            const T (&wk)[K], int64_t N, int64_t v, T (&u)[K][3],
                                            T (&x)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = mean ? load_once<NT>(&mean[c * N + v]) : (T)0;
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
            u[kk][c] = load_once<NT>(&U[(int64_t)(kk * 3 + c) * N + v]);
            x[c] = fma_t(wk[kk], u[kk][c], x[c]);
        }
    }
}

}  // namespace pcas
