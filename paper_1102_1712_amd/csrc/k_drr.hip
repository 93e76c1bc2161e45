// a4: forward projection P f and a6: back-projection P^T r.
//
// Forward: one lane per ray; a wave marches an 8 x 8 tile of neighbouring
// rays, whose samples at equal index sit within a few voxels of each other,
// so the 8-neighbour gathers of a wave hit a handful of cache lines.
//
// Adjoint: the exact transpose of the forward without global atomics.  One
// wavefront owns a 16 x 16 x 8 voxel brick held in LDS.  It visits every
// ray whose pixel lies in the detector footprint of the brick (plus a
// one-voxel apron), re-creates exactly the samples of that ray whose 2x2x2
// cell touches the brick (same ray record, same sample_cell arithmetic as
// the forward), and adds dt * r * weight for the corners inside the brick.
// Each (sample, corner) pair therefore lands in exactly one brick, and the
// brick is written to HBM once.  Only the lanes of one wave touch a brick,
// so the LDS accumulation order is fixed and the result is reproducible.
#include "device_util.h"

namespace pcas {

template <typename T>
__device__ __forceinline__ T lerp_t(T a, T b, T z) {
    return fma_t(z, b - a, a);
}

template <typename T, bool SUMS>
__global__ __launch_bounds__(256) void k_drr_forward(int n0, int n1, int n2, int nu, int nv,
                                                     int tiles_u, const RayRec<T> *__restrict__ rays,
                                                     const T *__restrict__ f, T *__restrict__ p,
                                                     const T *__restrict__ y,
                                                     double *__restrict__ partials,
                                                     uint32_t *counter, double *__restrict__ sums) {
    const int nb = gridDim.x;
    const int bid = xcd_remap(blockIdx.x, nb);
    const int tu = bid % tiles_u, tv = bid / tiles_u;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int iu = tu * TILE_U + (wave & 1) * 8 + (lane & 7);
    const int iv = tv * TILE_V + (wave >> 1) * 8 + (lane >> 3);
    const bool valid = iu < nu && iv < nv;
    const int pix = iv * nu + iu;
    double pv = 0.0;
    if (valid) {
        const RayRec<T> r = rays[pix];
        const T e[3] = {r.e[0], r.e[1], r.e[2]};
        const T d[3] = {r.d[0], r.d[1], r.d[2]};
        const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
        double acc = 0.0;
        for (int s = 0; s < r.n; ++s) {
            int l[3];
            T z[3];
            sample_cell(e, d, s, n0, n1, n2, l, z);
            const T *b = f + (l[0] + s1 * l[1] + s2 * l[2]);
            const T v000 = b[0], v100 = b[1];
            const T v010 = b[s1], v110 = b[s1 + 1];
            const T v001 = b[s2], v101 = b[s2 + 1];
            const T v011 = b[s2 + s1], v111 = b[s2 + s1 + 1];
            const T x00 = lerp_t(v000, v100, z[0]), x10 = lerp_t(v010, v110, z[0]);
            const T x01 = lerp_t(v001, v101, z[0]), x11 = lerp_t(v011, v111, z[0]);
            const T y0 = lerp_t(x00, x10, z[1]), y1 = lerp_t(x01, x11, z[1]);
            acc += (double)lerp_t(y0, y1, z[2]);
        }
        const T pt = (T)((double)r.dt * acc);
        p[pix] = pt;
        pv = (double)pt;
    }
    if constexpr (SUMS) {
        const double yv = valid ? (double)y[pix] : 0.0;
        const double vals[3] = {pv, pv * yv, pv * pv};
        grid_reduce<3>(vals, partials, counter, sums, bid, nb, 1.0);
    }
}

int drr_forward_blocks(int nu, int nv) {
    return ((nu + TILE_U - 1) / TILE_U) * ((nv + TILE_V - 1) / TILE_V);
}

hipError_t launch_drr_forward(pcas_dtype dt, const VolDims &v, int nu, int nv, const void *rays,
                              const void *f, void *p, const void *y, double *partials,
                              uint32_t *counter, double *sums, hipStream_t s) {
    const int tiles_u = (nu + TILE_U - 1) / TILE_U;
    dim3 grid(drr_forward_blocks(nu, nv)), block(256);
    if (dt == PCAS_F32) {
        if (sums)
            hipLaunchKernelGGL((k_drr_forward<float, true>), grid, block, 0, s, v.n0, v.n1, v.n2, nu,
                               nv, tiles_u, (const RayRec<float> *)rays, (const float *)f,
                               (float *)p, (const float *)y, partials, counter, sums);
        else
            hipLaunchKernelGGL((k_drr_forward<float, false>), grid, block, 0, s, v.n0, v.n1, v.n2,
                               nu, nv, tiles_u, (const RayRec<float> *)rays, (const float *)f,
                               (float *)p, (const float *)nullptr, nullptr, nullptr, nullptr);
    } else {
        if (sums)
            hipLaunchKernelGGL((k_drr_forward<double, true>), grid, block, 0, s, v.n0, v.n1, v.n2,
                               nu, nv, tiles_u, (const RayRec<double> *)rays, (const double *)f,
                               (double *)p, (const double *)y, partials, counter, sums);
        else
            hipLaunchKernelGGL((k_drr_forward<double, false>), grid, block, 0, s, v.n0, v.n1, v.n2,
                               nu, nv, tiles_u, (const RayRec<double> *)rays, (const double *)f,
                               (double *)p, (const double *)nullptr, nullptr, nullptr, nullptr);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// LDS accumulator of a brick with a one-voxel halo on every side, so that
// all eight corners of any cell touching the brick have a slot; halo slots
// collect contributions that belong to neighbouring bricks and are dropped
// at write-out.  Slice pitch 18*18+1 words spreads z-neighbours over banks.
constexpr int ACC_YP = BRICK_X + 2;
constexpr int ACC_ZP = (BRICK_Y + 2) * ACC_YP + 1;
constexpr int ACC_WORDS = (BRICK_Z + 2) * ACC_ZP;
constexpr int QCAP = 128;   // queued rays per wave (two batches)

template <typename T>
__device__ __forceinline__ bool brick_sample_range(const RayRec<T> &r, const T (&lob)[3],
                                                   const T (&hib)[3], int *s0, int *s1) {
    T s_lo = (T)0, s_hi = (T)(r.n - 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (r.d[c] != (T)0) {
            const T inv = (T)1 / r.d[c];
            T ta = (lob[c] - r.e[c]) * inv - (T)0.5;
            T tb = (hib[c] - r.e[c]) * inv - (T)0.5;
            if (ta > tb) { const T tmp = ta; ta = tb; tb = tmp; }
            s_lo = ta > s_lo ? ta : s_lo;
            s_hi = tb < s_hi ? tb : s_hi;
        } else if (r.e[c] < lob[c] || r.e[c] > hib[c]) {
            return false;
        }
    }
    if (!(s_lo <= s_hi + (T)2)) return false;
    *s0 = max(0, (int)floor(s_lo) - 1);
    *s1 = min(r.n - 1, (int)ceil(s_hi) + 1);
    return *s0 <= *s1;
}

template <typename T>
__device__ __forceinline__ void flush_cell(T *acc, int base, const T (&cw)[8]) {
    if (base < 0) return;
    T *p = acc + base;
    atomicAdd(p, cw[0]);
    atomicAdd(p + 1, cw[1]);
    atomicAdd(p + ACC_YP, cw[2]);
    atomicAdd(p + ACC_YP + 1, cw[3]);
    atomicAdd(p + ACC_ZP, cw[4]);
    atomicAdd(p + ACC_ZP + 1, cw[5]);
    atomicAdd(p + ACC_ZP + ACC_YP, cw[6]);
    atomicAdd(p + ACC_ZP + ACC_YP + 1, cw[7]);
}

// One lane walks the queued ray's samples near the brick.  Samples whose
// cell has no corner in the brick are skipped; the eight corner weights of
// consecutive samples sharing a cell are summed in registers and added to
// LDS when the cell changes.
template <typename T>
__device__ __forceinline__ void splat_ray(T *acc, const RayRec<T> &r, T cst, int s0, int s1,
                                          int n0, int n1, int n2, const int (&lo)[3],
                                          const int (&hi)[3]) {
    const T e[3] = {r.e[0], r.e[1], r.e[2]};
    const T d[3] = {r.d[0], r.d[1], r.d[2]};
    int cur = -1;   // halo-array offset of the cell being accumulated
    T cw[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) cw[q] = (T)0;
    for (int s = s0; s <= s1; ++s) {
        int l[3];
        T z[3];
        sample_cell(e, d, s, n0, n1, n2, l, z);
        const int lx = l[0] - lo[0] + 1, ly = l[1] - lo[1] + 1, lz = l[2] - lo[2] + 1;
        const bool touches = lx >= 0 && lx <= hi[0] - lo[0] + 1 && ly >= 0 &&
                             ly <= hi[1] - lo[1] + 1 && lz >= 0 && lz <= hi[2] - lo[2] + 1;
        if (!touches) continue;
        const int base = lz * ACC_ZP + ly * ACC_YP + lx;
        if (base != cur) {
            flush_cell(acc, cur, cw);
#pragma unroll
            for (int q = 0; q < 8; ++q) cw[q] = (T)0;
            cur = base;
        }
        const T c1a = cst * ((T)1 - z[1]), c1b = cst * z[1];
        const T za = (T)1 - z[2], zb = z[2];
        const T w00 = c1a * za, w10 = c1b * za, w01 = c1a * zb, w11 = c1b * zb;
        const T xa = (T)1 - z[0], xb = z[0];
        cw[0] = fma_t(w00, xa, cw[0]);
        cw[1] = fma_t(w00, xb, cw[1]);
        cw[2] = fma_t(w10, xa, cw[2]);
        cw[3] = fma_t(w10, xb, cw[3]);
        cw[4] = fma_t(w01, xa, cw[4]);
        cw[5] = fma_t(w01, xb, cw[5]);
        cw[6] = fma_t(w11, xa, cw[6]);
        cw[7] = fma_t(w11, xb, cw[7]);
    }
    flush_cell(acc, cur, cw);
}

template <typename T, bool FORM_R>
__global__ __launch_bounds__(64) void k_drr_adjoint(VolDims vd, Frame fr, int nbx, int nby,
                                                    const RayRec<T> *__restrict__ rays,
                                                    const T *__restrict__ rp,
                                                    const T *__restrict__ y, double a, double b,
                                                    T *__restrict__ bp) {
    __shared__ T acc[ACC_WORDS];
    __shared__ int q_pix[QCAP], q_s0[QCAP], q_s1[QCAP];
    __shared__ T q_c[QCAP];
    const int n0 = vd.n0, n1 = vd.n1, n2 = vd.n2;
    const int nb = gridDim.x;
    const int bid = xcd_remap(blockIdx.x, nb);
    const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
    const int lo[3] = {bx * BRICK_X, by * BRICK_Y, bz * BRICK_Z};
    const int hi[3] = {min(lo[0] + BRICK_X, n0) - 1, min(lo[1] + BRICK_Y, n1) - 1,
                       min(lo[2] + BRICK_Z, n2) - 1};
    const int nn[3] = {n0, n1, n2};
    const int lane = threadIdx.x;
    for (int t = lane; t < ACC_WORDS; t += 64) acc[t] = (T)0;

    // Detector footprint of the region whose samples can reach the brick:
    // index box [lo - 1, hi + 1] clipped to the grid, projected through its
    // eight corners (the source is outside the volume, so every depth > 0).
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    if (lane < 8) {
        double rel[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int idx = ((lane >> c) & 1) ? min(hi[c] + 1, nn[c] - 1) : max(lo[c] - 1, 0);
            rel[c] = vd.origin[c] + idx * vd.spacing[c] - fr.src[c];
        }
        const double depth = rel[0] * fr.en[0] + rel[1] * fr.en[1] + rel[2] * fr.en[2];
        const double pu = (rel[0] * fr.eu[0] + rel[1] * fr.eu[1] + rel[2] * fr.eu[2]) * fr.sid / depth;
        const double pv = (rel[0] * fr.ev[0] + rel[1] * fr.ev[1] + rel[2] * fr.ev[2]) * fr.sid / depth;
        umin = umax = (pu - fr.offset_u) / fr.pitch_u + 0.5 * (fr.nu - 1);
        vmin = vmax = (pv - fr.offset_v) / fr.pitch_v + 0.5 * (fr.nv - 1);
    }
    umin = wave_min(umin);
    umax = wave_max(umax);
    vmin = wave_min(vmin);
    vmax = wave_max(vmax);
    // clamp in floating point first so the conversions stay in range
    const int iu0 = (int)fmin(fmax(floor(umin) - 1.0, 0.0), (double)fr.nu);
    const int iu1 = (int)fmin(fmax(ceil(umax) + 1.0, -1.0), (double)(fr.nu - 1));
    const int iv0 = (int)fmin(fmax(floor(vmin) - 1.0, 0.0), (double)fr.nv);
    const int iv1 = (int)fmin(fmax(ceil(vmax) + 1.0, -1.0), (double)(fr.nv - 1));
    const int W = iu1 - iu0 + 1, H = iv1 - iv0 + 1;
    // Candidate batches interleave the footprint: lane (lu, lv) of batch
    // (bu, bv) takes pixel (iu0 + lu*Su + bu, iv0 + lv*Sv + bv), so the rays
    // of one batch sit Su x Sv pixels apart and rarely share a cell.
    const int Su = W > 0 ? (W + 7) / 8 : 0;
    const int Sv = H > 0 ? (H + 7) / 8 : 0;
    const int ntiles = (W > 0 && H > 0) ? Su * Sv : 0;
    __syncthreads();

    const T lob[3] = {(T)(lo[0] - 1), (T)(lo[1] - 1), (T)(lo[2] - 1)};
    const T hib[3] = {(T)(hi[0] + 1), (T)(hi[1] + 1), (T)(hi[2] + 1)};
    int qn = 0;   // wave-uniform queue length
    for (int tile = 0; tile <= ntiles; ++tile) {
        if (tile < ntiles) {
            // candidate ray of this lane
            const int iu = iu0 + (lane & 7) * Su + tile % Su;
            const int iv = iv0 + (lane >> 3) * Sv + tile / Su;
            bool active = false;
            int pix = 0, s0 = 0, s1 = -1;
            T cst = (T)0;
            if (iu <= iu1 && iv <= iv1) {
                pix = iv * fr.nu + iu;
                const RayRec<T> r = rays[pix];
                if (r.n > 0) {
                    T rv;
                    if constexpr (FORM_R)
                        rv = (T)((double)rp[pix] - a * (double)y[pix] - b);
                    else
                        rv = rp[pix];
                    cst = r.dt * rv;
                    active = cst != (T)0 && brick_sample_range(r, lob, hib, &s0, &s1);
                }
            }
            const uint64_t mask = __ballot(active);
            if (active) {
                const int pos = qn + __popcll(mask & ((1ull << lane) - 1ull));
                q_pix[pos] = pix;
                q_s0[pos] = s0;
                q_s1[pos] = s1;
                q_c[pos] = cst;
            }
            qn += __popcll(mask);
            __syncthreads();
            if (qn < 64) continue;
        } else if (qn == 0) {
            break;
        }
        // drain one batch of up to 64 queued rays, one per lane
        if (lane < qn) {
            const int pix = q_pix[lane];
            const RayRec<T> r = rays[pix];
            splat_ray(acc, r, q_c[lane], q_s0[lane], q_s1[lane], n0, n1, n2, lo, hi);
        }
        const int rest = qn > 64 ? qn - 64 : 0;
        __syncthreads();
        if (lane < rest) {
            q_pix[lane] = q_pix[64 + lane];
            q_s0[lane] = q_s0[64 + lane];
            q_s1[lane] = q_s1[64 + lane];
            q_c[lane] = q_c[64 + lane];
        }
        __syncthreads();
        qn = rest;
    }
    __syncthreads();
    const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
    for (int t = lane; t < BRICK_X * BRICK_Y * BRICK_Z; t += 64) {
        const int li = t % BRICK_X, lj = (t / BRICK_X) % BRICK_Y, lk = t / (BRICK_X * BRICK_Y);
        const int i = lo[0] + li, j = lo[1] + lj, k = lo[2] + lk;
        if (i < n0 && j < n1 && k < n2)
            bp[i + s1 * j + s2 * k] = acc[(lk + 1) * ACC_ZP + (lj + 1) * ACC_YP + (li + 1)];
    }
}

hipError_t launch_drr_adjoint(pcas_dtype dt, const VolDims &v, const Frame &fr, const void *rays,
                              const void *r_or_p, const void *y, double a, double b, void *bp,
                              hipStream_t s) {
    const int nbx = (v.n0 + BRICK_X - 1) / BRICK_X;
    const int nby = (v.n1 + BRICK_Y - 1) / BRICK_Y;
    const int nbz = (v.n2 + BRICK_Z - 1) / BRICK_Z;
    dim3 grid(nbx * nby * nbz), block(64);
    if (dt == PCAS_F32) {
        if (y)
            hipLaunchKernelGGL((k_drr_adjoint<float, true>), grid, block, 0, s, v, fr, nbx, nby,
                               (const RayRec<float> *)rays, (const float *)r_or_p,
                               (const float *)y, a, b, (float *)bp);
        else
            hipLaunchKernelGGL((k_drr_adjoint<float, false>), grid, block, 0, s, v, fr, nbx, nby,
                               (const RayRec<float> *)rays, (const float *)r_or_p,
                               (const float *)nullptr, 0.0, 0.0, (float *)bp);
    } else {
        if (y)
            hipLaunchKernelGGL((k_drr_adjoint<double, true>), grid, block, 0, s, v, fr, nbx, nby,
                               (const RayRec<double> *)rays, (const double *)r_or_p,
                               (const double *)y, a, b, (double *)bp);
        else
            hipLaunchKernelGGL((k_drr_adjoint<double, false>), grid, block, 0, s, v, fr, nbx, nby,
                               (const RayRec<double> *)rays, (const double *)r_or_p,
                               (const double *)nullptr, 0.0, 0.0, (double *)bp);
    }
    return hipGetLastError();
}

}  // namespace pcas
