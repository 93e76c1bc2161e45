// Device helpers: wave64 / block reductions in double and the
// fixed-order grid reduction, finished by the last block to arrive or by a
// later launch (deterministic either way).
#pragma once

#include "internal.h"

namespace pcas {

// A lane's value moved by a DPP pattern (both halves of the double), zero in
// the lanes of rows that ROW_MASK leaves out.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Sum over the 64 lanes of a wave, returned to every lane (a butterfly of
// lane permutes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The same sum by register moves across lanes (pairs, quads, half rows and
// rows of 16, then the row broadcasts) instead of LDS permutes, then the
// last lane's total: no LDS round trips, for the single-block passes that
// finish a reduction (inside the large kernels the permute form keeps the
// register count down).  The order of the additions is fixed.
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_move<0xB1, 0xF>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E, 0xF>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141, 0xF>(v);   // row_half_mirror
    v += dpp_move<0x140, 0xF>(v);   // row_mirror: every lane holds its row's sum
    v += dpp_move<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)lo);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ double load_agent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_agent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums vals[0..NS) over the block (any multiple of 64 threads up to 1024)
// and stores the block's totals in partials[red_slot(NS, j, bid, nblocks)].
template <int NS>
__device__ void block_partials(const double (&vals)[NS], double *__restrict__ partials, int bid,
                               int nblocks) {
    static_assert(NS <= RED_SLOTS_WIDE, "too many reduction slots");
    __shared__ double sm[NS][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        double v = wave_sum(vals[j]);
        if (lane == 0) sm[j][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            double t = 0.0;
            for (int w = 0; w < nwaves; ++w) t += sm[j][w];
            store_agent(&partials[red_slot(NS, j, bid, nblocks)], t);
        }
    }
}

// The first `width` threads of the block (a multiple of 64, at most
// blockDim.x; every thread must call this) sum the partials of nblocks
// blocks in one fixed order: thread t takes blocks t, t + width, ..., then
// its wave's sum, then the width / 64 waves in order.  Any block thus gets
// the same bits for the same width; grid_reduce uses its own block width.
// Thread 0 returns scale * total in tot.  COHERENT reads through to the
// agent-coherent level (partials written by other blocks of this kernel).
template <int NS, bool COHERENT>
__device__ void sum_partials(const double *__restrict__ partials, int nblocks, double scale,
                             int width, double (&tot)[NS]) {
    __shared__ double sm[NS][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = width >> 6;
    double acc[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) acc[j] = 0.0;
    // unrolled so that several blocks' loads are in flight at once (the
    // order of the additions into acc[j] stays the same)
#pragma unroll 4
    for (int b = threadIdx.x; threadIdx.x < width && b < nblocks; b += width) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const double *q = &partials[red_slot(NS, j, b, nblocks)];
            acc[j] += COHERENT ? load_agent(q) : *q;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        double v = wave_sum_dpp(acc[j]);
        if (lane == 0 && wave < nwaves) sm[j][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            double t = 0.0;
            for (int w = 0; w < nwaves; ++w) t += sm[j][w];
            tot[j] = scale * t;
        }
    }
}

// block_partials, then the last block to arrive (an agent-scope counter)
// runs sum_partials and writes out[j].  Each block's counter increment is a
// release and only the last block acquires (the increments form one release
// sequence), so one L2 invalidate per launch instead of one per block.  The
// counter must be zero on entry; the last block resets it.  Every thread of
// every block must call this exactly once.
template <int NS>
__device__ void grid_reduce(const double (&vals)[NS], double *__restrict__ partials,
                            uint32_t *counter, double *__restrict__ out, int bid, int nblocks,
                            double scale) {
    __shared__ int is_last;
    block_partials<NS>(vals, partials, bid, nblocks);
    if (threadIdx.x == 0) {
        uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE,
                                               __HIP_MEMORY_SCOPE_AGENT);
        is_last = (prev == (uint32_t)(nblocks - 1));
    }
    __syncthreads();
    if (!is_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double tot[NS];
    sum_partials<NS, true>(partials, nblocks, scale, (int)blockDim.x, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NS; ++j) store_agent(&out[j], tot[j]);
        __hip_atomic_store(counter, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// In a kernel whose totals are finished by a later launch (counter ==
// nullptr): the block's partials only.  Otherwise grid_reduce.
template <int NS>
__device__ void reduce_or_defer(const double (&vals)[NS], double *__restrict__ partials,
                                uint32_t *counter, double *__restrict__ out, int bid, int nblocks,
                                double scale) {
    if (counter)
        grid_reduce<NS>(vals, partials, counter, out, bid, nblocks, scale);
    else
        block_partials<NS>(vals, partials, bid, nblocks);
}

// Split a displacement x (mm) into whole voxels and the fractional part
// (Eq. A.5's integer and fractional parts): d = x / spacing rounded once,
// l = floor(d), z = d - l, exactly.  Contraction is off here so that z is the
// fraction of the rounded d (in [0, 1)) and an integer d gives z = 0.
template <typename T>
__device__ __forceinline__ void split_disp(T x, T inv_s, int &l, T &z) {
#pragma clang fp contract(off)
    const T d = x * inv_s;
    const T fl = floor(d);
    l = (int)fl;
    z = d - fl;
}

__device__ __forceinline__ float clamp_t(float q, float top) {
    return __builtin_amdgcn_fmed3f(q, 0.0f, top);
}
__device__ __forceinline__ double clamp_t(double q, double top) {
    return fmin(fmax(q, 0.0), top);
}

// Largest index-space position a sample takes along an axis of n >= 2
// voxels: the representable value just below n - 1, so that the lower corner
// floor(q) is at most n - 2 and the fraction stays below 1.  (A sample lands
// on the last voxel centre only where a ray runs along the grid's far face;
// its weights then move by one ulp.)
template <typename T> __device__ __forceinline__ T below_last(int n);
template <> __device__ __forceinline__ float below_last<float>(int n) {
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, (float)(n - 1)) - 1u);
}
template <> __device__ __forceinline__ double below_last<double>(int n) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, (double)(n - 1)) - 1ull);
}

template <typename T> struct GridTop {
    T t[3];
};
template <typename T>
__device__ __forceinline__ GridTop<T> grid_top(int n0, int n1, int n2) {
    return {{below_last<T>(n0), below_last<T>(n1), below_last<T>(n2)}};
}

__device__ __forceinline__ float fract_t(float q) { return __builtin_amdgcn_fractf(q); }
__device__ __forceinline__ double fract_t(double q) { return __builtin_amdgcn_fract(q); }

// Position of a ray sample along one axis in voxel-index units, clamped to
// [0, top], split into the lower corner l and the fraction z (exact: q is
// non-negative, so z = q - floor(q) is representable).  sh is the sample
// index plus one half (exact in T), so the position is e + sh d with one
// rounding.  For a fixed ray, l is monotone in sh (every step here is).
template <typename T>
__device__ __forceinline__ void axis_cell(T e, T d, T sh, T top, int &l, T &z) {
    const T q = clamp_t(fma_t(sh, d, e), top);
    l = (int)q;
    z = fract_t(q);
}

// The three axes of a sample.  drr_forward and drr_adjoint both call this,
// so a sample's corners and weights are bit-identical in the two kernels.
template <typename T>
__device__ __forceinline__ void sample_cell(const T (&e)[3], const T (&d)[3], T sh,
                                            const GridTop<T> &top, int (&l)[3], T (&z)[3]) {
    axis_cell(e[0], d[0], sh, top.t[0], l[0], z[0]);
    axis_cell(e[1], d[1], sh, top.t[1], l[1], z[1]);
    axis_cell(e[2], d[2], sh, top.t[2], l[2], z[2]);
}

// Raw buffer access (gfx9-family descriptor): the eight neighbours of a cell
// are read through one 32-bit byte offset plus wave-uniform strides, and any
// offset past num_records reads as zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// The job of a batched launch that owns this block (jobs sorted by block0;
// the scan is wave-uniform).
template <typename Job>
__device__ __forceinline__ int job_of(const Job *__restrict__ jobs, int njobs) {
    int j = 0;
    while (j + 1 < njobs && (int)blockIdx.x >= jobs[j + 1].block0) ++j;
    return j;
}

}  // namespace pcas
