// a4: forward projection P f and a6: back-projection P^T r.
//
// Forward: each ray is marched by fwd_split(ts) lanes that take interleaved
// samples (s = seg, seg + split, ...); a wave covers a tile of neighbouring
// rays, whose samples at equal index sit within a few voxels of each other.
// A block stages the voxels its bundle of rays can reach slab by slab in LDS.
// The partial sums of a ray are combined by a fixed butterfly.
//
// Adjoint: the exact transpose of the forward without global atomics.  A
// 512-thread workgroup owns a 32 x 16 x 8 voxel brick held in LDS.  It
// visits every ray whose pixel lies in the detector footprint of the brick
// (plus a one-voxel apron), re-creates exactly the samples of that ray whose
// 2x2x2 cell touches the brick (same ray record, same sample_cell
// arithmetic as the forward), and adds dt * r * weight for the corners of
// that cell.  Each (sample, corner) pair therefore lands in exactly one
// brick, and the brick is written to HBM once.  Accumulation is in 64-bit
// fixed point with a per-brick scale chosen so that no partial sum can
// overflow; integer addition is associative, so the result does not depend
// on the order in which the four waves add, and is bit-for-bit reproducible.
#include <algorithm>
#include <type_traits>

#include "jacobian.h"

namespace pcas {

template <typename T>
__device__ __forceinline__ T lerp_t(T a, T b, T z) {
    return fma_t(z, b - a, a);
}

// Trilinear value from the eight corners of a cell (vXYZ: X, Y, Z = 0 or 1
// for the lower or upper corner), x pairs first, then y, then z.
template <typename T>
__device__ __forceinline__ T trilinear(T v000, T v100, T v010, T v110, T v001, T v101, T v011,
                                       T v111, const T (&z)[3]) {
    const T x00 = lerp_t(v000, v100, z[0]), x10 = lerp_t(v010, v110, z[0]);
    const T x01 = lerp_t(v001, v101, z[0]), x11 = lerp_t(v011, v111, z[0]);
    const T y0 = lerp_t(x00, x10, z[1]), y1 = lerp_t(x01, x11, z[1]);
    return lerp_t(y0, y1, z[2]);
}

// Value at a sample from the volume in global memory: corner byte offset vo,
// wave-uniform byte strides sb1 (y) and sb2 (z).
template <typename T>
__device__ __forceinline__ T gather_global(__amdgpu_buffer_rsrc_t rf, int vo, int sb1, int sb2,
                                           const T (&z)[3]) {
    constexpr int ES = (int)sizeof(T);
    const int sb12 = sb1 + sb2;
    const T v000 = buf_load(rf, vo, 0, T()), v100 = buf_load(rf, vo + ES, 0, T());
    const T v010 = buf_load(rf, vo, sb1, T()), v110 = buf_load(rf, vo + ES, sb1, T());
    const T v001 = buf_load(rf, vo, sb2, T()), v101 = buf_load(rf, vo + ES, sb2, T());
    const T v011 = buf_load(rf, vo, sb12, T()), v111 = buf_load(rf, vo + ES, sb12, T());
    return trilinear(v000, v100, v010, v110, v001, v101, v011, v111, z);
}

// Geometric ray of detector pixel (iu, iv) in voxel-index coordinates:
// points o + t q, t >= 0 (o is the source).
struct IdxRay {
    double o[3], q[3];
};

__host__ __device__ inline IdxRay pixel_ray(const VolDims &v, const Frame &fr, int iu, int iv) {
    const double u = (iu - 0.5 * (fr.nu - 1)) * fr.pitch_u + fr.offset_u;
    const double w = (iv - 0.5 * (fr.nv - 1)) * fr.pitch_v + fr.offset_v;
    IdxRay r;
    for (int c = 0; c < 3; ++c) {
        const double P = fr.det[c] + u * fr.eu[c] + w * fr.ev[c];
        r.o[c] = (fr.src[c] - v.origin[c]) * v.inv_s[c];
        r.q[c] = (P - fr.src[c]) * v.inv_s[c];
    }
    return r;
}

// Where the ray of pixel (iu, iv) crosses the plane AX = plane: the two
// other index coordinates (in increasing axis order).  False when the ray
// runs (almost) parallel to the plane or crosses it absurdly far away.
__host__ __device__ inline bool plane_point(const VolDims &v, const Frame &fr, int AX, int iu,
                                            int iv, double plane, double &pb, double &pc) {
    const IdxRay r = pixel_ray(v, fr, iu, iv);
    const int B = AX == 0 ? 1 : 0, C = AX == 2 ? 1 : 2;
    if (!(fabs(r.q[AX]) > 1e-9)) return false;
    const double t = (plane - r.o[AX]) / r.q[AX];
    pb = r.o[B] + t * r.q[B];
    pc = r.o[C] + t * r.q[C];
    return fabs(pb) < 1e9 && fabs(pc) < 1e9;
}

// Cell range [lo, hi] along an axis of n voxels holding positions in
// [mn, mx], widened by 1/20 cell (far above the rounding of sample positions
// in either precision, far below a cell) and clamped to the grid.
__host__ __device__ inline void cell_range(double mn, double mx, int n, int &lo, int &hi) {
    lo = (int)fmin(fmax(floor(mn - 0.05), 0.0), (double)(n - 2));
    hi = (int)fmin(fmax(floor(mx + 0.05), 0.0), (double)(n - 2));
}

// Cells that samples of a bundle of rays (pixels [iu0, iu1] x [iv0, iv1])
// can occupy across axis AX while their cell along AX lies in [A0, A0 + S):
// on every plane AX = const the bundle's crossing points lie in the convex
// quadrilateral of its four corner rays (a central projection maps the
// detector rectangle onto it), so the box of the corner rays' crossings of
// the planes AX = A0 - 1 and AX = A0 + S + 1 (points 0..7: corner = p & 3,
// far plane = p >> 2), slightly widened and clamped, holds every such
// sample's cell.
__host__ __device__ inline bool slab_corner_point(const VolDims &v, const Frame &fr, int AX,
                                                  int iu0, int iu1, int iv0, int iv1, int A0,
                                                  int S, int pt, double &pb, double &pc) {
    const double plane = (pt >> 2) ? (double)(A0 + S + 1) : (double)(A0 - 1);
    return plane_point(v, fr, AX, (pt & 1) ? iu1 : iu0, (pt & 2) ? iv1 : iv0, plane, pb, pc);
}

static bool slab_cells_host(const VolDims &v, const Frame &fr, int AX, int iu0, int iu1, int iv0,
                            int iv1, int A0, int S, int (&lo)[2], int (&hi)[2]) {
    double mn[2] = {1e300, 1e300}, mx[2] = {-1e300, -1e300};
    for (int pt = 0; pt < 8; ++pt) {
        double pb, pc;
        if (!slab_corner_point(v, fr, AX, iu0, iu1, iv0, iv1, A0, S, pt, pb, pc)) return false;
        mn[0] = fmin(mn[0], pb);
        mx[0] = fmax(mx[0], pb);
        mn[1] = fmin(mn[1], pc);
        mx[1] = fmax(mx[1], pc);
    }
    const int nb = AX == 0 ? v.n1 : v.n0;
    cell_range(mn[0], mx[0], nb, lo[0], hi[0]);
    cell_range(mn[1], mx[1], v.n2, lo[1], hi[1]);
    return true;
}

// Row pitch of a staged box, in voxels, for an extent e along x: e rounded
// up to 3 mod 8.  One LDS access of a wave reads cells of neighbouring rays
// and samples, a row or two and a column or two apart.  Cells whose index
// differs by dx + dy * pitch with |dx| <= 1, |dy| <= 2 or |dx| <= 2, |dy| <= 1
// then never differ by a multiple of 8 (nor of 16), so the voxels (16 bytes
// each for four interleaved FP32 volumes) fall in different bank groups;
// at pitches near a multiple of 8 they collide.
__host__ __device__ constexpr int box_pitch_x(int e) { return e + ((3 - e) & 7); }

// What the projection kernel does with each ray's value.
enum { FWD_WRITE = 0, FWD_SUMS = 1, FWD_DOT = 2, FWD_EVAL = 3 };

// LDS budget of the staged boxes: one volume 16 KB, several 32 KB.
constexpr int fwd_lds_bytes(int nv) { return nv == 1 ? FWD_LDS_BYTES : 2 * FWD_LDS_BYTES; }

// Forward projection of one bundle of tile_u(TS) x tile_v(TS) rays through NV
// volumes f[v * N + voxel] at once (same rays, same samples, same weights).
// The bundle walks the volume in slabs of `slab` cells along the axis AX
// its rays mostly travel (x or y): per slab the block copies the box of
// voxels its samples can touch (slab boxes from the bundle's corner rays)
// into LDS with coalesced row reads, then every lane takes its ray's samples
// whose cell lies in the slab from LDS.  The gathers thus hit LDS instead of
// the texture path; a lane with a sample outside the staged box (never
// expected) redoes that slab from global memory, so the result does not
// depend on the box estimate.  A block whose rays do not all travel the same
// way along AX (or that spans too many slabs) marches from global memory.
// Samples of a slab are summed in T and the slab sums in double; the order
// depends only on the geometry, so results are bit-for-bit reproducible.
//
// MODE FWD_WRITE / FWD_SUMS (NV = 1): p = P f, and for FWD_SUMS also
// (sum r0, sum r0 y, sum r0^2) for r0 = p - fit.a0 y - fit.b0 into
// out[0..2] (the host forms the objective from them: objective_from_moments).
// MODE FWD_DOT: the ray values
// q_v = (P f_v) are not stored; out[v] = 2 sum_rays r q_v with the residual
// r = p - a y - b of the stored projection p.  MODE FWD_EVAL (NV = K + 1):
// p = P f of volume 0 and the moment sums of launch_drr_forward_eval.
template <typename T, int AX, int NV, int MODE, int TS>
__device__ __forceinline__ void drr_forward_block(const VolDims &vd, const Frame &fr, int tiles_u,
                                                  int slab, const RayRec<T> *__restrict__ rays,
                                                  const T *__restrict__ f, T *__restrict__ p,
                                                  const T *__restrict__ y, double fa, double fb,
                                                  const FitArgs &fit, double *__restrict__ partials,
                                                  uint32_t *counter, double *__restrict__ out,
                                                  int lb, int nb) {
    constexpr int SPLIT = fwd_split(TS), WU = fwd_wu(TS), WV = fwd_wv(TS);
    constexpr int TU = tile_u(TS), TV = tile_v(TS);
    constexpr int CAPT = fwd_lds_bytes(NV) / (int)sizeof(T);   // all volumes
    constexpr int CAP = CAPT / NV;                               // one volume's box
    constexpr int ES = (int)sizeof(T);
    // NV >= 3: the box interleaves the volumes (element t of volume v at
    // t * NV + v), so that one sample's corners of every volume sit together
    constexpr bool IL = NV >= 3;
    __shared__ __align__(16) T box[CAPT];
    __shared__ int sbox[FWD_MAX_SLABS][4];
    __shared__ int sred[3];
    const int n0 = vd.n0, n1 = vd.n1, n2 = vd.n2;
    const int nn[3] = {n0, n1, n2};
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int nu = fr.nu, nv = fr.nv;
    const int bid = xcd_remap(lb, nb);
    const int tu = bid % tiles_u, tv = bid / tiles_u;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int seg = lane % SPLIT, rl = lane / SPLIT;
    const int iu = tu * TU + (wave & 1) * WU + rl % WU;
    const int iv = tv * TV + (wave >> 1) * WV + rl / WU;
    const bool valid = iu < nu && iv < nv;
    const int pix = iv * nu + iu;
    RayRec<T> r;
    if (valid) {
        r = rays[pix];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) r.e[c] = r.d[c] = (T)0;
        r.dt = (T)0;
        r.n = 0;
    }
    const T e[3] = {r.e[0], r.e[1], r.e[2]};
    const T d[3] = {r.d[0], r.d[1], r.d[2]};
    __amdgpu_buffer_rsrc_t rf[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) rf[v] = make_rsrc(f + v * N, (uint32_t)(N * ES));
    const int sb1 = n0 * ES, sb2 = n0 * n1 * ES;   // wave-uniform strides
    const GridTop<T> top = grid_top<T>(n0, n1, n2);

    // Slabs the bundle's samples span, and the direction they are crossed.
    if (tid == 0) {
        sred[0] = 0x7fffffff;
        sred[1] = -1;
        sred[2] = 0;
    }
    __syncthreads();
    if (r.n > 0 && seg == 0 && slab > 0) {
        int la0, la1;
        T zz;
        axis_cell(e[AX], d[AX], (T)0.5, top.t[AX], la0, zz);
        axis_cell(e[AX], d[AX], (T)(r.n - 1) + (T)0.5, top.t[AX], la1, zz);
        atomicMin(&sred[0], min(la0, la1) / slab);
        atomicMax(&sred[1], max(la0, la1) / slab);
        atomicOr(&sred[2], d[AX] > (T)0 ? 1 : (d[AX] < (T)0 ? 2 : 4));
    }
    __syncthreads();
    const int kmin = sred[0], kmax = sred[1], votes = sred[2];
    const bool use_slabs = (votes == 1 || votes == 2) && kmax - kmin < FWD_MAX_SLABS;

    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    const T shn = (T)r.n;          // sample s exists iff s + 1/2 < n
    T sh = (T)seg + (T)0.5;
    if (use_slabs) {
        const int iu0 = tu * TU, iu1 = min(iu0 + TU, nu) - 1;
        const int iv0 = tv * TV, iv1 = min(iv0 + TV, nv) - 1;
        // staged box of every slab: eight lanes per slab, one per corner ray
        // and plane, reduced with shuffles (keeps the FP64 geometry out of
        // the march's register budget)
        const int nsl = kmax - kmin + 1;
        for (int j0 = 0; j0 < nsl; j0 += 32) {
            const int j = j0 + (tid >> 3), pt = tid & 7;
            double mnb = 1e300, mxb = -1e300, mnc = 1e300, mxc = -1e300;
            int ok = 1;
            if (j < nsl) {
                double pb = 0.0, pc = 0.0;
                ok = slab_corner_point(vd, fr, AX, iu0, iu1, iv0, iv1, (kmin + j) * slab, slab, pt,
                                       pb, pc);
                mnb = mxb = pb;
                mnc = mxc = pc;
            }
#pragma unroll
            for (int m = 1; m < 8; m <<= 1) {
                mnb = fmin(mnb, __shfl_xor(mnb, m, 64));
                mxb = fmax(mxb, __shfl_xor(mxb, m, 64));
                mnc = fmin(mnc, __shfl_xor(mnc, m, 64));
                mxc = fmax(mxc, __shfl_xor(mxc, m, 64));
                ok &= __shfl_xor(ok, m, 64);
            }
            if (j < nsl && pt == 0) {
                int *sb = sbox[j];
                if (ok) {
                    constexpr int B = AX == 0 ? 1 : 0;
                    cell_range(mnb, mxb, nn[B], sb[0], sb[1]);
                    cell_range(mnc, mxc, n2, sb[2], sb[3]);
                } else {
                    sb[0] = 1;
                    sb[1] = 0;   // empty: march this slab from global memory
                    sb[2] = 1;
                    sb[3] = 0;
                }
            }
        }
        // the lane's next sample, computed once and carried across slabs.
        // The cell of a sample past the ray's end is computed as well (it is
        // clamped to the grid and never used: every loop tests `have` first);
        // computing it unconditionally spares the loops their register copies.
        int l[3];
        T z[3];
        bool have = sh < shn;
        sample_cell(e, d, sh, top, l, z);
        __syncthreads();
        for (int i = 0; i < nsl; ++i) {
            const int k = votes == 1 ? kmin + i : kmax - i;
            const int A0 = k * slab;
            const int *sb = sbox[k - kmin];
            // staged voxel box [o, o + ext) per axis
            int o[3], ext[3];
            o[AX] = A0;
            ext[AX] = min(A0 + slab, nn[AX] - 1) - A0 + 1;
            constexpr int B = AX == 0 ? 1 : 0;
            o[B] = sb[0];
            ext[B] = sb[1] - sb[0] + 2;
            o[2] = sb[2];
            ext[2] = sb[3] - sb[2] + 2;
            // the box's row pitch (in voxels) may exceed its extent, so that
            // neighbouring rows fall in other LDS banks
            const int ex = box_pitch_x(ext[0]), exy = ex * ext[1];
            const bool staged = sb[0] <= sb[1] && sb[2] <= sb[3] && ext[0] <= CAP &&
                                ext[1] <= CAP && ext[2] <= CAP && exy <= CAP &&
                                exy * ext[2] <= CAP;
            const int size = exy * ext[2];          // box elements with the padding
            const int count = ext[0] * ext[1] * ext[2];   // voxels staged
            if (staged) {
                const int e0 = ext[0], e1 = ext[1];
                const int n01 = n0 * n1;
                const int gbase = o[0] + n0 * (o[1] + n1 * o[2]);
                // the voxel (tx, ty, tz) of the box, read at byte go of each
                // volume and stored at element bt = tx + ty ex + tz exy
                auto stage = [&](int go, int bt) {
                    if constexpr (IL) {
                        T val[NV];
#pragma unroll
                        for (int v = 0; v < NV; ++v) val[v] = buf_load(rf[v], go, 0, T());
#pragma unroll
                        for (int v = 0; v < NV; ++v) box[bt * NV + v] = val[v];
                    } else {
#pragma unroll
                        for (int v = 0; v < NV; ++v) box[v * size + bt] = buf_load(rf[v], go, 0, T());
                    }
                };
                // Quotients by float: exact for dividends below 2^13 (the
                // rounding error stays well below the 0.5 / divisor margin of
                // (t + 0.5) / divisor).
                const float ie0 = 1.0f / (float)e0, ie1 = 1.0f / (float)e1;
                const int R = (int)(256.5f * ie0);   // whole rows per pass of the block
                if (R > 0) {
                    // lane tid takes column tx = tid % e0 of rows r0 = tid / e0,
                    // r0 + R, ...; row r is (ty, tz) = (r % e1, r / e1), and a step
                    // of R rows adds (Ry, Rz) with at most one carry into z
                    const int r0 = (int)(((float)tid + 0.5f) * ie0);
                    const int tx = tid - __mul24(r0, e0);
                    const int Rz = (int)(((float)R + 0.5f) * ie1), Ry = R - __mul24(Rz, e1);
                    const int tz = (int)(((float)r0 + 0.5f) * ie1);
                    int ty = r0 - __mul24(tz, e1);
                    // byte offsets in the volume step modulo 2^32 (the carry's
                    // n0 n1 - e1 n0 may be negative); every offset read is a
                    // voxel's, below 2^31.  Box elements are tx + r ex (exy = e1 ex).
                    uint32_t go = (uint32_t)((gbase + tx + __mul24(ty, n0) + tz * n01) * ES);
                    const uint32_t dgo = ((uint32_t)Ry * (uint32_t)n0 + (uint32_t)Rz * (uint32_t)n01) * ES;
                    const uint32_t cgo = ((uint32_t)n01 - (uint32_t)e1 * (uint32_t)n0) * ES;
                    int bt = tx + __mul24(r0, ex);
                    const int dbt = __mul24(R, ex);
                    const int rows = e1 * ext[2];
                    if (r0 < R) {
                        for (int r = r0; r < rows; r += R) {
                            stage((int)go, bt);
                            ty += Ry;
                            go += dgo;
                            bt += dbt;
                            if (ty >= e1) {
                                ty -= e1;
                                go += cgo;
                            }
                        }
                    }
                } else {
                    // rows longer than the block: voxel t = tx + e0 (ty + e1 tz)
                    for (int t = tid; t < count; t += 256) {
                        const int q = (int)(((float)t + 0.5f) * ie0);
                        const int tx = t - __mul24(q, e0);
                        const int tz = (int)(((float)q + 0.5f) * ie1);
                        const int ty = q - __mul24(tz, e1);
                        stage((gbase + tx + __mul24(ty, n0) + tz * n01) * ES,
                              tx + __mul24(ty, ex) + __mul24(tz, exy));
                    }
                }
            }
            __syncthreads();
            // byte pitches of the box (of one voxel's NV values when
            // interleaved); offsets fit 24-bit products
            constexpr int EV = IL ? NV * ES : ES;
            const int px = ex * EV, pxy = exy * EV;
            [[maybe_unused]] const int pv = size * ES;
            const char *boxb = (const char *)box;
            T part[NV];   // this slab's samples, added to acc once
#pragma unroll
            for (int v = 0; v < NV; ++v) part[v] = (T)0;
            const T sh0 = sh;
            bool miss = !staged;
            if (staged) {
                // A ray's cells are monotone in sh along every axis, so the box
                // holds all of a lane's samples in this slab iff it holds the
                // first and the last.  The march reads at offsets clamped into
                // the box (every corner read stays inside it) and the two ends
                // are checked after it; along AX the slab test bounds the cell.
                constexpr int B2 = AX == 0 ? 1 : 0;
                auto inside = [&](const int (&c)[3]) {
                    return (unsigned)(c[B2] - o[B2]) < (unsigned)(ext[B2] - 1) &&
                           (unsigned)(c[2] - o[2]) < (unsigned)(ext[2] - 1);
                };
                const bool first_in = inside(l);
                // byte offset of a cell = its index in box pitches x EV - obase
                // (mod 2^32: cells below the box wrap past omax), at most omax =
                // the offset of the box's last cell
                const uint32_t obase = (uint32_t)((o[0] + o[1] * ex + o[2] * exy) * EV);
                const uint32_t omax =
                    (uint32_t)(((ext[0] - 2) + (ext[1] - 2) * ex + (ext[2] - 2) * exy) * EV);
                while (have && (unsigned)(l[AX] - A0) < (unsigned)slab) {
                    const uint32_t idx = __umul24((uint32_t)l[2], (uint32_t)exy) +
                                         __umul24((uint32_t)l[1], (uint32_t)ex) + (uint32_t)l[0];
                    const int off = (int)min(idx * (uint32_t)EV - obase, omax);
                    if constexpr (NV >= 3) {
                        // several volumes: the eight corner weights once, then
                        // eight products per volume instead of seven lerps
                        const T c0 = (T)1 - z[0], c1 = (T)1 - z[1], c2 = (T)1 - z[2];
                        const T a00 = c0 * c1, a10 = z[0] * c1, a01 = c0 * z[1], a11 = z[0] * z[1];
                        const T w000 = a00 * c2, w100 = a10 * c2, w010 = a01 * c2, w110 = a11 * c2;
                        const T w001 = a00 * z[2], w101 = a10 * z[2], w011 = a01 * z[2],
                                w111 = a11 * z[2];
                        const char *c = boxb + off;
                        const T *q0 = (const T *)c, *q1 = (const T *)(c + px);
                        const T *q2 = (const T *)(c + pxy), *q3 = (const T *)(c + pxy + px);
                        // the slab's running sum takes the eight products directly
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            T t = fma_t(w000, q0[v], part[v]);
                            t = fma_t(w100, q0[NV + v], t);
                            t = fma_t(w010, q1[v], t);
                            t = fma_t(w110, q1[NV + v], t);
                            t = fma_t(w001, q2[v], t);
                            t = fma_t(w101, q2[NV + v], t);
                            t = fma_t(w011, q3[v], t);
                            part[v] = fma_t(w111, q3[NV + v], t);
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            const char *c = boxb + (off + v * pv);
                            const T *c0 = (const T *)c, *c1 = (const T *)(c + px);
                            const T *c2 = (const T *)(c + pxy), *c3 = (const T *)(c + pxy + px);
                            part[v] += trilinear(c0[0], c0[1], c1[0], c1[1], c2[0], c2[1], c3[0],
                                                 c3[1], z);
                        }
                    }
                    sh += (T)SPLIT;
                    have = sh < shn;
                    sample_cell(e, d, sh, top, l, z);
                }
                if (sh != sh0) {   // the lane took samples in this slab
                    int lq[3];
                    T zq[3];
                    sample_cell(e, d, sh - (T)SPLIT, top, lq, zq);
                    miss = !(first_in && inside(lq));
                }
            }
            if (miss) {
                // a sample outside the staged box (or no box): redo this lane's
                // samples of the slab from global memory
#pragma unroll
                for (int v = 0; v < NV; ++v) part[v] = (T)0;
                sh = sh0;
                have = sh < shn;
                sample_cell(e, d, sh, top, l, z);
                while (have && (unsigned)(l[AX] - A0) < (unsigned)slab) {
                    const int go = (l[0] + n0 * (l[1] + n1 * l[2])) * ES;
#pragma unroll
                    for (int v = 0; v < NV; ++v) part[v] += gather_global(rf[v], go, sb1, sb2, z);
                    sh += (T)SPLIT;
                    have = sh < shn;
                    sample_cell(e, d, sh, top, l, z);
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += (double)part[v];
            __syncthreads();
        }
    } else {
        for (; sh < shn; sh += (T)SPLIT) {
            int l[3];
            T z[3];
            sample_cell(e, d, sh, top, l, z);
            const int go = (l[0] + n0 * (l[1] + n1 * l[2])) * ES;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += (double)gather_global(rf[v], go, sb1, sb2, z);
        }
    }
    // combine the SPLIT interleaved partial sums of a ray (same butterfly
    // order in every lane of the group, so they agree bit for bit)
#pragma unroll
    for (int m = 1; m < SPLIT; m <<= 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += __shfl_xor(acc[v], m, 64);
    }
    const bool writer = valid && seg == 0;
    if constexpr (MODE == FWD_DOT) {
        double vals[NV];
        const double rr = writer ? (double)p[pix] - fa * (double)y[pix] - fb : 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) vals[v] = rr * ((double)r.dt * acc[v]);
        reduce_or_defer<NV>(vals, partials, counter, out, bid, nb, 2.0);
    } else {
        double pv = 0.0;
        if (writer) {
            const T pt = (T)((double)r.dt * acc[0]);
            p[pix] = pt;
            pv = (double)pt;
        }
        if constexpr (MODE == FWD_SUMS) {
            const double yv = writer ? (double)y[pix] : 0.0;
            const double rv = writer ? pv - fit.a0 * yv - fit.b0 : 0.0;
            const double vals[3] = {rv, rv * yv, rv * rv};
            reduce_or_defer<3>(vals, partials, counter, out, bid, nb, 1.0);
        } else if constexpr (MODE == FWD_EVAL) {
            // volume 0 is f, volumes 1.. its Jacobian volumes: the objective's
            // moments and, per mode, the sums that give the gradient's
            // residual dot product at whatever fit the moments select
            const double yv = writer ? (double)y[pix] : 0.0;
            const double rv = writer ? pv - fit.a0 * yv - fit.b0 : 0.0;
            constexpr int KV = NV - 1;
            double vals[eval_sums(KV)];
            vals[0] = rv;
            vals[1] = rv * yv;
            vals[2] = rv * rv;
            vals[3] = vals[4] = vals[5] = 0.0;
#pragma unroll
            for (int v = 1; v < NV; ++v) {
                const double q = writer ? (double)r.dt * acc[v] : 0.0;
                vals[3 + 3 * v] = q * rv;
                vals[4 + 3 * v] = q * yv;
                vals[5 + 3 * v] = q;
            }
#pragma unroll
            for (int i = 0, t = 3 + 3 * NV; i < KV; ++i)
#pragma unroll
                for (int j = i; j < KV; ++j, ++t) vals[t] = vals[8 + 3 * i] * vals[8 + 3 * j];
            reduce_or_defer<eval_sums(KV)>(vals, partials, counter, out, bid, nb, 1.0);
        }
    }
}

template <typename T, int AX, int NV, int MODE, int TS>
__global__ __launch_bounds__(256) void k_drr_forward(VolDims vd, Frame fr, int tiles_u, int slab,
                                                     const RayRec<T> *__restrict__ rays,
                                                     const T *__restrict__ f, T *__restrict__ p,
                                                     const T *__restrict__ y, double fa, double fb,
                                                     FitArgs fit, double *__restrict__ partials,
                                                     uint32_t *counter, double *__restrict__ out) {
    drr_forward_block<T, AX, NV, MODE, TS>(vd, fr, tiles_u, slab, rays, f, p, y, fa, fb, fit,
                                           partials, counter, out, blockIdx.x, gridDim.x);
}

// Several requests' projections (with the fit sums) in one launch.
template <typename T, int AX>
__global__ __launch_bounds__(256) void k_drr_forward_batch(const FwdJob *__restrict__ jobs,
                                                           int njobs) {
    const int j = job_of(jobs, njobs);
    const FwdJob &J = jobs[j];
    drr_forward_block<T, AX, 1, FWD_SUMS, 0>(J.vd, J.fr, J.tiles_u, J.slab,
                                          (const RayRec<T> *)J.rays, (const T *)J.f, (T *)J.p,
                                          (const T *)J.y, 0.0, 0.0, J.fit, J.partials, J.counter,
                                          J.out, blockIdx.x - J.block0, J.nblocks);
}

// Several requests' fused-evaluation projections in one launch.
template <typename T, int AX, int K, int TS>
__global__ __launch_bounds__(256) void k_drr_forward_eval_batch(const FwdJob *__restrict__ jobs,
                                                                int njobs) {
    const int j = job_of(jobs, njobs);
    const FwdJob &J = jobs[j];
    drr_forward_block<T, AX, K + 1, FWD_EVAL, TS>(J.vd, J.fr, J.tiles_u, J.slab,
                                              (const RayRec<T> *)J.rays, (const T *)J.f,
                                              (T *)J.p, (const T *)J.y, 0.0, 0.0, J.fit,
                                              J.partials, J.counter, J.out,
                                              blockIdx.x - J.block0, J.nblocks);
}

int drr_forward_blocks(int nu, int nv, int ts) {
    const int TU = tile_u(ts), TV = tile_v(ts);
    return ((nu + TU - 1) / TU) * ((nv + TV - 1) / TV);
}

// Slab axis and thickness for a projection: the in-plane axis (x or y) the
// central ray advances fastest along in index units, and the thickest slab
// (32, 16 or 8 cells) whose staged boxes fit the LDS budget for bundles at
// the centre, edges and corners of the detector.  slab 0 means "no slabs".
static void forward_plan(const VolDims &v, const Frame &fr, int cap, int ts, int *axis,
                         int *slab) {
    const double ax = fabs(fr.en[0]) * v.inv_s[0], ay = fabs(fr.en[1]) * v.inv_s[1];
    const int AX = ay > ax ? 1 : 0;
    const int na = AX == 0 ? v.n0 : v.n1;
    const int TU = tile_u(ts), TV = tile_v(ts);
    const int tiles_u = (fr.nu + TU - 1) / TU, tiles_v = (fr.nv + TV - 1) / TV;
    *axis = AX;
    *slab = 0;
    for (int S = 32; S >= 8; S >>= 1) {
        if ((na + S - 1) / S > FWD_MAX_SLABS) break;
        bool fits = true;
        for (int gv = 0; gv < 3 && fits; ++gv)
            for (int gu = 0; gu < 3 && fits; ++gu) {
                const int tu = gu * (tiles_u - 1) / 2, tv = gv * (tiles_v - 1) / 2;
                const int iu0 = tu * TU, iu1 = std::min(iu0 + TU, fr.nu) - 1;
                const int iv0 = tv * TV, iv1 = std::min(iv0 + TV, fr.nv) - 1;
                for (int A0 = 0; A0 <= na - 2 && fits; A0 += S) {
                    int lo[2], hi[2];
                    if (!slab_cells_host(v, fr, AX, iu0, iu1, iv0, iv1, A0, S, lo, hi)) {
                        fits = false;
                        break;
                    }
                    const int eb = hi[0] - lo[0] + 2, ec = hi[1] - lo[1] + 2;
                    const long long size = AX == 0
                        ? (long long)box_pitch_x(S + 1) * eb * ec
                        : (long long)box_pitch_x(eb) * (S + 1) * ec;
                    if (size > cap) fits = false;
                }
            }
        if (fits) {
            *slab = S;
            return;
        }
    }
}

// FP32 projections of three or more volumes take tile shape 1 when its
// boxes fit slabs of some thickness (8 cells at least); otherwise, and for
// one or two volumes, shape 0.  On the clinical workload at seven angles,
// shape 1 took the four-volume projection 3-18% below shape 0, also where it
// needed thinner slabs, and the one-volume projection 15-27% above it.
ForwardPlan plan_drr_forward(pcas_dtype dt, const VolDims &v, const Frame &fr, int nvol) {
    ForwardPlan pl;
    const int es = dt == PCAS_F32 ? 4 : 8;
    const int cap = fwd_lds_bytes(nvol) / es / nvol;
    if (dt == PCAS_F32 && nvol >= 3) {
        forward_plan(v, fr, cap, 1, &pl.axis, &pl.slab);
        if (pl.slab > 0) {
            pl.tile = 1;
            return pl;
        }
    }
    forward_plan(v, fr, cap, 0, &pl.axis, &pl.slab);
    pl.tile = 0;
    return pl;
}

template <typename T, int AX, int NV, int MODE, int TS>
static void launch_fwd(const VolDims &v, const Frame &fr, int slab, const void *rays,
                       const void *f, void *p, const void *y, double a, double b,
                       const FitArgs &fit, double *partials, uint32_t *counter, double *out,
                       hipStream_t s) {
    const int tiles_u = (fr.nu + tile_u(TS) - 1) / tile_u(TS);
    const dim3 grid(drr_forward_blocks(fr.nu, fr.nv, TS));
    hipLaunchKernelGGL((k_drr_forward<T, AX, NV, MODE, TS>), grid, dim3(FWD_THREADS), 0, s, v, fr,
                       tiles_u, slab, (const RayRec<T> *)rays, (const T *)f, (T *)p,
                       (const T *)y, a, b, fit, partials, counter, out);
}

// Shape 1 is instantiated only where the plan can pick it (FP32, NV >= 3).
template <typename T, int NV>
constexpr bool has_shape1() { return sizeof(T) == 4 && NV >= 3; }

template <typename T, int NV, int MODE>
static void launch_fwd_axis(const ForwardPlan &pl, const VolDims &v, const Frame &fr,
                            const void *rays, const void *f, void *p, const void *y, double a,
                            double b, const FitArgs &fit, double *partials, uint32_t *counter,
                            double *out, hipStream_t s) {
    if constexpr (has_shape1<T, NV>()) {
        if (pl.tile == 1) {
            if (pl.axis == 0)
                launch_fwd<T, 0, NV, MODE, 1>(v, fr, pl.slab, rays, f, p, y, a, b, fit, partials,
                                              counter, out, s);
            else
                launch_fwd<T, 1, NV, MODE, 1>(v, fr, pl.slab, rays, f, p, y, a, b, fit, partials,
                                              counter, out, s);
            return;
        }
    }
    if (pl.axis == 0)
        launch_fwd<T, 0, NV, MODE, 0>(v, fr, pl.slab, rays, f, p, y, a, b, fit, partials, counter,
                                      out, s);
    else
        launch_fwd<T, 1, NV, MODE, 0>(v, fr, pl.slab, rays, f, p, y, a, b, fit, partials, counter,
                                      out, s);
}

static FitArgs no_fit() {
    FitArgs fa{FIT_NONE, 1.0, 0.0, 0.0, 0.0, 0.0};
    return fa;
}

hipError_t launch_drr_forward(pcas_dtype dt, const VolDims &v, const Frame &fr,
                              const ForwardPlan &plan, const void *rays, const void *f, void *p,
                              const void *y, const FitArgs *fit, double *partials,
                              uint32_t *counter, double *sums, hipStream_t s) {
    const FitArgs fa = fit ? *fit : no_fit();
    if (dt == PCAS_F32) {
        if (sums)
            launch_fwd_axis<float, 1, FWD_SUMS>(plan, v, fr, rays, f, p, y, 0.0, 0.0, fa, partials,
                                                counter, sums, s);
        else
            launch_fwd_axis<float, 1, FWD_WRITE>(plan, v, fr, rays, f, p, nullptr, 0.0, 0.0, fa,
                                                 nullptr, nullptr, nullptr, s);
    } else {
        if (sums)
            launch_fwd_axis<double, 1, FWD_SUMS>(plan, v, fr, rays, f, p, y, 0.0, 0.0, fa, partials,
                                                 counter, sums, s);
        else
            launch_fwd_axis<double, 1, FWD_WRITE>(plan, v, fr, rays, f, p, nullptr, 0.0, 0.0, fa,
                                                  nullptr, nullptr, nullptr, s);
    }
    return hipGetLastError();
}

FwdJob make_fwd_job(const VolDims &v, const Frame &fr, const ForwardPlan &plan, const void *rays,
                    const void *f, void *p, const void *y, const FitArgs &fit, double *partials,
                    uint32_t *counter, double *sums) {
    FwdJob J;
    J.vd = v;
    J.fr = fr;
    J.tiles_u = (fr.nu + tile_u(plan.tile) - 1) / tile_u(plan.tile);
    J.slab = plan.slab;
    J.rays = rays;
    J.f = f;
    J.p = p;
    J.y = y;
    J.fit = fit;
    J.partials = partials;
    J.counter = counter;
    J.out = sums;
    J.block0 = 0;
    J.nblocks = drr_forward_blocks(fr.nu, fr.nv, plan.tile);
    return J;
}

hipError_t launch_drr_forward_sums_batch(pcas_dtype dt, int axis, const FwdJob *jobs, int njobs,
                                         int total_blocks, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    const dim3 grid(total_blocks), block(256);
    if (dt == PCAS_F32) {
        if (axis == 0)
            hipLaunchKernelGGL((k_drr_forward_batch<float, 0>), grid, block, 0, s, jobs, njobs);
        else
            hipLaunchKernelGGL((k_drr_forward_batch<float, 1>), grid, block, 0, s, jobs, njobs);
    } else {
        if (axis == 0)
            hipLaunchKernelGGL((k_drr_forward_batch<double, 0>), grid, block, 0, s, jobs, njobs);
        else
            hipLaunchKernelGGL((k_drr_forward_batch<double, 1>), grid, block, 0, s, jobs, njobs);
    }
    return hipGetLastError();
}

template <typename T, int K, int TS>
static void eval_batch_shape(int axis, const FwdJob *jobs, int njobs, int total_blocks,
                             hipStream_t s) {
    if (axis == 0)
        hipLaunchKernelGGL((k_drr_forward_eval_batch<T, 0, K, TS>), dim3(total_blocks), dim3(256),
                           0, s, jobs, njobs);
    else
        hipLaunchKernelGGL((k_drr_forward_eval_batch<T, 1, K, TS>), dim3(total_blocks), dim3(256),
                           0, s, jobs, njobs);
}

template <typename T, int K>
static hipError_t eval_batch_axis(int axis, int tile, const FwdJob *jobs, int njobs,
                                  int total_blocks, hipStream_t s) {
    if constexpr (has_shape1<T, K + 1>()) {
        if (tile == 1) {
            eval_batch_shape<T, K, 1>(axis, jobs, njobs, total_blocks, s);
            return hipSuccess;
        }
    }
    if (tile != 0) return hipErrorInvalidValue;
    eval_batch_shape<T, K, 0>(axis, jobs, njobs, total_blocks, s);
    return hipSuccess;
}

hipError_t launch_drr_forward_eval_batch(pcas_dtype dt, int K, int axis, int tile,
                                         const FwdJob *jobs, int njobs, int total_blocks,
                                         hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
#define D(TT, KK)                                                                                  \
    case KK:                                                                                       \
        if (hipError_t e = eval_batch_axis<TT, KK>(axis, tile, jobs, njobs, total_blocks, s))     \
            return e;                                                                              \
        break
    if (dt == PCAS_F32) {
        switch (K) { D(float, 1); D(float, 2); D(float, 3); D(float, 4);
                     D(float, 5); D(float, 6); D(float, 7); D(float, 8);
                     default: return hipErrorInvalidValue; }
    } else {
        switch (K) { D(double, 1); D(double, 2); D(double, 3); D(double, 4);
                     D(double, 5); D(double, 6); D(double, 7); D(double, 8);
                     default: return hipErrorInvalidValue; }
    }
#undef D
    return hipGetLastError();
}

hipError_t launch_drr_forward_dot(pcas_dtype dt, const VolDims &v, const Frame &fr,
                                  const ForwardPlan &plan, int K, const void *rays, const void *J,
                                  const void *p, const void *y, double a, double b,
                                  double *partials, uint32_t *counter, double *g_out,
                                  hipStream_t s) {
    void *pp = const_cast<void *>(p);
    const FitArgs fa = no_fit();
#define D(TT, KK)                                                                                  \
    case KK:                                                                                       \
        launch_fwd_axis<TT, KK, FWD_DOT>(plan, v, fr, rays, J, pp, y, a, b, fa, partials, counter, \
                                         g_out, s);                                                \
        break
    if (dt == PCAS_F32) {
        switch (K) { D(float, 1); D(float, 2); D(float, 3); D(float, 4);
                     D(float, 5); D(float, 6); D(float, 7); D(float, 8);
                     default: return hipErrorInvalidValue; }
    } else {
        switch (K) { D(double, 1); D(double, 2); D(double, 3); D(double, 4);
                     D(double, 5); D(double, 6); D(double, 7); D(double, 8);
                     default: return hipErrorInvalidValue; }
    }
#undef D
    return hipGetLastError();
}

hipError_t launch_drr_forward_eval(pcas_dtype dt, const VolDims &v, const Frame &fr,
                                   const ForwardPlan &plan, int K, const void *rays,
                                   const void *vols, void *p, const void *y, const FitArgs &fit,
                                   double *partials, uint32_t *counter, double *sums,
                                   hipStream_t s) {
#define D(TT, KK)                                                                                  \
    case KK:                                                                                       \
        launch_fwd_axis<TT, KK + 1, FWD_EVAL>(plan, v, fr, rays, vols, p, y, 0.0, 0.0, fit,        \
                                              partials, counter, sums, s);                         \
        break
    if (dt == PCAS_F32) {
        switch (K) { D(float, 1); D(float, 2); D(float, 3); D(float, 4);
                     D(float, 5); D(float, 6); D(float, 7); D(float, 8);
                     default: return hipErrorInvalidValue; }
    } else {
        switch (K) { D(double, 1); D(double, 2); D(double, 3); D(double, 4);
                     D(double, 5); D(double, 6); D(double, 7); D(double, 8);
                     default: return hipErrorInvalidValue; }
    }
#undef D
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bounds on the trilinear weights one voxel receives (they size the
// back-projection's fixed-point accumulators).

// A ray with n >= 2 samples has dt >= step / 2, and its largest per-sample
// index step is >= dt / (sqrt(3) max spacing); the tent weights one ray
// gives a voxel then sum to at most 1/h + 1.  (A ray with one sample gives
// at most 1.)
__host__ __device__ inline double ray_weight_bound(const VolDims &v, const Frame &fr) {
    const double smax = fmax(v.spacing[0], fmax(v.spacing[1], v.spacing[2]));
    return 2.0 * sqrt(3.0) * smax / fr.step + 2.0;
}

// Bound on the summed trilinear weight all rays give one voxel whose support
// cube (index half-width 1) lies in the index box [b0, b1] (and, as every
// sample does, in the grid box): (P^T 1)(v) <= step * bound.
//
// One ray: its samples advance by h_a = dt |dir_a| / s_a per sample along
// index axis a, and a tent of half-width 1 sampled at spacing h sums to at
// most 1/h + 1 (a Riemann sum of its unit integral, off by at most h times
// its peak), so the ray gives the voxel at most dt (1/h_a + 1) =
// s_a / |dir_a| + dt <= s_a / |dir_a| + step.  Over the rays through the box
// |dir_a| >= min|rel_a| / max|rel| (rel = point - source) on any axis where
// rel_a keeps one sign; some axis always has |dir_a| >= 1/sqrt(3), which
// gives sqrt(3) max s + step for any ray.
//
// The rays: detector coordinates u = SID (rel.eu) / D with depth D = rel.en.
// Over the voxel's cube rel.eu varies by at most W_u = sum_c 2 s_c |eu_c|
// and D by at most W_n = sum_c 2 s_c |en_c|, so u varies by at most
// (SID / D_min)(W_u + A_u W_n / D_min), A_u the largest |rel.eu| over the
// box (D_min and A_u sit at box corners: both are linear in the point); an
// interval of that length holds at most floor(length / pitch_u) + 1 pixel
// centres, and likewise along v.
//
// *adds (if not null) bounds the samples that reach the voxel: per ray at
// most floor(diam / (step / 2)) + 1 lie in the cube (a ray of two or more
// samples has dt >= step / 2; diam = 2 sqrt(sum s_c^2)).  Infinite when the
// box reaches the source's plane.
__host__ __device__ inline double region_weight_bound(const VolDims &v, const Frame &fr,
                                                      const int (&b0)[3], const int (&b1)[3],
                                                      double *adds) {
    double dmin = INFINITY, au = 0.0, av = 0.0, rmax = 0.0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int corner = 0; corner < 8; ++corner) {
        double rel[3], depth = 0.0, pu = 0.0, pv = 0.0, r2 = 0.0;
        for (int c = 0; c < 3; ++c)
            rel[c] = v.origin[c] + (((corner >> c) & 1) ? b1[c] : b0[c]) * v.spacing[c] - fr.src[c];
        for (int c = 0; c < 3; ++c) {
            depth += rel[c] * fr.en[c];
            pu += rel[c] * fr.eu[c];
            pv += rel[c] * fr.ev[c];
            r2 += rel[c] * rel[c];
            lo[c] = fmin(lo[c], rel[c]);
            hi[c] = fmax(hi[c], rel[c]);
        }
        dmin = fmin(dmin, depth);
        au = fmax(au, fabs(pu));
        av = fmax(av, fabs(pv));
        rmax = fmax(rmax, sqrt(r2));
    }
    if (!(dmin > 0.0)) {
        if (adds) *adds = INFINITY;
        return INFINITY;
    }
    const double smax = fmax(v.spacing[0], fmax(v.spacing[1], v.spacing[2]));
    double ray = sqrt(3.0) * smax + fr.step;
    for (int a = 0; a < 3; ++a) {
        const double m = lo[a] > 0.0 ? lo[a] : (hi[a] < 0.0 ? -hi[a] : 0.0);
        if (m > 0.0) ray = fmin(ray, v.spacing[a] * rmax / m + fr.step);
    }
    double wu = 0.0, wv = 0.0, wn = 0.0, diam = 0.0;
    for (int c = 0; c < 3; ++c) {
        wu += 2.0 * v.spacing[c] * fabs(fr.eu[c]);
        wv += 2.0 * v.spacing[c] * fabs(fr.ev[c]);
        wn += 2.0 * v.spacing[c] * fabs(fr.en[c]);
        diam += v.spacing[c] * v.spacing[c];
    }
    diam = 2.0 * sqrt(diam);
    const double lu = fr.sid / dmin * (wu + au * wn / dmin), lv = fr.sid / dmin * (wv + av * wn / dmin);
    const double nu = fmin(floor(lu / fr.pitch_u) + 1.0, (double)fr.nu);
    const double nv = fmin(floor(lv / fr.pitch_v) + 1.0, (double)fr.nv);
    if (adds) *adds = nu * nv * (floor(2.0 * diam / fr.step) + 1.0);
    return ray / fr.step * nu * nv;
}

// The bound over one back-projection brick: every voxel of its halo box
// [lo - 1, hi + 1], whose support cubes lie in [lo - 2, hi + 2] (clipped).
__host__ __device__ inline double brick_weight_bound(const VolDims &v, const Frame &fr, int brick,
                                                     double *adds) {
    const int nbx = (v.n0 + BRICK_X - 1) / BRICK_X, nby = (v.n1 + BRICK_Y - 1) / BRICK_Y;
    const int bx = brick % nbx, by = (brick / nbx) % nby, bz = brick / (nbx * nby);
    const int lo[3] = {bx * BRICK_X, by * BRICK_Y, bz * BRICK_Z};
    const int n[3] = {v.n0, v.n1, v.n2};
    const int ext[3] = {BRICK_X, BRICK_Y, BRICK_Z};
    int r0[3], r1[3];
    for (int c = 0; c < 3; ++c) {
        const int h = (lo[c] + ext[c] < n[c] ? lo[c] + ext[c] : n[c]) - 1;
        r0[c] = lo[c] - 2 > 0 ? lo[c] - 2 : 0;
        r1[c] = h + 2 < n[c] - 1 ? h + 2 : n[c] - 1;
    }
    return region_weight_bound(v, fr, r0, r1, adds);
}

double brick_weight_bound_host(const VolDims &v, const Frame &fr, int brick) {
    return brick_weight_bound(v, fr, brick, nullptr);
}

// The same over the whole grid: (P^T 1)(v) <= step * bound for every voxel.
double backprojection_weight_bound(const VolDims &v, const Frame &fr) {
    const int b0[3] = {0, 0, 0}, b1[3] = {v.n0 - 1, v.n1 - 1, v.n2 - 1};
    return region_weight_bound(v, fr, b0, b1, nullptr);
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
// at write-out.  The slice pitch, one word more than the (BRICK_Y + 2) x
// (BRICK_X + 2) slice, spreads z-neighbours over banks.
constexpr int ACC_YP = BRICK_X + 2;
constexpr int ACC_ZP = (BRICK_Y + 2) * ACC_YP + 1;
constexpr int ACC_WORDS = (BRICK_Z + 2) * ACC_ZP;
// Ring queue of rays per wave (a power of two, at least one 64-ray tile).
// 64 rather than 128 entries: the queues are most of a block's LDS, and
// the smaller ones let 7 instead of 5 blocks share a CU (the fused gradient
// kernel measured 428 against 460 us).
#ifndef PCAS_ADJ_QCAP
#define PCAS_ADJ_QCAP 64
#endif
#ifndef PCAS_ADJ_RUN
#define PCAS_ADJ_RUN 8
#endif
constexpr int QCAP = PCAS_ADJ_QCAP;
constexpr int ADJ_RUN = PCAS_ADJ_RUN;   // samples per lane between queue refills

// Fixed-point image of one already-scaled contribution v as a 64-bit two's
// complement integer.  float: |v| <= 2^30, truncated toward zero and
// sign-extended (one unit is at most 2^-30 of the largest contribution, far
// below the float product's own rounding); double: |v| <= 2^50, rounded to
// nearest by reading the mantissa of v + 1.5 * 2^52.
__device__ __forceinline__ unsigned long long fixed_of(float v) {
    return (unsigned long long)(long long)(int)v;
}
__device__ __forceinline__ unsigned long long fixed_of(double v) {
    const double m = v + 6755399441055744.0;
    return __builtin_bit_cast(unsigned long long, m) - 0x4338000000000000ull;
}
// 32-bit image of an already-scaled float contribution, |v| < 2^31, rounded to
// nearest (the accumulator of the solver's FP32 gradient, whose scale comes
// from the measured per-brick bound).  A voxel near the source takes ~10^4
// adds at ~20 bits each; truncation's bias (half a unit per add, one sign
// where the residual is smooth) would add up with the count, rounding's
// errors only with its square root.  v_cvt_rpi_i32_f32 gives floor(v + 0.5)
// in one instruction (ties go up; on gfx950 it matched the exact value for
// 4M floats from 2^-2 to 2^30, ties included), against a round and a
// convert: this conversion runs eight times per sample.
__device__ __forceinline__ unsigned int fixed32_of(float v) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return (unsigned int)r;
}
__device__ __forceinline__ long long acc_value(unsigned int a) { return (long long)(int)a; }
__device__ __forceinline__ long long acc_value(unsigned long long a) { return (long long)a; }
template <bool A32, typename V>
__device__ __forceinline__ auto acc_image(V v) {
    if constexpr (A32)
        return fixed32_of(v);
    else
        return fixed_of(v);
}
template <typename T> struct FixedRange;
template <> struct FixedRange<float> { static constexpr double per_add = 1073741824.0; };       // 2^30
template <> struct FixedRange<double> { static constexpr double per_add = 1125899906842624.0; };  // 2^50

// Samples of ray r whose 2x2x2 cell may touch the brick [lo, hi]: the
// parameter range where every coordinate lies in [lo - 1, hi + 1], widened
// by one sample each side to absorb rounding in this estimate (the cell
// test in the sample loop is exact).
__device__ __forceinline__ float rcp_approx(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_approx(double x) { return 1.0 / x; }

template <typename T>
__device__ __forceinline__ bool brick_sample_range(const RayRec<T> &r, const T (&lob)[3],
                                                   const T (&hib)[3], int *s0, int *s1) {
    T s_lo = (T)0, s_hi = (T)(r.n - 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (r.d[c] != (T)0) {
            const T inv = rcp_approx(r.d[c]);
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

template <typename T, bool FORM_R>
__device__ __forceinline__ T residual_at(const T *__restrict__ rp, const T *__restrict__ y, double a,
                                         double b, int pix) {
    if constexpr (FORM_R)
        return (T)((double)rp[pix] - a * (double)y[pix] - b);
    else
        return rp ? rp[pix] : (T)1;   // no residual: the all-ones image
}

// Whether sample s of a ray has its cell (lower corner) in the halo box
// [lom, lom + ext) -- the same sample_cell arithmetic as the sample loop.
template <typename T>
__device__ __forceinline__ bool sample_in_box(const T (&e)[3], const T (&d)[3], int s,
                                              const GridTop<T> &top, const int (&lom)[3],
                                              const int (&ext)[3]) {
    int l[3];
    T z[3];
    sample_cell(e, d, (T)s + (T)0.5, top, l, z);
    return (unsigned)(l[0] - lom[0]) < (unsigned)ext[0] &&
           (unsigned)(l[1] - lom[1]) < (unsigned)ext[1] &&
           (unsigned)(l[2] - lom[2]) < (unsigned)ext[2];
}

// Slot of global cell l in a brick's halo array whose origin cell sits at
// word `base` of the global layout: l2 ZP + l1 YP + l0 - base.  Two
// v_mad_u32_u24 (full rate; cell indices are below 2^24), written out
// because the compiler otherwise folds `base` into the products and falls
// back to quarter-rate 32-bit multiplies.
__device__ __forceinline__ unsigned halo_slot(const int (&l)[3], unsigned base) {
    unsigned t, u;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(t) : "v"(l[1]), "s"(ACC_YP), "v"((unsigned)l[0] - base));
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(u) : "v"(l[2]), "s"(ACC_ZP), "v"(t));
    return u;
}

// Accumulator modes of drr_adjoint_block.
enum {
    ADJ_ACC64 = 0,        // 64-bit fixed point (drr_adjoint; FP64 gradients)
    ADJ_ACC32 = 1         // FP32: 32-bit fixed point (drr_adjoint32 and the fused gradient)
};

// hb bounds the summed weight one ray can give one voxel (samples within the
// voxel's cube of index half-width 1, each of weight at most 1).
//
// Work distribution: the rays of the brick's detector footprint with
// samples in the brick's halo box go into a per-wave ring queue (geometry,
// exact sample range and scaled dt * r); every lane takes a ray, walks
// ADJ_RUN samples, and lanes whose ray is done take the next queued one, so
// lanes stay busy whatever the spread of ray lengths.  A ray's range is
// first estimated from the box in continuous coordinates, then trimmed at
// both ends by re-creating the end samples' cells: along a ray every cell
// coordinate is monotone in the sample index, so the samples whose cell lies
// in the box form one interval, and the trimmed range is exactly that
// interval.  The sample loop therefore adds every sample it visits, with no
// per-sample test.  Each sample adds its eight corner weights to the LDS
// accumulator in fixed point (per-brick power-of-two scale).  Integer
// addition is associative, so the brick's sums do not depend on which lane
// adds when.
//
// Scale: every contribution is |dt r w| <= step * rmax = C (rmax the largest
// |r| of the footprint), and every voxel total of the brick, halo slots
// included, is at most C min(hb * footprint pixels, vb) with vb the
// brick's weight bound (brick_weight_bound).  ADJ_ACC64: contributions <= FixedRange, totals
// < 2^62.  ADJ_ACC32: contributions are rounded to
// nearest (errors grow with the square root of the add count instead of
// its count), and totals plus half a unit per add (at most `adds` of them)
// stay below 2^31.
//
// K = 0: bp is written.  K > 0 (the solver's
// gradient): bp never leaves the chip; each brick voxel's value is chained
// at once through the warp Jacobian (Eq. A.8 and the modes, as grad_w does)
// and the block sums of bp * sum_c U_kc df/dx_c go through the fixed-order
// grid reduction into g_out[k] (times 2).
template <typename T, bool FORM_R, int K, int ACCM>
__device__ __forceinline__ void drr_adjoint_block(const VolDims &vd, const Frame &fr, int nbx,
                                                  int nby, double hb,
                                                  const RayRec<T> *__restrict__ rays,
                                                  const T *__restrict__ rp,
                                                  const T *__restrict__ y, double a, double b,
                                                  T *__restrict__ bp, const T *__restrict__ f0,
                                                  const T *__restrict__ mean,
                                                  const T *__restrict__ U, const WVec &w,
                                                  double *__restrict__ partials,
                                                  uint32_t *counter, double *__restrict__ g_out,
                                                  int lb, int nb, int split) {
    constexpr bool ACC32 = std::is_same<T, float>::value && ACCM != ADJ_ACC64;
    using AccT = typename std::conditional<ACC32, unsigned int, unsigned long long>::type;
    __shared__ AccT acc[ACC_WORDS];
    __shared__ T q_f[ADJ_WAVES][7][QCAP];       // e[3], d[3], scaled dt * r
    __shared__ int q_s[ADJ_WAVES][2][QCAP];     // first and last sample
    __shared__ double red[ADJ_WAVES];
    const int n0 = vd.n0, n1 = vd.n1, n2 = vd.n2;
    // Bricks go round-robin over the XCDs in launch order: only bricks inside
    // the x-ray cone carry work, so contiguous per-XCD ranges would leave the
    // XCDs that hold the outer z-slabs idle.  With K > 0, `split` blocks may
    // share one brick's footprint rays (block lb: brick lb % bricks, part
    // lb / bricks): each part chains its own partial sums, and the chain being
    // linear in P^T r, the parts meet in the block reduction.
    const int nbricks = nb / split, bid = lb % nbricks, part = lb / nbricks;
    const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
    const int lo[3] = {bx * BRICK_X, by * BRICK_Y, bz * BRICK_Z};
    const int hi[3] = {min(lo[0] + BRICK_X, n0) - 1, min(lo[1] + BRICK_Y, n1) - 1,
                       min(lo[2] + BRICK_Z, n2) - 1};
    const int nn[3] = {n0, n1, n2};
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int t = tid; t < ACC_WORDS; t += ADJ_THREADS) acc[t] = 0;

    // Detector footprint of the region whose samples can reach the brick:
    // index box [lo - 1, hi + 1] clipped to the grid, projected through its
    // eight corners (the source is outside the volume, so every depth > 0).
    // Every wave computes it (identically).
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
    const int npix = (W > 0 && H > 0) ? W * H : 0;

    // Per-brick fixed-point scale S (a power of two, so scaling dt * r by it
    // is exact) from the largest |r| in the footprint and the brick's weight
    // bound.
    double rmax = 0.0;
    for (int t = tid; t < npix; t += ADJ_THREADS) {
        const int pix = (iv0 + t / W) * fr.nu + (iu0 + t % W);
        rmax = fmax(rmax, fabs((double)residual_at<T, FORM_R>(rp, y, a, b, pix)));
    }
    rmax = wave_max(rmax);
    if (lane == 0) red[wave] = rmax;
    __syncthreads();
    for (int q = 0; q < ADJ_WAVES; ++q) rmax = fmax(rmax, red[q]);
    const double C = fr.step * rmax * (1.0 + 1e-6);   // 1e-6: the products' rounding in T
    double adds;
    const double vb = brick_weight_bound(vd, fr, bid, &adds);
    const double bw = fmin(hb * (double)npix, vb);
    double Sd = 0.0;
    if (C > 0.0 && bw < INFINITY) {
        double lim;
        if constexpr (ACC32) {
            // totals <= C bw; at most `adds` adds per voxel, each off by <= 1/2
            // unit (the floor assumes fewer than 2^31 samples reach one voxel)
            lim = fmax(2147483647.0 - 0.5 * adds - 1.0, 1073741824.0) / (C * bw);
        } else {
            lim = fmin(FixedRange<T>::per_add / C, 4611686018427387904.0 / (C * bw));   // 2^62
        }
        int ex;
        frexp(fmin(lim, 1e300), &ex);
        Sd = ldexp(0.5, ex);   // the largest power of two not above the limit
    }

    const GridTop<T> top = grid_top<T>(n0, n1, n2);
    const T lob[3] = {(T)(lo[0] - 1), (T)(lo[1] - 1), (T)(lo[2] - 1)};
    const T hib[3] = {(T)(hi[0] + 1), (T)(hi[1] + 1), (T)(hi[2] + 1)};
    const int ext[3] = {hi[0] - lo[0] + 2, hi[1] - lo[1] + 2, hi[2] - lo[2] + 2};
    const int lom[3] = {lo[0] - 1, lo[1] - 1, lo[2] - 1};   // halo origin
    // Word offset of the global cell (0, 0, 0) in the halo array, so that a
    // cell's slot is l2 ZP + l1 YP + l0 - base (unsigned arithmetic; every
    // visited cell lies in the box).
    const unsigned base = (unsigned)(lom[2] * ACC_ZP + lom[1] * ACC_YP + lom[0]);
    // Candidate tiles interleave the footprint: lane (lu, lv) of tile (bu,
    // bv) takes pixel (iu0 + lu*Su + bu, iv0 + lv*Sv + bv), so the rays of one
    // tile sit Su x Sv pixels apart; tiles go round-robin to the waves.
    const int Su = W > 0 ? (W + 7) / 8 : 0;
    const int Sv = H > 0 ? (H + 7) / 8 : 0;
    const int ntiles = (Sd > 0.0 && npix > 0) ? Su * Sv : 0;
    T(*qf)[QCAP] = q_f[wave];
    int(*qs)[QCAP] = q_s[wave];
    const uint64_t lt = (1ull << lane) - 1ull;
    int head = 0, tail = 0;   // wave-uniform ring positions
    int tile = part * ADJ_WAVES + wave;
    bool busy = false;
    T e[3] = {0, 0, 0}, d[3] = {0, 0, 0}, cst = (T)0, sh = (T)0, sh_end = (T)0;
    __syncthreads();   // accumulator cleared
    for (;;) {
        // top up the queue while a whole tile of candidates fits
        while (tile < ntiles && tail - head <= QCAP - 64) {
            const int iu = iu0 + (lane & 7) * Su + tile % Su;
            const int iv = iv0 + (lane >> 3) * Sv + tile / Su;
            bool active = false;
            int s0 = 0, s1 = -1;
            T c = (T)0;
            RayRec<T> r;
            if (iu <= iu1 && iv <= iv1) {
                const int pix = iv * fr.nu + iu;
                r = rays[pix];
                if (r.n > 0) {
                    c = (T)((double)r.dt * (double)residual_at<T, FORM_R>(rp, y, a, b, pix) * Sd);
                    active = c != (T)0 && brick_sample_range(r, lob, hib, &s0, &s1);
                }
            }
            if (active) {
                // trim the estimate to the samples whose cell lies in the box
                while (s0 <= s1 && !sample_in_box(r.e, r.d, s0, top, lom, ext)) ++s0;
                while (s1 > s0 && !sample_in_box(r.e, r.d, s1, top, lom, ext)) --s1;
                active = s0 <= s1;
            }
            const uint64_t mask = __ballot(active);
            if (active) {
                const int q = (tail + __popcll(mask & lt)) & (QCAP - 1);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    qf[k][q] = r.e[k];
                    qf[3 + k][q] = r.d[k];
                }
                qf[6][q] = c;
                qs[0][q] = s0;
                qs[1][q] = s1;
            }
            tail += __popcll(mask);
            tile += ADJ_WAVES * split;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // idle lanes take queued rays in lane order
        const uint64_t idle = __ballot(!busy);
        const int avail = tail - head;
        if (!busy) {
            const int rank = __popcll(idle & lt);
            if (rank < avail) {
                const int q = (head + rank) & (QCAP - 1);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    e[k] = qf[k][q];
                    d[k] = qf[3 + k][q];
                }
                cst = qf[6][q];
                sh = (T)qs[0][q] + (T)0.5;
                sh_end = (T)qs[1][q] + (T)0.5;
                busy = true;
            }
        }
        head += min(__popcll(idle), avail);
        // Wait for the refill's LDS reads here, once per run: otherwise every
        // sample of the run below waits for all LDS operations in flight (the
        // previous sample's eight adds included), because along the path where
        // a lane had no sample the reads would still be outstanding.
        __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt and expcnt unconstrained
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (__ballot(busy) == 0ull) {
            if (tile >= ntiles) break;   // queue empty (idle lanes took all) and no tiles left
            continue;
        }
        for (int it = 0; it < ADJ_RUN; ++it) {
            if (busy) {
                int l[3];
                T z[3];
                sample_cell(e, d, sh, top, l, z);
                AccT *pa = acc + halo_slot(l, base);
                // corner weights: yz pairs, then each split along x, the
                // upper share first and the lower one as the difference
                const T c1b = cst * z[1], c1a = cst - c1b;
                const T w01 = c1a * z[2], w00 = c1a - w01;
                const T w11 = c1b * z[2], w10 = c1b - w11;
                const T w00b = w00 * z[0], w10b = w10 * z[0], w01b = w01 * z[0], w11b = w11 * z[0];
                atomicAdd(pa, acc_image<ACC32>(w00 - w00b));
                atomicAdd(pa + 1, acc_image<ACC32>(w00b));
                atomicAdd(pa + ACC_YP, acc_image<ACC32>(w10 - w10b));
                atomicAdd(pa + ACC_YP + 1, acc_image<ACC32>(w10b));
                atomicAdd(pa + ACC_ZP, acc_image<ACC32>(w01 - w01b));
                atomicAdd(pa + ACC_ZP + 1, acc_image<ACC32>(w01b));
                atomicAdd(pa + ACC_ZP + ACC_YP, acc_image<ACC32>(w11 - w11b));
                atomicAdd(pa + ACC_ZP + ACC_YP + 1, acc_image<ACC32>(w11b));
                sh += (T)1;
                busy = sh <= sh_end;
            }
        }
    }
    __syncthreads();
    const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
    const double inv_S = Sd > 0.0 ? 1.0 / Sd : 0.0;
    if constexpr (K == 0) {
        for (int t = tid; t < BRICK_X * BRICK_Y * BRICK_Z; t += ADJ_THREADS) {
            const int li = t % BRICK_X, lj = (t / BRICK_X) % BRICK_Y, lk = t / (BRICK_X * BRICK_Y);
            const int i = lo[0] + li, j = lo[1] + lj, k = lo[2] + lk;
            if (i < n0 && j < n1 && k < n2) {
                const long long v = acc_value(acc[(lk + 1) * ACC_ZP + (lj + 1) * ACC_YP + (li + 1)]);
                bp[i + s1 * j + s2 * k] = (T)((double)v * inv_S);
            }
        }
    } else {
        const int64_t N = (int64_t)n0 * n1 * n2;
        T wk[K];
#pragma unroll
        for (int kk = 0; kk < K; ++kk) wk[kk] = (T)w.w[kk];
        const T is0 = (T)vd.inv_s[0], is1 = (T)vd.inv_s[1], is2 = (T)vd.inv_s[2];
        double gacc[K];
#pragma unroll
        for (int kk = 0; kk < K; ++kk) gacc[kk] = 0.0;
        if (Sd > 0.0) {
            for (int t = tid; t < BRICK_X * BRICK_Y * BRICK_Z; t += ADJ_THREADS) {
                const int li = t % BRICK_X, lj = (t / BRICK_X) % BRICK_Y, lk = t / (BRICK_X * BRICK_Y);
                const int i = lo[0] + li, j = lo[1] + lj, k = lo[2] + lk;
                if (i >= n0 || j >= n1 || k >= n2) continue;
                const long long v = acc_value(acc[(lk + 1) * ACC_ZP + (lj + 1) * ACC_YP + (li + 1)]);
                const T bpv = (T)((double)v * inv_S);
                if (bpv == (T)0) continue;
                const int64_t vox = i + s1 * j + s2 * k;
                T u[K][3], x[3], jac[3];
                voxel_field<T, K, false>(mean, U, wk, N, vox, u, x);
                if (!voxel_jacobian(f0, n0, n1, n2, i, j, k, x, is0, is1, is2, jac)) continue;
                const T j0 = jac[0] * bpv, j1 = jac[1] * bpv, j2 = jac[2] * bpv;
#pragma unroll
                for (int kk = 0; kk < K; ++kk)
                    gacc[kk] += (double)fma_t(u[kk][0], j0, fma_t(u[kk][1], j1, u[kk][2] * j2));
            }
        }
        reduce_or_defer<K>(gacc, partials, counter, g_out, lb, nb, 2.0);
    }
}

template <typename T, bool FORM_R, int K, int ACCM>
__global__ __launch_bounds__(ADJ_THREADS) void k_drr_adjoint(VolDims vd, Frame fr, int nbx, int nby,
                                                     double hb,
                                                     const RayRec<T> *__restrict__ rays,
                                                     const T *__restrict__ rp,
                                                     const T *__restrict__ y, double a, double b,
                                                     T *__restrict__ bp, const T *__restrict__ f0,
                                                     const T *__restrict__ mean,
                                                     const T *__restrict__ U, WVec w,
                                                     double *__restrict__ partials,
                                                     uint32_t *counter, double *__restrict__ g_out,
                                                     const double *__restrict__ gate, int split) {
    if (gate) {   // a speculative gradient: (a, b, go) from the device's decision
        if (gate[2] == 0.0) return;
        a = gate[0];
        b = gate[1];
    }
    drr_adjoint_block<T, FORM_R, K, ACCM>(vd, fr, nbx, nby, hb, rays, rp, y, a, b, bp, f0,
                                          mean, U, w, partials, counter, g_out, blockIdx.x,
                                          gridDim.x, split);
}

// Several requests' gradients (back-projection + chain) in one launch.
template <typename T, int K>
__global__ __launch_bounds__(ADJ_THREADS) void k_drr_adjoint_batch(const AdjJob *__restrict__ jobs,
                                                           int njobs) {
    const int j = job_of(jobs, njobs);
    const AdjJob &J = jobs[j];
    constexpr int ACCM = std::is_same<T, float>::value ? ADJ_ACC32 : ADJ_ACC64;
    double a = J.a, b = J.b;
    if (J.gate) {   // a speculative gradient: (a, b, go) from the request's gate
        if (J.gate[2] == 0.0) return;
        a = J.gate[0];
        b = J.gate[1];
    }
    drr_adjoint_block<T, true, K, ACCM>(J.vd, J.fr, J.nbx, J.nby, J.hb,
                                        (const RayRec<T> *)J.rays, (const T *)J.p,
                                        (const T *)J.y, a, b, (T *)nullptr, (const T *)J.f0,
                                        (const T *)J.mean, (const T *)J.U, J.w, J.partials,
                                        J.counter, J.g_out, blockIdx.x - J.block0, J.nblocks,
                                        J.split);
}

int drr_adjoint_blocks(const VolDims &v) {
    return ((v.n0 + BRICK_X - 1) / BRICK_X) * ((v.n1 + BRICK_Y - 1) / BRICK_Y) *
           ((v.n2 + BRICK_Z - 1) / BRICK_Z);
}

// Liveness of the bricks for one projection: the brick's box with its
// one-voxel halo (which holds every sample whose cell touches a voxel of the
// brick), clipped to the grid and projected through its eight corners, in
// detector pixel coordinates as the back-projection's footprint.  The image
// of a box in front of the source lies in the convex hull of its corners'
// images, so a box whose corner images all fall more than a pixel off the
// detector meets no ray; a corner at or behind the source's plane keeps the
// brick live.
__host__ __device__ inline bool brick_live(const VolDims &vd, const Frame &fr, int bid) {
    const int nbx = (vd.n0 + BRICK_X - 1) / BRICK_X, nby = (vd.n1 + BRICK_Y - 1) / BRICK_Y;
    const int b[3] = {bid % nbx, (bid / nbx) % nby, bid / (nbx * nby)};
    const int ext[3] = {BRICK_X, BRICK_Y, BRICK_Z}, n[3] = {vd.n0, vd.n1, vd.n2};
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    bool behind = false;
    for (int corner = 0; corner < 8; ++corner) {
        double rel[3];
        for (int c = 0; c < 3; ++c) {
            const int lo = b[c] * ext[c];
            const int hi = (lo + ext[c] < n[c] ? lo + ext[c] : n[c]) - 1;
            const int idx = ((corner >> c) & 1) ? (hi + 1 < n[c] - 1 ? hi + 1 : n[c] - 1)
                                                : (lo - 1 > 0 ? lo - 1 : 0);
            rel[c] = vd.origin[c] + idx * vd.spacing[c] - fr.src[c];
        }
        const double depth = rel[0] * fr.en[0] + rel[1] * fr.en[1] + rel[2] * fr.en[2];
        if (!(depth > 0.0)) {
            behind = true;
            continue;
        }
        const double pu = (rel[0] * fr.eu[0] + rel[1] * fr.eu[1] + rel[2] * fr.eu[2]) * fr.sid / depth;
        const double pv = (rel[0] * fr.ev[0] + rel[1] * fr.ev[1] + rel[2] * fr.ev[2]) * fr.sid / depth;
        const double u = (pu - fr.offset_u) / fr.pitch_u + 0.5 * (fr.nu - 1);
        const double v = (pv - fr.offset_v) / fr.pitch_v + 0.5 * (fr.nv - 1);
        umin = fmin(umin, u);
        umax = fmax(umax, u);
        vmin = fmin(vmin, v);
        vmax = fmax(vmax, v);
    }
    const bool hit = umax >= -1.0 && umin <= (double)fr.nu && vmax >= -1.0 && vmin <= (double)fr.nv;
    return behind || hit;
}

__global__ __launch_bounds__(256) void k_brick_live(VolDims vd, Frame fr, uint8_t *__restrict__ live) {
    const int bid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = ((vd.n0 + BRICK_X - 1) / BRICK_X) * ((vd.n1 + BRICK_Y - 1) / BRICK_Y) *
                   ((vd.n2 + BRICK_Z - 1) / BRICK_Z);
    if (bid >= nb) return;
    live[bid] = brick_live(vd, fr, bid) ? 1 : 0;
}

int64_t live_voxels(const VolDims &v, const Frame &fr) {
    const int nbx = (v.n0 + BRICK_X - 1) / BRICK_X, nby = (v.n1 + BRICK_Y - 1) / BRICK_Y;
    int64_t n = 0;
    for (int bid = 0; bid < drr_adjoint_blocks(v); ++bid) {
        if (!brick_live(v, fr, bid)) continue;
        const int lo[3] = {bid % nbx * BRICK_X, bid / nbx % nby * BRICK_Y, bid / (nbx * nby) * BRICK_Z};
        n += (int64_t)(min(lo[0] + BRICK_X, v.n0) - lo[0]) * (min(lo[1] + BRICK_Y, v.n1) - lo[1]) *
             (min(lo[2] + BRICK_Z, v.n2) - lo[2]);
    }
    return n;
}

hipError_t launch_brick_live(const VolDims &v, const Frame &fr, uint8_t *live, hipStream_t s) {
    const int nb = drr_adjoint_blocks(v);
    hipLaunchKernelGGL(k_brick_live, dim3((nb + 255) / 256), dim3(256), 0, s, v, fr, live);
    return hipGetLastError();
}

// Blocks per brick of the fused gradient: enough to give the chip two
// blocks per CU on small grids (64^3 has 64 bricks), 1 from 512 bricks up.
int adjoint_chain_split(const VolDims &v) {
    const int nb = drr_adjoint_blocks(v);
    int split = 1;
    while (split < 8 && nb * split < 512) split *= 2;
    return split;
}

int drr_adjoint_chain_blocks(const VolDims &v) { return drr_adjoint_blocks(v) * adjoint_chain_split(v); }

template <typename T, bool FORM_R, int K, int ACCM>
static void launch_adj(const VolDims &v, const Frame &fr, const void *rays, const void *r_or_p,
                       const void *y, double a, double b, void *bp, const void *f0,
                       const void *mean, const void *U, const WVec &w, double *partials,
                       uint32_t *counter, double *g_out, hipStream_t s,
                       const double *gate = nullptr) {
    const int split = K > 0 ? adjoint_chain_split(v) : 1;   // bp is written whole: one block per brick
    const int nbx = (v.n0 + BRICK_X - 1) / BRICK_X;
    const int nby = (v.n1 + BRICK_Y - 1) / BRICK_Y;
    hipLaunchKernelGGL((k_drr_adjoint<T, FORM_R, K, ACCM>), dim3(drr_adjoint_blocks(v) * split),
                       dim3(ADJ_THREADS), 0, s, v, fr, nbx, nby, ray_weight_bound(v, fr),
                       (const RayRec<T> *)rays, (const T *)r_or_p, (const T *)y, a, b, (T *)bp,
                       (const T *)f0, (const T *)mean, (const T *)U, w, partials, counter, g_out,
                       gate, split);
}

template <typename T, int ACCM>
static void launch_adj_bp(const VolDims &v, const Frame &fr, const void *rays, const void *r_or_p,
                          const void *y, double a, double b, void *bp, hipStream_t s) {
    const WVec w{};
    if (y)
        launch_adj<T, true, 0, ACCM>(v, fr, rays, r_or_p, y, a, b, bp, nullptr, nullptr, nullptr, w,
                                     nullptr, nullptr, nullptr, s);
    else
        launch_adj<T, false, 0, ACCM>(v, fr, rays, r_or_p, nullptr, 0.0, 0.0, bp, nullptr, nullptr,
                                      nullptr, w, nullptr, nullptr, nullptr, s);
}

hipError_t launch_drr_adjoint(pcas_dtype dt, const VolDims &v, const Frame &fr, const void *rays,
                              const void *r_or_p, const void *y, double a, double b, void *bp,
                              bool acc32, hipStream_t s) {
    if (dt == PCAS_F32) {
        if (acc32)
            launch_adj_bp<float, ADJ_ACC32>(v, fr, rays, r_or_p, y, a, b, bp, s);
        else
            launch_adj_bp<float, ADJ_ACC64>(v, fr, rays, r_or_p, y, a, b, bp, s);
    } else {
        if (acc32) return hipErrorInvalidValue;
        launch_adj_bp<double, ADJ_ACC64>(v, fr, rays, r_or_p, y, a, b, bp, s);
    }
    return hipGetLastError();
}

hipError_t launch_drr_adjoint_chain(pcas_dtype dt, const VolDims &v, const Frame &fr, int K,
                                    const void *rays, const void *p, const void *y, double a,
                                    double b, const void *f0, const void *mean, const void *U,
                                    const double *w, double *partials, uint32_t *counter,
                                    double *g_out, hipStream_t s, const double *gate) {
    WVec wv{};
    for (int k = 0; k < K; ++k) wv.w[k] = w[k];
#define A(TT, KK, MM)                                                                             \
    case KK:                                                                                      \
        launch_adj<TT, true, KK, MM>(v, fr, rays, p, y, a, b, nullptr, f0, mean, U, wv, partials, \
                                     counter, g_out, s, gate);                                    \
        break
    if (dt == PCAS_F32) {
        switch (K) { A(float, 1, ADJ_ACC32); A(float, 2, ADJ_ACC32); A(float, 3, ADJ_ACC32);
                     A(float, 4, ADJ_ACC32); A(float, 5, ADJ_ACC32); A(float, 6, ADJ_ACC32);
                     A(float, 7, ADJ_ACC32); A(float, 8, ADJ_ACC32);
                     default: return hipErrorInvalidValue; }
    } else {
        switch (K) { A(double, 1, ADJ_ACC64); A(double, 2, ADJ_ACC64); A(double, 3, ADJ_ACC64);
                     A(double, 4, ADJ_ACC64); A(double, 5, ADJ_ACC64); A(double, 6, ADJ_ACC64);
                     A(double, 7, ADJ_ACC64); A(double, 8, ADJ_ACC64);
                     default: return hipErrorInvalidValue; }
    }
#undef A
    return hipGetLastError();
}

AdjJob make_adj_job(const VolDims &v, const Frame &fr, int K, const void *rays, const void *p,
                    const void *y, double a, double b, const void *f0, const void *mean,
                    const void *U, const double *w, double *partials, uint32_t *counter,
                    double *g_out) {
    AdjJob J;
    J.vd = v;
    J.fr = fr;
    J.nbx = (v.n0 + BRICK_X - 1) / BRICK_X;
    J.nby = (v.n1 + BRICK_Y - 1) / BRICK_Y;
    J.hb = ray_weight_bound(v, fr);
    J.rays = rays;
    J.p = p;
    J.y = y;
    J.a = a;
    J.b = b;
    J.f0 = f0;
    J.mean = mean;
    J.U = U;
    J.w = WVec{};
    for (int k = 0; k < K; ++k) J.w.w[k] = w[k];
    J.partials = partials;
    J.counter = counter;
    J.g_out = g_out;
    J.block0 = 0;
    J.split = adjoint_chain_split(v);
    J.nblocks = drr_adjoint_blocks(v) * J.split;
    return J;
}

hipError_t launch_drr_adjoint_chain_batch(pcas_dtype dt, int K, const AdjJob *jobs, int njobs,
                                          int total_blocks, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
#define A(TT, KK)                                                                                 \
    case KK:                                                                                      \
        hipLaunchKernelGGL((k_drr_adjoint_batch<TT, KK>), dim3(total_blocks), dim3(ADJ_THREADS), 0, s,     \
                           jobs, njobs);                                                          \
        break
    if (dt == PCAS_F32) {
        switch (K) { A(float, 1); A(float, 2); A(float, 3); A(float, 4);
                     A(float, 5); A(float, 6); A(float, 7); A(float, 8);
                     default: return hipErrorInvalidValue; }
    } else {
        switch (K) { A(double, 1); A(double, 2); A(double, 3); A(double, 4);
                     A(double, 5); A(double, 6); A(double, 7); A(double, 8);
                     default: return hipErrorInvalidValue; }
    }
#undef A
    return hipGetLastError();
}

}  // namespace pcas
