// grad_w without a caller workspace: the reduction partials and the
// last-block counter live in one file-scope device array per GPU, so the
// call allocates nothing (for callers that cannot allocate).
#include <mutex>

#include "host.h"

namespace pcas {
namespace {

// Partials of GRAD_BLOCKS_MAX blocks (RED_SLOTS doubles each), then the
// grid reduction's counter.
constexpr size_t NOALLOC_PARTIALS = (size_t)GRAD_BLOCKS_MAX * RED_SLOTS * sizeof(double);
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_PARTIALS + 256;
static_assert(NOALLOC_PARTIALS % 256 == 0, "counter offset alignment");

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
void *scratch_ptr[MAX_DEVICES] = {nullptr};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the array's name is a host-side stand-in, not a
// device address).
hipError_t device_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace pcas

using namespace pcas;
using namespace pcas::host;

extern "C" size_t grad_w_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" int grad_w_noalloc(pcas_dtype dtype, const pcas_vol *vol, int32_t K, const void *f0,
                              const void *mean, const void *U, const double *w, const void *bp,
                              double *g_out, void *stream) {
    if (!dtype_ok(dtype) || K < 1 || K > PCAS_MAX_K) return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    if (!f0 || !U || !w || !bp || !g_out) return PCAS_EINVAL;
    if (!finite_vec(w, K)) return PCAS_ENONFINITE;
    const size_t need = (size_t)grad_w_blocks(nvox_of(vol)) * RED_SLOTS * sizeof(double);
    if (need > NOALLOC_PARTIALS) return PCAS_EWORKSPACE;
    void *base = nullptr;
    HIPCHK(device_scratch(&base));
    double *partials = (double *)base;
    uint32_t *counter = (uint32_t *)((char *)base + NOALLOC_PARTIALS);
    hipStream_t s = (hipStream_t)stream;
    // the array keeps the last call's contents: the counter starts at zero
    HIPCHK(launch_fill_u32(counter, 1, 0u, s));
    HIPCHK(launch_grad_w(dtype, make_dims(vol), K, f0, mean, U, w, bp, partials, counter, g_out, s));
    return PCAS_OK;
}
