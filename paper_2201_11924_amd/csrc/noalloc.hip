// simsense_compute_noalloc: the whole depth path of one pair without a handle
// and without any device allocation.  The scratch a handle would allocate (census
// maps, per-direction path values, per-pixel results) lives in one file-scope
// device array of fixed size; the kernels are the handle path's own, with the
// aggregation launched one block per line block (no work list to upload).
#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)SIMSENSE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, at a per-GPU address; host code only ever uses the address
// hipGetSymbolAddress returns for the current device (the array's name on the
// host is a stand-in, not a device address).
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mutex;
void *g_scratch_ptr[kMaxDevices];

// the device address of this device's copy of the array, looked up once per device
int scratch_for_current_device(uint8_t **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return SIMSENSE_ERR_DEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) return SIMSENSE_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return SIMSENSE_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = (uint8_t *)g_scratch_ptr[dev];
    return SIMSENSE_OK;
}

}  // namespace

using namespace ss;

extern "C" int simsense_compute_noalloc(const simsense_params *params, const uint8_t *left, const uint8_t *right,
                                        int32_t pitch, float *depth, float *disp, uint8_t *flags, void *stream)
{
    int rc = validate(params);
    if (rc != SIMSENSE_OK) return rc;
    if (!left || !right || !depth) return SIMSENSE_ERR_NULL_POINTER;
    if (pitch < params->width) return SIMSENSE_ERR_INVALID_ARGUMENT;
    const Layout l = layout(params);
    if (l.total > kScratchBytes) return SIMSENSE_ERR_TOO_LARGE;
    uint8_t *base = nullptr;
    rc = scratch_for_current_device(&base);
    if (rc != SIMSENSE_OK) return rc;

    // a handle on the stack: its buffers point into the static scratch, the
    // aggregation runs one block per line block, profiling is off
    simsense_handle h{};
    init_handle(&h, params);
    carve_scratch(&h, base, l);
    h.tuning.struct_size = sizeof(h.tuning);
    h.tuning.horizontal_lanes = 0;
    h.tuning.blocks_per_cu = 0;
    h.profiling = false;
    // every scratch byte a call reads is written earlier in the same call, so
    // nothing needs clearing between calls
    hipStream_t s = (hipStream_t)stream;
    rc = enqueue_match(&h, left, right, pitch, s);
    if (rc != SIMSENSE_OK) return rc;
    simsense_outputs o{};
    o.depth = depth;
    o.disp = disp;
    o.flags = flags;
    return enqueue_post(&h, h.masked, h.flags_pre, &o, s);
}
