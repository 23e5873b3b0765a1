// memory.hip -- optional allocator for the caller's large device buffers (workspaces).
//
// A plain allocation of several GiB made after the device has been through many allocations and
// frees can be built from many small physical pieces, each needing its own address translation.
// Kernels that walk several multi-GiB arrays at once then wait on translation: the 3D FGP
// iteration, which streams thirteen volume-sized arrays, took 3.0 instead of 2.0 ms on a
// 256 x 1024^2 volume whose dual buffers sat in such an allocation.  device_alloc asks the
// driver for physically contiguous memory first and falls back to an ordinary allocation.
#include "internal.h"

using namespace ps;

namespace {

struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" ps_status device_alloc(size_t bytes, int32_t device, void **out, int32_t *contiguous) {
    clear_error();
    if (!out) return fail(PS_EINVAL, "null output pointer");
    *out = nullptr;
    if (contiguous) *contiguous = 0;
    if (bytes == 0) return fail(PS_EINVAL, "zero-byte allocation");
    int count = 0;
    PS_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(PS_EINVAL, "device %d of %d", device, count);
    DeviceScope scope(device);
    if (scope.err != hipSuccess) return fail(PS_EHIP, "hipSetDevice(%d): %s", device, hipGetErrorString(scope.err));
    void *p = nullptr;
    if (hipExtMallocWithFlags(&p, bytes, hipDeviceMallocContiguous) == hipSuccess && p) {
        if (contiguous) *contiguous = 1;
        *out = p;
        return PS_OK;
    }
    // the failed attempt leaves its error as the thread's last error: clear it, so that the next
    // launch check does not report it
    (void)hipGetLastError();
    p = nullptr;
    PS_HIP(hipMalloc(&p, bytes));
    *out = p;
    return PS_OK;
}

extern "C" ps_status device_free(void *ptr) {
    clear_error();
    if (!ptr) return PS_OK;
    hipPointerAttribute_t attr{};
    PS_HIP(hipPointerGetAttributes(&attr, ptr));
    if (attr.type != hipMemoryTypeDevice) return fail(PS_EINVAL, "not device memory");
    DeviceScope scope(attr.device);
    if (scope.err != hipSuccess) return fail(PS_EHIP, "hipSetDevice(%d): %s", attr.device, hipGetErrorString(scope.err));
    // work queued on any stream may still use the buffer
    PS_HIP(hipDeviceSynchronize());
    PS_HIP(hipFree(ptr));
    return PS_OK;
}
