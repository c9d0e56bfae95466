// qcl_propagate_batch_static: the batched propagation with the library's
// own workspace, for callers that cannot allocate device memory.
//
// The workspace (the batch descriptors and one tile counter per kernel
// class) lives in a file-scope device array of QCL_STATIC_WORKSPACE_BYTES;
// every GPU the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel: that name is a
// host-side stand-in, not a device address.  The device address is taken
// once per device, with that device current, by hipGetSymbolAddress on the
// entry point's first call there, and used from then on.  The descriptor
// upload kernel rewrites the whole image (counters included) on every call,
// so nothing carries over from the previous call; calls whose execution
// overlaps on one device race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qcl_internal.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[QCL_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];  // device address of scratch, per device (NULL until resolved)

}  // namespace

extern "C" qcl_status qcl_propagate_batch_static(const qcl_batch_item *items, int32_t n_items, void *stream)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return qcl::set_error(QCL_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return qcl::set_error(QCL_ERR_UNSUPPORTED, "device %d is beyond the %d this library tracks", dev, kMaxDevices);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return qcl::set_error(QCL_ERR_DEVICE, "hipGetSymbolAddress of the static workspace: %s",
                                      hipGetErrorString(e));
            g_scratch_ptr[dev] = p;
        }
        ptr = g_scratch_ptr[dev];
    }
    return qcl::propagate_batch_in(items, n_items, ptr, QCL_STATIC_WORKSPACE_BYTES, stream, true);
}
