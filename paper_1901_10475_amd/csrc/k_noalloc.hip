// k_noalloc.hip -- the graph-capturable query with its workspace in a fixed
// device array, for callers that cannot allocate (code under hipGraph capture,
// serving loops, harnesses that forbid allocation).
#include <mutex>

#include "cd_internal.h"

namespace {

// The query's workspace: two node-pair queues of max(N, 65536) entries, the
// control block and, per record slot of the capacity, raw and sorted records,
// flags, positions and scan/radix scratch.  64 MiB holds, for example, a tree
// of 2 M boxes with 1 M record slots.  Every device the library runs on holds
// its own copy until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // the array's device address, per device

}  // namespace

extern "C" size_t cd_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int cd_query_pairs_async_noalloc(const cd_tree *tree, cd_pair *out, int64_t capacity,
                                            unsigned long long *count_dev,
                                            unsigned int *status_dev, cd_stream_t stream)
{
    if (!tree)
        return cd::set_error(CD_E_INVALID, "tree is NULL");
    if (tree->count < 0)
        return cd::set_error(CD_E_INVALID, "tree is not built");
    if (capacity < 1 || capacity > 0xFFFFFFFEll)
        return cd::set_error(CD_E_INVALID, "capacity must be in [1, 2^32 - 2]");
    size_t need = cd_query_pairs_ws(tree->count, capacity);
    if (need > kScratchBytes)
        return cd::set_error(CD_E_WORKSPACE,
                             "a query of %lld boxes with %lld record slots needs %zu bytes of "
                             "workspace; the fixed scratch holds %zu (use cd_query_pairs_async "
                             "with a caller workspace)",
                             (long long)tree->count, (long long)capacity, need, kScratchBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return cd::set_error(CD_E_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return cd::set_error(CD_E_DEVICE, "device %d beyond the %d devices with scratch", dev,
                             kMaxDevices);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            // the array's name is a host-side stand-in; its address on the
            // current device comes from the runtime, once per device
            e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess)
                return cd::set_error(CD_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                                     hipGetErrorString(e));
            g_scratch_ptr[dev] = ptr;
        }
        ptr = g_scratch_ptr[dev];
    }
    // the async query clears every counter and flag it reads with fill kernels
    // before use, so the previous call's contents do not matter
    return cd_query_pairs_async(tree, out, capacity, count_dev, status_dev, ptr, kScratchBytes,
                                stream);
}
