// k_copy.hip -- a plain streaming copy: the achievable HBM bandwidth against
// which the other kernels' rooflines are read (and a kernel of known byte
// count for calibrating the HBM byte counters).
#include "cd_internal.h"

namespace cd {

namespace {

constexpr int kCopyThreads = 256;

// One 16-byte word per lane and a grid that covers the buffer once: measured
// fastest on MI355X (6.2 TB/s read + write over 4 GiB, against 4.4-5.2 TB/s
// for grid-stride loops of 1-8 words per lane at 1 024-16 384 workgroups and
// 4.9 TB/s for hipMemcpy).  Stores are non-temporal: the copy's output is not
// read again by this kernel.
__global__ __launch_bounds__(kCopyThreads) void k_stream_copy(const uint4 *__restrict__ src,
                                                              uint4 *__restrict__ dst,
                                                              uint64_t words, uint64_t first)
{
    uint64_t i = first + (uint64_t)blockIdx.x * kCopyThreads + threadIdx.x;
    if (i >= words)
        return;
    uint4 v = src[i];
    __builtin_nontemporal_store(v.x, &dst[i].x);
    __builtin_nontemporal_store(v.y, &dst[i].y);
    __builtin_nontemporal_store(v.z, &dst[i].z);
    __builtin_nontemporal_store(v.w, &dst[i].w);
}

}  // namespace

hipError_t launch_stream_copy(const void *src, void *dst, uint64_t words, hipStream_t s)
{
    // launches of at most 2^30 words (2^22 workgroups) each
    const uint64_t per = uint64_t(1) << 30;
    for (uint64_t first = 0; first < words; first += per) {
        uint64_t n = words - first < per ? words - first : per;
        unsigned grid = (unsigned)((n + kCopyThreads - 1) / kCopyThreads);
        hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(kCopyThreads), 0, s,
                           (const uint4 *)src, (uint4 *)dst, words, first);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace cd
