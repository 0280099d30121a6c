// Plain device-to-device streaming copy: the bandwidth reference that the
// solver's achieved HBM throughput is compared with (and the known-size kernel
// that calibrates the hardware traffic counters).  Not part of the method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tled.h"

namespace {

constexpr int kCopyBlock = 256;

// Grid-stride over float4 elements, four independent loads in flight per thread.
__global__ __launch_bounds__(kCopyBlock) void stream_copy_kernel(const float4 *__restrict__ src,
                                                                 float4 *__restrict__ dst, size_t n) {
    const size_t stride = size_t(gridDim.x) * kCopyBlock;
    size_t i = size_t(blockIdx.x) * kCopyBlock + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" tled_status tled_stream_copy(int device, void *dst, const void *src, size_t bytes, void *hip_stream) {
    if (!dst || !src || bytes == 0 || bytes % 16 || (uintptr_t(dst) | uintptr_t(src)) % 16) return TLED_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return TLED_E_HIP;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return TLED_E_HIP;
    const size_t n = bytes / 16;
    // eight resident workgroups per CU, never more than the elements need
    const size_t want = (n + kCopyBlock - 1) / kCopyBlock, cap = size_t(cus) * 8;
    const unsigned grid = unsigned(want < cap ? want : cap);
    hipLaunchKernelGGL(stream_copy_kernel, dim3(grid), dim3(kCopyBlock), 0, static_cast<hipStream_t>(hip_stream),
                       static_cast<const float4 *>(src), static_cast<float4 *>(dst), n);
    return hipGetLastError() == hipSuccess ? TLED_OK : TLED_E_HIP;
}
