// The bandwidth reference of the roofline: a plain streaming copy with the
// widest accesses (16 bytes per lane, 8 per thread in flight), timed by the
// benchmark on the same buffer rotation as the filter.
#include "rsg_internal.h"

namespace rsg {
namespace dev {

constexpr int kCopyUnroll = 8;

__global__ __launch_bounds__(256) void k_stream_copy(const uint4* __restrict__ s, uint4* __restrict__ d, size_t n16)
{
    const size_t base = size_t(blockIdx.x) * (256 * kCopyUnroll) + threadIdx.x;
    uint4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {          // a select, not a conditional store: v stays in registers
        const size_t i = base + size_t(u) * 256;
        v[u] = (i < n16) ? s[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + size_t(u) * 256;
        if (i < n16) d[i] = v[u];
    }
}

__global__ void k_copy_tail(const uint8_t* __restrict__ s, uint8_t* __restrict__ d, size_t n)
{
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

}  // namespace dev
}  // namespace rsg

extern "C" int rsg_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream)
{
    using namespace rsg;
    if (!d_src || !d_dst) return set_error(RSG_EINVAL, "rsg_stream_copy: NULL pointer");
    if ((reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst)) % 16)
        return set_error(RSG_EINVAL, "rsg_stream_copy: buffers must be 16-byte aligned");
    if (bytes == 0) return RSG_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n16 = bytes / 16;
    const size_t per_block = size_t(256) * dev::kCopyUnroll;
    if (n16) {
        const size_t blocks = (n16 + per_block - 1) / per_block;
        if (blocks > 0x7fffffffu) return set_error(RSG_EUNSUPPORTED, "rsg_stream_copy: %zu bytes is too large", bytes);
        hipLaunchKernelGGL(dev::k_stream_copy, dim3(unsigned(blocks)), dim3(256), 0, st,
                           static_cast<const uint4*>(d_src), static_cast<uint4*>(d_dst), n16);
    }
    const size_t tail = bytes - n16 * 16;
    if (tail)
        hipLaunchKernelGGL(dev::k_copy_tail, dim3(1), dim3(64), 0, st, static_cast<const uint8_t*>(d_src) + n16 * 16,
                           static_cast<uint8_t*>(d_dst) + n16 * 16, tail);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(RSG_EDEVICE, "copy launch failed: %s", hipGetErrorString(e));
    return RSG_OK;
}
