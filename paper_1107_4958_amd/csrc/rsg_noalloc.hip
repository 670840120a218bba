// rsg_gauss_filter_noalloc: rsg_gauss_filter for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
// The only device memory the single-image path needs beyond the caller's
// images is the two-pass path's intermediate (4 H W C bytes); here it is a
// file-scope device array of fixed size.  Its device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is handed to kernels.
#include "rsg_internal.h"

#include <mutex>

namespace rsg {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;          // 16 Mi four-byte words
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint32_t scratch[kScratchBytes / 4];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (NULL on failure).
void* scratch_on(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace rsg

extern "C" int rsg_gauss_filter_noalloc(const void* d_src, void* d_dst, int H, int W, int C, rsg_dtype dt,
                                        double sigma, int K, rsg_boundary b, void* stream)
{
    using namespace rsg;
    rsg_image_desc d;
    d.src = d_src;
    d.dst = d_dst;
    d.H = H;
    d.W = W;
    d.C = C;
    d.src_stride = 0;
    d.dst_stride = 0;
    d.dt = dt;
    d.sigma = sigma;
    d.K = K;
    d.b = b;
    d.boxes = nullptr;
    ImgParams ip;
    int rc = plan_image(d, &ip);
    if (rc != RSG_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ip.path != kPathTwoPass) return launch_single(ip, st);     // the fused kernel uses no scratch memory
    const size_t need = mid_bytes(ip);
    if (need > kScratchBytes)
        return set_error(RSG_ENOMEM, "two-pass intermediate of %zu bytes exceeds the %zu-byte scratch of the no-alloc entry point",
                         need, kScratchBytes);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(RSG_EDEVICE, "hipGetDevice failed");
    void* mid = scratch_on(dev);
    if (!mid) return set_error(RSG_EDEVICE, "cannot look up the scratch array on device %d", dev);
    return launch_two_pass_into(ip, mid, st);
}
