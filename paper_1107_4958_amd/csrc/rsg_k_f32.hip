// Kernel instantiations for one element type (see rsg_device.h); the FP32
// unit also holds the z pass of volumes (rsg_zpass.h).
#include "rsg_dispatch.h"
#include "rsg_zpass.h"

namespace rsg {

int launch_single_f32(const ImgParams& ip, hipStream_t stream)
{
    return dispatch::launch_single_t<dev::TrF32>(ip, stream);
}

int launch_batch_class_f32(const BatchClassLaunch& b, hipStream_t stream)
{
    return dispatch::launch_batch_t<dev::TrF32>(b, stream);
}

int launch_pass_f32(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t stream)
{
    return dispatch::launch_pass_t<dev::TrF32>(ip, pass, pp, stream);
}

int launch_pass_batch_f32(const PassBatchLaunch& b, hipStream_t stream)
{
    return dispatch::launch_pass_batch_t<dev::TrF32>(b, stream);
}

int launch_zpass_f32(const ZParams& zp, int kt, int wpb, hipStream_t stream)
{
    constexpr int PFZ = 4;                  // slices prefetched ahead (4 measured 0-5 % faster than 8 and 16)
    const void* fn = nullptr;
    switch (kt) {
    case 3: fn = reinterpret_cast<const void*>(dev::k_zpass<3, PFZ>); break;
    case 4: fn = reinterpret_cast<const void*>(dev::k_zpass<4, PFZ>); break;
    case 5: fn = reinterpret_cast<const void*>(dev::k_zpass<5, PFZ>); break;
    default: return set_error(RSG_EUNSUPPORTED, "no z-pass kernel for %d taps", kt);
    }
    const uint32_t lds = uint32_t(wpb) * uint32_t(zp.L) * uint32_t(kWave) * 4u;
    int rc = dispatch::set_lds_limit(fn, lds);
    if (rc != RSG_OK) return rc;
    const dim3 grid((zp.ntasks + wpb - 1) / wpb), block(wpb * kWave);
    switch (kt) {
    case 3: hipLaunchKernelGGL((dev::k_zpass<3, PFZ>), grid, block, lds, stream, zp); break;
    case 4: hipLaunchKernelGGL((dev::k_zpass<4, PFZ>), grid, block, lds, stream, zp); break;
    default: hipLaunchKernelGGL((dev::k_zpass<5, PFZ>), grid, block, lds, stream, zp); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(RSG_EDEVICE, "z-pass launch failed: %s", hipGetErrorString(e));
    return RSG_OK;
}

}  // namespace rsg
