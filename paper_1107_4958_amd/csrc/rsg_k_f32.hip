// Kernel instantiations for one element type (see rsg_device.h).
#include "rsg_dispatch.h"

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

}  // namespace rsg
