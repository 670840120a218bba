// Kernel instantiations for one element type (see rsg_device.h).
#include "rsg_dispatch.h"

namespace rsg {

int launch_single_bf16(const ImgParams& ip, hipStream_t stream)
{
    return dispatch::launch_single_t<dev::TrBF16>(ip, stream);
}

int launch_batch_class_bf16(const BatchClassLaunch& b, hipStream_t stream)
{
    return dispatch::launch_batch_t<dev::TrBF16>(b, stream);
}

int launch_pass_bf16(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t stream)
{
    return dispatch::launch_pass_t<dev::TrBF16>(ip, pass, pp, stream);
}

int launch_pass_batch_bf16(const PassBatchLaunch& b, hipStream_t stream)
{
    return dispatch::launch_pass_batch_t<dev::TrBF16>(b, stream);
}

}  // namespace rsg
