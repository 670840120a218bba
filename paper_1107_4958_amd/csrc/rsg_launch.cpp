// Launch paths: one image (one fused kernel launch) and batches (one
// persistent launch per (element type, channel count, tap count) class,
// all on the caller's stream).
#include "rsg_internal.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

namespace rsg {

int launch_single(const ImgParams& ip, hipStream_t stream)
{
    switch (ip.dtype) {
    case RSG_U8: return launch_single_u8(ip, stream);
    case RSG_F32: return launch_single_f32(ip, stream);
    case RSG_F16: return launch_single_f16(ip, stream);
    case RSG_BF16: return launch_single_bf16(ip, stream);
    default: return set_error(RSG_EINVAL, "bad dtype %d", ip.dtype);
    }
}

int launch_batch_class(const BatchClassLaunch& b, hipStream_t stream)
{
    switch (b.dtype) {
    case RSG_U8: return launch_batch_class_u8(b, stream);
    case RSG_F32: return launch_batch_class_f32(b, stream);
    case RSG_F16: return launch_batch_class_f16(b, stream);
    case RSG_BF16: return launch_batch_class_bf16(b, stream);
    default: return set_error(RSG_EINVAL, "bad dtype %d", b.dtype);
    }
}

namespace {
constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }
constexpr int kMaxClasses = 4 * 4 * 3;   // dtype x C x taps
}  // namespace

// Workspace: [counters, one per class][ImgParams x nimg][BatchTask x ntasks]
size_t batch_workspace_bytes(int nimg, int ntasks)
{
    return up(sizeof(unsigned) * kMaxClasses) + up(sizeof(ImgParams) * size_t(nimg)) +
           up(sizeof(BatchTask) * size_t(ntasks));
}

int launch_batch(const ImgParams* h_imgs, int nimg, const BatchTask* h_tasks, int ntasks, void* d_ws,
                 size_t ws_bytes, hipStream_t stream, void* h_stage)
{
    const size_t need = batch_workspace_bytes(nimg, ntasks);
    if (ws_bytes < need) return set_error(RSG_ENOMEM, "workspace too small: %zu < %zu", ws_bytes, need);
    // group the tasks by kernel class, keeping their order inside a class
    std::map<std::tuple<int, int, int>, std::vector<BatchTask>> classes;
    for (int t = 0; t < ntasks; ++t) {
        const ImgParams& ip = h_imgs[h_tasks[t].img];
        classes[std::make_tuple(ip.dtype, ip.C, ip.kt)].push_back(h_tasks[t]);
    }
    std::vector<char> pageable;
    char* host = static_cast<char*>(h_stage);
    if (!host) {
        pageable.assign(need, 0);
        host = pageable.data();
    } else {
        std::memset(host, 0, need);
    }
    const size_t o_img = up(sizeof(unsigned) * kMaxClasses);
    const size_t o_task = o_img + up(sizeof(ImgParams) * size_t(nimg));
    std::memcpy(host + o_img, h_imgs, sizeof(ImgParams) * size_t(nimg));
    size_t pos = 0;
    for (auto& kv : classes) {
        std::memcpy(host + o_task + pos * sizeof(BatchTask), kv.second.data(), sizeof(BatchTask) * kv.second.size());
        pos += kv.second.size();
    }
    hipError_t e = hipMemcpyAsync(d_ws, host, need, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return set_error(RSG_EDEVICE, "workspace copy failed: %s", hipGetErrorString(e));

    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    char* ws = static_cast<char*>(d_ws);
    pos = 0;
    int ci = 0;
    for (auto& kv : classes) {
        BatchClassLaunch b;
        b.dtype = std::get<0>(kv.first);
        b.C = std::get<1>(kv.first);
        b.kt = std::get<2>(kv.first);
        b.lds = 0;
        for (const BatchTask& t : kv.second) b.lds = std::max(b.lds, h_imgs[t.img].lds_bytes);
        // resident waves per CU are bounded by LDS (160 KiB per CU on gfx950)
        int per_cu = b.lds ? int((160u * 1024u) / b.lds) : 16;
        per_cu = std::max(1, std::min(per_cu, 16));
        b.ntasks = int(kv.second.size());
        b.grid = std::max(1, std::min(b.ntasks, ncu * per_cu));
        b.d_imgs = reinterpret_cast<const ImgParams*>(ws + o_img);
        b.d_tasks = reinterpret_cast<const BatchTask*>(ws + o_task) + pos;
        b.d_counter = reinterpret_cast<unsigned*>(ws) + ci;
        int rc = launch_batch_class(b, stream);
        if (rc != RSG_OK) return rc;
        pos += kv.second.size();
        ++ci;
    }
    return RSG_OK;
}

}  // namespace rsg
