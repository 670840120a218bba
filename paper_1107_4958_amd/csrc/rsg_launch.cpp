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

int launch_pass(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t stream)
{
    switch (ip.dtype) {
    case RSG_U8: return launch_pass_u8(ip, pass, pp, stream);
    case RSG_F32: return launch_pass_f32(ip, pass, pp, stream);
    case RSG_F16: return launch_pass_f16(ip, pass, pp, stream);
    case RSG_BF16: return launch_pass_bf16(ip, pass, pp, stream);
    default: return set_error(RSG_EINVAL, "bad dtype %d", ip.dtype);
    }
}

namespace {

PassParams pass_params(const ImgParams& ip, int pass, void* mid)
{
    PassParams pp;
    std::memset(&pp, 0, sizeof(pp));
    const int es = dtype_size(ip.dtype);
    const int WC = ip.W * ip.C;
    const int npl = ip.pnpl[pass];
    if (pass == 0) {                       // image rows -> intermediate (W*C) x H
        pp.src = ip.src;
        pp.dst = mid;
        pp.src_stride = ip.src_stride;
        pp.dst_stride = ip.H;
        pp.rows = ip.H;
        pp.len = WC;
        // chunk loads use the widest of 16 / 8 / 4 bytes that divides the chunk
        const int cb = npl * es;
        const int g = cb % 16 == 0 ? 16 : (cb % 8 == 0 ? 8 : (cb % 4 == 0 ? 4 : 0));
        const uintptr_t a = reinterpret_cast<uintptr_t>(ip.src);
        pp.vec = g > 0 && a % g == 0 && (ip.src_stride * es) % g == 0;
    } else {                               // intermediate rows (image columns) -> image
        pp.src = mid;
        pp.dst = ip.dst;
        pp.src_stride = ip.H;
        pp.dst_stride = ip.dst_stride;
        pp.rows = WC;
        pp.len = ip.H;
        pp.vec = (int64_t(ip.H) * 4) % 16 == 0;
    }
    pp.R = ip.R;
    for (int k = 0; k < RSG_MAX_K; ++k) {
        pp.r[k] = ip.r[k];
        pp.wf[k] = ip.wf[k];
        pp.m[k] = ip.m[k];
    }
    pp.dc32 = ip.dc32;
    pp.G2 = ip.G2;
    pp.G2half = ip.G2half;
    pp.invG2 = ip.invG2;
    pp.boundary = ip.boundary;
    const int hw = (2 * ip.R + 1) * (pass == 0 ? ip.C : 1);
    pp.win_pitch = pass_win_pitch(npl, hw);
    pp.win_shift = (4 - hw % 4) % 4;
    return pp;
}

// Both passes on `stream`, through an intermediate allocated in stream order.
int launch_two_pass(const ImgParams& ip, hipStream_t stream)
{
    void* mid = nullptr;
    const size_t bytes = size_t(ip.H) * size_t(ip.W) * size_t(ip.C) * 4;
    if (hipMallocAsync(&mid, bytes, stream) != hipSuccess)
        return set_error(RSG_ENOMEM, "cannot allocate the %zu-byte intermediate of the two-pass path", bytes);
    int rc = launch_pass(ip, 0, pass_params(ip, 0, mid), stream);
    if (rc == RSG_OK) rc = launch_pass(ip, 1, pass_params(ip, 1, mid), stream);
    if (hipFreeAsync(mid, stream) != hipSuccess && rc == RSG_OK)
        rc = set_error(RSG_EDEVICE, "cannot release the two-pass intermediate");
    return rc;
}

}  // namespace

int launch_single(const ImgParams& ip, hipStream_t stream)
{
    if (ip.path == kPathTwoPass) return launch_two_pass(ip, stream);
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
    // images planned for the two-pass path run their two passes after the
    // persistent launches, on the same stream
    for (int i = 0; i < nimg; ++i) {
        if (h_imgs[i].path != kPathTwoPass) continue;
        int rc = launch_single(h_imgs[i], stream);
        if (rc != RSG_OK) return rc;
    }
    return RSG_OK;
}

}  // namespace rsg
