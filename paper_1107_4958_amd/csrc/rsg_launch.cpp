// Launch paths, all on the caller's stream: one image (one fused kernel
// launch, or the two launches of the two-pass path around a stream-ordered
// intermediate) and batches (one persistent launch per fused class of
// element type, channel count, tap count and form, then the two-pass images'
// row blocks grouped per pass instantiation, with every intermediate carved
// from the caller's workspace).
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
    const int step = ip.step > 1 ? ip.step : 1;
    const int WoC = (ip.W + step - 1) / step * ip.C;   // intermediate rows: kept pixels x channels
    const int npl = ip.pnpl[pass];
    pp.ostep = step;
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
        pp.rows = WoC;
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
    pp.qsh = ip.qsh;
    pp.boundary = ip.boundary;
    const int hw = (2 * ip.R + 1) * (pass == 0 ? ip.C : 1);
    pp.win_pitch = pass_win_pitch(npl, hw);
    pp.win_shift = (4 - hw % 4) % 4;
    return pp;
}

}  // namespace

size_t mid_bytes(const ImgParams& ip)
{
    if (ip.path != kPathTwoPass) return 0;
    const int step = ip.step > 1 ? ip.step : 1;
    return size_t(ip.H) * size_t((ip.W + step - 1) / step) * size_t(ip.C) * 4;
}

int launch_two_pass_into(const ImgParams& ip, void* mid, hipStream_t stream)
{
    int rc = launch_pass(ip, 0, pass_params(ip, 0, mid), stream);
    if (rc == RSG_OK) rc = launch_pass(ip, 1, pass_params(ip, 1, mid), stream);
    return rc;
}

namespace {

// Both passes on `stream`, through an intermediate allocated in stream order
// (the single-image entry points take no workspace).
int launch_two_pass(const ImgParams& ip, hipStream_t stream)
{
    void* mid = nullptr;
    const size_t bytes = mid_bytes(ip);
    if (hipMallocAsync(&mid, bytes, stream) != hipSuccess)
        return set_error(RSG_ENOMEM, "cannot allocate the %zu-byte intermediate of the two-pass path", bytes);
    int rc = launch_two_pass_into(ip, mid, stream);
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
constexpr int kMaxClasses = 4 * 4 * 3 * 2;   // dtype x C x taps x (one or wide_nc(C) columns per lane)
}  // namespace

int64_t pass_blocks(const ImgParams* imgs, int nimg)
{
    int64_t n = 0;
    for (int i = 0; i < nimg; ++i)
        if (imgs[i].path == kPathTwoPass) n += imgs[i].ntasks;
    return n;
}

// Workspace: [counters, one per class][ImgParams x nimg][task entries x ntasks]
// [PassParams x 2 nimg] (the header), then one intermediate per two-pass
// image.  Task entries (8 bytes) are the fused images' BatchTasks followed by
// the (pass parameters, row block) pairs of the two-pass images.
size_t batch_header_bytes(int nimg, int64_t ntasks)
{
    return up(sizeof(unsigned) * kMaxClasses) + up(sizeof(ImgParams) * size_t(nimg)) +
           up(sizeof(BatchTask) * size_t(ntasks)) + up(sizeof(PassParams) * 2 * size_t(nimg));
}

size_t batch_mid_bytes(const ImgParams* imgs, int nimg)
{
    size_t b = 0;
    for (int i = 0; i < nimg; ++i) b += up(mid_bytes(imgs[i]));
    return b;
}

size_t batch_workspace_bytes(const ImgParams* imgs, int nimg, int64_t ntasks)
{
    return batch_header_bytes(nimg, ntasks) + batch_mid_bytes(imgs, nimg);
}

int launch_batch(const ImgParams* h_imgs, int nimg, const BatchTask* h_tasks, int ntasks, void* d_ws,
                 size_t ws_bytes, hipStream_t stream, void* h_stage)
{
    static_assert(sizeof(BatchTask) == sizeof(int2), "task entries share one region");
    const int64_t nblocks = pass_blocks(h_imgs, nimg);
    const size_t hdr = batch_header_bytes(nimg, ntasks + nblocks);
    const size_t need = hdr + batch_mid_bytes(h_imgs, nimg);
    if (ws_bytes < need) return set_error(RSG_ENOMEM, "workspace too small: %zu < %zu", ws_bytes, need);

    // fused images: group the tasks by kernel class, keeping their order
    std::map<std::tuple<int, int, int, int, int>, std::vector<BatchTask>> classes;
    for (int t = 0; t < ntasks; ++t) {
        const ImgParams& ip = h_imgs[h_tasks[t].img];
        // channel-planar images run the one-channel kernel
        classes[std::make_tuple(ip.dtype, ip.pstride > 1 ? 1 : ip.C, ip.kt, ip.co, ip.co ? ip.nc : 1)].push_back(h_tasks[t]);
    }

    // two-pass images: intermediates after the header, pass parameters 2j
    // (A) and 2j + 1 (B) for the j-th of them, row blocks grouped by
    // instantiation
    std::vector<int> two;
    for (int i = 0; i < nimg; ++i)
        if (h_imgs[i].path == kPathTwoPass) two.push_back(i);
    std::vector<PassParams> pps(2 * two.size());
    using PassKey = std::tuple<int, int, int, int, int, int, int>;   // pass, dtype, C, npl, kt, stages, rows
    std::map<PassKey, std::vector<int2>> pclasses;
    std::map<PassKey, uint32_t> plds;
    {
        size_t off = hdr;
        for (size_t j = 0; j < two.size(); ++j) {
            const ImgParams& ip = h_imgs[two[j]];
            void* slice = static_cast<char*>(d_ws) + off;
            off += up(mid_bytes(ip));
            for (int pass = 0; pass < 2; ++pass) {
                pps[2 * j + pass] = pass_params(ip, pass, slice);
                const PassKey key(pass, ip.dtype, pass == 0 ? ip.C : 1, ip.pnpl[pass], ip.kt, ip.pst[pass],
                                  ip.ptr[pass]);
                const int rows = pps[2 * j + pass].rows;
                auto& v = pclasses[key];
                for (int blk = 0; blk < (rows + ip.ptr[pass] - 1) / ip.ptr[pass]; ++blk)
                    v.push_back(int2{int(2 * j + pass), blk});
                plds[key] = std::max(plds[key], ip.plds[pass]);
            }
        }
    }

    std::vector<char> pageable;
    char* host = static_cast<char*>(h_stage);
    if (!host) {
        pageable.assign(hdr, 0);
        host = pageable.data();
    } else {
        std::memset(host, 0, hdr);
    }
    const size_t o_img = up(sizeof(unsigned) * kMaxClasses);
    const size_t o_task = o_img + up(sizeof(ImgParams) * size_t(nimg));
    const size_t o_pp = o_task + up(sizeof(BatchTask) * size_t(ntasks + nblocks));
    std::memcpy(host + o_img, h_imgs, sizeof(ImgParams) * size_t(nimg));
    size_t pos = 0;
    for (auto& kv : classes) {
        std::memcpy(host + o_task + pos * sizeof(BatchTask), kv.second.data(), sizeof(BatchTask) * kv.second.size());
        pos += kv.second.size();
    }
    for (auto& kv : pclasses) {
        std::memcpy(host + o_task + pos * sizeof(int2), kv.second.data(), sizeof(int2) * kv.second.size());
        pos += kv.second.size();
    }
    if (!pps.empty()) std::memcpy(host + o_pp, pps.data(), sizeof(PassParams) * pps.size());
    hipError_t e = hipMemcpyAsync(d_ws, host, hdr, hipMemcpyHostToDevice, stream);
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
        b.co = std::get<3>(kv.first);
        b.nc = std::get<4>(kv.first);
        b.lds = 0;
        for (const BatchTask& t : kv.second) {
            const ImgParams& ip = h_imgs[t.img];
            b.lds = std::max(b.lds, b.co ? ip.lds_bytes + 4 * kBatchSlotWords : ip.lds_one);
        }
        // resident workgroups per CU are bounded by LDS (160 KiB per CU on
        // gfx950); extra workgroups only start late and find the list empty
        int per_cu = b.lds ? int((160u * 1024u) / b.lds) : 16;
        per_cu = std::max(1, std::min(per_cu, b.co ? 8 : 16));
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
    // two-pass images: every pass-A class, then every pass-B class (the map
    // orders the keys by pass first), so each image's pass B follows its A
    for (auto& kv : pclasses) {
        PassBatchLaunch b;
        b.pass = std::get<0>(kv.first);
        b.dtype = std::get<1>(kv.first);
        b.C = std::get<2>(kv.first);
        b.npl = std::get<3>(kv.first);
        b.kt = std::get<4>(kv.first);
        b.stages = std::get<5>(kv.first);
        b.tr = std::get<6>(kv.first);
        b.lds = plds[kv.first];
        b.d_pps = reinterpret_cast<const PassParams*>(ws + o_pp);
        b.d_tasks = reinterpret_cast<const int2*>(ws + o_task) + pos;
        b.ntasks = int(kv.second.size());
        const int rc = launch_pass_batch(b, stream);
        if (rc != RSG_OK) return rc;
        pos += kv.second.size();
    }
    return RSG_OK;
}

int launch_pass_batch(const PassBatchLaunch& b, hipStream_t stream)
{
    switch (b.dtype) {
    case RSG_U8: return launch_pass_batch_u8(b, stream);
    case RSG_F32: return launch_pass_batch_f32(b, stream);
    case RSG_F16: return launch_pass_batch_f16(b, stream);
    case RSG_BF16: return launch_pass_batch_bf16(b, stream);
    default: return set_error(RSG_EINVAL, "bad dtype %d", b.dtype);
    }
}

}  // namespace rsg
