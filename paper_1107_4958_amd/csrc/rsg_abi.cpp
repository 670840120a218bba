// C ABI entry points (include/rsg.h).  Marshalling and validation only; the
// filtering runs in the kernels of rsg_device.h, rsg_twopass.h and
// rsg_zpass.h (instantiated in rsg_k_*.hip), the fit in rsg_fit.cpp, volumes
// in rsg_volume.cpp and serving in rsg_server.cpp.
#include "rsg_internal.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

namespace rsg {

namespace {
thread_local std::string g_last_error;
}

int set_error(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// Plans every image and builds the flat work list of a batched launch.
int plan_batch(const rsg_image_desc* d, int n, std::vector<ImgParams>& imgs, std::vector<BatchTask>& tasks,
               int hs_pref)
{
    if (!d || n < 1) return set_error(RSG_EINVAL, "batch needs n >= 1 descriptors");
    imgs.resize(n);
    tasks.clear();
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        int rc = plan_image(d[i], &imgs[i], 1, hs_pref);
        if (rc != RSG_OK) {
            std::string msg = g_last_error;
            return set_error(rc, "image %d: %s", i, msg.c_str());
        }
        total += imgs[i].ntasks;                  // fused tasks or two-pass row blocks
    }
    // uint8 results are exact integers whatever the segment height, so a batch
    // may give its fused uint8 images longer segments (fewer halo rows) as
    // long as the batch keeps enough tasks to fill the device; float images
    // keep their own plan (their rounding follows the segment boundaries)
    if (hs_pref <= 0) {
        constexpr int64_t kTarget = 4096;
        int64_t fixed = 0, strips = 0;
        for (int i = 0; i < n; ++i) {
            if (imgs[i].path != kPathFused) continue;
            if (imgs[i].dtype == RSG_U8) strips += int64_t(imgs[i].nstrips) * std::max(1, imgs[i].nslices);
            else fixed += imgs[i].ntasks;
        }
        if (strips > 0) {
            const int64_t segs = std::max<int64_t>(1, (kTarget - fixed + strips - 1) / strips);
            for (int i = 0; i < n; ++i) {
                ImgParams& ip = imgs[i];
                if (ip.path != kPathFused || ip.dtype != RSG_U8) continue;
                const int hs = int(std::max<int64_t>(ip.hs, (ip.H + segs - 1) / segs));
                if (hs == ip.hs) continue;
                ImgParams longer;
                if (plan_image(d[i], &longer, 1, hs) == RSG_OK && longer.path == kPathFused) {
                    total += int64_t(longer.ntasks) - ip.ntasks;
                    ip = longer;
                }
            }
        }
    }
    if (total > (int64_t(1) << 30)) return set_error(RSG_EUNSUPPORTED, "batch too large");
    tasks.reserve(size_t(total));
    // queue the longest tasks first (rows streamed x row span scanned per
    // task), so the last workgroups to finish run short tasks; per-image
    // results do not depend on the order
    auto task_cost = [&](int i) {
        const ImgParams& ip = imgs[i];
        const int64_t cols = int64_t(kWave) * std::max(1, ip.nc) + int64_t(2 * ip.R + 1) * (ip.pstride > 1 ? 1 : ip.C);
        return int64_t(std::min(ip.hs, ip.H) + 2 * ip.R + 1) * cols;
    };
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return task_cost(a) > task_cost(b); });
    for (int i : order)
        if (imgs[i].path == kPathFused)       // two-pass images are launched on their own
            for (int t = 0; t < imgs[i].ntasks; ++t) tasks.push_back(BatchTask{i, t});
    return RSG_OK;
}

}  // namespace rsg

extern "C" {

int rsg_plan_shape(const rsg_image_desc* d, int32_t* seg_height, int32_t* tasks, uint32_t* lds_bytes)
{
    using namespace rsg;
    if (!d) return set_error(RSG_EINVAL, "rsg_plan_shape: NULL descriptor");
    ImgParams ip;
    const int rc = plan_image(*d, &ip);
    if (rc != RSG_OK) return rc;
    if (seg_height) *seg_height = ip.hs;
    if (tasks) *tasks = ip.ntasks;
    if (lds_bytes) *lds_bytes = ip.lds_bytes;
    return RSG_OK;
}

int rsg_tune_path(int32_t path)
{
    using namespace rsg;
    if (path < 0 || path > 3)
        return set_error(RSG_EINVAL, "path must be 0 (planner), 1 (fused), 2 (two-pass) or 3 (fused, one wave per task)");
    set_path_override(path);
    return RSG_OK;
}

int rsg_tune_columns(int32_t columns)
{
    using namespace rsg;
    if (columns < 0 || columns > 3)
        return set_error(RSG_EINVAL, "task form must be 0 (planner), 1 (one column), 2 (wide) or 3 (channel-planar)");
    set_nc_override(columns);
    return RSG_OK;
}

int rsg_tune_layout(int32_t first)
{
    using namespace rsg;
    if (first < 0 || first >= kLayouts) return set_error(RSG_EINVAL, "layout must be in 0..%d", kLayouts - 1);
    set_layout_override(first);
    return RSG_OK;
}

int rsg_tune_stores(int32_t form)
{
    using namespace rsg;
    if (form < 0 || form > 2)
        return set_error(RSG_EINVAL, "store form must be 0 (planner), 1 (one per lane and row) or 2 (staged)");
    set_stores_override(form);
    return RSG_OK;
}

int rsg_tune_override(int32_t seg_height)
{
    using namespace rsg;
    if (seg_height < 0) return set_error(RSG_EINVAL, "segment height must be >= 0");
    set_hs_override(seg_height);
    return RSG_OK;
}

int rsg_fit_boxes(double sigma, int K, rsg_boxes* out)
{
    return rsg::make_boxes(sigma, K, RSG_FIT_SCALED, out);
}

int rsg_fit_boxes_ex(double sigma, int K, rsg_fit_method method, rsg_boxes* out)
{
    return rsg::make_boxes(sigma, K, int(method), out);
}

int rsg_gauss_filter(const void* d_src, void* d_dst, int H, int W, int C, rsg_dtype dt, double sigma,
                     int K, rsg_boundary b, void* stream)
{
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
    rsg::ImgParams ip;
    int rc = rsg::plan_image(d, &ip);
    if (rc != RSG_OK) return rc;
    return rsg::launch_single(ip, static_cast<hipStream_t>(stream));
}

int rsg_gauss_filter_strided(const void* d_src, void* d_dst, int H, int W, int C, rsg_dtype dt, double sigma,
                             int K, const rsg_boxes* boxes, rsg_boundary b, int step, void* stream)
{
    rsg_image_desc d;
    d.src = d_src;
    d.dst = d_dst;
    d.H = H;
    d.W = W;
    d.C = C;
    d.src_stride = 0;
    d.dst_stride = 0;
    d.dt = dt;
    d.sigma = boxes ? boxes->sigma : sigma;
    d.K = boxes ? boxes->K : K;
    d.b = b;
    d.boxes = boxes;
    rsg::ImgParams ip;
    int rc = rsg::plan_image(d, &ip, step);
    if (rc != RSG_OK) return rc;
    return rsg::launch_single(ip, static_cast<hipStream_t>(stream));
}

int rsg_box_filter(const void* d_src, void* d_dst, int H, int W, int C, rsg_dtype dt, const rsg_boxes* boxes,
                   rsg_boundary b, void* stream)
{
    if (!boxes) return rsg::set_error(RSG_EINVAL, "boxes is NULL");
    rsg_image_desc d;
    d.src = d_src;
    d.dst = d_dst;
    d.H = H;
    d.W = W;
    d.C = C;
    d.src_stride = 0;
    d.dst_stride = 0;
    d.dt = dt;
    d.sigma = boxes->sigma;
    d.K = boxes->K;
    d.b = b;
    d.boxes = boxes;
    rsg::ImgParams ip;
    int rc = rsg::plan_image(d, &ip);
    if (rc != RSG_OK) return rc;
    return rsg::launch_single(ip, static_cast<hipStream_t>(stream));
}

int rsg_filter_batch_workspace(const rsg_image_desc* d, int n, size_t* bytes)
{
    if (!bytes) return rsg::set_error(RSG_EINVAL, "bytes is NULL");
    std::vector<rsg::ImgParams> imgs;
    std::vector<rsg::BatchTask> tasks;
    int rc = rsg::plan_batch(d, n, imgs, tasks);
    if (rc != RSG_OK) return rc;
    *bytes = rsg::batch_workspace_bytes(imgs.data(), n, int64_t(tasks.size()) + rsg::pass_blocks(imgs.data(), n));
    return RSG_OK;
}

int rsg_filter_batch(const rsg_image_desc* d, int n, void* d_workspace, size_t ws_bytes, void* stream)
{
    if (!d_workspace) return rsg::set_error(RSG_EINVAL, "workspace is NULL");
    std::vector<rsg::ImgParams> imgs;
    std::vector<rsg::BatchTask> tasks;
    int rc = rsg::plan_batch(d, n, imgs, tasks);
    if (rc != RSG_OK) return rc;
    return rsg::launch_batch(imgs.data(), n, tasks.data(), int(tasks.size()), d_workspace, ws_bytes,
                             static_cast<hipStream_t>(stream));
}

const char* rsg_last_error(void)
{
    return rsg::g_last_error.c_str();
}

}  // extern "C"
