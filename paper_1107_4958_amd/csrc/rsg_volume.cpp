// Volumes: the separable filter of Sections 3.3-3.4 with one more pass per
// extra axis (Section 4's d-dimensional remark).  Every z-slice is filtered
// along x and y into a stream-ordered FP32 intermediate: one fused launch
// over the stack of slices (all slices share one plan), or for wide boxes
// the batched two-pass path.  Then the z pass (rsg_zpass.h) filters the
// intermediate along z into the destination.
#include "rsg_internal.h"

#include <algorithm>
#include <cstring>
#include <vector>

extern "C" int rsg_gauss_filter_3d(const void* d_src, void* d_dst, int D, int H, int W, int C, rsg_dtype dt,
                                   double sigma, int K, const rsg_boxes* boxes, rsg_boundary b, void* stream)
{
    using namespace rsg;
    if (!d_src || !d_dst) return set_error(RSG_EINVAL, "NULL volume pointer");
    if (D < 1) return set_error(RSG_EINVAL, "D must be >= 1 (got %d)", D);
    if (dt != RSG_F32) return set_error(RSG_EUNSUPPORTED, "volumes are filtered in FP32 only");
    if (H < 1 || W < 1 || C < 1 || C > 4) return set_error(RSG_EINVAL, "bad slice shape %d x %d x %d", H, W, C);
    const int64_t plane = int64_t(H) * W * C;
    const int64_t total = plane * D;
    if (total > (int64_t(1) << 40)) return set_error(RSG_EUNSUPPORTED, "volume too large");
    const int64_t ncols = (plane + kWave - 1) / kWave;
    if (ncols > (int64_t(1) << 28)) return set_error(RSG_EUNSUPPORTED, "slice too large");
    {
        const char* s0 = static_cast<const char*>(d_src);
        const char* t0 = static_cast<const char*>(d_dst);
        if (s0 < t0 + total * 4 && t0 < s0 + total * 4) return set_error(RSG_EINVAL, "source and destination overlap");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);

    // plan the slices (src slice -> intermediate slice); the plan validates
    // sigma, K, the boxes and the boundary
    void* mid = nullptr;
    if (hipMallocAsync(&mid, size_t(total) * 4, st) != hipSuccess)
        return set_error(RSG_ENOMEM, "cannot allocate the %lld-byte intermediate of the volume",
                         (long long)(total * 4));
    std::vector<rsg_image_desc> descs(D);
    for (int z = 0; z < D; ++z) {
        rsg_image_desc& d = descs[z];
        d.src = static_cast<const char*>(d_src) + plane * z * 4;
        d.dst = static_cast<char*>(mid) + plane * z * 4;
        d.H = H;
        d.W = W;
        d.C = C;
        d.src_stride = 0;
        d.dst_stride = 0;
        d.dt = RSG_F32;
        d.sigma = boxes ? boxes->sigma : sigma;
        d.K = boxes ? boxes->K : K;
        d.b = b;
        d.boxes = boxes;
    }
    // Segments: the slices already give the launch its parallelism, so each
    // task takes a whole slice column (halo 2R + 1 rows per H rows) unless
    // the volume has too few strips to fill the device.
    const int64_t strips = int64_t(D) * ((int64_t(W) * C + kWave - 1) / kWave);
    const int64_t per_strip = std::max<int64_t>(1, (1024 + strips - 1) / strips);
    const int hs_pref = int(std::max<int64_t>(16, (H + per_strip - 1) / per_strip));
    std::vector<ImgParams> imgs(1);
    std::vector<BatchTask> tasks;
    int rc = plan_image(descs[0], &imgs[0], 1, hs_pref, false);   // the stack takes the slice index
    void* ws = nullptr;
    size_t ws_bytes = 0;
    if (rc == RSG_OK && imgs[0].path == kPathFused && int64_t(imgs[0].ntasks) * D <= (int64_t(1) << 30)) {
        ImgParams stack = imgs[0];             // one launch over the stack of slices
        stack.nslices = D;
        stack.slice_stride = plane;
        stack.ntasks = imgs[0].ntasks * D;
        rc = launch_single(stack, st);
    } else if (rc == RSG_OK) {                 // two-pass slices: the batched path
        rc = plan_batch(descs.data(), D, imgs, tasks, hs_pref);
        if (rc == RSG_OK) {
            ws_bytes = batch_workspace_bytes(imgs.data(), D, int64_t(tasks.size()) + pass_blocks(imgs.data(), D));
            if (hipMallocAsync(&ws, ws_bytes, st) != hipSuccess)
                rc = set_error(RSG_ENOMEM, "cannot allocate the %zu-byte slice workspace", ws_bytes);
        }
        if (rc == RSG_OK)
            rc = launch_batch(imgs.data(), D, tasks.data(), int(tasks.size()), ws, ws_bytes, st, nullptr);
    }

    if (rc == RSG_OK) {                        // the z pass, intermediate -> destination
        const ImgParams& ip = imgs[0];
        ZParams zp;
        std::memset(&zp, 0, sizeof(zp));
        zp.src = static_cast<const float*>(mid);
        zp.dst = static_cast<float*>(d_dst);
        zp.plane = plane;
        zp.D = D;
        zp.R = ip.R;
        zp.L = 2 * ip.R + 2;
        zp.boundary = b;
        for (int k = 0; k < RSG_MAX_K; ++k) {
            zp.r[k] = ip.r[k];
            zp.wf[k] = ip.wf[k];
        }
        zp.dc32 = ip.dc32;
        zp.ncols = int(ncols);
        // enough tasks to fill the device (about 8192: fewer, longer segments
        // pay less halo and measured faster than 16384), segments no shorter
        // than needed
        const int64_t target = 8192;
        int64_t nsegs = std::max<int64_t>(1, std::min<int64_t>((target + ncols - 1) / ncols, (D + 7) / 8));
        zp.hz = int((D + nsegs - 1) / nsegs);
        nsegs = (D + zp.hz - 1) / zp.hz;
        if (ncols * nsegs > (int64_t(1) << 30)) {
            rc = set_error(RSG_EUNSUPPORTED, "too many z-pass tasks");
        } else {
            zp.ntasks = int(ncols * nsegs);
            const int64_t per_wave = int64_t(zp.L) * kWave * 4;
            if (per_wave > 160 * 1024) {
                rc = set_error(RSG_EUNSUPPORTED, "z pass: box half-width %d needs more LDS than a workgroup has", ip.R);
            } else {
                const int wpb = int(std::max<int64_t>(1, std::min<int64_t>(4, (160 * 1024) / per_wave)));
                rc = launch_zpass_f32(zp, ip.kt, wpb, st);
            }
        }
    }
    if (ws && hipFreeAsync(ws, st) != hipSuccess && rc == RSG_OK)
        rc = set_error(RSG_EDEVICE, "cannot release the slice workspace");
    if (hipFreeAsync(mid, st) != hipSuccess && rc == RSG_OK)
        rc = set_error(RSG_EDEVICE, "cannot release the volume intermediate");
    return rc;
}
