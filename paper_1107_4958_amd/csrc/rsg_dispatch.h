// Host-side dispatch from a planned image (or batch class) to the kernel
// instantiation for its element type, channel count, scan chunk and tap
// count (fused kernel), or pass, chunk, staging and rows per workgroup
// (two-pass kernel).  Included once per element type so the instantiations
// compile in parallel translation units.
#pragma once

#include "rsg_device.h"
#include "rsg_twopass.h"

namespace rsg {
namespace dispatch {

// Row-scan layouts per channel count, matching scan_layout().
template <int C> struct Layouts {
    static constexpr int S[4] = {16, 32, 64, 64};
    static constexpr int N[4] = {C == 3 ? 12 : 8, C == 3 ? 12 : 8, C == 3 ? 12 : 8, C == 3 ? 24 : 16};
};

inline int set_lds_limit(const void* fn, uint32_t bytes)
{
    if (bytes <= 64u * 1024u) return RSG_OK;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) != hipSuccess)
        return set_error(RSG_EUNSUPPORTED, "device refuses %u bytes of LDS per workgroup", bytes);
    return RSG_OK;
}

template <class Tr, int C, int SEG, int NPL, int KT>
int launch_one(const ImgParams& ip, hipStream_t st)
{
    if (ip.co) {
        constexpr int NCW = wide_nc(C);
        if (ip.nc != 1 && ip.nc != NCW) return set_error(RSG_EINVAL, "no kernel for %d columns per lane", ip.nc);
        auto fn = (ip.nc == NCW) ? dev::k_single_co<Tr, C, SEG, NPL, KT, NCW> : dev::k_single_co<Tr, C, SEG, NPL, KT, 1>;
        int rc = set_lds_limit(reinterpret_cast<const void*>(fn), ip.lds_bytes);
        if (rc != RSG_OK) return rc;
        hipLaunchKernelGGL(fn, dim3(ip.ntasks), dim3(kCoWaves * kWave), ip.lds_bytes, st, ip);
        return RSG_OK;
    }
    auto fn = dev::k_single<Tr, C, SEG, NPL, KT>;
    int rc = set_lds_limit(reinterpret_cast<const void*>(fn), ip.lds_bytes);
    if (rc != RSG_OK) return rc;
    hipLaunchKernelGGL(fn, dim3(ip.ntasks), dim3(kWave), ip.lds_bytes, st, ip);
    return RSG_OK;
}

template <class Tr, int C, int SEG, int NPL>
int launch_k(const ImgParams& ip, hipStream_t st)
{
    switch (ip.kt) {
    case 3: return launch_one<Tr, C, SEG, NPL, 3>(ip, st);
    case 4: return launch_one<Tr, C, SEG, NPL, 4>(ip, st);
    case 5: return launch_one<Tr, C, SEG, NPL, 5>(ip, st);
    default: return set_error(RSG_EUNSUPPORTED, "no kernel for %d taps", ip.kt);
    }
}

template <class Tr, int C>
int launch_layout(const ImgParams& ip, hipStream_t st)
{
    using Lo = Layouts<C>;
    if (ip.seg == Lo::S[0] && ip.npl == Lo::N[0]) return launch_k<Tr, C, Lo::S[0], Lo::N[0]>(ip, st);
    if (ip.seg == Lo::S[1] && ip.npl == Lo::N[1]) return launch_k<Tr, C, Lo::S[1], Lo::N[1]>(ip, st);
    if (ip.seg == Lo::S[2] && ip.npl == Lo::N[2]) return launch_k<Tr, C, Lo::S[2], Lo::N[2]>(ip, st);
    if (ip.seg == Lo::S[3] && ip.npl == Lo::N[3]) return launch_k<Tr, C, Lo::S[3], Lo::N[3]>(ip, st);
    return set_error(RSG_EUNSUPPORTED, "no kernel for C=%d seg=%d npl=%d", C, ip.seg, ip.npl);
}

template <class Tr>
int launch_single_t(const ImgParams& ip, hipStream_t st)
{
    int rc;
    // channel-planar tasks run the kernel of one channel
    switch (ip.pstride > 1 ? 1 : ip.C) {
    case 1: rc = launch_layout<Tr, 1>(ip, st); break;
    case 2: rc = launch_layout<Tr, 2>(ip, st); break;
    case 3: rc = launch_layout<Tr, 3>(ip, st); break;
    case 4: rc = launch_layout<Tr, 4>(ip, st); break;
    default: return set_error(RSG_EINVAL, "bad channel count %d", ip.C);
    }
    if (rc != RSG_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(RSG_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return RSG_OK;
}

template <class Tr, int C, int KT>
int batch_one(const BatchClassLaunch& b, hipStream_t st)
{
    using Lo = Layouts<C>;
    if (b.co) {
        constexpr int NCW = wide_nc(C);
        if (b.nc != 1 && b.nc != NCW) return set_error(RSG_EINVAL, "no batch kernel for %d columns per lane", b.nc);
        auto fn = (b.nc == NCW) ? dev::k_batch_co<Tr, C, KT, NCW, Lo::S[0], Lo::N[0], Lo::S[1], Lo::N[1], Lo::S[2],
                                                  Lo::N[2], Lo::S[3], Lo::N[3]>
                                : dev::k_batch_co<Tr, C, KT, 1, Lo::S[0], Lo::N[0], Lo::S[1], Lo::N[1], Lo::S[2],
                                                  Lo::N[2], Lo::S[3], Lo::N[3]>;
        int rc = set_lds_limit(reinterpret_cast<const void*>(fn), b.lds);
        if (rc != RSG_OK) return rc;
        hipLaunchKernelGGL(fn, dim3(b.grid), dim3(kCoWaves * kWave), b.lds, st, b.d_imgs, b.d_tasks, b.ntasks,
                           b.d_counter);
        return RSG_OK;
    }
    auto fn = dev::k_batch<Tr, C, KT, Lo::S[0], Lo::N[0], Lo::S[1], Lo::N[1], Lo::S[2], Lo::N[2], Lo::S[3], Lo::N[3]>;
    int rc = set_lds_limit(reinterpret_cast<const void*>(fn), b.lds);
    if (rc != RSG_OK) return rc;
    hipLaunchKernelGGL(fn, dim3(b.grid), dim3(kWave), b.lds, st, b.d_imgs, b.d_tasks, b.ntasks, b.d_counter);
    return RSG_OK;
}

template <class Tr, int C>
int batch_k(const BatchClassLaunch& b, hipStream_t st)
{
    switch (b.kt) {
    case 3: return batch_one<Tr, C, 3>(b, st);
    case 4: return batch_one<Tr, C, 4>(b, st);
    case 5: return batch_one<Tr, C, 5>(b, st);
    default: return set_error(RSG_EUNSUPPORTED, "no batch kernel for %d taps", b.kt);
    }
}

template <class Tr>
int launch_batch_t(const BatchClassLaunch& b, hipStream_t st)
{
    int rc;
    switch (b.C) {
    case 1: rc = batch_k<Tr, 1>(b, st); break;
    case 2: rc = batch_k<Tr, 2>(b, st); break;
    case 3: rc = batch_k<Tr, 3>(b, st); break;
    case 4: rc = batch_k<Tr, 4>(b, st); break;
    default: return set_error(RSG_EINVAL, "bad channel count %d", b.C);
    }
    if (rc != RSG_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(RSG_EDEVICE, "batch launch failed: %s", hipGetErrorString(e));
    return RSG_OK;
}

// ---- two-pass path ----
template <class Tr> struct PassOutOf;
template <> struct PassOutOf<dev::TrU8> { static constexpr int v = dev::kOutU8; };
template <> struct PassOutOf<dev::TrF32> { static constexpr int v = dev::kOutF32; };
template <> struct PassOutOf<dev::TrF16> { static constexpr int v = dev::kOutF16; };
template <> struct PassOutOf<dev::TrBF16> { static constexpr int v = dev::kOutBF16; };

// A pass launch: one image (pb == nullptr) or a batch class; TR rows per workgroup.
template <class TrIn, int OUT, int C, int NPL, int KT, int ST, int TR>
int pass_one(const PassParams* pp, const PassBatchLaunch* pb, uint32_t lds, hipStream_t st)
{
    if (pb) {
        auto fn = dev::k_pass_batch<TrIn, OUT, C, NPL, KT, ST, TR>;
        int rc = set_lds_limit(reinterpret_cast<const void*>(fn), lds);
        if (rc != RSG_OK) return rc;
        hipLaunchKernelGGL(fn, dim3(pb->ntasks), dim3(TR * kWave), lds, st, pb->d_pps, pb->d_tasks);
        return RSG_OK;
    }
    auto fn = dev::k_pass<TrIn, OUT, C, NPL, KT, ST, TR>;
    int rc = set_lds_limit(reinterpret_cast<const void*>(fn), lds);
    if (rc != RSG_OK) return rc;
    const int grid = (pp->rows + TR - 1) / TR;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(TR * kWave), lds, st, *pp);
    return RSG_OK;
}

// 8-row workgroups exist for the wide multi-channel windows of pass A only (C >= 2)
template <class TrIn, int OUT, int C, int NPL, int KT, int ST>
int pass_tr(int tr, const PassParams* pp, const PassBatchLaunch* pb, uint32_t lds, hipStream_t st)
{
    if (tr == dev::kPassRows) return pass_one<TrIn, OUT, C, NPL, KT, ST, dev::kPassRows>(pp, pb, lds, st);
    if constexpr (C >= 2) {
        if (tr == 8) return pass_one<TrIn, OUT, C, NPL, KT, ST, 8>(pp, pb, lds, st);
    }
    return set_error(RSG_EUNSUPPORTED, "no pass kernel with %d rows per workgroup for C=%d", tr, C);
}

template <class TrIn, int OUT, int C, int NPL, int ST>
int pass_k(int kt, int tr, const PassParams* pp, const PassBatchLaunch* pb, uint32_t lds, hipStream_t st)
{
    switch (kt) {
    case 3: return pass_tr<TrIn, OUT, C, NPL, 3, ST>(tr, pp, pb, lds, st);
    case 4: return pass_tr<TrIn, OUT, C, NPL, 4, ST>(tr, pp, pb, lds, st);
    case 5: return pass_tr<TrIn, OUT, C, NPL, 5, ST>(tr, pp, pb, lds, st);
    default: return set_error(RSG_EUNSUPPORTED, "no pass kernel for %d taps", kt);
    }
}

// samples per lane: 8 or 16 (24 / 12 for three channels: whole pixels);
// one or two staging tiles
template <class TrIn, int OUT, int C>
int pass_npl(int npl, int stages, int kt, int tr, const PassParams* pp, const PassBatchLaunch* pb, uint32_t lds,
             hipStream_t st)
{
    constexpr int N0 = (C == 3) ? 12 : 8;
    constexpr int N1 = 2 * N0;
    if (npl == N0) return stages == 2 ? pass_k<TrIn, OUT, C, N0, 2>(kt, tr, pp, pb, lds, st)
                                      : pass_k<TrIn, OUT, C, N0, 1>(kt, tr, pp, pb, lds, st);
    if (npl == N1) return stages == 2 ? pass_k<TrIn, OUT, C, N1, 2>(kt, tr, pp, pb, lds, st)
                                      : pass_k<TrIn, OUT, C, N1, 1>(kt, tr, pp, pb, lds, st);
    return set_error(RSG_EUNSUPPORTED, "no pass kernel for %d samples per lane", npl);
}

// pass 0 (A: image -> intermediate) or 1 (B: intermediate -> image)
template <class Tr>
int pass_any(int pass, int C, int npl, int stages, int kt, int tr, const PassParams* pp, const PassBatchLaunch* pb,
             uint32_t lds, hipStream_t st)
{
    if (pass == 0) {
        constexpr int OUT = Tr::kInt ? dev::kOutMidU32 : dev::kOutMidF32;
        switch (C) {
        case 1: return pass_npl<Tr, OUT, 1>(npl, stages, kt, tr, pp, pb, lds, st);
        case 2: return pass_npl<Tr, OUT, 2>(npl, stages, kt, tr, pp, pb, lds, st);
        case 3: return pass_npl<Tr, OUT, 3>(npl, stages, kt, tr, pp, pb, lds, st);
        case 4: return pass_npl<Tr, OUT, 4>(npl, stages, kt, tr, pp, pb, lds, st);
        default: return set_error(RSG_EINVAL, "bad channel count %d", C);
        }
    }
    using Mid = typename std::conditional<Tr::kInt, dev::TrU32, dev::TrF32>::type;
    return pass_npl<Mid, PassOutOf<Tr>::v, 1>(npl, stages, kt, tr, pp, pb, lds, st);
}

template <class Tr>
int launch_pass_batch_t(const PassBatchLaunch& b, hipStream_t st)
{
    int rc = pass_any<Tr>(b.pass, b.C, b.npl, b.stages, b.kt, b.tr, nullptr, &b, b.lds, st);
    if (rc != RSG_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(RSG_EDEVICE, "pass launch failed: %s", hipGetErrorString(e));
    return RSG_OK;
}

template <class Tr>
int launch_pass_t(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t st)
{
    int rc = pass_any<Tr>(pass, ip.C, ip.pnpl[pass], ip.pst[pass], ip.kt, ip.ptr[pass], &pp, nullptr, ip.plds[pass],
                          st);
    if (rc != RSG_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(RSG_EDEVICE, "pass launch failed: %s", hipGetErrorString(e));
    return RSG_OK;
}

}  // namespace dispatch
}  // namespace rsg
