// Device code of the fused running-sum Gaussian filter for gfx950 (MI355X).
//
// One 64-lane wave owns one task: a strip of 64 consecutive sample-columns
// (lane l owns column s0 + l) and a segment of hs output rows of one image.
// It streams down the image in groups of G input rows:
//
//   row pass (Section 3.3, Eq. alg1 / indep, along x), per input row:
//     the row span [s0 - (R+1)C, s0 + 64 + RC) is loaded lane-contiguous
//     (lane l holds NPL consecutive samples; border samples extended by
//     replicate or zero), its running sum I is built with a serial per-lane
//     scan per channel plus a DPP scan of the lane totals and written to LDS;
//     each lane then takes T(s) = sum_k w_k (I(s + r_k C) - I(s - (r_k+1) C)).
//   column pass (Section 3.4, the same along y):
//     each lane adds T to its running column sum J, writes J to an LDS ring
//     holding the last 2R + 1 + G rows and emits, for the row R behind the
//     newest, out = sum_k w_k (J(y + r_k) - J(y - r_k - 1)).
//
// All G rows of a group are scanned before one barrier, so the LDS reads of
// the box differences issue back to back; the next group's global loads are
// in flight while the current group is processed.
//
// FP32 / FP16 / BF16 accumulate in FP32.  Running sums are tile-local and
// offset: each row subtracts its first span sample (added back through the
// DC gain of the boxes) and each column its first T value, which keeps the
// summed magnitudes, and hence the rounding of the differences, small.
// uint8 uses exact uint32 arithmetic (differences are exact modulo 2^32 and
// every box sum is < 2^32), integer weights m_k and one exact rounding of
// U / G^2.
//
// There is no MFMA: the method costs 4K additions and 2K multiplications per
// pixel (Table 1), far below the HBM ridge point.
#pragma once

#include <hip/hip_fp16.h>

#include "rsg_internal.h"

namespace rsg {
namespace dev {

// --------------------------------------------------------------------------
// DPP wave scans (gfx9 row_shr / row_bcast / wave_shr controls)
// --------------------------------------------------------------------------
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROWMASK, 0xf, true));
}

__device__ __forceinline__ uint32_t addv(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ float addv(float a, float b) { return a + b; }
__device__ __forceinline__ uint32_t bits(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t bits(float v) { return __float_as_uint(v); }
template <class T> __device__ __forceinline__ T frombits(uint32_t v);
template <> __device__ __forceinline__ uint32_t frombits<uint32_t>(uint32_t v) { return v; }
template <> __device__ __forceinline__ float frombits<float>(uint32_t v) { return __uint_as_float(v); }

// Exclusive prefix over the 64 lanes (lane 0 gets 0).
template <class T>
__device__ __forceinline__ T wave_exclusive_scan(T x)
{
    x = addv(x, frombits<T>(dpp<kDppRowShr1, 0xf>(bits(x))));
    x = addv(x, frombits<T>(dpp<kDppRowShr2, 0xf>(bits(x))));
    x = addv(x, frombits<T>(dpp<kDppRowShr4, 0xf>(bits(x))));
    x = addv(x, frombits<T>(dpp<kDppRowShr8, 0xf>(bits(x))));
    x = addv(x, frombits<T>(dpp<kDppRowBcast15, 0xa>(bits(x))));
    x = addv(x, frombits<T>(dpp<kDppRowBcast31, 0xc>(bits(x))));
    return frombits<T>(dpp<kDppWaveShr1, 0xf>(bits(x)));
}

// --------------------------------------------------------------------------
// Element types
// --------------------------------------------------------------------------
struct TrU8 {
    using In = uint8_t;
    using Acc = uint32_t;
    static constexpr int kSize = 1;
    static constexpr bool kInt = true;
    __device__ static Acc unpack(const uint32_t* w, int i) { return (w[i >> 2] >> (8 * (i & 3))) & 0xffu; }
    __device__ static uint32_t pack_raw(In v, int i) { return uint32_t(v) << (8 * (i & 3)); }
};
struct TrF32 {
    using In = float;
    using Acc = float;
    static constexpr int kSize = 4;
    static constexpr bool kInt = false;
    __device__ static Acc unpack(const uint32_t* w, int i) { return __uint_as_float(w[i]); }
    __device__ static uint32_t pack_raw(In v, int) { return __float_as_uint(v); }
    __device__ static void store(In* p, float v) { *p = v; }
};
struct TrF16 {
    using In = uint16_t;
    using Acc = float;
    static constexpr int kSize = 2;
    static constexpr bool kInt = false;
    __device__ static Acc unpack(const uint32_t* w, int i)
    {
        return __half2float(__ushort_as_half(uint16_t(w[i >> 1] >> (16 * (i & 1)))));
    }
    __device__ static uint32_t pack_raw(In v, int i) { return uint32_t(v) << (16 * (i & 1)); }
    __device__ static void store(In* p, float v) { *p = __half_as_ushort(__float2half_rn(v)); }
};
struct TrBF16 {
    using In = uint16_t;
    using Acc = float;
    static constexpr int kSize = 2;
    static constexpr bool kInt = false;
    __device__ static Acc unpack(const uint32_t* w, int i)
    {
        return __uint_as_float(((w[i >> 1] >> (16 * (i & 1))) & 0xffffu) << 16);
    }
    __device__ static uint32_t pack_raw(In v, int i) { return uint32_t(v) << (16 * (i & 1)); }
    __device__ static void store(In* p, float v)
    {
        const uint32_t u = __float_as_uint(v);                       // finite v
        *p = uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);       // round to nearest even
    }
};

__device__ __forceinline__ int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// Raw chunk of NPL samples held in 32-bit words until it is consumed.
template <class Tr, int NPL>
struct Chunk {
    static constexpr int kBytes = NPL * Tr::kSize;
    static constexpr int kWords = (kBytes + 3) / 4;
    uint32_t w[kWords];
};

// Load this lane's chunk of one row.  `cs` is the chunk's first sample
// (row-relative, a multiple of C); WC = W*C.
template <class Tr, int C, int NPL>
__device__ __forceinline__ void load_chunk(Chunk<Tr, NPL>& ch, const typename Tr::In* rowp, int cs, int WC,
                                           int W, bool vec, bool replicate)
{
    constexpr int kBytes = Chunk<Tr, NPL>::kBytes;
    if (vec && cs >= 0 && cs + NPL <= WC) {
        const char* p = reinterpret_cast<const char*>(rowp + cs);
        if constexpr (kBytes % 16 == 0) {
#pragma unroll
            for (int k = 0; k < kBytes / 16; ++k) {
                const uint4 v = *reinterpret_cast<const uint4*>(p + 16 * k);
                ch.w[4 * k + 0] = v.x; ch.w[4 * k + 1] = v.y; ch.w[4 * k + 2] = v.z; ch.w[4 * k + 3] = v.w;
            }
        } else if constexpr (kBytes % 8 == 0) {
#pragma unroll
            for (int k = 0; k < kBytes / 8; ++k) {
                const uint2 v = *reinterpret_cast<const uint2*>(p + 8 * k);
                ch.w[2 * k + 0] = v.x; ch.w[2 * k + 1] = v.y;
            }
        } else if constexpr (kBytes % 4 == 0) {
#pragma unroll
            for (int k = 0; k < kBytes / 4; ++k) ch.w[k] = *reinterpret_cast<const uint32_t*>(p + 4 * k);
        } else {   // 2-byte granules (uint8 with NPL = 2, 6, ...)
#pragma unroll
            for (int k = 0; k < Chunk<Tr, NPL>::kWords; ++k) ch.w[k] = 0;
#pragma unroll
            for (int k = 0; k < kBytes / 2; ++k)
                ch.w[k >> 1] |= uint32_t(*reinterpret_cast<const uint16_t*>(p + 2 * k)) << (16 * (k & 1));
        }
        return;
    }
    // border or unaligned rows: one element at a time, extended per boundary
#pragma unroll
    for (int k = 0; k < Chunk<Tr, NPL>::kWords; ++k) ch.w[k] = 0;
    const int x0 = floor_div(cs, C);
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        int x = x0 + i / C;
        const int c = i % C;
        bool inside = (x >= 0 && x < W);
        if (!inside && replicate) { x = x < 0 ? 0 : W - 1; inside = true; }
        if (inside) ch.w[(i * Tr::kSize) / 4] |= Tr::pack_raw(rowp[x * C + c], i);
    }
}

// uint8 output: round half up of U / G^2, exactly.  N = U + floor(G^2/2) < 256 G^2.
__device__ __forceinline__ uint32_t exact_round_div(uint64_t U, const ImgParams& ip)
{
    const uint64_t N = U + ip.G2half;
    const float nf = float(uint32_t(N >> 32)) * 4294967296.0f + float(uint32_t(N));
    uint32_t q = uint32_t(nf * ip.invG2);
    const uint64_t prod = uint64_t(q) * ip.G2;
    if (prod > N) q -= 1;
    else if (N - prod >= ip.G2) q += 1;
    return q;
}

// Rows per group: keep two groups of raw chunks within ~64 VGPRs.
template <int NPL, int SIZE>
struct GroupRows {
    static constexpr int kWords = (NPL * SIZE + 3) / 4;
    static constexpr int value = kWords <= 4 ? 8 : (kWords <= 8 ? 4 : 2);
};

// --------------------------------------------------------------------------
// One task: 64 sample-columns x hs output rows.
// --------------------------------------------------------------------------
template <class Tr, int C, int NPL, int KT>
__device__ __forceinline__ void run_task(const ImgParams& ip, int task, uint32_t* lds)
{
    using In = typename Tr::In;
    using Acc = typename Tr::Acc;
    constexpr bool kInt = Tr::kInt;
    constexpr int G = GroupRows<NPL, Tr::kSize>::value;
    constexpr int PW = kWave * NPL;           // LDS width of one running-sum row
    const int lane = threadIdx.x;
    const int WC = ip.W * C;
    const int strip = task % ip.nstrips;
    const int seg = task / ip.nstrips;
    const int s0 = strip * kWave;
    const int y0 = seg * ip.hs;
    const int hs = min(ip.hs, ip.H - y0);
    const int R = ip.R;
    const int L = ip.L;
    const int H = ip.H;
    const bool replicate = (ip.boundary == RSG_REPLICATE);
    const bool vec = ip.vec != 0;

    const int a0 = floor_div(s0 - (R + 1) * C, ip.align) * ip.align;
    const int off = s0 - a0;                  // span index of this strip's first sample
    const int cs = a0 + NPL * lane;           // this lane's chunk

    Acc* P = reinterpret_cast<Acc*>(lds);     // G rows x PW
    Acc* ring = P + G * PW;                   // L rows x 64

    int tp[KT], tm[KT];                       // LDS indices of the box ends
    float wf[KT];
    uint32_t wm[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        tp[k] = off + lane + ip.r[k] * C;
        tm[k] = off + lane - (ip.r[k] + 1) * C;
        wf[k] = ip.wf[k];
        wm[k] = ip.m[k];
    }
    const float dc = ip.dc32;

    const In* src = reinterpret_cast<const In*>(ip.src);
    In* dst = reinterpret_cast<In*>(ip.dst);
    const int s = s0 + lane;                  // this lane's column
    const bool s_ok = s < WC;

    const int niter = 2 * R + 1 + hs;
    const int ngroups = (niter + G - 1) / G;
    const int ybase = y0 - R - 1;

    auto load_group = [&](Chunk<Tr, NPL>* buf, int g) {
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int it = g * G + j;
            if (it < niter) {
                int y = ybase + it;
                const bool inside = (y >= 0 && y < H);
                if (inside || replicate) {
                    y = y < 0 ? 0 : (y >= H ? H - 1 : y);
                    load_chunk<Tr, C, NPL>(buf[j], src + int64_t(y) * ip.src_stride, cs, WC, ip.W, vec, replicate);
                }
            }
        }
    };

    Chunk<Tr, NPL> nxt[G];
    load_group(nxt, 0);

    Acc colacc = Acc(0);
    float c2 = 0.0f;                          // column offset (float types)
    int slot0 = 0;                            // ring slot of the group's first row

    for (int g = 0; g < ngroups; ++g) {
        Chunk<Tr, NPL> cur[G];
#pragma unroll
        for (int j = 0; j < G; ++j) cur[j] = nxt[j];
        if (g + 1 < ngroups) load_group(nxt, g + 1);
        const int it0 = g * G;

        // ---- row running sums of the group (Eq. alg1) ----
        float rowoff[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            rowoff[j] = 0.0f;
            const int it = it0 + j;
            const int y = ybase + it;
            const bool live = (it < niter) && (replicate || (y >= 0 && y < H));
            if (live) {
                Acc v[NPL];
#pragma unroll
                for (int i = 0; i < NPL; ++i) v[i] = Tr::unpack(cur[j].w, i);
                if constexpr (!kInt) {
                    // offset: the span sample held first by the lane at the strip start
                    const float c = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v[0]), off / NPL));
                    rowoff[j] = c;
#pragma unroll
                    for (int i = 0; i < NPL; ++i) v[i] -= c;
                }
#pragma unroll
                for (int i = C; i < NPL; ++i) v[i] = v[i] + v[i - C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const Acc ex = wave_exclusive_scan<Acc>(v[NPL - C + c]);
#pragma unroll
                    for (int i = c; i < NPL; i += C) v[i] = v[i] + ex;
                }
#pragma unroll
                for (int i = 0; i < NPL; ++i) P[j * PW + lane * NPL + i] = v[i];
            }
        }
        __syncthreads();

        // ---- box differences along the row (Eq. indep) ----
        Acc T[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int it = it0 + j;
            const int y = ybase + it;
            const bool live = (it < niter) && (replicate || (y >= 0 && y < H));
            Acc t = Acc(0);
            if (live) {
                const Acc* Pj = P + j * PW;
                if constexpr (kInt) {
#pragma unroll
                    for (int k = 0; k < KT; ++k) t += __umul24(wm[k], Pj[tp[k]] - Pj[tm[k]]);
                } else {
                    t = rowoff[j] * dc;
#pragma unroll
                    for (int k = 0; k < KT; ++k) t = fmaf(wf[k], Pj[tp[k]] - Pj[tm[k]], t);
                }
            }
            T[j] = t;
        }

        // ---- running sums down the columns, into the ring (Eq. alg1) ----
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int it = it0 + j;
            if (it < niter) {
                if constexpr (kInt) {
                    colacc += T[j];
                } else {
                    if (it == 0) c2 = T[j];
                    colacc += T[j] - c2;
                }
                int sl = slot0 + j;
                sl -= (sl >= L) ? L : 0;
                ring[sl * kWave + lane] = colacc;
            }
        }

        // ---- box differences down the columns, for row y - R (Eq. indep) ----
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int it = it0 + j;
            if (it < niter && it >= 2 * R + 1) {
                int sl = slot0 + j;
                sl -= (sl >= L) ? L : 0;
                const int yo = ybase + it - R;
                In* orow = dst + int64_t(yo) * ip.dst_stride;
                if constexpr (kInt) {
                    uint64_t U = 0;
#pragma unroll
                    for (int k = 0; k < KT; ++k) {
                        int a = sl - R + ip.r[k];
                        int b = sl - R - ip.r[k] - 1;
                        a += (a < 0) ? L : 0;
                        b += (b < 0) ? L : 0;
                        U += uint64_t(wm[k]) * uint32_t(ring[a * kWave + lane] - ring[b * kWave + lane]);
                    }
                    if (s_ok) orow[s] = In(exact_round_div(U, ip));
                } else {
                    float o = c2 * dc;
#pragma unroll
                    for (int k = 0; k < KT; ++k) {
                        int a = sl - R + ip.r[k];
                        int b = sl - R - ip.r[k] - 1;
                        a += (a < 0) ? L : 0;
                        b += (b < 0) ? L : 0;
                        o = fmaf(wf[k], ring[a * kWave + lane] - ring[b * kWave + lane], o);
                    }
                    if (s_ok) Tr::store(orow + s, o);
                }
            }
        }
        slot0 += G;
        slot0 -= (slot0 >= L) ? L : 0;
    }
}

// Task order: blocks are dealt to the 8 XCDs round-robin; give each XCD a
// contiguous range of tasks (a horizontal band of strips) so strips that
// share halo columns share an L2.
__device__ __forceinline__ int xcd_task(int b, int n)
{
    const int x = b % kXcds;
    const int i = b / kXcds;
    const int q = n / kXcds;
    const int rem = n % kXcds;
    return x * q + min(x, rem) + i;
}

template <class Tr, int C, int NPL, int KT>
__global__ __launch_bounds__(64) void k_single(ImgParams ip)
{
    extern __shared__ uint32_t lds[];
    run_task<Tr, C, NPL, KT>(ip, xcd_task(blockIdx.x, ip.ntasks), lds);
}

// Persistent batch kernel for one (dtype, C, K) class: each wave pops
// (image, task) items off a shared counter until the list is exhausted.
template <class Tr, int C, int KT, int N0, int N1, int N2, int N3>
__global__ __launch_bounds__(64) void k_batch(const ImgParams* __restrict__ imgs,
                                              const BatchTask* __restrict__ tasks, int ntasks,
                                              unsigned* __restrict__ counter)
{
    extern __shared__ uint32_t lds[];
    for (;;) {
        unsigned t = 0;
        if (threadIdx.x == 0) t = atomicAdd(counter, 1u);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
        if (t >= unsigned(ntasks)) break;
        const BatchTask bt = tasks[t];
        const ImgParams& ip = imgs[bt.img];
        const int npl = ip.npl;
        if (npl == N0) run_task<Tr, C, N0, KT>(ip, bt.task, lds);
        else if (N1 && npl == N1) run_task<Tr, C, (N1 ? N1 : N0), KT>(ip, bt.task, lds);
        else if (N2 && npl == N2) run_task<Tr, C, (N2 ? N2 : N0), KT>(ip, bt.task, lds);
        else if (N3 && npl == N3) run_task<Tr, C, (N3 ? N3 : N0), KT>(ip, bt.task, lds);
        __syncthreads();
    }
}

}  // namespace dev
}  // namespace rsg
