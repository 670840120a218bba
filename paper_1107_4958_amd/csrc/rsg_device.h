// Device code of the fused running-sum Gaussian filter for gfx950 (MI355X).
//
// A task is a strip of 64 consecutive sample-columns (lane c owns column
// s0 + c in the column pass) and a segment of hs output rows of one image.
// It streams down the image in groups of G input rows, either on one wave
// (both passes, software-pipelined: stream_task) or on a workgroup of
// kCoWaves waves that split every step of rows between them, each running
// both passes on its own block and exchanging the column sums' carries
// through LDS (stream_task_co, the default):
//
//   row pass (Section 3.3, Eq. alg1 / indep, along x): the wave splits into
//     G = 64 / SEG segments of SEG lanes; segment j takes one input row,
//     lane q of the segment holds NPL consecutive samples of the row span
//     [s0 - (R+1)C, s0 + 64 + RC) (border samples replicated, reflected or
//     zero).  The running sum I of each row is a serial scan inside the lane
//     plus a DPP scan of the lane totals across the segment; the G rows of
//     running sums go to LDS.  Then every lane (now: a column) takes
//     T(s) = sum_k w_k (I(s + r_k C) - I(s - (r_k+1) C)) for each row.
//   column pass (Section 3.4, the same along y): running column sums J of T
//     in an LDS ring holding at least the last 2R + 2 rows, and for the row R
//     behind each summed row out = sum_k w_k (J(y + r_k) - J(y - r_k - 1)).
//
// Global memory is addressed through buffer descriptors with row offsets in
// SGPRs: border zero-padding and dropped stores (rows outside the task, lanes
// past the image) use an out-of-range offset instead of branches, so every
// step issues a fixed number of memory instructions and the next steps'
// loads stay in flight while the current one is processed.
//
// FP32 / FP16 / BF16 accumulate in FP32.  Running sums are tile-local and
// offset: each group of rows subtracts one of its samples (added back
// through the DC gain of the boxes) and each column a constant of its own,
// which keeps the summed magnitudes, and hence the rounding of the
// differences, small.  Zero extension takes no offsets: outside samples must
// enter the sums as 0, or a box lying mostly outside the image would be a
// small difference of large sums.  uint8 uses exact uint32 arithmetic
// (differences are exact modulo 2^32 and every box sum is < 2^32), integer
// weights m_k, a uint64 column combine and one exact integer rounding of
// U / G^2.
//
// There is no MFMA: the method costs 4K additions and 2K multiplications per
// pixel (Table 1), far below the HBM ridge point.
#pragma once

#include <hip/hip_fp16.h>

#include <type_traits>

#include "rsg_internal.h"

namespace rsg {
namespace dev {

// Cache policy of the output stores.  The output is written once and never
// read back by the kernel: where a wave's store of a row covers whole 128-byte
// lines (two or more bytes per lane), it streams past the caches
// (non-temporal), which keeps the input's halo rows and shared span columns
// resident in L2 (4096^2 FP32: 45.8 -> 43.6 us; non-temporal loads instead
// cost 30 %).  Byte-per-lane stores (uint8, one column per lane) stay cached,
// so that the L2 merges their 64-byte pieces before they reach memory
// (non-temporal, they wrote 1.4 x the output bytes).
constexpr int kStoreNT = 2;
template <int BYTES_PER_LANE> constexpr int kStorePolicy = (BYTES_PER_LANE >= 2) ? kStoreNT : 0;

typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v3u __attribute__((ext_vector_type(3)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------------------
// DPP (gfx9 row_shr / row_bcast controls)
// --------------------------------------------------------------------------
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppRowNewBcast7 = 0x157;     // gfx90a+: every lane of a 16-lane row reads lane 7 of it

// Lanes in rows / banks masked off receive 0.
template <int CTRL, int ROWMASK, int BANKMASK = 0xf>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROWMASK, BANKMASK, true));
}

__device__ __forceinline__ uint32_t addv(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ float addv(float a, float b) { return a + b; }
__device__ __forceinline__ uint32_t subv(uint32_t a, uint32_t b) { return a - b; }
__device__ __forceinline__ float subv(float a, float b) { return a - b; }
__device__ __forceinline__ uint32_t bits(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t bits(float v) { return __float_as_uint(v); }
template <class T> __device__ __forceinline__ T frombits(uint32_t v);
template <> __device__ __forceinline__ uint32_t frombits<uint32_t>(uint32_t v) { return v; }
template <> __device__ __forceinline__ float frombits<float>(uint32_t v) { return __uint_as_float(v); }

// Inclusive scan across segments of SEG lanes (8, 16, 32 or 64).
template <int SEG, class T>
__device__ __forceinline__ T segment_inclusive_scan(T x)
{
    x = addv(x, frombits<T>(dpp<kDppRowShr1, 0xf>(bits(x))));
    x = addv(x, frombits<T>(dpp<kDppRowShr2, 0xf>(bits(x))));
    x = addv(x, frombits<T>(dpp<kDppRowShr4, 0xf>(bits(x))));
    x = addv(x, frombits<T>(dpp<kDppRowShr8, 0xf>(bits(x))));
    // 8-lane segments: lanes 8..15 of each row drop the total of lanes 0..7 (banks 2 and 3 only)
    if constexpr (SEG == 8) x = subv(x, frombits<T>(dpp<kDppRowNewBcast7, 0xf, 0xc>(bits(x))));
    if constexpr (SEG >= 32) x = addv(x, frombits<T>(dpp<kDppRowBcast15, 0xa>(bits(x))));
    if constexpr (SEG >= 64) x = addv(x, frombits<T>(dpp<kDppRowBcast31, 0xc>(bits(x))));
    return x;
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
};
struct TrF32 {
    using In = float;
    using Acc = float;
    static constexpr int kSize = 4;
    static constexpr bool kInt = false;
    __device__ static Acc unpack(const uint32_t* w, int i) { return __uint_as_float(w[i]); }
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
};

__device__ __forceinline__ int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// Boundary extension of index i on an axis of n samples: the index whose
// sample stands at i, or -1 for a zero sample.  Replicate clamps; reflect is
// the half-sample symmetric extension (f(-1) = f(0), f(n) = f(n - 1)),
// periodic with period 2n so that boxes wider than the axis are defined.
__device__ __forceinline__ int ext_index(int i, int n, int boundary)
{
    if (i >= 0 && i < n) return i;
    if (boundary == RSG_REPLICATE) return i < 0 ? 0 : n - 1;
    if (boundary == RSG_REFLECT) {
        const int p = 2 * n;
        int m = i % p;
        m += (m < 0) ? p : 0;
        return m < n ? m : p - 1 - m;
    }
    return -1;
}

// Raw chunk of NPL samples held in 32-bit words until it is consumed.
template <class Tr, int NPL>
struct Chunk {
    static constexpr int kBytes = NPL * Tr::kSize;
    static constexpr int kWords = (kBytes + 3) / 4;
    uint32_t w[kWords];
};

constexpr int kBufDword3 = 0x00020000;         // gfx9-family raw buffer descriptor, word 3
// The planner keeps every offset a task really touches below 2^30 and
// descriptors hold at most 2^30 bytes, so offsets in [2^30, 2^31) are out of
// range: loads there read 0 and stores there are dropped.
constexpr int64_t kMaxRecords = int64_t(1) << 30;
constexpr int kDropOffset = 0x60000000;
constexpr uint32_t kDropColumn = 0x40000000u;   // column offset of lanes past the image

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes)
{
    const int n = int(bytes < kMaxRecords ? bytes : kMaxRecords);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, n, kBufDword3);
}

// Interior chunk: unchecked vector accesses of the widest granule that
// divides the chunk (16, 8 or 4 bytes); the planner aligns chunk starts to it.
template <class Tr, int NPL>
__device__ __forceinline__ void load_chunk_vec(Chunk<Tr, NPL>& ch, __amdgpu_buffer_rsrc_t rs, int voff, int soff)
{
    constexpr int kBytes = Chunk<Tr, NPL>::kBytes;
    static_assert(kBytes % 4 == 0, "chunk must be whole dwords");
    constexpr int kGran = (kBytes % 16 == 0) ? 16 : ((kBytes % 8 == 0) ? 8 : 4);
#pragma unroll
    for (int k = 0; k < kBytes / kGran; ++k) {
        if constexpr (kGran == 16) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16 * k, soff, 0);
            ch.w[4 * k + 0] = v[0]; ch.w[4 * k + 1] = v[1]; ch.w[4 * k + 2] = v[2]; ch.w[4 * k + 3] = v[3];
        } else if constexpr (kGran == 8) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff + 8 * k, soff, 0);
            ch.w[2 * k + 0] = v[0]; ch.w[2 * k + 1] = v[1];
        } else {
            ch.w[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff + 4 * k, soff, 0);
        }
    }
}

// Border chunk: element by element at precomputed offsets (clamped for
// REPLICATE, kDropOffset -> 0 for ZERO).
template <class Tr, int NPL>
__device__ __forceinline__ void load_chunk_elem(Chunk<Tr, NPL>& ch, __amdgpu_buffer_rsrc_t rs, const int* eoff,
                                                int soff)
{
#pragma unroll
    for (int k = 0; k < Chunk<Tr, NPL>::kWords; ++k) ch.w[k] = 0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        uint32_t raw;
        if constexpr (Tr::kSize == 1) raw = __builtin_amdgcn_raw_buffer_load_b8(rs, eoff[i], soff, 0);
        else if constexpr (Tr::kSize == 2) raw = __builtin_amdgcn_raw_buffer_load_b16(rs, eoff[i], soff, 0);
        else raw = __builtin_amdgcn_raw_buffer_load_b32(rs, eoff[i], soff, 0);
        ch.w[(i * Tr::kSize) / 4] |= raw << (8 * ((i * Tr::kSize) % 4));
    }
}

// uint8 output: round half up of U / G^2, exactly, in integer arithmetic.
// The caller accumulates N = U + floor(G^2 / 2) < 256 G^2 <= 2^56 (the sum
// starts at floor(G^2 / 2)); the result is Q = floor(N / G^2).  N >> qsh
// (qsh per image: the shift that brings 256 G^2 below 2^32) converts to FP32
// in one instruction; scaled by invG2s = 2^qsh / G^2 it is within 2^-13 of
// N / G^2 (the dropped bits are below 2^-23 of G^2, and three roundings of
// 2^-24 relative on a value below 257 stay under 2^-15).  So N / G^2 + 1 -
// 2^-11, estimated, truncates to Q + 1 or Q and is never negative, and one
// comparison of N with that candidate times G^2 (a 64-bit product, G^2 <
// 2^48) decides.
__device__ __forceinline__ uint32_t round_quotient(uint64_t N, uint64_t G2, float invG2s, int qsh)
{
    const float nf = float(uint32_t(N >> qsh));
    const uint32_t q1 = uint32_t(fmaf(nf, invG2s, 1.0f - 0.00048828125f));
    uint64_t P = uint64_t(q1) * uint64_t(uint32_t(G2));
    P += uint64_t(__umul24(q1, uint32_t(G2 >> 32))) << 32;
    return q1 - ((N < P) ? 1u : 0u);
}
__device__ __forceinline__ uint32_t round_quotient(uint64_t N, const ImgParams& ip)
{
    return round_quotient(N, ip.G2, ip.invG2, ip.qsh);
}

// One element at byte offset `boff` of a buffer, as float.
template <class Tr>
__device__ __forceinline__ float Tr_load_one(__amdgpu_buffer_rsrc_t rs, int boff)
{
    uint32_t w[1];
    if constexpr (Tr::kSize == 1) w[0] = __builtin_amdgcn_raw_buffer_load_b8(rs, boff, 0, 0);
    else if constexpr (Tr::kSize == 2) w[0] = __builtin_amdgcn_raw_buffer_load_b16(rs, boff, 0, 0);
    else w[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, boff, 0, 0);
    return float(Tr::unpack(w, 0));
}

// Orders this wave's LDS writes before its later reads (one-wave groups).
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class Tr>
__device__ __forceinline__ void store_out(__amdgpu_buffer_rsrc_t rs, int voff, int soff, float v);
template <>
__device__ __forceinline__ void store_out<TrF32>(__amdgpu_buffer_rsrc_t rs, int voff, int soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, voff, soff, kStorePolicy<4>);
}
template <>
__device__ __forceinline__ void store_out<TrF16>(__amdgpu_buffer_rsrc_t rs, int voff, int soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), rs, voff, soff, kStorePolicy<2>);
}
template <>
__device__ __forceinline__ void store_out<TrBF16>(__amdgpu_buffer_rsrc_t rs, int voff, int soff, float v)
{
    const uint32_t u = __float_as_uint(v);                          // finite v
    __builtin_amdgcn_raw_buffer_store_b16(uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16), rs, voff, soff, kStorePolicy<2>);
}

// NC consecutive output samples of one lane at byte offset vo: one vector
// store when every sample is inside the row (`full`) and the type allows it
// (`vec`: 2-byte element types need the destination aligned to the group),
// else one store per sample, those at or past `nlive` dropped.
template <class Tr, int NC>
__device__ __forceinline__ void store_group(__amdgpu_buffer_rsrc_t rs, int vo, const uint32_t (&w)[NC], bool full,
                                            int nlive, bool vec)
{
    constexpr int es = Tr::kSize;
    constexpr int pol = kStorePolicy<es * NC>;
    if constexpr (NC == 1) {
        if constexpr (es == 4) __builtin_amdgcn_raw_buffer_store_b32(w[0], rs, vo, 0, pol);
        else if constexpr (es == 2) __builtin_amdgcn_raw_buffer_store_b16(uint16_t(w[0]), rs, vo, 0, pol);
        else __builtin_amdgcn_raw_buffer_store_b8(uint8_t(w[0]), rs, vo, 0, pol);
        return;
    } else {
        if (full && (es == 4 || vec)) {
            if constexpr (es == 4) {
                if constexpr (NC == 2) {
                    __builtin_amdgcn_raw_buffer_store_b64((v2u){w[0], w[1]}, rs, vo, 0, pol);
                } else if constexpr (NC == 3) {
                    __builtin_amdgcn_raw_buffer_store_b96((v3u){w[0], w[1], w[2]}, rs, vo, 0, pol);
                } else {
                    __builtin_amdgcn_raw_buffer_store_b128((v4u){w[0], w[1], w[2], w[3]}, rs, vo, 0, pol);
                }
            } else if constexpr (es == 2 && NC == 2) {
                __builtin_amdgcn_raw_buffer_store_b32(w[0] | (w[1] << 16), rs, vo, 0, pol);
            } else if constexpr (es == 1 && NC == 2) {
                __builtin_amdgcn_raw_buffer_store_b16(uint16_t(w[0] | (w[1] << 8)), rs, vo, 0, pol);
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    // strided element stores: partial lines, left to the L2 to merge
                    if constexpr (es == 2) __builtin_amdgcn_raw_buffer_store_b16(uint16_t(w[c]), rs, vo + 2 * c, 0, 0);
                    else __builtin_amdgcn_raw_buffer_store_b8(uint8_t(w[c]), rs, vo + c, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int o = (c < nlive) ? vo + c * es : kDropOffset;
                if constexpr (es == 4) __builtin_amdgcn_raw_buffer_store_b32(w[c], rs, o, 0, 0);
                else if constexpr (es == 2) __builtin_amdgcn_raw_buffer_store_b16(uint16_t(w[c]), rs, o, 0, 0);
                else __builtin_amdgcn_raw_buffer_store_b8(uint8_t(w[c]), rs, o, 0, 0);
            }
        }
    }
}
// The stored bits of an FP32 result in the element type (round to nearest even).
template <class Tr> __device__ __forceinline__ uint32_t out_bits(float v);
template <> __device__ __forceinline__ uint32_t out_bits<TrF32>(float v) { return __float_as_uint(v); }
template <> __device__ __forceinline__ uint32_t out_bits<TrF16>(float v)
{
    return __half_as_ushort(__float2half_rn(v));
}
template <> __device__ __forceinline__ uint32_t out_bits<TrBF16>(float v)
{
    const uint32_t u = __float_as_uint(v);                          // finite v
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// NC consecutive LDS words of one lane (8- or 16-byte aligned for NC = 2, 4).
template <class Acc, int NC>
__device__ __forceinline__ void lds_put(Acc* p, const Acc (&v)[NC])
{
    if constexpr (NC == 2) {
        *reinterpret_cast<v2u*>(p) = (v2u){bits(v[0]), bits(v[1])};
    } else if constexpr (NC == 4) {
        *reinterpret_cast<v4u*>(p) = (v4u){bits(v[0]), bits(v[1]), bits(v[2]), bits(v[3])};
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) p[c] = v[c];
    }
}
template <class Acc, int NC>
__device__ __forceinline__ void lds_get(const Acc* p, Acc (&v)[NC])
{
    if constexpr (NC == 2) {
        const v2u t = *reinterpret_cast<const v2u*>(p);
        v[0] = frombits<Acc>(t[0]);
        v[1] = frombits<Acc>(t[1]);
    } else if constexpr (NC == 4) {
        const v4u t = *reinterpret_cast<const v4u*>(p);
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = frombits<Acc>(t[c]);
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = p[c];
    }
}

// Per-task constants.
struct TaskGeom {
    int s0, y0, hs, a0, off, niter, ybase;
    int o0;                                    // first output sample of the strip (strided output: kept samples)
    int emit0;                                 // first iteration that emits a row (a multiple of G)
    int64_t slice_off;                         // byte offset of the task's slice (stacked images)
};

// --------------------------------------------------------------------------
// The streaming loop of one task.  The column ring keeps L = roundup(2R + 1
// + G, G) rows of running column sums plus G mirror rows (slots 0..G-1 are
// also written at L..L+G-1), so the taps of a whole group are read at
// (per-group base) + (row * ring pitch) without any per-row modulo.
//
// Iteration `it` reads input row ybase + it and emits output row
// ybase + it - R.  The task starts 2R + 1 + pre rows above its first output
// row, pre < G chosen so that emission starts on a group boundary: a group
// either emits all of its rows or none, and the output offset of row j of a
// group is one add away from the group's.
// --------------------------------------------------------------------------
template <class Tr, int C, int SEG, int NPL, int KT, bool EDGE>
__device__ __forceinline__ void stream_task(const ImgParams& ip, const TaskGeom& tg, uint32_t* lds)
{
    using Acc = typename Tr::Acc;
    constexpr bool kInt = Tr::kInt;
    constexpr int G = kWave / SEG;             // rows per group
    constexpr int PP = row_tile_pitch(SEG, NPL);   // LDS pitch of the row-sum tile
    constexpr int RP = kWave;                      // LDS pitch of the column ring
    constexpr int PF = kPrefetch;
    static_assert(PF % 2 == 0, "the loop alternates the two row tiles, so it unrolls by an even count");
    constexpr int es = Tr::kSize;
    const int lane = threadIdx.x;
    const int jrow = lane / SEG;               // row pass: row within the group
    const int q = lane % SEG;                  // row pass: chunk within the row
    const int R = ip.R;
    const int L = ip.L;
    const int H = ip.H;
    const int W = ip.W;
    const int WC = W * C;
    const int boundary = ip.boundary;

    Acc* P = reinterpret_cast<Acc*>(lds);      // 2 tiles of G rows x PW running sums (pitch PP)
    Acc* ring = P + 2 * G * PP;                // (L + G) rows x 64 column sums (pitch RP)

    // ---- source / destination descriptors (task-relative row offsets) ----
    const int y_lo = max(0, tg.ybase);        // loads clamp rows into [y_lo, H - 1]
    const int y_hi = H - 1;
    const int64_t sstride = ip.src_stride * es;
    const int64_t dstride = ip.dst_stride * es;
    const char* sbase = reinterpret_cast<const char*>(ip.src) + tg.slice_off + int64_t(y_lo) * sstride;
    const __amdgpu_buffer_rsrc_t rs_src = make_rsrc(sbase, int64_t(y_hi - y_lo) * sstride + int64_t(WC) * es);
    const char* dbase = reinterpret_cast<const char*>(ip.dst) + tg.slice_off + int64_t(tg.y0) * dstride;
    const __amdgpu_buffer_rsrc_t rs_dst = make_rsrc(dbase, int64_t(tg.hs - 1) * dstride + int64_t(WC) * es);
    const int s = tg.s0 + lane;                // this lane's column
    // Output row k of the task is stored at ocol + k * dstride: lanes past the
    // image start out of range, rows past the task end beyond the descriptor.
    const uint32_t ocol = (s < WC) ? uint32_t(s * es) : kDropColumn;
    const uint32_t dstr = uint32_t(dstride);

    // ---- row-pass chunk offsets ----
    // Each row segment loads a different input row, so the row offset is a
    // per-lane (VGPR) part of the buffer offset; the descriptor and soffset
    // stay uniform.
    const int cs = tg.a0 + NPL * q;            // first span sample of this lane's chunk
    const int vec_voff = cs * es;
    int eoff[EDGE ? NPL : 1];
    if constexpr (EDGE) {
        const int x0 = floor_div(cs, C);
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int x = x0 + i / C;
            const int xe = ext_index(x, W, boundary);
            eoff[i] = (xe >= 0) ? (xe * C + i % C) * es : -1;    // -1: zero sample
        }
    }
    const int sstride32 = int(sstride);
    auto load = [&](Chunk<Tr, NPL>& ch, int g) {
        const int y = tg.ybase + g * G + jrow;
        // Every row a task needs maps into [y_lo, H - 1]; rows past the task
        // end (re-read, unused) may not, and then read as 0 or any row.
        const int ye = ext_index(y, H, boundary);
        const bool zero_row = ye < 0;                     // ZERO boundary: rows outside read as 0
        const int rowoff = (zero_row ? 0 : ye - y_lo) * sstride32;
        if constexpr (EDGE) {
            int vo[NPL];
#pragma unroll
            for (int i = 0; i < NPL; ++i) vo[i] = (eoff[i] < 0 || zero_row) ? kDropOffset : eoff[i] + rowoff;
            load_chunk_elem<Tr, NPL>(ch, rs_src, vo, 0);
        } else {
            load_chunk_vec<Tr, NPL>(ch, rs_src, zero_row ? kDropOffset : vec_voff + rowoff, 0);
        }
    };

    // ---- combine taps ----
    int tp[KT], tm[KT];                        // LDS indices of the row box ends
    float wf[KT];
    uint32_t wm[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        tp[k] = tg.off + lane + ip.r[k] * C;
        tm[k] = tg.off + lane - (ip.r[k] + 1) * C;
        wf[k] = ip.wf[k];
        wm[k] = ip.m[k];
    }
    const float dc = ip.dc32;

    const int ngroups = (tg.niter + G - 1) / G;

    // Prologue: the first PF groups' loads, in order, each followed by G
    // dropped stores, so the memory-operation sequence before the loop
    // matches the one around its back edge and the loop's waits stay exact.
    Chunk<Tr, NPL> buf[PF];
#pragma unroll
    for (int b = 0; b < PF; ++b) {
        __builtin_amdgcn_sched_barrier(0);
        load(buf[b], b);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < G; ++j) {         // distinct offsets: not merged by the compiler
            if constexpr (kInt) __builtin_amdgcn_raw_buffer_store_b8(uint8_t(0), rs_dst, kDropOffset - 64 * (b * G + j), 0, kStorePolicy<1>);
            else store_out<Tr>(rs_dst, kDropOffset - 64 * (b * G + j), 0, 0.0f);
        }
    }
    __builtin_amdgcn_sched_barrier(0);

    Acc colacc = Acc(0);
    float c2 = 0.0f;                           // column offset (float types): T of the task's first row
    float c2dc = 0.0f;
    int slot0 = 0;                             // ring slot of the first row of the queued group
    Acc Tq[G];                                 // row-pass result of the group queued for the column pass

    // Row pass, first half: consume the group's chunk, reuse its registers
    // for the load of group g + PF (so the loop-carried buffers are written
    // in place and each load is waited for PF groups after it was issued),
    // scan the rows and write them to the LDS tile.  Returns the group's
    // offset (float types): the first span sample of its first row (lane 0),
    // subtracted from every sample and restored through the DC gain.
    auto row_scan = [&](int g, Chunk<Tr, NPL>& bf, int t) -> float {
        __builtin_amdgcn_sched_barrier(0);
        Acc v[NPL];
        float off = 0.0f;
        if constexpr (!kInt) {
            off = (boundary == RSG_ZERO) ? 0.0f
                                         : __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(Tr::unpack(bf.w, 0))));
#pragma unroll
            for (int i = 0; i < NPL; ++i) v[i] = Tr::unpack(bf.w, i) - off;
        } else {
#pragma unroll
            for (int i = 0; i < NPL; ++i) v[i] = Tr::unpack(bf.w, i);
        }
        __builtin_amdgcn_sched_barrier(0);
        load(bf, g + PF);
        __builtin_amdgcn_sched_barrier(0);

        // running sum of this lane's row over its span (Eq. alg1)
#pragma unroll
        for (int i = C; i < NPL; ++i) v[i] = v[i] + v[i - C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const Acc tot = v[NPL - C + c];
            const Acc ex = segment_inclusive_scan<SEG>(tot) - tot;     // exclusive within the segment
#pragma unroll
            for (int i = c; i < NPL; i += C) v[i] = v[i] + ex;
        }
        using Acc4 = typename std::conditional<kInt, uint4, float4>::type;
        Acc4* dst4 = reinterpret_cast<Acc4*>(P + (t * G + jrow) * PP + q * NPL);   // 16-byte stores
#pragma unroll
        for (int h = 0; h < NPL / 4; ++h) {
            Acc4 t4;
            t4.x = v[4 * h + 0]; t4.y = v[4 * h + 1]; t4.z = v[4 * h + 2]; t4.w = v[4 * h + 3];
            dst4[h] = t4;
        }
        return off;
    };

    // Row pass, second half (after the tile is visible): box differences
    // along the rows (Eq. indep), lane = column.  The reads are issued as one
    // batch (row_reads) before any of them is used (row_combine).
    using Taps = Acc[G][2 * KT];
    auto row_reads = [&](Taps& pv, int t) {
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const Acc* Pj = P + (t * G + j) * PP;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                pv[j][2 * k] = Pj[tp[k]];
                pv[j][2 * k + 1] = Pj[tm[k]];
            }
        }
    };
    auto row_combine = [&](const Taps& pv, Acc (&T)[G], float init) {
#pragma unroll
        for (int j = 0; j < G; ++j) {
            Acc t;
            if constexpr (kInt) {
                t = 0;
#pragma unroll
                for (int k = 0; k < KT; ++k) t += __umul24(wm[k], pv[j][2 * k] - pv[j][2 * k + 1]);
            } else {
                t = fmaf(wf[0], pv[j][0] - pv[j][1], init);
#pragma unroll
                for (int k = 1; k < KT; ++k) t = fmaf(wf[k], pv[j][2 * k] - pv[j][2 * k + 1], t);
            }
            T[j] = t;
        }
    };

    // Column pass, first half: running sums down the columns (Eq. alg1) of
    // the queued group into the ring.  Float rows arrive as T + off * dc
    // (the group offset restores the row's true box sums, folded into the
    // row combine) and enter the sums as (T + off * dc) - c2: c2, the task's
    // first row, keeps the column sums small.  (The multi-wave form computes
    // exactly the same values, so every form agrees bit for bit.)
    auto col_push = [&]() {
        const int wbase = slot0 * RP + lane;
        Acc cj[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if constexpr (kInt) colacc += Tq[j];
            else colacc += Tq[j] - c2;
            cj[j] = colacc;
            ring[wbase + j * RP] = colacc;
        }
        if (slot0 == 0) {                           // slots 0 .. G-1 also live at L .. L+G-1
#pragma unroll
            for (int j = 0; j < G; ++j) ring[(L + j) * RP + lane] = cj[j];
        }
    };

    // Column pass, second half (after the ring rows are visible): box
    // differences down the columns (Eq. indep) for the rows R behind the
    // queued group's rows (col_reads issues the reads, col_combine uses them
    // and stores the outputs).
    auto col_reads = [&](Taps& rv) {
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            int a = slot0 - R + ip.r[k];
            int b = slot0 - R - ip.r[k] - 1;
            a += (a < 0) ? L : 0;
            b += (b < 0) ? L : 0;
            const int bp = a * RP + lane;
            const int bm = b * RP + lane;
#pragma unroll
            for (int j = 0; j < G; ++j) {
                rv[j][2 * k] = ring[bp + j * RP];
                rv[j][2 * k + 1] = ring[bm + j * RP];
            }
        }
    };
    auto col_combine = [&](int gq, const Taps& rv) {
        const int it0 = gq * G;
        const uint32_t og = (it0 >= tg.emit0) ? ocol + uint32_t(it0 - tg.emit0) * dstr : uint32_t(kDropOffset);
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int voff = int(og + uint32_t(j) * dstr);
            if constexpr (kInt) {
                // U = sum m_k D_k < 256 G^2: exact in uint64
                uint64_t N = ip.G2half;
#pragma unroll
                for (int k = 0; k < KT; ++k) N += uint64_t(wm[k]) * uint64_t(rv[j][2 * k] - rv[j][2 * k + 1]);
                __builtin_amdgcn_raw_buffer_store_b8(uint8_t(round_quotient(N, ip)), rs_dst, voff, 0, kStorePolicy<1>);
            } else {
                float o = c2dc;
#pragma unroll
                for (int k = 0; k < KT; ++k) o = fmaf(wf[k], rv[j][2 * k] - rv[j][2 * k + 1], o);
                store_out<Tr>(rs_dst, voff, 0, o);
            }
        }
    };

    auto dropped_stores = [&](int base) {      // distinct offsets: not merged by the compiler
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if constexpr (kInt) __builtin_amdgcn_raw_buffer_store_b8(uint8_t(0), rs_dst, kDropOffset - 64 * (base + j), 0, kStorePolicy<1>);
            else store_out<Tr>(rs_dst, kDropOffset - 64 * (base + j), 0, 0.0f);
        }
    };

    // Software pipeline.  Step g (g >= 1):
    //   1. row pass of group g + 1 up to its tile write (tile (g + 1) & 1),
    //   2. row differences of group g from the tile reads issued in step g - 1,
    //   3. column outputs of group g - 1 from the ring reads issued in step g - 1,
    //   4. column sums of group g into the ring,
    //   5. one fence, then the reads for steps 2 and 3 of step g + 1.
    // The reads of step 5 are served while step g + 1 runs its row scan.
    // Steps with no real rows (before the first emitted row, past the task)
    // store to dropped offsets, so every step issues the same memory
    // operations and the loop's waits stay exact.
    Taps pv, rv;
    float off_cur = row_scan(0, buf[0], 0);      // group 0
    dropped_stores(PF * G);
    wave_lds_fence();
    row_reads(pv, 0);
    {   // step 0: group 1's row scan, group 0's row differences and column sums
        const float off_next = row_scan(1, buf[1 % PF], 1);
        Acc T[G];
        float init = 0.0f;
        if constexpr (!kInt) init = off_cur * dc;
        row_combine(pv, T, init);
        if constexpr (!kInt) {
            c2 = (boundary == RSG_ZERO) ? 0.0f : T[0];  // the column offset: the task's first row
            c2dc = c2 * dc;
        }
        dropped_stores(PF * G + G);
#pragma unroll
        for (int j = 0; j < G; ++j) Tq[j] = T[j];
        col_push();
        wave_lds_fence();
        row_reads(pv, 1);
        col_reads(rv);
        off_cur = off_next;
    }
    const int nsteps = (ngroups + PF - 1) / PF * PF;   // steps 1 .. nsteps: column outputs of groups 0 .. nsteps - 1
    for (int g = 1; g < nsteps + 1; g += PF) {
#pragma unroll
        for (int b = 0; b < PF; ++b) {
            const int gg = g + b;
            const float off_next = row_scan(gg + 1, buf[(2 + b) % PF], b & 1);
            float init = 0.0f;
            if constexpr (!kInt) init = off_cur * dc;
            Acc T[G];
            row_combine(pv, T, init);
            col_combine(gg - 1, rv);
            slot0 += G;
            slot0 -= (slot0 >= L) ? L : 0;
#pragma unroll
            for (int j = 0; j < G; ++j) Tq[j] = T[j];
            col_push();
            wave_lds_fence();
            row_reads(pv, b & 1);                // tile of group gg + 1
            col_reads(rv);
            off_cur = off_next;
        }
    }
}

// --------------------------------------------------------------------------
// Cooperative form of the streaming loop: one task per workgroup of
// kCoWaves waves that share the strip.  Step m covers iterations
// [m MB, (m + 1) MB), MB = kCoWaves * RB (RB = co_rows(NC): 8 rows, 4 for
// the wide column form); wave w takes the block of RB iterations starting at
// m MB + w RB and runs both passes on it:
//
//   row pass    its groups of G rows (loads prefetched one step ahead in
//               the wave's own sequence, running sums, row tile, Eq. indep
//               along x) -> T of its RB rows in registers;
//   column sums the block's running sums of T (Eq. alg1 down the column,
//               in registers), its total to LDS; barrier; the block's carry
//               (sum of the earlier blocks' totals, added in the same order
//               by every wave) makes them the strip's running sums, written
//               to the LDS ring; barrier;
//   column out  K box differences down the column (Eq. indep) for the
//               block's rows, read from the ring, and one store per row.
//
// The ring holds L >= MB + 2R + 1 rows (a multiple of RB) plus RB
// mirror rows, so the taps of a block are read at (per-block slot) + row
// without a modulo.  Two barriers per step of MB rows, all waves doing the
// same work, several steps of loads in flight: the strip streams without a
// serial chain of LDS round trips per row.  Float columns sum T - c with c a
// per-column constant (the input sample at the task's first row), restored
// through the DC gain of the boxes, so the sums stay at the size of local
// variations (under zero extension only samples inside the image are
// offset, and each box takes back the share of its inside samples).
//
// Iteration `it` reads input row ybase + it and, for it >= 2R + 1, emits
// output row ybase + it - R.  Rows past the task are stored to dropped
// offsets, so every step issues the same memory operations and the waits
// for the prefetched loads stay exact.
// --------------------------------------------------------------------------
template <class Tr, int C, int SEG, int NPL, int KT, bool EDGE, int NC = 1, bool ZX = false, int NW_ = kCoWaves,
          int RB_ = co_rows(NC), bool TS = false>
__device__ __forceinline__ void stream_task_co(const ImgParams& ip, const TaskGeom& tg, uint32_t* lds)
{
    using Acc = typename Tr::Acc;
    constexpr bool kInt = Tr::kInt;
    constexpr int G = kWave / SEG;
    constexpr int PW = SEG * NPL;
    constexpr int PP = row_tile_pitch(SEG, NPL);
    constexpr int RP = kWave * NC;             // words per ring row (the strip's columns)
    constexpr int NW = NW_;                    // waves per task
    constexpr int RB = RB_;                    // rows per wave per step
    constexpr int NGW = RB / G;                // row groups per wave per step
    constexpr int MB = NW * RB;                // rows per step
    constexpr int PF = (NGW >= 2) ? 2 : 1;     // groups of loads in flight per wave (one step ahead)
    static_assert(RB % G == 0 && NGW % PF == 0, "a step holds whole groups and whole prefetch rounds");
    static_assert(PW <= PP, "tile pitch");
    constexpr int es = Tr::kSize;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // uniform: scalar slot arithmetic
    const int lane = threadIdx.x % kWave;
    const int R = ip.R;
    const int L = ip.Lco;
    const int H = ip.H;
    const int W = ip.W;
    const int WC = W * C;
    const int boundary = ip.boundary;
    // samples from one pixel to the next: 1, or the image's channel count
    // for channel-planar tasks (C = 1 here; the slice offset selects the channel)
    const int ps = ip.pstride > 1 ? ip.pstride : 1;

    // LDS: [row tiles NW x G x PP][block totals NW x RP][ring (L + RB) x RP]
    Acc* Pt = reinterpret_cast<Acc*>(lds) + wave * G * PP;
    Acc* X = reinterpret_cast<Acc*>(lds) + NW * G * PP;
    Acc* ring = X + NW * RP;

    const float dc = ip.dc32;
    float wf[KT];
    uint32_t wm[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        wf[k] = ip.wf[k];
        wm[k] = ip.m[k];
    }
    const int64_t sstride = ip.src_stride * es;
    const int64_t dstride = ip.dst_stride * es;
    const int nsteps = (tg.niter + MB - 1) / MB;
    [[maybe_unused]] const uint64_t G2 = ip.G2, G2half = ip.G2half;   // uint8 rounding
    [[maybe_unused]] const float invG2 = ip.invG2;
    [[maybe_unused]] const int qsh = ip.qsh;

    // ---------------- row-pass setup ----------------
    const int jrow = lane / SEG;
    const int q = lane % SEG;
    const int y_lo = max(0, tg.ybase);
    // groups whose rows all lie in [y_lo, H) start at y_lo + [0, fast_n)
    const int fast_n = max(0, H - G - y_lo + 1);
    const char* sbase = reinterpret_cast<const char*>(ip.src) + tg.slice_off + int64_t(y_lo) * sstride;
    const __amdgpu_buffer_rsrc_t rs_src = make_rsrc(sbase, int64_t(H - 1 - y_lo) * sstride + int64_t(WC) * ps * es);
    const int cs = tg.a0 + NPL * q;
    const int vec_voff = cs * es;
    int eoff[EDGE ? NPL : 1];
    if constexpr (EDGE) {
        const int x0 = floor_div(cs, C);
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int x = x0 + i / C;
            const int xe = ext_index(x, W, boundary);
            eoff[i] = (xe >= 0) ? (xe * C + i % C) * ps * es : -1;
        }
    }
    const int sstride32 = int(sstride);
    // 4-byte samples on a border task: a lane whose chunk lies inside the row
    // loads it as vectors, the others per element; each lane's other load
    // reads out of range (zeros), and the two are ORed when the group is
    // used, so no branch diverges and every wait stays exact
    constexpr bool kSplit = EDGE && Tr::kSize == 4;
    const bool lane_vec = ip.vec && cs >= 0 && cs + NPL <= WC;
    // Offsets of a group whose rows all lie in [y_lo, H): this lane's row
    // within the group and column in VGPRs (fixed for the task), the group's
    // first row in the scalar offset.  Other groups extend each lane's row.
    const int jrow_off = jrow * sstride32;
    const int fast_vec = (kSplit ? lane_vec : true) ? vec_voff + jrow_off : kDropOffset;
    int fast_elem[EDGE ? NPL : 1];
    if constexpr (EDGE) {
#pragma unroll
        for (int i = 0; i < NPL; ++i)
            fast_elem[i] = ((kSplit && lane_vec) || eoff[i] < 0) ? kDropOffset : eoff[i] + jrow_off;
    }
    // group gq of this wave: iterations (gq / NGW) MB + wave RB + (gq % NGW) G + [0, G)
    auto load = [&](Chunk<Tr, NPL>& ch, Chunk<Tr, NPL>& ech, int gq) {
        const int it = (gq / NGW) * MB + wave * RB + (gq % NGW) * G;
        const int yg = tg.ybase + it;
        if (unsigned(yg - y_lo) < unsigned(fast_n)) {
            const int soff = (yg - y_lo) * sstride32;
            if constexpr (kSplit) {
                load_chunk_vec<Tr, NPL>(ch, rs_src, fast_vec, soff);
                load_chunk_elem<Tr, NPL>(ech, rs_src, fast_elem, soff);
            } else if constexpr (EDGE) {
                load_chunk_elem<Tr, NPL>(ch, rs_src, fast_elem, soff);
            } else {
                load_chunk_vec<Tr, NPL>(ch, rs_src, fast_vec, soff);
            }
            return;
        }
        const int y = yg + jrow;
        const int ye = ext_index(y, H, boundary);
        const bool zero_row = ye < 0;
        const int rowoff = (zero_row ? 0 : ye - y_lo) * sstride32;
        if constexpr (kSplit) {
            load_chunk_vec<Tr, NPL>(ch, rs_src, (lane_vec && !zero_row) ? vec_voff + rowoff : kDropOffset, 0);
            int vo[NPL];
#pragma unroll
            for (int i = 0; i < NPL; ++i)
                vo[i] = (lane_vec || eoff[i] < 0 || zero_row) ? kDropOffset : eoff[i] + rowoff;
            load_chunk_elem<Tr, NPL>(ech, rs_src, vo, 0);
        } else if constexpr (EDGE) {
            int vo[NPL];
#pragma unroll
            for (int i = 0; i < NPL; ++i) vo[i] = (eoff[i] < 0 || zero_row) ? kDropOffset : eoff[i] + rowoff;
            load_chunk_elem<Tr, NPL>(ch, rs_src, vo, 0);
        } else {
            load_chunk_vec<Tr, NPL>(ch, rs_src, zero_row ? kDropOffset : vec_voff + rowoff, 0);
        }
    };
    // ---------------- this lane's columns ----------------
    // The lane owns NC consecutive output samples oidx0 .. oidx0 + NC - 1 of
    // the output row, centred on input samples s .. s + NC - 1.  A strided
    // output (NC = 1) keeps every ostep-th pixel, compacted: the strip then
    // covers 64 kept samples, so the row taps and the column pass run at
    // kept columns only.  Every lane's samples lie inside the row tile,
    // lanes past the end of the row included.
    const int ostep = (NC == 1 && ip.step > 1) ? ip.step : 1;
    const int orow_len = (ostep > 1) ? (W + ostep - 1) / ostep * C : WC;
    const int oidx0 = tg.o0 + lane * NC;
    const int s = (ostep > 1) ? (oidx0 / C) * ostep * C + oidx0 % C : oidx0;
    const int colL = s - tg.a0;
    int tp[KT], tm[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        tp[k] = colL + ip.r[k] * C;
        tm[k] = colL - (ip.r[k] + 1) * C;
    }

    // ---------------- column setup ----------------
    // Output rows of this task: y0 .. y0 + hs - 1, or with a strided output
    // the kept rows oq0 .. oq1 - 1 of the output image; rows outside the
    // descriptor and samples past the row are stored to out-of-range offsets.
    int oq0 = tg.y0, nrows = tg.hs;
    const uint32_t ocol = (oidx0 < orow_len) ? uint32_t(oidx0 * ps * es) : kDropColumn;
    const bool lane_full = oidx0 + NC <= orow_len;
    const int nlive = orow_len - oidx0;
    const bool ovec = ip.ovec != 0;
    if (ostep > 1) {
        oq0 = (tg.y0 + ostep - 1) / ostep;
        nrows = (tg.y0 + tg.hs - 1) / ostep - oq0 + 1;
    }
    const char* dbase = reinterpret_cast<char*>(ip.dst) + tg.slice_off + int64_t(oq0) * dstride;
    const __amdgpu_buffer_rsrc_t rs_dst =
        make_rsrc(dbase, nrows > 0 ? int64_t(nrows - 1) * dstride + int64_t(orow_len) * ps * es : 0);
    const uint32_t dstr = uint32_t(dstride);
    // Float offsets.  Each group of rows subtracts one of its samples (off)
    // and each column the input sample at the task's first row (cf); they
    // come back through the boxes' DC gain.  Under zero extension only the
    // samples inside the image are offset, and a box takes back the offset
    // of its samples inside the image: dcx (along x, per lane) and dcy
    // (along y, per output row) replace the DC gain near the borders, so
    // outside samples still enter every sum as exact zeros.
    constexpr bool zext = ZX;                  // float samples under zero extension
    static_assert(!ZX || !kInt, "integer sums take no offsets");
    float cf[NC], cdc[NC], dcx[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        cf[c] = 0.0f;
        dcx[c] = dc;
    }
    int off_lane = 0;                          // zext: a lane of row 0 of a group whose first sample is inside
    uint32_t col_in = ~0u;                     // zext, border tasks: bit i = sample i of the lane's chunk inside
    if constexpr (!kInt) {
        const int yc = zext ? min(max(tg.ybase, 0), H - 1) : ext_index(tg.ybase, H, boundary);   // >= y_lo
#pragma unroll
        for (int c = 0; c < NC; ++c)
            cf[c] = Tr_load_one<Tr>(rs_src, (yc - y_lo) * sstride32 + min(s + c, WC - 1) * ps * es);
        if (zext) {
            off_lane = min(SEG - 1, max(0, (NPL - 1 - tg.a0) / NPL));
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int x = min(s + c, WC - 1) / C;
                float d = 0.0f;
#pragma unroll
                for (int k = 0; k < KT; ++k)
                    d = fmaf(wf[k], float(min(x + ip.r[k], W - 1) - max(x - ip.r[k], 0) + 1), d);
                dcx[c] = d;
            }
            if constexpr (EDGE) {
                col_in = 0;
#pragma unroll
                for (int i = 0; i < NPL; ++i) col_in |= (eoff[i] >= 0) ? (1u << i) : 0u;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) cdc[c] = cf[c] * dc;
    // zext: sum_k w_k (rows of box k inside the image) for output row y
    auto dc_rows = [&](int y) {
        if (y >= R && y < H - R) return dc;
        float d = 0.0f;
#pragma unroll
        for (int k = 0; k < KT; ++k) d = fmaf(wf[k], float(min(y + ip.r[k], H - 1) - max(y - ip.r[k], 0) + 1), d);
        return d;
    };

    constexpr int NST = TS ? 2 : RB;           // stores per wave per step
    static_assert(!TS || (NC == 1 && es == 4 && RB == 8 && !EDGE && !ZX), "staged stores: FP32, interior, one column per lane");
    auto dropped_stores = [&](int base) {      // distinct offsets: not merged by the compiler
#pragma unroll
        for (int j = 0; j < NST; ++j) {
            if constexpr (kInt) __builtin_amdgcn_raw_buffer_store_b8(uint8_t(0), rs_dst, kDropOffset - 64 * (base + j), 0, kStorePolicy<1>);
            else store_out<Tr>(rs_dst, kDropOffset - 64 * (base + j), 0, 0.0f);
        }
    };

    // Prologue: the first PF groups' loads and RB dropped stores, the memory
    // operations that precede the loop's first wait as they precede it
    // around the back edge.
    Chunk<Tr, NPL> buf[PF];
    Chunk<Tr, NPL> ebuf[kSplit ? PF : 1];
#pragma unroll
    for (int b = 0; b < PF; ++b) {
        __builtin_amdgcn_sched_barrier(0);
        load(buf[b], ebuf[kSplit ? b : 0], b);
    }
    __builtin_amdgcn_sched_barrier(0);
    dropped_stores(0);
    __builtin_amdgcn_sched_barrier(0);

    Acc carry[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) carry[c] = Acc(0);
    int slot_m = 0;                            // ring slot of iteration m MB
    for (int m = 0; m < nsteps; ++m) {
        Acc T[RB][NC];
#pragma unroll
        for (int g = 0; g < NGW; ++g) {
            const int b = g % PF;
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (kSplit) {
#pragma unroll
                for (int k = 0; k < Chunk<Tr, NPL>::kWords; ++k) buf[b].w[k] |= ebuf[b].w[k];
            }
            Acc v[NPL];
            float off = 0.0f;
            const int yg = tg.ybase + m * MB + wave * RB + g * G;     // the group's first input row
            if constexpr (!kInt) {
                const uint32_t x0 = __float_as_uint(Tr::unpack(buf[b].w, 0));
                if (zext) {
                    off = __uint_as_float(__builtin_amdgcn_readlane(x0, off_lane));
                    const bool row_in = unsigned(yg + jrow) < unsigned(H);
#pragma unroll
                    for (int i = 0; i < NPL; ++i)
                        v[i] = (row_in && ((col_in >> i) & 1u)) ? Tr::unpack(buf[b].w, i) - off : 0.0f;
                } else {
                    off = __uint_as_float(__builtin_amdgcn_readfirstlane(x0));
#pragma unroll
                    for (int i = 0; i < NPL; ++i) v[i] = Tr::unpack(buf[b].w, i) - off;
                }
            } else {
#pragma unroll
                for (int i = 0; i < NPL; ++i) v[i] = Tr::unpack(buf[b].w, i);
            }
            __builtin_amdgcn_sched_barrier(0);
            load(buf[b], ebuf[kSplit ? b : 0], m * NGW + g + PF);
            __builtin_amdgcn_sched_barrier(0);
            // running sums along the row (Eq. alg1)
#pragma unroll
            for (int i = C; i < NPL; ++i) v[i] = v[i] + v[i - C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const Acc tot = v[NPL - C + c];
                const Acc ex = segment_inclusive_scan<SEG>(tot) - tot;
#pragma unroll
                for (int i = c; i < NPL; i += C) v[i] = v[i] + ex;
            }
            using Acc4 = typename std::conditional<kInt, uint4, float4>::type;
            Acc4* dst4 = reinterpret_cast<Acc4*>(Pt + jrow * PP + q * NPL);
#pragma unroll
            for (int h = 0; h < NPL / 4; ++h) {
                Acc4 t4;
                t4.x = v[4 * h]; t4.y = v[4 * h + 1]; t4.z = v[4 * h + 2]; t4.w = v[4 * h + 3];
                dst4[h] = t4;
            }
            wave_lds_fence();
            // row box differences (Eq. indep), lane = column; floats add the
            // group offset's share (none for rows outside the image)
            float od[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) od[c] = off * dcx[c];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const Acc* Pj = Pt + j * PP;
                const bool jin = !zext || unsigned(yg + j) < unsigned(H);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const float init = jin ? od[c] : 0.0f;
                    Acc t;
                    if constexpr (kInt) {
                        t = 0;
#pragma unroll
                        for (int k = 0; k < KT; ++k) t += __umul24(wm[k], Pj[tp[k] + c] - Pj[tm[k] + c]);
                    } else {
                        t = fmaf(wf[0], Pj[tp[0] + c] - Pj[tm[0] + c], init);
#pragma unroll
                        for (int k = 1; k < KT; ++k) t = fmaf(wf[k], Pj[tp[k] + c] - Pj[tm[k] + c], t);
                    }
                    T[g * G + j][c] = t;
                }
            }
        }

        // ---- column running sums of the block (Eq. alg1), then its carry ----
        {   // T becomes the block's running sums J
            Acc run[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                run[c] = Acc(0);
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    if constexpr (kInt) {
                        run[c] += T[i][c];
                    } else {
                        const bool iin = !zext || unsigned(tg.ybase + m * MB + wave * RB + i) < unsigned(H);
                        run[c] += T[i][c] - (iin ? cf[c] : 0.0f);
                    }
                    T[i][c] = run[c];
                }
            }
            lds_put<Acc, NC>(X + wave * RP + lane * NC, run);
        }
        __syncthreads();
        Acc cw[NC];
        {
            Acc acc[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                acc[c] = carry[c];
                cw[c] = carry[c];
            }
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                Acc xv[NC];
                lds_get<Acc, NC>(X + v * RP + lane * NC, xv);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    cw[c] = (v == wave) ? acc[c] : cw[c];
                    acc[c] += xv[c];
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) carry[c] = acc[c];
        }
        int sb = slot_m + wave * RB;
        sb -= (sb >= L) ? L : 0;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
#pragma unroll
            for (int c = 0; c < NC; ++c) T[i][c] = cw[c] + T[i][c];
            lds_put<Acc, NC>(ring + (sb + i) * RP + lane * NC, T[i]);
        }
        if (sb == 0) {                         // slots 0 .. RB-1 also live at L .. L+RB-1
#pragma unroll
            for (int i = 0; i < RB; ++i) lds_put<Acc, NC>(ring + (L + i) * RP + lane * NC, T[i]);
        }
        __syncthreads();

        // ---- column box differences (Eq. indep) and stores ----
        int ta[KT], tb[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            ta[k] = sb - R + ip.r[k];
            tb[k] = sb - R - ip.r[k] - 1;
            ta[k] += (ta[k] < 0) ? L : 0;
            tb[k] += (tb[k] < 0) ? L : 0;
        }
        // output row of block row i: k = (first iteration of the block) + i - (2R + 1);
        // its byte offset in the output (scalar), or the dropped offset
        const int kb = m * MB + wave * RB - tg.emit0;
        int soff[RB];
        if (ostep == 1) {
            uint32_t ob = uint32_t(kb) * dstr;
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                soff[i] = (unsigned(kb + i) < unsigned(tg.hs)) ? int(ob) : kDropOffset;
                ob += dstr;
            }
        } else {
            const int yb = tg.y0 + kb;
            int qrow = floor_div(yb, ostep);
            int rr = yb - qrow * ostep;
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int k = kb + i;
                soff[i] = (k >= 0 && k < tg.hs && rr == 0) ? int(uint32_t(qrow - oq0) * dstr) : kDropOffset;
                if (++rr == ostep) { rr = 0; ++qrow; }
            }
        }
        // the stored bits of the lane's NC results of block row i from its taps rv
        auto combine = [&](const Acc (&rv)[2 * KT][NC], int i, uint32_t (&w)[NC]) {
            const float dcy = zext ? dc_rows(tg.y0 + kb + i) : dc;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if constexpr (kInt) {
                    uint64_t N = G2half;
#pragma unroll
                    for (int k2 = 0; k2 < KT; ++k2)
                        N += uint64_t(wm[k2]) * uint64_t(rv[2 * k2][c] - rv[2 * k2 + 1][c]);
                    w[c] = round_quotient(N, G2, invG2, qsh);
                } else {
                    float o = zext ? cf[c] * dcy : cdc[c];
#pragma unroll
                    for (int k2 = 0; k2 < KT; ++k2) o = fmaf(wf[k2], rv[2 * k2][c] - rv[2 * k2 + 1][c], o);
                    w[c] = out_bits<Tr>(o);
                }
            }
        };
        auto combine_store = [&](const Acc (&rv)[2 * KT][NC], int i) {
            const int vo = int(ocol + uint32_t(soff[i]));
            uint32_t w[NC];
            combine(rv, i, w);
            store_group<Tr, NC>(rs_dst, vo, w, lane_full, nlive, ovec);
        };
        if constexpr (TS) {
            // Staged stores: the wave's RB x 64 results go through its row
            // tile (unused until the next step's row pass; one wave's LDS
            // accesses complete in order) and leave as 16-byte stores, four
            // whole 256-byte row pieces per instruction instead of one.
            constexpr int HB = (8 * KT <= 48) ? 4 : 2;
            static_assert(G * PP >= RB * kWave, "the row tile holds the staged results");
            uint32_t* stg = reinterpret_cast<uint32_t*>(Pt);
#pragma unroll
            for (int h = 0; h < RB / HB; ++h) {
                __builtin_amdgcn_sched_barrier(0);
                Acc rv[HB][2 * KT][NC];
#pragma unroll
                for (int k = 0; k < KT; ++k) {
#pragma unroll
                    for (int i = 0; i < HB; ++i) {
                        lds_get<Acc, NC>(ring + (ta[k] + h * HB + i) * RP + lane * NC, rv[i][2 * k]);
                        lds_get<Acc, NC>(ring + (tb[k] + h * HB + i) * RP + lane * NC, rv[i][2 * k + 1]);
                    }
                }
#pragma unroll
                for (int i = 0; i < HB; ++i) {
                    uint32_t w[1];
                    combine(rv[i], h * HB + i, w);
                    stg[(h * HB + i) * kWave + lane] = w[0];
                }
            }
            wave_lds_fence();
            // piece idx = lane + 64 j: block row idx / 16, columns 4 (idx % 16) ..
            const uint32_t sb0 = uint32_t(tg.o0 * es);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int idx = lane + kWave * j;
                const int k = kb + (idx >> 4);
                const v4u val = *reinterpret_cast<const v4u*>(stg + idx * 4);
                const int vo = (unsigned(k) < unsigned(tg.hs)) ? int(sb0 + uint32_t(k) * dstr + uint32_t(idx & 15) * 16u)
                                                               : kDropOffset;
                __builtin_amdgcn_raw_buffer_store_b128(val, rs_dst, vo, 0, kStorePolicy<16>);
            }
        } else if (ostep == 1) {
            // every row: the taps of HB rows at a time (fewer live registers)
            constexpr int HB = (8 * KT * NC <= 48) ? 4 : ((4 * KT * NC <= 48) ? 2 : 1);
            static_assert(RB % HB == 0, "whole sub-blocks");
#pragma unroll
            for (int h = 0; h < RB / HB; ++h) {
                __builtin_amdgcn_sched_barrier(0);
                Acc rv[HB][2 * KT][NC];
#pragma unroll
                for (int k = 0; k < KT; ++k) {
#pragma unroll
                    for (int i = 0; i < HB; ++i) {
                        lds_get<Acc, NC>(ring + (ta[k] + h * HB + i) * RP + lane * NC, rv[i][2 * k]);
                        lds_get<Acc, NC>(ring + (tb[k] + h * HB + i) * RP + lane * NC, rv[i][2 * k + 1]);
                    }
                }
#pragma unroll
                for (int i = 0; i < HB; ++i) combine_store(rv[i], h * HB + i);
            }
        } else if constexpr (NC == 1) {
            // strided output: only kept rows read their taps and combine (a
            // uniform test); a dropped row still issues one store, out of range
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                if (soff[i] != kDropOffset) {
                    Acc rv[2 * KT][NC];
#pragma unroll
                    for (int k = 0; k < KT; ++k) {
                        rv[2 * k][0] = ring[(ta[k] + i) * RP + lane];
                        rv[2 * k + 1][0] = ring[(tb[k] + i) * RP + lane];
                    }
                    combine_store(rv, i);
                } else {
                    if constexpr (kInt) __builtin_amdgcn_raw_buffer_store_b8(uint8_t(0), rs_dst, kDropOffset - 64 * i, 0, kStorePolicy<1>);
                    else store_out<Tr>(rs_dst, kDropOffset - 64 * i, 0, 0.0f);
                }
            }
        }
        slot_m += MB;
        slot_m -= (slot_m >= L) ? L : 0;
    }
}

// One task: 64 NC sample-columns x hs output rows of image `ip`, on one
// wave (CO = false, NC = 1) or on a workgroup of kCoWaves waves (CO = true)
// whose lanes own NC consecutive columns each.
template <class Tr, int C, int SEG, int NPL, int KT, bool CO = false, int NC = 1>
__device__ __forceinline__ void run_task(const ImgParams& ip, int task, uint32_t* lds)
{
    constexpr int G = kWave / SEG;
    TaskGeom tg;
    tg.slice_off = 0;
    if (ip.nslices > 1) {                      // a stack of equal images: slice-major task order
        const int per = ip.nstrips * ip.nsegs;
        const int slice = task / per;
        task -= slice * per;
        tg.slice_off = int64_t(slice) * ip.slice_stride * Tr::kSize;
    }
    const int strip = task % ip.nstrips;
    const int seg = task / ip.nstrips;
    // the one-wave form starts pre < G rows earlier, so that emission starts
    // on a group boundary; the cooperative form emits per row
    const int pre = CO ? 0 : (G - (2 * ip.R + 1) % G) % G;
    tg.s0 = strip * kWave * NC;
    tg.o0 = tg.s0;
    if (CO && ip.step > 1) {                   // a strip of 64 kept output samples: its first input sample
        tg.s0 = (tg.o0 / C) * ip.step * C + tg.o0 % C;
    }
    tg.y0 = seg * ip.hs;
    tg.hs = min(ip.hs, ip.H - tg.y0);
    tg.a0 = floor_div(tg.s0 - (ip.R + 1) * C, ip.align) * ip.align;
    tg.off = tg.s0 - tg.a0;
    tg.emit0 = 2 * ip.R + 1 + pre;
    tg.niter = tg.emit0 + tg.hs;
    tg.ybase = tg.y0 - ip.R - 1 - pre;
    const int WC = ip.W * C;
    const bool interior = ip.vec && tg.a0 >= 0 && tg.a0 + SEG * NPL <= WC;
    if constexpr (CO) {
        // float images under zero extension take the masked offsets (an
        // instantiation of their own, so other images pay nothing for them)
        if constexpr (!Tr::kInt) {
            if (ip.boundary == RSG_ZERO) {
                if (interior) stream_task_co<Tr, C, SEG, NPL, KT, false, NC, true>(ip, tg, lds);
                else stream_task_co<Tr, C, SEG, NPL, KT, true, NC, true>(ip, tg, lds);
                return;
            }
        }
        // FP32 images planned with staged stores: interior tasks whose
        // output rows are 16-byte aligned store through the row tile
        if constexpr (NC == 1 && Tr::kSize == 4) {
            const uintptr_t db = reinterpret_cast<uintptr_t>(ip.dst) + uintptr_t(tg.slice_off);
            if (ip.staged && interior && ip.step <= 1 && ip.pstride <= 1 && (db % 16) == 0 &&
                ((ip.dst_stride * 4) % 16) == 0) {
                stream_task_co<Tr, C, SEG, NPL, KT, false, NC, false, kCoWaves, co_rows(NC), true>(ip, tg, lds);
                return;
            }
        }
        if (interior) stream_task_co<Tr, C, SEG, NPL, KT, false, NC>(ip, tg, lds);
        else stream_task_co<Tr, C, SEG, NPL, KT, true, NC>(ip, tg, lds);
    } else {
        if (interior) stream_task<Tr, C, SEG, NPL, KT, false>(ip, tg, lds);
        else stream_task<Tr, C, SEG, NPL, KT, true>(ip, tg, lds);
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

// One task per workgroup of kCoWaves waves (the cooperative form).
template <class Tr, int C, int SEG, int NPL, int KT, int NC>
__global__ __launch_bounds__(kCoWaves * kWave) void k_single_co(ImgParams ip)
{
    extern __shared__ uint32_t lds[];
    run_task<Tr, C, SEG, NPL, KT, true, NC>(ip, xcd_task(blockIdx.x, ip.ntasks), lds);
}

template <class Tr, int C, int SEG, int NPL, int KT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_single(ImgParams ip)
{
    extern __shared__ uint32_t lds[];
    run_task<Tr, C, SEG, NPL, KT>(ip, xcd_task(blockIdx.x, ip.ntasks), lds);
}

// Persistent batch kernel for one (dtype, C, K) class: each wave pops
// (image, task) items off a shared counter until the list is exhausted.
// The image's scan layout (SEG, NPL) selects among four instantiations.
template <class Tr, int C, int KT, int S0, int N0, int S1, int N1, int S2, int N2, int S3, int N3>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_batch(const ImgParams* __restrict__ imgs,
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
        if (ip.seg == S0 && ip.npl == N0) run_task<Tr, C, S0, N0, KT>(ip, bt.task, lds);
        else if (ip.seg == S1 && ip.npl == N1) run_task<Tr, C, S1, N1, KT>(ip, bt.task, lds);
        else if (ip.seg == S2 && ip.npl == N2) run_task<Tr, C, S2, N2, KT>(ip, bt.task, lds);
        else if (ip.seg == S3 && ip.npl == N3) run_task<Tr, C, S3, N3, KT>(ip, bt.task, lds);
        __syncthreads();
    }
}

// Persistent batch kernel, cooperative form: each workgroup pops (image,
// task) items and runs them on its kCoWaves waves.  LDS word 0 carries the
// popped index to every wave; the task's LDS starts 16 bytes later.
template <class Tr, int C, int KT, int NC, int S0, int N0, int S1, int N1, int S2, int N2, int S3, int N3>
__global__ __launch_bounds__(kCoWaves * kWave) void k_batch_co(const ImgParams* __restrict__ imgs,
                                                              const BatchTask* __restrict__ tasks, int ntasks,
                                                              unsigned* __restrict__ counter)
{
    extern __shared__ uint32_t lds[];
    uint32_t* tl = lds + kBatchSlotWords;
    for (;;) {
        if (threadIdx.x == 0) lds[0] = atomicAdd(counter, 1u);
        __syncthreads();
        const unsigned t = __builtin_amdgcn_readfirstlane(lds[0]);
        if (t >= unsigned(ntasks)) break;                  // the same for every wave
        const BatchTask bt = tasks[t];
        const ImgParams& ip = imgs[bt.img];
        if (ip.seg == S0 && ip.npl == N0) run_task<Tr, C, S0, N0, KT, true, NC>(ip, bt.task, tl);
        else if (ip.seg == S1 && ip.npl == N1) run_task<Tr, C, S1, N1, KT, true, NC>(ip, bt.task, tl);
        else if (ip.seg == S2 && ip.npl == N2) run_task<Tr, C, S2, N2, KT, true, NC>(ip, bt.task, tl);
        else if (ip.seg == S3 && ip.npl == N3) run_task<Tr, C, S3, N3, KT, true, NC>(ip, bt.task, tl);
        __syncthreads();                                   // every wave is done with the slot and the tiles
    }
}

}  // namespace dev
}  // namespace rsg
