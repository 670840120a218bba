// Device code of the fused running-sum Gaussian filter for gfx950 (MI355X).
//
// A task is a strip of 64 consecutive sample-columns (lane c owns column
// s0 + c in the column pass) and a segment of hs output rows of one image.
// It streams down the image in groups of G input rows, either on one wave
// (both passes, software-pipelined: stream_task) or on a workgroup whose
// row-pass and column-pass waves hand each group over through LDS
// (stream_task_pc, the default):
//
//   row pass (Section 3.3, Eq. alg1 / indep, along x): the row-pass wave splits into
//     G = 64 / SEG segments of SEG lanes; segment j takes input row
//     (group start + j), lane q of the segment holds NPL consecutive samples
//     of the row span [s0 - (R+1)C, s0 + 64 + RC) (border samples replicated,
//     reflected or zero).  The running sum I of each row is a serial scan inside the
//     lane plus a DPP scan of the lane totals across the segment; the G rows
//     of running sums go to LDS.  Then every lane (now: a column) takes
//     T(s) = sum_k w_k (I(s + r_k C) - I(s - (r_k+1) C)) for each row.
//   column pass (Section 3.4, the same along y): each lane adds T to its
//     running column sum J, writes J to an LDS ring holding the last
//     L >= 2R + 1 + G rows and emits, for the row R behind the newest,
//     out = sum_k w_k (J(y + r_k) - J(y - r_k - 1)).
//
// Global memory is addressed through buffer descriptors with row offsets in
// SGPRs: border zero-padding and dropped stores (rows outside the task, lanes
// past the image) use an out-of-range offset instead of branches, so every
// group issues a fixed number of memory instructions and the next groups'
// loads stay in flight while the current one is processed.
//
// FP32 / FP16 / BF16 accumulate in FP32.  Running sums are tile-local and
// offset: each group of rows subtracts one of its samples (added back
// through the DC gain of the boxes) and each column its first T value, which
// keeps the summed magnitudes, and hence the rounding of the differences,
// small.  Both forms perform the same FP32 operations in the same order.
// uint8 uses exact uint32 arithmetic (differences are exact modulo 2^32 and
// every box sum is < 2^32), integer weights m_k and one exact rounding of
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

// uint8 output: round half up of U / G^2, exactly.  N = U + floor(G^2/2) < 256 G^2.
__device__ __forceinline__ uint32_t exact_round_div_u(uint64_t U, uint64_t G2, uint64_t G2half, float invG2)
{
    const uint64_t N = U + G2half;
    const float nf = float(uint32_t(N >> 32)) * 4294967296.0f + float(uint32_t(N));
    uint32_t q = uint32_t(nf * invG2);
    const uint64_t prod = uint64_t(q) * G2;
    if (prod > N) q -= 1;
    else if (N - prod >= G2) q += 1;
    return q;
}
__device__ __forceinline__ uint32_t exact_round_div(uint64_t U, const ImgParams& ip)
{
    return exact_round_div_u(U, ip.G2, ip.G2half, ip.invG2);
}

// The same in FP64 for U < 2^53 given exactly as a double (sum of FP64
// products that are all exact): quotient estimate from the reciprocal, then
// one exact remainder N - q G^2 (an FMA) decides a +-1 correction.
__device__ __forceinline__ uint32_t exact_round_div_f64(double U, double G2, double G2half, double invG2)
{
    const double N = U + G2half;                       // exact: < 2^53
    double q = floor(N * invG2);
    const double r = fma(-q, G2, N);                   // exact remainder
    q += (r >= G2) ? 1.0 : 0.0;
    q -= (r < 0.0) ? 1.0 : 0.0;
    return uint32_t(q);
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
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, voff, soff, 0);
}
template <>
__device__ __forceinline__ void store_out<TrF16>(__amdgpu_buffer_rsrc_t rs, int voff, int soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), rs, voff, soff, 0);
}
template <>
__device__ __forceinline__ void store_out<TrBF16>(__amdgpu_buffer_rsrc_t rs, int voff, int soff, float v)
{
    const uint32_t u = __float_as_uint(v);                          // finite v
    __builtin_amdgcn_raw_buffer_store_b16(uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16), rs, voff, soff, 0);
}

// Per-task constants.
struct TaskGeom {
    int s0, y0, hs, a0, off, niter, ybase;
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
    constexpr int PW = SEG * NPL;              // span capacity
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
            if constexpr (kInt) __builtin_amdgcn_raw_buffer_store_b8(uint8_t(0), rs_dst, kDropOffset - 64 * (b * G + j), 0, 0);
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
            off = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(Tr::unpack(bf.w, 0))));
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
                // U = sum m_k D_k < 2^52: every product and partial sum is an
                // exact FP64 value, and FP64 FMAs run at the FP32 rate here
                double U = 0.0;
#pragma unroll
                for (int k = 0; k < KT; ++k)
                    U = fma(double(wm[k]), double(uint32_t(rv[j][2 * k] - rv[j][2 * k + 1])), U);
                __builtin_amdgcn_raw_buffer_store_b8(uint8_t(exact_round_div_f64(U, ip.G2d, ip.G2halfd, ip.invG2d)),
                                                     rs_dst, voff, 0, 0);
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
            if constexpr (kInt) __builtin_amdgcn_raw_buffer_store_b8(uint8_t(0), rs_dst, kDropOffset - 64 * (base + j), 0, 0);
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
            c2 = T[0];                                  // the column offset: the task's first row
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
// Producer / consumer form of the streaming loop: one task per workgroup of
// kProducers + 1 waves.  The row pass is independent from row to row, so
// waves 0 .. NPR-1 each run it for every NPR-th group (loads, running sums,
// row box differences) and hand the group's row results to the last wave
// through an LDS queue; that wave runs the column pass of the groups in
// order (running column sums in the ring, column box differences, stores).
// Step s covers groups s NPR .. s NPR + NPR - 1 and ends, for the row-pass
// waves, in one workgroup barrier: at barrier s queue slot s & 1 holds the
// step's groups, and the slot the row-pass waves fill next was read by the
// column-pass wave before it reached barrier s.  Every wave takes the same
// number of barriers.  The split multiplies the waves per task without
// adding halo rows, and each wave's chain of dependent LDS round trips is a
// fraction of the one-wave form's.
// --------------------------------------------------------------------------
template <class Tr, int C, int SEG, int NPL, int KT, bool EDGE>
__device__ __forceinline__ void stream_task_pc(const ImgParams& ip, const TaskGeom& tg, uint32_t* lds)
{
    using Acc = typename Tr::Acc;
    constexpr bool kInt = Tr::kInt;
    constexpr int G = kWave / SEG;
    constexpr int PW = SEG * NPL;
    constexpr int PP = row_tile_pitch(SEG, NPL);
    constexpr int RP = kWave;
    constexpr int PF = kPrefetch;
    constexpr int es = Tr::kSize;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int R = ip.R;
    const int L = ip.L;
    const int H = ip.H;
    const int W = ip.W;
    const int WC = W * C;
    const int boundary = ip.boundary;
    static_assert(PW <= PP, "tile pitch");

    constexpr int NPR = kProducers;
    // LDS: [row tiles NPR x G x PP][queue 2 x NPR x G x 64][ring (L + G) x 64]
    Acc* P = reinterpret_cast<Acc*>(lds);
    Acc* Q = P + NPR * G * PP;
    Acc* ring = Q + 2 * NPR * G * kWave;

    const int ngroups = (tg.niter + G - 1) / G;
    // steps of NPR groups, a multiple of PF; every wave: one barrier per step
    const int nsteps = (ngroups + NPR * PF - 1) / (NPR * PF) * PF;
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

    if (wave < NPR) {
        // ---------------- row pass of groups wave, wave + NPR, ... ----------------
        Acc* Pt = P + wave * G * PP;
        const int jrow = lane / SEG;
        const int q = lane % SEG;
        const int y_lo = max(0, tg.ybase);
        const char* sbase = reinterpret_cast<const char*>(ip.src) + tg.slice_off + int64_t(y_lo) * sstride;
        const __amdgpu_buffer_rsrc_t rs_src = make_rsrc(sbase, int64_t(H - 1 - y_lo) * sstride + int64_t(WC) * es);
        const int cs = tg.a0 + NPL * q;
        const int vec_voff = cs * es;
        int eoff[EDGE ? NPL : 1];
        if constexpr (EDGE) {
            const int x0 = floor_div(cs, C);
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                const int x = x0 + i / C;
                const int xe = ext_index(x, W, boundary);
                eoff[i] = (xe >= 0) ? (xe * C + i % C) * es : -1;
            }
        }
        const int sstride32 = int(sstride);
        // 4-byte samples on a border task: a lane whose chunk lies inside the
        // row loads it as vectors, the others per element; each lane's other
        // load reads out of range (zeros), and the two are ORed when the group
        // is used, so no branch diverges and every wait stays exact
        constexpr bool kSplit = EDGE && Tr::kSize == 4;
        const bool lane_vec = ip.vec && cs >= 0 && cs + NPL <= WC;
        auto load = [&](Chunk<Tr, NPL>& ch, Chunk<Tr, NPL>& ech, int st) {    // the group of step st
            const int y = tg.ybase + (st * NPR + wave) * G + jrow;
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
        int tp[KT], tm[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            tp[k] = tg.off + lane + ip.r[k] * C;
            tm[k] = tg.off + lane - (ip.r[k] + 1) * C;
        }
        Chunk<Tr, NPL> buf[PF];
        Chunk<Tr, NPL> ebuf[kSplit ? PF : 1];
#pragma unroll
        for (int b = 0; b < PF; ++b) {          // this wave issues loads only: every wait is exact
            __builtin_amdgcn_sched_barrier(0);
            load(buf[b], ebuf[kSplit ? b : 0], b);
        }
        __builtin_amdgcn_sched_barrier(0);
        for (int g = 0; g < nsteps; g += PF) {
#pragma unroll
            for (int b = 0; b < PF; ++b) {
                const int gg = g + b;
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (kSplit) {
#pragma unroll
                    for (int k = 0; k < Chunk<Tr, NPL>::kWords; ++k) buf[b].w[k] |= ebuf[b].w[k];
                }
                Acc v[NPL];
                float off = 0.0f;
                if constexpr (!kInt) {
                    off = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(Tr::unpack(buf[b].w, 0))));
#pragma unroll
                    for (int i = 0; i < NPL; ++i) v[i] = Tr::unpack(buf[b].w, i) - off;
                } else {
#pragma unroll
                    for (int i = 0; i < NPL; ++i) v[i] = Tr::unpack(buf[b].w, i);
                }
                __builtin_amdgcn_sched_barrier(0);
                load(buf[b], ebuf[kSplit ? b : 0], gg + PF);
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
                // row box differences (Eq. indep), lane = column; floats add
                // the group offset's share
                float init = 0.0f;
                if constexpr (!kInt) init = off * dc;
                Acc T[G];
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const Acc* Pj = Pt + j * PP;
                    Acc t;
                    if constexpr (kInt) {
                        t = 0;
#pragma unroll
                        for (int k = 0; k < KT; ++k) t += __umul24(wm[k], Pj[tp[k]] - Pj[tm[k]]);
                    } else {
                        t = fmaf(wf[0], Pj[tp[0]] - Pj[tm[0]], init);
#pragma unroll
                        for (int k = 1; k < KT; ++k) t = fmaf(wf[k], Pj[tp[k]] - Pj[tm[k]], t);
                    }
                    T[j] = t;
                }
                Acc* Qs = Q + ((gg & 1) * NPR + wave) * G * kWave;
#pragma unroll
                for (int j = 0; j < G; ++j) Qs[j * kWave + lane] = T[j];
                __syncthreads();
            }
        }
    } else {
        // ---------------- column pass ----------------
        // Output rows of this task: y0 .. y0 + hs - 1, or with a strided
        // output (every ostep-th row and pixel, compacted) the kept rows
        // oq0 .. oq1 - 1 of the output image; rows outside the descriptor
        // and dropped columns are stored to out-of-range offsets.
        const int ostep = ip.step > 1 ? ip.step : 1;
        const int s = tg.s0 + lane;
        int oq0 = tg.y0, nrows = tg.hs, orow_len = WC;
        uint32_t ocol = (s < WC) ? uint32_t(s * es) : kDropColumn;
        if (ostep > 1) {
            oq0 = (tg.y0 + ostep - 1) / ostep;
            nrows = (tg.y0 + tg.hs - 1) / ostep - oq0 + 1;
            orow_len = (W + ostep - 1) / ostep * C;
            const int x = s / C;
            ocol = (s < WC && x % ostep == 0) ? uint32_t(((x / ostep) * C + (s - x * C)) * es) : kDropColumn;
        }
        const char* dbase = reinterpret_cast<char*>(ip.dst) + tg.slice_off + int64_t(oq0) * dstride;
        const __amdgpu_buffer_rsrc_t rs_dst =
            make_rsrc(dbase, nrows > 0 ? int64_t(nrows - 1) * dstride + int64_t(orow_len) * es : 0);
        const uint32_t dstr = uint32_t(dstride);
        Acc colacc = Acc(0);
        float c2 = 0.0f;
        float c2dc = 0.0f;
        int slot0 = 0;
        for (int st = 0; st < nsteps; ++st) {
            __syncthreads();
#pragma unroll 1
          for (int pq = 0; pq < NPR; ++pq) {
            const int g = st * NPR + pq;
            const Acc* Qs = Q + ((st & 1) * NPR + pq) * G * kWave;
            if constexpr (!kInt) {
                if (g == 0) {                    // the column offset: the task's first row
                    c2 = Qs[lane];
                    c2dc = c2 * dc;
                }
            }
            const int wbase = slot0 * RP + lane;
            Acc cj[G];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if constexpr (kInt) colacc += Qs[j * kWave + lane];
                else colacc += Qs[j * kWave + lane] - c2;
                cj[j] = colacc;
                ring[wbase + j * RP] = colacc;
            }
            if (slot0 == 0) {                       // slots 0 .. G-1 also live at L .. L+G-1
#pragma unroll
                for (int j = 0; j < G; ++j) ring[(L + j) * RP + lane] = cj[j];
            }
            wave_lds_fence();
            Acc rv[G][2 * KT];
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                int a = slot0 - R + ip.r[k];
                int b = slot0 - R - ip.r[k] - 1;
                a += (a < 0) ? L : 0;
                b += (b < 0) ? L : 0;
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    rv[j][2 * k] = ring[a * RP + lane + j * RP];
                    rv[j][2 * k + 1] = ring[b * RP + lane + j * RP];
                }
            }
            const int it0 = g * G;
            auto emit = [&](int j, int voff) {
                if constexpr (kInt) {
                    double U = 0.0;
#pragma unroll
                    for (int k = 0; k < KT; ++k)
                        U = fma(double(wm[k]), double(uint32_t(rv[j][2 * k] - rv[j][2 * k + 1])), U);
                    __builtin_amdgcn_raw_buffer_store_b8(uint8_t(exact_round_div_f64(U, ip.G2d, ip.G2halfd, ip.invG2d)),
                                                         rs_dst, voff, 0, 0);
                } else {
                    float o = c2dc;
#pragma unroll
                    for (int k = 0; k < KT; ++k) o = fmaf(wf[k], rv[j][2 * k] - rv[j][2 * k + 1], o);
                    store_out<Tr>(rs_dst, voff, 0, o);
                }
            };
            if (ostep == 1) {
                const uint32_t og = (it0 >= tg.emit0) ? ocol + uint32_t(it0 - tg.emit0) * dstr : uint32_t(kDropOffset);
#pragma unroll
                for (int j = 0; j < G; ++j) emit(j, int(og + uint32_t(j) * dstr));
            } else {
                // strided output: rows y = 0, ostep, 2 ostep, ... only (a
                // uniform test per row), stored at output row y / ostep
                const int yb = tg.y0 + it0 - tg.emit0;      // image row of this group's first output
                int q = floor_div(yb, ostep);
                int rr = yb - q * ostep;
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    if (rr == 0 && it0 + j >= tg.emit0)
                        emit(j, int(ocol + uint32_t(q - oq0) * dstr));
                    if (++rr == ostep) { rr = 0; ++q; }
                }
            }
            slot0 += G;
            slot0 -= (slot0 >= L) ? L : 0;
          }
        }
    }
}

// One task: 64 sample-columns x hs output rows of image `ip`.
template <class Tr, int C, int SEG, int NPL, int KT, bool PC = false>
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
    const int pre = (G - (2 * ip.R + 1) % G) % G;
    tg.s0 = strip * kWave;
    tg.y0 = seg * ip.hs;
    tg.hs = min(ip.hs, ip.H - tg.y0);
    tg.a0 = floor_div(tg.s0 - (ip.R + 1) * C, ip.align) * ip.align;
    tg.off = tg.s0 - tg.a0;
    tg.emit0 = 2 * ip.R + 1 + pre;
    tg.niter = tg.emit0 + tg.hs;
    tg.ybase = tg.y0 - ip.R - 1 - pre;
    const int WC = ip.W * C;
    const bool interior = ip.vec && tg.a0 >= 0 && tg.a0 + SEG * NPL <= WC;
    if constexpr (PC) {
        if (interior) stream_task_pc<Tr, C, SEG, NPL, KT, false>(ip, tg, lds);
        else stream_task_pc<Tr, C, SEG, NPL, KT, true>(ip, tg, lds);
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

// One task per workgroup of two waves (row-pass and column-pass waves).
template <class Tr, int C, int SEG, int NPL, int KT>
__global__ __launch_bounds__((kProducers + 1) * kWave) void k_single_pc(ImgParams ip)
{
    extern __shared__ uint32_t lds[];
    run_task<Tr, C, SEG, NPL, KT, true>(ip, xcd_task(blockIdx.x, ip.ntasks), lds);
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

// Persistent batch kernel, two-wave form: each workgroup pops (image, task)
// items and runs them as a row-pass / column-pass pair.  LDS word 0 carries
// the popped index to both waves; the task's LDS starts 16 bytes later.
template <class Tr, int C, int KT, int S0, int N0, int S1, int N1, int S2, int N2, int S3, int N3>
__global__ __launch_bounds__((kProducers + 1) * kWave) void k_batch_pc(const ImgParams* __restrict__ imgs,
                                                       const BatchTask* __restrict__ tasks, int ntasks,
                                                       unsigned* __restrict__ counter)
{
    extern __shared__ uint32_t lds[];
    uint32_t* tl = lds + kBatchSlotWords;
    for (;;) {
        if (threadIdx.x == 0) lds[0] = atomicAdd(counter, 1u);
        __syncthreads();
        const unsigned t = __builtin_amdgcn_readfirstlane(lds[0]);
        if (t >= unsigned(ntasks)) break;                  // the same for both waves
        const BatchTask bt = tasks[t];
        const ImgParams& ip = imgs[bt.img];
        if (ip.seg == S0 && ip.npl == N0) run_task<Tr, C, S0, N0, KT, true>(ip, bt.task, tl);
        else if (ip.seg == S1 && ip.npl == N1) run_task<Tr, C, S1, N1, KT, true>(ip, bt.task, tl);
        else if (ip.seg == S2 && ip.npl == N2) run_task<Tr, C, S2, N2, KT, true>(ip, bt.task, tl);
        else if (ip.seg == S3 && ip.npl == N3) run_task<Tr, C, S3, N3, KT, true>(ip, bt.task, tl);
        __syncthreads();                                   // both waves are done with the slot and the tiles
    }
}

}  // namespace dev
}  // namespace rsg
