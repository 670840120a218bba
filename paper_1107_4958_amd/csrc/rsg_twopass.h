// Two-pass path for wide boxes: each pass is a row filter whose output is
// stored transposed, so the second pass filters the image's columns as rows.
//
//   pass A: image rows (W*C interleaved samples, taps C samples apart)
//           -> intermediate (W*C) x H, FP32 (uint32 for uint8 images)
//   pass B: intermediate rows (one image column of one channel, H samples)
//           -> image H x W x C in the image's element type
//
// Both passes compute the same thing as the fused kernel (Section 3.3,
// Eq. alg1 / indep along x, then along y, Section 3.4); they only exchange
// the row-pass result through HBM.  The fused kernel keeps, per column, a
// ring of 2R + 2 running sums in LDS and re-reads 2R + 1 rows per segment;
// for wide boxes that ring caps occupancy and the halo dominates.  Here a
// wave streams one whole row in chunks of CW = 64 NPL samples and keeps only
// a window of (2R + 1) C running sums of the previous chunk, so every input
// sample is loaded once per pass.
//
// Workgroup: TR waves (16; 8 when a 16-row window would not fit the LDS),
// one row each.  Chunk k of a row loads input
// samples [k CW, (k + 1) CW) and emits outputs [k CW - R C, (k + 1) CW - R C)
// (the window reaches R C samples beyond each output).  The window holds
// running sums of positions [k CW - (2R + 1) C, (k + 1) CW); after the chunk
// its last (2R + 1) C entries move to the front.  Outputs go to an LDS
// staging tile [CW][TR + 1], then the workgroup stores them
// transposed: TR consecutive elements per output row.  With two
// staging tiles (ST = 2, when the LDS allows) chunk k + 1 fills the other
// tile while chunk k's stores drain, and one barrier per chunk suffices.
//
// Precision: integer inputs use exact uint32 running sums (differences are
// exact modulo 2^32).  Float inputs subtract a per-row reference (the row's
// first sample of each channel) before summing, restored through the DC gain
// of the boxes, and rebase the window to its first entry at every chunk, so
// no running sum spans more than CW + (2R + 1) C samples.  Under zero
// extension the reference is 0: outside samples would otherwise enter as
// minus the reference, and a box lying mostly outside the row would be a
// small difference of large sums.
#pragma once

#include "rsg_device.h"

namespace rsg {
namespace dev {

constexpr int kPassRows = 16;                  // waves (rows) per workgroup (8 for the widest windows)

// What a pass writes.
enum PassOut { kOutMidU32 = 0, kOutMidF32 = 1, kOutU8 = 2, kOutF32 = 3, kOutF16 = 4, kOutBF16 = 5 };

// Intermediate element as an input trait: exact uint32 running sums.
struct TrU32 {
    using In = uint32_t;
    using Acc = uint32_t;
    static constexpr int kSize = 4;
    static constexpr bool kInt = true;
    __device__ static Acc unpack(const uint32_t* w, int i) { return w[i]; }
};

template <int OUT> struct OutSize { static constexpr int v = (OUT == kOutU8) ? 1 : (OUT >= kOutF16 ? 2 : 4); };

// Stores one staged 32-bit word as the output element.  (Through the
// caches: a wave writes 16 consecutive elements of a row, partial lines that
// the L2 combines before they reach memory.)
template <int OUT>
__device__ __forceinline__ void store_pass_out(void* dst, int64_t idx, uint32_t w)
{
    if constexpr (OUT == kOutU8) static_cast<uint8_t*>(dst)[idx] = uint8_t(w);
    else if constexpr (OUT == kOutF16 || OUT == kOutBF16) static_cast<uint16_t*>(dst)[idx] = uint16_t(w);
    else static_cast<uint32_t*>(dst)[idx] = w;
}

// Boundary-extended position inside a row of `len` samples whose channels
// repeat every C samples (the pixel index is extended, the channel kept):
// -1 means a zero sample.
template <int C>
__device__ __forceinline__ int pass_clamp(int pos, int len, int boundary)
{
    if (pos >= 0 && pos < len) return pos;
    const int x = floor_div(pos, C);
    const int c = pos - x * C;
    const int xe = ext_index(x, len / C, boundary);
    return xe < 0 ? -1 : xe * C + c;
}

template <class TrIn, int OUT, int C, int NPL, int KT, int ST, int TR>
__device__ __forceinline__ void pass_rows(const PassParams& p, int block, uint32_t* lds)
{
    using Acc = typename TrIn::Acc;
    constexpr bool kInt = TrIn::kInt;
    constexpr int es = TrIn::kSize;
    constexpr int CW = kWave * NPL;
    constexpr int SP = TR + 1;                     // staging pitch (words): conflict-free row writes
    static_assert(NPL % C == 0 && NPL % 4 == 0, "chunk must hold whole pixels and 16-byte groups");
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int R = p.R;
    const int HW = (2 * R + 1) * C;                // window head: running sums kept from the previous chunk
    const int len = p.len;
    const int boundary = p.boundary;

    // per-wave window (the head starts so that the new part is 16-byte aligned)
    Acc* win = reinterpret_cast<Acc*>(lds) + wave * p.win_pitch + p.win_shift;
    uint32_t* stg0 = lds + TR * p.win_pitch;

    const int row0 = block * TR;
    const int row = min(row0 + wave, p.rows - 1);  // a wave past the last row repeats it and stores nothing
    const char* sbase = static_cast<const char*>(p.src) + int64_t(row) * p.src_stride * es;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(sbase, int64_t(len) * es);
    const bool vec = p.vec != 0;

    int tp[KT], tm[KT];
    float wf[KT];
    uint32_t wm[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        tp[k] = lane + (R + 1 + p.r[k]) * C;
        tm[k] = lane + (R - p.r[k]) * C;
        wf[k] = p.wf[k];
        wm[k] = p.m[k];
    }
    const float dc = p.dc32;

    // per-channel reference (float types) and the one of each output slot
    float off[C];
    float offo[NPL];
    if constexpr (!kInt) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            // zero extension keeps no reference: outside samples must stay 0,
            // or boxes reaching far outside would cancel against it
            const int q = pass_clamp<C>(c, len, RSG_REPLICATE);
            off[c] = (boundary == RSG_ZERO) ? 0.0f : Tr_load_one<TrIn>(rs, q * es);
        }
#pragma unroll
        for (int t = 0; t < NPL; ++t) {
            const int c = (lane + kWave * t) % C;   // output o = lane + 64 t has channel o mod C
            float v = off[0];
#pragma unroll
            for (int cc = 1; cc < C; ++cc) v = (c == cc) ? off[cc] : v;
            offo[t] = v;
        }
    }

    // Loads NPL samples at positions pos0 + NPL lane + i (boundary-extended),
    // minus the channel reference.
    auto load_samples = [&](int pos0, Acc (&v)[NPL]) {
        const int a = pos0 + NPL * lane;
        Chunk<TrIn, NPL> ch;
        if (vec && pos0 >= 0 && pos0 + CW <= len) {
            load_chunk_vec<TrIn, NPL>(ch, rs, a * es, 0);
        } else {
            int eo[NPL];
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
                const int q = pass_clamp<C>(a + i, len, boundary);
                eo[i] = q < 0 ? kDropOffset : q * es;
            }
            load_chunk_elem<TrIn, NPL>(ch, rs, eo, 0);
        }
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            if constexpr (kInt) v[i] = TrIn::unpack(ch.w, i);
            else v[i] = TrIn::unpack(ch.w, i) - off[i % C];
        }
    };

    // Running sums of NPL consecutive samples per lane with channel stride C,
    // continued from carry[c]; written to win[dst + NPL lane + i].
    auto scan_store = [&](Acc (&v)[NPL], const Acc (&carry)[C], int dst, bool aligned) {
#pragma unroll
        for (int i = C; i < NPL; ++i) v[i] = v[i] + v[i - C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const Acc tot = v[NPL - C + c];
            const Acc ex = segment_inclusive_scan<kWave>(tot) - tot + carry[c];
#pragma unroll
            for (int i = c; i < NPL; i += C) v[i] = v[i] + ex;
        }
        if (aligned) {
            using Acc4 = typename std::conditional<kInt, uint4, float4>::type;
            Acc4* d4 = reinterpret_cast<Acc4*>(win + dst + NPL * lane);
#pragma unroll
            for (int h = 0; h < NPL / 4; ++h) {
                Acc4 t4;
                t4.x = v[4 * h]; t4.y = v[4 * h + 1]; t4.z = v[4 * h + 2]; t4.w = v[4 * h + 3];
                d4[h] = t4;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NPL; ++i)
                if (NPL * lane + i < HW) win[dst + NPL * lane + i] = v[i];
        }
    };

    Acc carry[C];
#pragma unroll
    for (int c = 0; c < C; ++c) carry[c] = Acc(0);
    {   // head of chunk 0: positions [-HW, 0) (all boundary samples); HW <= CW
        Acc v[NPL];
        load_samples(-HW, v);
        scan_store(v, carry, 0, false);
        wave_lds_fence();
#pragma unroll
        for (int c = 0; c < C; ++c) carry[c] = win[HW - C + c];
    }

    const int nchunks = (len + R * C + CW - 1) / CW;
    constexpr int PFC = 1;                         // chunks of loads in flight ahead of the one in use
    Acc vq[PFC][NPL];
#pragma unroll
    for (int b = 0; b < PFC; ++b) load_samples(b * CW, vq[b]);
    for (int k = 0; k < nchunks; ++k) {
        Acc v[NPL];
#pragma unroll
        for (int i = 0; i < NPL; ++i) v[i] = vq[0][i];
#pragma unroll
        for (int b = 0; b + 1 < PFC; ++b)
#pragma unroll
            for (int i = 0; i < NPL; ++i) vq[b][i] = vq[b + 1][i];
        if (k + PFC < nchunks) load_samples((k + PFC) * CW, vq[PFC - 1]);   // chunks in flight
        scan_store(v, carry, HW, true);
        wave_lds_fence();

        uint32_t* stg = stg0 + (ST > 1 ? (k & 1) * CW * SP : 0);
        // outputs o = lane + 64 t of this chunk (position k CW - R C + o)
#pragma unroll
        for (int t = 0; t < NPL; ++t) {
            const int o = kWave * t;
            uint32_t word;
            if constexpr (OUT == kOutMidU32) {
                uint32_t s = 0;
#pragma unroll
                for (int kk = 0; kk < KT; ++kk) s += __umul24(wm[kk], win[o + tp[kk]] - win[o + tm[kk]]);
                word = s;
            } else if constexpr (OUT == kOutU8) {
                uint64_t N = p.G2half;                // exact: see the fused kernel
#pragma unroll
                for (int kk = 0; kk < KT; ++kk) N += uint64_t(wm[kk]) * uint64_t(win[o + tp[kk]] - win[o + tm[kk]]);
                word = round_quotient(N, p.G2, p.invG2, p.qsh);
            } else {
                float s = offo[t] * dc;
#pragma unroll
                for (int kk = 0; kk < KT; ++kk) s = fmaf(wf[kk], win[o + tp[kk]] - win[o + tm[kk]], s);
                if constexpr (OUT == kOutF16) word = __half_as_ushort(__float2half_rn(s));
                else if constexpr (OUT == kOutBF16) {
                    const uint32_t u = __float_as_uint(s);
                    word = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
                } else word = __float_as_uint(s);
            }
            stg[(o + lane) * SP + wave] = word;
        }

        // move the last HW running sums to the front; floats rebase them
        {
            Acc base[C];
#pragma unroll
            for (int c = 0; c < C; ++c) base[c] = kInt ? Acc(0) : win[CW + c];
            for (int j = lane; j < HW; j += kWave) {
                Acc x = win[CW + j];
                if constexpr (!kInt) {
                    Acc b = base[0];
#pragma unroll
                    for (int c = 1; c < C; ++c) b = (j % C == c) ? base[c] : b;
                    x = x - b;
                }
                win[j] = x;
            }
            wave_lds_fence();
#pragma unroll
            for (int c = 0; c < C; ++c) carry[c] = win[HW - C + c];
        }
        __syncthreads();

        // transposed store: element (x, row0 + w) for x = k CW - R C + o; a
        // strided pass keeps pixels x / C = 0, ostep, 2 ostep, ... and stores
        // pixel j ostep at j (channels kept)
        const int x0 = k * CW - R * C;
        const int ostep = p.ostep;
        for (int idx = threadIdx.x; idx < CW * TR; idx += TR * kWave) {
            const int o = idx / TR;
            const int w = idx % TR;
            const int x = x0 + o;
            if (x >= 0 && x < len && row0 + w < p.rows) {
                int xo = x;
                if (ostep > 1) {
                    const int px = x / C;
                    const int q = px / ostep;
                    if (px - q * ostep) continue;
                    xo = q * C + (x - px * C);
                }
                store_pass_out<OUT>(p.dst, int64_t(xo) * p.dst_stride + row0 + w, stg[o * SP + w]);
            }
        }
        // with two staging tiles the next chunk writes the other one; the
        // barrier of that chunk orders this chunk's reads before its reuse
        if (ST == 1) __syncthreads();
    }
}

template <class TrIn, int OUT, int C, int NPL, int KT, int ST, int TR>
__global__ __launch_bounds__(TR * kWave) void k_pass(PassParams p)
{
    extern __shared__ uint32_t lds[];
    pass_rows<TrIn, OUT, C, NPL, KT, ST, TR>(p, blockIdx.x, lds);
}

// The same pass over the row blocks of several images (one per workgroup).
template <class TrIn, int OUT, int C, int NPL, int KT, int ST, int TR>
__global__ __launch_bounds__(TR * kWave) void k_pass_batch(const PassParams* __restrict__ pps,
                                                           const int2* __restrict__ tasks)
{
    extern __shared__ uint32_t lds[];
    const int2 t = tasks[blockIdx.x];
    pass_rows<TrIn, OUT, C, NPL, KT, ST, TR>(pps[t.x], t.y, lds);
}

}  // namespace dev
}  // namespace rsg
