// The pass along z of a volume: D slices of `plane` = H W C FP32 samples.
// The separable filter takes one more 1D pass per extra axis (Section 4's
// d-dimensional remark); along z it is the same running sum (Eq. alg1) and
// K box differences (Eq. indep) as along y in the fused kernel.
//
// Task: 64 consecutive samples of a slice (lane = one z column) and a
// segment of hz output slices.  The lane walks positions t = z0 - R - 1 ..
// z0 + hz - 1 + R, keeps the running sum P of (f - c) (c: the column's first
// loaded value, restored through the boxes' DC gain, so sums stay at the size
// of local variations; 0 under zero extension) in an LDS ring of 2R + 2 entries, and emits slice
// z = t - R once the ring holds S(z + R) back to S(z - R - 1).  Loads of
// slice positions are prefetched PFZ steps ahead in registers; consecutive
// lanes read consecutive addresses.
#pragma once

#include "rsg_device.h"

namespace rsg {
namespace dev {

template <int KT, int PFZ>
__global__ __launch_bounds__(256) void k_zpass(ZParams p)
{
    extern __shared__ float zl[];
    const int wpb = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int task = blockIdx.x * wpb + wave;
    if (task >= p.ntasks) return;              // whole waves only; no barriers below
    const int L = p.L;
    float* ring = zl + wave * L * kWave;

    const int col = task % p.ncols;
    const int seg = task / p.ncols;
    const int64_t s = int64_t(col) * kWave + lane;
    const bool live = s < p.plane;
    const int64_t sl = live ? s : p.plane - 1;  // lanes past the slice read a valid sample, store nothing
    const int z0 = seg * p.hz;
    const int hz = min(p.hz, p.D - z0);
    const int R = p.R;
    const int niter = hz + 2 * R + 1;           // ring indices 0 .. niter - 1 (index 0: P = 0)
    const int tb = z0 - R - 1;                  // position of ring index 0

    float wf[KT];
    int rp[KT], rm[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        wf[k] = p.wf[k];
        rp[k] = -R + p.r[k];                    // S(z + r_k) relative to the newest index
        rm[k] = -R - p.r[k] - 1;                // S(z - r_k - 1)
    }
    const float dc = p.dc32;

    auto load = [&](int i) -> float {           // f at ring index i >= 1 (position tb + i)
        const int t = ext_index(tb + i, p.D, p.boundary);
        return t < 0 ? 0.0f : p.src[int64_t(t) * p.plane + sl];
    };

    float buf[PFZ];
#pragma unroll
    for (int j = 0; j < PFZ; ++j) buf[j] = load(1 + j);
    const float c = (p.boundary == RSG_ZERO) ? 0.0f : buf[0];    // zero extension: outside slices stay 0
    const float cdc = c * dc;

    float P = 0.0f;
    int wi = 0;                                 // ring slot of index i
    ring[lane] = 0.0f;
    for (int i0 = 1; i0 < niter; i0 += PFZ) {
#pragma unroll
        for (int j = 0; j < PFZ; ++j) {
            const int i = i0 + j;
            const float f = buf[j];
            buf[j] = load(min(i + PFZ, niter - 1));
            if (i < niter) {
                wi = (wi + 1 == L) ? 0 : wi + 1;
                P += f - c;
                ring[wi * kWave + lane] = P;
                if (i >= 2 * R + 1) {
                    float o = cdc;
#pragma unroll
                    for (int k = 0; k < KT; ++k) {
                        int a = wi + rp[k];
                        int b = wi + rm[k];
                        a += (a < 0) ? L : 0;
                        b += (b < 0) ? L : 0;
                        o = fmaf(wf[k], ring[a * kWave + lane] - ring[b * kWave + lane], o);
                    }
                    const int z = tb + i - R;
                    if (live) __builtin_nontemporal_store(o, p.dst + int64_t(z) * p.plane + s);   // output: not read back
                }
            }
        }
    }
}

}  // namespace dev
}  // namespace rsg
