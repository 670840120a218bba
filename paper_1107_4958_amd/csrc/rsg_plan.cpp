// Tile planning: validates one image descriptor, fits its boxes (cached, or
// checks the caller's), chooses the path (fused kernel, or two passes for
// wide boxes and strided output) and, for the fused path, the scan chunk and
// segment height of its tasks (strips are 64 sample-columns wide: one column
// per lane); for the two-pass path, the chunk, staging and rows per
// workgroup of each pass.
//
// The choice is a pure function of the image's own parameters (dtype, C, H,
// W, the box half-widths, boundary, pointer alignment), never of the batch it
// arrives in, so an image filters to the same bits alone or in a mix.  Shapes
// come from a tuning table (segment heights and the path, measured on the
// device by the package's autotune.py) when one is loaded, otherwise from
// the built-in rule below.
#include "rsg_internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace rsg {

namespace {

constexpr uint32_t kLdsLimit = 160u * 1024u;    // gfx950: 160 KiB of LDS per CU

int gcd_i(int a, int b) { while (b) { int t = a % b; a = b; b = t; } return a; }
int lcm_i(int a, int b) { return a / gcd_i(a, b) * b; }

// Tuning table (text): lines "dtype C rlo rhi nlo nhi hs [nc [lo]]", '#'
// starts a comment.  An image of dtype and channel count C whose largest
// half-width R lies in [rlo, rhi] and whose work size n = strips * H (strips
// of 64 samples) lies in [nlo, nhi] takes the fused kernel with segment
// height hs from the first matching line, or the two-pass path if hs is -1;
// nc > 1 selects the wide column form (wide_nc(C) columns per lane), 1 one
// column per lane, 0 or none the built-in rule; lo > 0 starts the search for
// a row-scan layout at layout lo (wider rows per group, fewer rows), 0 or
// none at the first.
struct TuneEntry { int dtype, C, rlo, rhi; int64_t nlo, nhi; int hs, nc, lo, st; };
std::once_flag g_tune_once;
std::vector<TuneEntry> g_tune;
std::atomic<int> g_hs_override{0};
std::atomic<int> g_path_override{0};
std::atomic<int> g_nc_override{0};
std::atomic<int> g_lo_override{0};
std::atomic<int> g_st_override{0};

// Two-pass geometry: the smallest chunk (64 NPL samples) that holds the
// window head (2R + 1) C and fits the LDS with one staging tile (0 if none
// does), and two staging tiles when those fit too; 16 rows per workgroup,
// else 8 (multi-channel rows, C >= 2, whose windows are the widest).
int pass_npl_for(int C, int hw, int* stages, int* tr)
{
    const int n0 = (C == 3) ? 12 : 8;
    for (int rows : {kPassRowsHost, 8}) {
        if (rows != kPassRowsHost && C < 2) break;
        for (int npl : {n0, 2 * n0})
            if (hw <= kWave * npl && pass_lds_bytes(npl, hw, 1, rows) <= kLdsLimit) {
                *stages = pass_lds_bytes(npl, hw, 2, rows) <= kLdsLimit ? 2 : 1;
                *tr = rows;
                return npl;
            }
    }
    return 0;
}

// Wide boxes favour the two-pass path: the fused kernel's column ring needs
// (2R + 2) x 256 bytes of LDS per wave and each segment re-reads 2R + 1 rows.
constexpr int kTwoPassMinRC = 40;

void load_tune_table()
{
    const char* path = std::getenv("RSG_TUNE_TABLE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t h = line.find('#');
        if (h != std::string::npos) line.resize(h);
        std::istringstream is(line);
        TuneEntry e;
        if (is >> e.dtype >> e.C >> e.rlo >> e.rhi >> e.nlo >> e.nhi >> e.hs && (e.hs > 0 || e.hs == -1)) {
            if (!(is >> e.nc) || e.nc < 0) e.nc = 0;
            if (!(is >> e.lo) || e.lo < 0 || e.lo >= kLayouts) e.lo = 0;
            if (!(is >> e.st) || e.st < 0 || e.st > 2) e.st = 0;
            g_tune.push_back(e);
        }
    }
}

bool tuned_hs(int dtype, int C, int R, int64_t n, int* hs, int* nc, int* lo, int* st)
{
    const int ov = g_hs_override.load(std::memory_order_relaxed);
    if (ov > 0) { *hs = ov; return true; }
    std::call_once(g_tune_once, load_tune_table);
    for (const auto& e : g_tune)
        if (e.dtype == dtype && e.C == C && R >= e.rlo && R <= e.rhi && n >= e.nlo && n <= e.nhi) {
            *hs = e.hs;
            *nc = e.nc;
            *lo = e.lo;
            *st = e.st;
            return true;
        }
    return false;
}

// Built-in segment height: minimise (rounds of resident waves) x (rows each
// wave streams), i.e. ceil(tasks / resident) * (hs + 2R + 1).
int default_hs(int H, int nstrips, int R, uint32_t lds)
{
    const int per_cu = std::max(1, std::min(8, int(kLdsLimit / std::max(lds, 1u))));
    const int64_t resident = int64_t(256) * per_cu;
    int best = 32;
    int64_t best_cost = -1;
    for (int hs : {32, 64, 128, 256, 512, 1024, 2048}) {
        const int h = std::min(hs, H);
        const int64_t tasks = int64_t(nstrips) * ((H + h - 1) / h);
        const int64_t rounds = (tasks + resident - 1) / resident;
        const int64_t cost = rounds * ((h + 2 * R + 1 + kCoStep - 1) / kCoStep * kCoStep);
        if (best_cost < 0 || cost <= best_cost) { best_cost = cost; best = h; }
        if (hs >= H) break;
    }
    return best;
}

}  // namespace

int check_boxes(const rsg_boxes& b, bool need_u8)
{
    if (b.K < 1 || b.K > RSG_MAX_K) return set_error(RSG_EINVAL, "boxes: K must be in 1..5 (got %d)", b.K);
    int64_t rmax = 0;
    for (int k = 0; k < b.K; ++k) {
        if (b.r[k] < 0 || b.r[k] > (1 << 26)) return set_error(RSG_EINVAL, "boxes: half-width %d out of range", b.r[k]);
        if (!std::isfinite(b.w32[k])) return set_error(RSG_EINVAL, "boxes: weight %d is not finite", k);
        rmax = std::max<int64_t>(rmax, b.r[k]);
    }
    if (need_u8) {
        if (!b.u8_ok) return set_error(RSG_EUNSUPPORTED, "boxes: no integer weights for uint8");
        int64_t G = 0;
        for (int k = 0; k < b.K; ++k) G += int64_t(b.m[k]) * (2 * int64_t(b.r[k]) + 1);
        if (G <= 0 || uint64_t(G) != b.G || G >= (int64_t(1) << 24) ||
            int64_t(255) * G * (2 * rmax + 1) >= (int64_t(1) << 32))
            return set_error(RSG_EINVAL, "boxes: inconsistent or oversized integer weights");
    }
    return RSG_OK;
}

void set_hs_override(int hs) { g_hs_override.store(hs > 0 ? hs : 0, std::memory_order_relaxed); }
void set_path_override(int path) { g_path_override.store(path, std::memory_order_relaxed); }
void set_nc_override(int nc) { g_nc_override.store(nc > 0 ? nc : 0, std::memory_order_relaxed); }
void set_layout_override(int lo) { g_lo_override.store(lo > 0 ? lo : 0, std::memory_order_relaxed); }
void set_stores_override(int st) { g_st_override.store(st > 0 ? st : 0, std::memory_order_relaxed); }

int plan_image(const rsg_image_desc& d, ImgParams* ip, int step, int hs_pref, bool planar_ok)
{
    if (step < 1) return set_error(RSG_EINVAL, "output step must be >= 1 (got %d)", step);
    if (!d.src || !d.dst) return set_error(RSG_EINVAL, "NULL image pointer");
    if (d.H < 1 || d.W < 1) return set_error(RSG_EINVAL, "H and W must be >= 1 (got %d x %d)", d.H, d.W);
    if (d.C < 1 || d.C > 4) return set_error(RSG_EINVAL, "C must be in 1..4 (got %d)", d.C);
    if (d.dt < RSG_U8 || d.dt > RSG_BF16) return set_error(RSG_EINVAL, "bad dtype %d", int(d.dt));
    if (d.b != RSG_REPLICATE && d.b != RSG_ZERO && d.b != RSG_REFLECT)
        return set_error(RSG_EINVAL, "bad boundary %d", int(d.b));
    const int64_t WC = int64_t(d.W) * d.C;
    if (WC > (int64_t(1) << 30) || d.H > (1 << 30)) return set_error(RSG_EUNSUPPORTED, "image too large");
    // the output: every step-th row and pixel, (Ho x Wo x C)
    const int64_t Ho = (d.H + step - 1) / step;
    const int64_t WoC = int64_t((d.W + step - 1) / step) * d.C;
    const int64_t ss = d.src_stride ? d.src_stride : WC;
    const int64_t ds = d.dst_stride ? d.dst_stride : WoC;
    if (ss < WC || ds < WoC) return set_error(RSG_EINVAL, "row stride smaller than the row");
    const int es = dtype_size(d.dt);
    {   // source and destination must not overlap
        const char* s0 = static_cast<const char*>(d.src);
        const char* s1 = s0 + (int64_t(d.H - 1) * ss + WC) * es;
        const char* t0 = static_cast<const char*>(d.dst);
        const char* t1 = t0 + ((Ho - 1) * ds + WoC) * es;
        if (s0 < t1 && t0 < s1) return set_error(RSG_EINVAL, "source and destination overlap");
    }

    rsg_boxes b;
    if (d.boxes) {
        int rc = check_boxes(*d.boxes, d.dt == RSG_U8);
        if (rc != RSG_OK) return rc;
        b = *d.boxes;
    } else {
        int rc = make_boxes(d.sigma, d.K, RSG_FIT_SCALED, &b);
        if (rc != RSG_OK) return rc;
    }
    if (d.dt == RSG_U8 && !b.u8_ok)
        return set_error(RSG_EUNSUPPORTED, "no integer weight scale for uint8 at sigma=%g K=%d", d.sigma, d.K);

    ImgParams p;
    std::memset(&p, 0, sizeof(p));
    p.src = d.src;
    p.dst = d.dst;
    p.src_stride = ss;
    p.dst_stride = ds;
    p.H = d.H;
    p.W = d.W;
    p.C = d.C;
    p.K = d.K;
    p.dtype = d.dt;
    p.boundary = d.b;
    int R = 0;
    for (int k = 0; k < d.K; ++k) {
        p.r[k] = b.r[k];
        p.wf[k] = b.w32[k];
        p.m[k] = b.m[k];
        R = std::max(R, int(b.r[k]));
    }
    p.R = R;
    if (d.dt == RSG_U8) {
        p.G2 = b.G * b.G;
        p.G2half = p.G2 / 2;
        // the estimate divides N >> qsh (< 2^32) by G^2 / 2^qsh
        int qsh = 0;
        while ((p.G2 << 8) > (uint64_t(1) << (32 + qsh))) ++qsh;
        p.qsh = qsh;
        p.invG2 = float(std::ldexp(1.0, qsh) / double(p.G2));
    }

    // taps: K < 3 is padded with zero-weight boxes of half-width 0
    p.kt = std::max(3, d.K);
    for (int k = d.K; k < p.kt; ++k) { p.r[k] = 0; p.wf[k] = 0.0f; p.m[k] = 0; }
    {
        double dc = 0.0;
        for (int k = 0; k < p.kt; ++k) dc += double(p.wf[k]) * (2.0 * p.r[k] + 1.0);
        p.dc32 = float(dc);
    }

    // ---- path: fused kernel, or two passes for wide boxes ----
    const int C = d.C;
    p.pnpl[0] = pass_npl_for(C, (2 * R + 1) * C, &p.pst[0], &p.ptr[0]);
    p.pnpl[1] = pass_npl_for(1, 2 * R + 1, &p.pst[1], &p.ptr[1]);
    const bool two_ok = p.pnpl[0] > 0 && p.pnpl[1] > 0;
    if (two_ok) {
        p.plds[0] = pass_lds_bytes(p.pnpl[0], (2 * R + 1) * C, p.pst[0], p.ptr[0]);
        p.plds[1] = pass_lds_bytes(p.pnpl[1], 2 * R + 1, p.pst[1], p.ptr[1]);
    }
    const int ov = g_path_override.load(std::memory_order_relaxed);
    int hs_t = 0, nc_t = 0, lo_t = 0, st_t = 0;
    const bool tabled = tuned_hs(d.dt, C, R, (WC + kWave - 1) / kWave * d.H, &hs_t, &nc_t, &lo_t, &st_t);
    const int lo_ov = g_lo_override.load(std::memory_order_relaxed);
    const int lo_first = lo_ov > 0 ? lo_ov : lo_t;      // first row-scan layout tried
    bool two = two_ok && (tabled ? hs_t < 0 : R * C >= kTwoPassMinRC);
    if (ov == 1 || ov == 3) two = false;
    // strided output: the fused two-wave form (which stores every step-th row
    // and pixel) when the fused path is chosen, else the two-pass path
    if (ov == 2 || (step > 1 && ov == 3)) {
        if (!two_ok) return set_error(RSG_EUNSUPPORTED, "two-pass path: box half-width %d too wide for C=%d", R, C);
        two = true;
    }

    // ---- row-scan layout: first (lanes per row, samples per lane) whose
    //      segment covers the row span [s0 - (R+1)C, s_last + RC] of a
    //      task's columns s0 .. s_last: 64 nc consecutive samples, or with a
    //      strided output the input samples of 64 consecutive kept samples.
    //      The cooperative form takes nc = wide_nc(C) columns per lane where
    //      the span and the LDS allow, else one. ----
    // single launches, batches and served images run the cooperative form
    // (kCoWaves waves per task); path override 3 selects the one-wave form
    const int co = (ov == 3) ? 0 : 1;
    int seg = 0, npl = 0, align = 1, nc = 1;
    // columns per lane: the override, else the table, else one.  3 asks for
    // channel-planar tasks: each task filters one channel of a multi-channel
    // image (the kernel of one channel, pixels C samples apart), so its row
    // span is 64 + 2R + 1 pixels of that channel instead of 64 + (2R + 1)C
    // interleaved samples for 64 / C pixels
    const int nc_ov = g_nc_override.load(std::memory_order_relaxed);
    const int nc_want = nc_ov > 0 ? nc_ov : (nc_t > 0 ? nc_t : 1);
    const bool planar_possible = co && step == 1 && C >= 2 && planar_ok;
    bool planar = planar_possible && nc_want == 3;
    const int CK = planar ? 1 : C;                       // channels of the kernel
    const int nc_first = (co && step == 1 && nc_want == 2) ? wide_nc(C) : 1;
    for (int nci = nc_first; nci >= 1 && !seg; nci = (nci > 1) ? 1 : 0) {
        int64_t cols = int64_t(kWave) * nci;            // samples (pixels when planar)
        if (step > 1) {
            int64_t np = 0;                          // pixels a strip of 64 kept samples spans
            for (int k = 0; k < C; ++k) np = std::max<int64_t>(np, ((kWave * k) % C + kWave - 1) / C + 1);
            cols = ((np - 1) * step + 1) * C;
        }
        for (int i = lo_first; i < kLayouts && !seg; ++i) {
            int sg, n;
            scan_layout(CK, i, &sg, &n);
            const int cb = n * es;                   // chunk bytes
            const int unit = gcd_i(cb, 16);          // vector load granule
            const int al = lcm_i(CK, std::max(1, unit / es));
            const int64_t span = cols + int64_t(2 * R + 1) * CK + al - 1;
            if (span > int64_t(sg) * n) continue;
            if (nci > 1 && tile_lds_bytes_co(sg, n, co_ring_rows(R, nci), nci) + 4u * kBatchSlotWords > kLdsLimit) break;
            seg = sg; npl = n; align = al; nc = nci;
        }
    }
    if (!seg && !two && !planar && planar_possible && !(two_ok && ov != 1 && ov != 3)) {
        // neither an interleaved span nor the two-pass window holds the
        // boxes: one channel per task needs only 64 + 2R + 1 pixels
        for (int i = lo_first; i < kLayouts && !seg; ++i) {
            int sg, n;
            scan_layout(1, i, &sg, &n);
            const int al = std::max(1, gcd_i(n * es, 16) / es);
            if (int64_t(kWave) + int64_t(2 * R + 1) + al - 1 > int64_t(sg) * n) continue;
            seg = sg; npl = n; align = al; nc = 1;
            planar = true;
        }
    }
    if (!seg && !two) {
        if (two_ok && ov != 1 && ov != 3) {
            two = true;
        } else {
            int sg, n;
            scan_layout(C, kLayouts - 1, &sg, &n);
            return set_error(RSG_EUNSUPPORTED, "box half-width %d too wide for C=%d (largest row span %d samples)",
                             R, C, sg * n);
        }
    }
    auto finish_two_pass = [&]() {
        p.path = kPathTwoPass;
        p.nstrips = int((WC + kWave - 1) / kWave);
        p.hs = d.H;
        p.nsegs = 1;
        p.step = step;
        p.ntasks = (d.H + p.ptr[0] - 1) / p.ptr[0] + int((WoC + p.ptr[1] - 1) / p.ptr[1]);
        p.lds_bytes = std::max(p.plds[0], p.plds[1]);
        *ip = p;
        return RSG_OK;
    };
    if (two) return finish_two_pass();
    p.seg = seg;
    p.npl = npl;
    p.align = align;
    {   // (channel-planar tasks read their channel element by element)
        const int unit = gcd_i(npl * es, 16);
        const uintptr_t sa = reinterpret_cast<uintptr_t>(d.src);
        p.vec = !planar && (sa % unit == 0) && ((ss * es) % unit == 0);
    }
    p.pstride = planar ? C : 1;
    p.G = kWave / seg;
    p.L = (2 * R + 1 + p.G + p.G - 1) / p.G * p.G;
    p.Lco = co_ring_rows(R, nc);
    p.co = co;
    p.nc = nc;
    {   // vector stores of a lane's columns: 2-byte and 1-byte elements need
        // the destination rows aligned to the group (4-byte ones: to the element)
        const int gb = nc * es;
        const uintptr_t da = reinterpret_cast<uintptr_t>(d.dst);
        p.ovec = (es == 4) || (nc > 1 && (gb & (gb - 1)) == 0 && da % gb == 0 && (ds * es) % gb == 0);
    }
    {   // output stores of FP32 cooperative one-column tasks: the override,
        // else the table, else staged where the kernel has four or five taps
        const int st_ov = g_st_override.load(std::memory_order_relaxed);
        const int st_want = st_ov > 0 ? st_ov : st_t;
        p.staged = (es == 4 && co && nc == 1 && !planar && step == 1) ? int(st_want == 2 || (st_want == 0 && p.kt >= 4)) : 0;
    }
    p.lds_one = tile_lds_bytes(seg, npl, p.L);
    p.lds_bytes = p.co ? tile_lds_bytes_co(seg, npl, p.Lco, p.nc) : p.lds_one;
    {   // the batch kernel of the cooperative form adds its task slot
        const uint32_t need = std::max(p.lds_bytes + (p.co ? 4u * kBatchSlotWords : 0u), p.lds_one);
        if (need > kLdsLimit)
            return set_error(RSG_EUNSUPPORTED, "tile needs %u bytes of LDS (limit %u)", need, kLdsLimit);
    }
    // a strip is 64 nc output samples (strided: 64 kept samples; planar: 64
    // pixels of one channel, the channels a stack of C slices one sample apart)
    p.nstrips = int((WoC / (planar ? C : 1) + int64_t(kWave) * nc - 1) / (int64_t(kWave) * nc));
    if (planar) {
        p.nslices = C;
        p.slice_stride = 1;
    }

    // ---- segment height ----
    int hs = hs_pref > 0 ? hs_pref
                         : ((tabled && hs_t > 0) ? hs_t : default_hs(d.H, p.nstrips * std::max(1, p.nslices), R, p.lds_bytes));
    hs = std::max(1, std::min(hs, d.H));
    {   // every offset a task touches (rows ybase .. ybase + its padded
        // iteration count, times the larger stride) must stay below 2^30
        const int64_t stride_b = std::max(ss, ds) * es;
        auto fits = [&](int h) {
            // (the cooperative form pads to whole steps of kCoStep rows and
            // prefetches into the next step; the one-wave form starts up to
            // G - 1 rows early and prefetches kPrefetch groups ahead)
            const int64_t rows = int64_t(h) + 2 * R + 1 + std::max(2 * kCoStep, (p.G - 1) + (2 * kPrefetch + 1) * p.G);
            return rows * stride_b + WC * es <= kOffsetLimit;
        };
        while (hs > 1 && !fits(hs)) hs = (hs + 1) / 2;
        if (!fits(hs)) {
            if (two_ok && ov != 1 && ov != 3) return finish_two_pass();     // it addresses every row on its own
            return set_error(RSG_EUNSUPPORTED, "row stride too large for a tile (%lld bytes, box half-width %d)",
                             (long long)stride_b, R);
        }
    }
    p.step = step;
    p.hs = hs;
    p.nsegs = (d.H + hs - 1) / hs;
    const int64_t nt = int64_t(p.nstrips) * p.nsegs * std::max(1, p.nslices);
    if (nt > (int64_t(1) << 30)) return set_error(RSG_EUNSUPPORTED, "too many tasks");
    p.ntasks = int(nt);
    *ip = p;
    return RSG_OK;
}

}  // namespace rsg
