// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "rsg.h"

#include <vector>

namespace rsg {

// Records the message for rsg_last_error() on this thread; returns `code`.
int set_error(int code, const char* fmt, ...);

// Section 4.2 sigma0 fit (cached per K) and per-sigma boxes.
int sigma0_fit(int K, bool quadratic_form, int* p, double* c, double* err);
int make_boxes(double sigma, int K, int method, rsg_boxes* out);   // method: rsg_fit_method
int check_boxes(const rsg_boxes& b, bool need_u8);                 // caller-supplied boxes
extern const double kSigma0Value;

constexpr int kWave = 64;          // CDNA wavefront width; also the strip width in samples
constexpr int kXcds = 8;           // MI355X: 8 accelerator complex dies
#ifndef RSG_PREFETCH
#define RSG_PREFETCH 2
#endif
constexpr int kPrefetch = RSG_PREFETCH;   // groups of row loads in flight per wave
constexpr int kCoWaves = 4;        // waves per task of the cooperative fused form
constexpr int kCoRows = 8;         // rows per wave per step of the cooperative form
constexpr int kCoStep = kCoWaves * kCoRows;   // rows per step
// The wide column form takes 4-row blocks: its ring, nc times as wide, is
// then shorter (measured 5-10 % faster than 8-row blocks at every sigma).
constexpr int co_rows(int nc) { return nc > 1 ? 4 : kCoRows; }
// Ring rows of the cooperative form: the step's rows and the 2R + 1 rows
// behind them, rounded to whole blocks (plus one block of mirror rows)
constexpr int co_ring_rows(int R, int nc) { return (kCoWaves * co_rows(nc) + 2 * R + 1 + co_rows(nc) - 1) / co_rows(nc) * co_rows(nc); }
// Columns per lane of the cooperative form on unstrided outputs: a task is
// 64 pixels wide for C = 3 (a lane owns one pixel's channels) and 128
// samples wide for C = 1, which shortens the row span per output sample and
// lets one vector access carry a lane's columns.
constexpr int wide_nc(int C) { return C == 1 ? 2 : (C == 3 ? 3 : 1); }
constexpr int64_t kOffsetLimit = int64_t(1) << 30;   // every byte offset a task touches stays below this

// Everything one image's kernel needs; plain data, copied to the device for
// batched launches and passed by value for single-image launches.
struct ImgParams {
    const void* src;
    void* dst;
    int64_t src_stride;            // elements per row
    int64_t dst_stride;
    int32_t H, W, C, K;
    int32_t dtype;                 // rsg_dtype
    int32_t boundary;              // rsg_boundary (REPLICATE or ZERO)
    int32_t kt;                    // taps in the kernel: max(K, 3) (extra taps carry weight 0)
    int32_t r[RSG_MAX_K];
    float wf[RSG_MAX_K];           // FP32 slice weights
    uint32_t m[RSG_MAX_K];         // uint8 integer weights
    float dc32;                    // sum_k wf_k (2 r_k + 1): DC gain of the FP32 boxes
    uint64_t G2;                   // G^2 (uint8 rounding denominator)
    uint64_t G2half;               // floor(G^2 / 2)
    float invG2;                   // 2^qsh / G^2 rounded to FP32 (quotient estimate)
    int32_t qsh;                   // shift that brings 256 G^2 below 2^32
    int32_t R;                     // max r
    // tile plan
    int32_t seg;                   // lanes per row in the row scan (16, 32, 64)
    int32_t npl;                   // samples per lane in the row scan
    int32_t G;                     // input rows per group = 64 / seg
    int32_t hs;                    // output rows per task
    int32_t L;                     // one-wave form: column ring length roundup(2R + 1 + G, G) (+ G mirror rows)
    int32_t Lco;                   // cooperative form: co_ring_rows(R, nc) (+ co_rows(nc) mirror rows)
    int32_t align;                 // span start alignment (samples)
    int32_t vec;                   // 1: rows allow vector loads of one chunk
    int32_t nstrips, nsegs, ntasks;
    int32_t variant;               // kernel instantiation
    uint32_t lds_bytes;            // dynamic LDS per workgroup of a single launch
    uint32_t lds_one;              // dynamic LDS of the one-wave fused form (batches, serving)
    // two-pass path (wide boxes): row filter + transposed store, twice
    int32_t path;                  // kPathFused or kPathTwoPass
    int32_t step;                  // output stride in pixels along both axes (1: every pixel; two-pass only)
    int32_t nslices;               // fused path: a stack of this many equal images (<= 1: one image)
    int64_t slice_stride;          // elements from one image of the stack to the next (source and destination)
    int32_t pstride;               // samples from one pixel to the next in a task (> 1: channel-planar tasks)
    int32_t co;                    // fused path: 1 = cooperative workgroups of kCoWaves waves, 0 = one wave
    int32_t nc;                    // cooperative form: consecutive columns per lane (1, or wide_nc(C))
    int32_t ovec;                  // the destination allows one vector store per lane's columns
    int32_t staged;                // FP32, one column per lane: interior tasks with 16-byte aligned
                                   // output rows stage each wave's results in LDS for 16-byte stores
    int32_t pnpl[2];               // samples per lane of pass A, pass B
    int32_t pst[2];                // staging tiles of pass A, pass B (1 or 2)
    uint32_t plds[2];              // LDS bytes per workgroup of pass A, pass B
    int32_t ptr[2];                // rows (waves) per workgroup of pass A, pass B (16, or 8 for wide windows)
};

constexpr int kPathFused = 0;
constexpr int kPathTwoPass = 1;

// One pass of the two-pass path: filter `rows` rows of `len` samples (taps C
// samples apart) and store the result transposed (element (x, row) at
// dst[x * dst_stride + row]).
// The pass along z of an FP32 volume (D slices of `plane` samples).
struct ZParams {
    const float* src;
    float* dst;
    int64_t plane;                 // samples per slice (H W C)
    int32_t D, R;
    int32_t hz;                    // output slices per task
    int32_t ncols;                 // 64-sample columns per slice
    int32_t ntasks;                // ncols x segments
    int32_t L;                     // ring length 2R + 2
    int32_t boundary;
    int32_t r[RSG_MAX_K];
    float wf[RSG_MAX_K];
    float dc32;
};
// Launches the z pass with `wpb` waves (tasks) per workgroup.
int launch_zpass_f32(const ZParams& zp, int kt, int wpb, hipStream_t stream);

struct PassParams {
    const void* src;
    void* dst;
    int64_t src_stride;            // elements per input row
    int64_t dst_stride;            // elements per output row (= input row count of the next pass)
    int32_t rows, len;
    int32_t R;
    int32_t r[RSG_MAX_K];
    float wf[RSG_MAX_K];
    uint32_t m[RSG_MAX_K];
    float dc32;
    uint64_t G2, G2half;
    float invG2;
    int32_t qsh;
    int32_t boundary;
    int32_t vec;                   // rows allow 16-byte chunk loads
    int32_t win_pitch;             // LDS words per wave window
    int32_t win_shift;             // window start offset (aligns its new part to 16 bytes)
    int32_t ostep;                 // store every ostep-th pixel of a row (1: all), compacted
};

// One unit of work of a batched launch.
struct BatchTask {
    int32_t img;
    int32_t task;                  // task index inside the image
};

// Plan for one image: validates, fits (cached), picks the tile shape.
// step > 1: strided output (two-pass path); hs_pref > 0: segment height of a
// fused plan chosen by the caller (volumes), instead of the table or rule
int plan_image(const rsg_image_desc& d, ImgParams* ip, int step = 1, int hs_pref = 0, bool planar_ok = true);
// Process-wide segment height that overrides the tuning table (0: none).
void set_hs_override(int hs);
// Process-wide path override (0: planner's choice, 1: fused, 2: two-pass).
void set_path_override(int path);
// Process-wide columns-per-lane override of the cooperative form (0: none,
// 1: one, 2: wide_nc(C), 3: channel-planar tasks for C >= 2).
void set_nc_override(int nc);
// Process-wide first row-scan layout the planner tries (0: the first that fits).
void set_layout_override(int lo);
// Process-wide output store form (0: the table, else the built-in rule;
// 1: one store per lane and row; 2: staged 16-byte stores).
void set_stores_override(int st);

// Launchers (rsg_kernels.hip).
int launch_single(const ImgParams& ip, hipStream_t stream);
int launch_single_u8(const ImgParams& ip, hipStream_t stream);
int launch_single_f32(const ImgParams& ip, hipStream_t stream);
int launch_single_f16(const ImgParams& ip, hipStream_t stream);
int launch_single_bf16(const ImgParams& ip, hipStream_t stream);
// Two-pass path: pass A (image -> intermediate) or pass B (intermediate -> image).
int launch_pass(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t stream);
int launch_pass_u8(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t stream);
int launch_pass_f32(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t stream);
int launch_pass_f16(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t stream);
int launch_pass_bf16(const ImgParams& ip, int pass, const PassParams& pp, hipStream_t stream);
// One launch of one pass over the two-pass images of a batch that share a
// kernel instantiation: workgroup b takes (pass parameters, row block) =
// d_tasks[b].
struct PassBatchLaunch {
    int dtype, pass, C, npl, kt, stages, tr;
    uint32_t lds;
    const PassParams* d_pps;
    const int2* d_tasks;
    int ntasks;
};
int launch_pass_batch(const PassBatchLaunch& b, hipStream_t stream);
int launch_pass_batch_u8(const PassBatchLaunch& b, hipStream_t stream);
int launch_pass_batch_f32(const PassBatchLaunch& b, hipStream_t stream);
int launch_pass_batch_f16(const PassBatchLaunch& b, hipStream_t stream);
int launch_pass_batch_bf16(const PassBatchLaunch& b, hipStream_t stream);
// Row blocks of the two-pass images of a batch (both passes).
int64_t pass_blocks(const ImgParams* imgs, int nimg);
// Plans every image and builds the flat work list of a batched launch.
int plan_batch(const rsg_image_desc* d, int n, std::vector<ImgParams>& imgs, std::vector<BatchTask>& tasks,
               int hs_pref = 0);
// Window geometry of one pass (shared by the planner and the launcher).
constexpr int kPassRowsHost = 16;
inline int pass_win_pitch(int npl, int hw) { return (kWave * npl + hw + 3 + 3) / 4 * 4; }
// tr: rows (waves) per workgroup; stages: staging tiles (2 lets the stores
// of chunk k overlap chunk k + 1)
inline uint32_t pass_lds_bytes(int npl, int hw, int stages, int tr = kPassRowsHost)
{
    return uint32_t(4 * (tr * pass_win_pitch(npl, hw) + stages * kWave * npl * (tr + 1)));
}
// One persistent launch over the tasks of one (dtype, C, kt) class.
struct BatchClassLaunch {
    int dtype, C, kt;
    int co;                        // 1: cooperative workgroups (LDS includes the task slot)
    int nc;                        // cooperative form: columns per lane
    int grid;
    uint32_t lds;
    const ImgParams* d_imgs;
    const BatchTask* d_tasks;
    int ntasks;
    unsigned* d_counter;
};
int launch_batch_class(const BatchClassLaunch& b, hipStream_t stream);
int launch_batch_class_u8(const BatchClassLaunch& b, hipStream_t stream);
int launch_batch_class_f32(const BatchClassLaunch& b, hipStream_t stream);
int launch_batch_class_f16(const BatchClassLaunch& b, hipStream_t stream);
int launch_batch_class_bf16(const BatchClassLaunch& b, hipStream_t stream);
// Row-scan layouts (lanes per row, samples per lane) instantiated per
// channel count, in the order the planner tries them.
constexpr int kLayouts = 4;
inline void scan_layout(int C, int i, int* seg, int* npl)
{
    static const int segs[kLayouts] = {16, 32, 64, 64};
    static const int n1[kLayouts] = {8, 8, 8, 16};      // C = 1, 2, 4
    static const int n3[kLayouts] = {12, 12, 12, 24};   // C = 3
    *seg = segs[i];
    *npl = (C == 3) ? n3[i] : n1[i];
}
// LDS row pitch (in 32-bit words) of the row-sum tiles.  The compiler pairs
// reads of one lane from consecutive tile rows into one ds_read2; a pitch of
// 32 (mod 64) words puts the pair in opposite halves of the 64 banks.  The
// column ring keeps the dense 64-word pitch (one word per lane).
constexpr int row_tile_pitch(int seg, int npl) { return seg * npl + 32; }
// Cooperative form: one row tile per wave, one block total per wave and
// column, and the ring of Lco + kCoRows rows (64 nc columns).
inline uint32_t tile_lds_bytes_co(int seg, int npl, int Lco, int nc)
{
    const int G = kWave / seg;
    return uint32_t(4 * (kCoWaves * G * row_tile_pitch(seg, npl) + (kCoWaves + Lco + co_rows(nc)) * kWave * nc));
}
// Two row tiles (double-buffered) and the ring of L + G rows.
inline uint32_t tile_lds_bytes(int seg, int npl, int L)
{
    const int G = kWave / seg;
    return uint32_t(4 * (2 * G * row_tile_pitch(seg, npl) + (L + G) * kWave));
}
// The two-wave batch kernel passes each popped task index through the first
// 16 bytes of LDS (which keeps the tiles 16-byte aligned).
constexpr int kBatchSlotWords = 4;

// Workspace of a batched launch: a header (class counters, ImgParams, task
// entries, PassParams), copied from the host at launch, then the
// intermediates of the batch's two-pass images, carved from the same
// caller-provided buffer.  ntasks: tasks of the fused images plus row blocks
// of the two-pass images.
size_t batch_header_bytes(int nimg, int64_t ntasks);
size_t batch_mid_bytes(const ImgParams* imgs, int nimg);
size_t batch_workspace_bytes(const ImgParams* imgs, int nimg, int64_t ntasks);
// h_stage: optional pinned host buffer of >= batch_header_bytes() used to
// stage the header (must not be reused before the copy has executed); NULL
// stages through pageable memory.  Allocates no device memory.
int launch_batch(const ImgParams* h_imgs, int nimg, const BatchTask* h_tasks, int ntasks,
                 void* d_ws, size_t ws_bytes, hipStream_t stream, void* h_stage = nullptr);
// Two-pass path of one image with its intermediate (>= mid_bytes(ip)) given.
size_t mid_bytes(const ImgParams& ip);
int launch_two_pass_into(const ImgParams& ip, void* mid, hipStream_t stream);

// Sizes of the element types.
inline int dtype_size(int dt) { return dt == RSG_U8 ? 1 : (dt == RSG_F32 ? 4 : 2); }

}  // namespace rsg
