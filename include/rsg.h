/*
 * rsg.h -- C ABI of the running-sum Gaussian filter for AMD Instinct MI355X
 * (gfx950).
 *
 * The method is Elboher & Werman, "Efficient and Accurate Gaussian Image
 * Filtering Using Running Sums" (arXiv 1107.4958):
 *   - a symmetric 1D kernel is a sum of K nested, centred boxes ("weighted
 *     slices", Section 3.2, Eq. S_i and Eq. ciwi);
 *   - a 1D pass builds the running sum I of the signal (Section 3.3,
 *     Eq. alg1) and outputs sum_k w_k (I(x + r_k) - I(x - r_k - 1)) at every
 *     sample (Eq. indep);
 *   - a 2D image is filtered along rows, then along the columns of the
 *     intermediate result (Section 3.4);
 *   - box half-widths and weights come from an exhaustive fit at
 *     sigma0 = 100/pi under the quadratic-form error of Section 4.1
 *     (Eq. mahal, autocorrelation of a 1/f spectrum), rescaled to the
 *     requested sigma by Eq. scale1 / scale2 (Section 4.2); other fit methods
 *     (l2 error, a direct fit at sigma) and caller-supplied boxes are offered
 *     too;
 *   - beyond 2D images: strided (downsampling) output and FP32 volumes (one
 *     more 1D pass along z).
 *
 * Conventions for every entry point:
 *   - functions never throw; they return RSG_OK (0) or a negative rsg_status;
 *     rsg_last_error() gives a message for the last failure on the calling
 *     thread;
 *   - images are interleaved H x W x C (C in 1..4), row stride in ELEMENTS
 *     (>= W*C), element type given by rsg_dtype; output dtype = input dtype;
 *   - device pointers are HIP device addresses owned by the caller; they must
 *     stay valid until the work on the given stream (or the server ticket) is
 *     complete; source and destination must not overlap;
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream);
 *     device work is asynchronous on it: launch errors are returned, faults
 *     surface at the caller's next synchronisation.
 */
#ifndef RSG_H
#define RSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSG_OK = 0,
    RSG_EINVAL = -1,        /* bad argument */
    RSG_ENOMEM = -2,        /* host allocation failed, or request exceeds a budget */
    RSG_EBUSY = -3,         /* queue full; try again later */
    RSG_ENOTFOUND = -4,     /* unknown ticket */
    RSG_EDEVICE = -5,       /* HIP runtime error */
    RSG_EUNSUPPORTED = -6   /* valid but not supported (e.g. K > 5) */
} rsg_status;

typedef enum { RSG_U8 = 0, RSG_F32 = 1, RSG_F16 = 2, RSG_BF16 = 3 } rsg_dtype;

/* Boundary extension of each axis (the paper names none).  REPLICATE clamps
 * indices to the image; ZERO treats samples outside as 0; REFLECT is the
 * half-sample symmetric extension (... c b a | a b c d | d c b ...), repeated
 * with period 2n, so boxes wider than the image are defined in every mode. */
typedef enum { RSG_REPLICATE = 0, RSG_ZERO = 1, RSG_REFLECT = 2 } rsg_boundary;

#define RSG_MAX_K 5

/* Box parameters for one (sigma, K).
 *   p, c      the sigma0 fit: inclusive half-widths 0 <= p_1 < ... < p_K <= 99
 *             of the K segments and their least-squares constants
 *             (Section 4.2, Table 2), fit_err its quadratic-form error;
 *   r         half-widths at sigma: r_k = floor(sigma * p_k / sigma0 + 1e-9)
 *             (Eq. scale1);
 *   w         slice weights w_k = (c_k - c_{k+1}) p_k / (2 r_k + 1)
 *             (Eq. scale2, c_{K+1} = 0), normalised so that
 *             sum_k w_k (2 r_k + 1) = 1; w32 = (float)w;
 *   m, G, s   integer weights of the exact uint8 path: m_k = rint(w_k 2^s),
 *             G = sum_k m_k (2 r_k + 1), with s the largest integer in
 *             [1, 23] such that G < 2^24 and 255 G (2 r_K + 1) < 2^32;
 *             u8_ok = 0 when no s qualifies (uint8 filtering then fails). */
typedef struct {
    int32_t K;
    int32_t p[RSG_MAX_K];
    double c[RSG_MAX_K];
    double fit_err;
    double sigma;
    int32_t r[RSG_MAX_K];
    double w[RSG_MAX_K];
    float w32[RSG_MAX_K];
    uint32_t m[RSG_MAX_K];
    uint64_t G;
    int32_t s;
    int32_t u8_ok;
} rsg_boxes;

/* Fit and rescale the boxes for (sigma, K) on the host, in FP64 (the
 * kernels compute in FP32 and in integers; FP64 is host-only).  The sigma0 search is exhaustive over all
 * C(100, K) partitions and is cached per K for the life of the process
 * (thread-safe).  sigma must be finite and > 0; K in 1..5.  This is the fit
 * every entry point uses unless the caller passes boxes of its own.
 * Errors: RSG_EINVAL (sigma, K, out == NULL), RSG_EUNSUPPORTED (K > 5). */
int rsg_fit_boxes(double sigma, int K, rsg_boxes* out);

/* Fit methods:
 *   RSG_FIT_SCALED     the paper's: the quadratic-form fit at sigma0 rescaled
 *                      to sigma (Section 4.2), as rsg_fit_boxes;
 *   RSG_FIT_SCALED_L2  the same with the l2 error (A = I), the error measure
 *                      the paper compares its quadratic form against;
 *   RSG_FIT_DIRECT     the Section 4 search run at sigma itself: the Gaussian
 *                      of s.d. sigma on M = max(ceil(pi sigma), K) half
 *                      samples, Phi on period 2M, r = p (the partition), w
 *                      the slices c_k - c_{k+1} normalised to unit DC gain
 *                      (p, c, fit_err describe this fit).  For sigma <=
 *                      100/pi, where rescaling floors half-widths together;
 *                      cached per (K, sigma), bounded. */
typedef enum { RSG_FIT_SCALED = 0, RSG_FIT_SCALED_L2 = 1, RSG_FIT_DIRECT = 2 } rsg_fit_method;

/* Boxes for (sigma, K) by one of the fit methods above.
 * Errors: as rsg_fit_boxes; RSG_EINVAL (bad method); RSG_EUNSUPPORTED
 * (RSG_FIT_DIRECT with sigma > 100/pi). */
int rsg_fit_boxes_ex(double sigma, int K, rsg_fit_method method, rsg_boxes* out);

/* Filter one image: rows by the K boxes, then columns (Sections 3.3-3.4), on
 * `stream`: one fused kernel launch, or for wide boxes two launches of a row
 * filter with a transposed store and an intermediate of H*W*C four-byte
 * words.  That intermediate is the one device allocation of this entry point
 * (and of rsg_box_filter and rsg_gauss_filter_strided): it is taken and
 * released in stream order (hipMallocAsync / hipFreeAsync on `stream`),
 * since the call has no workspace argument; rsg_filter_batch takes it from
 * the caller's workspace and rsg_gauss_filter_noalloc from a fixed scratch
 * array instead.  uint8 is computed in exact integers (uint32 running sums,
 * a uint64 column combine, one integer rounding at the end: round half up
 * of U / G^2);
 * FP32 / FP16 / BF16 load as FP32 and accumulate in FP32; FP16 / BF16
 * results are rounded to nearest even.  Row stride = W*C elements.
 * Errors: RSG_EINVAL (NULL pointers, H or W < 1, C not in 1..4, bad dtype,
 * sigma <= 0 or not finite, K not in 1..5, bad boundary), RSG_EUNSUPPORTED
 * (uint8 with no admissible integer scale, box wider than the kernel limits),
 * RSG_ENOMEM (no device memory for the intermediate), RSG_EDEVICE (launch
 * failure). */
int rsg_gauss_filter(const void* d_src, void* d_dst, int H, int W, int C, rsg_dtype dt,
                     double sigma, int K, rsg_boundary b, void* stream);

/* rsg_gauss_filter for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same plan, kernels and results, but the two-pass path's
 * intermediate lives in a scratch array of 64 MiB that the library holds on
 * each device it runs on until the process ends; the call allocates nothing
 * (no hipMalloc / hipFree / stream-ordered allocation).  The fused path
 * needs no scratch.  Every call on a device shares that device's array,
 * whose contents persist between calls (nothing in it needs to start at
 * zero: the row pass writes every intermediate element before the column
 * pass reads it); calls that overlap in time on one device race on it.
 * Errors: as rsg_gauss_filter; RSG_ENOMEM (the image takes the two-pass
 * path and its intermediate, 4 H W C bytes, exceeds 64 MiB: no launch is
 * made); RSG_EDEVICE (the array's device address cannot be found). */
int rsg_gauss_filter_noalloc(const void* d_src, void* d_dst, int H, int W, int C, rsg_dtype dt,
                             double sigma, int K, rsg_boundary b, void* stream);

/* rsg_gauss_filter with boxes the caller supplies (any fit method, or boxes
 * of its own): K in 1..5, half-widths r_k in [0, 2^26], FP32 weights w32
 * finite; for uint8 the integer form must be present (u8_ok) and consistent:
 * G = sum m_k (2 r_k + 1) < 2^24 and 255 G (2 r_max + 1) < 2^32.  Only K, r,
 * w32, m, G and u8_ok are read, during the call.
 * Errors: as rsg_gauss_filter; RSG_EINVAL (boxes NULL or inconsistent). */
int rsg_box_filter(const void* d_src, void* d_dst, int H, int W, int C, rsg_dtype dt,
                   const rsg_boxes* boxes, rsg_boundary b, void* stream);

/* Strided (downsampling) evaluation: the filtered image at every step-th row
 * and pixel only, out(i, j, c) = filtered(i step, j step, c), written as a
 * contiguous ceil(H/step) x ceil(W/step) x C image to d_dst (Eq. indep
 * evaluated on a sparser output grid, Section 3.3; the running sums still
 * cover every input sample).  Boxes: `boxes` if not NULL (as
 * rsg_box_filter), else rsg_fit_boxes(sigma, K).  The path is the one
 * rsg_gauss_filter would take: the fused kernel (its column pass stores
 * every step-th row and pixel only), or for wide boxes the two-pass path
 * (row filter keeping every step-th pixel into an intermediate of
 * ceil(W/step) C x H four-byte words, then the column filter keeping every
 * step-th row); step = 1 is rsg_gauss_filter / rsg_box_filter.
 * Errors: as rsg_gauss_filter / rsg_box_filter; RSG_EINVAL (step < 1);
 * RSG_EUNSUPPORTED (boxes too wide for the two-pass path: C = 3 beyond
 * r_max ~ 127, C = 4 beyond ~ 95). */
int rsg_gauss_filter_strided(const void* d_src, void* d_dst, int H, int W, int C, rsg_dtype dt, double sigma,
                             int K, const rsg_boxes* boxes, rsg_boundary b, int step, void* stream);

/* Filter a D x H x W x C FP32 volume (slice stride H*W*C, contiguous) with
 * the same K boxes along x, y and z: the separable method with one more 1D
 * pass for the third axis (Section 4 notes the extension to d dimensions).
 * Boxes: `boxes` if not NULL, else rsg_fit_boxes(sigma, K).  The slices are
 * filtered along x and y in one batched launch into a stream-ordered FP32
 * intermediate of D*H*W*C words, which a z-pass kernel filters along z into
 * d_dst (hipMallocAsync / hipFreeAsync on `stream`).  FP32 only: an exact
 * uint8 form would need G^3 * 255 < 2^64.
 * Errors: RSG_EINVAL (NULL pointers, D, H, W < 1, C not in 1..4, overlap,
 * bad sigma / K / boxes / boundary), RSG_EUNSUPPORTED (dt not FP32; boxes
 * wider than the kernels' limits: along z R <= 311), RSG_ENOMEM, RSG_EDEVICE. */
int rsg_gauss_filter_3d(const void* d_src, void* d_dst, int D, int H, int W, int C, rsg_dtype dt, double sigma,
                        int K, const rsg_boxes* boxes, rsg_boundary b, void* stream);

/* One image of a batch; strides in elements (0 means W*C). */
typedef struct {
    const void* src;
    void* dst;
    int32_t H, W, C;
    int64_t src_stride, dst_stride;
    rsg_dtype dt;
    double sigma;
    int32_t K;
    rsg_boundary b;
    const rsg_boxes* boxes;   /* NULL: rsg_fit_boxes(sigma, K); else these boxes (read during the call) */
} rsg_image_desc;

/* Bytes of device workspace rsg_filter_batch needs for these n images: the
 * work list (descriptors, task entries, counters) plus, for every image
 * planned on the two-pass path, its intermediate of 4 H W C bytes.
 * Errors: as rsg_gauss_filter for any descriptor, RSG_EINVAL (n < 1). */
int rsg_filter_batch_workspace(const rsg_image_desc* d, int n, size_t* bytes);

/* Filter n images of mixed size, channel count, dtype and sigma on
 * `stream`: one persistent launch per kernel class among the images planned
 * on the fused path (element type x channel count x tap count: a single
 * launch when the images share one), whose workgroups pop (image, task)
 * pairs from a shared counter, then for the images planned on the two-pass
 * path one launch per pass and pass instantiation.  The caller provides a
 * device workspace of at least rsg_filter_batch_workspace() bytes: the work
 * list is copied into it asynchronously on `stream` and the two-pass
 * intermediates are carved from it, so the workspace must not be reused
 * until the stream has passed this call.  The call allocates no device
 * memory.
 * Each image's result is bit-identical to rsg_gauss_filter on that image
 * alone: float images keep their single-image tile plan; uint8 images may
 * get longer segments in a batch (fewer halo rows), which cannot change
 * their exact integer results.
 * Errors: as rsg_gauss_filter, RSG_ENOMEM (ws_bytes too small). */
int rsg_filter_batch(const rsg_image_desc* d, int n, void* d_workspace, size_t ws_bytes,
                     void* stream);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of filter requests.                        */
/* ---------------------------------------------------------------------- */
typedef struct rsg_server rsg_server;

/* d_arena / arena_bytes: caller-owned device memory the server carves its
 * per-launch workspaces from: max_inflight equal slots, each holding one
 * launch's work list and the intermediates of its two-pass requests (the
 * server allocates no device memory).  hbm_budget: admission limit on the
 * sum of the in-flight requests' image bytes (src + dst); 0 means
 * unlimited.
 * max_inflight: launches outstanding at once (1..64); n_streams: HIP streams
 * the server creates (1..8); queue_depth: requests waiting for admission
 * (>= 1); max_batch: requests per launch (>= 1). */
typedef struct {
    void* d_arena;
    size_t arena_bytes;
    size_t hbm_budget;
    int32_t max_inflight;
    int32_t n_streams;
    int32_t queue_depth;
    int32_t max_batch;
} rsg_server_config;

/* Create a server and its scheduler thread on the current HIP device.
 * Errors: RSG_EINVAL (bad config), RSG_EDEVICE (stream creation). */
int rsg_server_create(const rsg_server_config* cfg, rsg_server** out);

/* Queue one request (device-resident src/dst, as rsg_image_desc); never
 * blocks (the scheduler plans and launches outside the server lock).
 * Requests are admitted in arrival order when the HBM budget, a free
 * in-flight slot and that slot's workspace allow, and batched with whatever
 * else is waiting into one batched launch (as rsg_filter_batch) while
 * earlier launches are still running on other slots and streams.
 * Errors: RSG_EINVAL (bad descriptor), RSG_ENOMEM (the request alone exceeds
 * the HBM budget, or its work list and intermediate exceed an arena slot),
 * RSG_EBUSY (queue full). */
int rsg_submit(rsg_server* s, const rsg_image_desc* req, uint64_t* ticket);

/* Timestamps are CLOCK_MONOTONIC nanoseconds. */
typedef struct {
    int32_t done;       /* 1 when the result is in dst */
    int32_t status;     /* RSG_OK or the failure of this request */
    uint64_t t_submit_ns, t_admit_ns, t_start_ns, t_done_ns;
} rsg_req_stats;

/* Non-blocking status of a ticket.  A ticket that is done is forgotten after
 * it has been reported once.  Errors: RSG_ENOTFOUND. */
int rsg_poll(rsg_server* s, uint64_t ticket, rsg_req_stats* out);

/* Drain all queued and in-flight work, stop the thread, free host state.  The
 * arena stays the caller's. */
int rsg_server_destroy(rsg_server* s);

/* ---------------------------------------------------------------------- */
/* Tile planning and tuning.                                               */
/* ---------------------------------------------------------------------- */
/* The tile plan rsg_gauss_filter / rsg_filter_batch would use for *d: the
 * segment height (output rows per task; every task covers 64 consecutive
 * samples of a row and streams 2R + 1 extra rows above its segment), the
 * number of tasks and the LDS bytes per task.  For an image planned on the
 * two-pass path the segment height is H, the tasks are the workgroups of
 * both passes (16 rows each; 8 in pass A for the widest multi-channel
 * windows) and the LDS is the larger pass's.  Host-only: d->src and d->dst
 * are compared but never dereferenced.  Segment heights come from the tuning
 * table named by the environment variable RSG_TUNE_TABLE (read once, lines
 * "dtype C rlo rhi nlo nhi hs [nc [lo [st]]]", with R the largest box
 * half-width, n the number of 64-sample strips times H, nc the columns per
 * lane of rsg_tune_columns, lo the first layout of rsg_tune_layout and st
 * the store form of rsg_tune_stores),
 * else from a built-in rule.  This is
 * the image's own plan; in a batch, uint8 images may get longer segments
 * (same results).  Any output pointer may be NULL.
 * Errors: as rsg_gauss_filter. */
int rsg_plan_shape(const rsg_image_desc* d, int32_t* seg_height, int32_t* tasks, uint32_t* lds_bytes);

/* Process-wide segment height used instead of the table and the built-in
 * rule (0 restores them); heights above H are clamped, and every result is
 * the same for any height up to FP32 rounding (bit-identical for uint8).
 * For the autotuner: it changes the plan of every later call on every
 * thread.  Errors: RSG_EINVAL (negative). */
int rsg_tune_override(int32_t seg_height);

/* Process-wide choice of kernel path for every later plan: 0 lets the
 * planner choose (the tuning table, else two passes for wide boxes,
 * R * C >= 40, when they fit), 1 forces the fused single-launch kernel
 * (workgroups of four waves per task, each wave running both passes on its
 * block of every step of rows), 2 forces the two-pass path (row filter into
 * an FP32 / uint32 intermediate stored transposed, then the same on the
 * intermediate; the intermediate, 4 H W C bytes, comes from where the entry
 * point takes it), 3 forces the fused kernel with one wave per task
 * (software-pipelined; batches planned under it use the one-wave batch
 * kernel too).  Results of the fused forms and of the two-pass path agree to
 * FP32 rounding and are bit-identical for uint8.  For the autotuner and
 * tests.
 * Errors: RSG_EINVAL (path not in 0..3); later plans return
 * RSG_EUNSUPPORTED when the forced path cannot hold the boxes. */
int rsg_tune_path(int32_t path);

/* Process-wide task form of the fused kernel for every later unstrided
 * plan: 0 lets the planner choose (the tuning table's optional field, else
 * 1); 1 gives each lane one sample column (strips of 64 interleaved
 * samples); 2 the wide form, where each lane owns two adjacent columns at
 * C = 1 (strips of 128 samples) or one pixel's three channels at C = 3
 * (strips of 64 pixels) and moves them with one vector access, at the price
 * of a larger LDS ring (C = 2 and 4, and images whose ring would not fit,
 * keep one column per lane); 3 channel-planar tasks on multi-channel images
 * (C >= 2): each task filters 64 pixels of one channel with the one-channel
 * kernel, reading its samples C apart, so its row span is 64 + 2R + 1
 * pixels instead of 64 + (2R + 1) C interleaved samples for 64 / C pixels
 * (volumes keep interleaved tasks).  Results agree to FP32 rounding
 * (bit-identical for uint8).  For the autotuner and tests.
 * Errors: RSG_EINVAL (not in 0..3). */
int rsg_tune_columns(int32_t columns);

/* Process-wide first row-scan layout of the fused kernel for every later
 * plan: 0 lets the planner choose (the tuning table's optional last field,
 * else the first layout whose rows cover the task's span), 1..3 start the
 * search at that layout.  Layouts are (lanes per row, samples per lane)
 * = (16, 8), (32, 8), (64, 8), (64, 16) at C = 1, 2, 4 and (16, 12), (32, 12),
 * (64, 12), (64, 24) at C = 3: later ones scan fewer, wider rows per group.
 * Results agree to FP32 rounding (bit-identical for
 * uint8).  For the autotuner and tests.  Errors: RSG_EINVAL (not in 0..3). */
int rsg_tune_layout(int32_t first);

/* Process-wide output store form of the fused kernel for every later FP32
 * plan with one column per lane: 0 lets the planner choose (the tuning
 * table's optional last field, else staged stores where the kernel has four
 * or five taps), 1 one store per lane and output row (4 bytes), 2 staged
 * stores: each wave writes its 8 x 64 results to its own LDS row tile and
 * stores them as 16-byte pieces of rows, on tasks whose column span lies
 * inside the image and whose output rows are 16-byte aligned (other tasks
 * keep the per-lane stores).  Results are bit-identical either way.  For the
 * autotuner and tests.  Errors: RSG_EINVAL (not in 0..2). */
int rsg_tune_stores(int32_t form);

/* ---------------------------------------------------------------------- */
/* Measurement.                                                            */
/* ---------------------------------------------------------------------- */
/* Copy `bytes` from d_src to d_dst on `stream` with a plain streaming copy
 * kernel (16-byte loads and stores, eight per thread in flight): the
 * achievable bandwidth the benchmark reports beside the filter's roofline.
 * Both buffers 16-byte aligned and not overlapping.
 * Errors: RSG_EINVAL (NULL or misaligned pointers), RSG_EUNSUPPORTED (more
 * than 2^31 blocks), RSG_EDEVICE (launch failure). */
int rsg_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream);

/* Message for the last failure on the calling thread ("" if none). */
const char* rsg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RSG_H */
