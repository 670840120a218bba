/*
 * Running-sum Gaussian filter: CPU ORACLE.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this code.  The product library (the HIP path) shares
 * nothing with it: no header, no helper, no table.  Everything here is plain
 * C in double precision (exact 64-bit integers for the uint8 path), written
 * for checking by eye against Elboher & Werman, "Efficient and Accurate
 * Gaussian Image Filtering Using Running Sums" (arXiv 1107.4958):
 *
 *   orc_phi        Section 4.1: the 1/f^2 autocorrelation model Phi, with the
 *                  missing DC value of the spectrum completed by a constant.
 *   orc_fit        Section 4.1 (quadratic-form error E2, Eq. "mahal") and
 *                  Section 4.2 (exhaustive search of the partition at sigma0).
 *   orc_scale      Section 4.2, Eq. "scale1"/"scale2" (per-sigma rescaling),
 *                  plus the readings listed below.
 *   orc_quant_u8   integer weights for exact uint8 filtering (a reading: the
 *                  paper has no integer scheme).
 *   orc_box_f64    the box approximation of Section 3 (Eq. "kerdec-1",
 *                  "S_i", "ciwi") applied separably (Section 3.4) by DIRECT
 *                  summation of every box: no running sums.
 *   orc_box_u8     the same in exact integers, rounded once at the end.
 *   orc_box3_f64   the same for a volume: one more pass along z.
 *   orc_gauss_f64  direct separable convolution with the sampled Gaussian
 *                  (the accuracy reference that replaces an exact library
 *                  Gaussian); orc_gauss_f64_points: the same at listed
 *                  output positions.
 *
 * Readings taken where the paper is silent or garbled:
 *   - slice weights w_i = c_i - c_{i+1} (c_{k+1} = 0): the printed index runs
 *     the other way, which does not telescope for the decreasing constants of
 *     Table 2;
 *   - half-widths p_i are inclusive: slice i covers |t| <= p_i, i.e. 2p_i+1
 *     samples, as the box difference I(x+p_i) - I(x-p_i-1) of Eq. "indep";
 *   - the Gaussian template is exp(-t^2 / (2 sigma0^2)) (the printed exponent
 *     has lost its minus sign);
 *   - the fit is over the full symmetric 2*100-1 samples t in [-99, 99]
 *     (t = 0 counted once), sigma0 = 100/pi;
 *   - Phi is the real inverse DFT over period N = 200 of S(u) = 1/u^2 on the
 *     integer frequency index u (folded: min(u, N-u)), S(0) = 16.5, and
 *     A_st = Phi((s - t) mod N);
 *   - the constants c are the least-squares optimum for each partition; only
 *     the partition is searched; ties go to the lexicographically smallest;
 *   - Eq. scale1 is evaluated as floor(sigma * p / sigma0 + 1e-9) so that a
 *     product that is an integer in exact arithmetic is not lost to rounding;
 *   - Eq. scale2 is applied as printed and the weights are then normalised to
 *     unit DC gain;
 *   - boundaries (the paper names none): replicate (clamp), zero extension,
 *     or reflect, the half-sample symmetric extension (... c b a | a b c d |
 *     d c b ...) repeated with period 2n for boxes wider than the axis;
 *     channels interleaved and filtered independently;
 *   - uint8 output: round half up of the exact rational U / G^2.
 * The direct fit at a target sigma (oracle/__init__.py, boxes_direct) runs
 * orc_fit on the Gaussian of that sigma with M = max(ceil(pi sigma), K) half
 * samples and Phi on period 2M, and takes r = p.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Section 4.1: Phi = real inverse DFT (period N) of the 1/u^2 spectrum.     */
/* Direct O(N^2) cosine sum, 1/N normalisation.                              */
/* ------------------------------------------------------------------------ */
void orc_phi(int N, double dc, double* phi)
{
    for (int l = 0; l < N; ++l) {
        double acc = 0.0;
        for (int u = 0; u < N; ++u) {
            double s;
            if (u == 0) {
                s = dc;
            } else {
                int f = (u < N - u) ? u : N - u;
                s = 1.0 / ((double)f * (double)f);
            }
            acc += s * cos(2.0 * ORC_PI * (double)u * (double)l / (double)N);
        }
        phi[l] = acc / (double)N;
    }
}

/* ------------------------------------------------------------------------ */
/* Section 4: the kernel-approximation problem at sigma0.                    */
/*                                                                          */
/* Samples t = -(nh-1) .. (nh-1), g(t) = exp(-t^2/(2 sigma0^2)).  A partition */
/* 0 <= p_1 < ... < p_k <= nh-1 defines k symmetric segments                 */
/*   seg_i = { t : p_{i-1} < |t| <= p_i },  p_0 = -1,                         */
/* and the approximation ghat(t) = c_i on seg_i, 0 beyond p_k.  The error is  */
/*   E2 = (g - ghat)^T A (g - ghat)                      (Eq. "mahal")        */
/* with A_st = Phi((s-t) mod N) (quadratic form) or A = I (plain l2).        */
/* For a fixed partition the optimal c solves M c = v with M = B^T A B,      */
/* v = B^T A g (B = segment indicator matrix) and E2 = g^T A g - v^T c.      */
/*                                                                          */
/* The block sums that make up M are read from a 2D summed-area table of     */
/* the "folded" matrix F[a][b] = sum of A over the sample pairs with |s| = a, */
/* |t| = b; v from a 1D prefix of the folded A g.                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nh;          /* half samples: t = 0 .. nh-1 */
    double* SA;      /* (nh+1)^2 summed-area table of F */
    double* Q;       /* nh+1 prefix of folded A g */
    double gAg;
} orc_problem;

static int orc_problem_build(int nh, double sigma0, int use_qf, int N, double dc,
                             orc_problem* pr)
{
    int n = 2 * nh - 1;              /* full symmetric sample count */
    double* A = (double*)malloc(sizeof(double) * (size_t)n * n);
    double* g = (double*)malloc(sizeof(double) * n);
    double* phi = NULL;
    if (!A || !g) { free(A); free(g); return -1; }
    if (use_qf) {
        phi = (double*)malloc(sizeof(double) * N);
        if (!phi) { free(A); free(g); return -1; }
        orc_phi(N, dc, phi);
    }
    for (int i = 0; i < n; ++i) {
        int t = i - (nh - 1);
        g[i] = exp(-(double)t * t / (2.0 * sigma0 * sigma0));
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (use_qf) {
                int lag = ((i - j) % N + N) % N;
                A[(size_t)i * n + j] = phi[lag];
            } else {
                A[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
            }
        }
    /* folded matrix F and folded vector q */
    double* F = (double*)calloc((size_t)nh * nh, sizeof(double));
    double* q = (double*)calloc((size_t)nh, sizeof(double));
    double gAg = 0.0;
    for (int i = 0; i < n; ++i) {
        int a = abs(i - (nh - 1));
        double Ag = 0.0;
        for (int j = 0; j < n; ++j) {
            int b = abs(j - (nh - 1));
            F[(size_t)a * nh + b] += A[(size_t)i * n + j];
            Ag += A[(size_t)i * n + j] * g[j];
        }
        q[a] += Ag;
        gAg += g[i] * Ag;
    }
    pr->nh = nh;
    pr->SA = (double*)calloc((size_t)(nh + 1) * (nh + 1), sizeof(double));
    pr->Q = (double*)calloc((size_t)(nh + 1), sizeof(double));
    for (int a = 0; a < nh; ++a)
        for (int b = 0; b < nh; ++b)
            pr->SA[(size_t)(a + 1) * (nh + 1) + (b + 1)] =
                F[(size_t)a * nh + b] + pr->SA[(size_t)a * (nh + 1) + (b + 1)] +
                pr->SA[(size_t)(a + 1) * (nh + 1) + b] - pr->SA[(size_t)a * (nh + 1) + b];
    for (int a = 0; a < nh; ++a) pr->Q[a + 1] = pr->Q[a] + q[a];
    pr->gAg = gAg;
    free(A); free(g); free(phi); free(F); free(q);
    return 0;
}

static void orc_problem_free(orc_problem* pr)
{
    free(pr->SA); free(pr->Q);
}

/* Solve the k x k SPD system M c = v by Cholesky; returns E2 = gAg - v.c, or
 * +inf when M is not positive definite. */
static double orc_partition_error(const orc_problem* pr, int k, const int* p, double* c)
{
    int nh1 = pr->nh + 1;
    int lo[8], hi[8];
    double M[8][8], L[8][8], v[8], z[8];
    for (int i = 0; i < k; ++i) {
        lo[i] = (i == 0) ? 0 : p[i - 1] + 1;
        hi[i] = p[i] + 1;
    }
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j < k; ++j)
            M[i][j] = pr->SA[(size_t)hi[i] * nh1 + hi[j]] - pr->SA[(size_t)lo[i] * nh1 + hi[j]]
                    - pr->SA[(size_t)hi[i] * nh1 + lo[j]] + pr->SA[(size_t)lo[i] * nh1 + lo[j]];
        v[i] = pr->Q[hi[i]] - pr->Q[lo[i]];
    }
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = M[i][j];
            for (int t = 0; t < j; ++t) s -= L[i][t] * L[j][t];
            if (i == j) {
                if (!(s > 0.0)) return INFINITY;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    for (int i = 0; i < k; ++i) {          /* L z = v */
        double s = v[i];
        for (int t = 0; t < i; ++t) s -= L[i][t] * z[t];
        z[i] = s / L[i][i];
    }
    for (int i = k - 1; i >= 0; --i) {     /* L^T c = z */
        double s = z[i];
        for (int t = i + 1; t < k; ++t) s -= L[t][i] * c[t];
        c[i] = s / L[i][i];
    }
    double vc = 0.0;
    for (int i = 0; i < k; ++i) vc += v[i] * c[i];
    return pr->gAg - vc;
}

/* Error and constants of one given partition (exposed for pinning). */
int orc_eval_partition(int nh, double sigma0, int use_qf, int N, double dc,
                       int k, const int* p, double* c, double* err)
{
    if (k < 1 || k > 8) return -1;
    for (int i = 0; i < k; ++i) {
        if (p[i] < 0 || p[i] >= nh) return -1;
        if (i > 0 && p[i] <= p[i - 1]) return -1;
    }
    orc_problem pr;
    if (orc_problem_build(nh, sigma0, use_qf, N, dc, &pr)) return -1;
    *err = orc_partition_error(&pr, k, p, c);
    orc_problem_free(&pr);
    return 0;
}

/* Exhaustive search over all C(nh, k) partitions (Section 4.2). */
int orc_fit(int nh, double sigma0, int use_qf, int N, double dc, int k,
            int* p_out, double* c_out, double* err_out)
{
    if (k < 1 || k > 8 || k > nh) return -1;
    orc_problem pr;
    if (orc_problem_build(nh, sigma0, use_qf, N, dc, &pr)) return -1;

    double best = INFINITY;
    int bestp[8] = {0};
    /* One task per value of p_1; each task enumerates p_2 < ... < p_k in
     * lexicographic order and keeps its first minimum. */
    #pragma omp parallel
    {
        double tbest = INFINITY;
        int tp[8] = {0};
        #pragma omp for schedule(dynamic, 1)
        for (int p1 = 0; p1 <= nh - k; ++p1) {
            int p[8];
            double c[8];
            p[0] = p1;
            for (int i = 1; i < k; ++i) p[i] = p1 + i;
            for (;;) {
                double e = orc_partition_error(&pr, k, p, c);
                if (e < tbest) {
                    tbest = e;
                    memcpy(tp, p, sizeof(int) * k);
                }
                /* next combination with p[0] fixed */
                int i = k - 1;
                while (i >= 1 && p[i] == nh - k + i) --i;
                if (i < 1) break;
                ++p[i];
                for (int j = i + 1; j < k; ++j) p[j] = p[j - 1] + 1;
            }
        }
        #pragma omp critical
        {
            int take = 0;
            if (tbest < best) take = 1;
            else if (tbest == best) {
                for (int i = 0; i < k; ++i) {
                    if (tp[i] != bestp[i]) { take = tp[i] < bestp[i]; break; }
                }
            }
            if (take) { best = tbest; memcpy(bestp, tp, sizeof(int) * k); }
        }
    }
    memcpy(p_out, bestp, sizeof(int) * k);
    *err_out = orc_partition_error(&pr, k, bestp, c_out);
    orc_problem_free(&pr);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 4.2, Eq. scale1 / scale2, then normalisation to unit DC gain.     */
/*   r_i = floor(sigma / sigma0 * p_i)   (evaluated with a 1e-9 guard)       */
/*   w_i = c_i - c_{i+1}            (slice weights, Section 3.2)             */
/*   what_i = w_i * p_i / (2 r_i + 1)                                        */
/*   what_i /= sum_j what_j (2 r_j + 1)                                      */
/* w32 are the single-precision roundings of the normalised weights.         */
/* ------------------------------------------------------------------------ */
int orc_scale(double sigma, double sigma0, int k, const int* p, const double* c,
              int* r, double* w, float* w32)
{
    if (!(sigma > 0.0) || k < 1 || k > 8) return -1;
    double z = 0.0;
    for (int i = 0; i < k; ++i) {
        double wi = c[i] - ((i + 1 < k) ? c[i + 1] : 0.0);
        /* a 1e-9 guard keeps exact integer products (sigma = sigma0) from
         * flooring to the integer below through FP64 rounding */
        double ri = floor(sigma * (double)p[i] / sigma0 + 1e-9);
        if (ri > 1.0e9) return -1;
        r[i] = (int)ri;
        w[i] = wi * (double)p[i] / (2.0 * r[i] + 1.0);
        z += w[i] * (2.0 * r[i] + 1.0);
    }
    if (!(z > 0.0)) return -1;
    for (int i = 0; i < k; ++i) {
        w[i] /= z;
        w32[i] = (float)w[i];
    }
    return 0;
}

/* Integer weights for exact uint8 filtering (a reading; the paper has none):
 * s is the largest integer in [1, 23] such that, with m_i = rint(w_i 2^s) and
 * G = sum m_i (2 r_i + 1), all m_i >= 0, G < 2^24 and
 * 255 * G * (2 r_max + 1) < 2^32.  Returns -1 when no s qualifies. */
int orc_quant_u8(int k, const int* r, const double* w, int64_t* m, int64_t* G, int* s_out)
{
    int rmax = 0;
    for (int i = 0; i < k; ++i) if (r[i] > rmax) rmax = r[i];
    for (int s = 23; s >= 1; --s) {
        int64_t g = 0;
        int ok = 1;
        for (int i = 0; i < k; ++i) {
            double mi = rint(ldexp(w[i], s));
            if (mi < 0.0) { ok = 0; break; }
            m[i] = (int64_t)mi;
            g += m[i] * (2 * (int64_t)r[i] + 1);
        }
        if (!ok) continue;
        if (g <= 0 || g >= ((int64_t)1 << 24)) continue;
        if ((int64_t)255 * g * (2 * (int64_t)rmax + 1) >= ((int64_t)1 << 32)) continue;
        *G = g;
        *s_out = s;
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Boundary extension along one axis of length n.                            */
/* ------------------------------------------------------------------------ */
static inline int orc_ext(int i, int n, int boundary, int* inside)
{
    if (i >= 0 && i < n) { *inside = 1; return i; }
    if (boundary == 0) { *inside = 1; return i < 0 ? 0 : n - 1; }   /* replicate */
    if (boundary == 2) {                                           /* reflect */
        /* half-sample symmetric extension: f(-1) = f(0), f(n) = f(n-1),
         * repeated with period 2n so that any offset is defined */
        int64_t p = 2 * (int64_t)n;
        int64_t m = (int64_t)i % p;
        if (m < 0) m += p;
        *inside = 1;
        return (int)(m < n ? m : p - 1 - m);
    }
    *inside = 0;                                                   /* zero */
    return 0;
}

/* Box approximation, FP64, direct summation (Section 3 + 3.4).
 *   T(y,x,c) = sum_j w_j sum_{a=-r_j..r_j} f(y, ext(x+a), c)
 *   g(y,x,c) = sum_j w_j sum_{b=-r_j..r_j} T(ext(y+b), x, c)
 * Layout: interleaved H x W x C, row stride W*C. */
int orc_box_f64(const double* src, int H, int W, int C, int k, const int* r,
                const double* w, int boundary, double* dst)
{
    if (H < 1 || W < 1 || C < 1 || k < 1) return -1;
    size_t n = (size_t)H * W * C;
    double* T = (double*)malloc(sizeof(double) * n);
    if (!T) return -1;
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                double acc = 0.0;
                for (int j = 0; j < k; ++j) {
                    double box = 0.0;
                    for (int a = -r[j]; a <= r[j]; ++a) {
                        int in;
                        int xx = orc_ext(x + a, W, boundary, &in);
                        if (in) box += src[((size_t)y * W + xx) * C + c];
                    }
                    acc += w[j] * box;
                }
                T[((size_t)y * W + x) * C + c] = acc;
            }
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                double acc = 0.0;
                for (int j = 0; j < k; ++j) {
                    double box = 0.0;
                    for (int b = -r[j]; b <= r[j]; ++b) {
                        int in;
                        int yy = orc_ext(y + b, H, boundary, &in);
                        if (in) box += T[((size_t)yy * W + x) * C + c];
                    }
                    acc += w[j] * box;
                }
                dst[((size_t)y * W + x) * C + c] = acc;
            }
    free(T);
    return 0;
}

/* The box approximation of a volume (Section 4's d-dimensional remark:
 * the separable filter takes one more 1D pass per axis).  FP64, direct
 * summation: each z-slice is filtered in 2D as orc_box_f64, then
 *   g(z,y,x,c) = sum_j w_j sum_{e=-r_j..r_j} S(ext(z+e), y, x, c).
 * Layout: D x H x W x C, slice stride H*W*C. */
int orc_box3_f64(const double* src, int D, int H, int W, int C, int k, const int* r,
                 const double* w, int boundary, double* dst)
{
    if (D < 1 || H < 1 || W < 1 || C < 1 || k < 1) return -1;
    size_t plane = (size_t)H * W * C;
    double* S = (double*)malloc(sizeof(double) * plane * D);
    if (!S) return -1;
    for (int z = 0; z < D; ++z) {
        if (orc_box_f64(src + plane * z, H, W, C, k, r, w, boundary, S + plane * z) != 0) {
            free(S);
            return -1;
        }
    }
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < D; ++z)
        for (size_t i = 0; i < plane; ++i) {
            double acc = 0.0;
            for (int j = 0; j < k; ++j) {
                double box = 0.0;
                for (int e = -r[j]; e <= r[j]; ++e) {
                    int in;
                    int zz = orc_ext(z + e, D, boundary, &in);
                    if (in) box += S[plane * zz + i];
                }
                acc += w[j] * box;
            }
            dst[plane * z + i] = acc;
        }
    free(S);
    return 0;
}

/* Box approximation in exact integers for uint8 images.
 *   T = sum_j m_j * (row box sum of f),  U = sum_j m_j * (column box sum of T)
 *   out = floor((U + floor(G^2/2)) / G^2)      (round half up of U / G^2)
 * Every partial sum is below 2^63. */
int orc_box_u8(const uint8_t* src, int H, int W, int C, int k, const int* r,
               const int64_t* m, int64_t G, int boundary, uint8_t* dst)
{
    if (H < 1 || W < 1 || C < 1 || k < 1 || G <= 0) return -1;
    size_t n = (size_t)H * W * C;
    int64_t* T = (int64_t*)malloc(sizeof(int64_t) * n);
    if (!T) return -1;
    int64_t G2 = G * G;
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                int64_t acc = 0;
                for (int j = 0; j < k; ++j) {
                    int64_t box = 0;
                    for (int a = -r[j]; a <= r[j]; ++a) {
                        int in;
                        int xx = orc_ext(x + a, W, boundary, &in);
                        if (in) box += src[((size_t)y * W + xx) * C + c];
                    }
                    acc += m[j] * box;
                }
                T[((size_t)y * W + x) * C + c] = acc;
            }
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                int64_t acc = 0;
                for (int j = 0; j < k; ++j) {
                    int64_t box = 0;
                    for (int b = -r[j]; b <= r[j]; ++b) {
                        int in;
                        int yy = orc_ext(y + b, H, boundary, &in);
                        if (in) box += T[((size_t)yy * W + x) * C + c];
                    }
                    acc += m[j] * box;
                }
                int64_t q = (acc + G2 / 2) / G2;
                dst[((size_t)y * W + x) * C + c] = (uint8_t)q;
            }
    free(T);
    return 0;
}

/* Sampled Gaussian, direct separable convolution in FP64: taps
 * exp(-t^2/(2 sigma^2)) for |t| <= R = ceil(6 sigma), normalised to sum 1. */
int orc_gauss_f64(const double* src, int H, int W, int C, double sigma, int boundary,
                  double* dst)
{
    if (H < 1 || W < 1 || C < 1 || !(sigma > 0.0)) return -1;
    int R = (int)ceil(6.0 * sigma);
    double* g = (double*)malloc(sizeof(double) * (2 * (size_t)R + 1));
    size_t n = (size_t)H * W * C;
    double* T = (double*)malloc(sizeof(double) * n);
    if (!g || !T) { free(g); free(T); return -1; }
    double z = 0.0;
    for (int t = -R; t <= R; ++t) { g[t + R] = exp(-(double)t * t / (2.0 * sigma * sigma)); z += g[t + R]; }
    for (int t = 0; t <= 2 * R; ++t) g[t] /= z;
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                double acc = 0.0;
                for (int a = -R; a <= R; ++a) {
                    int in;
                    int xx = orc_ext(x + a, W, boundary, &in);
                    if (in) acc += g[a + R] * src[((size_t)y * W + xx) * C + c];
                }
                T[((size_t)y * W + x) * C + c] = acc;
            }
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                double acc = 0.0;
                for (int b = -R; b <= R; ++b) {
                    int in;
                    int yy = orc_ext(y + b, H, boundary, &in);
                    if (in) acc += g[b + R] * T[((size_t)yy * W + x) * C + c];
                }
                dst[((size_t)y * W + x) * C + c] = acc;
            }
    free(g); free(T);
    return 0;
}

/* Pointwise versions for sampled checks at full size: the same sums as
 * orc_box_f64 / orc_box_u8, for a list of output positions only.  Each
 * output needs the row pass at the 2 r_max + 1 rows around it. */
int orc_box_f64_points(const double* src, int H, int W, int C, int k, const int* r,
                       const double* w, int boundary, int npts, const int64_t* ys,
                       const int64_t* xs, const int64_t* cs, double* out)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int pidx = 0; pidx < npts; ++pidx) {
        int y = (int)ys[pidx], x = (int)xs[pidx], c = (int)cs[pidx];
        double acc = 0.0;
        for (int j = 0; j < k; ++j) {
            double box = 0.0;
            for (int b = -r[j]; b <= r[j]; ++b) {
                int in;
                int yy = orc_ext(y + b, H, boundary, &in);
                if (!in) continue;
                double t = 0.0;
                for (int i = 0; i < k; ++i) {
                    double rb = 0.0;
                    for (int a = -r[i]; a <= r[i]; ++a) {
                        int in2;
                        int xx = orc_ext(x + a, W, boundary, &in2);
                        if (in2) rb += src[((size_t)yy * W + xx) * C + c];
                    }
                    t += w[i] * rb;
                }
                box += t;
            }
            acc += w[j] * box;
        }
        out[pidx] = acc;
    }
    return 0;
}

int orc_box_u8_points(const uint8_t* src, int H, int W, int C, int k, const int* r,
                      const int64_t* m, int64_t G, int boundary, int npts,
                      const int64_t* ys, const int64_t* xs, const int64_t* cs, uint8_t* out)
{
    int64_t G2 = G * G;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int pidx = 0; pidx < npts; ++pidx) {
        int y = (int)ys[pidx], x = (int)xs[pidx], c = (int)cs[pidx];
        int64_t acc = 0;
        for (int j = 0; j < k; ++j) {
            int64_t box = 0;
            for (int b = -r[j]; b <= r[j]; ++b) {
                int in;
                int yy = orc_ext(y + b, H, boundary, &in);
                if (!in) continue;
                int64_t t = 0;
                for (int i = 0; i < k; ++i) {
                    int64_t rb = 0;
                    for (int a = -r[i]; a <= r[i]; ++a) {
                        int in2;
                        int xx = orc_ext(x + a, W, boundary, &in2);
                        if (in2) rb += src[((size_t)yy * W + xx) * C + c];
                    }
                    t += m[i] * rb;
                }
                box += t;
            }
            acc += m[j] * box;
        }
        out[pidx] = (uint8_t)((acc + G2 / 2) / G2);
    }
    return 0;
}

/* The sampled-Gaussian reference at a list of output positions only: the
 * same separable sums as orc_gauss_f64 (|t| <= ceil(6 sigma), normalised
 * taps), evaluated directly around each point. */
int orc_gauss_f64_points(const double* src, int H, int W, int C, double sigma, int boundary, int npts,
                         const int64_t* ys, const int64_t* xs, const int64_t* cs, double* out)
{
    if (H < 1 || W < 1 || C < 1 || !(sigma > 0.0)) return -1;
    int R = (int)ceil(6.0 * sigma);
    double* g = (double*)malloc(sizeof(double) * (2 * (size_t)R + 1));
    if (!g) return -1;
    double z = 0.0;
    for (int t = -R; t <= R; ++t) { g[t + R] = exp(-(double)t * t / (2.0 * sigma * sigma)); z += g[t + R]; }
    for (int t = 0; t <= 2 * R; ++t) g[t] /= z;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int pidx = 0; pidx < npts; ++pidx) {
        int y = (int)ys[pidx], x = (int)xs[pidx], c = (int)cs[pidx];
        double acc = 0.0;
        for (int b = -R; b <= R; ++b) {
            int in;
            int yy = orc_ext(y + b, H, boundary, &in);
            if (!in) continue;
            double row = 0.0;
            for (int a = -R; a <= R; ++a) {
                int in2;
                int xx = orc_ext(x + a, W, boundary, &in2);
                if (in2) row += g[a + R] * src[((size_t)yy * W + xx) * C + c];
            }
            acc += g[b + R] * row;
        }
        out[pidx] = acc;
    }
    free(g);
    return 0;
}
