// Host-side kernel design for the running-sum Gaussian filter, in FP64.  FP64
// is used only on the host: here, and by the planner for two constants
// derived from these weights (the FP32 reciprocal of G^2 and the DC gain of
// the FP32 weights); the kernels compute in FP32 and in integers.
//
//   Section 4.1  quadratic-form kernel error E2 = (g - ghat)^T A (g - ghat)
//                (Eq. mahal) with A_st = Phi(s - t), Phi the autocorrelation
//                of a 1/f image: the inverse DFT of 1/u^2 with the missing DC
//                value completed as 16.5.
//   Section 4.2  exhaustive search over every partition of the 100 half
//                samples of a Gaussian with sigma0 = 100/pi; rescaling of the
//                half-widths (Eq. scale1) and weights (Eq. scale2) to sigma.
//
// Besides the paper's rescaled fit there are two more methods: the same with
// the l2 error (A = I, the paper's alternative error measure), and a direct
// fit at the target sigma: the search run on the Gaussian of that sigma over
// M = max(ceil(pi sigma), K) half samples with Phi on period 2M (the paper's
// problem at sigma0 is the case M = 100), taking r = p.  At small sigma the
// rescaled half-widths floor to a few repeated values; the direct fit keeps
// K distinct ones.
//
// The search visits partitions in lexicographic order as a tree: fixing
// p_1..p_d fixes the first d segments, hence the leading d x d block of the
// normal matrix M = B^T A B and the first d entries of v = B^T A g.  The
// Cholesky factor L of M and the forward solution z = L^-1 v are therefore
// built one row per tree level, and the error of a complete partition is
// g^T A g - |z|^2, an O(K) update at each leaf.
#include "rsg_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

namespace rsg {

namespace {

constexpr int kHalf = 100;                 // half samples t = 0..99 at sigma0
constexpr int kPeriod = 200;               // DFT period of Phi at sigma0
constexpr double kDc = 16.5;               // completed DC value of the spectrum
const double kSigma0 = 100.0 / M_PI;

struct FitProblem {
    int nh = kHalf;            // half samples t = 0..nh-1
    // block sums of the folded matrix over half-index ranges [a0, a1) x [b0, b1)
    std::vector<double> sat;   // (nh+1)^2 summed-area table
    std::vector<double> vpre;  // nh+1 prefix of the folded A g
    double gag = 0.0;

    double block(int a0, int a1, int b0, int b1) const {
        const int n = nh + 1;
        return sat[a1 * n + b1] - sat[a0 * n + b1] - sat[a1 * n + b0] + sat[a0 * n + b0];
    }
    double vsum(int a0, int a1) const { return vpre[a1] - vpre[a0]; }
};

// The problem of fitting the Gaussian of s.d. sig over nh half samples, with
// Phi on period N (quadratic form) or A = I (l2).
FitProblem build_problem(bool quadratic_form, int nh = kHalf, int N = kPeriod, double sig = kSigma0)
{
    // autocorrelation model: Phi(l) = (1/N) sum_u S(u) cos(2 pi u l / N)
    std::vector<double> phi(N, 0.0);
    if (quadratic_form) {
        for (int l = 0; l < N; ++l) {
            double acc = kDc;
            for (int u = 1; u < N; ++u) {
                const int f = std::min(u, N - u);
                acc += std::cos(2.0 * M_PI * double(u) * double(l) / double(N)) / (double(f) * f);
            }
            phi[l] = acc / N;
        }
    }
    auto A = [&](int s, int t) -> double {   // s, t signed sample positions
        if (!quadratic_form) return s == t ? 1.0 : 0.0;
        const int lag = ((s - t) % N + N) % N;
        return phi[lag];
    };
    auto g = [sig](int t) { return std::exp(-double(t) * t / (2.0 * sig * sig)); };

    // folded matrix over |s| = a, |t| = b: sum over the (one or two) signs
    std::vector<double> F(nh * nh, 0.0), q(nh, 0.0);
    for (int a = 0; a < nh; ++a) {
        const int na = a ? 2 : 1;
        for (int b = 0; b < nh; ++b) {
            const int nb = b ? 2 : 1;
            double acc = 0.0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) acc += A(i ? -a : a, j ? -b : b);
            F[a * nh + b] = acc;
        }
    }
    FitProblem pr;
    pr.nh = nh;
    // v = B^T A g folded; gAg over the full symmetric support
    for (int a = 0; a < nh; ++a) {
        double acc = 0.0;
        for (int b = 0; b < nh; ++b) acc += F[a * nh + b] * g(b);
        q[a] = acc;
        // q[a] sums (A g)_s over the signs s = +-a; g is symmetric, so
        // sum_a g(a) q[a] = g^T A g
        pr.gag += g(a) * acc;
    }
    const int n = nh + 1;
    pr.sat.assign(n * n, 0.0);
    for (int a = 0; a < nh; ++a)
        for (int b = 0; b < nh; ++b)
            pr.sat[(a + 1) * n + b + 1] = F[a * nh + b] + pr.sat[a * n + b + 1] +
                                          pr.sat[(a + 1) * n + b] - pr.sat[a * n + b];
    pr.vpre.assign(n, 0.0);
    for (int a = 0; a < nh; ++a) pr.vpre[a + 1] = pr.vpre[a] + q[a];
    return pr;
}

struct SearchState {
    int K;
    const FitProblem* pr;
    int lo[RSG_MAX_K], hi[RSG_MAX_K];   // segment half-index ranges [lo, hi)
    double L[RSG_MAX_K][RSG_MAX_K];
    double z[RSG_MAX_K];
    double zz[RSG_MAX_K + 1];           // running |z|^2 of the first d levels
    double best = -1.0;                 // max |z|^2 (== min error)
    int bestp[RSG_MAX_K];
};

// Fill row d of L and z for segment d = [lo[d], hi[d]); false if not PD.
inline bool factor_row(SearchState& st, int d)
{
    const FitProblem& pr = *st.pr;
    for (int j = 0; j <= d; ++j) {
        double mdj = pr.block(st.lo[d], st.hi[d], st.lo[j], st.hi[j]);
        for (int t = 0; t < j; ++t) mdj -= st.L[d][t] * st.L[j][t];
        if (j < d) {
            st.L[d][j] = mdj / st.L[j][j];
        } else {
            if (!(mdj > 0.0)) return false;
            st.L[d][d] = std::sqrt(mdj);
        }
    }
    double zd = pr.vsum(st.lo[d], st.hi[d]);
    for (int t = 0; t < d; ++t) zd -= st.L[d][t] * st.z[t];
    st.z[d] = zd / st.L[d][d];
    st.zz[d + 1] = st.zz[d] + st.z[d] * st.z[d];
    return true;
}

void descend(SearchState& st, int d, int pmin)
{
    const int last = st.pr->nh - (st.K - d); // largest p_d leaving room for the rest
    for (int p = pmin; p <= last; ++p) {
        st.lo[d] = (d == 0) ? 0 : st.hi[d - 1];
        st.hi[d] = p + 1;
        if (!factor_row(st, d)) continue;
        if (d + 1 == st.K) {
            if (st.zz[d + 1] > st.best) {    // strict: keeps the lexicographically first
                st.best = st.zz[d + 1];
                for (int i = 0; i < st.K; ++i) st.bestp[i] = st.hi[i] - 1;
            }
        } else {
            descend(st, d + 1, p + 1);
        }
    }
}

// Least-squares constants of one partition (plain Cholesky solve).
void solve_constants(const FitProblem& pr, int K, const int* p, double* c, double* err)
{
    double M[RSG_MAX_K][RSG_MAX_K], v[RSG_MAX_K], L[RSG_MAX_K][RSG_MAX_K], y[RSG_MAX_K];
    int lo[RSG_MAX_K], hi[RSG_MAX_K];
    for (int i = 0; i < K; ++i) { lo[i] = i ? p[i - 1] + 1 : 0; hi[i] = p[i] + 1; }
    for (int i = 0; i < K; ++i) {
        for (int j = 0; j < K; ++j) M[i][j] = pr.block(lo[i], hi[i], lo[j], hi[j]);
        v[i] = pr.vsum(lo[i], hi[i]);
    }
    for (int i = 0; i < K; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = M[i][j];
            for (int t = 0; t < j; ++t) s -= L[i][t] * L[j][t];
            L[i][j] = (i == j) ? std::sqrt(s) : s / L[j][j];
        }
    for (int i = 0; i < K; ++i) {
        double s = v[i];
        for (int t = 0; t < i; ++t) s -= L[i][t] * y[t];
        y[i] = s / L[i][i];
    }
    for (int i = K - 1; i >= 0; --i) {
        double s = y[i];
        for (int t = i + 1; t < K; ++t) s -= L[t][i] * c[t];
        c[i] = s / L[i][i];
    }
    double vc = 0.0;
    for (int i = 0; i < K; ++i) vc += v[i] * c[i];
    *err = pr.gag - vc;
}

struct Sigma0Fit {
    int K = 0;
    int p[RSG_MAX_K] = {0};
    double c[RSG_MAX_K] = {0};
    double err = 0.0;
};

Sigma0Fit run_search(int K, bool quadratic_form, int nh = kHalf, int N = kPeriod, double sig = kSigma0)
{
    const FitProblem pr = build_problem(quadratic_form, nh, N, sig);
    const int first_max = nh - K;
    unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<SearchState> states(first_max + 1);
    std::mutex mu;
    int next = 0;
    auto worker = [&]() {
        for (;;) {
            int p1;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (next > first_max) return;
                p1 = next++;
            }
            SearchState& st = states[p1];
            st.K = K;
            st.pr = &pr;
            st.zz[0] = 0.0;
            st.lo[0] = 0;
            st.hi[0] = p1 + 1;
            if (!factor_row(st, 0)) continue;
            if (K == 1) {
                st.best = st.zz[1];
                st.bestp[0] = p1;
            } else {
                descend(st, 1, p1 + 1);
            }
        }
    };
    std::vector<std::thread> pool;
    for (unsigned i = 0; i < nthreads; ++i) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
    // combine in p_1 order: strict improvement keeps the lexicographic first
    Sigma0Fit out;
    out.K = K;
    double best = -1.0;
    for (int p1 = 0; p1 <= first_max; ++p1) {
        if (states[p1].best > best) {
            best = states[p1].best;
            std::memcpy(out.p, states[p1].bestp, sizeof(int) * K);
        }
    }
    solve_constants(pr, K, out.p, out.c, &out.err);
    return out;
}

std::once_flag g_once[RSG_MAX_K + 1][2];
Sigma0Fit g_fit[RSG_MAX_K + 1][2];

// Direct fits, cached per (K, sigma); a small bounded cache (the search at
// M <= 100 half samples costs at most as much as the sigma0 search).
std::mutex g_direct_mu;
std::vector<std::pair<std::pair<int, double>, Sigma0Fit>> g_direct;
constexpr size_t kDirectCache = 256;

Sigma0Fit direct_fit(int K, double sigma, int M)
{
    {
        std::lock_guard<std::mutex> lk(g_direct_mu);
        for (const auto& e : g_direct)
            if (e.first.first == K && e.first.second == sigma) return e.second;
    }
    Sigma0Fit f = run_search(K, true, M, 2 * M, sigma);
    std::lock_guard<std::mutex> lk(g_direct_mu);
    if (g_direct.size() >= kDirectCache) g_direct.erase(g_direct.begin());
    g_direct.push_back({{K, sigma}, f});
    return f;
}

// uint8 fixed point: the largest s in [1, 23] with every m_k = rint(w_k 2^s)
// >= 0, G = sum m_k (2 r_k + 1) < 2^24 and 255 G (2 r_max + 1) < 2^32.
void quantize_u8(rsg_boxes& b)
{
    int64_t rmax = 0;
    for (int k = 0; k < b.K; ++k) rmax = std::max<int64_t>(rmax, b.r[k]);
    b.u8_ok = 0;
    for (int s = 23; s >= 1 && !b.u8_ok; --s) {
        int64_t G = 0;
        uint32_t m[RSG_MAX_K];
        bool neg = false;
        for (int k = 0; k < b.K; ++k) {
            const double mk = std::nearbyint(std::ldexp(b.w[k], s));
            if (mk < 0.0) { neg = true; break; }
            m[k] = uint32_t(mk);
            G += int64_t(m[k]) * (2 * int64_t(b.r[k]) + 1);
        }
        if (neg || G <= 0 || G >= (int64_t(1) << 24)) continue;
        if (int64_t(255) * G * (2 * rmax + 1) >= (int64_t(1) << 32)) continue;
        std::memcpy(b.m, m, sizeof(uint32_t) * b.K);
        b.G = uint64_t(G);
        b.s = s;
        b.u8_ok = 1;
    }
}

}  // namespace

const double kSigma0Value = 100.0 / M_PI;

int sigma0_fit(int K, bool quadratic_form, int* p, double* c, double* err)
{
    if (K < 1 || K > RSG_MAX_K) return RSG_EUNSUPPORTED;
    const int q = quadratic_form ? 1 : 0;
    std::call_once(g_once[K][q], [&] { g_fit[K][q] = run_search(K, quadratic_form); });
    const Sigma0Fit& f = g_fit[K][q];
    std::memcpy(p, f.p, sizeof(int) * K);
    std::memcpy(c, f.c, sizeof(double) * K);
    *err = f.err;
    return RSG_OK;
}

int make_boxes(double sigma, int K, int method, rsg_boxes* out)
{
    if (!out) return set_error(RSG_EINVAL, "rsg_fit_boxes: out is NULL");
    if (!(sigma > 0.0) || !std::isfinite(sigma))
        return set_error(RSG_EINVAL, "rsg_fit_boxes: sigma must be finite and > 0");
    if (K < 1) return set_error(RSG_EINVAL, "rsg_fit_boxes: K must be >= 1");
    if (K > RSG_MAX_K) return set_error(RSG_EUNSUPPORTED, "rsg_fit_boxes: K > 5 is not supported");
    if (method < RSG_FIT_SCALED || method > RSG_FIT_DIRECT)
        return set_error(RSG_EINVAL, "rsg_fit_boxes: bad fit method %d", method);
    rsg_boxes b;
    std::memset(&b, 0, sizeof(b));
    b.K = K;
    b.sigma = sigma;

    if (method == RSG_FIT_DIRECT) {
        const double mh = std::ceil(M_PI * sigma - 1e-9);
        if (mh > double(kHalf))
            return set_error(RSG_EUNSUPPORTED, "rsg_fit_boxes: the direct fit covers sigma <= 100/pi (got %g)", sigma);
        const int M = std::max(int(mh), K);
        const Sigma0Fit f = direct_fit(K, sigma, M);
        std::memcpy(b.p, f.p, sizeof(int) * K);
        std::memcpy(b.c, f.c, sizeof(double) * K);
        b.fit_err = f.err;
        // r = p; slice weights normalised to unit DC gain
        double dc = 0.0;
        for (int k = 0; k < K; ++k) {
            b.r[k] = b.p[k];
            b.w[k] = b.c[k] - (k + 1 < K ? b.c[k + 1] : 0.0);
            dc += b.w[k] * (2.0 * b.r[k] + 1.0);
        }
        if (!(dc > 0.0)) return set_error(RSG_EUNSUPPORTED, "rsg_fit_boxes: degenerate kernel");
        for (int k = 0; k < K; ++k) {
            b.w[k] /= dc;
            b.w32[k] = float(b.w[k]);
        }
        quantize_u8(b);
        *out = b;
        return RSG_OK;
    }

    sigma0_fit(K, method == RSG_FIT_SCALED, b.p, b.c, &b.fit_err);

    // Eq. scale1 / scale2, then unit DC gain
    double dc = 0.0;
    for (int k = 0; k < K; ++k) {
        const double slice = b.c[k] - (k + 1 < K ? b.c[k + 1] : 0.0);
        const double rk = std::floor(sigma * double(b.p[k]) / kSigma0Value + 1e-9);
        if (rk > 1.0e8) return set_error(RSG_EUNSUPPORTED, "rsg_fit_boxes: sigma too large");
        b.r[k] = int32_t(rk);
        b.w[k] = slice * double(b.p[k]) / (2.0 * b.r[k] + 1.0);
        dc += b.w[k] * (2.0 * b.r[k] + 1.0);
    }
    if (!(dc > 0.0)) return set_error(RSG_EUNSUPPORTED, "rsg_fit_boxes: degenerate kernel");
    for (int k = 0; k < K; ++k) {
        b.w[k] /= dc;
        b.w32[k] = float(b.w[k]);
    }
    quantize_u8(b);
    *out = b;
    return RSG_OK;
}

}  // namespace rsg
