// ldref.cpp -- CPU oracle for the per-frame hot path of the stereo lane detector of
// Fan & Dahnoun, "Real-Time Stereo Vision-Based Lane Detection System" (arXiv 1807.02752).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct reference that
// the GPU library is checked against.  Only the tests, the smoke check and the benchmark's
// CPU-baseline leg may load it; the product path never calls it and shares no code with it
// (no headers, helpers, tables or constants).  Build: g++ -std=c++17 -O2 -ffp-contract=off.
//
// Conventions: u = column 0..W-1, v = row 0..H-1, v_max = H-1.  All decision arithmetic is
// FP64 in the order written, with no contraction; std::fma appears only where written.
// Where the paper is silent, garbled or self-contradictory, the reading taken is named
// at the function (R1..R19 in the design notes).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

typedef __int128 i128;
typedef unsigned __int128 u128;

namespace {

// ------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
// 3", SC'11): ten rounds of two 64x64->128 multiplications with Weyl-sequence key bumps.
// Written from the published definition.
void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        u128 p0 = (u128)M0 * c0;
        u128 p1 = (u128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Exact integer -> double conversion used for the fit moments (R6): the magnitude is split
// into its two 64-bit halves, each converted, then recombined.
double i128_to_double(i128 v) {
    bool neg = v < 0;
    u128 a = neg ? (u128)(-v) : (u128)v;
    uint64_t hi = (uint64_t)(a >> 64), lo = (uint64_t)a;
    double d = (double)hi * 18446744073709551616.0 + (double)lo;
    return neg ? -d : d;
}

}  // namespace

extern "C" {

// Parameters of the method.  Defaults are the constants printed in the paper plus the
// readings for the silent ones.
struct ldref_params {
    int32_t chi;          // band half-height (Sec. 2.3.2): 25
    int32_t tau_y_max;    // v-disparity DP jump bound (Eq. vpy_estimation): 6
    int32_t tau_x_max;    // V_px DP jump bound (Eq. dense_vpx_estimation): 5
    int32_t lambda_y;     // DP smoothness weights (silent; R2, R12): 1
    int32_t lambda_x;
    double tr_y;          // RANSAC inlier tolerances (Sec. 2.2, 2.3.3): 4, 16
    double tr_x;
    int32_t eps_num;      // RANSAC exit fraction eps = 99/100 (Sec. 2.2, 2.3.3)
    int32_t eps_den;
    double varpi;         // road tolerance (Sec. 2.3.1): 3
    int32_t edge_t;       // Sobel magnitude threshold (Fig. 5 caption): 100
    double sigma_g;       // w_g width (Eq. sigma_g): 3.5
    int32_t nu;           // M_0 box half-sizes (Sec. 2.4): 1 (columns), 3 (rows)
    int32_t varsigma;
    int32_t n_hyp;        // RANSAC hypotheses per round (silent; R4): 64
    int32_t max_rounds;   // RANSAC round cap (silent; R4): 16
    double rho_lpv;       // lane threshold as a fraction of the deepest minimum (R18): 0.25
    int32_t d_nms;        // minimum lane separation, 0 -> max(8, W/64) (R18)
    int32_t weight_squared;  // 0: exponent as printed, 1: squared (Gaussian) reading (R15)
    int32_t vote;         // 0: q = G_x w_g (Sec. 2.4); 1: the prior work's vote (Sec. 2.4 opening)
    uint64_t seed;        // Philox key word 0 (R5)
};

void ldref_params_default(ldref_params* p) {
    p->chi = 25; p->tau_y_max = 6; p->tau_x_max = 5; p->lambda_y = 1; p->lambda_x = 1;
    p->tr_y = 4.0; p->tr_x = 16.0; p->eps_num = 99; p->eps_den = 100; p->varpi = 3.0;
    p->edge_t = 100; p->sigma_g = 3.5; p->nu = 1; p->varsigma = 3; p->n_hyp = 64;
    p->max_rounds = 16; p->rho_lpv = 0.25; p->d_nms = 0; p->weight_squared = 0; p->vote = 0; p->seed = 0;
}

void ldref_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    philox4x64_10(ctr, key, out);
}

// ------------------------------------------------------------------------------------
// O1 -- v-disparity histogram (Sec. 2.2: histogram of every image row of the disparity
// map).  R1: a pixel is valid iff its raw value is non-zero (the LRC check of Sec. 2.1.3
// writes 0 for rejected pixels); float values must also be finite and positive.
// D = raw (u8, f32) or raw/16 (u16 in 1/16 px); bin = min(d_max, floor(D + 0.5)).
static bool disparity_at(const void* disp, int64_t pitch, int fmt, int u, int v, double* D) {
    const uint8_t* row = (const uint8_t*)disp + (int64_t)v * pitch;
    if (fmt == 0) {
        uint8_t r = row[u];
        if (r == 0) return false;
        *D = (double)r;
        return true;
    } else if (fmt == 1) {
        float r;
        std::memcpy(&r, row + 4 * (int64_t)u, 4);
        if (!(std::isfinite(r) && r > 0.0f)) return false;
        *D = (double)r;
        return true;
    } else {
        uint16_t r;
        std::memcpy(&r, row + 2 * (int64_t)u, 2);
        if (r == 0) return false;
        *D = (double)r / 16.0;
        return true;
    }
}

static int disparity_bin(double D, int d_max) {
    double b = std::floor(D + 0.5);
    if (b > (double)d_max) return d_max;
    return (int)b;
}

int ldref_vdisp_hist(const void* disp, int64_t pitch, int W, int H, int fmt, int d_max,
                     int32_t* m_y /* H x (d_max+1) */) {
    std::memset(m_y, 0, sizeof(int32_t) * (size_t)H * (d_max + 1));
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            double D;
            if (!disparity_at(disp, pitch, fmt, u, v, &D)) continue;
            m_y[(int64_t)v * (d_max + 1) + disparity_bin(D, d_max)] += 1;
        }
    return 0;
}

// ------------------------------------------------------------------------------------
// O2 -- DP on the v-disparity map (Eq. energy_function, Eq. vpy_estimation).
// E_{d_max}(v) = -m_y(d_max, v); for d = d_max-1 .. 0:
//   E_d(v) = -m_y(d, v) + min_{0<=tau<=tau_max, v+tau<=v_max} [E_{d+1}(v+tau) + lambda*tau]
// R2: the road disparity grows towards the image bottom, so the row that carries d+1 lies
// at or below the row of d (v+tau), and the jump is penalised (lambda >= 0).
// Ties: smallest tau; start row v* = argmin E_0, smallest v.  The backtrace buffer has the
// size of the v-disparity map.  R3: path points without votes are dropped.
int ldref_vdisp_dp(const int32_t* m_y, int H, int d_max, int tau_max, int lambda,
                   int32_t* path_v /* d_max+1: row of every d */,
                   int32_t* pts_x /* v */, int32_t* pts_y /* d */, int32_t* n_pts) {
    const int D1 = d_max + 1;
    std::vector<int64_t> E(H), En(H);
    std::vector<int8_t> back((size_t)D1 * H, 0);
    for (int v = 0; v < H; ++v) E[v] = -(int64_t)m_y[(int64_t)v * D1 + d_max];
    for (int d = d_max - 1; d >= 0; --d) {
        for (int v = 0; v < H; ++v) {
            int64_t best = 0;
            int bt = -1;
            for (int t = 0; t <= tau_max && v + t <= H - 1; ++t) {
                int64_t c = E[v + t] + (int64_t)lambda * t;
                if (bt < 0 || c < best) { best = c; bt = t; }
            }
            En[v] = -(int64_t)m_y[(int64_t)v * D1 + d] + best;
            back[(size_t)d * H + v] = (int8_t)bt;
        }
        std::swap(E, En);
    }
    int vs = 0;
    for (int v = 1; v < H; ++v)
        if (E[v] < E[vs]) vs = v;
    int n = 0, v = vs;
    for (int d = 0; d <= d_max; ++d) {
        if (path_v) path_v[d] = v;
        if (m_y[(int64_t)v * D1 + d] > 0) { pts_x[n] = v; pts_y[n] = d; ++n; }
        if (d < d_max) v += back[(size_t)d * H + v];
    }
    *n_pts = n;
    return 0;
}

// ------------------------------------------------------------------------------------
// O4 -- least squares polynomial fit (Eq. vpy_least_square_fitting for degree 2,
// Eq. vpx_least_square_fitting / vpx_fitting for degree 4).  R6: the paper rescales the
// Vandermonde system by kappa to avoid overflow; the least-squares minimiser does not
// depend on the basis, so the fit is taken in the shifted, power-of-two scaled variable
// s = (x - center) / 2^k.  The normal-equation moments are exact integer sums, converted
// to FP64 and scaled by exact powers of two, then solved by Gaussian elimination without
// pivoting (i < j < l) and back substitution.  Returns 0 on success, 1 if singular.
int ldref_fit(const int32_t* x, const int32_t* y, const int32_t* idx, int n, int degree,
              int32_t center, int32_t kshift, double* coef /* degree+1, s basis */) {
    const int m = degree, nm = m + 1;
    i128 Sw[9] = {0}, Syw[5] = {0};
    for (int jj = 0; jj < n; ++jj) {
        int j = idx ? idx[jj] : jj;
        i128 w = (i128)x[j] - center;
        i128 pw = 1;
        for (int p = 0; p <= 2 * m; ++p) {
            Sw[p] += pw;
            if (p <= m) Syw[p] += pw * (i128)y[j];
            pw *= w;
        }
    }
    double A[5][5], b[5], sc[9];
    for (int p = 0; p <= 2 * m; ++p) sc[p] = std::ldexp(1.0, -kshift * p);
    for (int i = 0; i < nm; ++i) {
        for (int j = 0; j < nm; ++j) A[i][j] = i128_to_double(Sw[i + j]) * sc[i + j];
        b[i] = i128_to_double(Syw[i]) * sc[i];
    }
    for (int i = 0; i < nm; ++i) {
        if (!(A[i][i] > 0.0)) return 1;
        for (int j = i + 1; j < nm; ++j) {
            double f = A[j][i] / A[i][i];
            for (int l = i; l < nm; ++l) A[j][l] = A[j][l] - f * A[i][l];
            b[j] = b[j] - f * b[i];
        }
    }
    for (int i = nm - 1; i >= 0; --i) {
        double s = b[i];
        for (int l = i + 1; l < nm; ++l) s = s - A[i][l] * coef[l];
        coef[i] = s / A[i][i];
    }
    for (int i = 0; i < nm; ++i)
        if (!std::isfinite(coef[i])) return 1;
    return 0;
}

// Model value at integer x: Horner's rule in s = (x - center) * 2^-k.
static double eval_s(const double* coef, int degree, int32_t center, int32_t kshift, int32_t x) {
    double s = (double)(x - center) * std::ldexp(1.0, -kshift);
    double r = coef[degree];
    for (int p = degree - 1; p >= 0; --p) r = r * s + coef[p];
    return r;
}

// Model value of a raw-basis polynomial g(x) = sum g_p x^p (seeds given by a caller).
static double eval_raw(const double* g, int degree, int32_t x) {
    double xv = (double)x;
    double r = g[degree];
    for (int p = degree - 1; p >= 0; --p) r = r * xv + g[p];
    return r;
}

// s-basis coefficients -> raw-basis coefficients (reporting only; not used for decisions):
// the binomial expansion of c_p ((x - center) / 2^k)^p; C(p,q) and (-center)^(p-q) are
// small integers, formed exactly by repeated multiplication.
static void to_raw(const double* c, int degree, int32_t center, int32_t kshift, double* raw) {
    for (int q = 0; q <= degree; ++q) raw[q] = 0.0;
    for (int p = 0; p <= degree; ++p) {
        double cp = c[p] * std::ldexp(1.0, -kshift * p);
        double binom = 1.0;
        for (int q = 0; q <= p; ++q) {
            double pw = 1.0;
            for (int e = 0; e < p - q; ++e) pw = pw * -(double)center;
            double term = cp * binom * pw;
            raw[q] += term;
            binom = binom * (double)(p - q) / (double)(q + 1);
        }
    }
}

struct ldref_fit_out {
    int32_t ok;           // 1 if a model was fitted on the survivors
    int32_t flags;        // bit 0: no consensus (round cap or too few inliers)
    int32_t center, kshift;
    int32_t rounds;       // rounds executed
    int32_t n_survivors;  // points used in the final fit
    double coef[5];       // s-basis coefficients
    double raw[5];        // raw-basis coefficients (x = row index v)
};

// O5 -- one RANSAC sample: `s` distinct indices into a set of n_cur points, from the
// Philox words of counter (frame index, stage<<32 | round, hypothesis, block), block =
// 0, 1, ... (at most 16), key (seed, stream id); word w maps to floor(w * n_cur / 2^64).
// Returns how many distinct indices were drawn (s unless the blocks ran out).
int ldref_sample(int n_cur, int s, uint64_t seed, uint64_t stream_id, int64_t frame_idx, int stage,
                 int round, int hyp, int32_t* pick) {
    const uint64_t key[2] = {seed, stream_id};
    int got = 0;
    for (int blk = 0; blk < 16 && got < s; ++blk) {
        uint64_t ctr[4] = {(uint64_t)frame_idx, ((uint64_t)stage << 32) | (uint64_t)(uint32_t)round,
                           (uint64_t)hyp, (uint64_t)blk};
        uint64_t wds[4];
        philox4x64_10(ctr, key, wds);
        for (int q = 0; q < 4 && got < s; ++q) {
            int32_t ix = (int32_t)(uint64_t)(((u128)wds[q] * (u128)(uint64_t)n_cur) >> 64);
            bool dup = false;
            for (int e = 0; e < got; ++e) dup = dup || (pick[e] == ix);
            if (!dup) pick[got++] = ix;
        }
    }
    return got;
}

// ------------------------------------------------------------------------------------
// O3 + O5 -- RANSAC as in Alg. "beta estimation with the assist of RANSAC" and Alg.
// "gamma estimation with the assist of RANSAC": draw a random sample, fit, count inliers
// (residual^2 < tr), remove the outliers, repeat while the inlier fraction is below eps;
// finally refit on the surviving inliers.  R4: every round scores n_hyp random samples of
// degree+1 points and keeps the best (most inliers, lowest index on ties); a round whose
// best sample has fewer than max(degree+1, ceil(n0/10)) inliers stops the loop without
// removing anything.  R5: samples are drawn with Philox4x64-10, key (seed, stream id),
// counter (frame index, stage<<32 | round, hypothesis, block); each 64-bit word w gives
// index floor(w * n_cur / 2^64); repeated indices are skipped; at most 16 blocks.
// A sample with fewer than degree+1 distinct x is invalid.  Hypothesis 0 is replaced by the
// caller's seed model (raw basis) when one is given (a seed whose first coefficient is NaN
// counts as none).
// trace (nullable): 3 ints per round: best hypothesis, its inlier count, n_cur.
int ldref_ransac(const int32_t* x, const int32_t* y, int n0, int degree, double tr,
                 int n_hyp, int max_rounds, int eps_num, int eps_den, uint64_t seed,
                 uint64_t stream_id, int64_t frame_idx, int stage, const double* seed_raw,
                 ldref_fit_out* out, int32_t* trace) {
    std::memset(out, 0, sizeof(*out));
    const int s = degree + 1;
    if (n0 < s) { out->flags |= 1; return 0; }
    int32_t xmin = x[0], xmax = x[0];
    for (int j = 1; j < n0; ++j) { xmin = std::min(xmin, x[j]); xmax = std::max(xmax, x[j]); }
    const int32_t center = (xmin + xmax) >> 1;
    int32_t wmax = std::max(xmax - center, center - xmin);
    int32_t k = 0;
    while ((1 << k) < wmax) ++k;
    out->center = center; out->kshift = k;

    std::vector<int32_t> cur(n0);
    for (int j = 0; j < n0; ++j) cur[j] = j;
    const int need = std::max(s, (n0 + 9) / 10);
    bool converged = false;
    int r = 0;
    for (; r < max_rounds; ++r) {
        const int n_cur = (int)cur.size();
        int best_h = -1, best_n = -1;
        std::vector<double> best_model(5, 0.0);
        bool best_is_seed = false;
        for (int h = 0; h < n_hyp; ++h) {
            double model[5] = {0, 0, 0, 0, 0};
            bool is_seed = (h == 0 && seed_raw != nullptr && !std::isnan(seed_raw[0]));   // NaN: no seed
            if (is_seed) {
                for (int p = 0; p <= degree; ++p) model[p] = seed_raw[p];
            } else {
                int32_t pick[5];
                int got = ldref_sample(n_cur, s, seed, stream_id, frame_idx, stage, r, h, pick);
                if (got < s) continue;
                int distinct = 0;
                for (int e = 0; e < s; ++e) {
                    bool seen = false;
                    for (int f = 0; f < e; ++f) seen = seen || (x[cur[pick[f]]] == x[cur[pick[e]]]);
                    if (!seen) ++distinct;
                }
                if (distinct < s) continue;
                int32_t sel[5];
                for (int e = 0; e < s; ++e) sel[e] = cur[pick[e]];
                if (ldref_fit(x, y, sel, s, degree, center, k, model) != 0) continue;
            }
            int cnt = 0;
            for (int jj = 0; jj < n_cur; ++jj) {
                int j = cur[jj];
                double fv = is_seed ? eval_raw(model, degree, x[j]) : eval_s(model, degree, center, k, x[j]);
                double res = (double)y[j] - fv;
                if (res * res < tr) ++cnt;
            }
            if (cnt > best_n) {
                best_n = cnt; best_h = h; best_is_seed = is_seed;
                for (int p = 0; p < 5; ++p) best_model[p] = model[p];
            }
        }
        if (trace) { trace[3 * r] = best_h; trace[3 * r + 1] = best_n; trace[3 * r + 2] = n_cur; }
        if (best_h < 0 || best_n < need) { ++r; break; }
        std::vector<int32_t> keep;
        keep.reserve(best_n);
        for (int jj = 0; jj < n_cur; ++jj) {
            int j = cur[jj];
            double fv = best_is_seed ? eval_raw(best_model.data(), degree, x[j])
                                     : eval_s(best_model.data(), degree, center, k, x[j]);
            double res = (double)y[j] - fv;
            if (res * res < tr) keep.push_back(j);
        }
        bool done = (int64_t)eps_den * best_n >= (int64_t)eps_num * n_cur;
        cur.swap(keep);
        if (done) { converged = true; ++r; break; }
    }
    out->rounds = r;
    if (!converged) out->flags |= 1;
    out->n_survivors = (int)cur.size();
    // final refit on the survivors
    int distinct = 0;
    {
        std::vector<int32_t> xs;
        for (int j : cur) xs.push_back(x[j]);
        std::sort(xs.begin(), xs.end());
        for (size_t i = 0; i < xs.size(); ++i)
            if (i == 0 || xs[i] != xs[i - 1]) ++distinct;
    }
    if (distinct < s) return 0;
    if (ldref_fit(x, y, cur.data(), (int)cur.size(), degree, center, k, out->coef) != 0) return 0;
    out->ok = 1;
    to_raw(out->coef, degree, center, k, out->raw);
    return 0;
}

// ------------------------------------------------------------------------------------
// O6 -- road profile tables and road rows.  f(v) from beta; f'(v) = (c1 + 2 c2 s) 2^-k;
// V_py(v) = v - f(v)/f'(v) (Eq. vpy_equation).  R7: the road occupies rows v_h..v_max where
// v_h is the smallest row such that f > 0 and f' > 0 on every row from v_h to v_max (the
// rows strictly below the horizon root f^-1(0) of Sec. 2.3.1).
int ldref_road_tables(const ldref_fit_out* beta, int H, double* f, double* fp, double* vpy,
                      int32_t* v_h) {
    const double sc = std::ldexp(1.0, -beta->kshift);
    for (int v = 0; v < H; ++v) {
        double s = (double)(v - beta->center) * sc;
        double fv = beta->coef[2];
        fv = fv * s + beta->coef[1];
        fv = fv * s + beta->coef[0];
        double t = 2.0 * beta->coef[2];
        double d = (beta->coef[1] + t * s) * sc;
        f[v] = fv;
        fp[v] = d;
        vpy[v] = (double)v - fv / d;
    }
    int v = H - 1;
    while (v >= 0 && f[v] > 0.0 && fp[v] > 0.0) --v;
    *v_h = v + 1;
    return 0;
}

// ------------------------------------------------------------------------------------
// O7 -- Sobel gradient (Sec. 2.3.1).  R9: the raw grey image is differentiated (the
// bilateral pre-filter is a separate step).  G_x = d/du with weights (1,2,1) across rows,
// positive on a dark-to-light transition (Sec. 2.4); G_y = d/dv.  Border pixels are 0.
int ldref_sobel(const uint8_t* grey, int64_t pitch, int W, int H, int32_t* gx, int32_t* gy) {
    auto I = [&](int u, int v) { return (int32_t)grey[(int64_t)v * pitch + u]; };
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int32_t a = 0, b = 0;
            if (u >= 1 && u <= W - 2 && v >= 1 && v <= H - 2) {
                const int s[3] = {1, 2, 1};
                for (int t = -1; t <= 1; ++t) {
                    a += s[t + 1] * (I(u + 1, v + t) - I(u - 1, v + t));
                    b += s[t + 1] * (I(u + t, v + 1) - I(u + t, v - 1));
                }
            }
            gx[(int64_t)v * W + u] = a;
            gy[(int64_t)v * W + u] = b;
        }
    return 0;
}

// ------------------------------------------------------------------------------------
// Stereo disparity (Sec. 2.1): NCC block matching with the block statistics memorised from
// integral images (Alg. "integral image initialisation", Eq. integral_image, Eq. sigma_l_1,
// Eq. sigma_r_1, Eq. ncc_1), search range propagation row by row from the bottom (Eq. srp,
// Alg. "SRP-based disparity map estimation") and the left-right consistency check (Alg. "LRC
// check").  Readings (D1..D6):
// D1: block side 2 rho + 1, n = (2 rho + 1)^2; a pixel is matched only when its block lies in
//     the image (rho <= u <= W-1-rho, rho <= v <= H-1-rho), others get 0.  Disparity 0 marks
//     "no match" (the value the check writes), so the search range is 1..d_max.
// D2: with S = block sum, Q = block sum of squares (from the integral images) and
//     P = sum of I_l(i,j) I_r(i-d,j), the cost of Eq. ncc_1 equals
//     c = (n P - S_l S_r) / (sqrt(n Q_l - S_l^2) sqrt(n Q_r - S_r^2)); the integers are exact,
//     the quotient is FP64 in this order.  A block with n Q - S^2 = 0 (flat) is not scored.
// D3: the disparity is the scored candidate of largest c, ties to the smaller d; none -> 0.
//     A candidate is admissible when the other block lies in the image.
// D4: the bottom matched row searches 1..d_max; row v searches the union over the matched
//     columns k = u-1..u+1 of [l(k,v+1) - tau, l(k,v+1) + tau] clipped to 1..d_max, over the
//     neighbours with l(k,v+1) > 0; with none of them, 1..d_max again.
// D5: the right map is estimated the same way with the roles swapped (right block at x, left
//     block at x + d), its own propagation, the same statistics.
// D6: l(u,v) = l_lf(u,v) unless l_lf(u,v) = 0, u - l_lf(u,v) < 0, or
//     |l_lf(u,v) - l_rt(u - l_lf(u,v), v)| > tr, in which case 0.
namespace {
struct StereoStats {
    int W = 0, H = 0, rho = 0, n = 0;
    std::vector<int64_t> S, Q;   // block sums at every matchable centre (0 elsewhere)
};

// Alg. "integral image initialisation" for I and I^2, then the four-reference block sums.
StereoStats stereo_stats(const uint8_t* img, int64_t pitch, int W, int H, int rho) {
    StereoStats st;
    st.W = W; st.H = H; st.rho = rho; st.n = (2 * rho + 1) * (2 * rho + 1);
    std::vector<int64_t> In((size_t)W * H), In2((size_t)W * H);
    auto I = [&](int u, int v) { return (int64_t)img[(int64_t)v * pitch + u]; };
    auto at = [&](std::vector<int64_t>& a, int u, int v) -> int64_t& { return a[(size_t)v * W + u]; };
    at(In, 0, 0) = I(0, 0);
    at(In2, 0, 0) = I(0, 0) * I(0, 0);
    for (int u = 1; u < W; ++u) {
        at(In, u, 0) = at(In, u - 1, 0) + I(u, 0);
        at(In2, u, 0) = at(In2, u - 1, 0) + I(u, 0) * I(u, 0);
    }
    for (int v = 1; v < H; ++v) {
        at(In, 0, v) = at(In, 0, v - 1) + I(0, v);
        at(In2, 0, v) = at(In2, 0, v - 1) + I(0, v) * I(0, v);
    }
    for (int u = 1; u < W; ++u)
        for (int v = 1; v < H; ++v) {
            at(In, u, v) = at(In, u, v - 1) + at(In, u - 1, v) - at(In, u - 1, v - 1) + I(u, v);
            at(In2, u, v) = at(In2, u, v - 1) + at(In2, u - 1, v) - at(In2, u - 1, v - 1) + I(u, v) * I(u, v);
        }
    // r1 = In(u+rho, v+rho), r2 = In(u-rho-1, v-rho-1), r3 = In(u-rho-1, v+rho), r4 = In(u+rho, v-rho-1),
    // a reference left of column 0 or above row 0 being 0
    auto ref = [&](std::vector<int64_t>& a, int u, int v) -> int64_t { return (u < 0 || v < 0) ? 0 : at(a, u, v); };
    st.S.assign((size_t)W * H, 0);
    st.Q.assign((size_t)W * H, 0);
    for (int v = rho; v <= H - 1 - rho; ++v)
        for (int u = rho; u <= W - 1 - rho; ++u) {
            st.S[(size_t)v * W + u] = ref(In, u + rho, v + rho) + ref(In, u - rho - 1, v - rho - 1) -
                                      ref(In, u - rho - 1, v + rho) - ref(In, u + rho, v - rho - 1);
            st.Q[(size_t)v * W + u] = ref(In2, u + rho, v + rho) + ref(In2, u - rho - 1, v - rho - 1) -
                                      ref(In2, u - rho - 1, v + rho) - ref(In2, u + rho, v - rho - 1);
        }
    return st;
}

// One disparity map by SRP.  ref_left = 1: blocks of `a` at u matched against `b` at u - d
// (the left map); 0: `a` at x against `b` at x + d (the right map).
void stereo_srp(const uint8_t* a, const uint8_t* b, int64_t pitch, const StereoStats& sa, const StereoStats& sb,
                int d_max, int tau, int ref_left, uint8_t* out, double* cost_out) {
    const int W = sa.W, H = sa.H, rho = sa.rho, n = sa.n;
    auto A = [&](int u, int v) { return (int64_t)a[(int64_t)v * pitch + u]; };
    auto B = [&](int u, int v) { return (int64_t)b[(int64_t)v * pitch + u]; };
    for (int64_t i = 0; i < (int64_t)W * H; ++i) out[i] = 0;
    std::vector<uint8_t> scan(d_max + 2);
    for (int v = H - 1 - rho; v >= rho; --v) {
        for (int u = rho; u <= W - 1 - rho; ++u) {
            // D4: the search range
            std::fill(scan.begin(), scan.end(), 0);
            bool any = false;
            if (v < H - 1 - rho) {
                for (int k = u - 1; k <= u + 1; ++k) {
                    if (k < rho || k > W - 1 - rho) continue;
                    const int l = out[(int64_t)(v + 1) * W + k];
                    if (l <= 0) continue;
                    any = true;
                    for (int d = l - tau; d <= l + tau; ++d)
                        if (d >= 1 && d <= d_max) scan[d] = 1;
                }
            }
            if (!any)
                for (int d = 1; d <= d_max; ++d) scan[d] = 1;
            const int64_t Sa = sa.S[(size_t)v * W + u], Qa = sa.Q[(size_t)v * W + u];
            const int64_t Va = (int64_t)n * Qa - Sa * Sa;
            int best = 0;
            double bc = 0.0;
            if (Va > 0) {
                for (int d = 1; d <= d_max; ++d) {
                    if (!scan[d]) continue;
                    const int x = ref_left ? u - d : u + d;          // centre of the other block
                    if (x < rho || x > W - 1 - rho) continue;
                    const int64_t Sb = sb.S[(size_t)v * W + x], Qb = sb.Q[(size_t)v * W + x];
                    const int64_t Vb = (int64_t)n * Qb - Sb * Sb;
                    if (Vb <= 0) continue;
                    int64_t P = 0;
                    for (int j = v - rho; j <= v + rho; ++j)
                        for (int i = -rho; i <= rho; ++i) P += A(u + i, j) * B(x + i, j);
                    const double c = (double)((int64_t)n * P - Sa * Sb) / (std::sqrt((double)Va) * std::sqrt((double)Vb));
                    if (best == 0 || c > bc) { best = d; bc = c; }
                }
            }
            out[(int64_t)v * W + u] = (uint8_t)best;
            if (cost_out) cost_out[(int64_t)v * W + u] = best ? bc : 0.0;
        }
    }
}
}  // namespace

int ldref_stereo(const uint8_t* left, const uint8_t* right, int64_t pitch, int W, int H, int rho, int d_max, int tau,
                 int tr_lrc, uint8_t* disp_lf, uint8_t* disp_rt, uint8_t* disp, double* cost_lf) {
    if (rho < 1 || rho > 7 || d_max < 1 || d_max > 255 || tau < 0 || tr_lrc < 0 || W < 2 * rho + 1 || H < 2 * rho + 1)
        return -1;
    const StereoStats sl = stereo_stats(left, pitch, W, H, rho), sr = stereo_stats(right, pitch, W, H, rho);
    std::vector<uint8_t> lf((size_t)W * H), rt((size_t)W * H);
    stereo_srp(left, right, pitch, sl, sr, d_max, tau, 1, lf.data(), cost_lf);
    stereo_srp(right, left, pitch, sr, sl, d_max, tau, 0, rt.data(), nullptr);
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            const int l = lf[(size_t)v * W + u];
            int o = 0;
            if (l > 0 && u - l >= 0 && std::abs(l - (int)rt[(size_t)v * W + (u - l)]) <= tr_lrc) o = l;
            disp[(size_t)v * W + u] = (uint8_t)o;
        }
    if (disp_lf) std::memcpy(disp_lf, lf.data(), lf.size());
    if (disp_rt) std::memcpy(disp_rt, rt.data(), rt.size());
    return 0;
}

// The block statistics alone (pinned separately): S and Q at every matchable centre.
int ldref_stereo_stats(const uint8_t* img, int64_t pitch, int W, int H, int rho, int64_t* S, int64_t* Q) {
    if (rho < 1 || W < 2 * rho + 1 || H < 2 * rho + 1) return -1;
    const StereoStats st = stereo_stats(img, pitch, W, H, rho);
    std::memcpy(S, st.S.data(), sizeof(int64_t) * st.S.size());
    std::memcpy(Q, st.Q.data(), sizeof(int64_t) * st.Q.size());
    return 0;
}

// ------------------------------------------------------------------------------------
// Lane tracking across frames.  The paper names a tracking algorithm as future work (Sec. 4)
// without defining one; this is the reading taken (T1..T5).  T1: a track is a lane's start
// column x on row v_max with a rate dx in columns per frame; a frame first predicts every
// track, x_hat = x + dx.  T2: a frame without a road or a vanishing point has no detections.
// T3: detections are assigned to predicted tracks greedily, the closest pair |u - x_hat| first
// (ties to the lower track slot, then the lower detection index), only pairs within `gate`.
// T4: an alpha-beta filter updates a matched track, r = u - x_hat, x = x_hat + alpha r,
// dx = dx + beta r, hits + 1, misses = 0; an unmatched track keeps x = x_hat and counts a miss,
// and is dropped once misses > max_misses (the others keep their order).  T5: unmatched
// detections, in their order, start tracks (x = u, dx = 0, hits = 1) with consecutive ids
// while fewer than 16 tracks live.  A track with hits >= confirm is reported.  FP64, in the
// order written.
struct ldref_track {
    int32_t n, next_id;
    int64_t frames;
    int32_t id[16], hits[16], misses[16];
    double x[16], dx[16];
};

int ldref_track_update(ldref_track* s, const int32_t* u, int n_det, int valid, double alpha, double beta,
                       double gate, int max_misses) {
    if (!valid) n_det = 0;
    if (n_det > 16) n_det = 16;
    double xh[16];
    for (int t = 0; t < s->n; ++t) xh[t] = s->x[t] + s->dx[t];
    int match_t[16], match_d[16];
    for (int t = 0; t < 16; ++t) match_t[t] = -1;
    for (int d = 0; d < 16; ++d) match_d[d] = -1;
    for (;;) {
        int bt = -1, bd = -1;
        double best = 0.0;
        for (int t = 0; t < s->n; ++t) {
            if (match_t[t] >= 0) continue;
            for (int d = 0; d < n_det; ++d) {
                if (match_d[d] >= 0) continue;
                const double dist = std::fabs((double)u[d] - xh[t]);
                if (!(dist <= gate)) continue;
                if (bt < 0 || dist < best) { bt = t; bd = d; best = dist; }
            }
        }
        if (bt < 0) break;
        match_t[bt] = bd;
        match_d[bd] = bt;
    }
    for (int t = 0; t < s->n; ++t) {
        if (match_t[t] >= 0) {
            const double r = (double)u[match_t[t]] - xh[t];
            s->x[t] = xh[t] + alpha * r;
            s->dx[t] = s->dx[t] + beta * r;
            s->hits[t] += 1;
            s->misses[t] = 0;
        } else {
            s->x[t] = xh[t];
            s->misses[t] += 1;
        }
    }
    int k = 0;
    for (int t = 0; t < s->n; ++t) {
        if (s->misses[t] > max_misses) continue;
        s->id[k] = s->id[t]; s->hits[k] = s->hits[t]; s->misses[k] = s->misses[t];
        s->x[k] = s->x[t]; s->dx[k] = s->dx[t];
        ++k;
    }
    s->n = k;
    for (int d = 0; d < n_det; ++d) {
        if (match_d[d] >= 0 || s->n >= 16) continue;
        const int t = s->n++;
        s->id[t] = s->next_id++;
        s->hits[t] = 1;
        s->misses[t] = 0;
        s->x[t] = (double)u[d];
        s->dx[t] = 0.0;
    }
    s->frames += 1;
    return s->n;
}

// ------------------------------------------------------------------------------------
// Bilateral pre-filter (Sec. 2.3.1, Eq. bilateral_filter and the two weights defined after
// it): I_bf(u, v) = sum w_s w_r I / sum w_s w_r over the (2 rho + 1) x (2 rho + 1) window
// centred at (u, v), w_s = exp(-((i-u)^2 + (j-v)^2) / sigma_s^2) on the offset and
// w_r = exp(-(I(i,j) - I(u,v))^2 / sigma_r^2) on intensities scaled to [0, 1].
// Readings (B1..B4): window pixels outside the frame take part in neither sum (B1); sigma_s and
// sigma_r are single-precision numbers, and both weights are single-precision tables -- w_s per
// window offset, w_r per absolute grey difference 0..255 -- each the double-precision
// exponential rounded to float (B2); the sums run in single precision over the window row by
// row (j), left to right (i), the numerator accumulated by a fused multiply-add of the product
// weight with the intensity (B3); the output is the single-precision quotient rounded half up
// to u8, so the gradient after it stays integer (B4).  Rows v < row0 are not written; val
// (nullable, W x H) receives the quotients of the rows written.
int ldref_bilateral(const uint8_t* grey, int64_t pitch, int W, int H, int rho, float sigma_s, float sigma_r,
                    int row0, uint8_t* out, int64_t opitch, float* val) {
    if (rho < 1 || rho > 5 || !(sigma_s > 0.0f) || !(sigma_r > 0.0f)) return -1;
    const int n = 2 * rho + 1;
    const double ss = (double)sigma_s, sr = (double)sigma_r;
    std::vector<float> ws((size_t)n * n);
    for (int dy = -rho; dy <= rho; ++dy)
        for (int dx = -rho; dx <= rho; ++dx)
            ws[(size_t)(dy + rho) * n + (dx + rho)] = (float)std::exp(-(double)(dx * dx + dy * dy) / (ss * ss));
    float wr[256];
    for (int d = 0; d < 256; ++d) {
        const double x = (double)d / 255.0;
        wr[d] = (float)std::exp(-(x * x) / (sr * sr));
    }
    for (int v = std::max(row0, 0); v < H; ++v)
        for (int u = 0; u < W; ++u) {
            const int c = grey[(int64_t)v * pitch + u];
            float num = 0.0f, den = 0.0f;
            for (int j = v - rho; j <= v + rho; ++j)
                for (int i = u - rho; i <= u + rho; ++i) {
                    if (i < 0 || i >= W || j < 0 || j >= H) continue;
                    const int I = grey[(int64_t)j * pitch + i];
                    const float w = ws[(size_t)(j - v + rho) * n + (i - u + rho)] * wr[std::abs(I - c)];
                    num = std::fma(w, (float)I, num);
                    den = den + w;
                }
            const float q = num / den;
            if (val) val[(int64_t)v * W + u] = q;
            out[(int64_t)v * opitch + u] = (uint8_t)std::floor(q + 0.5f);
        }
    return 0;
}

// ------------------------------------------------------------------------------------
// Road mask + edges (Sec. 2.3.1): a pixel is on the road iff it is valid, lies on a road row
// v_h <= v <= v_max and |D - f(v)| <= varpi; a road pixel is an edge iff
// G_x^2 + G_y^2 > edge_t^2 (the magnitude read as Euclidean).  Edges are listed row-major.
// Returns the number of edges (written up to cap).
int ldref_road_edges(const uint8_t* grey, int64_t gpitch, const void* disp, int64_t dpitch, int W, int H,
                     int fmt, const double* f, int v_h, double varpi, int edge_t, int32_t* eu, int32_t* ev,
                     int32_t* egx, int32_t* egy, int cap) {
    std::vector<int32_t> gx((size_t)H * W), gy((size_t)H * W);
    ldref_sobel(grey, gpitch, W, H, gx.data(), gy.data());
    const int64_t t2 = (int64_t)edge_t * edge_t;
    int n = 0;
    for (int v = v_h; v <= H - 1; ++v)
        for (int u = 0; u < W; ++u) {
            double D;
            if (!disparity_at(disp, dpitch, fmt, u, v, &D)) continue;
            if (!(std::fabs(D - f[v]) <= varpi)) continue;
            int32_t a = gx[(int64_t)v * W + u], b = gy[(int64_t)v * W + u];
            if ((int64_t)a * a + (int64_t)b * b <= t2) continue;
            if (n < cap) { eu[n] = u; ev[n] = v; egx[n] = a; egy[n] = b; }
            ++n;
        }
    return n;
}

// O8 -- sparse V_px votes, Eq. sparse_vpx_estimation with the gradient read as the edge
// slope (R10): the edge tangent through (u, v) meets row V_py(v) at
//   x = u + (v - V_py(v)) * G_y / G_x.
// Vote column c = floor(x + 0.5) + floor(W/2), kept if 0 <= c < 2W (candidate columns run
// from -W/2 to 1.5 W, xi = 0.5 of Sec. 2.4); G_x = 0 casts no vote (-1).
int ldref_votes(const int32_t* eu, const int32_t* ev, const int32_t* egx, const int32_t* egy, int n,
                const double* vpy, int W, int32_t* bin) {
    const int W2 = 2 * W, half = W / 2;
    int kept = 0;
    for (int i = 0; i < n; ++i) {
        bin[i] = -1;
        if (egx[i] == 0) continue;
        double t = (double)ev[i] - vpy[ev[i]];
        double xv = (double)eu[i] + (t * (double)egy[i]) / (double)egx[i];
        double b = std::floor(xv + 0.5);
        if (b >= -(double)half && b < (double)(W2 - half)) { bin[i] = (int32_t)b + half; ++kept; }
    }
    return kept;
}

// O9 -- dense V_px accumulator (Alg. "Dense V_px accumulation", Sec. 2.3.2).  R11: the band
// is 2 chi + 1 rows centred on v, clipped to the road rows (the thinner top bands of the
// prose), each vote counting -varrho = -1:
//   m_x(c, v) = - sum_{v' = max(v - chi, v_h)}^{min(v + chi, v_max)} h(c, v').
// h is H x 2W vote counts; m_x is H x 2W (rows outside v_h..v_max untouched).
int ldref_band(const int32_t* h, int H, int W2, int v_h, int chi, int64_t* mx) {
    for (int v = v_h; v <= H - 1; ++v) {
        int lo = std::max(v - chi, v_h), hi = std::min(v + chi, H - 1);
        for (int c = 0; c < W2; ++c) {
            int64_t acc = 0;
            for (int vv = lo; vv <= hi; ++vv) acc += h[(size_t)vv * W2 + c];
            mx[(size_t)v * W2 + c] = -acc;
        }
    }
    return 0;
}

// O10 -- DP on the accumulator (Eq. dense_vpx_estimation), rows v_max -> v_h:
//   E_{v_max}(c) = m_x(c, v_max)
//   E_v(c) = m_x(c, v) + min_{|tau| <= tau_max, 0 <= c+tau < 2W} [E_{v+1}(c + tau) + lambda |tau|]
// R12: the smoothness term is read as lambda |tau|; ties go to the first strict minimum in
// the scan order tau = 0, -1, +1, -2, +2, ...; the start column is argmin E_{v_h} (smallest
// c); the backtrace runs down to v_max.  cpath[v] = c_v for v_h <= v <= v_max.
int ldref_row_dp(const int64_t* mx, int H, int W2, int v_h, int tau_max, int lambda, int32_t* cpath) {
    const int v_max = H - 1, R = v_max - v_h + 1;
    std::vector<int64_t> E(W2), En(W2);
    std::vector<int8_t> back((size_t)R * W2, 0);
    for (int c = 0; c < W2; ++c) E[c] = mx[(size_t)v_max * W2 + c];
    for (int v = v_max - 1; v >= v_h; --v) {
        for (int c = 0; c < W2; ++c) {
            int64_t best = E[c];
            int bt = 0;
            for (int a = 1; a <= tau_max; ++a)
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    int t = sgn * a, cc = c + t;
                    if (cc < 0 || cc >= W2) continue;
                    int64_t val = E[cc] + (int64_t)lambda * a;
                    if (val < best) { best = val; bt = t; }
                }
            En[c] = mx[(size_t)v * W2 + c] + best;
            back[(size_t)(v - v_h) * W2 + c] = (int8_t)bt;
        }
        std::swap(E, En);
    }
    int c = 0;
    for (int cc = 1; cc < W2; ++cc)
        if (E[cc] < E[c]) c = cc;
    for (int v = v_h; v <= v_max; ++v) {
        cpath[v] = c;
        if (v < v_max) c += back[(size_t)(v - v_h) * W2 + c];
    }
    return 0;
}

// O12 -- piecewise weight w_g (Eq. sigma_g).  R14: theta_e is the orientation of the edge
// line (tangent t = (-G_y, G_x)) and theta_Vp that of the ray r from the pixel to V_p(v);
// the angle between the two lines, delta, lies in [0, pi/2].  The gate delta <= pi/6 is the
// exact test dot^2 >= (3/4) |t|^2 |r|^2 (cos^2(pi/6) = 3/4).  R15: w_g = exp(-p / sigma_g^2)
// with p = delta / theta_s, theta_s = pi/36, as printed (squared = 1: exp(-p^2 / sigma_g^2)).
// q = G_x * w_g per edge.  Returns the number of edges that pass the gate.
// vote = 1 (A/B variant): the vote of the authors' prior work named at the opening of Sec. 2.4,
// V(e) = |grad(e)| cos(theta_e - theta_Vp), in place of G_x w_g.  R20: theta_e is the direction
// of the tangent t = (-G_y, G_x) (the gradient turned by +90 degrees, so the two edges of a
// marking point opposite ways) and theta_Vp the direction of the ray from V_p(v) to the pixel,
// p - V_p = -r; then V(e) = t . (-r) / |r| = -dot / |r|, no gate, 0 at V_p itself.  On a lane
// edge V(e) has the sign of G_x, so the box, M_1, the energies and the minima that follow are
// the paper's, with the vote swapped.  Returns n.
int ldref_weights(const int32_t* eu, const int32_t* ev, const int32_t* egx, const int32_t* egy, int n,
                  const double* vpx, const double* vpy, double sigma_g, int squared, double* q, int vote) {
    const double pi = 3.14159265358979323846;
    const double theta_s = pi / 36.0;
    const double sg2 = sigma_g * sigma_g;
    int kept = 0;
    for (int i = 0; i < n; ++i) {
        double tx = (double)(-egy[i]), ty = (double)egx[i];
        double rx = vpx[ev[i]] - (double)eu[i], ry = vpy[ev[i]] - (double)ev[i];
        double dot = tx * rx + ty * ry;
        double tt = tx * tx + ty * ty;
        double rr = rx * rx + ry * ry;
        if (vote) {
            q[i] = rr > 0.0 ? -dot / std::sqrt(rr) : 0.0;
            ++kept;
            continue;
        }
        double w = 0.0;
        if (dot * dot >= (0.75 * tt) * rr) {
            double cr = tx * ry - ty * rx;
            double delta = std::atan2(std::fabs(cr), std::fabs(dot));
            double pp = delta / theta_s;
            w = squared ? std::exp(-(pp * pp) / sg2) : std::exp(-pp / sg2);
            ++kept;
        }
        q[i] = (double)egx[i] * w;
    }
    return kept;
}

// O13 -- M_0 = sum of G_x w_g over a box of (2 nu + 1) columns x (2 varsigma + 1) rows
// (Alg. "Lane position validation"); M_1 = G * M_0 with the Sobel kernel
// G = [1,2,1]^T [1,0,-1] (R16: a true convolution, so M_1(u,v) =
// sum_y s_y (M_0(u+1, v+y) - M_0(u-1, v+y)), negative at the centre of a bright marking).
// Everything outside the image is zero.  q, m0, m1: H x W.
int ldref_m0m1(const double* q, int W, int H, int nu, int varsigma, double* m0, double* m1) {
    auto Q = [&](int u, int v) { return (u < 0 || u >= W || v < 0 || v >= H) ? 0.0 : q[(size_t)v * W + u]; };
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            double acc = 0.0;
            for (int xo = -nu; xo <= nu; ++xo)
                for (int yo = -varsigma; yo <= varsigma; ++yo) acc += Q(u + xo, v + yo);
            m0[(size_t)v * W + u] = acc;
        }
    auto M0 = [&](int u, int v) { return (u < 0 || u >= W || v < 0 || v >= H) ? 0.0 : m0[(size_t)v * W + u]; };
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            const double s[3] = {1.0, 2.0, 1.0};
            double acc = 0.0;
            for (int yo = -1; yo <= 1; ++yo) acc += s[yo + 1] * (M0(u + 1, v + yo) - M0(u - 1, v + yo));
            m1[(size_t)v * W + u] = acc;
        }
    return 0;
}

// O14 -- energy of every candidate (Eq. lane_energy, lambda_g = 1) along the track of
// Eq. lane_visualisation, which is the line through (u_{v+1}, v+1) and V_p(v+1) taken at
// row v:  u_v = B_v u_{v+1} + A_v,  A_v = V_px(v+1) / den,  B_v = (v - V_py(v+1)) / den,
// den = v + 1 - V_py(v+1).  R17: candidate i starts at u = i - floor(W/2) on row v_max
// (i = 0..2W-1, xi = 0.5); the column on row v is floor(u_v + 0.5); off-image columns add
// 0; the track stops on the first row whose den is not positive.
// E[i] = sum_{v = v_max .. v_end} M_1(col_i(v), v).  Returns v_end.
int ldref_energy(const double* m1, const double* vpx, const double* vpy, int W, int H, int v_h,
                 double* E, double* curves_for /* nullable: n_tracks x H */, const int32_t* track_start,
                 int n_tracks) {
    const int v_max = H - 1, W2 = 2 * W, half = W / 2;
    std::vector<double> Av(H, 0.0), Bv(H, 0.0);
    int v_end = v_max;
    for (int v = v_max - 1; v >= v_h; --v) {
        double den = (double)(v + 1) - vpy[v + 1];
        if (!(den > 0.0)) break;
        Av[v] = vpx[v + 1] / den;
        Bv[v] = ((double)v - vpy[v + 1]) / den;
        v_end = v;
    }
    if (E) {
        for (int i = 0; i < W2; ++i) {
            double u = (double)(i - half);
            double e = 0.0;
            for (int v = v_max; v >= v_end; --v) {
                if (v < v_max) u = std::fma(Bv[v], u, Av[v]);
                double xx = u + 0.5;
                if (xx >= 0.0 && xx < (double)W) e += m1[(size_t)v * W + (int)std::floor(xx)];
            }
            E[i] = e;
        }
    }
    if (curves_for) {
        const double nan = std::nan("");
        for (int l = 0; l < n_tracks; ++l) {
            double u = (double)track_start[l];
            for (int v = 0; v < H; ++v) curves_for[(size_t)l * H + v] = nan;
            for (int v = v_max; v >= v_end; --v) {
                if (v < v_max) u = std::fma(Bv[v], u, Av[v]);
                curves_for[(size_t)l * H + v] = u;
            }
        }
    }
    return v_end;
}

// O14 -- peak selection (Alg. "Lane position validation"): strict local minima of the
// energy histogram; R18: keep those below rho times the deepest value (none if that value
// is not negative), then greedily accept by (E ascending, i ascending) a minimum farther
// than d_nms columns from every accepted one, at most 16; report by ascending position.
int ldref_peaks(const double* E, int W2, int half, double rho, int d_nms, int32_t* u_start, double* e_lane) {
    double mn = E[0];
    for (int i = 1; i < W2; ++i) mn = std::min(mn, E[i]);
    std::vector<int> cand;
    if (mn < 0.0) {
        const double thr = rho * mn;
        for (int i = 1; i + 1 < W2; ++i)
            if (E[i] < E[i - 1] && E[i] < E[i + 1] && E[i] < thr) cand.push_back(i);
    }
    std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
        if (E[a] != E[b]) return E[a] < E[b];
        return a < b;
    });
    std::vector<int> acc;
    for (int i : cand) {
        if ((int)acc.size() >= 16) break;
        bool ok = true;
        for (int j : acc) ok = ok && (std::abs(i - j) > d_nms);
        if (ok) acc.push_back(i);
    }
    std::sort(acc.begin(), acc.end());
    for (size_t l = 0; l < acc.size(); ++l) {
        u_start[l] = acc[l] - half;
        e_lane[l] = E[acc[l]];
    }
    return (int)acc.size();
}

// ------------------------------------------------------------------------------------
// Full per-frame path.  Every array pointer in ldref_out is optional (nullable).
struct ldref_out {
    int32_t flags;        // 1 NOROAD, 2 NOVP, 4 no consensus in beta, 8 no consensus in gamma
    int32_t v_h;          // first road row
    int32_t v_end;        // last (top) row reached by the lane tracks
    int32_t n_lanes;
    int32_t n_my;         // points on the v-disparity path
    int32_t n_edges;      // road edge pixels
    int32_t n_votes;      // votes that landed in a column
    int32_t pad0;
    int32_t u_start[16];
    double energy_lane[16];
    ldref_fit_out beta;
    ldref_fit_out gamma;
    int32_t* m_y;          // H x (d_max+1)
    int32_t* my_path_v;    // d_max+1
    int32_t* my_x;         // d_max+1 (points kept)
    int32_t* my_y;
    double* f;             // H
    double* fp;            // H
    double* vpy;           // H
    double* vpx;           // H (NaN off-road)
    int32_t* edge_u;       // capacity edge_cap
    int32_t* edge_v;
    int32_t* edge_gx;
    int32_t* edge_gy;
    int32_t* edge_bin;     // vote column 0..2W-1, or -1
    double* edge_q;        // G_x * w_g
    int32_t edge_cap;
    int32_t pad1;
    int32_t* mx_path;      // H: column c_v (0..2W-1) on road rows, -1 elsewhere
    double* energy;        // 2W
    double* m1;            // H x W
    double* curves;        // 16 x H (NaN outside the track)
    int32_t* trace_beta;   // 3 x max_rounds
    int32_t* trace_gamma;  // 3 x max_rounds
};

// Inputs and outputs of the narrowed search (learned part; the steps are defined with the
// library's ld_detect_pruned, not by the paper).
struct ldref_learned {
    int32_t n_bands, delta_x, dilate, min_votes, seed_ransac, pad;
    const uint8_t* lane_bits;   // 4 x 16 x W decisions of the network, band k at k * 16 * W
    int32_t prune[16];          // out: bands, fallback bits, c_s, lo, hi, votes, est[4], cnt[4], kept, 0
    uint8_t* cand_mask;         // out, nullable: 2W
};

static int band_top(int v_h, int H, int nb, int k) {
    const int R = H - v_h;
    if (R < 16 || nb < 1) return -1;
    return (H - 16) - ((R - 16) * k) / nb;
}

int ldref_band_top(int v_h, int H, int nb, int k) { return band_top(v_h, H, nb, k); }

// Seed of the narrowed search: the vote columns of the road edges that the network marks on
// the band rows, one histogram per band and one pooled.  est[k] is the first column of the
// highest count of band k (-1 with no vote), cnt[k] its number of votes.  Returns the pooled
// argmax c_s (smallest on ties), or -1 when fewer than min_votes votes were pooled.
int ldref_seed(const int32_t* eu, const int32_t* ev, const int32_t* ebin, int ne, const uint8_t* lane_bits,
               int W, int H, int v_h, int nb, int min_votes, int32_t* est, int32_t* cnt, int32_t* total) {
    const int W2 = 2 * W;
    std::vector<int> hp(W2, 0), hb(W2);
    for (int k = 0; k < 4; ++k) { est[k] = -1; cnt[k] = 0; }
    for (int k = 0; k < nb; ++k) {
        const int top = band_top(v_h, H, nb, k);
        if (top < 0) break;
        std::fill(hb.begin(), hb.end(), 0);
        for (int i = 0; i < ne; ++i) {
            const int r = ev[i] - top;
            if (r < 0 || r >= 16 || ebin[i] < 0 || !lane_bits[((size_t)k * 16 + r) * W + eu[i]]) continue;
            hb[ebin[i]] += 1;
            hp[ebin[i]] += 1;
        }
        int tot = 0, best = 0;
        for (int c = 0; c < W2; ++c) { tot += hb[c]; if (hb[c] > hb[best]) best = c; }
        est[k] = tot > 0 ? best : -1;
        cnt[k] = tot;
    }
    int tot = 0, cs = 0;
    for (int c = 0; c < W2; ++c) { tot += hp[c]; if (hp[c] > hp[cs]) cs = c; }
    *total = tot;
    return tot < min_votes ? -1 : cs;
}

// The row DP of ldref_row_dp restricted to the columns lo..hi: the same recursion, tie order
// and backtrace, with every transition that leaves the window removed.  cpath[v] gets the
// column (0..W2-1) on the road rows.  Returns 1 when the path reaches an inner edge of the
// window (column lo with lo > 0, or column hi with hi < W2 - 1), else 0.
int ldref_window_dp(const int64_t* mx, int H, int W2, int v_h, int tau_max, int lambda, int lo, int hi,
                    int32_t* cpath) {
    const int v_max = H - 1, R = v_max - v_h + 1, win = hi - lo + 1;
    std::vector<int64_t> E(win), En(win);
    std::vector<int8_t> back((size_t)R * win, 0);
    for (int c = 0; c < win; ++c) E[c] = mx[(size_t)v_max * W2 + lo + c];
    for (int v = v_max - 1; v >= v_h; --v) {
        for (int c = 0; c < win; ++c) {
            int64_t best = E[c];
            int bt = 0;
            for (int a = 1; a <= tau_max; ++a)
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    const int cc = c + sgn * a;
                    if (cc < 0 || cc >= win) continue;
                    const int64_t val = E[cc] + (int64_t)lambda * a;
                    if (val < best) { best = val; bt = sgn * a; }
                }
            En[c] = mx[(size_t)v * W2 + lo + c] + best;
            back[(size_t)(v - v_h) * win + c] = (int8_t)bt;
        }
        std::swap(E, En);
    }
    int c = 0;
    for (int cc = 1; cc < win; ++cc)
        if (E[cc] < E[c]) c = cc;
    int touch = 0;
    for (int v = v_h; v <= v_max; ++v) {
        if ((lo > 0 && c == 0) || (hi < W2 - 1 && c == win - 1)) touch = 1;
        cpath[v] = lo + c;
        if (v < v_max) c += back[(size_t)(v - v_h) * win + c];
    }
    return touch;
}

// The track of Eq. lane_visualisation as one affine map of the start column per row:
// u_v = fma(a_v, u_start, b_v), with a_{v_max} = 1, b_{v_max} = 0 and, going up one row,
// a_v = B_v a_{v+1}, b_v = fma(B_v, b_{v+1}, A_v) (A_v, B_v as in the energy step).  Written for
// the rows max(v_lo, v_end) .. v_max.
int ldref_track_affine(const double* vpx, const double* vpy, int H, int v_end, int v_lo, double* a_out,
                       double* b_out) {
    const int v_max = H - 1;
    double a = 1.0, c = 0.0;
    for (int v = v_max; v >= std::max(v_lo, v_end); --v) {
        if (v < v_max) {
            const double den = (double)(v + 1) - vpy[v + 1];
            const double Av = vpx[v + 1] / den;
            const double Bv = ((double)v - vpy[v + 1]) / den;
            a = Bv * a;
            c = std::fma(Bv, c, Av);
        }
        a_out[v] = a;
        b_out[v] = c;
    }
    return 0;
}

// Candidate mask of the narrowed search: candidate i (u_start = i - W/2) is hit when its track
// column floor(u_v + 0.5) on a band row v >= v_end is a marked pixel; keep = hit dilated by
// `dilate` candidates.  Returns the number kept.
int ldref_cand_mask(const uint8_t* lane_bits, int W, int H, int v_h, int v_end, int nb, int dilate,
                    const double* vpx, const double* vpy, uint8_t* hit_out, uint8_t* keep_out) {
    const int W2 = 2 * W, half = W / 2, v_max = H - 1;
    std::vector<double> av(H, 0.0), bv(H, 0.0);
    const int top_hi = band_top(v_h, H, nb, nb - 1);
    ldref_track_affine(vpx, vpy, H, v_end, top_hi, av.data(), bv.data());
    std::vector<uint8_t> hit(W2, 0);
    for (int i = 0; i < W2; ++i) {
        const double us = (double)(i - half);
        for (int k = 0; k < nb && !hit[i]; ++k) {
            const int top = band_top(v_h, H, nb, k);
            for (int r = 0; r < 16; ++r) {
                const int v = top + r;
                if (v < v_end || v > v_max) continue;
                const double x = std::fma(av[v], us, bv[v]) + 0.5;
                if (x >= 0.0 && x < (double)W) {
                    const int col = (int)std::floor(x);
                    if (lane_bits[((size_t)k * 16 + r) * W + col]) { hit[i] = 1; break; }
                }
            }
        }
    }
    int kept = 0;
    for (int i = 0; i < W2; ++i) {
        uint8_t k = 0;
        for (int j = std::max(0, i - dilate); j <= std::min(W2 - 1, i + dilate); ++j) k |= hit[j];
        keep_out[i] = k;
        kept += k;
        if (hit_out) hit_out[i] = hit[i];
    }
    return kept;
}

static int detect_impl(const uint8_t* grey, int64_t gpitch, const void* disp, int64_t dpitch, int W, int H,
                       int fmt, int d_max, const ldref_params* P, uint64_t stream_id, int64_t frame_idx,
                       const double* seed_gamma, ldref_out* o, ldref_learned* L);

int ldref_detect(const uint8_t* grey, int64_t gpitch, const void* disp, int64_t dpitch, int W, int H,
                 int fmt, int d_max, const ldref_params* P, uint64_t stream_id, int64_t frame_idx,
                 const double* seed_gamma, ldref_out* o) {
    return detect_impl(grey, gpitch, disp, dpitch, W, H, fmt, d_max, P, stream_id, frame_idx, seed_gamma, o, nullptr);
}

int ldref_detect_pruned(const uint8_t* grey, int64_t gpitch, const void* disp, int64_t dpitch, int W, int H,
                        int fmt, int d_max, const ldref_params* P, uint64_t stream_id, int64_t frame_idx,
                        const double* seed_gamma, ldref_learned* L, ldref_out* o) {
    return detect_impl(grey, gpitch, disp, dpitch, W, H, fmt, d_max, P, stream_id, frame_idx, seed_gamma, o, L);
}

}  // extern "C"

static int detect_impl(const uint8_t* grey, int64_t gpitch, const void* disp, int64_t dpitch, int W, int H,
                       int fmt, int d_max, const ldref_params* P, uint64_t stream_id, int64_t frame_idx,
                       const double* seed_gamma, ldref_out* o, ldref_learned* L) {
    const int D1 = d_max + 1;
    const int W2 = 2 * W, half = W / 2, v_max = H - 1;
    o->flags = 0; o->v_h = H; o->v_end = H; o->n_lanes = 0; o->n_my = 0; o->n_edges = 0; o->n_votes = 0;
    std::memset(&o->beta, 0, sizeof(o->beta));
    std::memset(&o->gamma, 0, sizeof(o->gamma));
    const double nan = std::nan("");
    if (o->vpx) for (int v = 0; v < H; ++v) o->vpx[v] = nan;
    if (o->energy) for (int i = 0; i < W2; ++i) o->energy[i] = 0.0;
    if (o->curves) for (int i = 0; i < 16 * H; ++i) o->curves[i] = nan;
    if (o->mx_path) for (int v = 0; v < H; ++v) o->mx_path[v] = -1;
    if (o->m1) for (int64_t i = 0; i < (int64_t)H * W; ++i) o->m1[i] = 0.0;

    // S1: v-disparity histogram
    std::vector<int32_t> my((size_t)H * D1);
    ldref_vdisp_hist(disp, dpitch, W, H, fmt, d_max, my.data());
    if (o->m_y) std::memcpy(o->m_y, my.data(), sizeof(int32_t) * my.size());

    // S2: DP path on the v-disparity map
    std::vector<int32_t> pv(D1), px(D1), py(D1);
    int n_my = 0;
    ldref_vdisp_dp(my.data(), H, d_max, P->tau_y_max, P->lambda_y, pv.data(), px.data(), py.data(), &n_my);
    o->n_my = n_my;
    if (o->my_path_v) std::memcpy(o->my_path_v, pv.data(), sizeof(int32_t) * D1);
    if (o->my_x) { std::memcpy(o->my_x, px.data(), sizeof(int32_t) * n_my); std::memcpy(o->my_y, py.data(), sizeof(int32_t) * n_my); }

    // S3: beta by RANSAC, road tables, road rows
    ldref_ransac(px.data(), py.data(), n_my, 2, P->tr_y, P->n_hyp, P->max_rounds, P->eps_num, P->eps_den,
                 P->seed, stream_id, frame_idx, 0, nullptr, &o->beta, o->trace_beta);
    if (o->beta.flags & 1) o->flags |= 4;
    if (L) {
        for (int i = 0; i < 16; ++i) L->prune[i] = 0;
        L->prune[0] = L->n_bands;
        L->prune[1] = 1 | 4;          // no seed until one is found
        L->prune[2] = -1;
        L->prune[4] = -1;
        for (int k = 0; k < 4; ++k) L->prune[6 + k] = -1;
        L->prune[14] = 2 * W;
        if (L->cand_mask) for (int i = 0; i < 2 * W; ++i) L->cand_mask[i] = 1;
    }
    const int fb_flag = L ? 16 : 0;   // a frame that never reaches the narrowed search falls back
    if (!o->beta.ok) { o->flags |= 1 | fb_flag; return 0; }
    std::vector<double> f(H), fp(H), vpy(H);
    int32_t v_h = H;
    ldref_road_tables(&o->beta, H, f.data(), fp.data(), vpy.data(), &v_h);
    o->v_h = v_h;
    if (o->f) std::memcpy(o->f, f.data(), sizeof(double) * H);
    if (o->fp) std::memcpy(o->fp, fp.data(), sizeof(double) * H);
    if (o->vpy) std::memcpy(o->vpy, vpy.data(), sizeof(double) * H);
    const int R = v_max - v_h + 1;
    if (R < 8) { o->flags |= 1 | fb_flag; return 0; }

    // S4: gradient, road mask, edges
    const int cap = W * H;
    std::vector<int32_t> eu(cap), ev(cap), egx(cap), egy(cap), ebin(cap);
    int ne = ldref_road_edges(grey, gpitch, disp, dpitch, W, H, fmt, f.data(), v_h, P->varpi, P->edge_t,
                              eu.data(), ev.data(), egx.data(), egy.data(), cap);
    o->n_edges = ne;

    // S5: sparse V_px votes, per-row vote histogram h
    o->n_votes = ldref_votes(eu.data(), ev.data(), egx.data(), egy.data(), ne, vpy.data(), W, ebin.data());
    std::vector<int32_t> h((size_t)H * W2, 0);
    for (int i = 0; i < ne; ++i)
        if (ebin[i] >= 0) h[(size_t)ev[i] * W2 + ebin[i]] += 1;

    // S6 + S7: band accumulation and DP path M_x
    std::vector<int64_t> mx((size_t)H * W2, 0);
    ldref_band(h.data(), H, W2, v_h, P->chi, mx.data());
    std::vector<int32_t> cpath(H, -1);
    int fb = 0;
    std::vector<double> seed_line(5, 0.0);
    if (L) {
        // seed from the votes of marking edges on the bands
        const int nb = L->n_bands;
        int32_t est[4], cnt[4], tot = 0;
        int cs = ldref_seed(eu.data(), ev.data(), ebin.data(), ne, L->lane_bits, W, H, v_h, nb, L->min_votes, est,
                            cnt, &tot);
        int lo = 0, hi = -1;
        if (cs < 0) {
            fb = 1 | 4;
        } else {
            lo = std::max(0, cs - L->delta_x);
            hi = std::min(W2 - 1, cs + L->delta_x);
            if (W < 128) fb = 1 | 4;     // frames narrower than 128 columns take the full search
        }
        int klo = -1, khi = -1;
        for (int k = 0; k < nb; ++k)
            if (cnt[k] >= L->min_votes) { if (klo < 0) klo = k; khi = k; }
        if (cs >= 0 && L->seed_ransac) {
            if (klo >= 0 && khi != klo) {
                const double v0 = (double)(band_top(v_h, H, nb, klo) + 8), v1 = (double)(band_top(v_h, H, nb, khi) + 8);
                const double u0 = (double)(est[klo] - half), u1 = (double)(est[khi] - half);
                const double g1 = (u1 - u0) / (v1 - v0);
                seed_line[1] = g1;
                seed_line[0] = u0 - g1 * v0;
            } else {
                seed_line[0] = (double)((klo >= 0 ? est[klo] : cs) - half);
            }
        }
        L->prune[2] = cs; L->prune[3] = lo; L->prune[4] = hi; L->prune[5] = tot;
        for (int k = 0; k < 4; ++k) { L->prune[6 + k] = est[k]; L->prune[10 + k] = cnt[k]; }
        if (!(fb & 1)) {
            // the row DP of O10 restricted to columns lo..hi
            if (ldref_window_dp(mx.data(), H, W2, v_h, P->tau_x_max, P->lambda_x, lo, hi, cpath.data()))
                fb |= 1 | 8;
        }
        L->prune[1] = fb;
    }
    if (!L || (fb & 1)) ldref_row_dp(mx.data(), H, W2, v_h, P->tau_x_max, P->lambda_x, cpath.data());
    if (o->mx_path) std::memcpy(o->mx_path, cpath.data(), sizeof(int32_t) * H);
    std::vector<int32_t> mxv(R), mxu(R);
    for (int v = v_h; v <= v_max; ++v) { mxv[v - v_h] = v; mxu[v - v_h] = cpath[v] - half; }

    // S8: gamma by RANSAC and V_px(v) = g(v) (Eq. vpx_estimation); the narrowed search seeds
    // hypothesis 0 with the line through the band estimates when it has them (seed_ransac, no
    // fallback), and otherwise with the caller's seed, as the full search does
    const double* seed = (L && !(fb & 1) && L->seed_ransac) ? seed_line.data() : seed_gamma;
    ldref_ransac(mxv.data(), mxu.data(), R, 4, P->tr_x, P->n_hyp, P->max_rounds, P->eps_num, P->eps_den,
                 P->seed, stream_id, frame_idx, 1, seed, &o->gamma, o->trace_gamma);
    if (o->gamma.flags & 1) o->flags |= 8;
    if (L && (fb & 1)) o->flags |= 16;
    if (!o->gamma.ok) { o->flags |= 2; return 0; }
    std::vector<double> vpx(H, nan);
    for (int v = v_h; v <= v_max; ++v) vpx[v] = eval_s(o->gamma.coef, 4, o->gamma.center, o->gamma.kshift, v);
    if (o->vpx) std::memcpy(o->vpx, vpx.data(), sizeof(double) * H);

    // S9: weights q = G_x w_g on the road edges, scattered into an image-sized map
    std::vector<double> eq(ne > 0 ? ne : 1, 0.0);
    ldref_weights(eu.data(), ev.data(), egx.data(), egy.data(), ne, vpx.data(), vpy.data(), P->sigma_g,
                  P->weight_squared, eq.data(), P->vote);
    std::vector<double> q((size_t)H * W, 0.0);
    for (int i = 0; i < ne; ++i) q[(size_t)ev[i] * W + eu[i]] = eq[i];
    if (o->edge_u) {
        int n = std::min(ne, o->edge_cap);
        for (int i = 0; i < n; ++i) {
            o->edge_u[i] = eu[i]; o->edge_v[i] = ev[i]; o->edge_gx[i] = egx[i]; o->edge_gy[i] = egy[i];
            o->edge_bin[i] = ebin[i];
            if (o->edge_q) o->edge_q[i] = eq[i];
        }
    }

    // S10 + S11: M_0 and M_1
    std::vector<double> m0((size_t)H * W), m1((size_t)H * W);
    ldref_m0m1(q.data(), W, H, P->nu, P->varsigma, m0.data(), m1.data());
    if (o->m1) std::memcpy(o->m1, m1.data(), sizeof(double) * m1.size());

    // S12: candidate energies
    std::vector<double> E(W2, 0.0);
    o->v_end = ldref_energy(m1.data(), vpx.data(), vpy.data(), W, H, v_h, E.data(), nullptr, nullptr, 0);
    const int dn = P->d_nms > 0 ? P->d_nms : std::max(8, W / 64);
    if (L && !(fb & 1) && L->dilate >= 0) {
        // candidate mask: tracks through the band rows, u_v = fma(a_v, u_start, b_v)
        std::vector<uint8_t> keep(W2, 0);
        L->prune[14] = ldref_cand_mask(L->lane_bits, W, H, v_h, o->v_end, L->n_bands, L->dilate, vpx.data(),
                                       vpy.data(), nullptr, keep.data());
        if (L->cand_mask) std::memcpy(L->cand_mask, keep.data(), W2);
        std::vector<double> Em(W2);
        for (int i = 0; i < W2; ++i) Em[i] = keep[i] ? E[i] : 0.0;
        int32_t us[16];
        double el[16];
        const int n = ldref_peaks(Em.data(), W2, half, P->rho_lpv, dn, us, el);
        bool bad = n == 0;
        for (int l = 0; l < n; ++l) {
            const int i = us[l] + half;
            bad = bad || !keep[i - 1] || !keep[i + 1];
        }
        if (bad) {
            fb |= 2;
            L->prune[1] = fb;
            o->flags |= 16;
        } else {
            E = Em;
        }
    }
    if (o->energy) std::memcpy(o->energy, E.data(), sizeof(double) * W2);

    // S13: peaks and lane curves
    o->n_lanes = ldref_peaks(E.data(), W2, half, P->rho_lpv, dn, o->u_start, o->energy_lane);
    if (o->curves && o->n_lanes > 0)
        ldref_energy(m1.data(), vpx.data(), vpy.data(), W, H, v_h, nullptr, o->curves, o->u_start, o->n_lanes);
    return 0;
}

extern "C" {

}  // extern "C"
