// ld.hip -- MI355X (gfx950) kernels and C ABI of the lane-detection hot path.
//
// Method: Fan & Dahnoun, "Real-Time Stereo Vision-Based Lane Detection System"
// (arXiv 1807.02752), Sec. 2.2-2.4.  One launch of each kernel processes a whole batch of
// frames; per-pixel steps are spread over many workgroups per frame, the serial steps
// (dynamic programming, RANSAC, row sweeps) run one workgroup per frame out of LDS.
//
//   k_vdisp_hist   S1   v-disparity histogram (LDS bins, wave-aggregated atomics)
//   k_vdisp_fit    S2-3 DP on the v-disparity map, RANSAC road profile, V_py, road rows
//   k_edges        S4-5 Sobel on road rows, road mask, V_px vote column per edge
//   k_vpx_fit      S6-7 sliding band accumulator, row DP
//   k_vpx_ransac   S8   RANSAC V_px, track tables
//   k_energy       S9-12 w_g, M_0, M_1 row ring, candidate-by-row energy accumulation
//   k_peaks        S13  minima, threshold, suppression, lane curves
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <new>
#include <mutex>
#include <vector>
#include <type_traits>

#include "ld_device.h"
#include "ld_internal.h"

using namespace ldk;

namespace {

struct FitRes {
    int32_t ok, flags, center, kshift, rounds, n_surv;
    double coef[5];
    double raw[5];
};
static_assert(sizeof(FitRes) == sizeof(ld_fit), "FitRes must mirror ld_fit");

struct FrameInfo {
    int32_t flags, v_h, v_end, n_my, n_edges, n_votes, R, n_mx;
};

constexpr int kMaxRounds = 64;
constexpr int kBig = 0x3FFFFFFF;
constexpr int kMaxLds = 160 * 1024;   // LDS bytes a workgroup may hold on gfx950

// Device view of a frame object: sizes, parameters and the scratch carried between steps.
struct Dev {
    int W, H, D1, W2, half, fmt, d_max, B;
    int hist_rows;      // rows binned by one histogram workgroup
    int Hm;             // row stride of myT: H rounded up to 32, so a histogram workgroup's rows
                        // of one disparity fill whole 128-byte lines
    ld_params P;
    int32_t* myT;       // B x D1 x Hm  v-disparity counts, transposed (m_y(d, .) contiguous)
    uint8_t* back_y;    // B x D1 x H   v-disparity DP backtrace (tau)
    int32_t* my_pts;    // B x 2 x D1   DP path points with votes: rows, then disparities
    FitRes* fit;        // B x 2        beta, gamma
    FrameInfo* info;    // B
    double* tab;        // B x 6 x H    f, f', V_py, V_px, A_v, B_v
    int32_t* rowcnt;    // B x H        road edges per row
    ld_edge* edges;     // B x H x W    per-row edge buckets
    int8_t* back_x;     // B x H x ceil(2W/8) x 4 B   row-DP backtrace, 4-bit tie ranks
    int32_t* mxpath;    // B x H        row-DP path columns
    double* energy;     // B x 2W
    int32_t* trace;     // B x 2 x 3 x kMaxRounds
    float* qbuf;        // B x H x W    G_x w_g of every road edge, in bucket order
    uint32_t* rbound;   // B x H x 2    raw disparity interval of the road test per row
    uint8_t* lbits;     // B x 4 x 16 x W   network decisions on the bands (pruned search)
    int32_t* prune;     // B x 16       pruned-search state (LD_STATE_PRUNE layout)
    uint8_t* cmask;     // B x 2W       candidate mask of the pruned search
    double* seedg;      // B x 5        RANSAC hypothesis 0 of the pruned search (raw basis)
    const int32_t* nact;   // nullable device count: frames b >= *nact of a launch are skipped
    // nullable: run only the frames whose fallback bits prune[b][1] & only_bits are
    // non-zero (only_set = 1) or zero (only_set = 0)
    const int32_t* only;
    int only_bits, only_set;
};

constexpr int kPruneWords = 16;
constexpr int kFbPlainVpx = 1, kFbPlainEnergy = 2, kFbNoSeed = 4, kFbTouch = 8;

__device__ __forceinline__ bool frame_masked(const Dev& d, int b) {
    if (d.nact != nullptr && b >= *d.nact) return true;
    if (d.only != nullptr && (((d.only[b * kPruneWords + 1] & d.only_bits) != 0) != (d.only_set != 0))) return true;
    return false;
}

// ------------------------------------------------------------------------------------------
// Block-wide helpers (any multiple of 64 threads up to 1024)
__device__ __forceinline__ int nwaves() { return blockDim.x / kWave; }

__device__ __forceinline__ int block_max_i32(int x, int* red) {
    x = wave_max_i32(x);
    int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) red[w] = x;
    __syncthreads();
    int r = red[0];
    for (int i = 1; i < nwaves(); ++i) r = max(r, red[i]);
    return r;
}

__device__ __forceinline__ int block_min_i32(int x, int* red) {
    x = wave_min_i32(x);
    int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) red[w] = x;
    __syncthreads();
    int r = red[0];
    for (int i = 1; i < nwaves(); ++i) r = min(r, red[i]);
    return r;
}

__device__ __forceinline__ int block_sum_i32(int x, int* red) {
    x = wave_sum_i32(x);
    int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) red[w] = x;
    __syncthreads();
    int r = 0;
    for (int i = 0; i < nwaves(); ++i) r += red[i];
    return r;
}

// (value, index) argmin over the block, ties to the smaller index
__device__ __forceinline__ void block_argmin_i64(int64_t& v, int& i, int64_t* rv, int* ri) {
    wave_argmin_i64(v, i);
    int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) { rv[w] = v; ri[w] = i; }
    __syncthreads();
    v = rv[0];
    i = ri[0];
    for (int k = 1; k < nwaves(); ++k)
        if (rv[k] < v || (rv[k] == v && ri[k] < i)) { v = rv[k]; i = ri[k]; }
}

// ------------------------------------------------------------------------------------------
// RANSAC (Alg. "beta/gamma estimation with the assist of RANSAC").  Each round scores up to
// 64 random samples of DEG+1 points, one per lane of wave 0, and the points are split over
// the waves of the workgroup for the inlier count; the best sample's outliers are removed by a stable
// ballot compaction; the loop ends when the inliers reach eps of the round's points.  The
// final model is refitted on the survivors from exact 128-bit moments.
struct RansacShared {
    double models[kMaxHyp][5];
    int mvalid[kMaxHyp];            // 0 invalid, 1 fitted (s basis), 2 caller seed (raw basis)
    int counts[kMaxWaves][kMaxHyp];
    int wsum[kMaxWaves];
    int red[kMaxWaves];
    int best_h, best_n;
    i128 mred[kMaxWaves][14];
};

template <int DEG>
__device__ __forceinline__ bool is_inlier(const double* m, int kind, int center, int kshift, int x, int y,
                                          double tr) {
    double fv = (kind == 2) ? eval_raw<DEG>(m, x) : eval_s<DEG>(m, center, kshift, x);
    double res = (double)y - fv;
    return res * res < tr;
}

template <int DEG>
__device__ void ransac_block(const int* X, const int* Y, int n0, int* cur, int* cur2, uint32_t* bitmap,
                             int bitmap_words, RansacShared& S, double tr, const ld_params& P, uint64_t key1,
                             uint64_t ctr0, int stage, const double* seed_raw, FitRes* out, int* trace) {
    constexpr int s = DEG + 1;
    const int t = threadIdx.x, lane = lane_id(), wave = t / kWave, nw = nwaves(), nt = blockDim.x;
    FitRes res;
    res.ok = 0; res.flags = 0; res.center = 0; res.kshift = 0; res.rounds = 0; res.n_surv = 0;
    for (int p = 0; p < 5; ++p) { res.coef[p] = 0.0; res.raw[p] = 0.0; }
    if (n0 < s) {
        if (t == 0) { res.flags = 1; *out = res; }
        __syncthreads();
        return;
    }
    int xmn = 0x7fffffff, xmx = -0x7fffffff;
    for (int j = t; j < n0; j += nt) { xmn = min(xmn, X[j]); xmx = max(xmx, X[j]); }
    xmn = block_min_i32(xmn, S.red);
    xmx = block_max_i32(xmx, S.red);
    const int center = (xmn + xmx) >> 1;
    const int wmax = max(xmx - center, center - xmn);
    int k = 0;
    while ((1 << k) < wmax) ++k;
    res.center = center;
    res.kshift = k;
    for (int j = t; j < n0; j += nt) cur[j] = j;
    const int need = max(s, (n0 + 9) / 10);
    const int n_hyp = min(P.n_hyp, kMaxHyp);
    int n_cur = n0;
    bool converged = false;
    int r = 0;
    __syncthreads();
    for (; r < P.max_rounds; ++r) {
        // ---- phase A: one sample + fit per hypothesis (wave 0)
        if (t < n_hyp) {
            double model[5] = {0, 0, 0, 0, 0};
            int kind = 0;
            if (t == 0 && seed_raw != nullptr && !isnan(seed_raw[0])) {   // a NaN seed means none
                for (int p = 0; p <= DEG; ++p) model[p] = seed_raw[p];
                kind = 2;
            } else {
                // draw indices until s distinct ones; the picks stay in registers (every
                // array index below is static after unrolling)
                int pick[s];
#pragma unroll
                for (int e = 0; e < s; ++e) pick[e] = -1;
                int got = 0;
                for (int blk = 0; blk < 16 && got < s; ++blk) {
                    U64x4 w = philox4x64_10(ctr0, ((uint64_t)stage << 32) | (uint64_t)(uint32_t)r, (uint64_t)t,
                                            (uint64_t)blk, P.seed, key1);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int ix = (int)__umul64hi(w.w[q], (uint64_t)n_cur);
                        bool dup = false;
#pragma unroll
                        for (int e = 0; e < s; ++e) dup = dup || (e < got && pick[e] == ix);
                        const bool take = got < s && !dup;
#pragma unroll
                        for (int e = 0; e < s; ++e) pick[e] = (take && e == got) ? ix : pick[e];
                        got += take ? 1 : 0;
                    }
                }
                if (got == s) {
                    int px[s], py[s];
#pragma unroll
                    for (int e = 0; e < s; ++e) { px[e] = X[cur[pick[e]]]; py[e] = Y[cur[pick[e]]]; }
                    bool distinct = true;
#pragma unroll
                    for (int e = 1; e < s; ++e)
#pragma unroll
                        for (int f = 0; f < e; ++f) distinct = distinct && (px[f] != px[e]);
                    if (distinct) {
                        Moments M;
                        moments_zero(M);
#pragma unroll
                        for (int e = 0; e < s; ++e) moments_add<DEG>(M, px[e], py[e], center);
                        kind = solve_moments<DEG>(M, k, model) ? 1 : 0;
                    }
                }
            }
            for (int p = 0; p < 5; ++p) S.models[t][p] = model[p];
            S.mvalid[t] = kind;
        }
        __syncthreads();
        // ---- phase B: inlier counts, hypothesis = lane, points split over the waves
        {
            const int h = lane;
            int cnt = -1;
            if (h < n_hyp && S.mvalid[h] != 0) {
                double m[5];
#pragma unroll
                for (int p = 0; p < 5; ++p) m[p] = S.models[h][p];
                const int kind = S.mvalid[h];
                int c4[4] = {0, 0, 0, 0};
                int jj = wave;
                for (; jj + 3 * nw < n_cur; jj += 4 * nw) {   // four independent evaluations
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int j = cur[jj + u * nw];
                        c4[u] += is_inlier<DEG>(m, kind, center, k, X[j], Y[j], tr) ? 1 : 0;
                    }
                }
                for (; jj < n_cur; jj += nw) {
                    const int j = cur[jj];
                    c4[0] += is_inlier<DEG>(m, kind, center, k, X[j], Y[j], tr) ? 1 : 0;
                }
                cnt = (c4[0] + c4[1]) + (c4[2] + c4[3]);
            }
            S.counts[wave][h] = cnt;
        }
        __syncthreads();
        // ---- phase C: best hypothesis (most inliers, lowest index)
        if (wave == 0) {
            int tot = -1;
            if (lane < n_hyp && S.counts[0][lane] >= 0) {
                tot = 0;
                for (int w = 0; w < nw; ++w) tot += S.counts[w][lane];
            }
            int bn = tot, bh = lane;
            for (int o = 32; o > 0; o >>= 1) {
                int on = __shfl_xor(bn, o, kWave), oh = __shfl_xor(bh, o, kWave);
                if (on > bn || (on == bn && oh < bh)) { bn = on; bh = oh; }
            }
            if (lane == 0) { S.best_h = bn >= 0 ? bh : -1; S.best_n = bn; }
        }
        __syncthreads();
        const int best_h = S.best_h, best_n = S.best_n;
        if (trace && t == 0) { trace[3 * r] = best_h; trace[3 * r + 1] = best_n; trace[3 * r + 2] = n_cur; }
        if (best_h < 0 || best_n < need) { ++r; break; }
        // ---- phase D: keep the inliers of the best sample, in order
        {
            const double* m = S.models[best_h];
            const int kind = S.mvalid[best_h];
            int base = 0;
            for (int c0 = 0; c0 < n_cur; c0 += nt) {
                int jj = c0 + t, j = 0;
                bool pred = false;
                if (jj < n_cur) {
                    j = cur[jj];
                    pred = is_inlier<DEG>(m, kind, center, k, X[j], Y[j], tr);
                }
                uint64_t bal = __ballot(pred);
                int wpre = __popcll(bal & lanes_below());
                if (lane == 0) S.wsum[wave] = __popcll(bal);
                __syncthreads();
                int off = base, tot = 0;
                for (int w = 0; w < nw; ++w) {
                    if (w < wave) off += S.wsum[w];
                    tot += S.wsum[w];
                }
                if (pred) cur2[off + wpre] = j;
                base += tot;
                __syncthreads();
            }
        }
        const bool done = (int64_t)P.eps_den * best_n >= (int64_t)P.eps_num * n_cur;
        int* tmp = cur; cur = cur2; cur2 = tmp;
        n_cur = best_n;
        __syncthreads();
        if (done) { converged = true; ++r; break; }
    }
    res.rounds = r;
    res.flags = converged ? 0 : 1;
    res.n_surv = n_cur;
    // ---- final fit on the survivors: distinct abscissae, exact moments, solve
    for (int i = t; i < bitmap_words; i += nt) bitmap[i] = 0u;
    __syncthreads();
    for (int jj = t; jj < n_cur; jj += nt) {
        int x = X[cur[jj]];
        atomicOr(&bitmap[x >> 5], 1u << (x & 31));
    }
    __syncthreads();
    int pc = 0;
    for (int i = t; i < bitmap_words; i += nt) pc += __popc(bitmap[i]);
    const int distinct = block_sum_i32(pc, S.red);
    Moments M;
    moments_zero(M);
    for (int jj = t; jj < n_cur; jj += nt) moments_add<DEG>(M, X[cur[jj]], Y[cur[jj]], center);
    for (int p = 0; p <= 2 * DEG; ++p) M.sw[p] = wave_sum_i128(M.sw[p]);
    for (int p = 0; p <= DEG; ++p) M.syw[p] = wave_sum_i128(M.syw[p]);
    if (lane == 0) {
        for (int p = 0; p <= 2 * DEG; ++p) S.mred[wave][p] = M.sw[p];
        for (int p = 0; p <= DEG; ++p) S.mred[wave][9 + p] = M.syw[p];
    }
    __syncthreads();
    if (t == 0) {
        if (distinct >= s) {
            Moments T;
            moments_zero(T);
            for (int w = 0; w < nw; ++w) {
                for (int p = 0; p <= 2 * DEG; ++p) T.sw[p] += S.mred[w][p];
                for (int p = 0; p <= DEG; ++p) T.syw[p] += S.mred[w][9 + p];
            }
            if (solve_moments<DEG>(T, k, res.coef)) {
                res.ok = 1;
                to_raw<DEG>(res.coef, center, k, res.raw);
            }
        }
        *out = res;
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------------------
// S1: v-disparity histogram m_y(d, v) (Sec. 2.2).  A workgroup bins hist_rows rows of one
// frame into LDS; within a wave, the lanes that share the first active lane's bin are merged
// by ballot into one LDS atomic and the other lanes add directly (a road row puts most
// pixels into one or two bins, so one merge removes most of the same-address traffic; merging
// two or three bins this way measured slower).  Rows
// are taken four at a time, and the raw values of the next four rows are loaded while the
// current four are binned, so a wave always has a group of loads in flight.  The counts
// leave transposed, hist_rows consecutive rows per disparity.
constexpr int kHistGroup = 4;
constexpr int kHistMerge = 1;

template <int FMT> struct RawPixel { using T = uint8_t; };
template <> struct RawPixel<LD_DISP_F32> { using T = float; };
template <> struct RawPixel<LD_DISP_U16Q4> { using T = uint16_t; };

// Bin of one raw disparity value; false for the invalid ones (0 in the integer formats,
// non-positive or non-finite in F32), so a load masked to 0 is never counted.
template <int FMT>
__device__ __forceinline__ bool disp_bin(typename RawPixel<FMT>::T x, int d_max, int& bin) {
    if (FMT == LD_DISP_U8) {
        bin = min((int)x, d_max);
        return x != 0;
    } else if (FMT == LD_DISP_F32) {
        if (!(isfinite((float)x) && (float)x > 0.0f)) return false;
        double b = floor((double)x + 0.5);
        bin = b > (double)d_max ? d_max : (int)b;
        return true;
    } else {
        bin = min(((int)x + 8) >> 4, d_max);
        return x != 0;
    }
}

template <int FMT, int NPT>
__device__ __forceinline__ void hist_load(const typename RawPixel<FMT>::T* base, int64_t pitch_px, int W, int t,
                                          int g, int rows, typename RawPixel<FMT>::T (&dst)[kHistGroup][NPT]) {
#pragma unroll
    for (int r = 0; r < kHistGroup; ++r) {
        const typename RawPixel<FMT>::T* row = base + (int64_t)min(g + r, rows - 1) * pitch_px;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int u = t + k * kBlock;
            dst[r][k] = (g + r < rows && u < W) ? row[u] : typename RawPixel<FMT>::T(0);
        }
    }
}

template <int FMT, int NPT>
__global__ __launch_bounds__(kBlock) void k_vdisp_hist(Dev d, const uint8_t* disp, int64_t pitch, int32_t* vdisp_out) {
    using Raw = typename RawPixel<FMT>::T;
    extern __shared__ int hist[];   // hist_rows x D1
    const int hr = d.hist_rows;
    const int b = blockIdx.y, v0 = blockIdx.x * hr, t = threadIdx.x, lane = lane_id();
    if (frame_masked(d, b)) return;
    const int D1 = d.D1, W = d.W, H = d.H;
    const int rows = min(hr, H - v0);
    const Raw* base = reinterpret_cast<const Raw*>(disp + ((int64_t)b * H + v0) * pitch);
    const int64_t pitch_px = pitch / (int64_t)sizeof(Raw);
    Raw nxt[kHistGroup][NPT];
    hist_load<FMT, NPT>(base, pitch_px, W, t, 0, rows, nxt);
    for (int i = t; i < hr * D1; i += kBlock) hist[i] = 0;
    __syncthreads();
    for (int g = 0; g < rows; g += kHistGroup) {
        int bins[kHistGroup][NPT];
        bool ok[kHistGroup][NPT];
#pragma unroll
        for (int r = 0; r < kHistGroup; ++r)
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                bins[r][k] = 0;
                ok[r][k] = disp_bin<FMT>(nxt[r][k], d.d_max, bins[r][k]);
            }
        if (g + kHistGroup < rows) hist_load<FMT, NPT>(base, pitch_px, W, t, g + kHistGroup, rows, nxt);
#pragma unroll
        for (int r = 0; r < kHistGroup; ++r) {
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                bool pend = ok[r][k];
                const int bin = bins[r][k];
                int* hrow = hist + (g + r) * D1;
                uint64_t act = __ballot(pend);
                // up to kHistMerge distinct bins of the wave are merged, each into one atomic
                // by its first lane; the lanes left over (many distinct bins) add one each
#pragma unroll
                for (int it = 0; it < kHistMerge; ++it) {
                    if (act == 0) break;
                    const int leader = __ffsll((unsigned long long)act) - 1;
                    const int b0 = __builtin_amdgcn_readlane(bin, leader);   // uniform: no LDS round trip
                    const bool same = pend && bin == b0;
                    const uint64_t m = __ballot(same);
                    if (lane == leader) atomicAdd(&hrow[b0], __popcll(m));
                    pend = pend && !same;
                    act &= ~m;
                }
                if (act != 0 && pend) atomicAdd(&hrow[bin], 1);
            }
        }
    }
    __syncthreads();
    for (int i = t; i < rows * D1; i += kBlock) {
        const int dd = i / rows, r = i % rows;
        d.myT[((int64_t)b * D1 + dd) * d.Hm + v0 + r] = hist[r * D1 + dd];
    }
    if (vdisp_out) {
        for (int i = t; i < rows * D1; i += kBlock) {
            const int r = i / D1, dd = i % D1;
            vdisp_out[((int64_t)b * H + v0 + r) * D1 + dd] = hist[r * D1 + dd];
        }
    }
}

// ------------------------------------------------------------------------------------------
// S2 + S3: DP on the v-disparity map (Eq. vpy_estimation), RANSAC road profile beta
// (Alg. "beta estimation"), tables f, f', V_py (Eq. vpy_equation) and the road rows.  One
// workgroup per frame; E lives in two LDS rows, the backtrace in global memory.
// The road test of Sec. 2.3.1, valid(raw) and |D(raw) - f| <= varpi in FP64, as an interval
// of raw pixel values.  D is non-decreasing in the raw value over the valid values (u8:
// 1..255, u16: 1..65535, f32: the bit patterns of positive finite floats) and the rounded
// difference D - f is non-decreasing in D, so the passing raw values form one interval
// [lo, hi]; both ends are found by bisection on the same FP64 predicate.  Every invalid raw
// value (0, negative, infinite or NaN floats) lies outside it.  lo > hi when it is empty.
__device__ __forceinline__ double raw_to_d(int fmt, uint32_t r) {
    if (fmt == LD_DISP_U8) return (double)r;
    if (fmt == LD_DISP_U16Q4) return (double)r / 16.0;
    return (double)__uint_as_float(r);
}

__device__ void road_interval(int fmt, double f, double varpi, uint32_t& lo, uint32_t& hi) {
    const uint32_t top = fmt == LD_DISP_U8 ? 255u : (fmt == LD_DISP_U16Q4 ? 65535u : 0x7F7FFFFFu);
    lo = 1u;
    hi = 0u;
    // smallest r with D(r) - f >= -varpi
    if (!(raw_to_d(fmt, top) - f >= -varpi)) return;
    uint32_t a = 1u, z = top;
    if (!(raw_to_d(fmt, a) - f >= -varpi)) {
        while (z - a > 1u) {            // predicate false at a, true at z
            const uint32_t m = a + (z - a) / 2u;
            if (raw_to_d(fmt, m) - f >= -varpi) z = m; else a = m;
        }
        a = z;
    }
    // largest r with D(r) - f <= varpi
    if (!(raw_to_d(fmt, 1u) - f <= varpi)) return;
    uint32_t x = 1u, y = top;
    if (!(raw_to_d(fmt, y) - f <= varpi)) {
        while (y - x > 1u) {            // predicate true at x, false at y
            const uint32_t m = x + (y - x) / 2u;
            if (raw_to_d(fmt, m) - f <= varpi) x = m; else y = m;
        }
    } else {
        x = y;
    }
    lo = a;
    hi = x;
}

constexpr int kVdRows = 4;                 // rows per thread in the v-disparity DP
constexpr int kVdWalk = 32;                // DP steps of the backtrace staged in LDS per walk chunk
constexpr int kVdWalkCols = 257;           // staged rows per step (covers kVdWalk steps of tau_max)
constexpr int kVdPad = 8;                  // padding rows after each DP row
constexpr int kVdPadKey = 0x3FFFFFF0;      // padding key: above any real key, and twice it fits int32

__global__ __launch_bounds__(1024) void k_vdisp_fit(Dev d, const uint64_t* stream_ids, const int64_t* frame_idx,
                                                    double* beta_out) {
    extern __shared__ unsigned char smem[];
    __shared__ RansacShared S;
    __shared__ int64_t rv[kMaxWaves];
    __shared__ int ri[kMaxWaves];
    __shared__ int s_n, s_v;
    const int b = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
    if (frame_masked(d, b)) return;
    const int H = d.H, D1 = d.D1, d_max = d.d_max;
    // DP rows hold E << 4 (E <= 0, low 4 bits zero); the kVdPad entries past row H - 1 hold a
    // key that loses to every real one
    int* E0 = reinterpret_cast<int*>(smem);
    int* E1 = E0 + H + kVdPad;
    int* PX = E1 + H + kVdPad;
    int* PY = PX + D1;
    int* cur = PY + D1;
    int* cur2 = cur + D1;
    uint32_t* bitmap = reinterpret_cast<uint32_t*>(cur2 + D1);
    const int bm_words = (H + 31) / 32;
    uint8_t* win = reinterpret_cast<uint8_t*>(bitmap + bm_words);   // kVdWalk x kVdWalkCols
    uint8_t* back = d.back_y + (int64_t)b * D1 * H;
    const int Hm = d.Hm;
    const int32_t* myT = d.myT + (int64_t)b * D1 * Hm;
    const int tau_max = d.P.tau_y_max, lam = d.P.lambda_y;

    for (int v = t; v < H; v += nt) {
        E0[v] = -myT[(int64_t)d_max * Hm + v] * 16;
        d.rowcnt[(int64_t)b * H + v] = 0;
    }
    if (t < kVdPad) { E0[H + t] = kVdPadKey; E1[H + t] = kVdPadKey; }
    // step costs of the packed keys: 16 lambda tau + tau for an allowed jump, the padding key
    // for tau > tau_max (so the key loses), for the window of up to 8 rows read at once
    int addc[9];
#pragma unroll
    for (int tau = 1; tau <= 8; ++tau) addc[tau] = tau <= tau_max ? 16 * lam * tau + tau : kVdPadKey;
    // the column m_y(d, .) of the next DP step is loaded while the current one is computed
    int nxt[kVdRows];
#pragma unroll
    for (int k = 0; k < kVdRows; ++k) {
        const int v = t + k * nt;
        nxt[k] = (d_max >= 1 && v < H) ? myT[(int64_t)(d_max - 1) * Hm + v] : 0;
    }
    __syncthreads();
    int* Ec = E0;
    int* En = E1;
    for (int dd = d_max - 1; dd >= 0; --dd) {
        int curm[kVdRows];
#pragma unroll
        for (int k = 0; k < kVdRows; ++k) curm[k] = nxt[k];
        if (dd >= 1) {
#pragma unroll
            for (int k = 0; k < kVdRows; ++k) {
                const int v = t + k * nt;
                nxt[k] = v < H ? myT[(int64_t)(dd - 1) * Hm + v] : 0;
            }
        }
#pragma unroll
        for (int k = 0; k < kVdRows; ++k) {
            const int v = t + k * nt;
            if (v < H) {
                if (tau_max <= 8) {
                    // key of jump tau: (E(v + tau) + lambda tau) << 4 | tau; the minimum is the
                    // smallest cost, and among equal costs the smallest tau (the strict-< scan
                    // over tau = 0, 1, ...).  Rows past H - 1 read the padding.
                    int e[9];
#pragma unroll
                    for (int j = 0; j <= 8; ++j) e[j] = Ec[v + j];
                    int m = e[0];
#pragma unroll
                    for (int tau = 1; tau <= 8; ++tau) m = min(m, e[tau] + addc[tau]);
                    En[v] = (m & -16) - curm[k] * 16;
                    back[(int64_t)dd * H + v] = (uint8_t)(m & 15);
                } else {
                    int best = Ec[v] >> 4, bt = 0;
                    for (int tau = 1; tau <= tau_max && v + tau <= H - 1; ++tau) {
                        const int c = (Ec[v + tau] >> 4) + lam * tau;
                        if (c < best) { best = c; bt = tau; }
                    }
                    En[v] = (best - curm[k]) * 16;
                    back[(int64_t)dd * H + v] = (uint8_t)bt;
                }
            }
        }
        __syncthreads();
        int* tmp = Ec; Ec = En; En = tmp;
    }
    int64_t bv = INT64_MAX;
    int bi = 0x7fffffff;
    for (int v = t; v < H; v += nt)
        if ((int64_t)Ec[v] < bv) { bv = Ec[v]; bi = v; }
    block_argmin_i64(bv, bi, rv, ri);
    // backtrace: stage the rows the path can reach in the next kVdWalk steps, then one thread
    // follows it (the path moves down by at most tau_max rows per step)
    const int steps = max(1, min(kVdWalk, (kVdWalkCols - 1) / max(1, tau_max)));
    if (t == 0) s_v = bi;
    __syncthreads();
    for (int d0 = 0; d0 <= d_max; d0 += steps) {
        const int v0 = s_v;
        const int nst = min(steps, d_max - d0);               // steps with a backtrace entry
        const int ncols = min(H - v0, tau_max * steps + 1);
        for (int i = t; i < nst * ncols; i += nt) {
            const int r = i / ncols, c = i % ncols;
            win[r * kVdWalkCols + c] = back[(int64_t)(d0 + r) * H + v0 + c];
        }
        __syncthreads();
        if (t == 0) {
            int v = v0;
            const int last = min(d0 + steps - 1, d_max);
            for (int dd = d0; dd <= last; ++dd) {
                cur[dd] = v;                                    // row of disparity dd on the path
                if (dd < d_max) v += win[(dd - d0) * kVdWalkCols + (v - v0)];
            }
            s_v = v;
        }
        __syncthreads();
    }
    // keep the path points that carry votes, in order of disparity (stable ballot compaction)
    {
        const int lane = lane_id(), wave = t / kWave, nw = nwaves();
        int base = 0;
        for (int c0 = 0; c0 <= d_max; c0 += nt) {
            const int dd = c0 + t;
            const bool pred = dd <= d_max && myT[(int64_t)dd * Hm + cur[dd]] > 0;
            const uint64_t bal = __ballot(pred);
            if (lane == 0) S.wsum[wave] = __popcll(bal);
            __syncthreads();
            int off = base, tot = 0;
            for (int w = 0; w < nw; ++w) {
                if (w < wave) off += S.wsum[w];
                tot += S.wsum[w];
            }
            if (pred) {
                const int o = off + __popcll(bal & lanes_below());
                PX[o] = cur[dd];
                PY[o] = dd;
            }
            base += tot;
            __syncthreads();
        }
        if (t == 0) s_n = base;
        __syncthreads();
    }
    const int n_my = s_n;
    for (int i = t; i < n_my; i += nt) {
        d.my_pts[(int64_t)b * 2 * D1 + i] = PX[i];
        d.my_pts[(int64_t)b * 2 * D1 + D1 + i] = PY[i];
    }
    const uint64_t sid = stream_ids ? stream_ids[b] : 0ull;
    const uint64_t fid = frame_idx ? (uint64_t)frame_idx[b] : (uint64_t)b;
    FitRes* fit = d.fit + 2 * b;
    ransac_block<2>(PX, PY, n_my, cur, cur2, bitmap, bm_words, S, d.P.tr_y, d.P, sid, fid, 0, nullptr, fit,
                    d.trace + (int64_t)b * 6 * kMaxRounds);
    // tables and road rows
    const FitRes& beta = *fit;
    const int ok = beta.ok;
    double* tf = d.tab + (int64_t)b * 6 * H;
    double* tfp = tf + H;
    double* tvpy = tf + 2 * H;
    double* tvpx = tf + 3 * H;
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    int bad = -1;
    if (ok) {
        const double sc = ldexp(1.0, -beta.kshift);
        for (int v = t; v < H; v += nt) {
            double s = (double)(v - beta.center) * sc;
            double fv = beta.coef[2];
            fv = fv * s + beta.coef[1];
            fv = fv * s + beta.coef[0];
            double tt = 2.0 * beta.coef[2];
            double dv = (beta.coef[1] + tt * s) * sc;
            tf[v] = fv;
            tfp[v] = dv;
            tvpy[v] = (double)v - fv / dv;
            tvpx[v] = nan;
            if (!(fv > 0.0 && dv > 0.0)) bad = max(bad, v);
            uint32_t lo, hi;
            road_interval(d.fmt, fv, d.P.varpi, lo, hi);
            d.rbound[((int64_t)b * H + v) * 2] = lo;
            d.rbound[((int64_t)b * H + v) * 2 + 1] = hi;
        }
    } else {
        for (int v = t; v < H; v += nt) { tf[v] = nan; tfp[v] = nan; tvpy[v] = nan; tvpx[v] = nan; }
    }
    bad = block_max_i32(bad, S.red);
    if (t == 0) {
        FrameInfo fi;
        fi.flags = (beta.flags & 1) ? LD_FLAG_NOCONS_Y : 0;
        fi.v_h = ok ? bad + 1 : H;
        fi.R = H - fi.v_h;
        if (!ok || fi.R < 8) fi.flags |= LD_FLAG_NOROAD;
        fi.v_end = H;
        fi.n_my = n_my;
        fi.n_edges = 0;
        fi.n_votes = 0;
        fi.n_mx = 0;
        d.info[b] = fi;
        if (beta_out) {
            for (int p = 0; p < 3; ++p) beta_out[3 * b + p] = ok ? beta.raw[p] : nan;
        }
    }
}

// ------------------------------------------------------------------------------------------
// S4 + S5: Sobel gradient on the road rows, edge test, road mask (Sec. 2.3.1) and the V_px
// vote of every road edge (Eq. sparse_vpx_estimation with the gradient read as the edge
// slope).
//
// A workgroup takes kEdgeStrip rows of one frame across its whole width: wave w owns the 256
// columns from 256 w, four consecutive columns per lane, and walks the rows down.  A row is
// loaded as one aligned dword per lane (plus the dwords left and right of the wave's span for
// its first and last lane); the six bytes a lane needs (columns ub-1 .. ub+4) come from its own
// dword and its neighbours' by DPP lane shifts.  The loads go through a buffer resource bounded
// by the frame's rows, so a dword outside the frame reads as 0 and is never fetched (those
// bytes feed no result: the gradient is only taken at 1 <= u <= W-2, 1 <= v <= H-2).  Rows go
// in groups of three, the loads of the next group issued before the current one is worked on.
// Only the grey image is streamed: the edge test needs no disparity.  The edge pixels of a
// wave are queued in LDS and, in batches of 64, each lane gathers the raw disparity of one
// queued pixel, applies the road test (an integer compare against the row's raw interval),
// takes the vote column and appends the record to its row's bucket (LDS slot counters of the
// strip, so every bucket of the strip, and its count, is written by this workgroup alone and
// nothing carries over from an earlier call).
template <int N> using IntC = std::integral_constant<int, N>;

constexpr int kEdgeStrip = 32;                        // rows per workgroup
constexpr int kEdgeCols = 4 * kWave;                  // columns per wave
constexpr int kEdgeQueue = 512;                       // queued edge pixels per wave
constexpr int kEdgeFlushAt = kEdgeQueue - kEdgeCols;  // a row queues at most kEdgeCols
static_assert(sizeof(ld_edge) == 8, "an edge record is written as one 8-byte store");

template <int FMT>
__device__ __forceinline__ uint32_t disp_raw(const uint8_t* row, int u) {
    if (FMT == LD_DISP_U8) return row[u];
    if (FMT == LD_DISP_F32) return reinterpret_cast<const uint32_t*>(row)[u];
    return reinterpret_cast<const uint16_t*>(row)[u];
}

// Vote column of an edge: floor(x + 0.5) with x = u + (tt * gy) / gx in IEEE FP64, each
// operation rounded as written.  The quotient is first taken as p * (1/gx) with the
// reciprocal refined by two Newton steps and one residual correction, which is within an ulp
// or two of the rounded quotient; the floor of x + 0.5 can differ from the exact one only
// when x + 0.5 lies within a few ulps of an integer, and there (and for non-finite values)
// the rounded division is taken.  Returns the bin or -1 when the column is outside
// [-half, W2 - half).
__device__ __forceinline__ int vote_bin(double tt, int gy, int gx, int u, int half, int W2) {
    const double p = tt * (double)gy;
    const double g = (double)gx;
    double r = __builtin_amdgcn_rcp(g);
    r = fma(r, fma(-g, r, 1.0), r);
    r = fma(r, fma(-g, r, 1.0), r);
    double q = p * r;
    q = fma(fma(-g, q, p), r, q);
    double y = ((double)u + q) + 0.5;
    double bf = floor(y);
    const double fr = y - bf;
    if (!(fr >= 0x1p-30 && fr <= 1.0 - 0x1p-30)) bf = floor(((double)u + p / g) + 0.5);
    return (bf >= -(double)half && bf < (double)(W2 - half)) ? (int)bf + half : -1;
}

__device__ __forceinline__ uint32_t dpp_from_prev(uint32_t x) {   // lane l gets lane l-1's x
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t dpp_from_next(uint32_t x) {   // lane l gets lane l+1's x
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, false);
}

template <int FMT>
__global__ __launch_bounds__(1024) void k_edges(Dev d, const uint8_t* grey, int64_t gpitch, const uint8_t* disp,
                                                int64_t dpitch) {
    extern __shared__ __attribute__((aligned(16))) unsigned char esm[];   // strip tables, then the wave queues
    const int b = blockIdx.y, s0 = blockIdx.x * kEdgeStrip;
    if (frame_masked(d, b)) return;
    const int W = d.W, H = d.H, t = threadIdx.x, lane = lane_id(), wave = t / kWave;
    const int rows = min(kEdgeStrip, H - s0);
    double* svpy = reinterpret_cast<double*>(esm);                      // V_py of the strip's rows
    uint32_t* sbnd = reinterpret_cast<uint32_t*>(svpy + kEdgeStrip);    // raw road interval per row
    int* scnt = reinterpret_cast<int*>(sbnd + 2 * kEdgeStrip);          // edges per row
    uint2* queue = reinterpret_cast<uint2*>(scnt + kEdgeStrip) + wave * kEdgeQueue;
    const FrameInfo fi = d.info[b];
    const bool road = !(fi.flags & LD_FLAG_NOROAD);
    if (t < kEdgeStrip) {
        scnt[t] = 0;
        if (road && t < rows) {
            const int64_t v = (int64_t)b * H + s0 + t;
            svpy[t] = d.tab[(int64_t)b * 6 * H + 2 * H + s0 + t];
            sbnd[2 * t] = d.rbound[2 * v];
            sbnd[2 * t + 1] = d.rbound[2 * v + 1];
        }
    }
    __syncthreads();
    const int vs = max(max(s0, road ? fi.v_h : H), 1), ve = min(s0 + rows - 1, H - 2);
    const int ub = wave * kEdgeCols + 4 * lane;
    if (vs <= ve) {
        // the frame's rows through a buffer resource: base aligned down to a dword, records up
        // to the end of the frame's last row rounded up to a dword
        const uintptr_t fbase = (uintptr_t)(grey + (int64_t)b * H * gpitch);
        const uintptr_t abase = fbase & ~(uintptr_t)3;
        const int nrec = (int)((((fbase + (uintptr_t)((int64_t)H * gpitch)) + 3) & ~(uintptr_t)3) - abase);
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(abase), 0, nrec, 0x00020000);
        // every lane issues both loads; the extra one is fetched only by the first and last
        // lane (the others give an offset past the records, which reads 0 without a fetch)
        const int xoff = lane == 0 ? -4 : (lane == kWave - 1 ? 4 : INT32_MIN);
        struct RowD { uint32_t own, ext; };
        auto load_row = [&](int v) -> RowD {
            const uintptr_t ra = fbase + (uintptr_t)((int64_t)min(max(v, 0), H - 1) * gpitch);
            const int off = (int)((ra & ~(uintptr_t)3) - abase) + ub;
            RowD r;
            r.own = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
            r.ext = __builtin_amdgcn_raw_buffer_load_b32(rs, xoff == INT32_MIN ? INT32_MIN : off + xoff, 0, 0);
            return r;
        };
        // columns ub-1 .. ub+4 of row v
        auto unpack = [&](const RowD& r, int v, int* x) {
            const uint32_t sh = (uint32_t)((fbase + (uintptr_t)((int64_t)min(max(v, 0), H - 1) * gpitch)) & 3);
            uint32_t dp = dpp_from_prev(r.own), dn = dpp_from_next(r.own);
            if (lane == 0) dp = r.ext;
            if (lane == kWave - 1) dn = r.ext;
            const uint32_t mid = __builtin_amdgcn_alignbyte(dn, r.own, sh);   // ub .. ub+3
            const uint32_t lft = __builtin_amdgcn_alignbyte(r.own, dp, 3u);   // ub-sh-1 .. ub-sh+2
            x[0] = (int)((lft >> (8u * sh)) & 255u);
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k + 1] = (int)((mid >> (8 * k)) & 255u);
            x[5] = (int)((dn >> (8u * sh)) & 255u);
        };
        const int t2 = d.P.edge_t * d.P.edge_t;
        bool colok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) colok[k] = ub + k >= 1 && ub + k <= W - 2;
        int qn = 0;
        const uint8_t* dframe = disp + (int64_t)b * H * dpitch;
        ld_edge* eframe = d.edges + (int64_t)b * H * W;
        auto flush = [&]() {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            for (int i0 = 0; i0 < qn; i0 += kWave) {
                const int i = i0 + lane;
                if (i < qn) {
                    const uint2 e = queue[i];
                    const int u = (int)(e.x & 0xffffu), r = (int)(e.y >> 16);
                    const int gx = (int)(int16_t)(e.x >> 16), gy = (int)(int16_t)(e.y & 0xffffu);
                    const int v = s0 + r;
                    const uint32_t raw = disp_raw<FMT>(dframe + (int64_t)v * dpitch, u);
                    if (raw >= sbnd[2 * r] && raw <= sbnd[2 * r + 1]) {
                        const int bin = gx != 0 ? vote_bin((double)v - svpy[r], gy, gx, u, d.half, d.W2) : -1;
                        const int slot = atomicAdd(&scnt[r], 1);
                        reinterpret_cast<uint2*>(eframe + (int64_t)v * W)[slot] =
                            make_uint2(e.x, (uint32_t)(uint16_t)gy | ((uint32_t)(uint16_t)bin << 16));
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            qn = 0;
        };
        // Ring of three unpacked rows (rotated by renaming: at the step of phase P, rows v-1 and
        // v sit in U[(P+2)%3] and U[P], and row v+1 is unpacked into U[(P+1)%3]) and two sets of
        // three rows of loads: a group of steps consumes one set, whose loads were issued a
        // whole group earlier, after issuing the other set's loads for the next group.  Steps
        // past the strip's last row compute masked rows.
        int U[3][6];
        RowD LA[3], LB[3];
        LA[0] = load_row(vs - 1);
        LA[1] = load_row(vs);
        unpack(LA[0], vs - 1, U[2]);
        unpack(LA[1], vs, U[0]);
        LA[0] = load_row(vs + 1);
        LA[1] = load_row(vs + 2);
        LA[2] = load_row(vs + 3);
        int v = vs;
        auto step = [&](auto Pc, const RowD& row_next) {
            constexpr int P = decltype(Pc)::value;
            constexpr int A = (P + 2) % 3, M = P % 3, C = (P + 1) % 3;
            const bool rowok = v <= ve;
            unpack(row_next, v + 1, U[C]);
            int S[6], T[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                S[j] = U[A][j] + 2 * U[M][j] + U[C][j];
                T[j] = U[C][j] - U[A][j];
            }
            uint64_t bal[4];
            int gxk[4], gyk[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                gxk[k] = S[k + 2] - S[k];
                gyk[k] = T[k] + 2 * T[k + 1] + T[k + 2];
                const int m2 = __mul24(gxk[k], gxk[k]) + __mul24(gyk[k], gyk[k]);
                bal[k] = __ballot(colok[k] & rowok & (m2 > t2));
            }
            if ((bal[0] | bal[1] | bal[2] | bal[3]) != 0) {
                int off = qn;
                const uint32_t rv = (uint32_t)(v - s0) << 16;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (bal[k] != 0) {
                        if ((bal[k] >> lane) & 1ull)
                            queue[off + __popcll(bal[k] & lanes_below())] =
                                make_uint2((uint32_t)(ub + k) | ((uint32_t)gxk[k] << 16),
                                           ((uint32_t)gyk[k] & 0xffffu) | rv);
                        off += __popcll(bal[k]);
                    }
                }
                qn = off;
                if (qn >= kEdgeFlushAt) flush();
            }
            ++v;
        };
        while (v <= ve) {
#pragma unroll
            for (int j = 0; j < 3; ++j) LB[j] = load_row(v + 4 + j);
            step(IntC<0>{}, LA[0]);
            step(IntC<1>{}, LA[1]);
            step(IntC<2>{}, LA[2]);
            if (v > ve) break;
#pragma unroll
            for (int j = 0; j < 3; ++j) LA[j] = load_row(v + 4 + j);
            step(IntC<3>{}, LB[0]);
            step(IntC<4>{}, LB[1]);
            step(IntC<5>{}, LB[2]);
        }
        flush();
    }
    __syncthreads();
    if (t < rows) d.rowcnt[(int64_t)b * H + s0 + t] = scnt[t];
}

// ------------------------------------------------------------------------------------------
// S6 + S7 + S8: band accumulator m_x (Alg. "Dense V_px accumulation", a band of 2 chi + 1 rows
// clipped to the road), DP path over the 2W vote columns (Eq. dense_vpx_estimation), RANSAC
// quartic gamma (Alg. "gamma estimation"), V_px table (Eq. vpx_estimation) and the
// coefficients of the lane track of Eq. lane_visualisation.  One workgroup per frame, one
// thread per run of kDpRun consecutive columns.
//
// DP step.  The value E + lambda|tau| and the tie rank of tau in the scan order
// 0, -1, +1, -2, +2, ... (0..10) are packed into one key (value << 4 | rank): the minimum key
// is the minimum value with the first tau of the scan order, which is exactly the
// first-strict-minimum rule.  With Sh = E << 4 the key of tau = -a is
// Sh(c') - (16 lambda + 2) c' + ((16 lambda + 2) c - 1) and of tau = +a is
// Sh(c') + (16 lambda + 2) c' - (16 lambda + 2) c (c' = c + tau), so each side is a plain
// minimum of a per-column term over a window, plus a per-c constant.  The rank (4 bits) is
// the backtrace, eight columns per 32-bit word.
constexpr int kDpRun = 8;
constexpr int kFitWalk = 16;         // rows of the backtrace per register chunk of the walk

// The band edges of one row, up to kBandPer per thread (a row holds at most W edges and the
// workgroup has at least W/4 threads).
constexpr int kBandPer = 4;

__device__ __forceinline__ void band_load(const ld_edge* row_edges, int cnt, int* bins) {
#pragma unroll
    for (int k = 0; k < kBandPer; ++k) {
        const int i = threadIdx.x + k * blockDim.x;
        bins[k] = i < cnt ? row_edges[i].bin : -1;
    }
}

__device__ __forceinline__ int* smem_i(unsigned char* p) { return reinterpret_cast<int*>(p); }

// position of column c (c >= -8) in a run-interleaved row with NR runs
__device__ __forceinline__ int ipos(int c, int NR) { return (c & (kDpRun - 1)) * NR + (c >> 3) + 1; }

__device__ __forceinline__ void band_apply(const int* bins, int sign, int* hist, int NR) {
#pragma unroll
    for (int k = 0; k < kBandPer; ++k)
        if (bins[k] >= 0) atomicAdd(&hist[ipos(bins[k], NR)], sign);
}

__device__ __forceinline__ int rank_to_tau(int r) { return r == 0 ? 0 : ((r & 1) ? -((r + 1) >> 1) : (r >> 1)); }
// rank_to_tau(r) + 8 in bits 4r .. 4r+3 for r = 0 .. 10
constexpr uint64_t kRankTau = [] {
    uint64_t x = 0;
    for (int r = 0; r <= 10; ++r) x |= (uint64_t)((r == 0 ? 0 : ((r & 1) ? -((r + 1) >> 1) : (r >> 1))) + 8) << (4 * r);
    return x;
}();

// S8: RANSAC of the quartic through the path points (PX = rows, PY = u columns), V_px and the
// track tables, frame info.
__device__ void vpx_fit_tail(Dev& d, int b, FrameInfo fi, int* PX, int* PY, int* cur, int* cur2, uint32_t* bitmap,
                             int bm_words, RansacShared& S, const uint64_t* stream_ids, const int64_t* frame_idx,
                             const double* seed, double* vp_out) {
    const int t = threadIdx.x, nt = blockDim.x;
    const int H = d.H, v_max = H - 1, v_h = fi.v_h, R = v_max - v_h + 1;
    double* tf = d.tab + (int64_t)b * 6 * H;
    double* tvpy = tf + 2 * H;
    double* tvpx = tf + 3 * H;
    double* tA = tf + 4 * H;
    double* tB = tf + 5 * H;
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    const uint64_t sid = stream_ids ? stream_ids[b] : 0ull;
    const uint64_t fid = frame_idx ? (uint64_t)frame_idx[b] : (uint64_t)b;
    FitRes* fit = d.fit + 2 * b + 1;
    ransac_block<4>(PX, PY, R, cur, cur2, bitmap, bm_words, S, d.P.tr_x, d.P, sid, fid, 1,
                    seed, fit,
                    d.trace + (int64_t)b * 6 * kMaxRounds + 3 * kMaxRounds);
    const FitRes& g = *fit;
    int bad = v_h - 1;
    if (g.ok) {
        for (int v = t; v < H; v += nt)
            tvpx[v] = (v >= v_h) ? eval_s<4>(g.coef, g.center, g.kshift, v) : nan;
    }
    __syncthreads();
    if (g.ok) {
        for (int v = v_h + t; v <= v_max - 1; v += nt) {
            const double den = (double)(v + 1) - tvpy[v + 1];
            if (!(den > 0.0)) {
                bad = max(bad, v);
            } else {
                tA[v] = tvpx[v + 1] / den;
                tB[v] = ((double)v - tvpy[v + 1]) / den;
            }
        }
    }
    bad = block_max_i32(bad, S.red);
    if (t == 0) {
        fi.flags |= (g.flags & 1) ? LD_FLAG_NOCONS_X : 0;
        if (!g.ok) fi.flags |= LD_FLAG_NOVP;
        fi.v_end = g.ok ? bad + 1 : H;
        fi.n_mx = R;
        d.info[b] = fi;
    }
    if (vp_out) {
        for (int v = t; v < H; v += nt) {
            const bool road = v >= v_h && g.ok;
            vp_out[((int64_t)b * H + v) * 2] = road ? tvpx[v] : nan;
            vp_out[((int64_t)b * H + v) * 2 + 1] = v >= v_h ? tvpy[v] : nan;
        }
    }
}

// NRC: the run count NR of the interleaved rows as a compile-time constant (>= nwords + 2,
// so the LDS offsets of the window below become immediates), or 0 for nwords + 2 at run time.
// Seven waves per SIMD (72 VGPRs, a few bytes spilled outside the row loop) leave room for
// four 320-thread frames on every CU however their waves fall on its SIMDs, so a 1024-frame
// batch runs in one round; at six waves per SIMD some CUs held only three of them.
template <int MAXT, int NRC>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(7))) void k_vpx_fit(Dev d) {
    extern __shared__ unsigned char smem[];
    __shared__ int64_t rv[kMaxWaves];
    __shared__ int ri[kMaxWaves];
    __shared__ int red[kMaxWaves];
    const int b = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
    if (frame_masked(d, b)) return;
    const int H = d.H, W2 = d.W2, v_max = H - 1;
    const int nwords = (W2 + kDpRun - 1) / kDpRun;
    FrameInfo fi = d.info[b];
    for (int v = t; v < H; v += nt) d.mxpath[(int64_t)b * H + v] = -1;
    if (fi.flags & LD_FLAG_NOROAD) return;
    const int v_h = fi.v_h, R = v_max - v_h + 1, chi = d.P.chi;
    // DP rows and the band histogram are stored run-interleaved, column c at
    // (c mod 8) * NR + c / 8 + 1, so that the lanes of a wave (one run of 8 columns each)
    // touch consecutive words; runs -1 and nruns are padding (kBig).
    const int NR = NRC > 0 ? NRC : nwords + 2;
    const int WP = kDpRun * NR;
    int* hist = reinterpret_cast<int*>(smem);   // WP, interleaved, 16 x the band's votes
    int* Sa = hist + WP;                 // E << 4
    int* Sb = Sa + WP;
    int* cntL = Sb + WP;                 // per-row edge counts
    const ld_edge* fedges = d.edges + (int64_t)b * H * d.W;
    for (int v = t; v < H; v += nt) cntL[v] = d.rowcnt[(int64_t)b * H + v];
    for (int i = t; i < WP; i += nt) { hist[i] = 0; Sa[i] = kBig; Sb[i] = kBig; }
    __syncthreads();
    int ne = 0;
    for (int v = v_h + t; v <= v_max; v += nt) ne += cntL[v];
    ne = block_sum_i32(ne, red);
    int nv = 0;   // votes that landed in a column (counted as each row enters the band)
    // initial band rows max(v_max - chi, v_h) .. v_max, four rows of loads in flight at a time
    for (int v = max(v_max - chi, v_h); v <= v_max; v += 4) {
        int bins[4][kBandPer];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = v + j;
            band_load(fedges + (int64_t)r * d.W, r <= v_max ? cntL[r] : 0, bins[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int k = 0; k < kBandPer; ++k) nv += bins[j][k] >= 0 ? 1 : 0;
            band_apply(bins[j], 16, hist, NR);
        }
    }
    __syncthreads();
    for (int c = t; c < W2; c += nt) Sa[ipos(c, NR)] = -hist[ipos(c, NR)];
    __syncthreads();
    const int tau_max = d.P.tau_x_max;
    const int slope = 16 * d.P.lambda_x + 2;
    uint32_t* back = reinterpret_cast<uint32_t*>(d.back_x) + (int64_t)b * H * nwords;
    const int c0 = t * kDpRun;
    // each thread's window Sh(c0-5 .. c0+12) of a DP row: window column c0 - 5 + j sits at int
    // index t + K[j] (K uniform over the workgroup: K[j] = ((3 + j) mod 8) NR + (3 + j) div 8)
    constexpr int kWin = kDpRun + 10;
    int K[kWin];
#pragma unroll
    for (int j = 0; j < kWin; ++j) K[j] = ((3 + j) & (kDpRun - 1)) * NR + ((3 + j) >> 3);
    const bool full5 = tau_max == 5;
    // band rows entering / leaving at the next DP row: each thread's first edge of both rows is
    // prefetched one row ahead (one register each keeps the kernel at 80 VGPRs); the edges past
    // the first blockDim.x of a row (rare) are read when the row is applied
    auto first_bin = [&](int r, bool in) -> int {
        const int n = in ? cntL[r] : 0;
        return t < n ? fedges[(int64_t)r * d.W + t].bin : -1;
    };
    auto rest_apply = [&](int r, bool in, int sign) {
        const int n = in ? cntL[r] : 0;
        for (int i = t + nt; i < n; i += nt) {
            const int c = fedges[(int64_t)r * d.W + i].bin;
            if (c >= 0) {
                atomicAdd(&hist[ipos(c, NR)], 16 * sign);
                nv += sign > 0 ? 1 : 0;
            }
        }
    };
    int nadd, nrem;
    {
        const int v = v_max - 1;
        const int ra = v - chi, rr = v + chi + 1;
        nadd = first_bin(max(ra, 0), ra >= v_h);
        nrem = first_bin(min(rr, v_max), rr <= v_max);
    }
    // bits of the backtrace word that belong to columns below W2
    const uint32_t wmask = c0 + kDpRun <= W2 ? 0xFFFFFFFFu : (1u << (4 * max(W2 - c0, 0))) - 1u;
    int parity = 0;   // 0: read Sa, write Sb
    // The row recursion, instantiated once for the full window (tau_max = 5) and once for a
    // narrower one, so the per-column minima carry no run-time test.  The per-c constant of
    // the window minima cancels between the shifted terms and the result, so only the
    // uniform offsets slope * (j - 5) and slope * k enter.
    auto dp_rows = [&](auto full) {
        constexpr bool kFull = decltype(full)::value;
        for (int v = v_max - 1; v >= v_h; --v) {
            const int cadd = nadd, crem = nrem;
            if (v - 1 >= v_h) {
                const int ra = v - 1 - chi, rr = v + chi;
                nadd = first_bin(max(ra, 0), ra >= v_h);
                nrem = first_bin(min(rr, v_max), rr <= v_max);
            }
            nv += cadd >= 0 ? 1 : 0;
            if (cadd >= 0) atomicAdd(&hist[ipos(cadd, NR)], 16);
            if (crem >= 0) atomicAdd(&hist[ipos(crem, NR)], -16);
            {
                const int ra = v - chi, rr = v + chi + 1;
                rest_apply(max(ra, 0), ra >= v_h, 1);
                rest_apply(min(rr, v_max), rr <= v_max, -1);
            }
            __syncthreads();
            if (c0 < W2) {
                const int* src = (parity ? Sb : Sa) + t;
                int* dst = (parity ? Sa : Sb) + t;
                const int* hs = hist + t;
                int w[kWin], h[kDpRun], TL[kWin], TR[kWin];
#pragma unroll
                for (int j = 0; j < kWin; ++j) w[j] = src[K[j]];
#pragma unroll
                for (int k = 0; k < kDpRun; ++k) h[k] = hs[K[k + 5]];
#pragma unroll
                for (int j = 0; j < kWin; ++j) {
                    TL[j] = w[j] - slope * (j - 5);     // tau < 0 terms, less slope * c
                    TR[j] = w[j] + slope * (j - 5);     // tau > 0 terms, plus slope * c
                }
                uint32_t word = 0;
#pragma unroll
                for (int k = 0; k < kDpRun; ++k) {
                    int lm, rm;
                    if constexpr (kFull) {
                        lm = min(min(min(TL[k], TL[k + 1]), min(TL[k + 2], TL[k + 3])), TL[k + 4]);
                        rm = min(min(min(TR[k + 6], TR[k + 7]), min(TR[k + 8], TR[k + 9])), TR[k + 10]);
                    } else {
                        lm = kBig; rm = kBig;
#pragma unroll
                        for (int a = 1; a <= 5; ++a)
                            if (a <= tau_max) { lm = min(lm, TL[k + 5 - a]); rm = min(rm, TR[k + 5 + a]); }
                    }
                    const int key = min(w[k + 5], min(lm + (slope * k - 1), rm - slope * k));
                    // (E_min - votes) << 4; columns past W2 keep the padding value
                    dst[K[k + 5]] = c0 + k < W2 ? (key & -16) - h[k] : kBig;
                    word |= (uint32_t)(key & 15) << (4 * k);
                }
                back[(int64_t)v * nwords + t] = word & wmask;
            }
            __syncthreads();
            parity ^= 1;
        }
    };
    if (full5) dp_rows(std::true_type{});
    else dp_rows(std::false_type{});
    int* Sc = parity ? Sb : Sa;
    int64_t bvv = INT64_MAX;
    int bi = 0x7fffffff;
    for (int c = t; c < W2; c += nt) {
        const int64_t e = Sc[ipos(c, NR)] >> 4;
        if (e < bvv) { bvv = e; bi = c; }
    }
    block_argmin_i64(bvv, bi, rv, ri);
    // backtrace, by wave 0: lane l holds word w0 + l of each of kFitWalk rows (64 words = 512
    // columns), with the next chunk in flight; the column is wave-uniform, so a step is a
    // readlane and a few scalar operations.  The path moves at most 5 columns a row, so from
    // the start column c of a chunk it stays within c +- 5 kFitWalk over this chunk and within
    // c +- 10 kFitWalk over the next, which the next chunk's words (centred on c) cover.
    if (t < kWave) {
        const int l = t;
        int c = bi;
        auto wbase = [&](int col) { return max(0, min((col >> 3) - 31, nwords - kWave)); };
        uint32_t bk[kFitWalk], bn[kFitWalk];
        auto load_chunk = [&](int v0, int w0, uint32_t (&dst)[kFitWalk]) {
            const int wi = min(w0 + l, nwords - 1);
#pragma unroll
            for (int r = 0; r < kFitWalk; ++r) {
                const int v = min(v0 + r, v_max - 1);          // rows v < v_max hold an entry
                dst[r] = back[(int64_t)v * nwords + wi];
            }
        };
        int wcur = wbase(c);
        load_chunk(v_h, wcur, bk);
        for (int v0 = v_h; v0 <= v_max; v0 += kFitWalk) {
            const int wnext = wbase(c);
            load_chunk(v0 + kFitWalk, wnext, bn);          // clamped rows: always a full chunk
            int pv = 0;
#pragma unroll
            for (int r = 0; r < kFitWalk; ++r) {
                const int v = v0 + r;
                if (v <= v_max) {
                    if (l == r) pv = c;
                    if (v < v_max) {
                        const uint32_t word = __builtin_amdgcn_readlane(bk[r], (c >> 3) - wcur);
                        c += rank_to_tau((int)((word >> (4 * (c & 7))) & 15u));
                    }
                }
            }
            if (l < kFitWalk && v0 + l <= v_max) d.mxpath[(int64_t)b * H + v0 + l] = pv;
#pragma unroll
            for (int r = 0; r < kFitWalk; ++r) bk[r] = bn[r];
            wcur = wnext;
        }
    }
    nv = block_sum_i32(nv, red);
    if (t == 0) {
        fi.n_edges = ne;
        fi.n_votes = nv;
        d.info[b] = fi;
    }
}

// S8 for every frame: RANSAC of the quartic through the row-DP path (read back from the path
// columns), V_px and the track tables.  One 128-thread workgroup per frame (the RANSAC's
// registers allow many per CU).  Hypothesis 0: the seed of the narrowed search for the frames
// that kept one (pruned = 1), otherwise the caller's seed rows.
// Three waves per frame: the inlier counts of a round split the points over the waves, and
// three 192-thread workgroups per CU still hold every frame of a 1024 batch at once.
#ifndef LD_RANSAC_THREADS
#define LD_RANSAC_THREADS 192
#endif
constexpr int kRansacThreads = LD_RANSAC_THREADS;
__global__ __launch_bounds__(kRansacThreads) void k_vpx_ransac(Dev d, const uint64_t* stream_ids, const int64_t* frame_idx,
                                                    const double* seed_gamma, int pruned, double* vp_out) {
    extern __shared__ unsigned char smem[];
    __shared__ RansacShared S;
    const int b = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
    if (frame_masked(d, b)) return;
    const int H = d.H, v_max = H - 1;
    const FrameInfo fi = d.info[b];
    double* tf = d.tab + (int64_t)b * 6 * H;
    for (int v = t; v < H; v += nt) {
        tf[4 * H + v] = 0.0;
        tf[5 * H + v] = 0.0;
    }
    if (fi.flags & LD_FLAG_NOROAD) {
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        if (vp_out)
            for (int v = t; v < H; v += nt) {
                vp_out[((int64_t)b * H + v) * 2] = nan;
                vp_out[((int64_t)b * H + v) * 2 + 1] = nan;
            }
        return;
    }
    const int v_h = fi.v_h;
    int* PX = reinterpret_cast<int*>(smem);
    int* PY = PX + H;
    int* cur = PY + H;
    int* cur2 = cur + H;
    uint32_t* bitmap = reinterpret_cast<uint32_t*>(cur2 + H);
    const int bm_words = (H + 31) / 32;
    for (int v = v_h + t; v <= v_max; v += nt) {
        PX[v - v_h] = v;
        PY[v - v_h] = d.mxpath[(int64_t)b * H + v] - d.half;
    }
    __syncthreads();
    // hypothesis 0: the narrowed search's own seed when it has one (no fallback, a seed line
    // drawn), else the caller's seed (NaN first coefficient or NULL: none)
    const double* seed = seed_gamma ? seed_gamma + 5 * (int64_t)b : nullptr;
    if (pruned && !(d.prune[(int64_t)b * kPruneWords + 1] & kFbPlainVpx) && !isnan(d.seedg[5 * (int64_t)b]))
        seed = d.seedg + 5 * (int64_t)b;
    vpx_fit_tail(d, b, fi, PX, PY, cur, cur2, bitmap, bm_words, S, stream_ids, frame_idx, seed, vp_out);
}

// ------------------------------------------------------------------------------------------
// S9 - S12: piecewise weight w_g (Eq. sigma_g), q = G_x w_g, M_0 (box of 3 columns x 7 rows),
// M_1 = Sobel-x of M_0 (Alg. "Lane position validation"), and the energy of every candidate
// along its track (Eq. lane_energy, Eq. lane_visualisation).
//
// One workgroup per frame.  First q is computed for every road edge (each wave a group of rows)
// into a per-edge buffer.  Then the road rows are swept upwards.  At the step of row v every
// thread pushes its NC columns (consecutive when NC is odd, a stride coprime with the LDS
// banks; else t, t + 256, ...) of the dense q row v-4 (scattered into LDS during the previous
// step) into a 9-row register ring (rows v-4..v+4) and forms V(x, v) = sum_y s_y C(x, v+y),
// C = vertical 7-row sums, with the zero padding of M_0 outside the image (a uniform branch:
// rows strictly inside take both neighbours without a select), while the edges of row v-5 are
// scattered into the other q row; after the step's one barrier the column owners form
// M_1(u, v) = sum_{dx} V(u+1+dx) - sum_{dx} V(u-1+dx) (terms outside the image dropped, on the
// few edge lanes only; consecutive columns share their three-column sums) into one of two LDS
// rows, and every candidate adds M_1 at its track column of row v+1.  The q, V and M_1 rows are
// double-buffered by row parity, so one barrier per row orders every write before its reads.
// Rows are padded to the NC * 256 columns the threads own (the columns past W hold zeros), so
// the column loops carry no bounds test.  The row loop is unrolled nine times so that the ring
// rotates by renaming registers instead of moving them.
// mode 0 / 1: G_x w_g with the exponent as printed / squared; mode 2: the prior work's vote
// |grad| cos(theta_e - theta_Vp) = t . (p - V_p) / |p - V_p| = -dot / |r|, in FP64 (no gate)
__device__ __forceinline__ float edge_q(const ld_edge& ed, int r, double vx, double vy, float inv_sg2, int sq) {
    const double tx = (double)(-ed.gy), ty = (double)ed.gx;
    const double rx = vx - (double)ed.u, ry = vy - (double)r;
    const double dot = tx * rx + ty * ry;
    const double tt = tx * tx + ty * ty;
    const double rr = rx * rx + ry * ry;
    if (sq == 2) return rr > 0.0 ? (float)(-dot / sqrt(rr)) : 0.0f;
    if (!(dot * dot >= (0.75 * tt) * rr)) return 0.0f;
    const double cr = tx * ry - ty * rx;
    const float delta = atan2f((float)fabs(cr), (float)fabs(dot));
    const float p = delta * (float)(36.0 / 3.14159265358979323846);
    const float w = sq ? expf(-(p * p) * inv_sg2) : expf(-p * inv_sg2);
    return (float)ed.gx * w;
}

template <int NC, int NT>
__global__ __launch_bounds__(kBlock) void k_energy(Dev d, const uint8_t* cand_mask, float* energy_out) {
    extern __shared__ float fsm[];
    const int b = blockIdx.x, t = threadIdx.x, lane = lane_id(), wave = t / kWave;
    if (frame_masked(d, b)) return;
    const int W = d.W, H = d.H, W2 = d.W2, v_max = H - 1;
    const FrameInfo fi = d.info[b];
    double* Eout = d.energy + (int64_t)b * W2;
    if (fi.flags & (LD_FLAG_NOROAD | LD_FLAG_NOVP)) {
        for (int i = t; i < W2; i += kBlock) {
            Eout[i] = 0.0;
            if (energy_out) energy_out[(int64_t)b * W2 + i] = 0.0f;
        }
        return;
    }
    constexpr int WP = NC * kBlock;  // columns owned by the threads (>= W)
    // a thread owns NC consecutive columns when NC is odd (a stride coprime with the LDS banks),
    // else columns t, t + 256, ...
    constexpr bool kConsec = NC % 2 == 1;
    auto col = [&](int k) { return kConsec ? t * NC + k : t + k * kBlock; };
    // by row parity: dense q rows; V rows, column u at u + 2 (two zero columns each side); M_1
    // rows (entries >= W stay 0)
    auto qb = [&](int par) -> float* { return fsm + par * WP; };
    auto Vp = [&](int par) -> float* { return fsm + 2 * WP + par * (WP + 4); };
    auto mb = [&](int par) -> float* { return fsm + 4 * WP + 8 + par * (WP + 1); };
    const double* tf = d.tab + (int64_t)b * 6 * H;
    const double* tvpy = tf + 2 * H;
    const double* tvpx = tf + 3 * H;
    const double* tA = tf + 4 * H;
    const double* tB = tf + 5 * H;
    const int v_h = fi.v_h, v_end = fi.v_end;
    const float inv_sg2 = (float)(1.0 / (d.P.sigma_g * d.P.sigma_g));
    const int sq = d.P.vote ? 2 : d.P.weight_squared;
    const ld_edge* edges = d.edges + (int64_t)b * H * W;
    float* qbuf = d.qbuf + (int64_t)b * H * W;
    const int32_t* rowcnt = d.rowcnt + (int64_t)b * H;

    // q of every road edge: a wave takes kQRows rows at a time and loads two edge slots per
    // lane (i = lane, lane + 64) of each, every load of the group issued before any q is
    // formed (clamped to the row's W slots; the counts mask them); longer rows go on in a loop
    constexpr int kQRows = 4;
    for (int r0 = v_h + wave * kQRows; r0 <= v_max; r0 += (kBlock / kWave) * kQRows) {
        int cnt[kQRows];
        double vx[kQRows], vy[kQRows];
        ld_edge e0[kQRows], e1[kQRows];
#pragma unroll
        for (int j = 0; j < kQRows; ++j) {
            const int r = min(r0 + j, v_max);
            cnt[j] = r0 + j <= v_max ? rowcnt[r] : 0;
            vx[j] = tvpx[r];
            vy[j] = tvpy[r];
            e0[j] = edges[(int64_t)r * W + min(lane, W - 1)];
            e1[j] = edges[(int64_t)r * W + min(lane + kWave, W - 1)];
        }
#pragma unroll
        for (int j = 0; j < kQRows; ++j) {
            const int r = r0 + j;
            if (lane < cnt[j]) qbuf[(int64_t)r * W + lane] = edge_q(e0[j], r, vx[j], vy[j], inv_sg2, sq);
            if (lane + kWave < cnt[j]) qbuf[(int64_t)r * W + lane + kWave] = edge_q(e1[j], r, vx[j], vy[j], inv_sg2, sq);
            for (int i = lane + 2 * kWave; i < cnt[j]; i += kWave)
                qbuf[(int64_t)r * W + i] = edge_q(edges[(int64_t)r * W + i], r, vx[j], vy[j], inv_sg2, sq);
        }
    }
    for (int i = t; i < 6 * WP + 10; i += kBlock) fsm[i] = 0.0f;
    float ring[NC][9];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int j = 0; j < 9; ++j) ring[k][j] = 0.0f;
    double uu[NT], ee[NT];
    bool live[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int i = t + k * kBlock;
        uu[k] = (double)(i - d.half);
        ee[k] = 0.0;
        live[k] = i < W2 && (cand_mask == nullptr || cand_mask[(int64_t)b * W2 + i] != 0);
    }
    __syncthreads();

    // the next row to scatter: its count and each thread's first edge are loaded a step ahead
    // (from a clamped, always valid index; the count masks them when they are used)
    int nx_r = -1, nx_cnt = 0, nx_u = 0;
    float nx_q = 0.0f;
    auto prefetch = [&](int r) {
        const int rr = min(max(r, 0), v_max), i = min(t, W - 1);
        nx_r = r;
        nx_cnt = (r >= v_h && r <= v_max) ? rowcnt[rr] : 0;
        nx_u = edges[(int64_t)rr * W + i].u;
        nx_q = qbuf[(int64_t)rr * W + i];
    };
    auto scatter_next = [&](float* q) {
        if (t < nx_cnt) q[nx_u] = nx_q;
        for (int i = t + kBlock; i < nx_cnt; i += kBlock)
            q[edges[(int64_t)nx_r * W + i].u] = qbuf[(int64_t)nx_r * W + i];
    };
    // slot S of the ring takes the newest row; reads and re-zeroes the owned columns of q
    auto push = [&](auto Sc, float* q) {
        constexpr int S = decltype(Sc)::value;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int u = col(k);
            ring[k][S] = q[u];
            q[u] = 0.0f;
        }
    };
    // the track of every live candidate moves to row w and adds M_1(col, w); a track outside
    // the image (or a dead candidate) reads the zero entry W (ee is never -0, so adding +0
    // leaves it unchanged).  The tracks are finite (A_v, B_v are finite on the swept rows);
    // the conversion saturates, so the unsigned compare also rejects x < 0 and huge x.
    // A_w, B_w are loaded one step before their row's turn (fma(1, u, 0) = u for w = v_max).
    double cA = 0.0, cB = 1.0;
    auto coef = [&](int w) {
        const bool upd = w < v_max;
        cA = upd ? tA[w] : 0.0;
        cB = upd ? tB[w] : 1.0;
    };
    auto candidates = [&](const float* m1row) {
        const double A = cA, Bc = cB;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            uu[k] = fma(Bc, uu[k], A);
            const int c = (int)floor(uu[k] + 0.5);
            const bool in = live[k] & ((unsigned)c < (unsigned)W);   // no branch: both are computed
            ee[k] += (double)m1row[in ? c : W];
        }
    };
    // rows v_max .. v_max-3 enter slots 0, 8, 7, 6; rows below the image stay zero; row
    // v_max-4 waits in its q row for the first step
    prefetch(v_max);
    scatter_next(qb(v_max & 1));               __syncthreads(); push(IntC<0>{}, qb(v_max & 1));
    prefetch(v_max - 1);
    scatter_next(qb((v_max - 1) & 1));         __syncthreads(); push(IntC<8>{}, qb((v_max - 1) & 1));
    prefetch(v_max - 2);
    scatter_next(qb((v_max - 2) & 1));         __syncthreads(); push(IntC<7>{}, qb((v_max - 2) & 1));
    prefetch(v_max - 3);
    scatter_next(qb((v_max - 3) & 1));         __syncthreads(); push(IntC<6>{}, qb((v_max - 3) & 1));
    prefetch(v_max - 4);
    scatter_next(qb((v_max - 4) & 1));
    prefetch(v_max - 5);
    __syncthreads();
    int v = v_max;
    // one row: newest ring slot S holds row v-4, slot (S + j) % 9 row v-4+j
    auto step = [&](auto Sc) -> bool {
        constexpr int S = decltype(Sc)::value;
        if (v < v_end) return false;
        const int par = v & 1;
        push(Sc, qb(par));               // row v - 4 (same parity as v)
        const bool up = v >= 1, dn = v + 1 <= v_max;   // M_0 is zero outside the image rows
        // (uniform over the workgroup: the rows strictly inside the image take both terms
        // without a per-column select)
        auto vcol = [&](auto both) {
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int u = col(k);
                float r[9];
#pragma unroll
                for (int j = 0; j < 9; ++j) r[j] = ring[k][(S + j) % 9];
                const float s5 = (((r[2] + r[3]) + r[4]) + r[5]) + r[6];
                const float cm1 = (r[0] + r[1]) + s5;   // C(v-1): rows v-4..v+2
                const float c0 = (r[1] + s5) + r[7];    // C(v):   rows v-3..v+3
                const float cp1 = (s5 + r[7]) + r[8];   // C(v+1): rows v-2..v+4
                float V = 2.0f * c0;
                if constexpr (decltype(both)::value) {
                    V += cm1;
                    V += cp1;
                } else {
                    V += up ? cm1 : 0.0f;
                    V += dn ? cp1 : 0.0f;
                }
                Vp(par)[u + 2] = V;
            }
        };
        if (up && dn) vcol(std::bool_constant<true>{}); else vcol(std::bool_constant<false>{});
        scatter_next(qb(par ^ 1));       // row v - 5
        prefetch(v - 6);
        __syncthreads();
        float* mrow = mb(par);
        const float* vr = Vp(par);
        // the three-column sums (the one over columns u-2 .. u, M_0 at u-1, is the one over
        // u .. u+2, M_0 at u+1, of the column two to the left: shared by consecutive columns)
        float g1[NC], g2[NC];
        if constexpr (kConsec) {
            float vv[NC + 4], T3[NC + 2];
#pragma unroll
            for (int j = 0; j < NC + 4; ++j) vv[j] = vr[t * NC + j];
#pragma unroll
            for (int j = 0; j < NC + 2; ++j) T3[j] = (vv[j] + vv[j + 1]) + vv[j + 2];
#pragma unroll
            for (int k = 0; k < NC; ++k) { g1[k] = T3[k + 2]; g2[k] = T3[k]; }
        } else {
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int u = col(k);
                g1[k] = (vr[u + 2] + vr[u + 3]) + vr[u + 4];
                g2[k] = (vr[u] + vr[u + 1]) + vr[u + 2];
            }
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int u = col(k);
            float m1 = g1[k] - g2[k];
            // the columns at the image edges and past it (a few lanes of a few waves)
            if (u < 1 || u >= W - 1) m1 = u < W ? (u + 1 <= W - 1 ? g1[k] : 0.0f) - (u >= 1 ? g2[k] : 0.0f) : 0.0f;
            mrow[u] = m1;
        }
        if (v < v_max) candidates(mb(par ^ 1));   // row v + 1
        coef(v);                       // for this row's candidates in the next step
        --v;
        return true;
    };
    while (step(IntC<5>{}) && step(IntC<4>{}) && step(IntC<3>{}) && step(IntC<2>{}) && step(IntC<1>{}) &&
           step(IntC<0>{}) && step(IntC<8>{}) && step(IntC<7>{}) && step(IntC<6>{})) {
    }
    if (v_end <= v_max) {
        __syncthreads();
        candidates(mb(v_end & 1));
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int i = t + k * kBlock;
        if (i < W2) {
            Eout[i] = ee[k];
            if (energy_out) energy_out[(int64_t)b * W2 + i] = (float)ee[k];
        }
    }
}

// ------------------------------------------------------------------------------------------
// S13: strict local minima of the energies, below rho * (deepest energy); greedy suppression
// of minima within d_nms of a deeper accepted one; lane curves by iterating the track.
__global__ __launch_bounds__(kBlock) void k_peaks(Dev d, ld_lanes* lanes_out, float* curves_out) {
    extern __shared__ unsigned char smem[];
    __shared__ int64_t rv[kMaxWaves];
    __shared__ int ri[kMaxWaves];
    __shared__ double dred[kMaxWaves];
    __shared__ int acc[LD_MAX_LANES];
    __shared__ int s_nacc;
    const int b = blockIdx.x, t = threadIdx.x;
    if (frame_masked(d, b)) return;
    const int W2 = d.W2, H = d.H, v_max = H - 1;
    const FrameInfo fi = d.info[b];
    const double* E = d.energy + (int64_t)b * W2;
    uint8_t* alive = smem;   // W2
    const double* tA = d.tab + (int64_t)b * 6 * H + 4 * H;
    const double* tB = tA + H;
    double mn = INFINITY;
    for (int i = t; i < W2; i += kBlock) mn = fmin(mn, E[i]);
    for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, kWave));
    if (lane_id() == 0) dred[t / kWave] = mn;
    __syncthreads();
    mn = dred[0];
    for (int w = 1; w < nwaves(); ++w) mn = fmin(mn, dred[w]);
    const bool any = !(fi.flags & (LD_FLAG_NOROAD | LD_FLAG_NOVP)) && mn < 0.0;
    const double thr = d.P.rho_lpv * mn;
    for (int i = t; i < W2; i += kBlock) {
        bool a = any && i >= 1 && i + 1 < W2 && E[i] < E[i - 1] && E[i] < E[i + 1] && E[i] < thr;
        alive[i] = a ? 1 : 0;
    }
    if (t == 0) s_nacc = 0;
    __syncthreads();
    const int dn = d.P.d_nms > 0 ? d.P.d_nms : max(8, d.W / 64);
    for (int it = 0; it < LD_MAX_LANES; ++it) {
        // argmin over the alive minima by (E, i); E is compared through its order-preserving
        // 64-bit image so that ties fall to the smaller index
        int64_t key = INT64_MAX;
        int idx = 0x7fffffff;
        for (int i = t; i < W2; i += kBlock)
            if (alive[i]) {
                const int64_t bits = __double_as_longlong(E[i]);
                const int64_t k = bits >= 0 ? bits : (bits ^ 0x7fffffffffffffffLL);
                if (k < key || (k == key && i < idx)) { key = k; idx = i; }
            }
        block_argmin_i64(key, idx, rv, ri);
        if (idx == 0x7fffffff) break;
        if (t == 0) acc[s_nacc++] = idx;
        for (int i = t; i < W2; i += kBlock)
            if (alive[i] && abs(i - idx) <= dn) alive[i] = 0;
        __syncthreads();
    }
    __syncthreads();
    const int n = s_nacc;
    if (t == 0) {
        for (int i = 1; i < n; ++i) {
            int x = acc[i], j = i - 1;
            while (j >= 0 && acc[j] > x) { acc[j + 1] = acc[j]; --j; }
            acc[j + 1] = x;
        }
        ld_lanes L;
        L.n = n;
        L.flags = fi.flags;
        L.v_h = fi.v_h;
        L.v_end = fi.v_end;
        for (int l = 0; l < LD_MAX_LANES; ++l) {
            L.u_start[l] = l < n ? acc[l] - d.half : 0;
            L.energy[l] = l < n ? (float)E[acc[l]] : 0.0f;
        }
        lanes_out[b] = L;
    }
    __syncthreads();
    if (curves_out) {
        float* cv = curves_out + (int64_t)b * LD_MAX_LANES * H;
        const float fnan = __int_as_float(0x7fc00000);
        for (int i = t; i < LD_MAX_LANES * H; i += kBlock) cv[i] = fnan;
        __syncthreads();
        if (t < n) {
            double u = (double)(acc[t] - d.half);
            for (int v = v_max; v >= fi.v_end; --v) {
                if (v < v_max) u = fma(tB[v], u, tA[v]);
                cv[(int64_t)t * H + v] = (float)u;
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Pruned search (learned part, not in the paper).  The network's decisions on a few bands of
// road rows (lbits) select the edges that lie on lane markings; their V_px vote columns give a
// seed for the V_px path, the DP then runs inside a window around the seed, and the tracks of
// the candidates through the bands decide which candidates are scored.  Any sign that the
// narrowed search may differ from the full one sends the frame back to the full search.
__device__ __forceinline__ int band_top(const Dev& d, int v_h, int nb, int k) { return ldi_band_top(v_h, d.H, nb, k); }

// Seed: per-band histograms of the vote columns of marking edges; pooled argmax c_s; window;
// RANSAC hypothesis 0 (line through the lowest and the highest band estimates).  One workgroup
// per frame; LDS 2 x 2W ints.
__global__ __launch_bounds__(kBlock) void k_seed(Dev d, int nb, int delta, int min_votes, int seed_ransac) {
    extern __shared__ int hs[];
    __shared__ int64_t rv[kMaxWaves];
    __shared__ int ri[kMaxWaves];
    __shared__ int red[kMaxWaves];
    const int b = blockIdx.x, t = threadIdx.x;
    if (frame_masked(d, b)) return;
    const int W = d.W, W2 = d.W2, H = d.H;
    const FrameInfo fi = d.info[b];
    int32_t* pr = d.prune + (int64_t)b * kPruneWords;
    double* sg = d.seedg + (int64_t)b * 5;
    int* hb = hs;          // band histogram
    int* hp = hs + W2;     // pooled histogram
    for (int i = t; i < 2 * W2; i += kBlock) hs[i] = 0;
    int est[LDI_MAX_BANDS], cnt[LDI_MAX_BANDS];
    for (int k = 0; k < LDI_MAX_BANDS; ++k) { est[k] = -1; cnt[k] = 0; }
    const bool road = !(fi.flags & LD_FLAG_NOROAD);
    const ld_edge* fe = d.edges + (int64_t)b * H * W;
    const uint8_t* lb = d.lbits + (int64_t)b * LDI_MAX_BANDS * LDI_BAND_ROWS * W;
    __syncthreads();
    for (int k = 0; k < nb && road; ++k) {
        const int top = band_top(d, fi.v_h, nb, k);
        if (top < 0) break;
        for (int r = 0; r < LDI_BAND_ROWS; ++r) {
            const int v = top + r, n = d.rowcnt[(int64_t)b * H + v];
            for (int i = t; i < n; i += kBlock) {
                const ld_edge e = fe[(int64_t)v * W + i];
                if (e.bin >= 0 && lb[(k * LDI_BAND_ROWS + r) * W + e.u]) {
                    atomicAdd(&hb[e.bin], 1);
                    atomicAdd(&hp[e.bin], 1);
                }
            }
        }
        __syncthreads();
        int64_t key = INT64_MAX;
        int bi = 0x7fffffff, tot = 0;
        for (int c = t; c < W2; c += kBlock) {
            const int h = hb[c];
            tot += h;
            if (h > 0 && -(int64_t)h < key) { key = -(int64_t)h; bi = c; }
            hb[c] = 0;
        }
        tot = block_sum_i32(tot, red);
        block_argmin_i64(key, bi, rv, ri);
        est[k] = tot > 0 ? bi : -1;
        cnt[k] = tot;
    }
    int64_t key = INT64_MAX;
    int bi = 0x7fffffff, tot = 0;
    for (int c = t; c < W2; c += kBlock) {
        const int h = hp[c];
        tot += h;
        if (h > 0 && -(int64_t)h < key) { key = -(int64_t)h; bi = c; }
    }
    tot = block_sum_i32(tot, red);
    block_argmin_i64(key, bi, rv, ri);
    if (t == 0) {
        int fb = 0, cs = -1, lo = 0, hi = -1;
        if (!road || tot < min_votes) {
            fb = kFbPlainVpx | kFbNoSeed;
        } else {
            cs = bi;
            lo = max(0, cs - delta);
            hi = min(W2 - 1, cs + delta);
            if (W < 128) fb = kFbPlainVpx | kFbNoSeed;   // the window backtrace needs 128 B per row
        }
        // hypothesis 0: line through the lowest and the highest band with min_votes votes
        int klo = -1, khi = -1;
        for (int k = 0; k < nb; ++k)
            if (cnt[k] >= min_votes) { if (klo < 0) klo = k; khi = k; }
        for (int p = 0; p < 5; ++p) sg[p] = 0.0;
        if (cs >= 0 && seed_ransac) {
            if (klo >= 0 && khi != klo) {
                const double v0 = (double)(band_top(d, fi.v_h, nb, klo) + 8), v1 = (double)(band_top(d, fi.v_h, nb, khi) + 8);
                const double u0 = (double)(est[klo] - d.half), u1 = (double)(est[khi] - d.half);
                const double g1 = (u1 - u0) / (v1 - v0);
                sg[1] = g1;
                sg[0] = u0 - g1 * v0;
            } else {
                sg[0] = (double)((klo >= 0 ? est[klo] : cs) - d.half);
            }
        } else {
            sg[0] = __longlong_as_double(0x7ff8000000000000LL);   // no seed
        }
        pr[0] = nb; pr[1] = fb; pr[2] = cs; pr[3] = lo; pr[4] = hi; pr[5] = tot;
        for (int k = 0; k < 4; ++k) { pr[6 + k] = est[k]; pr[10 + k] = cnt[k]; }
        pr[14] = 0; pr[15] = 0;
    }
}

// Windowed V_px search: band accumulator and row DP on columns lo..hi only (transitions
// leaving the window are not allowed), the same tie order as the full DP, backtrace, a check
// that the path never reaches an inner edge of the window.  One wave per frame: lane l keeps
// window columns 4l .. 4l+3 (16 E of the previous row and the column counts) in registers and
// takes the neighbours' values from lanes l-2 .. l+2 by DPP wave shifts, so a row needs no
// barrier; the band deltas of a row go through LDS atomics, from the road rows' vote columns
// staged in LDS before the sweep; the backtrace (the rank of tau, 4 bits per column,
// 128 B per row) goes to the frame's backtrace buffer and is walked 32 rows at a time from
// registers.  Needs W >= 128 (the buffer holds W bytes per row); narrower frames use the full
// search.
constexpr int kWalkChunk = 32;

__device__ __forceinline__ int shfl_i(int x, int src) { return __shfl(x, src, kWave); }
__device__ __forceinline__ int min3_i(int a, int b, int c) { return min(min(a, b), c); }
// x of lane l - 1 (kBig on lane 0) and of lane l + 1 (kBig on lane 63): DPP wave shifts by one
__device__ __forceinline__ int lane_prev(int x) { return __builtin_amdgcn_update_dpp(kBig, x, 0x138, 0xF, 0xF, false); }
__device__ __forceinline__ int lane_next(int x) { return __builtin_amdgcn_update_dpp(kBig, x, 0x130, 0xF, 0xF, false); }
// the same shifts filling with 0 (lane 0, lane 63)
__device__ __forceinline__ int lane_prev0(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int lane_next0(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true); }
constexpr int kBig16 = 0x3FFFFFF0;

__global__ __launch_bounds__(256) void k_vpx_window(Dev d, int stage_cap, int wave_bytes, int nframes) {
    extern __shared__ unsigned char smem_all[];
    // blockDim.x / 64 frames per workgroup, one per wave with its own LDS slice: the waves of
    // a workgroup go to different SIMDs, so a batch of four frames per CU runs one wave per SIMD
    // the frame's values are wave-uniform: kept in scalar registers, so every loop below
    // branches on scalars
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int b = (int)blockIdx.x * (int)(blockDim.x / kWave) + wv, l = lane_id();
    if (b >= nframes || frame_masked(d, b)) return;
    unsigned char* smem = smem_all + (size_t)wv * wave_bytes;
    int32_t* pr = d.prune + (int64_t)b * kPruneWords;
    if (__builtin_amdgcn_readfirstlane(pr[1]) & kFbPlainVpx) return;
    const int H = d.H, W2 = d.W2, v_max = H - 1;
    FrameInfo fi = d.info[b];
    for (int v = l; v < H; v += kWave) d.mxpath[(int64_t)b * H + v] = -1;
    const int v_h = __builtin_amdgcn_readfirstlane(fi.v_h), chi = d.P.chi, R = v_max - v_h + 1;
    const int lo = __builtin_amdgcn_readfirstlane(pr[3]), hi = __builtin_amdgcn_readfirstlane(pr[4]);
    const int win = hi - lo + 1;
    int* dlt = reinterpret_cast<int*>(smem);                 // 256 band deltas of a row + 64 lane sinks
    int* cntL = dlt + 256 + kWave;                            // H
    int* path = cntL + H;                                     // H + 1 (the last: touch flag)
    int* roff = path + H + 1;                                 // R + 1 <= H + 1
    uint8_t* wb = reinterpret_cast<uint8_t*>(roff + H + 1);               // stage_cap bytes
    uint16_t* back = reinterpret_cast<uint16_t*>(d.back_x) + (int64_t)b * H * ((W2 + kDpRun - 1) / kDpRun) * 2;
    const ld_edge* fe = d.edges + (int64_t)b * H * d.W;
    // the road rows' edge counts (the search reads no other row), eight loads per lane in
    // flight before the first is stored
    for (int base = 0; base < R; base += 8 * kWave) {
        int cn[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) cn[k] = d.rowcnt[(int64_t)b * H + v_h + min(base + k * kWave + l, R - 1)];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (base + k * kWave + l < R) cntL[v_h + base + k * kWave + l] = cn[k];
    }
    for (int i = l; i < 256; i += kWave) dlt[i] = 0;
    {   // exclusive prefix of the road rows' edge counts, 64 rows per wave scan
        int carry = 0;
        for (int base = 0; base < R; base += kWave) {
            const int own = base + l < R ? cntL[v_h + base + l] : 0;
            int x = own;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(x, o, kWave);
                if (l >= o) x += y;
            }
            if (base + l < R) roff[base + l] = carry + x - own;
            carry += __shfl(x, kWave - 1, kWave);
        }
        if (l == 0) roff[R] = carry;
    }
    const int ne = __builtin_amdgcn_readfirstlane(roff[R]);
    // window offset of every road edge's vote column (255: outside the window or no vote),
    // loaded eight rows at a time with every load of the group in flight
    const bool staged = ne <= stage_cap;
    auto woff = [&](int c) -> uint8_t { return (c >= lo && c <= hi) ? (uint8_t)(c - lo) : (uint8_t)255; };
    int nv = 0;
    if (staged) {
        // Groups of 16 rows, two in flight while a third is written to LDS: lane l loads the
        // vote columns of entries l and l + 64 of every row of a group (the window search needs
        // W >= 128, so both lie in the row's slots; entries past the row's count and rows past
        // v_max, read as row v_max, are loaded and not used).  The two register sets are
        // written in turn, so no copy waits on loads in flight.  Lane l holds the count and
        // offset (offset << 16 | count) of row v_h + 64 m + l of the current 64-row chunk m.
        uint8_t* junk = reinterpret_cast<uint8_t*>(dlt + 256 + l);   // stores of lanes without an entry
        const int ng = (R + 15) / 16;
        auto load_group = [&](int g, int (&c)[16][2]) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const ld_edge* row = fe + (int64_t)min(v_h + 16 * g + k, v_max) * d.W;
                c[k][0] = row[l].bin;
                c[k][1] = row[l + kWave].bin;
            }
        };
        int desc = 0;
        auto store_group = [&](int g, const int (&c)[16][2]) {
            if ((g & 3) == 0) {
                const int r = 16 * g + l;
                desc = r < R ? (roff[r] << 16 | cntL[v_h + r]) : 0;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int r = 16 * g + k;
                if (r >= R) break;
                const int rd = __builtin_amdgcn_readlane(desc, r & 63);
                const int n = rd & 0xFFFF, o = rd >> 16;
                const bool e0 = l < n, e1 = l + kWave < n;
                nv += (e0 && c[k][0] >= 0 ? 1 : 0) + (e1 && c[k][1] >= 0 ? 1 : 0);
                *(e0 ? wb + o + l : junk) = woff(c[k][0]);
                *(e1 ? wb + o + l + kWave : junk) = woff(c[k][1]);
                if (n > 2 * kWave) {                 // long rows: 8 loads in flight
                    const int v = v_h + r;
                    for (int i0 = l + 2 * kWave; i0 < n; i0 += 8 * kWave) {
                        int cc[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int i = i0 + j * kWave;
                            cc[j] = i < n ? fe[(int64_t)v * d.W + i].bin : -1;
                        }
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int i = i0 + j * kWave;
                            if (i < n) {
                                nv += cc[j] >= 0 ? 1 : 0;
                                wb[o + i] = woff(cc[j]);
                            }
                        }
                    }
                }
            }
        };
        int ca[16][2], cb[16][2];
        load_group(0, ca);
        load_group(1, cb);
        for (int g = 0; g < ng; g += 2) {
            store_group(g, ca);
            load_group(g + 2, ca);
            if (g + 1 < ng) store_group(g + 1, cb);
            load_group(g + 3, cb);
        }
    } else {
        for (int v = v_h; v <= v_max; ++v)
            for (int i = l; i < cntL[v]; i += kWave) nv += fe[(int64_t)v * d.W + i].bin >= 0 ? 1 : 0;
    }
    // band rows entering (sign +1) or leaving (-1) the accumulator
    auto apply = [&](int r, int sign) {
        const int n = cntL[r];
        const int o = staged ? roff[r - v_h] : 0;
        for (int base = 0; base < n; base += kWave) {
            const int i = base + l;
            int key = -1;
            if (i < n) {
                if (staged) {
                    const int c = wb[o + i];
                    key = c != 255 ? c : -1;
                } else {
                    const int c = fe[(int64_t)r * d.W + i].bin;
                    key = (c >= lo && c <= hi) ? c - lo : -1;
                }
            }
            if (key >= 0) atomicAdd(&dlt[key], sign);
        }
    };
    for (int r = max(v_max - chi, v_h); r <= v_max; ++r) apply(r, 16);
    // S = 16 E of the own columns (kBig16 outside the window), H = 16 x the column's band count
    // (the deltas are applied in units of 16); the registers hold S - kBig16, so the columns
    // outside the window and beyond the wave's ends are 0 and the wave shifts fill with 0.
    // kBig16 is a multiple of 16, so the rank bits and the update below are unchanged by the
    // offset, and it exceeds every reachable |16 E|.  A candidate from column c + tau costs
    // S(c + tau) + slope |tau| - [tau < 0] with slope = 16 lambda + 2, i.e. 16 (E + lambda |tau|)
    // plus the rank of tau in the tie order 0, -1, +1, -2, +2, ..., so one min picks the cost
    // and the tie; offsets are taken relative to the lane's first column 4l.
    int Hc[4], S[4];
    bool inw[4];
    {
        const int4 q = *reinterpret_cast<const int4*>(dlt + 4 * l);
        Hc[0] = q.x; Hc[1] = q.y; Hc[2] = q.z; Hc[3] = q.w;
        *reinterpret_cast<int4*>(dlt + 4 * l) = make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        inw[j] = 4 * l + j < win;
        S[j] = inw[j] ? -Hc[j] - kBig16 : 0;
    }
    const int tau_max = d.P.tau_x_max, slope = 16 * d.P.lambda_x + 2;
    // one row of the DP from the previous row's S and this row's H (returns the 4-bit ranks)
    auto dp_row = [&]() -> uint32_t {
        // w[p] = S of column 4l - 5 + p of the previous row (p = 0 .. 13)
        int w[14];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w[1 + j] = lane_prev0(S[j]);
            w[5 + j] = S[j];
            w[9 + j] = lane_next0(S[j]);
        }
        w[0] = lane_prev0(w[4]);
        w[13] = lane_next0(w[9]);
        int lm[4], rm[4];
        if (tau_max == 5) {
            // TL[p] = w[p] + slope (5 - p) for p = 0 .. 7 and TR[p] = w[p] + slope (p - 5) for
            // p = 6 .. 13; the minima over five consecutive entries share their middle terms
            int TL[8], TR[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                TL[p] = w[p] + slope * (5 - p);
                TR[p] = w[p + 6] + slope * (p + 1);
            }
            const int cl = min3_i(TL[2], TL[3], TL[4]);
            lm[0] = min3_i(TL[0], TL[1], cl);
            lm[1] = min3_i(TL[1], cl, TL[5]);
            lm[2] = min3_i(cl, TL[5], TL[6]);
            lm[3] = min3_i(TL[3], TL[4], min3_i(TL[5], TL[6], TL[7]));
            const int cr = min3_i(TR[2], TR[3], TR[4]);
            rm[0] = min3_i(TR[0], TR[1], cr);
            rm[1] = min3_i(TR[1], cr, TR[5]);
            rm[2] = min3_i(cr, TR[5], TR[6]);
            rm[3] = min3_i(TR[3], TR[4], min3_i(TR[5], TR[6], TR[7]));
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                lm[j] = 0; rm[j] = 0;
#pragma unroll
                for (int a = 1; a <= 5; ++a)
                    if (a <= tau_max) {
                        lm[j] = min(lm[j], w[j + 5 - a] + slope * (a - j));
                        rm[j] = min(rm[j], w[j + 5 + a] + slope * (a + j));
                    }
            }
        }
        uint32_t bits = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int key = min3_i(w[5 + j], lm[j] + (slope * j - 1), rm[j] - slope * j);
            S[j] = inw[j] ? (key & ~15) - Hc[j] : 0;
            bits |= (uint32_t)(key & 15) << (4 * j);
        }
        return bits;
    };
    auto take_deltas = [&]() {
        // the wave's LDS operations complete in order: the deltas are final here
        const int4 q = *reinterpret_cast<const int4*>(dlt + 4 * l);
        *reinterpret_cast<int4*>(dlt + 4 * l) = make_int4(0, 0, 0, 0);
        Hc[0] += q.x; Hc[1] += q.y; Hc[2] += q.z; Hc[3] += q.w;
    };
    if (staged) {
        // Row v (v = v_max - 1 - t) adds the votes of row v - chi and removes those of row
        // v + chi + 1.  Lane l holds the two lists' heads (offset << 16 | count) of row
        // t0 + l of the current 64-row chunk, taken by readlane; the own entries of the next
        // row's lists are read while the current row is computed.  Lanes without an entry
        // add to their own sink word.
        int* sink = dlt + 256 + l;
        auto heads = [&](int t0, int& hA, int& hR) {
            const int v = v_max - 1 - t0 - l, ra = v - chi, rr = v + chi + 1;
            hA = (v >= v_h && ra >= v_h) ? (roff[ra - v_h] << 16 | cntL[ra]) : 0;
            hR = (v >= v_h && rr <= v_max) ? (roff[rr - v_h] << 16 | cntL[rr]) : 0;
        };
        auto own_slot = [&](int hd) -> int* {
            const int n = hd & 0xFFFF, o = hd >> 16;
            const int c = wb[l < n ? o + l : 0];
            return (l < n && c != 255) ? dlt + c : sink;
        };
        int hA, hR;
        heads(0, hA, hR);
        int* pA = own_slot(__builtin_amdgcn_readlane(hA, 0));
        int* pR = own_slot(__builtin_amdgcn_readlane(hR, 0));
        for (int t = 0; t < R - 1; ++t) {
            const int v = v_max - 1 - t;
            const int cA = __builtin_amdgcn_readlane(hA, t & 63), cR = __builtin_amdgcn_readlane(hR, t & 63);
            atomicAdd(pA, 16);
            atomicAdd(pR, -16);
            const int nA = cA & 0xFFFF, nR = cR & 0xFFFF;
            for (int i0 = kWave; i0 < max(nA, nR); i0 += kWave) {     // long lists
                const int i = i0 + l;
                const int ca = i < nA ? wb[(cA >> 16) + i] : 255;
                const int cr = i < nR ? wb[(cR >> 16) + i] : 255;
                atomicAdd(ca != 255 ? dlt + ca : sink, 16);
                atomicAdd(cr != 255 ? dlt + cr : sink, -16);
            }
            if (((t + 1) & 63) == 0) heads(t + 1, hA, hR);
            pA = own_slot(__builtin_amdgcn_readlane(hA, (t + 1) & 63));
            pR = own_slot(__builtin_amdgcn_readlane(hR, (t + 1) & 63));
            take_deltas();
            back[(int64_t)(v - v_h) * kWave + l] = (uint16_t)dp_row();
        }
    } else {
        for (int v = v_max - 1; v >= v_h; --v) {
            if (v - chi >= v_h) apply(v - chi, 16);
            if (v + chi + 1 <= v_max) apply(v + chi + 1, -16);
            take_deltas();
            back[(int64_t)(v - v_h) * kWave + l] = (uint16_t)dp_row();
        }
    }
    // start column: argmin over the window of E at v_h, ties to the smaller column
    int64_t bv = INT64_MAX;
    int bc = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (4 * l + j < win && (int64_t)(S[j] >> 4) < bv) { bv = S[j] >> 4; bc = 4 * l + j; }
    wave_argmin_i64(bv, bc);
    __threadfence_block();   // the backtrace stores are complete before the wave reads them back
    // Walk: the backtrace words of kWalkChunk rows in registers (lane l holds columns
    // 4l .. 4l+3 of each row) with the next chunk in flight; the column is wave-uniform, so a
    // step is a readlane and a few scalar operations.  Lane r keeps the path of row v0 + r.
    int c = __builtin_amdgcn_readfirstlane(bc), touch = 0;
    auto load_chunk = [&](int v0, uint32_t (&dst)[kWalkChunk]) {
#pragma unroll
        for (int r = 0; r < kWalkChunk; ++r) {
            const int v = min(v0 + r, v_max - 1);          // rows v < v_max hold an entry
            dst[r] = back[(int64_t)max(v - v_h, 0) * kWave + l];
        }
    };
    auto walk_chunk = [&](int v0, const uint32_t (&bk)[kWalkChunk]) {
        int pv = 0;
#pragma unroll
        for (int r = 0; r < kWalkChunk; ++r) {
            const int v = v0 + r;
            if (v <= v_max) {
                if (l == r) pv = lo + c;
                if (v < v_max) {
                    const uint32_t word = __builtin_amdgcn_readlane(bk[r], c >> 2);
                    const int rank = (int)((word >> (4 * (c & 3))) & 15u);
                    c += (int)((kRankTau >> (4 * rank)) & 15u) - 8;
                }
            }
        }
        if (l < kWalkChunk && v0 + l <= v_max) path[v0 + l] = pv;
    };
    // two chunks in flight, the register sets written in turn (row loads are clamped, so
    // every chunk is a full set of loads)
    uint32_t ba[kWalkChunk], bb[kWalkChunk];
    load_chunk(v_h, ba);
    load_chunk(v_h + kWalkChunk, bb);
    for (int v0 = v_h; v0 <= v_max; v0 += 2 * kWalkChunk) {
        walk_chunk(v0, ba);
        load_chunk(v0 + 2 * kWalkChunk, ba);
        if (v0 + kWalkChunk <= v_max) walk_chunk(v0 + kWalkChunk, bb);
        load_chunk(v0 + 3 * kWalkChunk, bb);
    }
    // the path touches an inner edge of the window (a column the window cut off could have
    // been reached): the frame goes back to the full search
    for (int v = v_h + l; v <= v_max; v += kWave) {
        const int pc = path[v];
        if ((lo > 0 && pc == lo) || (hi < W2 - 1 && pc == hi)) touch = 1;
    }
    touch = __any(touch) ? 1 : 0;
    nv = wave_sum_i32(nv);
    if (touch) {
        if (l == 0) pr[1] |= kFbPlainVpx | kFbTouch;
        return;
    }
    for (int v = v_h + l; v <= v_max; v += kWave) d.mxpath[(int64_t)b * H + v] = path[v];
    if (l == 0) {
        fi.n_edges = ne;
        fi.n_votes = nv;
        d.info[b] = fi;
    }
}

// Candidate mask: candidate i is kept when its track meets a marking pixel on a band row, then
// dilated.  Frames on the plain V_px search keep every candidate.  One workgroup per frame.
__global__ __launch_bounds__(kBlock) void k_cand_mask(Dev d, int nb, int dilate) {
    extern __shared__ unsigned char smem[];
    __shared__ double ta[LDI_MAX_BANDS * LDI_BAND_ROWS], tb[LDI_MAX_BANDS * LDI_BAND_ROWS];
    __shared__ int red[kMaxWaves];
    const int b = blockIdx.x, t = threadIdx.x;
    if (frame_masked(d, b)) return;
    const int W = d.W, W2 = d.W2, H = d.H, v_max = H - 1;
    int32_t* pr = d.prune + (int64_t)b * kPruneWords;
    uint8_t* cm = d.cmask + (int64_t)b * W2;
    const FrameInfo fi = d.info[b];
    if ((pr[1] & kFbPlainVpx) || (fi.flags & (LD_FLAG_NOROAD | LD_FLAG_NOVP)) || dilate < 0) {
        for (int i = t; i < W2; i += kBlock) cm[i] = 1;
        if (t == 0) pr[14] = W2;
        return;
    }
    const int wpr = (W + 31) / 32;
    uint32_t* bits = reinterpret_cast<uint32_t*>(smem);            // nb x 16 x wpr
    uint8_t* hit = reinterpret_cast<uint8_t*>(bits + nb * LDI_BAND_ROWS * wpr);   // W2
    const uint8_t* lb = d.lbits + (int64_t)b * LDI_MAX_BANDS * LDI_BAND_ROWS * W;
    for (int w = t; w < nb * LDI_BAND_ROWS * wpr; w += kBlock) {
        const int row = w / wpr, c0 = (w % wpr) * 32;
        uint32_t x = 0;
        for (int j = 0; j < 32 && c0 + j < W; ++j) x |= (lb[row * W + c0 + j] ? 1u : 0u) << j;
        bits[w] = x;
    }
    const double* tA = d.tab + (int64_t)b * 6 * H + 4 * H;
    const double* tB = tA + H;
    const int v_end = fi.v_end;
    const int top_hi = band_top(d, fi.v_h, nb, nb - 1);
    if (t == 0) {
        double a = 1.0, c = 0.0;
        for (int v = v_max; v >= top_hi; --v) {
            if (v < v_max) {
                a = tB[v] * a;
                c = fma(tB[v], c, tA[v]);
            }
            for (int k = 0; k < nb; ++k) {
                const int r = v - band_top(d, fi.v_h, nb, k);
                if (r >= 0 && r < LDI_BAND_ROWS) { ta[k * LDI_BAND_ROWS + r] = a; tb[k * LDI_BAND_ROWS + r] = c; }
            }
        }
    }
    __syncthreads();
    for (int i = t; i < W2; i += kBlock) {
        const double us = (double)(i - d.half);
        uint8_t h = 0;
        for (int k = 0; k < nb && !h; ++k) {
            const int top = band_top(d, fi.v_h, nb, k);
            for (int r = 0; r < LDI_BAND_ROWS; ++r) {
                if (top + r < v_end) continue;
                const double x = fma(ta[k * LDI_BAND_ROWS + r], us, tb[k * LDI_BAND_ROWS + r]) + 0.5;
                if (x >= 0.0 && x < (double)W) {
                    const int col = (int)floor(x);
                    if ((bits[(k * LDI_BAND_ROWS + r) * wpr + (col >> 5)] >> (col & 31)) & 1u) { h = 1; break; }
                }
            }
        }
        hit[i] = h;
    }
    __syncthreads();
    int kept = 0;
    for (int i = t; i < W2; i += kBlock) {
        uint8_t k = 0;
        for (int j = max(0, i - dilate); j <= min(W2 - 1, i + dilate); ++j) k |= hit[j];
        cm[i] = k;
        kept += k;
    }
    kept = block_sum_i32(kept, red);
    if (t == 0) pr[14] = kept;
}

// After the masked energies and peaks: a frame on the narrowed search falls back to the full
// energies when it found no lane or a lane sits next to a pruned candidate.  Marks
// LD_FLAG_FALLBACK on every frame that used any part of the full search.
__global__ void k_lane_check(Dev d, ld_lanes* lanes, int nframes, int pruning) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nframes || frame_masked(d, b)) return;
    int32_t* pr = d.prune + (int64_t)b * kPruneWords;
    const uint8_t* cm = d.cmask + (int64_t)b * d.W2;
    int fb = pr[1];
    const FrameInfo fi = d.info[b];
    if (!pruning) pr[14] = d.W2;        // candidates kept: all
    if (pruning && !(fb & kFbPlainVpx) && !(fi.flags & (LD_FLAG_NOROAD | LD_FLAG_NOVP))) {
        const int n = lanes[b].n;
        bool bad = n == 0;
        for (int l = 0; l < n; ++l) {
            const int i = lanes[b].u_start[l] + d.half;
            bad = bad || cm[i - 1] == 0 || cm[i + 1] == 0;
        }
        if (bad) fb |= kFbPlainEnergy;
    }
    pr[1] = fb;
    if (fb & (kFbPlainVpx | kFbPlainEnergy)) {
        d.info[b].flags = fi.flags | LD_FLAG_FALLBACK;
        lanes[b].flags |= LD_FLAG_FALLBACK;
    }
}

}  // namespace

// ==========================================================================================
// Host side: frame objects and the C ABI.
// k_vdisp_hist, k_vdisp_fit, k_edges, k_vpx_fit, k_energy, k_peaks, then the pruned search:
// k_cnn_fwd, k_seed, k_vpx_window, k_cand_mask + k_lane_check, then k_vpx_ransac
constexpr int kNumKernels = 11;

struct ProfEvent {
    int kernel;
    hipEvent_t start, stop;
};

struct ld_frame_s {
    Dev d;
    bool prof = false;                  // bracket every kernel launch with HIP events
    std::vector<ProfEvent> pending;     // recorded, not yet read
    std::vector<ProfEvent> pool;        // reusable event pairs
    double acc_ms[kNumKernels] = {};
    int64_t calls[kNumKernels] = {};
    int batch;          // allocated frames
    int active;         // frames processed by the next calls
    void* mem;          // one device allocation holding all scratch
    size_t mem_bytes;
    int device;
    hipStream_t last;
    int stage;          // 0 nothing, 1 vdisp done, 2 vp done, 3 energy done
    int bands;          // bands of the last network decisions (0 none since the last ld_vdisp)
};

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int elem_size(int fmt) { return fmt == LD_DISP_U8 ? 1 : (fmt == LD_DISP_F32 ? 4 : 2); }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

ld_status launch_ok() { return hipGetLastError() == hipSuccess ? LD_OK : LD_E_HIP; }

// Optional per-kernel timing: an event pair on the launch stream around one kernel.
struct ProfScope {
    ld_frame f;
    int kernel;
    hipStream_t st;
    ProfEvent ev;
    bool on;
    ProfScope(ld_frame f_, int k, hipStream_t s) : f(f_), kernel(k), st(s), on(f_->prof) {
        if (!on) return;
        if (f->pool.empty()) {
            ProfEvent e;
            e.kernel = 0;
            if (hipEventCreate(&e.start) != hipSuccess || hipEventCreate(&e.stop) != hipSuccess) { on = false; return; }
            f->pool.push_back(e);
        }
        ev = f->pool.back();
        f->pool.pop_back();
        ev.kernel = kernel;
        (void)hipEventRecord(ev.start, st);
    }
    ~ProfScope() {
        if (!on) return;
        (void)hipEventRecord(ev.stop, st);
        f->pending.push_back(ev);
    }
};

int vdisp_fit_threads(const Dev& d) {
    return std::min(1024, std::max(256, ((d.H + kVdRows - 1) / kVdRows + 63) / 64 * 64));
}

size_t vdisp_fit_lds(const Dev& d) {
    return sizeof(int) * (2 * ((size_t)d.H + kVdPad) + 4 * (size_t)d.D1) + sizeof(uint32_t) * ((d.H + 31) / 32) +
           (size_t)kVdWalk * kVdWalkCols;
}

int vpx_fit_threads(const Dev& d) {
    const int runs = (d.W2 + kDpRun - 1) / kDpRun;
    return std::min(1024, std::max(64, (runs + 63) / 64 * 64));
}

// the compile-time run count k_vpx_fit<512, NRC> uses for this width (0: none fits)
int vpx_fit_nrc(const Dev& d) {
    const int nr = (d.W2 + kDpRun - 1) / kDpRun + 2;
    for (int c : {64, 128, 256, 320, 512})
        if (nr <= c) return c;
    return 0;
}

size_t vpx_fit_lds(const Dev& d) {
    const int nrc = vpx_fit_nrc(d);
    const size_t WP = (size_t)kDpRun * (nrc > 0 ? nrc : (d.W2 + kDpRun - 1) / kDpRun + 2);
    return sizeof(int) * (3 * WP + (size_t)d.H);
}

size_t edges_lds(int nwaves) {
    return (sizeof(double) + 3 * sizeof(uint32_t)) * kEdgeStrip + sizeof(uint2) * kEdgeQueue * (size_t)nwaves;
}

size_t energy_lds(int nc) { return sizeof(float) * (6 * (size_t)nc * kBlock + 10); }

// Raise a kernel's dynamic LDS limit once per size (later launches, including those recorded
// into a captured graph, issue nothing but the launch).
template <typename K>
void allow_lds(K kernel, size_t bytes) {
    static size_t granted = 0;   // one counter per kernel instantiation
    if (bytes > 32 * 1024 && bytes > granted) {
        if (hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
            granted = bytes;
        else
            (void)hipGetLastError();
    }
}

constexpr int kRegions = 18;

// Byte offsets and sizes of the regions of one frame object's device allocation.
size_t frame_layout(int width, int height, int batch, int d_max, size_t* off, size_t* sz) {
    const size_t B = (size_t)batch, H = (size_t)height, W = (size_t)width, D1 = (size_t)d_max + 1, W2 = 2 * (size_t)width;
    const size_t s[kRegions] = {
        B * D1 * ((H + 31) / 32 * 32) * 4,   // myT (rows padded to 32)
        B * D1 * H,                     // back_y
        B * 2 * D1 * 4,                 // my_pts
        B * 2 * sizeof(FitRes),         // fit
        B * sizeof(FrameInfo),          // info
        B * 6 * H * 8,                  // tab
        B * H * 4,                      // rowcnt
        B * H * W * sizeof(ld_edge),    // edges
        B * H * ((W2 + kDpRun - 1) / kDpRun) * 4,   // back_x (4 bits per column)
        B * H * 4,                      // mxpath
        B * W2 * 8,                     // energy
        B * 6 * kMaxRounds * 4,         // trace
        B * H * W * 4,                  // qbuf
        B * H * 2 * 4,                  // rbound
        B * LDI_MAX_BANDS * LDI_BAND_ROWS * W,   // lbits
        B * kPruneWords * 4,            // prune
        B * W2,                         // cmask
        B * 5 * 8,                      // seedg
    };
    size_t o = 0;
    for (int i = 0; i < kRegions; ++i) {
        sz[i] = s[i];
        off[i] = o;
        o += align_up(s[i]);
    }
    return o;
}

ld_status check_params(const ld_params& p) {
    if (p.chi < 0 || p.tau_y_max < 0 || p.tau_y_max > 255 || p.tau_x_max < 0 || p.tau_x_max > 5) return LD_E_INVAL;
    if (p.lambda_y < 0 || p.lambda_x < 0 || p.lambda_y > 1000 || p.lambda_x > 1000) return LD_E_INVAL;
    if (p.n_hyp < 1 || p.n_hyp > kMaxHyp || p.max_rounds < 1 || p.max_rounds > kMaxRounds) return LD_E_INVAL;
    if (p.eps_num < 0 || p.eps_den < 1 || p.edge_t < 0 || p.edge_t > 46340) return LD_E_INVAL;
    if (p.nu != 1 || p.varsigma != 3) return LD_E_INVAL;    // the kernels are built for the paper's box
    if (!(p.sigma_g > 0.0) || !(p.tr_x >= 0.0) || !(p.tr_y >= 0.0) || !(p.varpi >= 0.0)) return LD_E_INVAL;
    if (p.d_nms < 0 || (p.weight_squared != 0 && p.weight_squared != 1) || (p.vote != 0 && p.vote != 1))
        return LD_E_INVAL;
    return LD_OK;
}

// Point the scratch fields of d at the regions of one allocation laid out by frame_layout.
void bind_regions(Dev& d, char* base, const size_t* off) {
    d.myT = reinterpret_cast<int32_t*>(base + off[0]);
    d.back_y = reinterpret_cast<uint8_t*>(base + off[1]);
    d.my_pts = reinterpret_cast<int32_t*>(base + off[2]);
    d.fit = reinterpret_cast<FitRes*>(base + off[3]);
    d.info = reinterpret_cast<FrameInfo*>(base + off[4]);
    d.tab = reinterpret_cast<double*>(base + off[5]);
    d.rowcnt = reinterpret_cast<int32_t*>(base + off[6]);
    d.edges = reinterpret_cast<ld_edge*>(base + off[7]);
    d.back_x = reinterpret_cast<int8_t*>(base + off[8]);
    d.mxpath = reinterpret_cast<int32_t*>(base + off[9]);
    d.energy = reinterpret_cast<double*>(base + off[10]);
    d.trace = reinterpret_cast<int32_t*>(base + off[11]);
    d.qbuf = reinterpret_cast<float*>(base + off[12]);
    d.rbound = reinterpret_cast<uint32_t*>(base + off[13]);
    d.lbits = reinterpret_cast<uint8_t*>(base + off[14]);
    d.prune = reinterpret_cast<int32_t*>(base + off[15]);
    d.cmask = reinterpret_cast<uint8_t*>(base + off[16]);
    d.seedg = reinterpret_cast<double*>(base + off[17]);
    d.nact = nullptr;
    d.only = nullptr;
    d.only_bits = 0;
    d.only_set = 0;
}

// Sizes, parameters and derived launch constants of a frame object (no device memory).
ld_status init_dev(Dev& d, int32_t width, int32_t height, int32_t batch, int32_t fmt, int32_t d_max,
                   const ld_params* p) {
    if (width < 8 || width > 4096 || height < 8 || height > 4096 || batch < 1 || batch > 65535) return LD_E_INVAL;
    if (fmt < 0 || fmt > 2 || d_max < 1 || d_max > 1023) return LD_E_INVAL;
    ld_params P;
    ld_params_default(&P);
    if (p) P = *p;
    if (check_params(P) != LD_OK) return LD_E_INVAL;
    // the row DP keeps (E << 4 | rank) in int32: E >= -width * height * (2 chi + 1)
    if ((int64_t)width * height * (2 * (int64_t)P.chi + 1) + 5 * (int64_t)P.lambda_x >= ((int64_t)1 << 27)) return LD_E_INVAL;
    d.W = width; d.H = height; d.D1 = d_max + 1; d.W2 = 2 * width; d.half = width / 2; d.fmt = fmt;
    d.d_max = d_max; d.B = batch; d.P = P;
    d.hist_rows = std::max(kHistGroup, std::min(32, (8192 / d.D1) / kHistGroup * kHistGroup));
    d.Hm = (height + 31) / 32 * 32;
    return LD_OK;
}

template <int FMT>
void launch_hist(int npt, dim3 g, size_t lds, hipStream_t st, const Dev& d, const uint8_t* dp, int64_t pitch,
                 int32_t* out) {
    if (npt <= 1) hipLaunchKernelGGL((k_vdisp_hist<FMT, 1>), g, dim3(kBlock), lds, st, d, dp, pitch, out);
    else if (npt <= 2) hipLaunchKernelGGL((k_vdisp_hist<FMT, 2>), g, dim3(kBlock), lds, st, d, dp, pitch, out);
    else if (npt <= 4) hipLaunchKernelGGL((k_vdisp_hist<FMT, 4>), g, dim3(kBlock), lds, st, d, dp, pitch, out);
    else if (npt <= 5) hipLaunchKernelGGL((k_vdisp_hist<FMT, 5>), g, dim3(kBlock), lds, st, d, dp, pitch, out);
    else if (npt <= 8) hipLaunchKernelGGL((k_vdisp_hist<FMT, 8>), g, dim3(kBlock), lds, st, d, dp, pitch, out);
    else hipLaunchKernelGGL((k_vdisp_hist<FMT, 16>), g, dim3(kBlock), lds, st, d, dp, pitch, out);
}

// S1 for the active frames of f
ld_status run_hist(ld_frame f, const void* disp, int64_t pitch, int32_t* vdisp_out, hipStream_t st) {
    Dev& d = f->d;
    dim3 g1((d.H + d.hist_rows - 1) / d.hist_rows, f->active);
    const size_t l1 = sizeof(int) * d.hist_rows * d.D1;
    const uint8_t* dp = static_cast<const uint8_t*>(disp);
    ProfScope ps(f, 0, st);
    const int npt = (d.W + kBlock - 1) / kBlock;
    if (d.fmt == LD_DISP_U8) launch_hist<LD_DISP_U8>(npt, g1, l1, st, d, dp, pitch, vdisp_out);
    else if (d.fmt == LD_DISP_F32) launch_hist<LD_DISP_F32>(npt, g1, l1, st, d, dp, pitch, vdisp_out);
    else launch_hist<LD_DISP_U16Q4>(npt, g1, l1, st, d, dp, pitch, vdisp_out);
    return launch_ok();
}

// S2-S3 for the active frames of f
ld_status run_vdisp_fit(ld_frame f, const uint64_t* sid, const int64_t* fidx, double* beta_out, hipStream_t st) {
    Dev& d = f->d;
    const size_t l2 = vdisp_fit_lds(d);
    allow_lds(k_vdisp_fit, l2);
    {
        ProfScope ps(f, 1, st);
        hipLaunchKernelGGL(k_vdisp_fit, dim3(f->active), dim3(vdisp_fit_threads(d)), l2, st, d, sid, fidx, beta_out);
    }
    return launch_ok();
}

ld_status run_vdisp(ld_frame f, const void* disp, int64_t pitch, const uint64_t* sid, const int64_t* fidx,
                    int32_t* vdisp_out, double* beta_out, hipStream_t st) {
    const ld_status s = run_hist(f, disp, pitch, vdisp_out, st);
    return s == LD_OK ? run_vdisp_fit(f, sid, fidx, beta_out, st) : s;
}

ld_status run_edges(ld_frame f, const uint8_t* grey, int64_t gp, const void* disp, int64_t dpt, hipStream_t st) {
    Dev& d = f->d;
    const int nw = (d.W + kEdgeCols - 1) / kEdgeCols;
    dim3 g3((d.H + kEdgeStrip - 1) / kEdgeStrip, f->active);
    const size_t lds = edges_lds(nw);
    const uint8_t* dp = static_cast<const uint8_t*>(disp);
    ProfScope ps(f, 2, st);
    if (d.fmt == LD_DISP_U8) {
        allow_lds(k_edges<LD_DISP_U8>, lds);
        hipLaunchKernelGGL(k_edges<LD_DISP_U8>, g3, dim3(nw * kWave), lds, st, d, grey, gp, dp, dpt);
    } else if (d.fmt == LD_DISP_F32) {
        allow_lds(k_edges<LD_DISP_F32>, lds);
        hipLaunchKernelGGL(k_edges<LD_DISP_F32>, g3, dim3(nw * kWave), lds, st, d, grey, gp, dp, dpt);
    } else {
        allow_lds(k_edges<LD_DISP_U16Q4>, lds);
        hipLaunchKernelGGL(k_edges<LD_DISP_U16Q4>, g3, dim3(nw * kWave), lds, st, d, grey, gp, dp, dpt);
    }
    return launch_ok();
}

// the full band accumulator and row DP of S6-S7 for the frames that `d` selects
ld_status run_vpx_dp(ld_frame f, const Dev& d, hipStream_t st) {
    const size_t l4 = vpx_fit_lds(d);
    const int nt4 = vpx_fit_threads(d);
    ProfScope ps(f, 3, st);
    const int nrc = vpx_fit_nrc(d);
    auto launch = [&](auto kernel) {
        allow_lds(kernel, l4);
        hipLaunchKernelGGL(kernel, dim3(f->active), dim3(nt4), l4, st, d);
    };
    if (nt4 <= 512) {
        switch (nrc) {
            case 64: launch(k_vpx_fit<512, 64>); break;
            case 128: launch(k_vpx_fit<512, 128>); break;
            case 256: launch(k_vpx_fit<512, 256>); break;
            case 320: launch(k_vpx_fit<512, 320>); break;
            case 512: launch(k_vpx_fit<512, 512>); break;
            default: launch(k_vpx_fit<512, 0>); break;
        }
    } else {
        launch(k_vpx_fit<1024, 0>);
    }
    return launch_ok();
}

// S8 for every active frame
ld_status run_vpx_ransac(ld_frame f, const uint64_t* sid, const int64_t* fidx, const double* seed_gamma, int pruned,
                         double* vp_out, hipStream_t st) {
    const Dev& d = f->d;
    const size_t l = sizeof(int) * 4 * (size_t)d.H + sizeof(uint32_t) * ((d.H + 31) / 32);
    allow_lds(k_vpx_ransac, l);
    ProfScope ps(f, 10, st);
    hipLaunchKernelGGL(k_vpx_ransac, dim3(f->active), dim3(kRansacThreads), l, st, d, sid, fidx, seed_gamma, pruned, vp_out);
    return launch_ok();
}

ld_status run_vp(ld_frame f, const uint8_t* grey, int64_t gp, const void* disp, int64_t dpt, const uint64_t* sid,
                 const int64_t* fidx, const double* seed_gamma, double* vp_out, hipStream_t st) {
    ld_status s = run_edges(f, grey, gp, disp, dpt, st);
    if (s == LD_OK) s = run_vpx_dp(f, f->d, st);
    if (s == LD_OK) s = run_vpx_ransac(f, sid, fidx, seed_gamma, 0, vp_out, st);
    return s;
}

template <int NC, int NT>
void launch_energy(ld_frame f, const Dev& d, const uint8_t* mask, float* eout, hipStream_t st) {
    const size_t l = energy_lds(NC);
    allow_lds(k_energy<NC, NT>, l);
    hipLaunchKernelGGL((k_energy<NC, NT>), dim3(f->active), dim3(kBlock), l, st, d, mask, eout);
}

ld_status run_energy(ld_frame f, const uint8_t* mask, float* eout, hipStream_t st, const Dev* dsel = nullptr) {
    ProfScope ps(f, 4, st);
    const Dev& d = dsel ? *dsel : f->d;
    const int nc = (d.W + kBlock - 1) / kBlock;
    if (nc <= 1) launch_energy<1, 2>(f, d, mask, eout, st);
    else if (nc <= 2) launch_energy<2, 4>(f, d, mask, eout, st);
    else if (nc <= 3) launch_energy<3, 6>(f, d, mask, eout, st);
    else if (nc <= 4) launch_energy<4, 8>(f, d, mask, eout, st);
    else if (nc <= 5) launch_energy<5, 10>(f, d, mask, eout, st);
    else if (nc <= 6) launch_energy<6, 12>(f, d, mask, eout, st);
    else if (nc <= 8) launch_energy<8, 16>(f, d, mask, eout, st);
    else if (nc <= 12) launch_energy<12, 24>(f, d, mask, eout, st);
    else launch_energy<16, 32>(f, d, mask, eout, st);
    return launch_ok();
}

ld_status run_peaks(ld_frame f, ld_lanes* lanes, float* curves, hipStream_t st, const Dev* dsel = nullptr) {
    ProfScope ps(f, 5, st);
    const Dev& d = dsel ? *dsel : f->d;
    hipLaunchKernelGGL(k_peaks, dim3(f->active), dim3(kBlock), (size_t)d.W2, st, d, lanes, curves);
    return launch_ok();
}

ld_status check_images(ld_frame f, const uint8_t* grey, int64_t gp, const void* disp, int64_t dpt) {
    const Dev& d = f->d;
    const int es = elem_size(d.fmt);
    if (disp == nullptr || dpt < (int64_t)d.W * es || dpt % es != 0 || !aligned(disp, es)) return LD_E_INVAL;
    // the edge kernel addresses a frame's grey rows with 32-bit offsets
    if (grey != nullptr && (gp < d.W || (int64_t)d.H * gp > (int64_t)INT32_MAX - 4096)) return LD_E_INVAL;
    return LD_OK;
}

// Every step of ld_detect on the active frames of f, on one stream.
ld_status detect_all(ld_frame f, const uint8_t* grey, int64_t gp, const void* disp, int64_t dpt,
                     const uint64_t* sid, const int64_t* fidx, ld_lanes* lanes, float* curves, hipStream_t st) {
    f->last = st;
    ld_status s = run_vdisp(f, disp, dpt, sid, fidx, nullptr, nullptr, st);
    if (s == LD_OK) s = run_vp(f, grey, gp, disp, dpt, sid, fidx, nullptr, nullptr, st);
    if (s == LD_OK) s = run_energy(f, nullptr, nullptr, st);
    if (s == LD_OK) s = run_peaks(f, lanes, curves, st);
    f->stage = s == LD_OK ? 3 : 0;
    f->bands = 0;
    return s;
}

}  // namespace

// Scratch of ld_detect_noalloc: a fixed device array, one copy per GPU for the life of the
// process.  Host code never uses the name `scratch` as an address: the device address of each
// GPU's copy is taken once per device with hipGetSymbolAddress (that device current) and kept
// in scratch_ptr.  Every ld_detect_noalloc call on a GPU uses that GPU's copy, so calls that
// overlap on one GPU (different streams or threads without ordering) race on it.
constexpr size_t kNoAllocBytes = LD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
char* scratch_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array (set up on the first call on that device).
ld_status noalloc_scratch(char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LD_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return LD_E_INVAL;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return LD_E_HIP;
        }
        scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    *out = scratch_ptr[dev];
    return LD_OK;
}

}  // namespace

extern "C" {

void ld_params_default(ld_params* p) {
    if (!p) return;
    p->chi = 25; p->tau_y_max = 6; p->tau_x_max = 5; p->lambda_y = 1; p->lambda_x = 1;
    p->tr_y = 4.0; p->tr_x = 16.0; p->eps_num = 99; p->eps_den = 100; p->varpi = 3.0;
    p->edge_t = 100; p->sigma_g = 3.5; p->nu = 1; p->varsigma = 3; p->n_hyp = 64; p->max_rounds = 16;
    p->rho_lpv = 0.25; p->d_nms = 0; p->weight_squared = 0; p->vote = 0; p->seed = 0;
}

const char* ld_status_string(ld_status s) {
    switch (s) {
        case LD_OK: return "ok";
        case LD_E_INVAL: return "invalid argument";
        case LD_E_NOMEM: return "out of device memory";
        case LD_E_HIP: return "HIP runtime error";
        case LD_E_STATE: return "step called out of order";
        case LD_E_BUSY: return "queue full, retry later";
    }
    return "unknown status";
}

ld_status ld_frame_create(int32_t width, int32_t height, int32_t batch, int32_t fmt, int32_t d_max,
                          const ld_params* p, ld_frame* out) {
    if (!out) return LD_E_INVAL;
    *out = nullptr;
    Dev d0{};
    if (init_dev(d0, width, height, batch, fmt, d_max, p) != LD_OK) return LD_E_INVAL;
    ld_frame f = new (std::nothrow) ld_frame_s();
    if (!f) return LD_E_NOMEM;
    Dev& d = f->d;
    d = d0;
    size_t off[kRegions], sz[kRegions];
    const size_t o = frame_layout(width, height, batch, d_max, off, sz);

    if (hipGetDevice(&f->device) != hipSuccess) { delete f; return LD_E_HIP; }
    if (hipMalloc(&f->mem, o) != hipSuccess) { (void)hipGetLastError(); delete f; return LD_E_NOMEM; }
    f->mem_bytes = o;
    bind_regions(d, static_cast<char*>(f->mem), off);
    // small state starts zeroed so that introspection of an unprocessed frame is defined
    if (hipMemset(d.info, 0, sz[4]) != hipSuccess || hipMemset(d.trace, 0xff, sz[11]) != hipSuccess ||
        hipMemset(d.fit, 0, sz[3]) != hipSuccess || hipMemset(d.prune, 0, sz[15]) != hipSuccess ||
        hipMemset(d.lbits, 0, sz[14]) != hipSuccess || hipMemset(d.cmask, 1, sz[16]) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(f->mem);
        delete f;
        return LD_E_HIP;
    }
    f->batch = batch;
    f->active = batch;
    f->last = nullptr;
    f->stage = 0;
    f->bands = 0;
    *out = f;
    return LD_OK;
}

ld_status ld_frame_destroy(ld_frame f) {
    if (!f) return LD_OK;
    ld_status s = LD_OK;
    if (hipStreamSynchronize(f->last) != hipSuccess) s = LD_E_HIP;
    for (auto& e : f->pending) { (void)hipEventDestroy(e.start); (void)hipEventDestroy(e.stop); }
    for (auto& e : f->pool) { (void)hipEventDestroy(e.start); (void)hipEventDestroy(e.stop); }
    if (hipFree(f->mem) != hipSuccess) s = LD_E_HIP;
    delete f;
    return s;
}

ld_status ld_frame_set_active(ld_frame f, int32_t n) {
    if (!f || n < 1 || n > f->batch) return LD_E_INVAL;
    f->active = n;
    return LD_OK;
}

ld_status ld_vdisp(ld_frame f, const void* disp, int64_t disp_pitch, const uint64_t* stream_ids,
                   const int64_t* frame_idx, int32_t* vdisp_out, double* beta_out, void* hip_stream) {
    LdRange rr_("ld_vdisp");
    if (!f) return LD_E_INVAL;
    if (check_images(f, nullptr, 0, disp, disp_pitch) != LD_OK) return LD_E_INVAL;
    if ((stream_ids && !aligned(stream_ids, 8)) || (frame_idx && !aligned(frame_idx, 8))) return LD_E_INVAL;
    if ((vdisp_out && !aligned(vdisp_out, 4)) || (beta_out && !aligned(beta_out, 8))) return LD_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    ld_status s = run_vdisp(f, disp, disp_pitch, stream_ids, frame_idx, vdisp_out, beta_out, st);
    f->last = st;
    if (s == LD_OK) f->stage = 1;
    f->bands = 0;
    return s;
}

ld_status ld_vp_ransac(ld_frame f, const uint8_t* grey, int64_t grey_pitch, const void* disp, int64_t disp_pitch,
                       const uint64_t* stream_ids, const int64_t* frame_idx, const double* seed_gamma,
                       double* vp_out, void* hip_stream) {
    LdRange rr_("ld_vp_ransac");
    if (!f) return LD_E_INVAL;
    if (!grey || check_images(f, grey, grey_pitch, disp, disp_pitch) != LD_OK) return LD_E_INVAL;
    if ((stream_ids && !aligned(stream_ids, 8)) || (frame_idx && !aligned(frame_idx, 8))) return LD_E_INVAL;
    if ((seed_gamma && !aligned(seed_gamma, 8)) || (vp_out && !aligned(vp_out, 8))) return LD_E_INVAL;
    if (f->stage < 1) return LD_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    ld_status s = run_vp(f, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, seed_gamma, vp_out, st);
    f->last = st;
    if (s == LD_OK) f->stage = 2;
    return s;
}

ld_status ld_lane_energy(ld_frame f, const uint8_t* cand_mask, float* energy_out, void* hip_stream) {
    LdRange rr_("ld_lane_energy");
    if (!f) return LD_E_INVAL;
    if (energy_out && !aligned(energy_out, 4)) return LD_E_INVAL;
    if (f->stage < 2) return LD_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    ld_status s = run_energy(f, cand_mask, energy_out, st);
    f->last = st;
    if (s == LD_OK) f->stage = 3;
    return s;
}

ld_status ld_peaks(ld_frame f, ld_lanes* lanes_out, float* curves_out, void* hip_stream) {
    LdRange rr_("ld_peaks");
    if (!f || !lanes_out || !aligned(lanes_out, 4)) return LD_E_INVAL;
    if (curves_out && !aligned(curves_out, 4)) return LD_E_INVAL;
    if (f->stage < 3) return LD_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    ld_status s = run_peaks(f, lanes_out, curves_out, st);
    f->last = st;
    return s;
}

ld_status ld_detect(ld_frame f, const uint8_t* grey, int64_t grey_pitch, const void* disp, int64_t disp_pitch,
                    const uint64_t* stream_ids, const int64_t* frame_idx, ld_lanes* lanes_out, float* curves_out,
                    void* hip_stream) {
    LdRange rr_("ld_detect");
    if (!f || !lanes_out || !aligned(lanes_out, 4)) return LD_E_INVAL;
    if (!grey || check_images(f, grey, grey_pitch, disp, disp_pitch) != LD_OK) return LD_E_INVAL;
    if ((stream_ids && !aligned(stream_ids, 8)) || (frame_idx && !aligned(frame_idx, 8))) return LD_E_INVAL;
    if (curves_out && !aligned(curves_out, 4)) return LD_E_INVAL;
    return detect_all(f, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, lanes_out, curves_out,
                      static_cast<hipStream_t>(hip_stream));
}

ld_status ld_detect_noalloc(int32_t width, int32_t height, int32_t batch, int32_t fmt, int32_t d_max,
                            const ld_params* p, const uint8_t* grey, int64_t grey_pitch, const void* disp,
                            int64_t disp_pitch, const uint64_t* stream_ids, const int64_t* frame_idx,
                            ld_lanes* lanes_out, float* curves_out, void* hip_stream) {
    LdRange rr_("ld_detect_noalloc");
    ld_frame_s fr;                      // host state on the stack; prof stays off (no event pool)
    if (init_dev(fr.d, width, height, batch, fmt, d_max, p) != LD_OK) return LD_E_INVAL;
    if (!lanes_out || !aligned(lanes_out, 4)) return LD_E_INVAL;
    if (!grey || check_images(&fr, grey, grey_pitch, disp, disp_pitch) != LD_OK) return LD_E_INVAL;
    if ((stream_ids && !aligned(stream_ids, 8)) || (frame_idx && !aligned(frame_idx, 8))) return LD_E_INVAL;
    if (curves_out && !aligned(curves_out, 4)) return LD_E_INVAL;
    size_t off[kRegions], sz[kRegions];
    if (frame_layout(width, height, batch, d_max, off, sz) > kNoAllocBytes) return LD_E_NOMEM;
    char* base = nullptr;
    const ld_status s = noalloc_scratch(&base);
    if (s != LD_OK) return s;
    bind_regions(fr.d, base, off);
    fr.batch = batch;
    fr.active = batch;
    fr.mem = nullptr;
    fr.mem_bytes = 0;
    (void)hipGetDevice(&fr.device);
    return detect_all(&fr, grey, grey_pitch, disp, disp_pitch, stream_ids, frame_idx, lanes_out, curves_out,
                      static_cast<hipStream_t>(hip_stream));
}

ld_status ld_detect_pruned(ld_frame f, ld_cnn n, const uint8_t* grey, int64_t grey_pitch, const void* disp,
                           int64_t disp_pitch, const uint64_t* stream_ids, const int64_t* frame_idx,
                           const double* seed_gamma, ld_lanes* lanes_out, float* curves_out, void* hip_stream) {
    LdRange rr_("ld_detect_pruned");
    if (!f || !n || !lanes_out || !aligned(lanes_out, 4)) return LD_E_INVAL;
    if (seed_gamma && !aligned(seed_gamma, 8)) return LD_E_INVAL;
    if (!grey || check_images(f, grey, grey_pitch, disp, disp_pitch) != LD_OK) return LD_E_INVAL;
    if ((stream_ids && !aligned(stream_ids, 8)) || (frame_idx && !aligned(frame_idx, 8))) return LD_E_INVAL;
    if (curves_out && !aligned(curves_out, 4)) return LD_E_INVAL;
    const ld_cnn_config* c = ldi_cnn_config(n);
    if (!c || !(f->d.P.varpi > 0.0)) return LD_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    f->last = st;
    Dev& d = f->d;
    const int nb = c->n_bands;
    ld_status s = run_vdisp(f, disp, disp_pitch, stream_ids, frame_idx, nullptr, nullptr, st);
    f->stage = s == LD_OK ? 1 : 0;
    f->bands = 0;
    // the edges first: without the candidate mask the network decisions are read only at voting
    // road edges of the band rows, so the network skips the column tiles that hold none
    if (s == LD_OK) s = run_edges(f, grey, grey_pitch, disp, disp_pitch, st);
    if (s == LD_OK) {
        ProfScope ps(f, 6, st);
        s = ldi_cnn_bits(n, f, grey, grey_pitch, disp, disp_pitch, nullptr, c->dilate < 0 ? 1 : 0, st);
    }
    if (s == LD_OK) {
        ProfScope ps(f, 7, st);
        const size_t ls = sizeof(int) * 2 * (size_t)d.W2;
        allow_lds(k_seed, ls);
        hipLaunchKernelGGL(k_seed, dim3(f->active), dim3(kBlock), ls, st, d, nb, c->delta_x, c->min_votes,
                           c->seed_ransac);
        s = launch_ok();
    }
    if (s == LD_OK) {
        ProfScope ps(f, 8, st);
        const int cap = std::min(16384, std::max(4096, 16 * d.W));   // staged road edges (bytes)
        const size_t lw = sizeof(int) * (256 + kWave + 3 * (size_t)d.H + 2) + cap;
        const int wave_bytes = (int)((lw + 15) / 16 * 16);
        const int fpw = std::max(1, std::min(4, kMaxLds / wave_bytes));   // frames per workgroup
        allow_lds(k_vpx_window, (size_t)fpw * wave_bytes);
        hipLaunchKernelGGL(k_vpx_window, dim3((f->active + fpw - 1) / fpw), dim3(kWave * fpw), (size_t)fpw * wave_bytes,
                           st, d, cap, wave_bytes, f->active);
        s = launch_ok();
    }
    Dev full = d;                       // frames sent back to the full V_px search
    full.only = d.prune;
    full.only_bits = kFbPlainVpx;
    full.only_set = 1;
    if (s == LD_OK) s = run_vpx_dp(f, full, st);
    if (s == LD_OK) s = run_vpx_ransac(f, stream_ids, frame_idx, seed_gamma, 1, nullptr, st);
    // without candidate pruning every candidate is kept: no mask, and no frame is sent back
    // to the full energies
    const bool pruning = c->dilate >= 0;
    if (s == LD_OK && pruning) {
        ProfScope ps(f, 9, st);
        const size_t lm = sizeof(uint32_t) * nb * LDI_BAND_ROWS * (size_t)((d.W + 31) / 32) + (size_t)d.W2;
        allow_lds(k_cand_mask, lm);
        hipLaunchKernelGGL(k_cand_mask, dim3(f->active), dim3(kBlock), lm, st, d, nb, c->dilate);
        s = launch_ok();
    }
    if (s == LD_OK) s = run_energy(f, pruning ? d.cmask : nullptr, nullptr, st);
    if (s == LD_OK) s = run_peaks(f, lanes_out, curves_out, st);
    if (s == LD_OK) {
        ProfScope ps(f, 9, st);
        hipLaunchKernelGGL(k_lane_check, dim3((f->active + 63) / 64), dim3(64), 0, st, d, lanes_out, f->active,
                           pruning ? 1 : 0);
        s = launch_ok();
    }
    Dev again = d;                      // frames sent back to the full energies
    again.only = d.prune;
    again.only_bits = kFbPlainEnergy;
    again.only_set = 1;
    if (s == LD_OK && pruning) s = run_energy(f, nullptr, nullptr, st, &again);
    if (s == LD_OK && pruning) s = run_peaks(f, lanes_out, curves_out, st, &again);
    f->stage = s == LD_OK ? 3 : 0;
    if (s == LD_OK) f->bands = nb;
    return s;
}

ld_status ld_sync(ld_frame f) {
    if (!f) return LD_E_INVAL;
    return hipStreamSynchronize(f->last) == hipSuccess ? LD_OK : LD_E_HIP;
}

ld_status ld_frame_profile(ld_frame f, int32_t enable) {
    if (!f) return LD_E_INVAL;
    if (hipStreamSynchronize(f->last) != hipSuccess) return LD_E_HIP;
    for (auto& e : f->pending) f->pool.push_back(e);
    f->pending.clear();
    for (int k = 0; k < kNumKernels; ++k) { f->acc_ms[k] = 0.0; f->calls[k] = 0; }
    f->prof = enable != 0;
    return LD_OK;
}

ld_status ld_frame_kernel_times(ld_frame f, double* ms_out, int64_t* calls_out, int32_t n) {
    if (!f || !ms_out || n < 1) return LD_E_INVAL;
    ld_status s = LD_OK;
    for (auto& e : f->pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(e.stop) != hipSuccess || hipEventElapsedTime(&ms, e.start, e.stop) != hipSuccess) {
            s = LD_E_HIP;
        } else {
            f->acc_ms[e.kernel] += ms;
            f->calls[e.kernel] += 1;
        }
        f->pool.push_back(e);
    }
    f->pending.clear();
    for (int k = 0; k < n && k < kNumKernels; ++k) {
        ms_out[k] = f->acc_ms[k];
        if (calls_out) calls_out[k] = f->calls[k];
    }
    return s;
}

ld_status ld_frame_read(ld_frame f, int32_t what, int32_t b, void* dst, int64_t bytes, void* hip_stream) {
    if (!f || !dst || b < 0 || b >= f->batch) return LD_E_INVAL;
    const Dev& d = f->d;
    const void* src = nullptr;
    size_t n = 0;
    switch (what) {
        case LD_STATE_INFO: src = d.info + b; n = sizeof(FrameInfo); break;
        case LD_STATE_MY_PATH: src = d.my_pts + (size_t)b * 2 * d.D1; n = sizeof(int32_t) * 2 * d.D1; break;
        case LD_STATE_BETA: src = d.fit + 2 * (size_t)b; n = sizeof(FitRes); break;
        case LD_STATE_GAMMA: src = d.fit + 2 * (size_t)b + 1; n = sizeof(FitRes); break;
        case LD_STATE_TABLES: src = d.tab + (size_t)b * 6 * d.H; n = sizeof(double) * 6 * d.H; break;
        case LD_STATE_ROWCOUNT: src = d.rowcnt + (size_t)b * d.H; n = sizeof(int32_t) * d.H; break;
        case LD_STATE_EDGES: src = d.edges + (size_t)b * d.H * d.W; n = sizeof(ld_edge) * d.H * d.W; break;
        case LD_STATE_MX_PATH: src = d.mxpath + (size_t)b * d.H; n = sizeof(int32_t) * d.H; break;
        case LD_STATE_ENERGY: src = d.energy + (size_t)b * d.W2; n = sizeof(double) * d.W2; break;
        case LD_STATE_TRACE: src = d.trace + (size_t)b * 6 * kMaxRounds; n = sizeof(int32_t) * 6 * kMaxRounds; break;
        case LD_STATE_LANE_BITS:
            src = d.lbits + (size_t)b * LDI_MAX_BANDS * LDI_BAND_ROWS * d.W;
            n = (size_t)LDI_MAX_BANDS * LDI_BAND_ROWS * d.W;
            break;
        case LD_STATE_PRUNE: src = d.prune + (size_t)b * kPruneWords; n = sizeof(int32_t) * kPruneWords; break;
        case LD_STATE_CAND_MASK: src = d.cmask + (size_t)b * d.W2; n = (size_t)d.W2; break;
        default: return LD_E_INVAL;
    }
    if (bytes < (int64_t)n) return LD_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    return hipMemcpyAsync(dst, src, n, hipMemcpyDefault, st) == hipSuccess ? LD_OK : LD_E_HIP;
}

}  // extern "C"

// ==========================================================================================
// Internal hooks for the serving layer (ld_server.hip); not part of the C ABI.
ld_status ldi_frame_bind_count(ld_frame f, const int32_t* d_count) {
    if (!f) return LD_E_INVAL;
    f->d.nact = d_count;
    return LD_OK;
}

const ld_fit* ldi_frame_fits(ld_frame f) { return f ? reinterpret_cast<const ld_fit*>(f->d.fit) : nullptr; }

ld_status ldi_frame_get_view(ld_frame f, ldi_frame_view* v) {
    if (!f || !v) return LD_E_INVAL;
    const Dev& d = f->d;
    v->W = d.W; v->H = d.H; v->fmt = d.fmt; v->d_max = d.d_max; v->batch = f->batch; v->active = f->active;
    v->stage = f->stage;
    v->varpi = d.P.varpi;
    v->tab = d.tab;
    v->info = reinterpret_cast<const int32_t*>(d.info);
    v->lane_bits = d.lbits;
    v->nact = d.nact;
    v->edges = d.edges;
    v->rowcnt = d.rowcnt;
    return LD_OK;
}

ld_status ldi_frame_set_last(ld_frame f, void* stream) {
    if (!f) return LD_E_INVAL;
    f->last = static_cast<hipStream_t>(stream);
    return LD_OK;
}

ld_status ldi_frame_mark_bands(ld_frame f, int32_t n_bands, void* stream) {
    if (!f) return LD_E_INVAL;
    f->bands = n_bands;
    f->last = static_cast<hipStream_t>(stream);
    return LD_OK;
}

size_t ldi_frame_bytes(int32_t width, int32_t height, int32_t batch, int32_t d_max) {
    size_t off[kRegions], sz[kRegions];
    return frame_layout(width, height, batch, d_max, off, sz);
}
