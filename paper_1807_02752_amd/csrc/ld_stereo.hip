// ld_stereo.hip -- disparity maps of rectified stereo pairs (Sec. 2.1): NCC block matching on
// memorised block statistics (Eq. ncc_1 with Eq. sigma_l_1 / sigma_r_1), search range
// propagation from the bottom row up (Eq. srp, Alg. "SRP-based disparity map estimation") and the
// left-right consistency check (Alg. "LRC check").
//
// Definitions (the same on the CPU check): a pixel is matched only when its (2 rho + 1)^2 block
// lies in the image, 0 meaning "no match", candidates 1..d_max whose other block lies in the
// image too.  With S, Q the block sum and sum of squares, P the sum of products of the two
// blocks and n the block size, the cost is (n P - S_a S_b) / (sqrt(n Q_a - S_a^2) sqrt(n Q_b -
// S_b^2)): integers exactly, the quotient in FP64 in that order; a flat block (n Q = S^2) is not
// scored; the largest cost wins, ties to the smaller disparity.  Row v searches the union of
// [l - tau, l + tau] over the matched neighbours u-1..u+1 of row v+1 with l > 0, else 1..d_max.
// The right map is the same search with the roles of the images swapped (the other block at
// x + d); the check keeps l(u) when |l(u) - l_right(u - l(u))| <= tr.
//
// Layout: one workgroup per frame sweeps the rows from the bottom, its two halves the left and
// the right map in step; each half keeps the statistics of its own image, which the other half
// reads as its partner's, so an image's ring, column sums, block sums and variances are formed
// once for both maps.  The 2 rho + 1 image rows of both images sit in LDS rings (one new row
// per step into the slot of the row that leaves, fetched from HBM while the row before it is
// matched), stored word-interleaved (word g
// of all slots together) so that a block's words are constant offsets from one address; the
// sum of products takes the rows in slot order for both blocks, which leaves it unchanged.  The
// column sums over the ring follow each new row incrementally, the block sums of a row come
// from the column sums four columns a thread, and the square roots of the block variances are
// kept per column (FP64), so a candidate costs its 2 rho + 1 rows of byte dot products, a
// subtraction, a multiplication and a division.  A pixel with a matched neighbour below scores
// its few propagated candidates (up to three runs) in one loop of its own lane; a pixel without
// one (every pixel of the first row) searches all of 1..d_max, which would hold up the 63 other
// lanes of its wave, so such pixels are queued: many (the first row) are taken one a lane, few
// one a wave with a candidate per lane and a reduction over the wave.  The propagation makes
// the rows of a frame sequential; frames are independent workgroups.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "ld.h"
#include "ld_internal.h"

namespace {

constexpr int kT = 512;        // sweep threads per map: a workgroup holds both maps of a frame, 16 waves
constexpr int kWaves = kT / 64;
constexpr int kRowWords = 2;   // words of a new row per thread and image: widths up to 4 kT kRowWords
constexpr int kPad = 8;        // zero columns on both sides of the column sums (block sums four at a time)
constexpr int kTL = 320;       // consistency check threads (a 1242-pixel row in one workgroup)
constexpr int kLrcPx = 4;      // consistency check pixels a thread
constexpr int kLrcRows = 8;    // consistency check rows a workgroup
constexpr int kNone = 1 << 20; // an absent neighbour in the sorted propagation bounds

__host__ __device__ constexpr size_t round16(size_t x) { return (x + 15) / 16 * 16; }

size_t stereo_lds(int W, int rho) {
    const size_t Wp = (size_t)(W + 3) / 4 * 4;
    const size_t rows = 2 * (size_t)rho + 1;
    return round16(2 * rows * Wp)                      // image rings (u8)
           + 4 * sizeof(int32_t) * (Wp + 2 * kPad)     // column sums S, Q of both images
           + 2 * sizeof(int32_t) * Wp                  // block sums S of both images
           + 2 * sizeof(double) * Wp                   // sqrt of the block variances of both images
           + 4 * Wp                                    // disparities of the previous and the current row, both maps
           + 2 * sizeof(uint16_t) * Wp + 16;           // queues of full-range pixels and their lengths, both maps
}

template <int RHO>
__global__ __launch_bounds__(2 * kT) void k_stereo(const uint8_t* left, int64_t lp, const uint8_t* right, int64_t rp,
                                               int W, int H, const int32_t* nact, int nframes, int d_max, int tau,
                                               uint8_t* lf, uint8_t* rt) {
    constexpr int K = 2 * RHO + 1, N = K * K;
    constexpr int NW = (K + 3) / 4;                                   // words of a block row
    constexpr uint32_t kLastMask = (K % 4 == 0) ? 0xFFFFFFFFu : ((1u << (8 * (K % 4))) - 1u);
    constexpr int kC = (RHO + 3) / 4;                                 // column-sum quads either side
    extern __shared__ __align__(16) unsigned char smem[];
    // NW words holding bytes o .. o + 4 NW - 1 of the row in slot j of a ring whose word g of
    // slot j is word g K + j (the words past a row's last byte lie in the LDS allocation, their
    // bytes are cleared or unused)
    auto fetch = [&](const uint32_t* ring, int j, int o, uint32_t (&w)[NW]) {
        const uint32_t* r = ring + (o >> 2) * K + j;
        const uint32_t s = (uint32_t)(o & 3);
        uint32_t x[NW + 1];
#pragma unroll
        for (int k = 0; k <= NW; ++k) x[k] = r[k * K];
#pragma unroll
        for (int k = 0; k < NW; ++k) w[k] = __builtin_amdgcn_alignbyte(x[k + 1], x[k], s);
    };
    const int b = blockIdx.x, t = threadIdx.x;
    const int nf = nact != nullptr ? min(*nact, nframes) : nframes;
    if (b >= nf) return;
    // the workgroup's first half sweeps the left map (own image left, blocks of the right image
    // at u - d), the second the right map (own image right, blocks of the left image at u + d);
    // each half keeps the ring, column sums, block sums and variances of its own image, which
    // the other half reads as the partner's
    const int m = t / kT, tm = t % kT;
    const uint8_t* ga = (m == 0 ? left + (int64_t)b * H * lp : right + (int64_t)b * H * rp);
    const int64_t pa = m == 0 ? lp : rp;
    uint8_t* out = (m == 0 ? lf : rt) + (int64_t)b * H * W;
    const int sgn = m == 0 ? -1 : 1;
    const int Wp = (W + 3) / 4 * 4, Wq = Wp / 4;
    uint32_t* ring0 = reinterpret_cast<uint32_t*>(smem);
    uint32_t* ring1 = ring0 + K * Wq;
    int32_t* colS0 = reinterpret_cast<int32_t*>(smem + round16(2 * (size_t)K * Wp)) + kPad;
    int32_t* colQ0 = colS0 + Wp + 2 * kPad;
    int32_t* colS1 = colQ0 + Wp + 2 * kPad;
    int32_t* colQ1 = colS1 + Wp + 2 * kPad;
    int32_t* S0 = colQ1 + Wp + kPad;
    int32_t* S1 = S0 + Wp;
    double* sq0 = reinterpret_cast<double*>(S1 + Wp);
    double* sq1 = sq0 + Wp;
    uint8_t* pc = reinterpret_cast<uint8_t*>(sq1 + Wp);
    uint16_t* queues = reinterpret_cast<uint16_t*>(pc + 4 * Wp);
    int* qns = reinterpret_cast<int*>(queues + 2 * Wp);
    uint32_t* ringA = m == 0 ? ring0 : ring1;
    uint32_t* ringB = m == 0 ? ring1 : ring0;
    uint8_t* ringA8 = reinterpret_cast<uint8_t*>(ringA);
    int32_t* colS_a = m == 0 ? colS0 : colS1;
    int32_t* colQ_a = m == 0 ? colQ0 : colQ1;
    int32_t* S_a = m == 0 ? S0 : S1;
    const int32_t* S_b = m == 0 ? S1 : S0;
    double* sq_a = m == 0 ? sq0 : sq1;
    const double* sq_b = m == 0 ? sq1 : sq0;
    uint8_t* prev = pc + (2 * m) * Wp;
    uint8_t* cur = pc + (2 * m + 1) * Wp;
    uint16_t* queue = queues + m * Wp;
    int* qn = qns + m;
    // rows outside the matched band are 0 (every row when no block fits)
    const bool none = W < K || H < K;
    for (int v = 0; v < H; ++v) {
        if (!none && v >= RHO && v <= H - 1 - RHO) continue;
        for (int u = tm; u < W; u += kT) out[(int64_t)v * W + u] = 0;
    }
    if (none) return;
    // the first 2 rho + 1 rows of the own image (slot v mod K), bytes past the width cleared;
    // its column sums
    const int vb = H - 1 - RHO;
    for (int v = vb - RHO; v <= vb + RHO; ++v) {
        const int slot = v % K;
        for (int u = tm; u < Wp; u += kT) ringA8[((u >> 2) * K + slot) * 4 + (u & 3)] = u < W ? ga[(int64_t)v * pa + u] : 0;
    }
    for (int i = tm; i < kPad; i += kT) {
        colS_a[-1 - i] = colQ_a[-1 - i] = 0;
        colS_a[Wp + i] = colQ_a[Wp + i] = 0;
    }
    if (tm == 0) *qn = 0;
    __syncthreads();
    for (int u = tm; u < Wp; u += kT) {
        int sa = 0, qa = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int x = ringA8[((u >> 2) * K + j) * 4 + (u & 3)];
            sa += x; qa += x * x;
        }
        colS_a[u] = sa; colQ_a[u] = qa;
    }
    // the candidate of disparity d for the pixel at u: its cost against the best so far (bc
    // starts at -inf), the first strictly larger one kept (with d increasing that leaves ties to
    // the smaller d).  The numerator n P - S_a S_b is exact in 32 bits (each product below 2^30
    // for rho <= 5); a candidate whose block leaves the image or is flat is scored at a stand-in
    // position and not taken
    auto score = [&](const uint32_t (&A)[K][NW], int u, int Sa, double da, int d, int& best, double& bc) {
        const int x = u + sgn * d;
        const bool inr = (unsigned)(x - RHO) <= (unsigned)(W - 1 - 2 * RHO);
        const int xc = inr ? x : RHO;
        const double db = sq_b[xc];
        uint32_t P = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            uint32_t Bw[NW];
            fetch(ringB, j, xc - RHO, Bw);
#pragma unroll
            for (int k = 0; k < NW; ++k) P = __builtin_amdgcn_udot4(A[j][k], Bw[k], P, false);
        }
        const int num = N * (int)P - Sa * S_b[xc];
        const double c = (double)num / (da * db);
        const bool take = inr & (db > 0.0) & (c > bc);
        best = take ? d : best;
        bc = take ? c : bc;
    };
    auto own_block = [&](int u, uint32_t (&A)[K][NW]) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            fetch(ringA, j, u - RHO, A[j]);
            A[j][NW - 1] &= kLastMask;        // the bytes past the block are cleared
        }
    };
    for (int v = vb; v >= RHO; --v) {
        const bool more = v > RHO;             // a row v - rho - 1 follows
        const int vlo = v - RHO;
        __syncthreads();
        // block sums and sqrt(n Q - S^2) of the own image, four columns a thread (0 where no
        // block fits)
        for (int g = tm; g < Wq; g += kT) {
            int cs[2][4 * (2 * kC + 1)];
            const int32_t* arr[2] = {colS_a, colQ_a};
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
                for (int c = -kC; c <= kC; ++c) {
                    const int4 q = *reinterpret_cast<const int4*>(arr[a] + 4 * (g + c));
                    cs[a][4 * (c + kC) + 0] = q.x; cs[a][4 * (c + kC) + 1] = q.y;
                    cs[a][4 * (c + kC) + 2] = q.z; cs[a][4 * (c + kC) + 3] = q.w;
                }
            }
            int bs[2][4];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                int s_ = 0;
#pragma unroll
                for (int mm = -RHO; mm <= RHO; ++mm) s_ += cs[a][4 * kC + mm];
                bs[a][0] = s_;
#pragma unroll
                for (int i = 1; i < 4; ++i) {
                    s_ += cs[a][4 * kC + i + RHO] - cs[a][4 * kC + i - 1 - RHO];
                    bs[a][i] = s_;
                }
            }
            int4 oa;
            double qa4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = 4 * g + i;
                const bool fits = u >= RHO && u <= W - 1 - RHO;
                const int va = N * bs[1][i] - bs[0][i] * bs[0][i];
                qa4[i] = fits && va > 0 ? sqrt((double)va) : 0.0;
                (&oa.x)[i] = fits ? bs[0][i] : 0;
            }
            *reinterpret_cast<int4*>(S_a + 4 * g) = oa;
#pragma unroll
            for (int i = 0; i < 4; i += 2)
                *reinterpret_cast<double2*>(sq_a + 4 * g + i) = make_double2(qa4[i], qa4[i + 1]);
        }
        __syncthreads();
        // the own image's next row from HBM while this one is matched: four bytes a word for
        // words tm and tm + kT, byte loads at clamped positions (their values are masked when
        // the words are put together), so that nothing waits for them before the row is done
        uint32_t ra[kRowWords][4];
        {
            const uint8_t* pa0 = ga + (int64_t)(more ? vlo - 1 : vlo) * pa;
#pragma unroll
            for (int k = 0; k < kRowWords; ++k)
#pragma unroll
                for (int i = 0; i < 4; ++i) ra[k][i] = pa0[min(4 * (tm + k * kT) + i, W - 1)];
        }
        // pixels with a matched neighbour below: the union of [l - tau, l + tau] over those
        // neighbours, in increasing d, in the pixel's own lane; the others are queued
        const bool first = v == vb;
        for (int u = tm; u < W; u += kT) {
            int best = 0;
            if (u >= RHO && u <= W - 1 - RHO && sq_a[u] > 0.0) {
                int l0 = 0, l1 = 0, l2 = 0;
                if (!first) {
                    l0 = u - 1 >= RHO ? prev[u - 1] : 0;
                    l1 = prev[u];
                    l2 = u + 1 <= W - 1 - RHO ? prev[u + 1] : 0;
                }
                if ((l0 | l1 | l2) == 0) {
                    queue[atomicAdd(qn, 1)] = (uint16_t)u;
                } else {
                    int s0 = l0 ? l0 : kNone, s1 = l1 ? l1 : kNone, s2 = l2 ? l2 : kNone;
                    {   // s0 <= s1 <= s2
                        const int a = min(s0, s1), c = max(s0, s1);
                        const int hi3 = max(c, s2), mid = min(c, s2);
                        s0 = min(a, mid); s1 = max(a, mid); s2 = hi3;
                    }
                    // the union as up to three disjoint runs in increasing order
                    int a0 = max(s0 - tau, 1), b0 = min(s0 + tau, d_max), a1 = 1, b1 = 0, a2 = 1, b2 = 0;
                    if (s1 < kNone) {
                        const int lo = s1 - tau, hi = min(s1 + tau, d_max);
                        if (lo <= b0 + 1) b0 = max(b0, hi); else { a1 = lo; b1 = hi; }
                    }
                    if (s2 < kNone) {
                        const int lo = s2 - tau, hi = min(s2 + tau, d_max);
                        if (b1 >= a1) {
                            if (lo <= b1 + 1) b1 = max(b1, hi); else { a2 = lo; b2 = hi; }
                        } else {
                            if (lo <= b0 + 1) b0 = max(b0, hi); else { a1 = lo; b1 = hi; }
                        }
                    }
                    uint32_t A[K][NW];
                    own_block(u, A);
                    const int Sa = S_a[u];
                    const double da = sq_a[u];
                    double bc = -__builtin_inf();
                    // one loop over all the candidates (a lane's runs follow each other
                    // without waiting for the other lanes' runs to end)
                    const int n = (b0 - a0 + 1) + max(b1 - a1 + 1, 0) + max(b2 - a2 + 1, 0);
                    int d = a0, e = b0;
                    for (int k = 0; k < n; ++k) {
                        score(A, u, Sa, da, d, best, bc);
                        const bool nx = d == e;
                        d = nx ? a1 : d + 1;
                        e = nx ? b1 : e;
                        a1 = nx ? a2 : a1;
                        b1 = nx ? b2 : b1;
                    }
                }
            }
            cur[u] = (uint8_t)best;
        }
        __syncthreads();
        // queued pixels: many (the first row) one a lane over all of 1..d_max; few one a wave,
        // candidates 1 + lane, 65 + lane, ..., then the best (largest cost, then smallest d)
        // over the wave.  Both halves take the barrier when either map queued any.
        const int nq = *qn;
        if (qns[0] > 0 || qns[1] > 0) {
            if (nq >= kT / 2) {
                for (int q = tm; q < nq; q += kT) {
                    const int u = queue[q];
                    uint32_t A[K][NW];
                    own_block(u, A);
                    const int Sa = S_a[u];
                    const double da = sq_a[u];
                    int best = 0;
                    double bc = -__builtin_inf();
                    for (int d = 1; d <= d_max; ++d) score(A, u, Sa, da, d, best, bc);
                    cur[u] = (uint8_t)best;
                }
            } else if (nq > 0) {
                const int wv = tm >> 6, lane = tm & 63;
                for (int q = wv; q < nq; q += kWaves) {
                    const int u = queue[q];
                    uint32_t A[K][NW];
                    own_block(u, A);
                    const int Sa = S_a[u];
                    const double da = sq_a[u];
                    int best = 0;
                    double bc = -__builtin_inf();
                    for (int d = 1 + lane; d <= d_max; d += 64) score(A, u, Sa, da, d, best, bc);
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) {
                        const double oc = __shfl_xor(bc, off);
                        const int od = __shfl_xor(best, off);
                        if (od != 0 && (best == 0 || oc > bc || (oc == bc && od < best))) { best = od; bc = oc; }
                    }
                    if (lane == 0) cur[u] = (uint8_t)best;
                }
            }
            __syncthreads();
        }
        // the own image's next row replaces row v + rho in its ring and column sums; the row out
        if (more) {
            const int slot = (v + RHO) % K;
#pragma unroll
            for (int k = 0; k < kRowWords; ++k) {
                const int g = tm + k * kT;
                if (g >= Wq) continue;
                uint32_t na = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * g + i < W) na |= ra[k][i] << (8 * i);
                const uint32_t oa = ringA[g * K + slot];
                ringA[g * K + slot] = na;
                int4 s1 = *reinterpret_cast<int4*>(colS_a + 4 * g), q1 = *reinterpret_cast<int4*>(colQ_a + 4 * g);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int xn = (na >> (8 * i)) & 0xFF, xo = (oa >> (8 * i)) & 0xFF;
                    (&s1.x)[i] += xn - xo; (&q1.x)[i] += xn * xn - xo * xo;
                }
                *reinterpret_cast<int4*>(colS_a + 4 * g) = s1; *reinterpret_cast<int4*>(colQ_a + 4 * g) = q1;
            }
        }
        for (int u = tm; u < W; u += kT) out[(int64_t)v * W + u] = cur[u];
        if (tm == 0) *qn = 0;
        uint8_t* tmp = prev; prev = cur; cur = tmp;
    }
}

// l(u) = l_left(u) unless it is 0, u - l(u) < 0 or |l(u) - l_right(u - l(u))| > tr.  A workgroup
// takes kLrcRows rows of a frame (grid: row groups, frames), kLrcPx consecutive pixels a thread.
template <int PX>
__global__ __launch_bounds__(kTL) void k_lrc(const uint8_t* lf, const uint8_t* rt, int W, int H, const int32_t* nact,
                                            int nframes, int tr, uint8_t* out, int64_t op) {
    const int b = blockIdx.y;
    const int nf = nact != nullptr ? min(*nact, nframes) : nframes;
    if (b >= nf) return;
    for (int v = blockIdx.x * kLrcRows; v < min(H, (int)(blockIdx.x + 1) * kLrcRows); ++v) {
        const uint8_t* L = lf + ((int64_t)b * H + v) * W;
        const uint8_t* R = rt + ((int64_t)b * H + v) * W;
        uint8_t* O = out + ((int64_t)b * H + v) * op;
        for (int u0 = threadIdx.x * PX; u0 < W; u0 += kTL * PX) {
            uint8_t l[PX];
#pragma unroll
            for (int k = 0; k < PX; ++k) l[k] = L[min(u0 + k, W - 1)];
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int u = u0 + k, lk = l[k];
                if (u >= W) break;
                int o = 0;
                if (lk > 0 && u - lk >= 0 && abs(lk - (int)R[u - lk]) <= tr) o = lk;
                O[u] = (uint8_t)o;
            }
        }
    }
}

// The same check over the maps as one flat array when the left map and the output are whole
// words apart and the output rows are contiguous: a thread loads a word of four disparities,
// gathers their right-map partners (same row: u - l >= 0) and stores a word.
__global__ __launch_bounds__(256) void k_lrc_words(const uint8_t* lf, const uint8_t* rt, int W, int64_t HW,
                                                  const int32_t* nact, int nframes, int tr, uint8_t* out) {
    const int nf = nact != nullptr ? min(*nact, nframes) : nframes;
    const int64_t total = (int64_t)nf * HW;
    const int64_t p0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (p0 >= total) return;
    const int64_t row = p0 / W;
    int u = (int)(p0 - row * W);
    if (p0 + 4 <= total) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(lf + p0);
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l = (int)((w >> (8 * i)) & 0xFFu);
            const int ui = u + i < W ? u + i : u + i - W;     // a word spans at most two rows
            if (l > 0 && ui - l >= 0 && abs(l - (int)rt[p0 + i - l]) <= tr) o |= (uint32_t)l << (8 * i);
        }
        *reinterpret_cast<uint32_t*>(out + p0) = o;
    } else {
        for (int64_t p = p0; p < total; ++p, ++u) {      // the last few bytes
            if (u == W) u = 0;
            const int l = lf[p];
            out[p] = (l > 0 && u - l >= 0 && abs(l - (int)rt[p - l]) <= tr) ? (uint8_t)l : 0;
        }
    }
}

template <int RHO>
void launch(const uint8_t* left, int64_t lp, const uint8_t* right, int64_t rp, const ldi_frame_view& V, int tau,
            uint8_t* lf, uint8_t* rt, hipStream_t st) {
    const size_t lds = stereo_lds(V.W, RHO);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_stereo<RHO>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_stereo<RHO>, dim3(V.active), dim3(2 * kT), lds, st, left, lp, right, rp, V.W, V.H, V.nact,
                       V.active, V.d_max, tau, lf, rt);
}

}  // namespace

extern "C" ld_status ld_stereo(ld_frame f, const uint8_t* left, int64_t left_pitch, const uint8_t* right,
                               int64_t right_pitch, int32_t rho, int32_t tau, int32_t tr_lrc, uint8_t* disp_out,
                               int64_t disp_pitch, uint8_t* disp_lf, uint8_t* disp_rt, void* hip_stream) {
    LdRange rr_("ld_stereo");
    ldi_frame_view V;
    if (!f || !left || !right || !disp_out || !disp_lf || !disp_rt || ldi_frame_get_view(f, &V) != LD_OK)
        return LD_E_INVAL;
    if (rho < 1 || rho > 5 || tau < 0 || tau > 255 || tr_lrc < 0 || V.d_max > 255) return LD_E_INVAL;
    if (left_pitch < V.W || right_pitch < V.W || disp_pitch < V.W) return LD_E_INVAL;
    if (stereo_lds(V.W, rho) > 160 * 1024 || V.W > 4 * kT * kRowWords) return LD_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (V.active > 0) {
        switch (rho) {
            case 1: launch<1>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
            case 2: launch<2>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
            case 3: launch<3>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
            case 4: launch<4>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
            default: launch<5>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
        }
        const int64_t HW = (int64_t)V.W * V.H;
        if (disp_pitch == V.W && ((uintptr_t)disp_lf & 3) == 0 && ((uintptr_t)disp_out & 3) == 0) {
            const int64_t words = (V.active * HW + 3) / 4;
            hipLaunchKernelGGL(k_lrc_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, disp_lf, disp_rt,
                               V.W, HW, V.nact, V.active, tr_lrc, disp_out);
        } else {
            const unsigned gx = (unsigned)((V.H + kLrcRows - 1) / kLrcRows);
            hipLaunchKernelGGL(k_lrc<kLrcPx>, dim3(gx, V.active), dim3(kTL), 0, st, disp_lf, disp_rt, V.W, V.H,
                               V.nact, V.active, tr_lrc, disp_out, disp_pitch);
        }
    }
    if (hipGetLastError() != hipSuccess) return LD_E_HIP;
    return ldi_frame_set_last(f, hip_stream);
}
