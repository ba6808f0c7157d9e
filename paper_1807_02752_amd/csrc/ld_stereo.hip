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
// Layout: one workgroup per (frame, map) sweeps the rows from the bottom; the 2 rho + 1 image
// rows of both images sit in an LDS ring (one new row per step), the block sums of the current
// row are formed from column sums in LDS, and the square roots of the block variances are kept
// per column (FP64), so a candidate costs its 2 rho + 1 squared products, a subtraction, a
// multiplication and a division.  The propagation makes the rows of a frame sequential; frames
// and the two maps are independent workgroups.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "ld.h"
#include "ld_internal.h"

namespace {

constexpr int kT = 512;        // sweep threads: 8 waves, two sweeps per CU (LDS) keep 4 waves per SIMD
constexpr int kTL = 256;       // consistency check threads

size_t stereo_lds(int W, int rho) {
    const size_t Wp = (size_t)(W + 3) / 4 * 4;
    const size_t rows = 2 * (size_t)rho + 1;
    return 2 * rows * Wp                       // image rings (u8)
           + 4 * sizeof(int32_t) * W           // column sums S, Q of both images
           + 2 * sizeof(int32_t) * W           // block sums S of both images
           + 2 * sizeof(double) * W            // sqrt of the block variances of both images
           + 2 * Wp;                           // disparities of the previous and the current row
}

template <int RHO>
__global__ __launch_bounds__(kT) void k_stereo(const uint8_t* left, int64_t lp, const uint8_t* right, int64_t rp,
                                               int W, int H, const int32_t* nact, int nframes, int d_max, int tau,
                                               uint8_t* lf, uint8_t* rt) {
    constexpr int K = 2 * RHO + 1, N = K * K;
    constexpr int NW = (K + 3) / 4;                                   // words of a block row
    constexpr uint32_t kLastMask = (K % 4 == 0) ? 0xFFFFFFFFu : ((1u << (8 * (K % 4))) - 1u);
    extern __shared__ __align__(16) unsigned char smem[];
    // NW words of a row holding bytes o .. o + 4 NW - 1 (rows start on a word; the word after a
    // row's last byte lies in the LDS allocation, its bytes are cleared or unused)
    auto fetch = [&](const uint8_t* row, int o, uint32_t (&w)[NW]) {
        const uint32_t* r = reinterpret_cast<const uint32_t*>(row) + (o >> 2);
        const uint32_t s = (uint32_t)(o & 3);
        uint32_t x[NW + 1];
#pragma unroll
        for (int k = 0; k <= NW; ++k) x[k] = r[k];
#pragma unroll
        for (int k = 0; k < NW; ++k) w[k] = __builtin_amdgcn_alignbyte(x[k + 1], x[k], s);
    };
    const int b = blockIdx.x, t = threadIdx.x;
    const int nf = nact != nullptr ? min(*nact, nframes) : nframes;
    if (b >= nf) return;
    const bool is_left = blockIdx.y == 0;
    // the map's own image is a (blocks at u), the other b (blocks at u - d or u + d)
    const uint8_t* ga = (is_left ? left + (int64_t)b * H * lp : right + (int64_t)b * H * rp);
    const uint8_t* gb = (is_left ? right + (int64_t)b * H * rp : left + (int64_t)b * H * lp);
    const int64_t pa = is_left ? lp : rp, pb = is_left ? rp : lp;
    uint8_t* out = (is_left ? lf : rt) + (int64_t)b * H * W;
    const int sgn = is_left ? -1 : 1;
    const int Wp = (W + 3) / 4 * 4;
    uint8_t* ringA = smem;
    uint8_t* ringB = ringA + K * Wp;
    int32_t* colS_a = reinterpret_cast<int32_t*>(ringB + K * Wp);
    int32_t* colQ_a = colS_a + W;
    int32_t* colS_b = colQ_a + W;
    int32_t* colQ_b = colS_b + W;
    int32_t* S_a = colQ_b + W;
    int32_t* S_b = S_a + W;
    double* sq_a = reinterpret_cast<double*>(S_b + W);        // 8-byte aligned: 2 K Wp + 24 W bytes before it
    double* sq_b = sq_a + W;
    uint8_t* prev = reinterpret_cast<uint8_t*>(sq_b + W);
    uint8_t* cur = prev + Wp;
    // rows outside the matched band are 0 (every row when no block fits)
    const bool none = W < K || H < K;
    for (int v = 0; v < H; ++v) {
        if (!none && v >= RHO && v <= H - 1 - RHO) continue;
        for (int u = t; u < W; u += kT) out[(int64_t)v * W + u] = 0;
    }
    if (none) return;
    auto load_row = [&](int v) {
        const int slot = v % K;
        for (int u = t; u < W; u += kT) {
            ringA[slot * Wp + u] = ga[(int64_t)v * pa + u];
            ringB[slot * Wp + u] = gb[(int64_t)v * pb + u];
        }
    };
    const int vb = H - 1 - RHO;
    for (int v = vb - RHO; v <= vb + RHO; ++v) load_row(v);
    for (int v = vb; v >= RHO; --v) {
        if (v < vb) load_row(v - RHO);
        __syncthreads();
        // column sums over the block's rows, then the block sums and sqrt of n Q - S^2
        for (int u = t; u < W; u += kT) {
            int sa = 0, qa = 0, sb = 0, qb = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int slot = (v - RHO + j) % K;
                const int x = ringA[slot * Wp + u], y = ringB[slot * Wp + u];
                sa += x; qa += x * x; sb += y; qb += y * y;
            }
            colS_a[u] = sa; colQ_a[u] = qa; colS_b[u] = sb; colQ_b[u] = qb;
        }
        __syncthreads();
        for (int u = t; u < W; u += kT) {
            if (u < RHO || u > W - 1 - RHO) continue;
            int sa = 0, qa = 0, sb = 0, qb = 0;
#pragma unroll
            for (int i = -RHO; i <= RHO; ++i) {
                sa += colS_a[u + i]; qa += colQ_a[u + i]; sb += colS_b[u + i]; qb += colQ_b[u + i];
            }
            S_a[u] = sa; S_b[u] = sb;
            const int va = N * qa - sa * sa, vbv = N * qb - sb * sb;
            sq_a[u] = va > 0 ? sqrt((double)va) : 0.0;
            sq_b[u] = vbv > 0 ? sqrt((double)vbv) : 0.0;
        }
        __syncthreads();
        const bool first = v == vb;
        for (int u = t; u < W; u += kT) {
            int best = 0;
            if (u >= RHO && u <= W - 1 - RHO && sq_a[u] > 0.0) {
                // the search range: [lo, hi] and a membership test over the matched neighbours
                int l0 = 0, l1 = 0, l2 = 0;
                if (!first) {
                    l0 = u - 1 >= RHO ? prev[u - 1] : 0;
                    l1 = prev[u];
                    l2 = u + 1 <= W - 1 - RHO ? prev[u + 1] : 0;
                }
                const bool any = (l0 | l1 | l2) != 0;
                int lo = 1, hi = d_max;
                if (any) {
                    lo = 1 << 30; hi = -1;
                    if (l0) { lo = min(lo, l0 - tau); hi = max(hi, l0 + tau); }
                    if (l1) { lo = min(lo, l1 - tau); hi = max(hi, l1 + tau); }
                    if (l2) { lo = min(lo, l2 - tau); hi = max(hi, l2 + tau); }
                    lo = max(lo, 1);
                    hi = min(hi, d_max);
                }
                // the map's own block in registers, four bytes a word (the bytes past the block
                // are cleared, so the partner block's extra bytes add nothing)
                uint32_t A[K][NW];
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const int slot = (v - RHO + j) % K;
                    fetch(ringA + slot * Wp, u - RHO, A[j]);
                    A[j][NW - 1] &= kLastMask;
                }
                const int64_t Sa = S_a[u];
                const double da = sq_a[u];
                double bc = 0.0;
                for (int d = lo; d <= hi; ++d) {
                    if (any) {
                        const bool in = (l0 && abs(d - l0) <= tau) || (l1 && abs(d - l1) <= tau) ||
                                        (l2 && abs(d - l2) <= tau);
                        if (!in) continue;
                    }
                    const int x = u + sgn * d;
                    if (x < RHO || x > W - 1 - RHO) continue;
                    const double db = sq_b[x];
                    if (!(db > 0.0)) continue;
                    uint32_t P = 0;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const int slot = (v - RHO + j) % K;
                        uint32_t Bw[NW];
                        fetch(ringB + slot * Wp, x - RHO, Bw);
#pragma unroll
                        for (int k = 0; k < NW; ++k) P = __builtin_amdgcn_udot4(A[j][k], Bw[k], P, false);
                    }
                    const double c = (double)((int64_t)N * (int64_t)P - Sa * (int64_t)S_b[x]) / (da * db);
                    if (best == 0 || c > bc) { best = d; bc = c; }
                }
            }
            cur[u] = (uint8_t)best;
            out[(int64_t)v * W + u] = (uint8_t)best;
        }
        __syncthreads();
        for (int u = t; u < W; u += kT) prev[u] = cur[u];
    }
}

// l(u) = l_left(u) unless it is 0, u - l(u) < 0 or |l(u) - l_right(u - l(u))| > tr
__global__ __launch_bounds__(kTL) void k_lrc(const uint8_t* lf, const uint8_t* rt, int W, int H, const int32_t* nact,
                                            int nframes, int tr, uint8_t* out, int64_t op) {
    const int b = blockIdx.y;
    const int nf = nact != nullptr ? min(*nact, nframes) : nframes;
    if (b >= nf) return;
    const int64_t i = (int64_t)blockIdx.x * kTL + threadIdx.x;
    if (i >= (int64_t)W * H) return;
    const int v = (int)(i / W), u = (int)(i % W);
    const int64_t base = (int64_t)b * H * W;
    const int l = lf[base + i];
    int o = 0;
    if (l > 0 && u - l >= 0 && abs(l - (int)rt[base + (int64_t)v * W + (u - l)]) <= tr) o = l;
    out[((int64_t)b * H + v) * op + u] = (uint8_t)o;
}

template <int RHO>
void launch(const uint8_t* left, int64_t lp, const uint8_t* right, int64_t rp, const ldi_frame_view& V, int tau,
            uint8_t* lf, uint8_t* rt, hipStream_t st) {
    const size_t lds = stereo_lds(V.W, RHO);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_stereo<RHO>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_stereo<RHO>, dim3(V.active, 2), dim3(kT), lds, st, left, lp, right, rp, V.W, V.H, V.nact,
                       V.active, V.d_max, tau, lf, rt);
}

}  // namespace

extern "C" ld_status ld_stereo(ld_frame f, const uint8_t* left, int64_t left_pitch, const uint8_t* right,
                               int64_t right_pitch, int32_t rho, int32_t tau, int32_t tr_lrc, uint8_t* disp_out,
                               int64_t disp_pitch, uint8_t* disp_lf, uint8_t* disp_rt, void* hip_stream) {
    ldi_frame_view V;
    if (!f || !left || !right || !disp_out || !disp_lf || !disp_rt || ldi_frame_get_view(f, &V) != LD_OK)
        return LD_E_INVAL;
    if (rho < 1 || rho > 5 || tau < 0 || tau > 255 || tr_lrc < 0 || V.d_max > 255) return LD_E_INVAL;
    if (left_pitch < V.W || right_pitch < V.W || disp_pitch < V.W) return LD_E_INVAL;
    if (stereo_lds(V.W, rho) > 160 * 1024) return LD_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (V.active > 0) {
        switch (rho) {
            case 1: launch<1>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
            case 2: launch<2>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
            case 3: launch<3>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
            case 4: launch<4>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
            default: launch<5>(left, left_pitch, right, right_pitch, V, tau, disp_lf, disp_rt, st); break;
        }
        const int64_t px = (int64_t)V.W * V.H;
        hipLaunchKernelGGL(k_lrc, dim3((unsigned)((px + kTL - 1) / kTL), V.active), dim3(kTL), 0, st, disp_lf, disp_rt,
                           V.W, V.H, V.nact, V.active, tr_lrc, disp_out, disp_pitch);
    }
    if (hipGetLastError() != hipSuccess) return LD_E_HIP;
    return ldi_frame_set_last(f, hip_stream);
}
