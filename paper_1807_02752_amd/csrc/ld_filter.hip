// ld_filter.hip -- bilateral pre-filter of the grey images ahead of the gradient (Sec. 2.3.1,
// Eq. bilateral_filter with its spatial weight w_s and range weight w_r).
//
// I_bf(u, v) = sum w_s w_r I / sum w_s w_r over the (2 rho + 1)^2 window centred at (u, v),
// w_s = exp(-((i-u)^2 + (j-v)^2) / sigma_s^2), w_r = exp(-(I(i,j) - I(u,v))^2 / sigma_r^2) on
// intensities scaled to [0, 1].  The result is rounded to u8 (so the Sobel step after it stays
// integer), and because that rounding is a decision, the arithmetic is fixed: single-precision
// weight tables (w_s per window offset, w_r per absolute grey difference, each the
// double-precision exponential rounded to float, built on the host), single-precision sums in
// window order (rows top to bottom, each left to right), the numerator by a fused multiply-add,
// an IEEE quotient, rounding half up.  Window pixels outside the frame take part in neither sum.
//
// Layout on the GPU: a workgroup filters a 64 x 32 tile of one frame.  The tile and its rho
// halo are staged in LDS as 4 x grey (4 x 511 outside the frame), so |n - c| of two staged
// values is directly the byte offset of w_r in the LDS copy of the range table, whose entries
// 256 .. 511 are 0: a pixel outside the frame gets weight 0 and adds exactly nothing.  Thread
// (r, g) computes pixels 8g .. 8g+7 of tile row r: for each window row it reads the 8 + 2 rho
// staged values of that row once and uses them for its eight pixels.  The spatial weights are
// wave-uniform kernel arguments.  The arithmetic is FP32 VALU work, about five operations per
// window tap and pixel; HBM traffic is one read and one write of the image.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "ld.h"
#include "ld_internal.h"

namespace {

constexpr int kTileW = 64, kTileH = 32, kThreads = 256, kPix = 8;   // kPix columns per thread
constexpr int kMaxRho = 5;
constexpr int kOutside = 511;                 // staged value of a pixel outside the frame
constexpr int kLut = 512;                     // range-weight table entries in LDS

struct BfTables {
    float ws[(2 * kMaxRho + 1) * (2 * kMaxRho + 1)];   // row-major over (dy, dx)
    float wr[256];
};

template <int RHO>
__global__ __launch_bounds__(kThreads) void k_bilateral(ldi_frame_view V, const uint8_t* grey, int64_t gp,
                                                        uint8_t* out, int64_t op, BfTables T, int road_rows) {
    constexpr int N = 2 * RHO + 1;
    constexpr int SW = kTileW + 2 * RHO, SH = kTileH + 2 * RHO;
    constexpr int SP = (SW + 7) / 8 * 8;              // staged row pitch (u16), rows 16-byte aligned
    __shared__ __align__(16) uint16_t tile[SH * SP];
    __shared__ float lut[kLut];
    const int b = blockIdx.z, t = threadIdx.x;
    const int nf = V.nact != nullptr ? min(*V.nact, V.active) : V.active;
    if (b >= nf) return;
    const int W = V.W, H = V.H;
    int row0 = 0;
    if (road_rows) {
        const int flags = V.info[b * 8], v_h = V.info[b * 8 + 1];
        row0 = (flags & LD_FLAG_NOROAD) ? H : max(v_h - 1, 0);
    }
    const int r0 = blockIdx.y * kTileH, c0 = blockIdx.x * kTileW;
    if (r0 + kTileH <= row0) return;                   // the whole tile lies above the rows filtered
    const uint8_t* g = grey + (int64_t)b * H * gp;
    for (int i = t; i < SH * SW; i += kThreads) {
        const int y = i / SW, x = i % SW;
        const int v = r0 - RHO + y, u = c0 - RHO + x;
        const int val = (v >= 0 && v < H && u >= 0 && u < W) ? (int)g[(int64_t)v * gp + u] : kOutside;
        tile[y * SP + x] = (uint16_t)(4 * val);
    }
    for (int i = t; i < kLut; i += kThreads) lut[i] = i < 256 ? T.wr[i] : 0.0f;
    __syncthreads();
    const int r = t / (kTileW / kPix), gcol = (t % (kTileW / kPix)) * kPix;
    const unsigned char* lutb = reinterpret_cast<const unsigned char*>(lut);
    int c4[kPix];
    float num[kPix], den[kPix];
#pragma unroll
    for (int k = 0; k < kPix; ++k) {
        c4[k] = tile[(r + RHO) * SP + gcol + RHO + k];
        num[k] = 0.0f;
        den[k] = 0.0f;
    }
#pragma unroll 1
    for (int dy = -RHO; dy <= RHO; ++dy) {
        const uint16_t* srow = tile + (r + RHO + dy) * SP + gcol;
        int n4[kPix + 2 * RHO];
        float nv[kPix + 2 * RHO], ws[N];
#pragma unroll
        for (int x = 0; x < kPix + 2 * RHO; ++x) {
            n4[x] = srow[x];
            nv[x] = (float)(n4[x] >> 2);
        }
#pragma unroll
        for (int dx = 0; dx < N; ++dx) ws[dx] = T.ws[(dy + RHO) * N + dx];   // wave-uniform
#pragma unroll
        for (int k = 0; k < kPix; ++k) {
#pragma unroll
            for (int dx = -RHO; dx <= RHO; ++dx) {
                const int x = k + dx + RHO;
                const int d4 = (int)__builtin_amdgcn_sad_u16(n4[x], c4[k], 0u);   // |n - c|, one operation
                const float wr = *reinterpret_cast<const float*>(lutb + d4);
                const float w = ws[dx + RHO] * wr;
                num[k] = fmaf(w, nv[x], num[k]);
                den[k] = den[k] + w;
            }
            // one pixel's window row at a time: keeps the table reads in flight to 2 rho + 1
            // (the compiler would otherwise hoist every read of the row and spill)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const int v = r0 + r;
    if (v < row0 || v >= H) return;
    uint8_t* o = out + ((int64_t)b * H + v) * op;
#pragma unroll
    for (int k = 0; k < kPix; ++k) {
        const int u = c0 + gcol + k;
        if (u < W) {
            const float q = num[k] / den[k];
            o[u] = (uint8_t)floorf(q + 0.5f);
        }
    }
}

template <int RHO>
void launch(const ldi_frame_view& V, const uint8_t* grey, int64_t gp, uint8_t* out, int64_t op, const BfTables& T,
            int road_rows, hipStream_t st) {
    const dim3 grid((V.W + kTileW - 1) / kTileW, (V.H + kTileH - 1) / kTileH, V.active);
    hipLaunchKernelGGL(k_bilateral<RHO>, grid, dim3(kThreads), 0, st, V, grey, gp, out, op, T, road_rows);
}

}  // namespace

extern "C" ld_status ld_bilateral(ld_frame f, const uint8_t* grey, int64_t grey_pitch, uint8_t* out,
                                  int64_t out_pitch, int32_t rho, float sigma_s, float sigma_r, int32_t road_rows,
                                  void* hip_stream) {
    LdRange rr_("ld_bilateral");
    ldi_frame_view V;
    if (!f || !grey || !out || ldi_frame_get_view(f, &V) != LD_OK) return LD_E_INVAL;
    if (rho < 1 || rho > kMaxRho || !(sigma_s > 0.0f) || !(sigma_r > 0.0f) || !std::isfinite(sigma_s) ||
        !std::isfinite(sigma_r) || (road_rows != 0 && road_rows != 1))
        return LD_E_INVAL;
    if (grey_pitch < V.W || out_pitch < V.W) return LD_E_INVAL;
    // the two images must not overlap (the filter reads grey while out is written)
    const uintptr_t g0 = (uintptr_t)grey, g1 = g0 + (uintptr_t)((int64_t)V.active * V.H * grey_pitch);
    const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (uintptr_t)((int64_t)V.active * V.H * out_pitch);
    if (g0 < o1 && o0 < g1) return LD_E_INVAL;
    if (road_rows && V.stage < 1) return LD_E_STATE;
    BfTables T;
    const double ss = (double)sigma_s, sr = (double)sigma_r;
    const int n = 2 * rho + 1;
    for (int dy = -rho; dy <= rho; ++dy)
        for (int dx = -rho; dx <= rho; ++dx)
            T.ws[(dy + rho) * n + (dx + rho)] = (float)std::exp(-(double)(dx * dx + dy * dy) / (ss * ss));
    for (int d = 0; d < 256; ++d) {
        const double x = (double)d / 255.0;
        T.wr[d] = (float)std::exp(-(x * x) / (sr * sr));
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    switch (rho) {
        case 1: launch<1>(V, grey, grey_pitch, out, out_pitch, T, road_rows, st); break;
        case 2: launch<2>(V, grey, grey_pitch, out, out_pitch, T, road_rows, st); break;
        case 3: launch<3>(V, grey, grey_pitch, out, out_pitch, T, road_rows, st); break;
        case 4: launch<4>(V, grey, grey_pitch, out, out_pitch, T, road_rows, st); break;
        default: launch<5>(V, grey, grey_pitch, out, out_pitch, T, road_rows, st); break;
    }
    if (hipGetLastError() != hipSuccess) return LD_E_HIP;
    return ldi_frame_set_last(f, hip_stream);
}
