// ld_cnn.hip -- the candidate-pruning network on gfx950: features, three 3x3 convolutions
// (4 -> 16 -> 16 -> 1 channels, ReLU, zero padding) as BF16 MFMA tiles with FP32
// accumulation, the weighted cross-entropy, the backward pass (input and weight gradients on
// MFMA), a fixed-order gradient reduction and Adam on FP32 master weights.  The network is not
// part of the paper's method: it scores the pixels of a few bands of road rows so that the
// search for V_px and the lane candidates can be narrowed (see ld_detect_pruned).
//
// Geometry.  A band is 16 consecutive road rows taken as an image of its own: the convolutions
// pad with zeros above and below the band and left and right of the frame.  One workgroup owns
// 60 output columns of one band of one frame and recomputes the 3-column halo of each layer:
// layer 1 on u0-2 .. u0+61, layer 2 on u0-1 .. u0+62, layer 3 on u0 .. u0+63 (four 16-pixel
// tiles per row, the last columns of each layer unused).  Activations stay in LDS as
// [18 rows][72 columns][channels] BF16, column x holding u = u0 - 4 + x, rows 0 and 17 zero.
//
// MFMA v_mfma_f32_16x16x32_bf16, D = A B with lane l holding A[l%16][8(l/16) .. +7],
// B[8(l/16) .. +7][l%16] and D[4(l/16) .. +3][l%16].  Forward and input-gradient tiles take
// A = weights (rows = output channels), B = activations (columns = 16 pixels of a row), so a
// lane ends with 4 consecutive channels of one pixel; a K step of 32 is 2 taps x 16 channels
// (layer 1: 8 taps x 4 channels).  Weight gradients take K = 32 pixels of a row.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ld.h"
#include "ld_internal.h"

namespace {

constexpr int kNP = LD_CNN_PARAMS;
constexpr int kOffW1 = 0, kOffB1 = 576, kOffW2 = 592, kOffB2 = 2896, kOffW3 = 2912, kOffB3 = 3056;
constexpr int kPart = 3072;          // floats per workgroup partial: gradients, then the loss
constexpr int kLossSlot = 3064;
constexpr int kBR = LDI_BAND_ROWS;
constexpr int kCT = 60;              // output columns owned by a workgroup
constexpr int kXW = 72;              // LDS columns, u = u0 - 4 + x
constexpr int kLR = kBR + 2;         // LDS rows
constexpr int kT = 256;              // threads per workgroup (4 waves)
constexpr int kChunks = 28;          // packed A operands: 2 + 5 + 5 forward, 1 + 5 input gradient, 5 + 5 row sweep
constexpr int kFeatElems = kLR * kXW * 4;
constexpr int kActElems = kLR * kXW * 16;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_bits(float f) {   // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_val(uint32_t h) { return __uint_as_float(h << 16); }
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// bf16_bits(lo) | bf16_bits(hi) << 16 by the packed hardware conversion (also round to nearest even)
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float bf16_round(float f) { return bf16_val(bf16_bits(f)); }
// the low 16 bits hold a BF16 value > 0 (ReLU outputs are >= 0 or -0)
__device__ __forceinline__ bool positive(uint32_t h) { return (h & 0x7FFFu) != 0u && (h & 0x8000u) == 0u; }

__device__ __forceinline__ f32x4 mfma(uint4 a, uint4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// 8 BF16 values p[0], p[s], ..., p[7s] packed into one operand
__device__ __forceinline__ uint4 pack8(const uint16_t* p, int s) {
    uint4 r;
    r.x = (uint32_t)p[0] | ((uint32_t)p[s] << 16);
    r.y = (uint32_t)p[2 * s] | ((uint32_t)p[3 * s] << 16);
    r.z = (uint32_t)p[4 * s] | ((uint32_t)p[5 * s] << 16);
    r.w = (uint32_t)p[6 * s] | ((uint32_t)p[7 * s] << 16);
    return r;
}

__device__ __forceinline__ int tap_dy(int tap) { return tap / 3 - 1; }
__device__ __forceinline__ int tap_dx(int tap) { return tap % 3 - 1; }

struct Net {
    const uint4* wpk;      // kChunks x 64 lanes
    const float* master;   // kNP, FP32 (biases are read from here)
};

// ------------------------------------------------------------------------------------------
// Features of band rows top .. top+15, columns u0-3 .. u0+62 (x = 1 .. 66): I/255,
// |grad|/1020, atan2(G_y, G_x)/pi, clamp((D - f(v)) / varpi, -4, 4) (-4 where D is invalid),
// with the Sobel pair G_x = d/du, G_y = d/dv (weights 1, 2, 1, zero outside the frame).
// The grey rows top-1 .. top+16 and the disparities are first staged in LDS (every load of
// the workgroup in flight at once), then each pixel's features are formed from LDS.
constexpr int kGW = 72;              // staged grey columns u0-4 .. u0+67
constexpr int kDW = 66;              // staged disparity columns u0-3 .. u0+62
constexpr size_t kStageBytes = 18 * kGW + sizeof(float) * kBR * kDW + sizeof(double) * kBR;

// Features of the staged tile (grey rows top-1 .. top+16, columns u0-4 .. u0+67; disparities
// of rows top .. top+15, columns u0-3 .. u0+62; f(v) of the 16 rows) into feat at x = 1 .. 66
// of rows 1 .. 16; pixels outside the frame get zero features.
__device__ void features_from_stage(const ldi_frame_view& V, int u0, uint16_t* feat, const unsigned char* stage) {
    const int W = V.W, t = threadIdx.x;
    const uint8_t* gs = stage;
    const float* ds = reinterpret_cast<const float*>(stage + 18 * kGW);
    const double* fs = reinterpret_cast<const double*>(ds + kBR * kDW);
    const float inv_pi = (float)(1.0 / 3.14159265358979323846);
    for (int i = t; i < kBR * 66; i += kT) {
        const int r = i / 66, x = 1 + i % 66, u = u0 - 4 + x;
        uint2 pk = make_uint2(0u, 0u);
        if (u >= 0 && u < W) {
            const uint8_t* g0 = gs + r * kGW + x;          // row v-1, column u
            const uint8_t* g1 = g0 + kGW;
            const uint8_t* g2 = g1 + kGW;
            const int gx = ((int)g0[1] - (int)g0[-1]) + 2 * ((int)g1[1] - (int)g1[-1]) + ((int)g2[1] - (int)g2[-1]);
            const int gy = ((int)g2[-1] - (int)g0[-1]) + 2 * ((int)g2[0] - (int)g0[0]) + ((int)g2[1] - (int)g0[1]);
            // g * (1/255) rounds to the same BF16 as g / 255 for every grey value g
            const float c0 = (float)g1[0] * (float)(1.0 / 255.0);
            const float c1 = sqrtf((float)(gx * gx + gy * gy)) / 1020.0f;
            const float c2 = atan2f((float)gy, (float)gx) * inv_pi;
            const float D = ds[r * kDW + x - 1];
            float c3 = -4.0f;
            if (D > 0.0f) c3 = (float)fmin(fmax(((double)D - fs[r]) / V.varpi, -4.0), 4.0);
            pk.x = pack_bf16(c0, c1);
            pk.y = pack_bf16(c2, c3);
        }
        *reinterpret_cast<uint2*>(feat + ((r + 1) * kXW + x) * 4) = pk;
    }
}

// A disparity as the features see it: the value in pixels, or -1 where it is invalid.
__device__ __forceinline__ float disp_value(const uint8_t* row, int u, int fmt) {
    if (fmt == LD_DISP_U8) {
        const int q = row[u];
        return q != 0 ? (float)q : -1.0f;
    } else if (fmt == LD_DISP_F32) {
        const float x32 = reinterpret_cast<const float*>(row)[u];
        return (isfinite(x32) && x32 > 0.0f) ? x32 : -1.0f;
    }
    const int q = reinterpret_cast<const uint16_t*>(row)[u];
    return q != 0 ? (float)q * 0.0625f : -1.0f;                       // exact: q / 16
}

// Features of band rows top .. top+15, columns u0-3 .. u0+62 (x = 1 .. 66): I/255,
// |grad|/1020, atan2(G_y, G_x)/pi, clamp((D - f(v)) / varpi, -4, 4) (-4 where D is invalid),
// with the Sobel pair G_x = d/du, G_y = d/dv (weights 1, 2, 1, zero outside the frame).
// The grey rows top-1 .. top+16 and the disparities are first staged in LDS (every load of
// the workgroup in flight at once), then each pixel's features are formed from LDS.
__device__ void build_features(const ldi_frame_view& V, int b, int top, int u0, const uint8_t* grey, int64_t gp,
                               const uint8_t* disp, int64_t dp, uint16_t* feat, unsigned char* stage) {
    const int W = V.W, H = V.H, t = threadIdx.x;
    uint8_t* gs = stage;                                            // 18 x kGW
    float* ds = reinterpret_cast<float*>(stage + 18 * kGW);          // 16 x kDW, D or -1 (invalid)
    double* fs = reinterpret_cast<double*>(ds + kBR * kDW);          // 16
    const uint8_t* gb = grey + (int64_t)b * H * gp;
    const uint8_t* db = disp + (int64_t)b * H * dp;
    for (int i = t; i < 18 * kGW; i += kT) {
        const int r = i / kGW, u = u0 - 4 + i % kGW, v = top - 1 + r;
        gs[i] = (v >= 0 && v < H && u >= 0 && u < W) ? gb[(int64_t)v * gp + u] : (uint8_t)0;
    }
    for (int i = t; i < kBR * kDW; i += kT) {
        const int r = i / kDW, u = u0 - 3 + i % kDW;
        ds[i] = (u >= 0 && u < W) ? disp_value(db + (int64_t)(top + r) * dp, u, V.fmt) : -1.0f;
    }
    if (t < kBR) fs[t] = V.tab[(int64_t)b * 6 * H + top + t];
    __syncthreads();
    features_from_stage(V, u0, feat, stage);
}

// The raw inputs of one tile held in registers between units: thread t holds the staged
// grey bytes t + 256k, the disparities t + 256k and (t < 16) f of band row t.
constexpr int kRawG = (18 * kGW + kT - 1) / kT;
constexpr int kRawD = (kBR * kDW + kT - 1) / kT;
struct RawTile {
    uint32_t g[kRawG];
    float d[kRawD];
    double f;
};

__device__ __forceinline__ void load_tile(const ldi_frame_view& V, int b, int top, int u0, const uint8_t* grey,
                                          int64_t gp, const uint8_t* disp, int64_t dp, RawTile& R) {
    const int W = V.W, H = V.H, t = threadIdx.x;
    const uint8_t* gb = grey + (int64_t)b * H * gp;
    const uint8_t* db = disp + (int64_t)b * H * dp;
#pragma unroll
    for (int k = 0; k < kRawG; ++k) {
        const int i = t + k * kT;
        const int r = i / kGW, u = u0 - 4 + i % kGW, v = top - 1 + r;
        R.g[k] = (i < 18 * kGW && v >= 0 && v < H && u >= 0 && u < W) ? (uint32_t)gb[(int64_t)v * gp + u] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kRawD; ++k) {
        const int i = t + k * kT;
        const int r = i / kDW, u = u0 - 3 + i % kDW;
        R.d[k] = (i < kBR * kDW && u >= 0 && u < W) ? disp_value(db + (int64_t)(top + r) * dp, u, V.fmt) : -1.0f;
    }
    R.f = t < kBR ? V.tab[(int64_t)b * 6 * H + top + t] : 0.0;
}

__device__ __forceinline__ void stage_tile(const RawTile& R, unsigned char* stage) {
    const int t = threadIdx.x;
    uint8_t* gs = stage;
    float* ds = reinterpret_cast<float*>(stage + 18 * kGW);
    double* fs = reinterpret_cast<double*>(ds + kBR * kDW);
#pragma unroll
    for (int k = 0; k < kRawG; ++k)
        if (t + k * kT < 18 * kGW) gs[t + k * kT] = (uint8_t)R.g[k];
#pragma unroll
    for (int k = 0; k < kRawD; ++k)
        if (t + k * kT < kBR * kDW) ds[t + k * kT] = R.d[k];
    if (t < kBR) fs[t] = R.f;
}

__device__ __forceinline__ void zero_lds(uint4* p, int n16) {
    for (int i = threadIdx.x; i < n16; i += kT) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// The cells of an activation buffer that the layers read but never write: the zero rows 0
// and 17 and columns 66..68 of the band rows (layer 1 writes x = 2..65, layer 2 reads up to
// x = 67, layer 3 up to x = 68).  Two uint4 per cell.
__device__ __forceinline__ void zero_act_border(uint16_t* act) {
    uint4* p = reinterpret_cast<uint4*>(act);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int i = threadIdx.x; i < 2 * kXW * 2; i += kT) {            // rows 0 and 17
        const int row = i < kXW * 2 ? 0 : kLR - 1;
        p[row * kXW * 2 + i % (kXW * 2)] = z;
    }
    for (int i = threadIdx.x; i < kBR * 3 * 2; i += kT) {            // rows 1..16, x = 66..68
        const int row = 1 + i / 6, x = 66 + (i % 6) / 2;
        p[(row * kXW + x) * 2 + (i & 1)] = z;
    }
}

// Layer 1 (4 -> 16): 64 tiles (16 rows x 4), 16 per wave; writes ReLU(z1) as BF16 to a1 at
// x = 2 .. 65, zero outside the frame.
__device__ void layer1(const uint16_t* feat, uint16_t* a1, const Net& N, int u0, int W) {
    const int lane = __lane_id(), wave = threadIdx.x / 64, n = lane & 15, g = lane >> 4;
    const uint4 A0 = N.wpk[lane], A1 = N.wpk[64 + lane];
    const float* b1 = N.master + kOffB1;
    float bias[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias[j] = b1[4 * g + j];
    const int t0 = 2 * g, t1 = 2 * g + 1;
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
        const int tile = wave + 4 * k, r = tile >> 2, x0 = 2 + 16 * (tile & 3);
        const uint16_t* base = feat + ((r + 1) * kXW + x0 + n) * 4;
        const uint2 p0 = *reinterpret_cast<const uint2*>(base + (tap_dy(t0) * kXW + tap_dx(t0)) * 4);
        const uint2 p1 = *reinterpret_cast<const uint2*>(base + (tap_dy(t1) * kXW + tap_dx(t1)) * 4);
        uint4 B1 = make_uint4(0u, 0u, 0u, 0u);
        if (g == 0) {
            const uint2 p8 = *reinterpret_cast<const uint2*>(base + (kXW + 1) * 4);   // tap 8: dy = dx = 1
            B1.x = p8.x;
            B1.y = p8.y;
        }
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = mfma(A0, make_uint4(p0.x, p0.y, p1.x, p1.y), acc);
        acc = mfma(A1, B1, acc);
        const int u = u0 - 4 + x0 + n;
        const bool in = u >= 0 && u < W;
        uint2 o;
        o.x = pack_bf16(fmaxf(acc[0] + bias[0], 0.0f), fmaxf(acc[1] + bias[1], 0.0f));
        o.y = pack_bf16(fmaxf(acc[2] + bias[2], 0.0f), fmaxf(acc[3] + bias[3], 0.0f));
        if (!in) o = make_uint2(0u, 0u);
        *reinterpret_cast<uint2*>(a1 + ((r + 1) * kXW + x0 + n) * 16 + 4 * g) = o;
    }
}

// 16-channel 3x3 convolution of `in` on the 64 tiles at x0 = xs + 16 ct; A = 5 packed chunks.
__device__ __forceinline__ void conv16(const uint16_t* in, int xs, const uint4* A, f32x4 (&acc)[16]) {
    const int lane = __lane_id(), wave = threadIdx.x / 64, n = lane & 15, g = lane >> 4;
    uint4 Ac[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) Ac[c] = A[c * 64 + lane];
    int off[5];
    bool val[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const int tap = 2 * c + (g >> 1);
        val[c] = tap < 9;
        off[c] = val[c] ? (tap_dy(tap) * kXW + tap_dx(tap)) * 16 + 8 * (g & 1) : 0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int tile = wave + 4 * k, r = tile >> 2, x0 = xs + 16 * (tile & 3);
        const uint16_t* base = in + ((r + 1) * kXW + x0 + n) * 16;
        f32x4 a = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const uint4 Bv = val[c] ? *reinterpret_cast<const uint4*>(base + off[c]) : make_uint4(0u, 0u, 0u, 0u);
            a = mfma(Ac[c], Bv, a);
        }
        acc[k] = a;
    }
}

// ReLU(acc + bias) as BF16 into `out` at the tiles of conv16(xs), zero outside the frame
__device__ __forceinline__ void store16(uint16_t* out, int xs, const f32x4 (&acc)[16], const float* bias_all, int u0,
                                        int W) {
    const int lane = __lane_id(), wave = threadIdx.x / 64, n = lane & 15, g = lane >> 4;
    float bias[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias[j] = bias_all[4 * g + j];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int tile = wave + 4 * k, r = tile >> 2, x0 = xs + 16 * (tile & 3);
        const int u = u0 - 4 + x0 + n;
        const bool in = u >= 0 && u < W;
        uint2 o;
        o.x = pack_bf16(fmaxf(acc[k][0] + bias[0], 0.0f), fmaxf(acc[k][1] + bias[1], 0.0f));
        o.y = pack_bf16(fmaxf(acc[k][2] + bias[2], 0.0f), fmaxf(acc[k][3] + bias[3], 0.0f));
        if (!in) o = make_uint2(0u, 0u);
        *reinterpret_cast<uint2*>(out + ((r + 1) * kXW + x0 + n) * 16 + 4 * g) = o;
    }
}

// 16-channel 3x3 convolution by a sweep over the input rows: wave w owns the 16 columns
// x0 = xs + 16 w of all 16 output rows.  Input row ri is read as two operands,
// P = [row ri, dx = -1 | row ri, dx = 0] and Q = [row ri, dx = +1 | row ri+1, dx = +1]; P feeds
// output rows ri+1, ri, ri-1 (weights of dy = -1, 0, +1), Q feeds output row ri+1 (dy = -1, 0
// of dx = +1) and output row ri-1 (dy = +1 of dx = +1, second half weighted zero).  Each output
// row takes its nine taps once; rows 0 and 17 of `in` are zero.  A = 5 packed chunks
// (P of dy = -1, 0, +1, then Q for row ri+1, Q for row ri-1).  acc[k] is LDS row k+1.
__device__ __forceinline__ void conv_rows(const uint16_t* in, int xs, const uint4* A, f32x4 (&acc)[16]) {
    const int lane = __lane_id(), wave = threadIdx.x / 64, n = lane & 15, g = lane >> 4;
    uint4 Ac[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) Ac[c] = A[c * 64 + lane];
    const int x = xs + 16 * wave + n;
    const uint16_t* pP = in + (x + (g < 2 ? -1 : 0)) * 16 + 8 * (g & 1);
    const uint16_t* pQ = in + ((g < 2 ? 0 : kXW) + x + 1) * 16 + 8 * (g & 1);
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // operands of row ri+1 are read while row ri is multiplied; the scheduling barrier keeps
    // the compiler from hoisting every row's reads (which would cost occupancy)
    uint4 Qn = *reinterpret_cast<const uint4*>(pQ), Pn = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int ri = 0; ri <= 16; ++ri) {
        const uint4 Q = Qn, P = Pn;
        if (ri + 1 <= 16) {
            Qn = *reinterpret_cast<const uint4*>(pQ + (ri + 1) * kXW * 16);
            Pn = *reinterpret_cast<const uint4*>(pP + (ri + 1) * kXW * 16);
        }
        if (ri >= 1) {
            if (ri + 1 <= 16) acc[ri] = mfma(Ac[0], P, acc[ri]);
            acc[ri - 1] = mfma(Ac[1], P, acc[ri - 1]);
            if (ri >= 2) acc[ri - 2] = mfma(Ac[2], P, acc[ri - 2]);
        }
        if (ri <= 15) acc[ri] = mfma(Ac[3], Q, acc[ri]);
        if (ri >= 2) acc[ri - 2] = mfma(Ac[4], Q, acc[ri - 2]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

__device__ __forceinline__ int frame_band_top(const ldi_frame_view& V, int b, int nb, int band) {
    const int flags = V.info[b * 8], v_h = V.info[b * 8 + 1];
    if (flags & LD_FLAG_NOROAD) return -1;
    return ldi_band_top(v_h, V.H, nb, band);
}

// ------------------------------------------------------------------------------------------
// Inference: decisions (z3 >= logit(theta)) into the frame's band buffer, optional P = sigmoid(z3).
// A workgroup takes kFwdUnits consecutive units (column tile, band, frame), column tiles of one
// band being consecutive units.  The raw inputs of the next unit are loaded into registers
// while the current one is computed, and the feature buffer is cleared once (its rows 0 and
// 17 are never written, every other cell read by layer 1 is written for each unit).  With
// `sparse`, a unit is evaluated only when a voting road edge (vote column >= 0) lies on its
// band rows and output columns; the others get zero decisions and load nothing.
constexpr int kFwdUnits = 4;
static_assert(kT / 64 == kFwdUnits, "wave w checks unit w");

__global__ __launch_bounds__(kT, 3) void k_cnn_fwd(ldi_frame_view V, Net N, int nb, float thr_logit,
                                                const uint8_t* grey, int64_t gp, const uint8_t* disp, int64_t dp,
                                                float* prob_out, int sparse) {
    extern __shared__ uint4 smem4[];
    uint16_t* feat = reinterpret_cast<uint16_t*>(smem4);
    uint16_t* act = feat + kFeatElems;
    unsigned char* stage = reinterpret_cast<unsigned char*>(act);    // the staged inputs live in act
    const int t = threadIdx.x, W = V.W;
    const int nct = (W + kCT - 1) / kCT;
    const int nf = V.nact != nullptr ? min(*V.nact, V.active) : V.active;
    const int total = nf * nb * nct;
    const int first = blockIdx.x * kFwdUnits;
    if (first >= total) return;
    const int count = min(kFwdUnits, total - first);
    __shared__ int tops[kFwdUnits];        // first band row of each unit, -1 without a band
    __shared__ int need[kFwdUnits];        // the unit is evaluated
    if (t < count) {
        const int q = (first + t) / nct;
        tops[t] = frame_band_top(V, q / nb, nb, q % nb);
    }
    zero_lds(smem4, kFeatElems / 8);
    __syncthreads();
    {   // sparse: wave w looks for a voting road edge on the band rows and columns of unit w
        const int w = t / 64, l = t % 64;
        bool any = !sparse;
        if (sparse && w < count && tops[w] >= 0) {
            const int unit = first + w, u0 = (unit % nct) * kCT;
            const int64_t row0 = (int64_t)((unit / nct) / nb) * V.H + tops[w];
            int cnt[kBR];
            ld_edge e[kBR];
#pragma unroll
            for (int r = 0; r < kBR; ++r) {
                cnt[r] = V.rowcnt[row0 + r];
                e[r] = V.edges[(row0 + r) * W + min(l, W - 1)];
            }
#pragma unroll
            for (int r = 0; r < kBR; ++r)
                any = any || (l < cnt[r] && e[r].bin >= 0 && e[r].u >= u0 && e[r].u < u0 + kCT);
            for (int r = 0; r < kBR; ++r)
                for (int i = l + 64; i < cnt[r]; i += 64) {
                    const ld_edge x = V.edges[(row0 + r) * W + i];
                    any = any || (x.bin >= 0 && x.u >= u0 && x.u < u0 + kCT);
                }
        }
        any = __any(any ? 1 : 0) != 0;
        if (l == 0 && w < kFwdUnits) need[w] = any ? 1 : 0;
    }
    __syncthreads();
    RawTile R;
    if (tops[0] >= 0 && need[0]) {
        const int q = first / nct;
        load_tile(V, q / nb, tops[0], (first % nct) * kCT, grey, gp, disp, dp, R);
    }
    const int lane = __lane_id(), wave = t / 64, n = lane & 15;
#pragma unroll 1
    for (int k = 0; k < count; ++k) {
        const int unit = first + k, ct = unit % nct, q = unit / nct, band = q % nb, b = q / nb;
        const int u0 = ct * kCT, top = need[k] ? tops[k] : -1;
        uint8_t* bits = V.lane_bits + ((int64_t)b * LDI_MAX_BANDS + band) * kBR * W;
        float* prob = prob_out ? prob_out + ((int64_t)b * nb + band) * kBR * W : nullptr;
        if (top < 0) {
            for (int i = t; i < kBR * kCT; i += kT) {
                const int r = i / kCT, u = u0 + i % kCT;
                if (u < W) {
                    bits[r * W + u] = 0;
                    if (prob) prob[r * W + u] = 0.0f;
                }
            }
        } else {
            __syncthreads();                   // the previous unit has finished reading act
            stage_tile(R, stage);
            __syncthreads();
            features_from_stage(V, u0, feat, stage);
        }
        if (k + 1 < count) {                   // the next unit's inputs stay in flight below
            const int un = unit + 1, qn = un / nct, tn = need[k + 1] ? tops[k + 1] : -1;
            if (tn >= 0) load_tile(V, qn / nb, tn, (un % nct) * kCT, grey, gp, disp, dp, R);
        }
        if (top < 0) continue;
        __syncthreads();
        zero_act_border(act);
        __syncthreads();
        layer1(feat, act, N, u0, W);
        __syncthreads();
        f32x4 acc[16];
        conv_rows(act, 3, N.wpk + 18 * 64, acc);
        __syncthreads();                       // every wave has read a1: a2 replaces it in place
        store16(act, 3, acc, N.master + kOffB2, u0, W);
        __syncthreads();
        conv_rows(act, 4, N.wpk + 23 * 64, acc);
        // layer 3 is packed into all 16 output rows of the tile, so every lane holds z of its
        // pixel for every band row; lane group g writes rows g, g + 4, g + 8, g + 12
        const int g = lane >> 4, col = 16 * wave + n, u = u0 + col;
        if (col < kCT && u < W) {
            const float b3 = N.master[kOffB3];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float zr = g == 0 ? acc[4 * j][0] : g == 1 ? acc[4 * j + 1][0] : g == 2 ? acc[4 * j + 2][0]
                                                                                             : acc[4 * j + 3][0];
                const int r = 4 * j + g;
                const float z = zr + b3;
                bits[r * W + u] = z >= thr_logit ? 1 : 0;
                if (prob) prob[r * W + u] = 1.0f / (1.0f + expf(-z));
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Training: forward, loss, backward and this workgroup's share of every gradient (its own
// 60 x 16 loss terms through the recomputed halo), written to one partial row.
__device__ __forceinline__ float softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }

__global__ __launch_bounds__(kT) void k_cnn_train(ldi_frame_view V, Net N, int nb, const uint8_t* grey, int64_t gp,
                                                  const uint8_t* disp, int64_t dp, const uint8_t* labels,
                                                  float pos_weight, float inv_norm, float* part) {
    extern __shared__ uint4 smem4[];
    uint16_t* feat = reinterpret_cast<uint16_t*>(smem4);
    uint16_t* a1 = feat + kFeatElems;            // a1, later dz1
    uint16_t* a2 = a1 + kActElems;               // a2, later dz2
    uint16_t* dz3 = a2 + kActElems;              // kLR x kXW
    float* red = reinterpret_cast<float*>(dz3 + kLR * kXW);   // 4 x 256 + 256 x 4 floats
    const int ct = blockIdx.x, band = blockIdx.y, b = blockIdx.z, t = threadIdx.x;
    const int lane = __lane_id(), wave = t / 64, n = lane & 15, g = lane >> 4;
    float* out = part + (((int64_t)b * nb + band) * gridDim.x + ct) * kPart;
    const int W = V.W, u0 = ct * kCT;
    const int top = (V.nact != nullptr && b >= *V.nact) ? -1 : frame_band_top(V, b, nb, band);
    if (top < 0) {
        for (int i = t; i < kPart; i += kT) out[i] = 0.0f;
        return;
    }
    zero_lds(smem4, (kFeatElems + 2 * kActElems + kLR * kXW) / 8);
    build_features(V, b, top, u0, grey, gp, disp, dp, feat, reinterpret_cast<unsigned char*>(red + 2048));
    __syncthreads();
    layer1(feat, a1, N, u0, W);
    __syncthreads();
    f32x4 acc[16];
    conv16(a1, 3, N.wpk + 2 * 64, acc);
    store16(a2, 3, acc, N.master + kOffB2, u0, W);
    __syncthreads();
    conv16(a2, 4, N.wpk + 7 * 64, acc);

    // ---- loss and dL/dz3 (BF16) of the owned pixels
    const uint8_t* lab = labels + ((int64_t)b * nb + band) * kBR * W;
    float loss = 0.0f, db3 = 0.0f;
    if (lane < 16) {
        const float b3 = N.master[kOffB3];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int tile = wave + 4 * k, r = tile >> 2, col = 16 * (tile & 3) + n, u = u0 + col;
            float gz = 0.0f;
            if (col < kCT && u < W) {
                const int y = lab[r * W + u];
                if (y != 255) {
                    const float z = acc[k][0] + b3;
                    const float s = 1.0f / (1.0f + expf(-z));
                    if (y) {
                        gz = pos_weight * (s - 1.0f) * inv_norm;
                        loss += pos_weight * softplus(-z) * inv_norm;
                    } else {
                        gz = s * inv_norm;
                        loss += softplus(z) * inv_norm;
                    }
                }
            }
            const uint32_t h = bf16_bits(gz);
            db3 += bf16_val(h);
            dz3[(r + 1) * kXW + 4 + 16 * (tile & 3) + n] = (uint16_t)h;
        }
    }
    __syncthreads();

    // ---- dW3[tap][c] = sum_q a2[q][c] dz3[q - off(tap)]: M = c, N = tap, K = 32 pixels of a row
    {
        f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
        const int tap = n;
        const int dyx = tap < 9 ? tap_dy(tap) * kXW + tap_dx(tap) : 0;
        for (int kc = wave; kc < 32; kc += 4) {
            const int rr = kc >> 1, xq = 3 + 32 * (kc & 1) + 8 * g;
            const uint4 A = pack8(a2 + ((rr + 1) * kXW + xq) * 16 + n, 16);
            const uint4 B = tap < 9 ? pack8(dz3 + (rr + 1) * kXW + xq - dyx, 1) : make_uint4(0u, 0u, 0u, 0u);
            d = mfma(A, B, d);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) red[wave * 256 + (4 * g + j) * 16 + n] = d[j];   // [c][tap]
    }
    __syncthreads();
    if (t < 144) {   // t = tap * 16 + c
        const int tap = t >> 4, c = t & 15;
        out[kOffW3 + t] = ((red[c * 16 + tap] + red[256 + c * 16 + tap]) + red[512 + c * 16 + tap]) +
                          red[768 + c * 16 + tap];
    }
    __syncthreads();

    // ---- dz2 = BF16(dL/da2 * (a2 > 0)) in place of a2; dL/da2[q][c] = sum_tap w3[tap][c] dz3[q - off(tap)]
    float cs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    {
        const uint4 A = N.wpk[12 * 64 + lane];
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int tile = wave + 4 * k, r = tile >> 2, x0 = 3 + 16 * (tile & 3);
            uint4 Bv = make_uint4(0u, 0u, 0u, 0u);
            const uint16_t* q = dz3 + (r + 1) * kXW + x0 + n;
            if (g == 0) {
                uint16_t v8[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v8[j] = q[-(tap_dy(j) * kXW + tap_dx(j))];
                Bv.x = v8[0] | ((uint32_t)v8[1] << 16);
                Bv.y = v8[2] | ((uint32_t)v8[3] << 16);
                Bv.z = v8[4] | ((uint32_t)v8[5] << 16);
                Bv.w = v8[6] | ((uint32_t)v8[7] << 16);
            } else if (g == 1) {
                Bv.x = q[-(kXW + 1)];   // tap 8
            }
            f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
            d = mfma(A, Bv, d);
            uint16_t* cell = a2 + ((r + 1) * kXW + x0 + n) * 16 + 4 * g;
            const uint2 av = *reinterpret_cast<const uint2*>(cell);
            float o[4];
            o[0] = positive(av.x) ? bf16_round(d[0]) : 0.0f;
            o[1] = positive(av.x >> 16) ? bf16_round(d[1]) : 0.0f;
            o[2] = positive(av.y) ? bf16_round(d[2]) : 0.0f;
            o[3] = positive(av.y >> 16) ? bf16_round(d[3]) : 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) cs[j] += o[j];
            uint2 w;
            w.x = bf16_bits(o[0]) | (bf16_bits(o[1]) << 16);
            w.y = bf16_bits(o[2]) | (bf16_bits(o[3]) << 16);
            *reinterpret_cast<uint2*>(cell) = w;
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[1024 + t * 4 + j] = cs[j];
    __syncthreads();
    if (t < 16) {   // db2[c], lanes with 4g <= c < 4g + 4 in a fixed order
        const int gg = t >> 2, j = t & 3;
        float s = 0.0f;
        for (int w = 0; w < 4; ++w)
            for (int nn = 0; nn < 16; ++nn) s += red[1024 + (w * 64 + gg * 16 + nn) * 4 + j];
        out[kOffB2 + t] = s;
    }

    // ---- dW2[tap][ci][co] = sum_q a1[q + off(tap)][ci] dz2[q][co]; wave w owns taps w, w+4, w+8
    {
        f32x4 d[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) d[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int kc = 0; kc < 32; ++kc) {
            const int rr = kc >> 1, xq = 3 + 32 * (kc & 1) + 8 * g;
            const uint4 B = pack8(a2 + ((rr + 1) * kXW + xq) * 16 + n, 16);            // dz2[q][co = n]
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int tap = wave + 4 * i;
                if (tap < 9) {
                    const uint4 A = pack8(a1 + ((rr + 1 + tap_dy(tap)) * kXW + xq + tap_dx(tap)) * 16 + n, 16);
                    d[i] = mfma(A, B, d[i]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int tap = wave + 4 * i;
            if (tap < 9)
#pragma unroll
                for (int j = 0; j < 4; ++j) out[kOffW2 + (tap * 16 + 4 * g + j) * 16 + n] = d[i][j];
        }
    }
    __syncthreads();

    // ---- dz1 = BF16(dL/da1 * (a1 > 0)) in place of a1; dL/da1 = conv of dz2 with the flipped,
    //      transposed w2 (5 chunks)
    float cs1[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    {
        uint4 Ac[5];
        int off[5];
        bool val[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            Ac[c] = N.wpk[(13 + c) * 64 + lane];
            const int tap = 2 * c + (g >> 1);
            val[c] = tap < 9;
            off[c] = val[c] ? -(tap_dy(tap) * kXW + tap_dx(tap)) * 16 + 8 * (g & 1) : 0;
        }
        f32x4 dd[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int tile = wave + 4 * k, r = tile >> 2, x0 = 2 + 16 * (tile & 3);
            const uint16_t* base = a2 + ((r + 1) * kXW + x0 + n) * 16;
            f32x4 a = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                const uint4 Bv = val[c] ? *reinterpret_cast<const uint4*>(base + off[c]) : make_uint4(0u, 0u, 0u, 0u);
                a = mfma(Ac[c], Bv, a);
            }
            dd[k] = a;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int tile = wave + 4 * k, r = tile >> 2, x0 = 2 + 16 * (tile & 3);
            uint16_t* cell = a1 + ((r + 1) * kXW + x0 + n) * 16 + 4 * g;
            const uint2 av = *reinterpret_cast<const uint2*>(cell);
            float o[4];
            o[0] = positive(av.x) ? bf16_round(dd[k][0]) : 0.0f;
            o[1] = positive(av.x >> 16) ? bf16_round(dd[k][1]) : 0.0f;
            o[2] = positive(av.y) ? bf16_round(dd[k][2]) : 0.0f;
            o[3] = positive(av.y >> 16) ? bf16_round(dd[k][3]) : 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) cs1[j] += o[j];
            uint2 w;
            w.x = bf16_bits(o[0]) | (bf16_bits(o[1]) << 16);
            w.y = bf16_bits(o[2]) | (bf16_bits(o[3]) << 16);
            *reinterpret_cast<uint2*>(cell) = w;
        }
    }
    __syncthreads();   // every wave has read dz2 and written its dz1 cells
#pragma unroll
    for (int j = 0; j < 4; ++j) red[1024 + t * 4 + j] = cs1[j];
    __syncthreads();
    if (t < 16) {
        const int gg = t >> 2, j = t & 3;
        float s = 0.0f;
        for (int w = 0; w < 4; ++w)
            for (int nn = 0; nn < 16; ++nn) s += red[1024 + (w * 64 + gg * 16 + nn) * 4 + j];
        out[kOffB1 + t] = s;
    }

    // ---- dW1[tap][ci][co] = sum_q x[q + off(tap)][ci] dz1[q][co]; M = 4 taps x 4 channels,
    //      wave w < 3 owns taps 4w .. 4w+3
    if (wave < 3) {
        f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
        const int tap = 4 * wave + (n >> 2), ci = n & 3;
        const int dyx = tap < 9 ? tap_dy(tap) * kXW + tap_dx(tap) : 0;
        for (int kc = 0; kc < 32; ++kc) {
            const int rr = kc >> 1, xq = 2 + 32 * (kc & 1) + 8 * g;
            const uint4 B = pack8(a1 + ((rr + 1) * kXW + xq) * 16 + n, 16);            // dz1[q][co = n]
            const uint4 A = tap < 9 ? pack8(feat + ((rr + 1) * kXW + xq + dyx) * 4 + ci, 4) : make_uint4(0u, 0u, 0u, 0u);
            d = mfma(A, B, d);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 4 * g + j, tp = 4 * wave + (m >> 2), c = m & 3;
            if (tp < 9) out[kOffW1 + (tp * 4 + c) * 16 + n] = d[j];
        }
    }

    // ---- loss and db3: wave sums, then the waves in order
    for (int o = 32; o > 0; o >>= 1) {
        loss += __shfl_xor(loss, o, 64);
        db3 += __shfl_xor(db3, o, 64);
    }
    __syncthreads();
    if (lane == 0) { red[2 * wave] = loss; red[2 * wave + 1] = db3; }
    __syncthreads();
    if (t == 0) {
        out[kLossSlot] = ((red[0] + red[2]) + red[4]) + red[6];
        out[kOffB3] = ((red[1] + red[3]) + red[5]) + red[7];
    }
}

// grad[i] = sum over the workgroups, in workgroup order
__global__ void k_cnn_reduce(const float* part, int nwg, float* grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kPart || (i >= kNP && i != kLossSlot)) return;
    float s = 0.0f;
    for (int w = 0; w < nwg; ++w) s += part[(int64_t)w * kPart + i];
    grad[i] = s;
}

__global__ void k_cnn_adam(float* master, float* m, float* v, const float* grad, float lr, float b1, float b2,
                           float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNP) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    master[i] = master[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 A operands from the FP32 masters (one thread per lane of a chunk)
__global__ void k_cnn_pack(const float* w, uint4* wpk) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= kChunks * 64) return;
    const int chunk = id / 64, l = id % 64, m = l & 15, g = l >> 4;
    uint32_t h[8];
    for (int j = 0; j < 8; ++j) {
        float x = 0.0f;
        if (chunk < 2) {                      // layer 1: tap 8c + 2g + j/4, input j%4, output m
            const int tap = 8 * chunk + 2 * g + j / 4;
            if (tap < 9) x = w[kOffW1 + (tap * 4 + j % 4) * 16 + m];
        } else if (chunk < 7) {               // layer 2: tap 2c + g/2, input 8(g%2) + j, output m
            const int tap = 2 * (chunk - 2) + g / 2;
            if (tap < 9) x = w[kOffW2 + (tap * 16 + 8 * (g & 1) + j) * 16 + m];
        } else if (chunk < 12) {              // layer 3: only output 0
            const int tap = 2 * (chunk - 7) + g / 2;
            if (tap < 9 && m == 0) x = w[kOffW3 + tap * 16 + 8 * (g & 1) + j];
        } else if (chunk == 12) {             // dL/da2: row = channel m, column = tap 8g + j
            const int tap = 8 * g + j;
            if (tap < 9) x = w[kOffW3 + tap * 16 + m];
        } else if (chunk < 18) {              // dL/da1: row = input m, K = (tap 2c + g/2, output 8(g%2) + j)
            const int tap = 2 * (chunk - 13) + g / 2;
            if (tap < 9) x = w[kOffW2 + (tap * 16 + m) * 16 + 8 * (g & 1) + j];
        } else {                              // row sweep, layer 2 (18 .. 22); layer 3 (23 .. 27) in all 16 rows
            const int c = (chunk - 18) % 5, hi = g >= 2, in = 8 * (g & 1) + j;
            int dy = 1, dx = 1;
            bool zero = false;
            if (c < 3) { dy = c - 1; dx = hi ? 0 : -1; }          // P of dy: dx = -1 | dx = 0
            else if (c == 3) { dy = hi ? 0 : -1; }                 // Q for row ri+1: dy = -1 | dy = 0
            else zero = hi;                                        // Q for row ri-1: dy = +1 | zero
            const int tap = (dy + 1) * 3 + (dx + 1);
            if (!zero) x = chunk < 23 ? w[kOffW2 + (tap * 16 + in) * 16 + m] : w[kOffW3 + tap * 16 + in];
        }
        h[j] = bf16_bits(x);
    }
    wpk[id] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// Labels: 1 within radius + radius_per_disp * f(v) columns of a detected lane curve on the
// band rows, else 0; 255 (ignored) where the frame has no band.
__global__ void k_cnn_labels(ldi_frame_view V, int nb, const ld_lanes* lanes, const float* curves, float radius,
                             float radius_per_disp, uint8_t* labels) {
    const int b = blockIdx.z, band = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int W = V.W, H = V.H;
    if (i >= kBR * W) return;
    if (V.nact != nullptr && b >= *V.nact) return;
    const int r = i / W, u = i % W;
    uint8_t* out = labels + ((int64_t)b * nb + band) * kBR * W;
    const int top = frame_band_top(V, b, nb, band);
    if (top < 0) { out[i] = 255; return; }
    const int v = top + r;
    const int nl = lanes[b].n;
    const float rad = radius + radius_per_disp * (float)V.tab[(int64_t)b * 6 * H + v];
    uint8_t y = 0;
    for (int l = 0; l < nl && l < LD_MAX_LANES; ++l) {
        const float c = curves[((int64_t)b * LD_MAX_LANES + l) * H + v];
        if (fabsf((float)u - c) <= rad) y = 1;   // NaN (track ended) compares false
    }
    out[i] = y;
}

constexpr size_t kFwdLds = sizeof(uint16_t) * (kFeatElems + kActElems);
static_assert(kStageBytes <= sizeof(uint16_t) * kActElems, "the staged inputs live in the activation buffer");
constexpr size_t kTrainLds =
    sizeof(uint16_t) * (kFeatElems + 2 * kActElems + kLR * kXW) + sizeof(float) * (1024 + 1024) + kStageBytes;

template <typename K>
void allow_lds(K kernel, size_t bytes) {
    static size_t granted = 0;
    if (bytes > granted) {
        if (hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
            granted = bytes;
        else
            (void)hipGetLastError();
    }
}

int col_tiles(int W) { return (W + kCT - 1) / kCT; }

}  // namespace

struct ld_cnn_s {
    ld_cnn_config cfg;
    void* mem;
    float* master;
    float* am;
    float* av;
    float* grad;     // kPart: gradients, loss at kLossSlot
    uint4* wpk;
    float* part;
    int64_t part_rows;
    int64_t step;
    hipStream_t last;
};

namespace {

ld_status hip_ok(hipError_t e) { return e == hipSuccess ? LD_OK : LD_E_HIP; }

ld_status repack(ld_cnn n, hipStream_t st) {
    hipLaunchKernelGGL(k_cnn_pack, dim3((kChunks * 64 + 255) / 256), dim3(256), 0, st, n->master, n->wpk);
    return hip_ok(hipGetLastError());
}

bool valid_config(const ld_cnn_config& c) {
    return c.n_bands >= 1 && c.n_bands <= LDI_MAX_BANDS && c.theta > 0.0f && c.theta < 1.0f && c.delta_x >= 1 &&
           c.delta_x <= 127 && c.dilate >= -1 && c.dilate <= 64 && c.min_votes >= 1 && c.max_batch >= 1 &&
           c.max_batch <= 65535 && c.max_width >= 8 && c.max_width <= 4096 &&
           (c.seed_ransac == 0 || c.seed_ransac == 1);
}

ld_status check_frame(ld_cnn n, ld_frame f, ldi_frame_view& V, const uint8_t* grey, int64_t gp, const void* disp,
                      int64_t dp) {
    if (!n || !f || !grey || !disp) return LD_E_INVAL;
    if (ldi_frame_get_view(f, &V) != LD_OK) return LD_E_INVAL;
    const int es = V.fmt == LD_DISP_U8 ? 1 : (V.fmt == LD_DISP_F32 ? 4 : 2);
    if (gp < V.W || dp < (int64_t)V.W * es || dp % es != 0 || ((uintptr_t)disp % es) != 0) return LD_E_INVAL;
    if (!(V.varpi > 0.0)) return LD_E_INVAL;
    if (V.stage < 1) return LD_E_STATE;
    return LD_OK;
}

}  // namespace

// Internal: decisions of the network into the frame's band buffer (used by ld_detect_pruned).
ld_status ldi_cnn_bits(ld_cnn n, ld_frame f, const uint8_t* grey, int64_t gp, const void* disp, int64_t dp,
                       float* prob_out, int sparse, hipStream_t st) {
    ldi_frame_view V;
    ld_status s = check_frame(n, f, V, grey, gp, disp, dp);
    if (s != LD_OK) return s;
    const int nb = n->cfg.n_bands;
    const double th = (double)n->cfg.theta;
    const float thr_logit = (float)std::log(th / (1.0 - th));
    allow_lds(k_cnn_fwd, kFwdLds);
    Net N{n->wpk, n->master};
    const int64_t units = (int64_t)col_tiles(V.W) * nb * V.active;
    hipLaunchKernelGGL(k_cnn_fwd, dim3((unsigned)((units + kFwdUnits - 1) / kFwdUnits)), dim3(kT), kFwdLds, st, V, N,
                       nb, thr_logit, grey, gp, static_cast<const uint8_t*>(disp), dp, prob_out, sparse);
    s = hip_ok(hipGetLastError());
    if (s == LD_OK) s = ldi_frame_mark_bands(f, nb, st);
    n->last = st;
    return s;
}

const ld_cnn_config* ldi_cnn_config(ld_cnn n) { return n ? &n->cfg : nullptr; }

extern "C" {

void ld_cnn_config_default(ld_cnn_config* c) {
    if (!c) return;
    c->n_bands = 1;
    c->theta = 0.5f;
    c->delta_x = 127;
    c->dilate = -1;
    c->min_votes = 8;
    c->max_batch = 32;
    c->max_width = 1920;
    c->seed_ransac = 0;
}

ld_status ld_cnn_create(const ld_cnn_config* cfg, const float* params, ld_cnn* out) {
    if (!out) return LD_E_INVAL;
    *out = nullptr;
    ld_cnn_config c;
    ld_cnn_config_default(&c);
    if (cfg) c = *cfg;
    if (!valid_config(c)) return LD_E_INVAL;
    ld_cnn n = new (std::nothrow) ld_cnn_s();
    if (!n) return LD_E_NOMEM;
    n->cfg = c;
    n->part_rows = (int64_t)c.max_batch * c.n_bands * col_tiles(c.max_width);
    const size_t fl = 4096;   // floats per small array (>= kPart)
    const size_t bytes = sizeof(float) * fl * 4 + sizeof(uint4) * kChunks * 64 + sizeof(float) * (size_t)n->part_rows * kPart;
    if (hipMalloc(&n->mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete n;
        return LD_E_NOMEM;
    }
    float* base = static_cast<float*>(n->mem);
    n->master = base;
    n->am = base + fl;
    n->av = base + 2 * fl;
    n->grad = base + 3 * fl;
    n->wpk = reinterpret_cast<uint4*>(base + 4 * fl);
    n->part = reinterpret_cast<float*>(n->wpk + kChunks * 64);
    n->step = 0;
    n->last = nullptr;
    ld_status s = hip_ok(hipMemset(n->mem, 0, sizeof(float) * fl * 4));
    if (s == LD_OK && params) s = hip_ok(hipMemcpy(n->master, params, sizeof(float) * kNP, hipMemcpyHostToDevice));
    if (s == LD_OK) s = repack(n, nullptr);
    if (s == LD_OK) s = hip_ok(hipDeviceSynchronize());
    if (s != LD_OK) {
        (void)hipFree(n->mem);
        delete n;
        return s;
    }
    *out = n;
    return LD_OK;
}

ld_status ld_cnn_destroy(ld_cnn n) {
    if (!n) return LD_OK;
    ld_status s = LD_OK;
    if (hipStreamSynchronize(n->last) != hipSuccess) s = LD_E_HIP;
    if (hipFree(n->mem) != hipSuccess) s = LD_E_HIP;
    delete n;
    return s;
}

ld_status ld_cnn_set_params(ld_cnn n, const float* params) {
    if (!n || !params) return LD_E_INVAL;
    if (hipStreamSynchronize(n->last) != hipSuccess) return LD_E_HIP;
    ld_status s = hip_ok(hipMemcpy(n->master, params, sizeof(float) * kNP, hipMemcpyHostToDevice));
    if (s == LD_OK) s = hip_ok(hipMemset(n->am, 0, sizeof(float) * 4096 * 2));
    n->step = 0;
    if (s == LD_OK) s = repack(n, nullptr);
    if (s == LD_OK) s = hip_ok(hipDeviceSynchronize());
    return s;
}

ld_status ld_cnn_get_params(ld_cnn n, float* params) {
    if (!n || !params) return LD_E_INVAL;
    if (hipStreamSynchronize(n->last) != hipSuccess) return LD_E_HIP;
    return hip_ok(hipMemcpy(params, n->master, sizeof(float) * kNP, hipMemcpyDeviceToHost));
}

// Checkpoint file: one header line of JSON, then the FP32 master weights, the Adam first and
// second moments (kNP little-endian float32 each, in that order).
namespace {

constexpr const char* kCkptFormat = "ld_cnn_checkpoint";
constexpr int kCkptVersion = 1;

std::string ckpt_header(const ld_cnn_s& n) {
    char buf[512];
    const ld_cnn_config& c = n.cfg;
    snprintf(buf, sizeof(buf),
             "{\"format\": \"%s\", \"version\": %d, \"params\": %d, \"step\": %lld, \"dtype\": \"float32\", "
             "\"arrays\": [\"master\", \"adam_m\", \"adam_v\"], \"config\": {\"n_bands\": %d, \"theta\": %.9g, "
             "\"delta_x\": %d, \"dilate\": %d, \"min_votes\": %d, \"max_batch\": %d, \"max_width\": %d, "
             "\"seed_ransac\": %d}}\n",
             kCkptFormat, kCkptVersion, kNP, (long long)n.step, c.n_bands, (double)c.theta, c.delta_x, c.dilate,
             c.min_votes, c.max_batch, c.max_width, c.seed_ransac);
    return buf;
}

// the number after "key": in a header line (false if absent)
bool ckpt_number(const std::string& h, const char* key, double& out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t p = h.find(k);
    if (p == std::string::npos) return false;
    const char* s = h.c_str() + p + k.size();
    char* end = nullptr;
    out = strtod(s, &end);
    return end != s;
}

}  // namespace

ld_status ld_cnn_save(ld_cnn n, const char* path) {
    if (!n || !path) return LD_E_INVAL;
    if (hipStreamSynchronize(n->last) != hipSuccess) return LD_E_HIP;
    std::vector<float> buf((size_t)3 * kNP);
    if (hipMemcpy(buf.data(), n->master, sizeof(float) * kNP, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(buf.data() + kNP, n->am, sizeof(float) * kNP, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(buf.data() + 2 * kNP, n->av, sizeof(float) * kNP, hipMemcpyDeviceToHost) != hipSuccess)
        return LD_E_HIP;
    const std::string h = ckpt_header(*n);
    FILE* fp = fopen(path, "wb");
    if (!fp) return LD_E_INVAL;
    const bool ok = fwrite(h.data(), 1, h.size(), fp) == h.size() &&
                    fwrite(buf.data(), sizeof(float), buf.size(), fp) == buf.size();
    const bool closed = fclose(fp) == 0;
    return ok && closed ? LD_OK : LD_E_INVAL;
}

ld_status ld_cnn_load(const char* path, const ld_cnn_config* cfg, ld_cnn* out) {
    if (!path || !out) return LD_E_INVAL;
    *out = nullptr;
    FILE* fp = fopen(path, "rb");
    if (!fp) return LD_E_INVAL;
    std::string h;
    int ch;
    while ((ch = fgetc(fp)) != EOF && ch != '\n' && h.size() < 4096) h.push_back((char)ch);
    std::vector<float> buf((size_t)3 * kNP);
    const bool got = ch == '\n' && fread(buf.data(), sizeof(float), buf.size(), fp) == buf.size() && fgetc(fp) == EOF;
    fclose(fp);
    double version = 0, params = 0, step = -1;
    if (!got || h.find(std::string("\"format\": \"") + kCkptFormat + "\"") == std::string::npos ||
        !ckpt_number(h, "version", version) || version != kCkptVersion || !ckpt_number(h, "params", params) ||
        params != kNP || !ckpt_number(h, "step", step) || step < 0 || step != std::floor(step))
        return LD_E_INVAL;
    ld_cnn_config c;
    if (cfg) {
        c = *cfg;
    } else {
        ld_cnn_config_default(&c);
        double x;
        if (ckpt_number(h, "n_bands", x)) c.n_bands = (int32_t)x;
        if (ckpt_number(h, "theta", x)) c.theta = (float)x;
        if (ckpt_number(h, "delta_x", x)) c.delta_x = (int32_t)x;
        if (ckpt_number(h, "dilate", x)) c.dilate = (int32_t)x;
        if (ckpt_number(h, "min_votes", x)) c.min_votes = (int32_t)x;
        if (ckpt_number(h, "max_batch", x)) c.max_batch = (int32_t)x;
        if (ckpt_number(h, "max_width", x)) c.max_width = (int32_t)x;
        if (ckpt_number(h, "seed_ransac", x)) c.seed_ransac = (int32_t)x;
    }
    if (!valid_config(c)) return LD_E_INVAL;
    ld_cnn n = nullptr;
    ld_status s = ld_cnn_create(&c, buf.data(), &n);
    if (s != LD_OK) return s;
    if (hipMemcpy(n->am, buf.data() + kNP, sizeof(float) * kNP, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->av, buf.data() + 2 * kNP, sizeof(float) * kNP, hipMemcpyHostToDevice) != hipSuccess) {
        ld_cnn_destroy(n);
        return LD_E_HIP;
    }
    n->step = (int64_t)step;
    *out = n;
    return LD_OK;
}

ld_status ld_cnn_forward(ld_cnn n, ld_frame f, const uint8_t* grey, int64_t grey_pitch, const void* disp,
                         int64_t disp_pitch, float* prob_out, void* hip_stream) {
    LdRange rr_("ld_cnn_forward");
    if (prob_out && ((uintptr_t)prob_out % 4) != 0) return LD_E_INVAL;
    return ldi_cnn_bits(n, f, grey, grey_pitch, disp, disp_pitch, prob_out, 0, static_cast<hipStream_t>(hip_stream));
}

ld_status ld_cnn_labels(ld_cnn n, ld_frame f, const ld_lanes* lanes, const float* curves, float radius,
                        float radius_per_disp, uint8_t* labels_out, void* hip_stream) {
    LdRange rr_("ld_cnn_labels");
    if (!n || !f || !lanes || !curves || !labels_out || !(radius >= 0.0f) || !(radius_per_disp >= 0.0f))
        return LD_E_INVAL;
    ldi_frame_view V;
    if (ldi_frame_get_view(f, &V) != LD_OK) return LD_E_INVAL;
    if (V.stage < 1) return LD_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_cnn_labels, dim3((kBR * V.W + 255) / 256, n->cfg.n_bands, V.active), dim3(256), 0, st, V,
                       n->cfg.n_bands, lanes, curves, radius, radius_per_disp, labels_out);
    n->last = st;
    return hip_ok(hipGetLastError());
}

ld_status ld_cnn_train_step(ld_cnn n, ld_frame f, const uint8_t* grey, int64_t grey_pitch, const void* disp,
                            int64_t disp_pitch, const uint8_t* labels, float pos_weight, float inv_norm, float lr,
                            float* loss_out, float* grad_out, void* hip_stream) {
    LdRange rr_("ld_cnn_train_step");
    ldi_frame_view V;
    ld_status s = check_frame(n, f, V, grey, grey_pitch, disp, disp_pitch);
    if (s != LD_OK) return s;
    if (!labels || !(pos_weight > 0.0f) || !(inv_norm > 0.0f) || !(lr >= 0.0f)) return LD_E_INVAL;
    const int nb = n->cfg.n_bands, nct = col_tiles(V.W);
    const int64_t nwg = (int64_t)V.active * nb * nct;
    if (nwg > n->part_rows) return LD_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    allow_lds(k_cnn_train, kTrainLds);
    Net N{n->wpk, n->master};
    hipLaunchKernelGGL(k_cnn_train, dim3(nct, nb, V.active), dim3(kT), kTrainLds, st, V, N, nb, grey, grey_pitch,
                       static_cast<const uint8_t*>(disp), disp_pitch, labels, pos_weight, inv_norm, n->part);
    if ((s = hip_ok(hipGetLastError())) != LD_OK) return s;
    hipLaunchKernelGGL(k_cnn_reduce, dim3((kPart + 255) / 256), dim3(256), 0, st, n->part, (int)nwg, n->grad);
    if ((s = hip_ok(hipGetLastError())) != LD_OK) return s;
    if (grad_out && hipMemcpyAsync(grad_out, n->grad, sizeof(float) * kNP, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return LD_E_HIP;
    if (loss_out &&
        hipMemcpyAsync(loss_out, n->grad + kLossSlot, sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return LD_E_HIP;
    if (lr > 0.0f) {
        n->step += 1;
        const double b1 = 0.9, b2 = 0.999;
        const float bc1 = (float)(1.0 - std::pow(b1, (double)n->step));
        const float bc2 = (float)(1.0 - std::pow(b2, (double)n->step));
        hipLaunchKernelGGL(k_cnn_adam, dim3((kNP + 255) / 256), dim3(256), 0, st, n->master, n->am, n->av, n->grad, lr,
                           (float)b1, (float)b2, 1e-8f, bc1, bc2);
        if ((s = hip_ok(hipGetLastError())) != LD_OK) return s;
        if ((s = repack(n, st)) != LD_OK) return s;
    }
    n->last = st;
    return LD_OK;
}

}  // extern "C"
