// ld_device.h -- device-side building blocks of the lane-detection kernels (gfx950,
// wave64).  Decision arithmetic (fits, inlier tests, vote bins, gates, track columns) is
// FP64 in a fixed operation order; the library is compiled with -ffp-contract=off so that
// no multiply-add is fused unless written as fma().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ld.h"

namespace ldk {

typedef __int128 i128;
typedef unsigned __int128 u128;

constexpr int kWave = 64;
constexpr int kBlock = 256;          // default workgroup size
constexpr int kMaxWaves = 16;        // up to 1024 threads per workgroup
constexpr int kMaxHyp = 64;          // one RANSAC hypothesis per lane of a wave

// ------------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int wave_sum_i32(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ __forceinline__ int wave_max_i32(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, kWave));
    return x;
}

__device__ __forceinline__ int wave_min_i32(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, kWave));
    return x;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int o) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    lo = __shfl_xor(lo, o, kWave);
    hi = __shfl_xor(hi, o, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// exact 128-bit sum across the wave (integer addition is associative: any order is exact)
__device__ __forceinline__ i128 wave_sum_i128(i128 x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t lo = shfl_xor_u64((uint64_t)(u128)x, o);
        uint64_t hi = shfl_xor_u64((uint64_t)((u128)x >> 64), o);
        x += (i128)(((u128)hi << 64) | (u128)lo);
    }
    return x;
}

// (value, index) minimum across the wave; ties go to the smaller index
__device__ __forceinline__ void wave_argmin_i64(int64_t& v, int& i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int64_t ov = (int64_t)shfl_xor_u64((uint64_t)v, o);
        int oi = __shfl_xor(i, o, kWave);
        if (ov < v || (ov == v && oi < i)) { v = ov; i = oi; }
    }
}

// ------------------------------------------------------------------------ Philox4x64-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds, each two 64x64->128
// products; the key advances by the Weyl constants between rounds.
struct U64x4 { uint64_t w[4]; };

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    U64x4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

// ------------------------------------------------------------------------ exact-moment LSF
// Least squares in s = (x - center) / 2^k from exact integer moments (any summation order
// gives the same integers), converted to FP64 half by half, then Gaussian elimination
// without pivoting and back substitution, all in a fixed order.
__device__ __forceinline__ double i128_to_f64(i128 v) {
    bool neg = v < 0;
    u128 a = neg ? (u128)(-v) : (u128)v;
    uint64_t hi = (uint64_t)(a >> 64), lo = (uint64_t)a;
    double d = (double)hi * 18446744073709551616.0 + (double)lo;
    return neg ? -d : d;
}

struct Moments {
    i128 sw[9];    // sum w^p, p = 0..2m
    i128 syw[5];   // sum y w^p, p = 0..m
};

__device__ __forceinline__ void moments_zero(Moments& M) {
#pragma unroll
    for (int p = 0; p < 9; ++p) M.sw[p] = 0;
#pragma unroll
    for (int p = 0; p < 5; ++p) M.syw[p] = 0;
}

// |w| < 2^12 and |y| < 2^14 (frames of at most 4096 rows and columns): w^p fits in int64 up
// to p = 5 and y w^p up to p = 4; the higher powers are exact 64 x 64 -> 128-bit products.
template <int DEG>
__device__ __forceinline__ void moments_add(Moments& M, int x, int y, int center) {
    const int64_t w = x - center;
    int64_t pw[6];
    pw[0] = 1;
#pragma unroll
    for (int p = 1; p <= 5; ++p) pw[p] = pw[p - 1] * w;
#pragma unroll
    for (int p = 0; p <= 2 * DEG; ++p) {
        if (p <= 5) M.sw[p] += (i128)pw[p];
        else M.sw[p] += (i128)pw[4] * (i128)pw[p - 4];
        if (p <= DEG) M.syw[p] += (i128)(pw[p] * (int64_t)y);
    }
}

// returns true on success (every pivot positive, finite coefficients)
template <int DEG>
__device__ bool solve_moments(const Moments& M, int kshift, double* coef) {
    constexpr int N = DEG + 1;
    double A[N][N], b[N], sc[2 * DEG + 1];
#pragma unroll
    for (int p = 0; p <= 2 * DEG; ++p) sc[p] = ldexp(1.0, -kshift * p);
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) A[i][j] = i128_to_f64(M.sw[i + j]) * sc[i + j];
        b[i] = i128_to_f64(M.syw[i]) * sc[i];
    }
    bool ok = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        ok = ok && (A[i][i] > 0.0);
#pragma unroll
        for (int j = i + 1; j < N; ++j) {
            double f = A[j][i] / A[i][i];
#pragma unroll
            for (int l = i; l < N; ++l) A[j][l] = A[j][l] - f * A[i][l];
            b[j] = b[j] - f * b[i];
        }
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int l = i + 1; l < N; ++l) s = s - A[i][l] * coef[l];
        coef[i] = s / A[i][i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) ok = ok && isfinite(coef[i]);
    return ok;
}

// model value at integer x, Horner in s
template <int DEG>
__device__ __forceinline__ double eval_s(const double* c, int center, int kshift, int x) {
    double s = (double)(x - center) * ldexp(1.0, -kshift);
    double r = c[DEG];
#pragma unroll
    for (int p = DEG - 1; p >= 0; --p) r = r * s + c[p];
    return r;
}

// raw-basis polynomial (caller seeds), Horner in x
template <int DEG>
__device__ __forceinline__ double eval_raw(const double* g, int x) {
    double xv = (double)x;
    double r = g[DEG];
#pragma unroll
    for (int p = DEG - 1; p >= 0; --p) r = r * xv + g[p];
    return r;
}

// s-basis -> raw basis (reporting only)
template <int DEG>
__device__ void to_raw(const double* c, int center, int kshift, double* raw) {
    for (int q = 0; q <= DEG; ++q) raw[q] = 0.0;
    for (int p = 0; p <= DEG; ++p) {
        double cp = c[p] * ldexp(1.0, -kshift * p);
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

}  // namespace ldk
