// convert.hip -- reduced-precision copies of the rows (bfloat16 and OCP
// FP8 e4m3 with a per-row scale), their squared norms, and small utility
// kernels of the query path.
//
// bfloat16: the upper 16 bits of the float32 pattern after round-to-nearest-
// even at bit 16.  e4m3 (OCP 8-bit floating point, E4M3): 1 sign, 4 exponent
// (bias 7), 3 mantissa bits; no infinities; 0x7F/0xFF are NaN; the largest
// finite magnitude is 448 = 1.75 * 2^8; subnormals step by 2^-9.  Rows are
// scaled by s = max|x| / 448 before rounding (nearest-even, saturating), so
// x ~= s * decode(code).  The squared norms are those of the rounded rows,
// which makes ||x||^2 - 2 q.x + ||q||^2 the exact distance between the
// rounded vectors up to the FP32 accumulation.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace gf {

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ __forceinline__ float bf16_value(uint16_t h) {
    return __uint_as_float(uint32_t(h) << 16);
}

__device__ __forceinline__ uint8_t e4m3_encode(float y) {
    const uint32_t sign = (__float_as_uint(y) >> 24) & 0x80u;
    const float a = fabsf(y);
    uint32_t code;
    if (!(a < 448.0f)) {
        code = 0x7Eu;                                   // saturate to 448
    } else if (a < 0.015625f) {                         // below 2^-6: subnormal
        code = uint32_t(rintf(a * 512.0f));             // 0..8 (8 = 2^-6, exp 1)
    } else {
        int e;
        (void)frexpf(a, &e);                            // a = f * 2^e, f in [0.5, 1)
        int E = e - 1;                                  // a = 1.m * 2^E
        int mant = int(rintf((ldexpf(a, -E) - 1.0f) * 8.0f));
        if (mant == 8) { mant = 0; E += 1; }
        code = uint32_t((E + 7) << 3) | uint32_t(mant);
        if (code > 0x7Eu) code = 0x7Eu;
    }
    return uint8_t(sign | code);
}

__device__ __forceinline__ float e4m3_value(uint8_t c) {
    const int E = (c >> 3) & 0xF, mant = c & 7;
    const float mag = (E == 0) ? ldexpf(float(mant), -9) : ldexpf(1.0f + float(mant) * 0.125f, E - 7);
    return (c & 0x80) ? -mag : mag;
}

// One wavefront per row.
__global__ void k_to_bf16(const float* X, int64_t n, int d, int64_t ldx, uint16_t* Y,
                          int64_t ldy, float* norm) {
    const int64_t row = int64_t(blockIdx.x) * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float* x = X + row * ldx;
    uint16_t* y = Y + row * ldy;
    float acc = 0.0f;
    for (int64_t j = lane; j < ldy; j += 64) {
        const uint16_t h = (j < d) ? bf16_rne(x[j]) : uint16_t(0);
        y[j] = h;
        const float v = bf16_value(h);
        acc = fmaf(v, v, acc);
    }
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0 && norm) norm[row] = acc;
}

__global__ void k_to_fp8(const float* X, int64_t n, int d, int64_t ldx, uint8_t* Y,
                         int64_t ldy, float* scale, float* norm) {
    const int64_t row = int64_t(blockIdx.x) * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float* x = X + row * ldx;
    uint8_t* y = Y + row * ldy;
    float mx = 0.0f;
    for (int j = lane; j < d; j += 64) mx = fmaxf(mx, fabsf(x[j]));
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    const float s = (mx > 0.0f) ? mx / 448.0f : 1.0f;
    float acc = 0.0f;
    for (int64_t j = lane; j < ldy; j += 64) {
        const uint8_t c = (j < d) ? e4m3_encode(x[j] / s) : uint8_t(0);
        y[j] = c;
        const float v = e4m3_value(c) * s;
        acc = fmaf(v, v, acc);
    }
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
        scale[row] = s;
        if (norm) norm[row] = acc;
    }
}

__global__ void k_pad_rows(const float* X, int64_t n, int d, float* Y, int64_t ldy) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n * ldy) return;
    const int64_t r = i / ldy, j = i % ldy;
    Y[i] = (j < d) ? X[r * d + j] : 0.0f;
}

// Flags a non-finite value in an [n][d] (stride ld) float matrix.
__global__ void k_check_finite(const float* X, int64_t n, int d, int64_t ld, uint32_t* bad) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n * int64_t(d)) return;
    const int64_t r = i / d, j = i % d;
    if (!isfinite(X[r * ld + j])) atomicOr(bad, 1u);
}

// [m][W][nq] word-major leaf bits -> [nq][m][W].
__global__ void k_leafbits_to_query_major(const uint32_t* src, int nq, int64_t words,
                                          uint32_t* dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= words * nq) return;
    const int64_t w = i / nq, q = i % nq;
    dst[q * words + w] = src[i];
}

// Decode table check: every e4m3 code through the hardware conversion and
// through the format definition (used by the tests).
__global__ void k_e4m3_decode_both(float* hw, float* sw) {
    const uint32_t c = threadIdx.x;   // 256 threads
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = __builtin_amdgcn_cvt_pk_f32_fp8(c, false);
    hw[c] = v.x;
    sw[c] = e4m3_value(uint8_t(c));
}

__global__ void k_e4m3_encode(const float* x, int n, uint8_t* y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = e4m3_encode(x[i]);
}

}  // namespace gf
