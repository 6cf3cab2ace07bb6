// Device-side building blocks shared by the librcp kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcp {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Counter-based Gaussian test matrix (Section 3.1: Gaussian random vectors
// omega_1..omega_l; Algorithm 1's test-matrix draw).  Philox4x32-10 from Salmon, Moraes,
// Dror, Shaw (SC'11): ten rounds of two 32x32->64 multiplies with the
// constants below, key bumped by the Weyl increments between rounds.

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        U4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return c;
}

// u = ((x >> 8) + 1) * 2^-24 in (0, 1], exact in float32.
__device__ __forceinline__ float uniform24(uint32_t x) {
    return (float)((x >> 8) + 1u) * 5.9604644775390625e-08f;
}

// Four N(0,1) values of row j, columns 4g..4g+3 of Omega (Box-Muller on the
// pairs (u0,u1) and (u2,u3); cos/sin of 2*pi*u through sinpi/cospi of 2u,
// which is exact in the argument).
__device__ __forceinline__ void omega4(uint64_t seed, uint32_t tag, uint64_t j, uint32_t g,
                                       float out[4]) {
    U4 c;
    c.x = (uint32_t)j;
    c.y = (uint32_t)(j >> 32);
    c.z = g;
    c.w = tag;
    const U4 x = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u0 = uniform24(x.x), u1 = uniform24(x.y);
    const float u2 = uniform24(x.z), u3 = uniform24(x.w);
    const float ra = sqrtf(-2.0f * logf(u0));
    const float rb = sqrtf(-2.0f * logf(u2));
    float sa, ca, sb, cb;
    sincospif(2.0f * u1, &sa, &ca);
    sincospif(2.0f * u3, &sb, &cb);
    out[0] = ra * ca;
    out[1] = ra * sa;
    out[2] = rb * cb;
    out[3] = rb * sb;
}

// Test-matrix kinds (values of rcp_problem.test_matrix generated in-kernel).
constexpr int kOmegaGaussian = 0;
constexpr int kOmegaUniform = 1;
constexpr int kOmegaHalton = 2;

// The first 64 primes: Halton base of columns 0..63.
__device__ __forceinline__ uint32_t halton_base(int c) {
    constexpr uint32_t p[64] = {2,   3,   5,   7,   11,  13,  17,  19,  23,  29,  31,  37,  41,
                                43,  47,  53,  59,  61,  67,  71,  73,  79,  83,  89,  97,  101,
                                103, 107, 109, 113, 127, 131, 137, 139, 149, 151, 157, 163, 167,
                                173, 179, 181, 191, 193, 197, 199, 211, 223, 227, 229, 233, 239,
                                241, 251, 257, 263, 269, 271, 277, 281, 283, 293, 307, 311};
    return p[c & 63];
}

// Radical inverse of i >= 1 in base b (digits mirrored about the radix
// point): the exact ratio num / b^digits, rounded once to float.
__device__ __forceinline__ float radical_inverse(uint64_t i, uint32_t b) {
    uint64_t num = 0, den = 1;
    while (i > 0) {
        const uint64_t q = i / b;
        num = num * b + (i - q * b);
        den *= b;
        i = q;
    }
    return (float)((double)num / (double)den);
}

// Four entries of row j, columns 4g..4g+3, of a test matrix of the given kind.
__device__ __forceinline__ void omega4k(int kind, uint64_t seed, uint32_t tag, uint64_t j,
                                        uint32_t g, float out[4]) {
    if (kind == kOmegaHalton) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = 4 * (int)g + v;
            out[v] = (c < 64) ? radical_inverse(j + 1, halton_base(c)) : 0.0f;
        }
        return;
    }
    if (kind == kOmegaUniform) {
        U4 c;
        c.x = (uint32_t)j;
        c.y = (uint32_t)(j >> 32);
        c.z = g;
        c.w = tag;
        const U4 x = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        out[0] = uniform24(x.x);
        out[1] = uniform24(x.y);
        out[2] = uniform24(x.z);
        out[3] = uniform24(x.w);
        return;
    }
    omega4(seed, tag, j, g, out);
}

__device__ __forceinline__ uint32_t omega_tag(uint32_t batch, uint32_t mode) {
    return (batch << 8) | (mode & 0xFFu);
}

// ---------------------------------------------------------------------------
// Matrix-core FP32 product: D(16x16) += A(16x4) B(4x16) on one wavefront.
// Lane layout (v_mfma_f32_16x16x4_f32): lane holds A[lane%16][lane/16],
// B[lane/16][lane%16] and D[4*(lane/16)+v][lane%16], v = 0..3.

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Reductions.

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float warp_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sum of one double; `red` holds >= blockDim.x/64 doubles.
// Every thread receives the total.  Contains two __syncthreads.
__device__ __forceinline__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = warp_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}


// x / d on the serial path of an elimination, where the IEEE division
// sequence (about ten dependent float64 operations) is the latency: the
// hardware reciprocal refined by two Newton steps, then one multiply; within
// about an ulp of the rounded quotient for finite nonzero d (a zero or NaN d
// gives NaN, which the callers' pivot tests reject).
__device__ __forceinline__ double div_pivot(double x, double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    return x * r;
}

// a double of lane `lane` (wave-uniform) to every lane of the wavefront
__device__ __forceinline__ double readlane_f64(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Exact-ish integer quotient of small non-negative values (< 2^22) by a
// positive divisor, using a float reciprocal plus one correction step.
__device__ __forceinline__ int small_div(int a, int d, float inv_d) {
    int q = (int)((float)a * inv_d);
    int r = a - q * d;
    if (r < 0) { --q; r += d; }
    if (r >= d) { ++q; }
    return q;
}

// ---------------------------------------------------------------------------
// 16-bit matrix-core operands (values of rcp_problem.precision)
constexpr int kPrecFp32 = 0;
constexpr int kPrecBf16 = 1;
constexpr int kPrecFp16 = 2;

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));

// four float32 values rounded to nearest even in the 16-bit operand format
template <int PR>
__device__ __forceinline__ s16x4 to_lp(float4 v) {
    if constexpr (PR == kPrecBf16) {
        const bf16x4_t b = {(__bf16)v.x, (__bf16)v.y, (__bf16)v.z, (__bf16)v.w};
        return __builtin_bit_cast(s16x4, b);
    } else {
        const f16x4_t h = {(_Float16)v.x, (_Float16)v.y, (_Float16)v.z, (_Float16)v.w};
        return __builtin_bit_cast(s16x4, h);
    }
}

// D += A B with A 16 x 16 (lane l: row l % 16, k = 4 (l / 16) .. + 3),
// B 16 x 16 (lane l: column l % 16, same k), float32 accumulation; D in the
// layout of mfma16x16x4.
template <int PR>
__device__ __forceinline__ f32x4 mfma_lp(s16x4 a, s16x4 b, f32x4 c) {
    if constexpr (PR == kPrecBf16)
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(f16x4_t, a),
                                                     __builtin_bit_cast(f16x4_t, b), c, 0, 0, 0);
}

// D += A B on the float64 matrix cores (v_mfma_f64_16x16x4_f64): A operand
// [i][k] in lane i + 16 k, B operand [k][j] in lane j + 16 k, result element
// v of lane l is [l / 16 + 4 v][l % 16].
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace rcp
