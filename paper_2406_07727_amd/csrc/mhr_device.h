// Device helpers shared by the query kernels: float-float (double-FP32)
// arithmetic, the two log-sigmoid evaluations, embedding row loads and the
// total order on candidate paths.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhr {

constexpr int kWave = 64;
constexpr float kLn2f = 0.693147180559945309417f;
constexpr float kUnit = 5.9604644775390625e-08f;  // 2^-24, unit roundoff of FP32

// ---------------------------------------------------------------------------
// Float-float arithmetic.  A value is hi + lo with |lo| <= ulp(hi)/2.  The
// error-free transformations are Knuth's TwoSum, Dekker's FastTwoSum and the
// FMA-based TwoProduct; the double-word sum and products follow Joldes,
// Muller and Popescu, "Tight and rigorous error bounds for basic building
// blocks of double-word arithmetic" (ACM TOMS 2017): relative error below
// 3u^2 for the sum and 5u^2 for the product.  Contraction is disabled here
// so the compiler cannot fuse the operations these transformations rely on.
// ---------------------------------------------------------------------------
struct ff {
    float hi, lo;
};

#pragma clang fp contract(off)

__device__ __forceinline__ ff two_sum(float a, float b) {
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ ff fast_two_sum(float a, float b) {  // needs |a| >= |b| or a == 0
    float s = a + b;
    float e = b - (s - a);
    return {s, e};
}

__device__ __forceinline__ ff two_prod(float a, float b) {
    float p = a * b;
    float e = __builtin_fmaf(a, b, -p);
    return {p, e};
}

__device__ __forceinline__ ff ff_add(ff x, ff y) {
    ff s = two_sum(x.hi, y.hi);
    ff t = two_sum(x.lo, y.lo);
    float c = s.lo + t.hi;
    ff v = fast_two_sum(s.hi, c);
    float w = t.lo + v.lo;
    return fast_two_sum(v.hi, w);
}

__device__ __forceinline__ ff ff_add_f(ff x, float y) {
    ff s = two_sum(x.hi, y);
    float v = x.lo + s.lo;
    return fast_two_sum(s.hi, v);
}

__device__ __forceinline__ ff ff_neg(ff x) { return {-x.hi, -x.lo}; }

__device__ __forceinline__ ff ff_mul(ff x, ff y) {
    ff c = two_prod(x.hi, y.hi);
    float tl = x.hi * y.lo;
    float cl2 = __builtin_fmaf(x.lo, y.hi, tl);
    float cl3 = c.lo + cl2;
    return fast_two_sum(c.hi, cl3);
}

__device__ __forceinline__ ff ff_mul_f(ff x, float y) {
    ff c = two_prod(x.hi, y);
    float cl3 = __builtin_fmaf(x.lo, y, c.lo);
    return fast_two_sum(c.hi, cl3);
}

#pragma clang fp contract(on)

// 1/n! for n = 0..13 as float-float constants, split at compile time.
struct ffc {
    float hi, lo;
};
__device__ constexpr ffc inv_fact_split(double v) {
    return {static_cast<float>(v), static_cast<float>(v - static_cast<double>(static_cast<float>(v)))};
}
__device__ constexpr ffc kInvFact[14] = {
    inv_fact_split(1.0),
    inv_fact_split(1.0),
    inv_fact_split(1.0 / 2.0),
    inv_fact_split(1.0 / 6.0),
    inv_fact_split(1.0 / 24.0),
    inv_fact_split(1.0 / 120.0),
    inv_fact_split(1.0 / 720.0),
    inv_fact_split(1.0 / 5040.0),
    inv_fact_split(1.0 / 40320.0),
    inv_fact_split(1.0 / 362880.0),
    inv_fact_split(1.0 / 3628800.0),
    inv_fact_split(1.0 / 39916800.0),
    inv_fact_split(1.0 / 479001600.0),
    inv_fact_split(1.0 / 6227020800.0),
};
// ln 2 split into a float and the float nearest to the remainder.
__device__ constexpr ffc kLn2ff = inv_fact_split(0.69314718055994530941723212145818);

// e^a for a <= 0 in float-float.  a = k ln2 + r with |r| <= ln2/2 (plus
// rounding), e^r from its Taylor series to degree 13 (truncation below
// 2^-50 for |r| < 0.35), scaled by 2^k.
__device__ inline ff ff_exp_nonpos(ff a) {
    if (a.hi < -103.0f) return {0.0f, 0.0f};
    float kf = rintf(a.hi * 1.4426950408889634f);
    ff kl = ff_mul_f(ff{kLn2ff.hi, kLn2ff.lo}, kf);
    ff r = ff_add(a, ff_neg(kl));
    ff p = {kInvFact[13].hi, kInvFact[13].lo};
#pragma unroll
    for (int n = 12; n >= 0; --n) p = ff_add(ff_mul(p, r), ff{kInvFact[n].hi, kInvFact[n].lo});
    int k = static_cast<int>(kf);
    return {ldexpf(p.hi, k), ldexpf(p.lo, k)};
}

// log(1 + z) for 0 < z <= 1 in float-float: one Newton step on e^y = 1 + z
// from the FP32 estimate y0 = log1pf(z):  y1 = y0 + (1 + z) e^{-y0} - 1.
// The step squares the relative error of y0 (a few 2^-24), leaving about
// 2^-46 after the float-float rounding.
__device__ inline ff ff_log1p_unit(ff z) {
    float y0 = log1pf(z.hi);
    ff e = ff_exp_nonpos(ff{-y0, 0.0f});
    ff t = ff_mul(ff_add_f(z, 1.0f), e);
    ff d = ff_add_f(t, -1.0f);
    return ff_add_f(d, y0);
}

// logsigmoid(x) = min(x, 0) - log1p(exp(-|x|)) in float-float.
__device__ inline ff ff_logsigmoid(ff x) {
    const bool neg = x.hi < 0.0f;
    ff v = neg ? ff_neg(x) : x;
    ff z = ff_exp_nonpos(ff_neg(v));
    ff g = (z.hi == 0.0f) ? ff{0.0f, 0.0f} : ff_log1p_unit(z);
    ff m = neg ? x : ff{0.0f, 0.0f};
    return ff_add(m, ff_neg(g));
}

// Generous bound on the float-float log-sigmoid error (absolute):
// 2^-42 (1 + |w|).
__device__ __forceinline__ float ff_logsigmoid_err(float w) { return 2.2737368e-13f * (1.0f + fabsf(w)); }

// Centred log-sigmoid in FP32: f(x) = logsigmoid(x) + ln 2
// = -log1p(expm1(-x) / 2).  Near x = 0, where every weight of these
// workloads lies, f(x) is about x/2, so its rounding error is relative to a
// value ~100x smaller than logsigmoid itself.  For x < -15, where expm1(-x)
// would overflow for large |x|, f = x + ln 2 - log1p(e^x) ~ x + ln 2 - e^x.
__device__ __forceinline__ float centred_logsigmoid(float x) {
    if (x >= -15.0f) return -log1pf(0.5f * expm1f(-x));
    return (x + kLn2f) - expf(x);
}

// Error model for centred_logsigmoid: 16 units of roundoff relative to
// |f| (expm1f and log1pf are accurate to a couple of ulps; the margin
// covers the composition).
__device__ __forceinline__ float centred_logsigmoid_err(float f) { return 16.0f * kUnit * fabsf(f); }

// The centred log-sigmoid with a rigorous bound on its FP32 error, for the
// fast pass.  For |x| <= 1/2 it uses f(x) = x/2 - log cosh(x/2) and the
// Taylor series of log cosh(y) (y = x/2, z = y^2):
//     z/2 - z^2/12 + z^3/45 - 17 z^4/2520 + 31 z^5/14175 - ...
// alternating with decreasing terms for |y| < pi/2; the first omitted term,
// 691 z^6/467775, is below 1e-10 for |y| <= 1/4.  Horner's rule in z costs
// five fused multiply-adds; its rounding error (the rounded constants, z,
// each step and the final subtraction) stays below 16 u (|x|/2 + z).
// Larger |x| (rare: x has a spread of about 1/d) take the library path.
__device__ __forceinline__ float centred_logsigmoid_e(float x, float &err) {
    if (fabsf(x) <= 0.5f) {
        const float y = 0.5f * x;
        const float z = y * y;
        float lc = 31.0f / 14175.0f;
        lc = fmaf(lc, z, -17.0f / 2520.0f);
        lc = fmaf(lc, z, 1.0f / 45.0f);
        lc = fmaf(lc, z, -1.0f / 12.0f);
        lc = fmaf(lc, z, 0.5f);
        lc = lc * z;
        err = 16.0f * kUnit * (fabsf(y) + z) + 1e-10f;
        return y - lc;
    }
    const float f = centred_logsigmoid(x);
    err = centred_logsigmoid_err(f);
    return f;
}

// gamma_n = n u / (1 - n u): the classical bound factor for n roundings.
__device__ __forceinline__ float gamma_n(int n) {
    float nu = static_cast<float>(n) * kUnit;
    return nu / (1.0f - nu) * 1.0001f;
}

// ---------------------------------------------------------------------------
// Embedding rows: 8 consecutive elements per lane.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

template <bool BF16>
__device__ __forceinline__ void load8(const void *base, size_t row, uint32_t d, uint32_t off, float (&v)[8]) {
    if (BF16) {
        const uint16_t *p = static_cast<const uint16_t *>(base) + row * d + off;
        uint4 u = *reinterpret_cast<const uint4 *>(p);
        v[0] = bf16_to_f32(u.x & 0xFFFFu); v[1] = bf16_to_f32(u.x >> 16);
        v[2] = bf16_to_f32(u.y & 0xFFFFu); v[3] = bf16_to_f32(u.y >> 16);
        v[4] = bf16_to_f32(u.z & 0xFFFFu); v[5] = bf16_to_f32(u.z >> 16);
        v[6] = bf16_to_f32(u.w & 0xFFFFu); v[7] = bf16_to_f32(u.w >> 16);
    } else {
        const float *p = static_cast<const float *>(base) + row * d + off;
        float4 a = *reinterpret_cast<const float4 *>(p);
        float4 b = *reinterpret_cast<const float4 *>(p + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    }
}

template <bool BF16>
__device__ __forceinline__ float load1(const void *base, size_t idx) {
    if (BF16) return bf16_to_f32(static_cast<const uint16_t *>(base)[idx]);
    return static_cast<const float *>(base)[idx];
}

// Cross-lane moves within rows of 16 lanes (DPP; no LDS traffic).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over an aligned group of G lanes (G a power of two, 4..64); every lane
// of the group receives the total.  Within a row: lane^1 and lane^2 by quad
// permutes, then the other quad of each half-row (half mirror), then the
// other half of the row (mirror); across rows: lane^16, lane^32.
__device__ __forceinline__ float group_sum(float v, int G) {
    v += dpp_f<0xB1>(v);                      // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);                      // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_f<0x141>(v);         // row_half_mirror
    if (G >= 16) v += dpp_f<0x140>(v);        // row_mirror
    if (G >= 32) v += __shfl_xor(v, 16, kWave);
    if (G >= 64) v += __shfl_xor(v, 32, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// Candidate paths and their total order: score descending (hi, then lo),
// then a, b, (r1, r2, r3) ascending.  rel packs r1 << 16 | r2 << 8 | r3.
// ---------------------------------------------------------------------------
struct Cand {
    float s;      // FP32 centred score (fast pass) or float-float hi (rescored)
    float s_lo;   // 0 (fast pass) or float-float lo
    uint32_t a, b, rel;
    float eps;    // error bound of the score
};

__device__ __forceinline__ bool cand_better(const Cand &x, const Cand &y) {
    if (x.s != y.s) return x.s > y.s;
    if (x.s_lo != y.s_lo) return x.s_lo > y.s_lo;
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    return x.rel < y.rel;
}

__device__ __forceinline__ Cand cand_sentinel() {
    Cand c;
    c.s = -__builtin_huge_valf();
    c.s_lo = 0.0f;
    c.a = 0xFFFFFFFFu; c.b = 0xFFFFFFFFu; c.rel = 0xFFFFFFFFu;
    c.eps = 0.0f;
    return c;
}

// Bitonic sort of n (a power of two) LDS candidates, best first, by the
// whole block.  Ends with a barrier.
__device__ inline void block_sort_cands(Cand *c, int n) {
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                int p = i ^ j;
                if (p > i) {
                    Cand x = c[i], y = c[p];
                    bool up = (i & k) == 0;  // this half ends best-first
                    bool swap = up ? cand_better(y, x) : cand_better(x, y);
                    if (swap) { c[i] = y; c[p] = x; }
                }
            }
            __syncthreads();
        }
    }
}

__host__ __device__ constexpr uint32_t next_pow2(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace mhr
