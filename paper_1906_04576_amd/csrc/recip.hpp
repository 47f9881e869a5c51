// Correctly rounded reciprocal without the IEEE division sequence.
//
// y0 = v_rcp_f32(d) is within one ulp of 1/d; one Newton-Raphson step done
// with fused multiply-adds (Markstein's reciprocal iteration: the residual
// e = 1 - d y0 is exact in an FMA, and y0 + e y0 is rounded once) gives the
// correctly rounded 1/d.  tests/native/recip_check.hip compares it with the
// IEEE division 1.0f / d for every float d in [2^-126, 2^126); outside that
// range (denormal d, or a denormal result) callers use the division.
#pragma once

namespace mr {

constexpr float kRecipLo = 0x1p-126f, kRecipHi = 0x1p126f;

// valid (equal to 1.0f / d) for kRecipLo <= d < kRecipHi
__device__ __forceinline__ float recip_fast(float d) {
    const float y0 = __builtin_amdgcn_rcpf(d);
    const float e = __builtin_fmaf(-d, y0, 1.0f);
    return __builtin_fmaf(e, y0, y0);
}

// 1.0f / d for d > 0 (any value for d <= 0 or NaN: callers discard it).
// The division runs only in waves that hold such an extreme d (a branch on
// the wave's ballot, so that it is not evaluated speculatively).
__device__ __forceinline__ float recip_pos(float d) {
    float r = recip_fast(d);
    const bool slow = (d > 0.0f && d < kRecipLo) || d >= kRecipHi;
    if (__builtin_expect(__ballot(slow) != 0, 0)) {
        if (slow) r = 1.0f / d;
    }
    return r;
}

// 1.0f / sqrtf(x) for x > 0: sqrtf of a positive finite float lies in
// [2^-75, 2^64], inside the exact range of recip_fast; 1/sqrt(+inf) = +0.
__device__ __forceinline__ float rsqrt_pos(float x) {
    return x < __builtin_inff() ? recip_fast(sqrtf(x)) : 0.0f;
}

}  // namespace mr
