// Device-side arithmetic of the REWL kernels: counter-based RNG, the
// deterministic exponential used by the acceptance tests, two-float (FP32
// compensated) arithmetic and wavefront reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// takes the 64-bit products of counter words 0 and 2 with two fixed
// multipliers, xors their high halves with words 1, 3 and the round key, and
// bumps the key by two Weyl constants.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                   (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
  }
  return c;
}

// Rounds [FIRST, LAST) of Philox4x32-10; round r uses the key bumped r
// times.  philox_rounds<0, 10> equals philox10.  Splitting lets a kernel
// spread the 10 rounds over latency gaps of other work.
template <int FIRST, int LAST>
__device__ __forceinline__ uint4 philox_rounds(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = FIRST; r < LAST; ++r) {
    const uint32_t kr0 = k0 + (uint32_t)r * 0x9E3779B9u;
    const uint32_t kr1 = k1 + (uint32_t)r * 0xBB67AE85u;
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ kr0, (uint32_t)p1,
                   (uint32_t)(p0 >> 32) ^ c.w ^ kr1, (uint32_t)p0);
  }
  return c;
}

// exp(x) for x in [-40, 0): x = n ln2 + r with n = rint(x / ln2) and r from a
// two-part split of ln2 (Cody and Waite); exp(r) by its degree-13 Taylor
// polynomial in Horner form with fused multiply-adds; result 2^n exp(r).
__device__ __forceinline__ double exp_det(double x) {
  const double n = rint(x * 0x1.71547652b82fep+0);
  double r = fma(-n, 0x1.62e42feep-1, x);
  r = fma(-n, 0x1.a39ef35793c76p-33, r);
  double p = 1.0 / 6227020800.0;
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)n);
}

// Single-precision counterpart for x in [-17, 0): degree-8 Taylor polynomial.
__device__ __forceinline__ float expf_det(float x) {
  const float n = rintf(x * 0x1.715476p+0f);
  float r = fmaf(-n, 0x1.62e000p-1f, x);
  r = fmaf(-n, 0x1.0bfbe8p-15f, r);
  float p = 1.0f / 40320.0f;
  p = fmaf(p, r, 1.0f / 5040.0f);
  p = fmaf(p, r, 1.0f / 720.0f);
  p = fmaf(p, r, 1.0f / 120.0f);
  p = fmaf(p, r, 1.0f / 24.0f);
  p = fmaf(p, r, 1.0f / 6.0f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  return ldexpf(p, (int)n);
}

// 53-bit uniform from two Philox words.
__device__ __forceinline__ uint64_t u53(uint32_t hi, uint32_t lo) {
  return (((uint64_t)hi << 32) | lo) >> 11;
}

// Accept with probability min[1, exp(delta)], u = u53 * 2^-53.  Below -40,
// exp(delta) < 2^-53, so only u == 0 accepts.
__device__ __forceinline__ bool accept64(uint64_t u, double delta) {
  if (delta >= 0.0) return true;
  if (delta < -40.0) return u == 0;
  return (double)u * 0x1p-53 < exp_det(delta);
}

// The same decision without branches: exp_det is evaluated for every lane
// (its argument clamped into [-40, 0]) and used only where delta lies in
// [-40, 0), so the outcome is bit-identical to accept64.
__device__ __forceinline__ bool accept64_flat(uint64_t u, double delta) {
  const double x = fmin(fmax(delta, -40.0), 0.0);
  const double e = exp_det(x);
  const bool mid = (double)u * 0x1p-53 < e;
  return (delta >= 0.0) || (delta < -40.0 ? (u == 0) : mid);
}

// Same with a 24-bit uniform (exp(-17) < 2^-24).
__device__ __forceinline__ bool accept32(uint32_t u, float delta) {
  if (delta >= 0.0f) return true;
  if (delta < -17.0f) return u == 0;
  return (float)u * 0x1p-24f < expf_det(delta);
}

__device__ __forceinline__ bool accept32_flat(uint32_t u, float delta) {
  const float x = fminf(fmaxf(delta, -17.0f), 0.0f);
  const float e = expf_det(x);
  const bool mid = (float)u * 0x1p-24f < e;
  return (delta >= 0.0f) || (delta < -17.0f ? (u == 0) : mid);
}

// ---- two-float arithmetic (Knuth's TwoSum, Dekker's FastTwoSum) ----
__device__ __forceinline__ void df_add1(float ah, float al, float b, float& rh, float& rl) {
  const float s = ah + b;
  const float bb = s - ah;
  float e = (ah - (s - bb)) + (b - bb);
  e = e + al;
  rh = s + e;
  rl = e - (rh - s);
}

__device__ __forceinline__ void df_add(float ah, float al, float bh, float bl, float& rh, float& rl) {
  const float s = ah + bh;
  const float bb = s - ah;
  float e = (ah - (s - bb)) + (bh - bb);
  e = e + (al + bl);
  rh = s + e;
  rl = e - (rh - s);
}

__device__ __forceinline__ void df_div_int(float ah, float al, int m, float& rh, float& rl) {
  const float fm = (float)m;
  const float qh = ah / fm;
  const float rem = fmaf(-qh, fm, ah);
  const float ql = (rem + al) / fm;
  rh = qh + ql;
  rl = ql - (rh - qh);
}

// ---- block reductions (wavefront shuffles, then LDS across waves) ----
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, 64));
  return v;
}

template <typename T, typename Op>
__device__ T block_reduce(T v, Op op, T* scratch) {
  v = wave_reduce(v, op);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T r = scratch[0];
  for (int i = 1; i < nw; ++i) r = op(r, scratch[i]);
  __syncthreads();
  return r;
}

}  // namespace rewl
