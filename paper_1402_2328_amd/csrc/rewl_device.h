// Device-side arithmetic of the REWL kernels: counter-based RNG, the
// deterministic exponential used by the acceptance tests, two-float (FP32
// compensated) arithmetic and wavefront reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl {

// x ^ y ^ z in one instruction (gfx950 three-input bitwise op, truth table
// 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t x, uint32_t y, uint32_t z) {
  return __builtin_amdgcn_bitop3_b32(x, y, z, 0x96);
}

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
    c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                   xor3((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
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
    c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, kr0), (uint32_t)p1,
                   xor3((uint32_t)(p0 >> 32), c.w, kr1), (uint32_t)p0);
  }
  return c;
}

// Fused multiply-add with all three operands in vector registers.  Written
// as the instruction itself because the compiler otherwise turns a Horner
// step with a loop-invariant coefficient into the accumulating form plus a
// register copy of the coefficient; the arithmetic is the same single
// rounding as fma().
__device__ __forceinline__ double fma_vvv(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// exp(x) for x in [-40, 0): x = n ln2 + r with n = rint(x / ln2) and r from a
// two-part split of ln2 (Cody and Waite); exp(r) by its degree-13 Taylor
// polynomial in Horner form with fused multiply-adds; result 2^n exp(r).
// exp_det_parts returns p = exp(r) and n, so that callers can fold a further
// power of two into the final scaling.
__device__ __forceinline__ double exp_det_parts(double x, int& n_out) {
  const double n = rint(x * 0x1.71547652b82fep+0);
  double r = fma(-n, 0x1.62e42feep-1, x);
  r = fma(-n, 0x1.a39ef35793c76p-33, r);
  double p = 1.0 / 6227020800.0;
  p = fma_vvv(p, r, 1.0 / 479001600.0);
  p = fma_vvv(p, r, 1.0 / 39916800.0);
  p = fma_vvv(p, r, 1.0 / 3628800.0);
  p = fma_vvv(p, r, 1.0 / 362880.0);
  p = fma_vvv(p, r, 1.0 / 40320.0);
  p = fma_vvv(p, r, 1.0 / 5040.0);
  p = fma_vvv(p, r, 1.0 / 720.0);
  p = fma_vvv(p, r, 1.0 / 120.0);
  p = fma_vvv(p, r, 1.0 / 24.0);
  p = fma_vvv(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  n_out = (int)n;
  return p;
}

__device__ __forceinline__ double exp_det(double x) {
  int n;
  const double p = exp_det_parts(x, n);
  return ldexp(p, n);
}

// Single-precision counterpart for x in [-17, 0): degree-8 Taylor polynomial.
__device__ __forceinline__ float expf_det_parts(float x, int& n_out) {
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
  n_out = (int)n;
  return p;
}

__device__ __forceinline__ float expf_det(float x) {
  int n;
  const float p = expf_det_parts(x, n);
  return ldexpf(p, n);
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

// The same decision without branches, from the two Philox words hi, lo of
// the uniform.  With x = delta clamped into [-40, 0]:
//   delta >= 0:   x = 0 and exp_det(0) = 1 exactly, and u * 2^-53 < 1 always;
//   delta < -40:  x = -40 and 0 < exp_det(-40) < 2^-53, so u * 2^-53 < it
//                 iff u == 0;
// so the single comparison u * 2^-53 < exp_det(x) is accept64.  Both sides
// are then scaled by 2^53 (exact): u = hi * 2^21 + (lo >> 11) is formed
// exactly in FP64 and compared with 2^(n+53) p.
__device__ __forceinline__ bool accept64_flat(uint32_t hi, uint32_t lo, double delta) {
  const double x = fmin(fmax(delta, -40.0), 0.0);
  int n;
  const double p = exp_det_parts(x, n);
  const double u = fma((double)hi, 0x1p21, (double)(lo >> 11));
  return u < ldexp(p, n + 53);
}

// Same with a 24-bit uniform (exp(-17) < 2^-24).
__device__ __forceinline__ bool accept32(uint32_t u, float delta) {
  if (delta >= 0.0f) return true;
  if (delta < -17.0f) return u == 0;
  return (float)u * 0x1p-24f < expf_det(delta);
}

// Branch-free accept32 (exp(-17) < 2^-24 and expf_det(0) = 1, as above):
// the comparison u < 2^(n+24) p on the 24-bit uniform u.
__device__ __forceinline__ bool accept32_flat(uint32_t u, float delta) {
  const float x = fminf(fmaxf(delta, -17.0f), 0.0f);
  int n;
  const float p = expf_det_parts(x, n);
  return (float)u < ldexpf(p, n + 24);
}

// Median of three signed integers: clamp(a, b, c) when b <= c, one
// v_med3_i32 either way.  The compiler turns the min/max form into the
// instruction and schedules it freely; written as inline asm it also gets
// wait states around it and fixes the order of the code near it.  Which
// of the two makes a loop faster is a matter of measurement (the sweep
// takes ASM for Ising and the min/max form for Potts).
template <bool ASM>
__device__ __forceinline__ int med3_i32(int a, int b, int c) {
  if constexpr (ASM) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
  } else {
    return max(min(a, b), min(max(a, b), c));
  }
}

// Fast exact acceptance.  A single-precision estimate e of exp(x), x the
// clamped delta, from the hardware base-2 exponential of x log2(e) has a
// relative error below 1e-5: x and log2(e) rounded to float (each < 2^-24
// relative, |x| <= 40) and the product rounded (< 58 * 2^-24 absolute) shift
// the exponent by < 1e-5 in total, and the instruction itself is accurate to
// about one float ulp.  The uniform u = u53 * 2^-53 lies in
// [hi 2^-32, (hi + 1) 2^-32).  With the slack s = 2^-10, far above that
// bound and above the float roundings of hi, hi + 1 and the two products
// (each < 2^-24 relative), u is surely below exp_det(x) when
// fl(fl(hi) + 1) <= fl(e (1 - s) 2^32), and surely not when
// fl(hi) > fl(e (1 + s) 2^32); only in between (probability about 2 s e per
// attempt) is accept64_flat evaluated.  The decision is therefore always
// accept64_flat's.  The estimate uses the unclamped delta: for delta >= 0
// only the first test can hold (e >= 1), and it is right since every such
// move is accepted; for delta < -40 the second test holds exactly when
// hi >= 1, and then u >= 2^-32 > exp_det(-40), a rejection; hi = 0 goes to
// the exact test.
__device__ __forceinline__ bool accept64_fast(uint32_t hi, uint32_t lo, double delta) {
  const float e = __builtin_amdgcn_exp2f((float)delta * 0x1.715476p+0f);
  const float h = (float)hi;
  const bool yes = h + 1.0f <= e * 0x1.ff8p+31f;  // (1 - 2^-10) 2^32
  const bool no = h > e * 0x1.004p+32f;           // (1 + 2^-10) 2^32
  bool a = yes;
  if (!yes && !no) a = accept64_flat(hi, lo, delta);
  return a;
}

// The same pre-test for the 24-bit uniform u of accept32_flat (u lies in
// [u, u + 1) 2^-24 exactly).
__device__ __forceinline__ bool accept32_fast(uint32_t u, float delta) {
  const float x = fminf(fmaxf(delta, -17.0f), 0.0f);
  const double e = (double)__builtin_amdgcn_exp2f(x * 0x1.715476p+0f);
  const double h = (double)u;
  const bool yes = h + 1.0 <= e * ((1.0 - 0x1p-10) * 0x1p24);
  const bool no = h >= e * ((1.0 + 0x1p-10) * 0x1p24);
  bool a = yes;
  if (!yes && !no) a = accept32_flat(u, delta);
  return a;
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
__device__ T block_reduce(T v, Op op, T* red) {
  v = wave_reduce(v, op);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  T r = red[0];
  for (int i = 1; i < nw; ++i) r = op(r, red[i]);
  __syncthreads();
  return r;
}

}  // namespace rewl
