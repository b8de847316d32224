// Internal definitions shared by the HIP sources of the Hessian-equation solver.
//
// Everything is compiled for gfx950 (CDNA4, 64-wide wavefronts) with
// -ffp-contract=off: fused multiply-adds are written explicitly with fma(),
// which keeps the error-free transformations of the double-double helpers exact.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/lrsdp.h"

namespace lrsdp {

constexpr int kWave = 64;

// ------------------------------------------------------------------ host-side errors

struct Status {
  int code = LRSDP_OK;
};

#define LRSDP_HIP(expr)                                                         \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      std::fprintf(stderr, "lrsdp: %s failed: %s (%s:%d)\n", #expr,             \
                   hipGetErrorString(e_), __FILE__, __LINE__);                  \
      return LRSDP_ERR_DEVICE;                                                  \
    }                                                                           \
  } while (0)

#define LRSDP_TRY(expr)               \
  do {                                \
    int s_ = (expr);                  \
    if (s_ < 0) return s_;            \
  } while (0)

inline int grid_for(int64_t work, int per_block, int cap = 1 << 20) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

// ------------------------------------------------------------------ device helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Deterministic block sum; every thread gets the result.  scratch: >= blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  return s;
}

// ------------------------------------------------------------------ double-double
// A value is hi + lo with |lo| <= ulp(hi)/2.  TwoSum (Knuth) and TwoProduct via FMA
// are error-free; the library is built with -ffp-contract=off so nothing is re-fused.

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  double e = fma(a, b, -p);
  return {p, e};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  double e = s.lo + t.hi;
  dd u = quick_two_sum(s.hi, e);
  e = u.lo + t.lo;
  return quick_two_sum(u.hi, e);
}

__device__ __forceinline__ dd dd_add_d(dd a, double b) {
  dd s = two_sum(a.hi, b);
  double e = s.lo + a.lo;
  return quick_two_sum(s.hi, e);
}

__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  double e = fma(a.lo, b, p.lo);
  return quick_two_sum(p.hi, e);
}

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  double e = fma(a.hi, b.lo, fma(a.lo, b.hi, p.lo));
  return quick_two_sum(p.hi, e);
}

// acc += a * b with a, b FP64 (b may carry a low part blo)
__device__ __forceinline__ dd dd_fma(dd acc, double a, double b) {
  dd p = two_prod(a, b);
  return dd_add(acc, p);
}

__device__ __forceinline__ dd dd_fma2(dd acc, double a, double bhi, double blo) {
  dd p = two_prod(a, bhi);
  p.lo = fma(a, blo, p.lo);
  return dd_add(acc, p);
}

// Compensated dot product (Ogita, Rump and Oishi, "Accurate sum and dot product", SIAM J. Sci.
// Comput. 26, 2005: Dot2).  s is the rounded running sum; c gathers every product's rounding
// error (TwoProduct) and every addition's (TwoSum).  The result s + c is as accurate as the dot
// product evaluated in twice the working precision, with an error below gamma_n^2 sum |x_i y_i|
// (n terms, gamma_n = n u / (1 - n u)).  Unlike a double-double accumulator, a term depends on
// the previous ones through one addition to s and one to c only, so the terms pipeline.
struct dot2 {
  double s = 0.0, c = 0.0;
};

// a += x (yhi + ylo); the product with the low part is folded into the product's error term
__device__ __forceinline__ void dot2_add(dot2& a, double x, double yhi, double ylo) {
  const dd p = two_prod(x, yhi);
  const double pe = fma(x, ylo, p.lo);
  const dd t = two_sum(a.s, p.hi);
  a.s = t.hi;
  a.c += t.lo + pe;
}

// s + c as a normalized double-double (TwoSum: |c| may exceed |s| after cancellation)
__device__ __forceinline__ dd dot2_result(const dot2& a) { return two_sum(a.s, a.c); }

__device__ __forceinline__ dd shfl_xor_dd(dd v, int o) {
  return {__shfl_xor(v.hi, o, kWave), __shfl_xor(v.lo, o, kWave)};
}

__device__ __forceinline__ dd wave_sum_dd(dd v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = dd_add(v, shfl_xor_dd(v, o));
  return v;
}

// Deterministic block sum in double-double; every thread gets the result.
// scratch: >= 2 * blockDim/64 doubles.
__device__ __forceinline__ dd block_sum_dd(dd v, double* scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum_dd(v);
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wid] = v.hi;
    scratch[2 * wid + 1] = v.lo;
  }
  __syncthreads();
  dd s = {0.0, 0.0};
  for (int i = 0; i < nw; ++i) s = dd_add(s, {scratch[2 * i], scratch[2 * i + 1]});
  return s;
}

// ------------------------------------------------------------------ bf16 helpers
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

}  // namespace lrsdp
