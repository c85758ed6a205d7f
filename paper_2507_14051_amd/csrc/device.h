// Device-side helpers for the gfx950 kernels: wave64 reductions, clamps and
// the deterministic block-partial scheme.  Included by the .hip files only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hlp {

constexpr int kBlock = 256;  // threads per block: 4 wave64s
constexpr int kWaves = kBlock / 64;

// Sum over the L lanes of an aligned lane group (L a power of two <= 64).
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Clamp that propagates NaN (comparisons with NaN are false) and resolves a
// tie at the lower bound first.
template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// 0 inside (lo, hi), 1 at or below lo, 2 at or above hi (lower tested first).
template <typename T>
__device__ __forceinline__ uint8_t clamp_code(T v, T lo, T hi) {
  return v <= lo ? uint8_t(1) : (v >= hi ? uint8_t(2) : uint8_t(0));
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Block-wide sum (and max for the quantities flagged in max_mask) of NQV
// per-thread values; thread 0 writes them to out[0..NQV).  Deterministic:
// fixed shuffle tree inside a wave, then waves in order.
template <int NQV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NQV], double* out,
                                                   unsigned max_mask = 0u) {
  __shared__ double sh[NQV][kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQV; ++q) {
    double r = ((max_mask >> q) & 1u) ? wave_max(v[q]) : wave_sum(v[q]);
    if (lane == 0) sh[q][w] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQV; ++q) {
      double r = sh[q][0];
      for (int k = 1; k < kWaves; ++k) r = ((max_mask >> q) & 1u) ? (sh[q][k] > r ? sh[q][k] : r) : r + sh[q][k];
      out[q] = r;
    }
  }
}

}  // namespace hlp
