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

// ---------------------------------------------------------------- row blocks
// The hot SpMVs walk "row blocks" built at setup.  A row is short (at most
// kRbSerial nonzeros), medium (at most kRbMed) or long.  A block holds
//  - up to kRbRows consecutive short rows whose nonzeros start in the same
//    kRbCap-sized chunk (so at most kRbCap + kRbSerial = kRbLds nonzeros):
//    products staged in LDS, each row summed by its own thread;
//  - or up to kWaves consecutive medium rows inside an aligned group of
//    kWaves rows: one wave per row, a fixed shuffle tree per wave;
//  - or one row (a long one, or a row cut off by the rules above): strided
//    partials over the whole block, a fixed shuffle tree, the waves in order.
// The kind is decided from the block's row and nonzero counts alone.
constexpr int kRbRows = kBlock;
constexpr int kRbCap = 2048;
constexpr int kRbSerial = 64;
constexpr int kRbMed = 1024;
constexpr int kRbLds = kRbCap + kRbSerial;

template <typename T>
__device__ __forceinline__ T block_sum_to0(T v) {
  __shared__ T sh[kWaves];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  T r = sh[0];
  for (int k = 1; k < kWaves; ++k) r += sh[k];
  __syncthreads();
  return r;  // every thread gets the block sum
}

// Each lane handles the nonzeros first + lane + k*STRIDE of [first, end) in
// batches of U: all index and value loads of a batch are issued, then all
// gathers, then the products, so a lane has a whole batch of gathers in
// flight instead of one.  U (2, 4 or 8) follows the lane's share of the
// range, so short ranges issue few masked loads and long ones deep batches.
constexpr int kRbUnroll = 8;

// NT: load the matrix arrays (idx, val) as streaming (non-temporal) data so a
// matrix larger than the caches does not evict the gathered vector.
template <bool NT, typename T>
__device__ __forceinline__ T ld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// STAGE: write each product to lds[q - first] instead of summing.
template <int STRIDE, int U, bool STAGE, bool NT, typename ACC, typename I, typename V, typename X>
__device__ __forceinline__ ACC strided_batches(const I* __restrict__ idx, const V* __restrict__ val,
                                               const X* __restrict__ vec, int xoff, int first, int end,
                                               int lane, ACC* lds) {
  ACC part = 0;
  for (int base = first + lane; base < end; base += STRIDE * U) {
    // Past the end, the clamped position repeats the last nonzero (a valid
    // address, so the loads need no branch) and its product is dropped.
    int ix[U];
    V vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = min(base + u * STRIDE, end - 1);
      ix[u] = (int)ld<NT>(idx + q);
      vv[u] = ld<NT>(val + q);
    }
    X g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = vec[ix[u] - xoff];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = base + u * STRIDE;
      const ACC prod = q < end ? (ACC)vv[u] * (ACC)g[u] : ACC(0);
      if constexpr (STAGE) {
        if (q < end) lds[q - first] = prod;
      } else {
        part += prod;
      }
    }
  }
  return part;
}

// The batch depth is uniform over the lanes that share [first, end) (a block
// or a wave).  Either way a lane adds its products in increasing position, so
// the result does not depend on the depth.
template <int STRIDE, bool STAGE, bool NT, typename ACC, typename I, typename V, typename X>
__device__ __forceinline__ ACC strided_products(const I* __restrict__ idx, const V* __restrict__ val,
                                                const X* __restrict__ vec, int xoff, int first, int end,
                                                int lane, ACC* lds) {
  const int per_lane = (end - first + STRIDE - 1) / STRIDE;
  if (per_lane <= 2)
    return strided_batches<STRIDE, 2, STAGE, NT, ACC>(idx, val, vec, xoff, first, end, lane, lds);
  if (per_lane <= 4)
    return strided_batches<STRIDE, 4, STAGE, NT, ACC>(idx, val, vec, xoff, first, end, lane, lds);
  return strided_batches<STRIDE, kRbUnroll, STAGE, NT, ACC>(idx, val, vec, xoff, first, end, lane, lds);
}

// lds[q0] + lds[q0 + 1] + ... + lds[q1 - 1], added in that order; the reads
// go out four at a time, the last one to three together (one read at a time
// would wait out the LDS latency for every term).
template <typename ACC>
__device__ __forceinline__ ACC lds_row_sum(const ACC* lds, int q0, int q1) {
  ACC acc = 0;
  int q = q0;
  for (; q + 4 <= q1; q += 4) {
    const ACC v0 = lds[q], v1 = lds[q + 1], v2 = lds[q + 2], v3 = lds[q + 3];
    acc += v0;
    acc += v1;
    acc += v2;
    acc += v3;
  }
  if (q < q1) {  // the last one to three, also read together
    const ACC v0 = lds[q], v1 = q + 1 < q1 ? lds[q + 1] : ACC(0), v2 = q + 2 < q1 ? lds[q + 2] : ACC(0);
    acc += v0;
    if (q + 1 < q1) acc += v1;
    if (q + 2 < q1) acc += v2;
  }
  return acc;
}

// Row sums of val .* vec[idx - xoff] (idx: int32, or uint16 offsets into a
// staged slice) over the calling block's nrows rows with
// nonzeros [ps, pe); thread t (own: t < nrows) holds the pointers [a0, a1) of
// its row and gets that row's sum (in a single-row block every thread gets
// it).  Deterministic in every kind of block.  (xoff: vec holds the slice of
// the vector that starts at index xoff, e.g. a slice staged in LDS.)
template <typename ACC, bool NT = false, typename I, typename V, typename X>
__device__ __forceinline__ ACC rb_dot(const I* __restrict__ idx, const V* __restrict__ val,
                                      const X* __restrict__ vec, int ps, int pe, int a0, int a1,
                                      bool own, int nrows, ACC* lds, int xoff = 0) {
  const int tid = threadIdx.x;
  if (nrows == 1)
    return block_sum_to0(strided_products<kBlock, false, NT, ACC>(idx, val, vec, xoff, ps, pe, tid, lds));
  if (pe - ps > nrows * kRbSerial) {  // medium rows (a block of short rows has at most kRbSerial per row)
    __shared__ int sh_ptr[kWaves + 1];
    __shared__ ACC sh_sum[kWaves];
    if (own) {
      sh_ptr[tid] = a0;
      if (tid == nrows - 1) sh_ptr[nrows] = a1;
    }
    __syncthreads();
    const int w = tid >> 6;
    if (w < nrows) {
      const ACC part =
          strided_products<64, false, NT, ACC>(idx, val, vec, xoff, sh_ptr[w], sh_ptr[w + 1], tid & 63, lds);
      const ACC sum = wave_sum(part);
      if ((tid & 63) == 0) sh_sum[w] = sum;
    }
    __syncthreads();
    return own ? sh_sum[tid] : ACC(0);
  }
  strided_products<kBlock, true, NT, ACC>(idx, val, vec, xoff, ps, pe, tid, lds);
  __syncthreads();
  const ACC acc = own ? lds_row_sum(lds, a0 - ps, a1 - ps) : ACC(0);
  __syncthreads();
  return acc;
}

}  // namespace hlp
