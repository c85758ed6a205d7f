// Setup kernels: input validation, CSR copy, explicit transpose (stable LSD
// radix sort of the column keys), diagonal rescaling, scaled vectors and the
// power iteration for ||A~||_2 (paper Sec. 3, "Stepsize").
#include <cmath>

#include "device.h"
#include "hlp_internal.h"

namespace hlp {

namespace {

inline int nblocks(int64_t threads) { return (int)((threads + kBlock - 1) / kBlock); }

// ----------------------------------------------------------------- validation
// flag bits (see abi.cpp for the messages)
enum : int {
  F_RP_ENDS = 1, F_RP_DEC = 2, F_COL_RANGE = 4, F_COL_ORDER = 8, F_VAL = 16,
  F_C = 32, F_NAN = 64, F_ORDER = 128, F_INF = 256
};

__global__ void k_validate_rowptr(const int64_t* __restrict__ rp, int32_t m, int64_t nnz,
                                  int32_t* flags) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i == 0 && rp[0] != 0) atomicOr(flags, F_RP_ENDS);
  if (i == 0 && rp[m] != nnz) atomicOr(flags, F_RP_ENDS);
  if (i < m && rp[i] > rp[i + 1]) atomicOr(flags, F_RP_DEC);
}

// One wave per row; the row pointers were validated before this launch.
__global__ void k_validate_rows(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const double* __restrict__ val, int32_t m, int32_t n,
                                int32_t* flags) {
  int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (i >= m) return;
  int f = 0;
  for (int64_t p = rp[i] + lane; p < rp[i + 1]; p += 64) {
    int32_t cj = col[p];
    if (cj < 0 || cj >= n) f |= F_COL_RANGE;
    if (p > rp[i] && col[p - 1] >= cj) f |= F_COL_ORDER;
    if (!finite(val[p])) f |= F_VAL;
  }
  if (f) atomicOr(flags, f);
}

__device__ __forceinline__ int bound_flags(double lo, double hi) {
  int f = 0;
  if (lo != lo || hi != hi) f |= F_NAN;
  if (lo > hi) f |= F_ORDER;
  if (lo == INFINITY || hi == -INFINITY) f |= F_INF;
  return f;
}

__global__ void k_validate_vectors(const double* __restrict__ c, const double* __restrict__ lc,
                                   const double* __restrict__ uc, const double* __restrict__ lv,
                                   const double* __restrict__ uv, int32_t m, int32_t n,
                                   int32_t* flags) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int f = 0;
  if (i < n) {
    if (!finite(c[i])) f |= F_C;
    f |= bound_flags(lv[i], uv[i]);
  }
  if (i < m) f |= bound_flags(lc[i], uc[i]);
  if (f) atomicOr(flags, f);
}

__global__ void k_rowptr32(const int64_t* __restrict__ rp64, int32_t* __restrict__ rp, int32_t m) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i <= m) rp[i] = (int32_t)rp64[i];
}

// ----------------------------------------------------------------- scan (int32, exclusive)
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int* total) {
  __shared__ int sw[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) sw[w] = inc;
  __syncthreads();
  int base = 0, tot = 0;
  for (int k = 0; k < kWaves; ++k) {
    if (k < w) base += sw[k];
    tot += sw[k];
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

__global__ void k_scan_partial(const int32_t* __restrict__ a, int64_t N, int32_t* __restrict__ bsum) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < N) s += a[base + k];
  int tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums in place.
__global__ void k_scan_top(int32_t* __restrict__ bsum, int64_t NB) {
  int carry = 0;
  for (int64_t off = 0; off < NB; off += kScanTile) {
    int64_t base = off + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = (base + k < NB) ? bsum[base + k] : 0;
      s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, &tot) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (base + k < NB) bsum[base + k] = ex;
      ex += v[k];
    }
    carry += tot;
    __syncthreads();
  }
}

__global__ void k_scan_apply(const int32_t* __restrict__ a, int32_t* __restrict__ out, int64_t N,
                             const int32_t* __restrict__ bsum) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < N) ? a[base + k] : 0;
    s += v[k];
  }
  int tot;
  int ex = block_exclusive_scan(s, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < N) out[base + k] = ex;
    ex += v[k];
  }
}

// ----------------------------------------------------------------- transpose
__global__ void k_row_of(const int32_t* __restrict__ rp, int32_t m, int32_t* __restrict__ rowof) {
  int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (i >= m) return;
  for (int p = rp[i] + lane; p < rp[i + 1]; p += 64) rowof[p] = (int32_t)i;
}

__global__ void k_init_keys(const int32_t* __restrict__ col, int64_t nnz, int32_t* __restrict__ k,
                            int32_t* __restrict__ v) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < nnz) {
    k[p] = col[p];
    v[p] = (int32_t)p;
  }
}

constexpr int kRadixItems = 16;
constexpr int kRadixTile = kBlock * kRadixItems;

// Per-tile digit histogram, stored digit-major: hist[d * nb + tile].
__global__ void k_radix_hist(const int32_t* __restrict__ keys, int64_t N, int shift,
                             int32_t* __restrict__ hist, int64_t nb) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
  for (int r = 0; r < kRadixItems; ++r) {
    int64_t e = base + r * kBlock + threadIdx.x;
    if (e < N) atomicAdd(&h[((uint32_t)keys[e] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: elements keep their input order within a digit.
__global__ void k_radix_scatter(const int32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                int32_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t N,
                                int shift, const int32_t* __restrict__ offs, int64_t nb) {
  __shared__ int gofs[256];
  __shared__ int run[256];
  __shared__ int cnt[kWaves][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  gofs[tid] = offs[(int64_t)tid * nb + blockIdx.x];
  run[tid] = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) cnt[k][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int r = 0; r < kRadixItems; ++r) {
    int64_t e = base + r * kBlock + tid;
    bool valid = e < N;
    int32_t key = valid ? kin[e] : 0;
    int32_t val = valid ? vin[e] : 0;
    uint32_t d = ((uint32_t)key >> shift) & 255u;
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot((d >> b) & 1u);
      match &= ((d >> b) & 1u) ? bb : ~bb;
    }
    int rank = __popcll(match & lt);
    if (valid && rank == 0) cnt[w][d] = __popcll(match);
    __syncthreads();
    {
      int acc = run[tid];
#pragma unroll
      for (int k = 0; k < kWaves; ++k) {
        int c = cnt[k][tid];
        cnt[k][tid] = acc;
        acc += c;
      }
      run[tid] = acc;
    }
    __syncthreads();
    if (valid) {
      int pos = gofs[d] + cnt[w][d] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kWaves; ++k) cnt[k][tid] = 0;
    __syncthreads();
  }
}

__global__ void k_count_cols(const int32_t* __restrict__ col, int64_t nnz, int32_t* __restrict__ cnt) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < nnz) atomicAdd(&cnt[col[p]], 1);
}

__global__ void k_gather_transpose(const int32_t* __restrict__ perm, const int32_t* __restrict__ rowof,
                                   const double* __restrict__ val, int64_t nnz,
                                   int32_t* __restrict__ trow, double* __restrict__ tval) {
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < nnz) {
    int32_t p = perm[k];
    trow[k] = rowof[p];
    tval[k] = val[p];
  }
}

// ----------------------------------------------------------------- row blocks
// Row kind: 0 short (at most kRbSerial nonzeros), 1 medium (at most kRbMed), 2 long.
__device__ __forceinline__ int row_kind(int len) { return len > kRbMed ? 2 : (len > kRbSerial ? 1 : 0); }

// Row r starts a block if r is a multiple of kRbRows, if its nonzeros start in
// another kRbCap-sized chunk than those of row r-1, if its kind differs from
// that of row r-1, if it is long (long rows stand alone), or if it is medium
// and r is a multiple of kWaves (medium rows go kWaves to a block at most);
// with period > 0 also every period-th row (the first row of each column panel).
__global__ void k_rb_flags(const int32_t* __restrict__ ptr, int32_t rows, int32_t period,
                           int32_t* __restrict__ flags) {
  int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= rows) return;
  int f = 1;
  if (r > 0) {
    const int p0 = ptr[r - 1], p1 = ptr[r], p2 = ptr[r + 1];
    const int k0 = row_kind(p1 - p0), k1 = row_kind(p2 - p1);
    f = (r % kRbRows == 0) || (p1 / kRbCap != p0 / kRbCap) || (k1 != k0) || (k1 == 2) ||
        (k1 == 1 && r % kWaves == 0) || (period > 0 && r % period == 0);
  }
  flags[r] = f;
}

__global__ void k_rb_scatter(const int32_t* __restrict__ flags, const int32_t* __restrict__ pos, int32_t rows,
                             int32_t* __restrict__ rb, int32_t* __restrict__ count) {
  int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= rows) return;
  if (flags[r]) rb[pos[r]] = (int32_t)r;
  if (r == rows - 1) {
    const int total = pos[r] + flags[r];
    rb[total] = rows;
    *count = total;
  }
}

// rbx[4b..4b+3] = {first row, end row, first nonzero, end nonzero} of block b.
__global__ void k_rb_expand(const int32_t* __restrict__ rb, const int32_t* __restrict__ ptr, int32_t rows,
                            const int32_t* __restrict__ count, int64_t cap, int32_t* __restrict__ rbx) {
  int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= rows || b >= *count || b >= cap) return;  // the host rejects count > cap
  const int s = rb[b], e = rb[b + 1];
  rbx[4 * b] = s;
  rbx[4 * b + 1] = e;
  rbx[4 * b + 2] = ptr[s];
  rbx[4 * b + 3] = ptr[e];
}

// ----------------------------------------------------------------- column panels
// Row classes: short (at most T nonzeros), long (more than T, below Ld) and,
// with Ld > 0, dense (at least Ld).  fl / fd flag the long / dense rows; the
// short part keeps the short rows' lengths.  All three get a terminal 0 so
// their exclusive scans end with the totals.
__global__ void k_pn_flags(const int32_t* __restrict__ rp, int32_t m, int32_t T, int32_t Ld,
                           int32_t* __restrict__ fl, int32_t* __restrict__ fd, int32_t* __restrict__ slen) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i > m) return;
  if (i == m) {
    fl[m] = 0;
    fd[m] = 0;
    slen[m] = 0;
    return;
  }
  const int len = rp[i + 1] - rp[i];
  const int dense = Ld > 0 && len >= Ld;
  const int lg = len > T && !dense;
  fl[i] = lg;
  fd[i] = dense;
  slen[i] = (lg || dense) ? 0 : len;
}

__global__ void k_pn_counts(const int32_t* __restrict__ plid, const int32_t* __restrict__ sp,
                            const int32_t* __restrict__ dlid, int32_t m, int32_t* __restrict__ counts) {
  counts[0] = plid[m];
  counts[1] = sp[m];
  counts[2] = dlid[m];
}

// Short rows copied into AS (in order); long rows listed in lrow[0, nL),
// dense rows in lrow[nL, nL + nD).
__global__ void k_pn_short(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const double* __restrict__ val, const float* __restrict__ val32,
                           const int32_t* __restrict__ plid, const int32_t* __restrict__ dlid,
                           const int32_t* __restrict__ sp, int32_t m, int32_t nL, int32_t* __restrict__ scol,
                           double* __restrict__ sval, float* __restrict__ sval32, int32_t* __restrict__ lrow) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= m) return;
  if (plid[i + 1] != plid[i]) {
    lrow[plid[i]] = (int32_t)i;
    return;
  }
  if (dlid[i + 1] != dlid[i]) {
    lrow[nL + dlid[i]] = (int32_t)i;
    return;
  }
  const int b = rp[i], d = sp[i] - b;
  for (int q = b; q < rp[i + 1]; ++q) {
    scol[q + d] = col[q];
    sval[q + d] = val[q];
    if (val32) sval32[q + d] = val32[q];
  }
}

// bit i: row i is long or dense (its update comes from panel sums)
__global__ void k_pn_bits(const int32_t* __restrict__ plid, const int32_t* __restrict__ dlid, int32_t m,
                          uint32_t* __restrict__ bits) {
  int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (w >= ((int64_t)m + 31) / 32) return;
  uint32_t b = 0;
  for (int k = 0; k < 32; ++k) {
    const int64_t i = w * 32 + k;
    if (i < m && (plid[i + 1] != plid[i] || dlid[i + 1] != dlid[i])) b |= 1u << k;
  }
  bits[w] = b;
}

__device__ int lower_col(const int32_t* __restrict__ col, int lo, int hi, int64_t c) {
  while (lo < hi) {
    const int mid = lo + (hi - lo) / 2;
    if (col[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Segment t = p*nL + l: the nonzeros of long row lrow[l] with columns in
// panel p; its length (terminal 0 at t = P*nL) and its first position in A~.
__global__ void k_pn_seg(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                         const int32_t* __restrict__ lrow, int32_t nL, int32_t P, int32_t W,
                         int32_t* __restrict__ seglen, int32_t* __restrict__ seg0) {
  int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t R = (int64_t)P * nL;
  if (t > R) return;
  if (t == R) {
    seglen[R] = 0;
    return;
  }
  const int p = (int)(t / nL), l = (int)(t % nL);
  const int i = lrow[l];
  const int a = rp[i], b = rp[i + 1];
  const int lo = lower_col(col, a, b, (int64_t)p * W);
  const int hi = lower_col(col, lo, b, (int64_t)(p + 1) * W);
  seglen[t] = hi - lo;
  seg0[t] = lo;
}

// One block per long row: each nonzero to its panel's segment, order kept.
// I = int32_t stores the column; I = uint16_t its offset in the panel (W <= 65536).
template <typename I>
__global__ void k_pn_long(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const double* __restrict__ val, const float* __restrict__ val32,
                          const int32_t* __restrict__ lrow, int32_t nL, int32_t W, const int32_t* __restrict__ pp,
                          const int32_t* __restrict__ seg0, I* __restrict__ pcol, double* __restrict__ pval,
                          float* __restrict__ pval32) {
  const int l = blockIdx.x;
  const int i = lrow[l];
  for (int q = rp[i] + threadIdx.x; q < rp[i + 1]; q += kBlock) {
    const int j = col[q];
    const int p = j / W;
    const int64_t t = (int64_t)p * nL + l;
    const int dst = pp[t] + (q - seg0[t]);
    pcol[dst] = sizeof(I) == 4 ? (I)j : (I)(j - p * W);
    pval[dst] = val[q];
    if (val32) pval32[dst] = val32[q];
  }
}

// A~^T's row indices with long and dense rows redirected to their entries of
// the compact copy of y (m + l, m + nL + d).
__global__ void k_pn_remap(const int32_t* __restrict__ row, const int32_t* __restrict__ plid,
                           const int32_t* __restrict__ dlid, int32_t m, int32_t nL, int64_t nnz,
                           int32_t* __restrict__ rowc) {
  int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= nnz) return;
  const int i = row[q];
  const int l = plid[i], d = dlid[i];
  rowc[q] = plid[i + 1] != l ? m + l : (dlid[i + 1] != d ? m + nL + d : i);
}

// Columns of A~^T split for the primal side of the dense rows: per column j,
// the count of its entries from other rows (cntR) and, per slice r of the
// compact dense index (slices of W), of its entries from dense rows (cntT).
// Within a column the entries go by increasing row, so by increasing dense
// index: the slices come in order.  Terminal zeros for the scans.
__global__ void k_tr_count(const int32_t* __restrict__ cp, const int32_t* __restrict__ row,
                           const int32_t* __restrict__ dlid, int32_t n, int32_t PT, int32_t W,
                           int32_t* __restrict__ cntR, int32_t* __restrict__ cntT) {
  int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j > n) return;
  if (j == n) {
    cntR[n] = 0;
    cntT[(int64_t)PT * n] = 0;
    return;
  }
  for (int r = 0; r < PT; ++r) cntT[(int64_t)r * n + j] = 0;
  int cr = 0, cur = -1, cc = 0;
  for (int q = cp[j]; q < cp[j + 1]; ++q) {
    const int i = row[q];
    const int d = dlid[i];
    if (dlid[i + 1] != d) {
      const int r = d / W;
      if (r != cur) {
        if (cur >= 0) cntT[(int64_t)cur * n + j] = cc;
        cur = r;
        cc = 0;
      }
      ++cc;
    } else {
      ++cr;
    }
  }
  if (cur >= 0) cntT[(int64_t)cur * n + j] = cc;
  cntR[j] = cr;
}

// The copies: ATR keeps the other rows' entries in order (long rows pointing
// to their compact y entry m + l), ATD the dense rows' entries by slice, each
// with the offset of its compact dense index d in the slice.
__global__ void k_tr_copy(const int32_t* __restrict__ cp, const int32_t* __restrict__ row,
                          const double* __restrict__ tval, const float* __restrict__ tval32,
                          const int32_t* __restrict__ dlid, const int32_t* __restrict__ plid, int32_t n, int32_t m,
                          int32_t W, const int32_t* __restrict__ cpR, const int32_t* __restrict__ ppT,
                          int32_t* __restrict__ rowR, double* __restrict__ tvalR, float* __restrict__ tval32R,
                          uint16_t* __restrict__ rowT, double* __restrict__ tvalT, float* __restrict__ tval32T) {
  int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  int pr = cpR[j], cur = -1, pt = 0;
  for (int q = cp[j]; q < cp[j + 1]; ++q) {
    const int i = row[q];
    const int d = dlid[i];
    if (dlid[i + 1] != d) {
      const int r = d / W;
      if (r != cur) {
        cur = r;
        pt = ppT[(int64_t)r * n + j];
      }
      rowT[pt] = (uint16_t)(d - r * W);  // offset in the slice
      tvalT[pt] = tval[q];
      if (tval32) tval32T[pt] = tval32[q];
      ++pt;
    } else {
      const int l = plid[i];
      rowR[pr] = plid[i + 1] != l ? m + l : i;
      tvalR[pr] = tval[q];
      if (tval32) tval32R[pr] = tval32[q];
      ++pr;
    }
  }
}

// First block of each panel (panels start blocks: see k_rb_flags).
__global__ void k_pn_starts(const int32_t* __restrict__ rbx, int32_t nb, int32_t nL, int32_t* __restrict__ pstart) {
  int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= nb) return;
  const int s = rbx[4 * b];
  if (s % nL == 0) pstart[s / nL] = (int32_t)b;
}

// ----------------------------------------------------------------- rescaling
// Per-row statistic of |d_r[i] a_ij d_c[j]| over a CSR (MAX or SUM), then
// rho = sqrt(stat) (1 for an empty row).  Used for both A (rows) and A^T
// (columns) by swapping the roles of d_r and d_c.
template <int L, bool SUM>
__global__ __launch_bounds__(kBlock) void k_row_stat(const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ idx,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ dself,
                                                     const double* __restrict__ dother, int32_t rows,
                                                     double* __restrict__ rho) {
  int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t i = t / L;
  int lane = threadIdx.x & (L - 1);
  double s = 0.0;
  if (i < rows) {
    double di = dself[i];
    for (int p = ptr[i] + lane; p < ptr[i + 1]; p += L) {
      double v = fabs(val[p]) * di * dother[idx[p]];
      s = SUM ? s + v : (v > s ? v : s);
    }
  }
  if (SUM) {
    s = group_sum<L>(s);
  } else {
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
      double o = __shfl_xor(s, off, 64);
      s = o > s ? o : s;
    }
  }
  if (i < rows && lane == 0) rho[i] = s > 0.0 ? sqrt(s) : 1.0;
}

__global__ void k_divide(double* __restrict__ d, const double* __restrict__ rho, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) d[i] = d[i] / rho[i];
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_apply_scaling(const int32_t* __restrict__ ptr,
                                                          const int32_t* __restrict__ idx,
                                                          const double* __restrict__ val0,
                                                          const double* __restrict__ dself,
                                                          const double* __restrict__ dother,
                                                          int32_t rows, double* __restrict__ out,
                                                          float* __restrict__ out32) {
  int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t i = t / L;
  int lane = threadIdx.x & (L - 1);
  if (i >= rows) return;
  double di = dself[i];
  for (int p = ptr[i] + lane; p < ptr[i + 1]; p += L) {
    double v = di * val0[p] * dother[idx[p]];
    out[p] = v;
    if (out32) out32[p] = (float)v;
  }
}

__global__ void k_scale_vectors(const double* __restrict__ c, const double* __restrict__ lc,
                                const double* __restrict__ uc, const double* __restrict__ lv,
                                const double* __restrict__ uv, const double* __restrict__ dr,
                                const double* __restrict__ dc, int32_t m, int32_t n,
                                double* __restrict__ ct, double* __restrict__ lct,
                                double* __restrict__ uct, double* __restrict__ lvt,
                                double* __restrict__ uvt, double* __restrict__ partials) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double q[2] = {0.0, 0.0};
  if (i < n) {
    double d = dc[i];
    ct[i] = d * c[i];
    lvt[i] = lv[i] / d;
    uvt[i] = uv[i] / d;
    q[0] = c[i] * c[i];
  }
  if (i < m) {
    double d = dr[i];
    lct[i] = d * lc[i];
    uct[i] = d * uc[i];
    if (finite(lc[i])) q[1] += lc[i] * lc[i];
    if (finite(uc[i])) q[1] += uc[i] * uc[i];
  }
  block_reduce_store<2>(q, partials + (int64_t)blockIdx.x * 2);
}

// ----------------------------------------------------------------- power iteration
// out = A~ x over row blocks; with partials, per-block sums of out^2.
__global__ __launch_bounds__(kBlock) void k_spmv_plain(const int32_t* __restrict__ rb,
                                                       const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ idx,
                                                       const double* __restrict__ val,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ out,
                                                       const PowerState* __restrict__ ps,
                                                       double* __restrict__ partials) {
  if (ps->done) return;
  __shared__ double lds[kRbLds];
  const int s = rb[blockIdx.x], e = rb[blockIdx.x + 1];
  const int i = s + threadIdx.x;
  const bool own = i < e;
  int a0 = 0, a1 = 0;
  if (own) {
    a0 = ptr[i];
    a1 = ptr[i + 1];
  }
  const double v = rb_dot<double>(idx, val, x, ptr[s], ptr[e], a0, a1, own, e - s, lds);
  double q[1] = {0.0};
  if (own) {
    out[i] = v;
    q[0] = v * v;
  }
  if (partials) block_reduce_store<1>(q, partials + blockIdx.x);
}

__global__ void k_power_finish(const double* __restrict__ partials, int64_t nb, PowerState* ps,
                               int32_t max_iter, double tol) {
  if (ps->done) return;
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kBlock) s += partials[b];
  double q[1] = {s};
  __shared__ double tot[1];
  block_reduce_store<1>(q, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  double nrm = sqrt(tot[0]);
  ps->it += 1;
  ps->s = nrm;
  if (nrm == 0.0) {
    ps->estimate = 0.0;
    ps->done = 1;
    return;
  }
  double root = sqrt(nrm);
  ps->root = root;
  if ((ps->has_prev && fabs(root - ps->prev_root) <= tol * root) || ps->it >= max_iter) {
    ps->estimate = root;
    ps->done = 1;
  }
  ps->prev_root = root;
  ps->has_prev = 1;
}

__global__ void k_power_reset(PowerState* ps) { *ps = PowerState{}; }

constexpr int64_t kSumDirect = 4096;  // partial counts up to this: summed by k_power_finish alone

// out[c] = sum of partials[c*chunk, min(nb, (c+1)*chunk)) in order (one block per chunk).
__global__ void k_sum_chunks(const double* __restrict__ partials, int64_t nb, int64_t chunk, double* __restrict__ out,
                             const PowerState* __restrict__ ps) {
  if (ps->done) return;
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = min(nb, b0 + chunk);
  double s = 0.0;
  for (int64_t b = b0 + threadIdx.x; b < b1; b += kBlock) s += partials[b];
  double q[1] = {s};
  block_reduce_store<1>(q, out + blockIdx.x);
}

__global__ void k_power_normalize(const double* __restrict__ w, double* __restrict__ v, int32_t n,
                                  const PowerState* __restrict__ ps) {
  int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < n && ps->s > 0.0) v[j] = w[j] / ps->s;
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_to_f32(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

// finalize for generic partial sums (block order) into dst[0..nq)
__global__ void k_finalize_sum(const double* __restrict__ partials, int64_t nb, int nq,
                               double* __restrict__ dst) {
  for (int q = 0; q < nq; ++q) {
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += kBlock) s += partials[b * nq + q];
    double v[1] = {s};
    __shared__ double tot[1];
    block_reduce_store<1>(v, tot);
    __syncthreads();
    if (threadIdx.x == 0) dst[q] = tot[0];
    __syncthreads();
  }
}

// ---- L dispatch
template <template <int> class F, typename... Args>
hipError_t dispatch_L(int L, Args... args) {
  switch (L) {
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 4: return F<4>::run(args...);
    case 8: return F<8>::run(args...);
    case 16: return F<16>::run(args...);
    case 32: return F<32>::run(args...);
    default: return F<64>::run(args...);
  }
}

template <int L>
struct RowStatMax {
  static hipError_t run(const int32_t* ptr, const int32_t* idx, const double* val, const double* ds,
                        const double* dot, int32_t rows, double* rho, hipStream_t s) {
    hipLaunchKernelGGL((k_row_stat<L, false>), dim3(nblocks((int64_t)rows * L)), dim3(kBlock), 0, s,
                       ptr, idx, val, ds, dot, rows, rho);
    return hipGetLastError();
  }
};
template <int L>
struct RowStatSum {
  static hipError_t run(const int32_t* ptr, const int32_t* idx, const double* val, const double* ds,
                        const double* dot, int32_t rows, double* rho, hipStream_t s) {
    hipLaunchKernelGGL((k_row_stat<L, true>), dim3(nblocks((int64_t)rows * L)), dim3(kBlock), 0, s,
                       ptr, idx, val, ds, dot, rows, rho);
    return hipGetLastError();
  }
};
template <int L>
struct ApplyScaling {
  static hipError_t run(const int32_t* ptr, const int32_t* idx, const double* val0, const double* ds,
                        const double* dot, int32_t rows, double* out, float* out32, hipStream_t s) {
    hipLaunchKernelGGL((k_apply_scaling<L>), dim3(nblocks((int64_t)rows * L)), dim3(kBlock), 0, s,
                       ptr, idx, val0, ds, dot, rows, out, out32);
    return hipGetLastError();
  }
};
hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t N, int32_t* tmp, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  int64_t NB = (N + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_partial, dim3((unsigned)NB), dim3(kBlock), 0, s, in, N, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, tmp, NB);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)NB), dim3(kBlock), 0, s, in, out, N, tmp);
  return hipGetLastError();
}

}  // namespace

// ============================================================================ launchers
hipError_t launch_validate_rowptr(const int64_t* rp, int32_t m, int64_t nnz, int32_t* flags,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_validate_rowptr, dim3(nblocks((int64_t)m + 1)), dim3(kBlock), 0, s, rp, m, nnz,
                     flags);
  return hipGetLastError();
}

hipError_t launch_validate_rows(const int64_t* rp, const int32_t* col, const double* val, int32_t m,
                                int32_t n, int32_t* flags, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_rows, dim3(nblocks((int64_t)m * 64)), dim3(kBlock), 0, s, rp, col, val,
                     m, n, flags);
  return hipGetLastError();
}

hipError_t launch_validate_vectors(const double* c, const double* lc, const double* uc,
                                   const double* lv, const double* uv, int32_t m, int32_t n,
                                   int32_t* flags, hipStream_t s) {
  int64_t N = m > n ? m : n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate_vectors, dim3(nblocks(N)), dim3(kBlock), 0, s, c, lc, uc, lv, uv, m, n,
                     flags);
  return hipGetLastError();
}

hipError_t launch_copy_csr(const int64_t* rp64, const int32_t* col, const double* val, int32_t m,
                           int64_t nnz, int32_t* rp, int32_t* col_out, double* val_out,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_rowptr32, dim3(nblocks((int64_t)m + 1)), dim3(kBlock), 0, s, rp64, rp, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    e = hipMemcpyAsync(col_out, col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(val_out, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s);
  }
  return e;
}

hipError_t launch_transpose(hlp_lp* lp) {
  hipStream_t s = lp->stream;
  const int64_t nnz = lp->nnz;
  const int32_t m = lp->m, n = lp->n;
  hipError_t e;
  // column pointers: counts then exclusive scan over n+1 entries (last count 0)
  int32_t* counts = lp->kB;  // n+1 ints fit: kB has max(nnz, n+1) entries
  e = hipMemsetAsync(counts, 0, sizeof(int32_t) * ((int64_t)n + 1), s);
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_count_cols, dim3(nblocks(nnz)), dim3(kBlock), 0, s, lp->col, nnz, counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = scan_exclusive(counts, lp->cp, (int64_t)n + 1, lp->scan_tmp, s)) != hipSuccess) return e;
  if (nnz == 0) return hipSuccess;
  // stable sort of (column, position) by column
  if (m > 0) {
    hipLaunchKernelGGL(k_row_of, dim3(nblocks((int64_t)m * 64)), dim3(kBlock), 0, s, lp->rp, m, lp->rowof);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_init_keys, dim3(nblocks(nnz)), dim3(kBlock), 0, s, lp->col, nnz, lp->kA, lp->vA);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int bits = 0;
  while (bits < 31 && ((int64_t)(n - 1) >> bits) > 0) ++bits;
  int32_t *kin = lp->kA, *vin = lp->vA, *kout = lp->kB, *vout = lp->vB;
  const int64_t nb = (nnz + kRadixTile - 1) / kRadixTile;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, nnz, shift, lp->hist, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(lp->hist, lp->hist, 256 * nb, lp->scan_tmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, vin, kout, vout, nnz,
                       shift, lp->hist, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t* t = kin; kin = kout; kout = t;
    t = vin; vin = vout; vout = t;
  }
  hipLaunchKernelGGL(k_gather_transpose, dim3(nblocks(nnz)), dim3(kBlock), 0, s, vin, lp->rowof,
                     lp->val0, nnz, lp->row, lp->tval0);
  return hipGetLastError();
}

hipError_t launch_build_row_blocks(hlp_lp* lp, const int32_t* ptr, int32_t rows, int32_t* rb, int32_t* rbx,
                                   int32_t* count, int32_t period, int64_t rbx_cap) {
  if (rows == 0) return hipSuccess;
  if (rows > lp->rbtmp_rows) return hipErrorInvalidValue;
  hipStream_t s = lp->stream;
  int32_t* flags = lp->rbtmp;
  int32_t* pos = lp->rbtmp + (lp->rbtmp_rows + 1);
  hipLaunchKernelGGL(k_rb_flags, dim3(nblocks(rows)), dim3(kBlock), 0, s, ptr, rows, period, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive(flags, pos, rows, lp->scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_rb_scatter, dim3(nblocks(rows)), dim3(kBlock), 0, s, flags, pos, rows, rb, count);
  hipLaunchKernelGGL(k_rb_expand, dim3(nblocks(rows)), dim3(kBlock), 0, s, rb, ptr, rows, (const int32_t*)count,
                     rbx_cap < 0 ? (int64_t)rows : rbx_cap, rbx);
  return hipGetLastError();
}

hipError_t launch_panel_split(hlp_lp* lp, int32_t T, int32_t Ld, int32_t* counts) {
  hipStream_t s = lp->stream;
  const int32_t m = lp->m;
  hipLaunchKernelGGL(k_pn_flags, dim3(nblocks((int64_t)m + 1)), dim3(kBlock), 0, s, lp->rp, m, T, Ld, lp->pscrA,
                     lp->pscrC, lp->pscrB);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive(lp->pscrA, lp->plid, (int64_t)m + 1, lp->scan_tmp, s)) != hipSuccess) return e;
  if ((e = scan_exclusive(lp->pscrC, lp->dlid, (int64_t)m + 1, lp->scan_tmp, s)) != hipSuccess) return e;
  if ((e = scan_exclusive(lp->pscrB, lp->sp, (int64_t)m + 1, lp->scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pn_counts, dim3(1), dim3(1), 0, s, lp->plid, lp->sp, lp->dlid, m, counts);
  return hipGetLastError();
}

namespace {
// Panel-major copy of the rows lrow[0, nrows): segment t = p*nrows + l, its
// row pointers pp (via the scratch arrays), then the nonzeros.
template <typename I>
hipError_t panel_copy(hlp_lp* lp, const int32_t* rows, int32_t nrows, int32_t P, int32_t W, int32_t* pp,
                      I* pcol, double* pval, float* pval32) {
  hipStream_t s = lp->stream;
  const int64_t R = (int64_t)P * nrows;
  if (nrows < 1 || R + 1 > lp->rbtmp_rows + 1) return hipErrorInvalidValue;
  const float* v32 = lp->precision == HLP_MIXED ? lp->val32 : nullptr;
  hipLaunchKernelGGL(k_pn_seg, dim3(nblocks(R + 1)), dim3(kBlock), 0, s, lp->rp, lp->col, rows, nrows, P, W,
                     lp->pscrA, lp->pscrB);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive(lp->pscrA, pp, R + 1, lp->scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pn_long<I>, dim3(nrows), dim3(kBlock), 0, s, lp->rp, lp->col, lp->val, v32, rows, nrows, W,
                     pp, lp->pscrB, pcol, pval, v32 ? pval32 : nullptr);
  return hipGetLastError();
}
}  // namespace

// Needs lp->panels, panel_w, nL, nD (and dense_P, dense_w if nD > 0) set.
hipError_t launch_panel_layout(hlp_lp* lp, int32_t* counts) {
  hipStream_t s = lp->stream;
  const int32_t m = lp->m, nL = lp->nL, nD = lp->nD;
  if (nL < 0 || nD < 0 || nL + nD < 1 || nL + nD > lp->nL_cap || nD > lp->nD_cap) return hipErrorInvalidValue;
  const float* v32 = lp->precision == HLP_MIXED ? lp->val32 : nullptr;
  hipLaunchKernelGGL(k_pn_short, dim3(nblocks(m)), dim3(kBlock), 0, s, lp->rp, lp->col, lp->val, v32, lp->plid,
                     lp->dlid, lp->sp, m, nL, lp->scol, lp->sval, lp->sval32, lp->lrow);
  hipLaunchKernelGGL(k_pn_bits, dim3(nblocks(((int64_t)m + 31) / 32)), dim3(kBlock), 0, s, lp->plid, lp->dlid, m,
                     lp->lbits);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_build_row_blocks(lp, lp->sp, m, lp->rbS, lp->rbxS, counts + 3)) != hipSuccess) return e;
  if (nL > 0) {
    if ((e = panel_copy(lp, lp->lrow, nL, lp->panels, lp->panel_w, lp->pp, lp->pcol, lp->pval, lp->pval32)) !=
        hipSuccess)
      return e;
    const int64_t R = (int64_t)lp->panels * nL;
    if ((e = launch_build_row_blocks(lp, lp->pp, (int32_t)R, lp->rbP, lp->rbxP, counts + 4, nL)) != hipSuccess)
      return e;
  }
  if (nD > 0) {
    if ((e = panel_copy(lp, lp->lrow + nL, nD, lp->dense_P, lp->dense_w, lp->ppD, lp->pcolD, lp->pvalD,
                        lp->pval32D)) != hipSuccess)
      return e;
    const int64_t RD = (int64_t)lp->dense_P * nD;
    if ((e = launch_build_row_blocks(lp, lp->ppD, (int32_t)RD, lp->rbD, lp->rbxD, counts + 5, nD,
                                     lp->capD_blocks)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

hipError_t launch_dense_transpose(hlp_lp* lp, int32_t* counts) {
  hipStream_t s = lp->stream;
  const int32_t n = lp->n, PT = lp->dense_PT;
  const int64_t RT = (int64_t)PT * n;
  if (lp->nD < 1 || PT < 1 || PT > lp->dense_PT_cap || RT + 1 > lp->rbtmp_rows + 1) return hipErrorInvalidValue;
  const float* t32 = lp->precision == HLP_MIXED ? lp->tval32 : nullptr;
  hipLaunchKernelGGL(k_tr_count, dim3(nblocks((int64_t)n + 1)), dim3(kBlock), 0, s, lp->cp, lp->row, lp->dlid, n,
                     PT, lp->dense_wT, lp->pscrB, lp->pscrA);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive(lp->pscrB, lp->cpR, (int64_t)n + 1, lp->scan_tmp, s)) != hipSuccess) return e;
  if ((e = scan_exclusive(lp->pscrA, lp->ppT, RT + 1, lp->scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tr_copy, dim3(nblocks(n)), dim3(kBlock), 0, s, lp->cp, lp->row, lp->tval, t32, lp->dlid,
                     lp->plid, n, lp->m, lp->dense_wT, lp->cpR, lp->ppT, lp->rowR, lp->tvalR,
                     t32 ? lp->tval32R : nullptr, lp->rowT, lp->tvalT, t32 ? lp->tval32T : nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_build_row_blocks(lp, lp->cpR, n, lp->rbR, lp->rbxR, counts + 6)) != hipSuccess) return e;
  return launch_build_row_blocks(lp, lp->ppT, (int32_t)RT, lp->rbT2, lp->rbxT2, counts + 7, n, lp->capT_blocks);
}

hipError_t launch_panel_remap(hlp_lp* lp) {
  if (lp->nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pn_remap, dim3(nblocks(lp->nnz)), dim3(kBlock), 0, lp->stream, lp->row, lp->plid, lp->dlid,
                     lp->m, lp->nL, lp->nnz, lp->rowc);
  return hipGetLastError();
}

hipError_t launch_panel_starts(const int32_t* rbx, int32_t nb, int32_t rows_per_panel, int32_t* pstart,
                               hipStream_t s) {
  if (nb < 1 || rows_per_panel < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pn_starts, dim3(nblocks(nb)), dim3(kBlock), 0, s, rbx, nb, rows_per_panel, pstart);
  return hipGetLastError();
}

hipError_t launch_rescale(hlp_lp* lp, int32_t ruiz_iters, int32_t pock_chambolle) {
  hipStream_t s = lp->stream;
  const int32_t m = lp->m, n = lp->n;
  hipError_t e;
  if ((e = launch_fill(lp->dr, 1.0, m, s)) != hipSuccess) return e;
  if ((e = launch_fill(lp->dc, 1.0, n, s)) != hipSuccess) return e;
  double* rho = lp->yh;  // free during setup
  double* kap = lp->xh;
  for (int pass = 0; pass < ruiz_iters + (pock_chambolle ? 1 : 0); ++pass) {
    bool sum = pass >= ruiz_iters;
    if (m > 0) {
      e = sum ? dispatch_L<RowStatSum>(lp->Lr, lp->rp, lp->col, lp->val0, lp->dr, lp->dc, m, rho, s)
              : dispatch_L<RowStatMax>(lp->Lr, lp->rp, lp->col, lp->val0, lp->dr, lp->dc, m, rho, s);
      if (e != hipSuccess) return e;
    }
    if (n > 0) {
      e = sum ? dispatch_L<RowStatSum>(lp->Lc, lp->cp, lp->row, lp->tval0, lp->dc, lp->dr, n, kap, s)
              : dispatch_L<RowStatMax>(lp->Lc, lp->cp, lp->row, lp->tval0, lp->dc, lp->dr, n, kap, s);
      if (e != hipSuccess) return e;
    }
    if (m > 0) hipLaunchKernelGGL(k_divide, dim3(nblocks(m)), dim3(kBlock), 0, s, lp->dr, rho, (int64_t)m);
    if (n > 0) hipLaunchKernelGGL(k_divide, dim3(nblocks(n)), dim3(kBlock), 0, s, lp->dc, kap, (int64_t)n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (m > 0) {
    e = dispatch_L<ApplyScaling>(lp->Lr, lp->rp, lp->col, lp->val0, lp->dr, lp->dc, m, lp->val, lp->val32, s);
    if (e != hipSuccess) return e;
  }
  if (n > 0) {
    e = dispatch_L<ApplyScaling>(lp->Lc, lp->cp, lp->row, lp->tval0, lp->dc, lp->dr, n, lp->tval,
                                 lp->tval32, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_scale_vectors(hlp_lp* lp, const double* c, const double* lc, const double* uc,
                                const double* lv, const double* uv) {
  hipStream_t s = lp->stream;
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return launch_fill(lp->results + SLOT_TMP * NQ, 0.0, 2, s);
  int nb = nblocks(N);
  hipLaunchKernelGGL(k_scale_vectors, dim3(nb), dim3(kBlock), 0, s, c, lc, uc, lv, uv, lp->dr, lp->dc,
                     lp->m, lp->n, lp->ct, lp->lct, lp->uct, lp->lvt, lp->uvt, lp->partials);
  hipLaunchKernelGGL(k_finalize_sum, dim3(1), dim3(kBlock), 0, s, lp->partials, (int64_t)nb, 2,
                     lp->results + SLOT_TMP * NQ);
  return hipGetLastError();
}

hipError_t launch_power(hlp_lp* lp, int32_t passes, int32_t first_pass, int32_t max_iter, double tol) {
  hipStream_t s = lp->stream;
  hipError_t e;
  const int32_t m = lp->m, n = lp->n;
  if (first_pass) {
    hipLaunchKernelGGL(k_power_reset, dim3(1), dim3(1), 0, s, lp->pstate);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fill(lp->pv, 1.0 / std::sqrt((double)n), n, s)) != hipSuccess) return e;
  }
  for (int k = 0; k < passes; ++k) {
    int64_t nbc = lp->nbT;
    if (lp->panels) {
      if ((e = launch_power_pass_panels(lp, &nbc)) != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(k_spmv_plain, dim3(lp->nbA), dim3(kBlock), 0, s, lp->rbA, lp->rp, lp->col, lp->val, lp->pv,
                         lp->pu, (const PowerState*)lp->pstate, (double*)nullptr);
      hipLaunchKernelGGL(k_spmv_plain, dim3(lp->nbT), dim3(kBlock), 0, s, lp->rbT, lp->cp, lp->row, lp->tval, lp->pu,
                         lp->pw, (const PowerState*)lp->pstate, lp->partials);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const double* sums = lp->partials;
    if (nbc > kSumDirect) {  // first pass: at most 256 chunk sums, in order
      const int64_t chunk = std::max<int64_t>(kSumDirect, (nbc + 255) / 256);
      const int32_t G = (int32_t)((nbc + chunk - 1) / chunk);
      hipLaunchKernelGGL(k_sum_chunks, dim3(G), dim3(kBlock), 0, s, lp->partials, nbc, chunk, lp->fin_scratch,
                         (const PowerState*)lp->pstate);
      sums = lp->fin_scratch;
      nbc = G;
    }
    hipLaunchKernelGGL(k_power_finish, dim3(1), dim3(kBlock), 0, s, sums, nbc, lp->pstate,
                       max_iter, tol);
    hipLaunchKernelGGL(k_power_normalize, dim3(nblocks(n)), dim3(kBlock), 0, s, lp->pw, lp->pv, n,
                       (const PowerState*)lp->pstate);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<double>, dim3(nblocks(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<float>, dim3(nblocks(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3(nblocks(n)), dim3(kBlock), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace hlp
