// Sparse X in CSR form (the paper's own data are sparse feature matrices,
// Sec. IV-A and V-A; Proposition 4 prices both products of the pass at
// O(nnz(X) l)): rows are samples; row i's entries are colidx[e], values[e]
// for e in [rowptr[i], rowptr[i + 1]). The pass of Algorithm 4, Algorithm 1's
// second pass and the projection with such an X. Every product gathers one
// k-vector (a row of Omega, of the sketch or of V) per stored entry, so the
// kernels are built to keep those rows in L2:
//
//  * k_csr_sketch_lists: Y = X Omega for the very sparse Omega, kept as row
//    lists of its nonzeros; each wave owns a row of Y in LDS.
//  * k_csr_block: Y = X B for a dense B (Gaussian Omega, or V for the
//    projection) over column blocks of B whose column slices fit an XCD's
//    L2, for rows with ordered columns; k_csr_spmm (one wave per row)
//    otherwise.
//  * the column-ordered form of a stripe of rows in row blocks, built on
//    the device by a stable LSD radix sort (own kernels: per-tile digit
//    counts, a prefix sum over (digit, tile), a ranked scatter), so every
//    column sum has a fixed order.
//  * k_csc_block: F += Y^T X, one row block per launch, one column slice of
//    the block's sketch rows per XCD, FP64 sums; columns are cut into
//    segments (one wave each) so a dense column does not serialise the
//    launch, the segments' partial sums added in segment order.
//
// G = Y^T Y uses the dense products. The inputs are checked on the device
// (rowptr[0] >= 0, nondecreasing, rowptr[m] = nnz; 0 <= colidx < n) before
// any kernel indexes with them.
#include "common.h"

#include <algorithm>
#include <utility>

namespace lspca {

// ---- exclusive prefix sums (int32 or int64 counts): per-tile sums, one
// workgroup scanning the tile sums, per-tile rescans adding the tile's
// offset. Integer sums, so the order does not matter for the result.
constexpr int kScanThreads = 256, kScanItems = 16, kScanTile = kScanThreads * kScanItems;

// Exclusive scan of v over the workgroup's 256 threads; *total gets the sum.
template <typename T>
__device__ T wg_exclusive_scan(T v, T *lds, T *total) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const T x = t >= d ? lds[t - d] : T(0);
    __syncthreads();
    lds[t] += x;
    __syncthreads();
  }
  *total = lds[kScanThreads - 1];
  const T incl = lds[t];
  __syncthreads();
  return incl - v;
}

// tile[] (kScanTile, LDS) <- in[b0 ...] (zeros past count), loaded striped
template <typename T>
__device__ void scan_load(const T *__restrict__ in, int64_t b0, int64_t count, T *tile) {
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) tile[i] = b0 + i < count ? in[b0 + i] : T(0);
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_tile_sums(const T *__restrict__ in, int64_t count,
                                                        T *__restrict__ sums) {
  __shared__ T tile[kScanTile];
  __shared__ T lds[kScanThreads];
  scan_load(in, (int64_t)blockIdx.x * kScanTile, count, tile);
  T v = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) v += tile[threadIdx.x * kScanItems + i];
  T total;
  (void)wg_exclusive_scan(v, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of one tile in LDS with a starting offset; returns the
// tile's total (every thread).
template <typename T>
__device__ T scan_tile_lds(T *tile, T *lds, T offset) {
  T v = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) v += tile[threadIdx.x * kScanItems + i];
  T total;
  T run = offset + wg_exclusive_scan(v, lds, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const T x = tile[threadIdx.x * kScanItems + i];
    tile[threadIdx.x * kScanItems + i] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

// In-place exclusive scan of the tile sums by one workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_scan_sums(T *__restrict__ sums, int64_t count) {
  __shared__ T tile[kScanTile];
  __shared__ T lds[kScanThreads];
  T carry = 0;
  for (int64_t b0 = 0; b0 < count; b0 += kScanTile) {
    scan_load(sums, b0, count, tile);
    const T total = scan_tile_lds(tile, lds, carry);
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
      if (b0 + i < count) sums[b0 + i] = tile[i];
    carry += total;
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_apply(const T *__restrict__ in, int64_t count,
                                                    const T *__restrict__ sums, T *__restrict__ out) {
  __shared__ T tile[kScanTile];
  __shared__ T lds[kScanThreads];
  const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
  scan_load(in, b0, count, tile);
  (void)scan_tile_lds(tile, lds, sums[blockIdx.x]);
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
    if (b0 + i < count) out[b0 + i] = tile[i];
}

template <typename T> size_t scan_temp_bytes(int64_t count) {
  return ((count + kScanTile - 1) / kScanTile) * sizeof(T) + 256;
}

// out[i] = sum of in[0 .. i) for i < count (in and out may not overlap).
template <typename T>
int exclusive_scan(const T *in, T *out, int64_t count, void *temp, size_t temp_bytes, hipStream_t s) {
  if (count <= 0) return LSPCA_OK;
  const int64_t tiles = (count + kScanTile - 1) / kScanTile;
  if (temp_bytes < (size_t)tiles * sizeof(T)) {
    set_error("scan: temporary buffer too small");
    return LSPCA_EINVAL;
  }
  T *sums = (T *)temp;
  hipLaunchKernelGGL(k_scan_tile_sums<T>, (unsigned)tiles, kScanThreads, 0, s, in, count, sums);
  LSPCA_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_sums<T>, 1, kScanThreads, 0, s, sums, tiles);
  LSPCA_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_apply<T>, (unsigned)tiles, kScanThreads, 0, s, in, count, (const T *)sums, out);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// ---- stable LSD radix sort of (key, value) pairs: digits of up to 10 bits,
// one pass for keys below 2^10, two below 2^20, three below 2^30. Per pass:
// digit counts of each tile of 4,096 pairs (LDS atomics; counts only), an
// exclusive scan of the counts in (digit, tile) order, then a scatter in
// which each pair's rank within its digit follows its position in the tile
// (earlier waves' quarters, earlier rounds, lower lanes), so equal keys keep
// their input order; the tile's pairs are placed in LDS grouped by digit and
// written out in that order, so each digit's pairs leave as one contiguous
// run.
constexpr int kSortMaxBits = 10, kSortBuckets = 1 << kSortMaxBits, kSortThreads = 256, kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;
static_assert(kSortBuckets % kScanThreads == 0, "digits per thread in the tile scan");

__global__ __launch_bounds__(256) void k_radix_count(const uint32_t *__restrict__ keys, int64_t cnt, int shift,
                                                     int dbits, int64_t ntiles, int32_t *__restrict__ counts) {
  __shared__ int32_t h[kSortBuckets];
  const int nb = 1 << dbits;
  for (int d = threadIdx.x; d < nb; d += kSortThreads) h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < cnt) atomicAdd(&h[(keys[i] >> shift) & (nb - 1)], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < nb; d += kSortThreads) counts[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin, int64_t cnt, int shift,
                                                       int dbits, int64_t ntiles, const int32_t *__restrict__ offs,
                                                       uint32_t *__restrict__ kout, uint32_t *__restrict__ vout) {
  // wave w ranks the tile's pairs [w * 1024, (w + 1) * 1024) in order (16
  // rounds of 64 lanes) against its own per-digit counts, so the waves need
  // no barrier until the tile's totals are combined
  __shared__ int32_t wrun[4][kSortBuckets];      // pairs of the digit ranked so far by the wave
  __shared__ int32_t start[kSortBuckets];        // the digit's first slot in the tile's order
  __shared__ int32_t obase[kSortBuckets];        // output position of slot 0 of the digit's run
  __shared__ uint32_t lk[kSortTile], lv[kSortTile];
  __shared__ int32_t scan_tmp[kScanThreads];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nb = 1 << dbits, mask = nb - 1;
  const uint64_t lower = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int d = t; d < nb; d += kSortThreads) wrun[0][d] = wrun[1][d] = wrun[2][d] = wrun[3][d] = 0;
  const int64_t base = (int64_t)blockIdx.x * kSortTile + w * (kSortTile / 4);
  uint32_t key[kSortRounds], val[kSortRounds];
  int slot[kSortRounds];
  // all of the wave's loads first, so they are in flight together
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    key[r] = i < cnt ? kin[i] : 0u;
    val[r] = i < cnt ? vin[i] : 0u;
  }
  __syncthreads();                                  // counters cleared
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool ok = base + r * 64 + lane < cnt;
    const int dig = (int)((key[r] >> shift) & mask);
    // lanes of this wave holding a pair of the same digit
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < kSortMaxBits; ++b) {
      if (b < dbits) {                              // uniform
        const bool bit = (dig >> b) & 1;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
      }
    }
    const int rank = __popcll(peers & lower);
    slot[r] = ok ? wrun[w][dig] + rank : -1;      // rank within the digit among the wave's pairs
    // the group's first lane moves the digit's count on (lanes of one wave
    // see their own LDS stores in order)
    if (ok && rank == 0) wrun[w][dig] += __popcll(peers);
  }
  __syncthreads();
  // the digits' starts in the tile: exclusive scan of the tile's counts
  // (contiguous digits per thread); each wave's run starts after the lower
  // waves' pairs of the digit
  {
    constexpr int per = kSortBuckets / kScanThreads;
    int32_t v[per], sum = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
      const int d = t * per + q;
      v[q] = d < nb ? wrun[0][d] + wrun[1][d] + wrun[2][d] + wrun[3][d] : 0;
      sum += v[q];
    }
    int32_t total;
    int32_t ex = wg_exclusive_scan<int32_t>(sum, scan_tmp, &total);
#pragma unroll
    for (int q = 0; q < per; ++q) {
      const int d = t * per + q;
      if (d < nb) {
        start[d] = ex;
        obase[d] = offs[(int64_t)d * ntiles + blockIdx.x] - ex;
      }
      ex += v[q];
    }
  }
  __syncthreads();
  {
    // slot offsets of this wave within each digit's run
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r)
      if (slot[r] >= 0) {
        const int dig = (int)((key[r] >> shift) & mask);
        int at = start[dig] + slot[r];
        for (int w2 = 0; w2 < w; ++w2) at += wrun[w2][dig];
        lk[at] = key[r];
        lv[at] = val[r];
      }
  }
  __syncthreads();
  const int64_t tb = (int64_t)blockIdx.x * kSortTile;
  const int n_tile = (int)(cnt - tb < kSortTile ? cnt - tb : kSortTile);
  for (int q = t; q < n_tile; q += kSortThreads) {
    const uint32_t k = lk[q];
    const int dig = (int)((k >> shift) & mask);
    const int64_t pos = (int64_t)obase[dig] + q;
    kout[pos] = k;
    vout[pos] = lv[q];
  }
}

static int sort_passes(int bits) { return bits <= kSortMaxBits ? 1 : (bits <= 2 * kSortMaxBits ? 2 : 3); }

size_t radix_temp_bytes(int64_t cnt) {
  const int64_t ntiles = (cnt + kSortTile - 1) / kSortTile;
  const int64_t nc = ntiles * kSortBuckets;
  return 2 * ws_bytes<int32_t>((size_t)nc) + scan_temp_bytes<int32_t>(nc);
}

// Stable sort of (keys, vals) by keys < 2^bits (bits <= 30). Returns in
// *in_place whether the result is in (keys, vals) (an even number of passes)
// rather than in (kout, vout); the other pair of buffers is overwritten.
int radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *kout, uint32_t *vout, int64_t cnt, int bits,
                     void *temp, size_t temp_bytes, bool *in_place, hipStream_t s) {
  *in_place = false;
  if (cnt <= 0) return LSPCA_OK;
  if (bits > 3 * kSortMaxBits) {
    set_error("radix sort: keys of %d bits", bits);
    return LSPCA_EINVAL;
  }
  if (cnt > 0x7fffffffLL || temp_bytes < radix_temp_bytes(cnt)) {
    set_error("radix sort: %lld pairs or temporary buffer too small", (long long)cnt);
    return LSPCA_EINVAL;
  }
  const int64_t ntiles = (cnt + kSortTile - 1) / kSortTile;
  const int passes = sort_passes(bits);
  const int dbits = (bits + passes - 1) / passes;
  const int64_t nc = ntiles << dbits;
  const size_t cbytes = ws_bytes<int32_t>((size_t)ntiles * kSortBuckets);
  int32_t *counts = (int32_t *)temp;
  int32_t *offs = (int32_t *)((char *)temp + cbytes);
  char *scan_tmp = (char *)temp + 2 * cbytes;
  const size_t scan_bytes = temp_bytes - 2 * cbytes;
  uint32_t *ki = keys, *vi = vals, *ko = kout, *vo = vout;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * dbits;
    hipLaunchKernelGGL(k_radix_count, (unsigned)ntiles, kSortThreads, 0, s, ki, cnt, shift, dbits, ntiles, counts);
    LSPCA_HIP(hipGetLastError());
    LSPCA_TRY(exclusive_scan<int32_t>(counts, offs, nc, scan_tmp, scan_bytes, s));
    hipLaunchKernelGGL(k_radix_scatter, (unsigned)ntiles, kSortThreads, 0, s, ki, vi, cnt, shift, dbits, ntiles,
                       offs, ko, vo);
    LSPCA_HIP(hipGetLastError());
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  *in_place = (passes % 2) == 0;
  return LSPCA_OK;
}


// ---- input check: flag bit 0 rowptr, bit 1 colidx
__global__ void k_csr_check(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                            int64_t m, int64_t n, int64_t nnz, int *flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t i = t; i <= m; i += stride) {
    const int64_t v = rowptr[i];
    if (i == 0 && v < 0) bad |= 1;
    if (i == m && v != nnz) bad |= 1;
    if (i < m && rowptr[i + 1] < v) bad |= 1;
  }
  // entries are read only where rowptr is valid
  const int64_t e0 = rowptr[0];
  if (!bad && e0 >= 0 && e0 <= nnz)
    for (int64_t e = e0 + t; e < nnz; e += stride) {
      const int32_t c = colidx[e];
      if (c < 0 || (int64_t)c >= n) bad |= 2;
    }
  if (bad) atomicOr(flag, bad);
}

int csr_check_launch(const int64_t *rowptr, const int32_t *colidx, int64_t m, int64_t n, int64_t nnz,
                     int *dflag, hipStream_t s) {
  LSPCA_TRY(zero_i32(dflag, 1, s));
  const int64_t work = (m + 1 > nnz ? m + 1 : nnz);
  const unsigned grid = (unsigned)std::min<int64_t>((work + 255) / 256, 4096);
  hipLaunchKernelGGL(k_csr_check, grid > 0 ? grid : 1, 256, 0, s, rowptr, colidx, m, n, nnz, dflag);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

int csr_check_result(const int *dflag, int64_t n, int64_t nnz, bool *unsorted, hipStream_t s) {
  int h = 0;
  LSPCA_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  LSPCA_HIP(hipStreamSynchronize(s));
  if (h & 1) {
    set_error("CSR rowptr must start at >= 0, be nondecreasing and end at nnz (%lld)", (long long)nnz);
    return LSPCA_EINVAL;
  }
  if (h & 2) {
    set_error("CSR colidx out of [0, n) (n = %lld)", (long long)n);
    return LSPCA_EINVAL;
  }
  if (unsorted) *unsorted = (h & 4) != 0;
  return LSPCA_OK;
}

int csr_check(const int64_t *rowptr, const int32_t *colidx, int64_t m, int64_t n, int64_t nnz,
              int *dflag, hipStream_t s) {
  LSPCA_TRY(csr_check_launch(rowptr, colidx, m, n, nnz, dflag, s));
  return csr_check_result(dflag, n, nnz, nullptr, s);
}

// sum over t in [t0, t1), in order, of v[t] * B[idx[t] * ldb + c] (coff:
// this lane's byte offset c * sizeof(T) within a row of B; idx and v are
// wave-uniform and read through the scalar cache). Groups of kGatherGroup
// gathers are issued together; the next group's indices (scalar loads) are
// fetched while the current group's gathers are outstanding.
#ifndef LSPCA_GATHER_GROUP
#define LSPCA_GATHER_GROUP 32
#endif
constexpr int kGatherGroup = LSPCA_GATHER_GROUP;

// Slices of the blocked sparse products (column sums and projection): a
// wave covers 64 columns per lane-column (W = 2 for FP32: one 8-byte gather
// of two adjacent columns per lane, 128 columns per slice; FP64: 64), and a
// slice of a block's rows is sized to one XCD's L2 (4 MiB). Measured at the
// sparse workload (k = 500): against one column per lane and 2 MiB slices,
// the column sums take 17% and the projection 11% less time.
#ifndef LSPCA_CSC_W
#define LSPCA_CSC_W 2
#endif
#ifndef LSPCA_CSC_L2_KIB
#define LSPCA_CSC_L2_KIB 4096
#endif
static int csc_slice(size_t esz) { return esz == 4 ? 64 * LSPCA_CSC_W : 64; }

template <typename T, typename ACC>
__device__ __forceinline__ ACC gather_dot(const int32_t *__restrict__ idx, const T *__restrict__ v,
                                          int64_t t0, int64_t t1, const T *__restrict__ B, int64_t ldb,
                                          uint32_t coff) {
  constexpr int G = kGatherGroup;
  ACC acc = ACC(0);
  int64_t t = t0;
  if (t + G <= t1) {
    int32_t r[G];
    T w[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      r[u] = idx[t + u];
      w[u] = v[t + u];
    }
    for (;;) {
      T y[G];
#pragma unroll
      for (int u = 0; u < G; ++u) y[u] = *(const T *)((const char *)(B + (int64_t)r[u] * ldb) + coff);
      const bool more = t + 2 * G <= t1;
      int32_t rn[G];
      T wn[G];
      if (more) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
          rn[u] = idx[t + G + u];
          wn[u] = v[t + G + u];
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) acc = fma((ACC)w[u], (ACC)y[u], acc);
      t += G;
      if (!more) break;
#pragma unroll
      for (int u = 0; u < G; ++u) {
        r[u] = rn[u];
        w[u] = wn[u];
      }
    }
  }
  for (; t < t1; ++t)
    acc = fma((ACC)v[t], (ACC) * (const T *)((const char *)(B + (int64_t)idx[t] * ldb) + coff), acc);
  return acc;
}

// gather_dot for two adjacent columns per lane (FP32 only): one 8-byte
// gather per entry, two FP64 sums (coff: byte offset of the first column).
template <typename ACC>
__device__ __forceinline__ void gather_dot2(const int32_t *__restrict__ idx, const float *__restrict__ v,
                                            int64_t t0, int64_t t1, const float *__restrict__ B, int64_t ldb,
                                            uint32_t coff, ACC &acc0, ACC &acc1) {
  constexpr int G = kGatherGroup;
  acc0 = ACC(0);
  acc1 = ACC(0);
  int64_t t = t0;
  if (t + G <= t1) {
    int32_t r[G];
    float w[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      r[u] = idx[t + u];
      w[u] = v[t + u];
    }
    for (;;) {
      float2 y[G];
#pragma unroll
      for (int u = 0; u < G; ++u) y[u] = *(const float2 *)((const char *)(B + (int64_t)r[u] * ldb) + coff);
      const bool more = t + 2 * G <= t1;
      int32_t rn[G];
      float wn[G];
      if (more) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
          rn[u] = idx[t + G + u];
          wn[u] = v[t + G + u];
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        acc0 = fma((ACC)w[u], (ACC)y[u].x, acc0);
        acc1 = fma((ACC)w[u], (ACC)y[u].y, acc1);
      }
      t += G;
      if (!more) break;
#pragma unroll
      for (int u = 0; u < G; ++u) {
        r[u] = rn[u];
        w[u] = wn[u];
      }
    }
  }
  for (; t < t1; ++t) {
    const float2 y = *(const float2 *)((const char *)(B + (int64_t)idx[t] * ldb) + coff);
    acc0 = fma((ACC)v[t], (ACC)y.x, acc0);
    acc1 = fma((ACC)v[t], (ACC)y.y, acc1);
  }
}

// ---- Y[i][c] = sum_e v_e B[col_e][c] for rows r0 + i, i < rows: one wave
// per row, lanes over 64 KQ columns per pass over the row's entries (taken
// in storage order). The entries' columns and values are wave-uniform
// (scalar loads); groups of GE entries (KQ gathers each) go in two buffers,
// the next group issued before the current group's products. Lanes past k
// gather column 0 and drop the result.
template <typename T, int KQ, int GE>
__global__ __launch_bounds__(256) void k_csr_spmm(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colidx,
                                                  const T *__restrict__ vals, int64_t r0, int64_t rows,
                                                  const T *__restrict__ B, int64_t ldb, int k,
                                                  T *__restrict__ Y, int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= rows) return;
  const int64_t e0 = rowptr[r0 + i], e1 = rowptr[r0 + i + 1];
  for (int cb = 0; cb < k; cb += 64 * KQ) {
    uint32_t off[KQ];                               // byte offsets (the base is wave-uniform)
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int c = cb + lane + 64 * q;
      off[q] = (c < k ? (uint32_t)c : 0u) * (uint32_t)sizeof(T);
    }
    T acc[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) acc[q] = T(0);
    int64_t e = e0;
    if (e + GE <= e1) {
      T va[GE], vb[GE], ya[GE][KQ], yb[GE][KQ];
#pragma unroll
      for (int u = 0; u < GE; ++u) {
        const T *Bj = B + (int64_t)colidx[e + u] * ldb;
        va[u] = vals[e + u];
#pragma unroll
        for (int q = 0; q < KQ; ++q) ya[u][q] = *(const T *)((const char *)Bj + off[q]);
      }
      for (;;) {
        const bool more = e + 2 * GE <= e1;
        if (more) {
#pragma unroll
          for (int u = 0; u < GE; ++u) {
            const T *Bj = B + (int64_t)colidx[e + GE + u] * ldb;
            vb[u] = vals[e + GE + u];
#pragma unroll
            for (int q = 0; q < KQ; ++q) yb[u][q] = *(const T *)((const char *)Bj + off[q]);
          }
        }
#pragma unroll
        for (int u = 0; u < GE; ++u)
#pragma unroll
          for (int q = 0; q < KQ; ++q) acc[q] = fma(va[u], ya[u][q], acc[q]);
        e += GE;
        if (!more) break;
        const bool more2 = e + 2 * GE <= e1;
        if (more2) {
#pragma unroll
          for (int u = 0; u < GE; ++u) {
            const T *Bj = B + (int64_t)colidx[e + GE + u] * ldb;
            va[u] = vals[e + GE + u];
#pragma unroll
            for (int q = 0; q < KQ; ++q) ya[u][q] = *(const T *)((const char *)Bj + off[q]);
          }
        }
#pragma unroll
        for (int u = 0; u < GE; ++u)
#pragma unroll
          for (int q = 0; q < KQ; ++q) acc[q] = fma(vb[u], yb[u][q], acc[q]);
        e += GE;
        if (!more2) break;
      }
    }
    for (; e < e1; ++e) {
      const T *Bj = B + (int64_t)colidx[e] * ldb;
      const T v = vals[e];
#pragma unroll
      for (int q = 0; q < KQ; ++q) acc[q] = fma(v, *(const T *)((const char *)Bj + off[q]), acc[q]);
    }
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int c = cb + lane + 64 * q;
      if (c < k) Y[i * ldy + c] = acc[q];
    }
  }
}

template <typename T>
static void spmm_kq(const int64_t *rowptr, const int32_t *colidx, const T *vals, int64_t r0, int64_t rows,
                    const T *B, int64_t ldb, int k, T *Y, int64_t ldy, unsigned grid, hipStream_t s) {
  constexpr int G8 = sizeof(T) == 8 ? 2 : 4;
  if (k <= 64)
    hipLaunchKernelGGL((k_csr_spmm<T, 1, 8>), grid, 256, 0, s, rowptr, colidx, vals, r0, rows, B, ldb, k, Y, ldy);
  else if (k <= 128)
    hipLaunchKernelGGL((k_csr_spmm<T, 2, 8>), grid, 256, 0, s, rowptr, colidx, vals, r0, rows, B, ldb, k, Y, ldy);
  else if (k <= 256)
    hipLaunchKernelGGL((k_csr_spmm<T, 4, 4>), grid, 256, 0, s, rowptr, colidx, vals, r0, rows, B, ldb, k, Y, ldy);
  else
    hipLaunchKernelGGL((k_csr_spmm<T, 8, G8>), grid, 256, 0, s, rowptr, colidx, vals, r0, rows, B, ldb, k, Y, ldy);
}

int launch_csr_spmm(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals,
                    int64_t r0, int64_t rows, const void *B, int64_t ldb, int k, void *Y, int64_t ldy,
                    hipStream_t s) {
  if (vdt != LSPCA_F32 && vdt != LSPCA_F64) {
    set_error("CSR values must be FP32 or FP64 (dtype %d)", (int)vdt);
    return LSPCA_ENOTSUP;
  }
  const size_t es = dtype_size(vdt);
  for (int64_t c0 = 0; c0 < rows; c0 += kCsrMaxRows) {      // grid size limit
    const int64_t cr = rows - c0 < kCsrMaxRows ? rows - c0 : kCsrMaxRows;
    const unsigned grid = (unsigned)((cr + 3) / 4);
    void *Yc = (char *)Y + (size_t)c0 * ldy * es;
    if (vdt == LSPCA_F32)
      spmm_kq<float>(rowptr, colidx, (const float *)vals, r0 + c0, cr, (const float *)B, ldb, k, (float *)Yc,
                     ldy, grid, s);
    else
      spmm_kq<double>(rowptr, colidx, (const double *)vals, r0 + c0, cr, (const double *)B, ldb, k,
                      (double *)Yc, ldy, grid, s);
    LSPCA_HIP(hipGetLastError());
  }
  return LSPCA_OK;
}

// ---- the very sparse Omega (entries -1, 0, +1) as row lists: row j's
// nonzeros are oc[t] for t in [optr[j], optr[j + 1]), in column order, each
// the column with the entry's sign in bit 31. Built from the materialised
// Omega (n x k, row-major, row pitch ldo); one wave per row.
template <typename T>
__global__ __launch_bounds__(256) void k_om_count(const T *__restrict__ Om, int64_t ldo, int64_t n, int k,
                                                  int32_t *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j <= n; j += (int64_t)gridDim.x * 4) {
    int c_nz = 0;
    if (j < n)
      for (int cb = 0; cb < k; cb += 64) {
        const int c = cb + lane;
        c_nz += __popcll(__ballot(c < k && Om[j * ldo + c] != T(0)));
      }
    if (lane == 0) cnt[j] = c_nz;                 // cnt[n] = 0 closes the scan
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_om_fill(const T *__restrict__ Om, int64_t ldo, int64_t n, int k,
                                                 const int32_t *__restrict__ optr, int32_t *__restrict__ oc) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < n; j += (int64_t)gridDim.x * 4) {
    int32_t base = optr[j];
    for (int cb = 0; cb < k; cb += 64) {
      const int c = cb + lane;
      const T v = c < k ? Om[j * ldo + c] : T(0);
      const uint64_t mask = __ballot(v != T(0));
      if (v != T(0)) oc[base + __popcll(mask & below)] = v < T(0) ? (int32_t)((uint32_t)c | 0x80000000u) : c;
      base += __popcll(mask);
    }
  }
}

size_t om_scan_bytes(int64_t n) { return scan_temp_bytes<int32_t>(n + 1); }

int build_omega_lists(lspca_dtype vdt, const void *Om, int64_t ldo, int64_t n, int k, int32_t *cnt,
                      int32_t *optr, int32_t *oc, void *temp, size_t temp_bytes, hipStream_t s) {
  const unsigned g = (unsigned)std::min<int64_t>((n + 1 + 3) / 4, 1 << 16);   // grid-stride over rows
  if (vdt == LSPCA_F32)
    hipLaunchKernelGGL(k_om_count<float>, g, 256, 0, s, (const float *)Om, ldo, n, k, cnt);
  else
    hipLaunchKernelGGL(k_om_count<double>, g, 256, 0, s, (const double *)Om, ldo, n, k, cnt);
  LSPCA_HIP(hipGetLastError());
  LSPCA_TRY(exclusive_scan<int32_t>(cnt, optr, n + 1, temp, temp_bytes, s));
  if (vdt == LSPCA_F32)
    hipLaunchKernelGGL(k_om_fill<float>, g, 256, 0, s, (const float *)Om, ldo, n, k, optr, oc);
  else
    hipLaunchKernelGGL(k_om_fill<double>, g, 256, 0, s, (const double *)Om, ldo, n, k, optr, oc);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// ---- Y = X Omega with Omega as row lists (very sparse kind): one wave per
// row, the row of Y accumulated in LDS. Lanes take 64 entries of the row at
// a time and add +-v for each listed column of their entry with LDS
// atomics, four list codes loaded at once; one wave owns the row, so the
// order of the adds is fixed by the instruction stream and the result is
// reproducible.
template <typename T>
__global__ void k_csr_sketch_lists(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                                   const T *__restrict__ vals, int64_t r0, int64_t rows,
                                   const int32_t *__restrict__ optr, const int32_t *__restrict__ oc, int k,
                                   T *__restrict__ Y, int64_t ldy) {
  extern __shared__ unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T *yl = (T *)smem + (size_t)wv * k;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
  if (i >= rows) return;
  for (int c = lane; c < k; c += 64) yl[c] = T(0);
  const int64_t e0 = rowptr[r0 + i], e1 = rowptr[r0 + i + 1];
  for (int64_t eb = e0; eb < e1; eb += 64) {
    const int64_t e = eb + lane;
    if (e < e1) {
      const int64_t j = colidx[e];
      const T v = vals[e];
      const int32_t a = optr[j], b = optr[j + 1];
      for (int32_t t = a; t < b; t += 4) {
        int32_t cd[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) cd[u] = oc[t + u < b ? t + u : b - 1];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (t + u < b) atomicAdd(&yl[cd[u] & 0x7fffffff], cd[u] < 0 ? -v : v);
      }
    }
  }
  for (int c = lane; c < k; c += 64) Y[i * ldy + c] = yl[c];
}

int launch_csr_sketch_lists(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals,
                            int64_t r0, int64_t rows, const int32_t *optr, const int32_t *oc, int k, void *Y,
                            int64_t ldy, hipStream_t s) {
  const size_t es = dtype_size(vdt);
  int waves = (int)std::min<int64_t>(4, 65536 / ((int64_t)k * es));
  waves = waves < 1 ? 1 : waves;
  const size_t lds = (size_t)waves * k * es;
  for (int64_t c0 = 0; c0 < rows; c0 += kCsrMaxRows) {
    const int64_t cr = rows - c0 < kCsrMaxRows ? rows - c0 : kCsrMaxRows;
    const unsigned grid = (unsigned)((cr + waves - 1) / waves);
    void *Yc = (char *)Y + (size_t)c0 * ldy * es;
    if (vdt == LSPCA_F32)
      hipLaunchKernelGGL(k_csr_sketch_lists<float>, grid, 64 * waves, lds, s, rowptr, colidx,
                         (const float *)vals, r0 + c0, cr, optr, oc, k, (float *)Yc, ldy);
    else
      hipLaunchKernelGGL(k_csr_sketch_lists<double>, grid, 64 * waves, lds, s, rowptr, colidx,
                         (const double *)vals, r0 + c0, cr, optr, oc, k, (double *)Yc, ldy);
    LSPCA_HIP(hipGetLastError());
  }
  return LSPCA_OK;
}

// ---- column-ordered form of a stripe of rows [r0, r0 + rows), entries
// [e0, e0 + cnt), in row blocks: list l = b * n + j holds the entries of
// column j in rows [b * rb, (b + 1) * rb) of the stripe, in row order. One
// wave per row, lanes over its entries.
__global__ __launch_bounds__(256) void k_csr_expand(const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ colidx, int64_t r0,
                                                    int64_t rows, int64_t e0, int64_t n, int64_t rb,
                                                    int32_t *__restrict__ keys, uint32_t *__restrict__ idx,
                                                    int32_t *__restrict__ rowof) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= rows) return;
  const int64_t a = rowptr[r0 + i], b = rowptr[r0 + i + 1];
  const int64_t kb = (i / rb) * n;
  for (int64_t e = a + (threadIdx.x & 63); e < b; e += 64) {
    keys[e - e0] = (int32_t)(kb + colidx[e]);
    idx[e - e0] = (uint32_t)(e - e0);
    rowof[e - e0] = (int32_t)i;
  }
}

__global__ void k_row_bounds(const int64_t *__restrict__ rowptr, int64_t rows, int64_t g, int64_t nb,
                             int64_t *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb) return;
  const int64_t r = t * g < rows ? t * g : rows;
  out[t] = rowptr[r];
}

int launch_row_bounds(const int64_t *rowptr, int64_t rows, int64_t g, int64_t nb, int64_t *out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_row_bounds, (unsigned)((nb + 255) / 256), 256, 0, s, rowptr, rows, g, nb, out);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// out[j * ldo + c] = V[j * k + c] in the value type (n x k FP64 in)
template <typename T>
__global__ void k_v_padded(const double *__restrict__ V, int64_t n, int k, T *__restrict__ out, int64_t ldo) {
  const int64_t count = n * k;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride)
    out[(t / k) * ldo + t % k] = (T)V[t];
}

int launch_v_padded(const double *V, int64_t n, int k, lspca_dtype vdt, void *out, int64_t ldo, hipStream_t s) {
  const unsigned grid = (unsigned)std::min<int64_t>((n * k + 255) / 256, 65536);
  if (vdt == LSPCA_F32)
    hipLaunchKernelGGL(k_v_padded<float>, grid, 256, 0, s, V, n, k, (float *)out, ldo);
  else
    hipLaunchKernelGGL(k_v_padded<double>, grid, 256, 0, s, V, n, k, (double *)out, ldo);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

template <typename T>
__global__ void k_csc_gather(const uint32_t *__restrict__ idx, const int32_t *__restrict__ rowof,
                             const T *__restrict__ vals, int64_t e0, int64_t cnt, int32_t *__restrict__ crow,
                             T *__restrict__ cval) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const uint32_t e = idx[t];
  crow[t] = rowof[e];
  cval[t] = vals[e0 + e];
}

// colptr[l] = first position of a key >= l in the sorted keys (l <= L)
__global__ void k_colptr(const int32_t *__restrict__ skeys, int64_t cnt, int64_t L, int64_t *__restrict__ colptr) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l > L) return;
  int64_t lo = 0, hi = cnt;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)skeys[mid] < l) lo = mid + 1;
    else hi = mid;
  }
  colptr[l] = lo;
}

static int key_bits(int64_t n) {
  int b = 1;
  while ((int64_t)1 << b < n) ++b;
  return b;
}

// Work split of the column sums: list l is cut into segments of at most S
// entries, [segoff[l], segoff[l + 1]) (segcol maps a segment to its list).
// Lists of two or more segments leave one partial row per segment in P,
// from slot moff[l] on.
__global__ void k_seg_count(const int64_t *__restrict__ colptr, int64_t L, int64_t S,
                            int64_t *__restrict__ segcnt) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l < L) segcnt[l] = (colptr[l + 1] - colptr[l] + S - 1) / S;
  else if (l == L) segcnt[L] = 0;
}

__global__ void k_multi_count(const int64_t *__restrict__ segoff, int64_t L, int64_t *__restrict__ mcnt) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l < L) {
    const int64_t ns = segoff[l + 1] - segoff[l];
    mcnt[l] = ns > 1 ? ns : 0;
  } else if (l == L) {
    mcnt[L] = 0;
  }
}

__global__ void k_seg_fill(const int64_t *__restrict__ segoff, int64_t L, int32_t *__restrict__ segcol) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  for (int64_t w = segoff[l]; w < segoff[l + 1]; ++w) segcol[w] = (int32_t)l;
}

CscShape csc_shape(int64_t rows, int64_t n, int64_t cnt, int k, size_t esz) {
  CscShape c;
  // rows per block: one column slice of the block's sketch rows fills an
  // XCD's L2 share; the lists (blocks x n) stay below 2^26
  const int64_t rb_l2 = (int64_t)(LSPCA_CSC_L2_KIB << 10) / (csc_slice(esz) * (int64_t)esz);
  int64_t nb = (rows + rb_l2 - 1) / rb_l2;
  const int64_t nb_max = std::max<int64_t>(1, ((int64_t)1 << 26) / n);
  nb = std::max<int64_t>(1, std::min(nb, nb_max));
  c.rb = (rows + nb - 1) / nb;
  c.rb = c.rb < 1 ? 1 : c.rb;
  c.nblocks = (rows + c.rb - 1) / c.rb;
  c.lists = c.nblocks * n;
  // segment length: partial rows of multi-segment lists (<= 2 cnt / S of
  // them) within 2 GiB
  int64_t S = (cnt * (int64_t)k * 16 + ((int64_t)1 << 31) - 1) >> 31;
  c.seg = S < 1024 ? 1024 : S;
  c.segs_max = c.lists + (cnt + c.seg - 1) / c.seg;
  c.partial_rows = 2 * ((cnt + c.seg - 1) / c.seg) + 1;
  return c;
}

size_t csc_temp_bytes(int64_t cnt, int64_t lists) {
  return std::max(radix_temp_bytes(cnt), scan_temp_bytes<int64_t>(lists + 1));
}

int build_csc(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals, int64_t r0,
              int64_t rows, int64_t e0, int64_t cnt, int64_t n, const CscShape &sh, CscBuffers &b,
              hipStream_t s) {
  const int64_t L = sh.lists;
  if (cnt > 0) {
    hipLaunchKernelGGL(k_csr_expand, (unsigned)((rows + 3) / 4), 256, 0, s, rowptr, colidx, r0, rows, e0, n,
                       sh.rb, b.keys, b.idx, b.rowof);
    LSPCA_HIP(hipGetLastError());
    bool in_place = false;
    LSPCA_TRY(radix_sort_pairs((uint32_t *)b.keys, b.idx, (uint32_t *)b.skeys, b.sidx, cnt, key_bits(L), b.temp,
                               b.temp_bytes, &in_place, s));
    if (in_place) {                               // sorted pairs in (keys, idx): swap the roles
      std::swap(b.keys, b.skeys);
      std::swap(b.idx, b.sidx);
    }
    b.crow = b.keys;                              // the unsorted keys are dead after the sort
    const unsigned g = (unsigned)((cnt + 255) / 256);
    if (vdt == LSPCA_F32)
      hipLaunchKernelGGL(k_csc_gather<float>, g, 256, 0, s, b.sidx, b.rowof, (const float *)vals, e0, cnt,
                         b.crow, (float *)b.cval);
    else
      hipLaunchKernelGGL(k_csc_gather<double>, g, 256, 0, s, b.sidx, b.rowof, (const double *)vals, e0, cnt,
                         b.crow, (double *)b.cval);
    LSPCA_HIP(hipGetLastError());
  }
  const unsigned gl = (unsigned)((L + 1 + 255) / 256);
  hipLaunchKernelGGL(k_colptr, gl, 256, 0, s, b.skeys, cnt, L, b.colptr);
  LSPCA_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_seg_count, gl, 256, 0, s, b.colptr, L, sh.seg, b.cnt);
  LSPCA_HIP(hipGetLastError());
  LSPCA_TRY(exclusive_scan<int64_t>(b.cnt, b.segoff, L + 1, b.temp, b.temp_bytes, s));
  hipLaunchKernelGGL(k_multi_count, gl, 256, 0, s, b.segoff, L, b.cnt);
  LSPCA_HIP(hipGetLastError());
  LSPCA_TRY(exclusive_scan<int64_t>(b.cnt, b.moff, L + 1, b.temp, b.temp_bytes, s));
  hipLaunchKernelGGL(k_seg_fill, (unsigned)((L + 255) / 256), 256, 0, s, b.segoff, L, b.segcol);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// ---- column sums of one row block b: Ft[j][c] += sum over list b n + j of
// cval[t] * Y[crow[t]][c] (FP64). Workgroup g takes the column slice
// g mod nslices (consecutive workgroups land on the 8 XCDs in turn, so each
// XCD's L2 holds one slice of the block's sketch rows); its waves take the
// block's segments in turn (their range is read on the device), lanes over
// the slice's columns, W adjacent columns each. Lists of one segment add into
// Ft directly; the others write partial rows, added by k_block_reduce in
// segment order.
template <typename T, int W>
__global__ __launch_bounds__(256) void k_csc_block(const int64_t *__restrict__ colptr,
                                                   const int64_t *__restrict__ segoff,
                                                   const int32_t *__restrict__ segcol,
                                                   const int64_t *__restrict__ moff,
                                                   const int32_t *__restrict__ crow,
                                                   const T *__restrict__ cval, int64_t lbase, int64_t n,
                                                   int64_t S, int nslices, const T *__restrict__ Y, int k,
                                                   int64_t ldy, double *__restrict__ Ft,
                                                   double *__restrict__ P) {
  const int lane = threadIdx.x & 63;
  // the wave index in a scalar register: every list quantity below is
  // wave-uniform and read through the scalar cache
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slice = (int)(blockIdx.x % (unsigned)nslices);
  const int c = slice * 64 * W + W * lane;
  const bool on = c < k;
  // byte offset from a row start (rows are padded to 128 bytes, so the
  // second column of a pair past k stays inside the row)
  const uint32_t coff = (on ? (uint32_t)c : 0u) * (uint32_t)sizeof(T);
  const int64_t wbeg = segoff[lbase], wend = segoff[lbase + n];
  const int64_t groups = gridDim.x / (unsigned)nslices;
  for (int64_t w = wbeg + (int64_t)(blockIdx.x / (unsigned)nslices) * 4 + wv; w < wend; w += groups * 4) {
    const int64_t l = segcol[w];
    const int64_t first = segoff[l], nseg = segoff[l + 1] - first;
    const int64_t t0 = colptr[l] + (w - first) * S;
    const int64_t t1 = t0 + S < colptr[l + 1] ? t0 + S : colptr[l + 1];
    double acc[W];
    if constexpr (W == 2)
      gather_dot2<double>(crow, cval, t0, t1, Y, ldy, coff, acc[0], acc[1]);
    else
      acc[0] = gather_dot<T, double>(crow, cval, t0, t1, Y, ldy, coff);
    const int64_t j = l - lbase;
#pragma unroll
    for (int q = 0; q < W; ++q)
      if (c + q < k) {
        if (nseg == 1) Ft[j * k + c + q] += acc[q];
        else P[(moff[l] + (w - first)) * k + c + q] = acc[q];
      }
  }
}

__global__ __launch_bounds__(256) void k_block_reduce(const int64_t *__restrict__ segoff,
                                                      const int64_t *__restrict__ moff, int64_t lbase,
                                                      int64_t n, const double *__restrict__ P, int k,
                                                      double *__restrict__ Ft) {
  const int lane = threadIdx.x & 63;
  for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < n; j += (int64_t)gridDim.x * 4) {
    const int64_t l = lbase + j;
    const int64_t nseg = segoff[l + 1] - segoff[l];
    if (nseg < 2) continue;
    const double *Pl = P + moff[l] * k;
    for (int c = lane; c < k; c += 64) {
      double sum = Pl[c];
      for (int64_t q = 1; q < nseg; ++q) sum += Pl[q * k + c];
      Ft[j * k + c] += sum;
    }
  }
}

int launch_csc_factor(lspca_dtype vdt, const CscBuffers &b, const CscShape &sh, int64_t n, int64_t cnt,
                      const void *Y, int k, int64_t ldy, double *Ft, hipStream_t s) {
  const int sw = csc_slice(dtype_size(vdt));
  const int nslices = (k + sw - 1) / sw;
  const int64_t per_block = n + (cnt + sh.seg - 1) / sh.seg;            // segments of one block, at most
  const int64_t groups = std::max<int64_t>(1, std::min<int64_t>((per_block + 3) / 4, 65536 / nslices));
  const unsigned grid = (unsigned)(groups * nslices);
  const unsigned gr = (unsigned)std::min<int64_t>((n + 3) / 4, 1 << 16);
  for (int64_t bk = 0; bk < sh.nblocks; ++bk) {
    const int64_t lbase = bk * n;
    if (vdt == LSPCA_F32)
      hipLaunchKernelGGL((k_csc_block<float, LSPCA_CSC_W>), grid, 256, 0, s, b.colptr, b.segoff, b.segcol, b.moff, b.crow,
                         (const float *)b.cval, lbase, n, sh.seg, nslices, (const float *)Y, k, ldy, Ft, b.P);
    else
      hipLaunchKernelGGL((k_csc_block<double, 1>), grid, 256, 0, s, b.colptr, b.segoff, b.segcol, b.moff, b.crow,
                         (const double *)b.cval, lbase, n, sh.seg, nslices, (const double *)Y, k, ldy, Ft, b.P);
    LSPCA_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_block_reduce, gr, 256, 0, s, b.segoff, b.moff, lbase, n, b.P, k, Ft);
    LSPCA_HIP(hipGetLastError());
  }
  return LSPCA_OK;
}

// ---- Z = X V by column blocks (rows with nondecreasing columns): block b
// holds the features [b nbc, (b + 1) nbc); pos[i][b] is the offset in row i
// of its first entry in block b. One wave per row: lanes take the block
// boundaries (lower bounds in the row's columns); the wave also flags a row
// whose columns decrease (bit 2 of flag). Reads stay in [0, nnz) whatever
// rowptr holds, so this may run before the check's result is known.
__global__ __launch_bounds__(256) void k_row_block_pos(const int64_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ colidx, int64_t rows,
                                                       int64_t nnz, int64_t nbc, int nblk,
                                                       int32_t *__restrict__ pos, int *flag) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= rows) return;
  int64_t a = rowptr[i], b = rowptr[i + 1];
  a = a < 0 ? 0 : (a > nnz ? nnz : a);
  b = b < a ? a : (b > nnz ? nnz : b);
  bool bad = false;
  for (int64_t e = a + lane; e + 1 < b; e += 64) bad |= colidx[e] > colidx[e + 1];
  if (__ballot(bad) != 0ull && lane == 0) atomicOr(flag, 4);
  for (int bk = lane; bk <= nblk; bk += 64) {
    const int64_t key = (int64_t)bk * nbc;
    int64_t lo = a, hi = b;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)colidx[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    pos[i * (nblk + 1) + bk] = (int32_t)(lo - a);
  }
}

// Block b of Z = X V: workgroup g takes the column slice g mod nslices (the
// XCD's L2 holds that slice of the block's rows of V), its waves take rows
// in turn, lanes over the slice's columns (W adjacent columns each); Z (+)=
// the block's sum.
template <typename T, int W>
__global__ __launch_bounds__(256) void k_csr_block(const int64_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colidx,
                                                   const T *__restrict__ vals, const int32_t *__restrict__ pos,
                                                   int nblk, int bk, int64_t rows, const T *__restrict__ V,
                                                   int64_t ldv, int k, int nslices, T *__restrict__ Z,
                                                   int64_t ldz) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slice = (int)(blockIdx.x % (unsigned)nslices);
  const int c = slice * 64 * W + W * lane;
  const bool on = c < k;
  const uint32_t coff = (on ? (uint32_t)c : 0u) * (uint32_t)sizeof(T);
  const int64_t groups = gridDim.x / (unsigned)nslices;
  for (int64_t i = (int64_t)(blockIdx.x / (unsigned)nslices) * 4 + wv; i < rows; i += groups * 4) {
    const int64_t base = rowptr[i];
    const int64_t t0 = base + pos[i * (nblk + 1) + bk], t1 = base + pos[i * (nblk + 1) + bk + 1];
    T acc[W];
    if constexpr (W == 2)
      gather_dot2<T>(colidx, vals, t0, t1, V, ldv, coff, acc[0], acc[1]);
    else
      acc[0] = gather_dot<T, T>(colidx, vals, t0, t1, V, ldv, coff);
#pragma unroll
    for (int q = 0; q < W; ++q)
      if (c + q < k) {
        if (bk == 0) Z[i * ldz + c + q] = acc[q];
        else Z[i * ldz + c + q] += acc[q];
      }
  }
}

// Bit 2 of flag when some row's columns decrease (one wave per row; reads
// stay in [0, nnz) whatever rowptr holds).
__global__ __launch_bounds__(256) void k_rows_sorted(const int64_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ colidx, int64_t rows,
                                                     int64_t nnz, int *flag) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= rows) return;
  int64_t a = rowptr[i], b = rowptr[i + 1];
  a = a < 0 ? 0 : (a > nnz ? nnz : a);
  b = b < a ? a : (b > nnz ? nnz : b);
  bool bad = false;
  for (int64_t e = a + lane; e + 1 < b; e += 64) bad |= colidx[e] > colidx[e + 1];
  if (__ballot(bad) != 0ull && lane == 0) atomicOr(flag, 4);
}

int launch_rows_sorted(const int64_t *rowptr, const int32_t *colidx, int64_t rows, int64_t nnz, int *dflag,
                       hipStream_t s) {
  for (int64_t r0 = 0; r0 < rows; r0 += kCsrMaxRows) {
    const int64_t cr = rows - r0 < kCsrMaxRows ? rows - r0 : kCsrMaxRows;
    hipLaunchKernelGGL(k_rows_sorted, (unsigned)((cr + 3) / 4), 256, 0, s, rowptr + r0, colidx, cr, nnz, dflag);
    LSPCA_HIP(hipGetLastError());
  }
  return LSPCA_OK;
}

int csr_blocks(int64_t n, size_t esz, int64_t *nbc) {
  // a slice of a block's rows of V fills one XCD's L2 share
  *nbc = (int64_t)(LSPCA_CSC_L2_KIB << 10) / (csc_slice(esz) * (int64_t)esz);
  return (int)((n + *nbc - 1) / *nbc);
}

int launch_row_block_pos(const int64_t *rowptr, const int32_t *colidx, int64_t rows, int64_t nnz, int64_t nbc,
                         int nblk, int32_t *pos, int *dflag, hipStream_t s) {
  hipLaunchKernelGGL(k_row_block_pos, (unsigned)((rows + 3) / 4), 256, 0, s, rowptr, colidx, rows, nnz, nbc,
                     nblk, pos, dflag);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

int launch_csr_blocked(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals,
                       const int32_t *pos, int nblk, int64_t rows, const void *V, int64_t ldv, int k, void *Z,
                       int64_t ldz, hipStream_t s) {
  const int sw = csc_slice(dtype_size(vdt));
  const int nslices = (k + sw - 1) / sw;
  const int64_t groups = std::max<int64_t>(1, std::min<int64_t>((rows + 3) / 4, 65536 / nslices));
  const unsigned grid = (unsigned)(groups * nslices);
  for (int bk = 0; bk < nblk; ++bk) {
    if (vdt == LSPCA_F32)
      hipLaunchKernelGGL((k_csr_block<float, LSPCA_CSC_W>), grid, 256, 0, s, rowptr, colidx, (const float *)vals, pos, nblk, bk,
                         rows, (const float *)V, ldv, k, nslices, (float *)Z, ldz);
    else
      hipLaunchKernelGGL((k_csr_block<double, 1>), grid, 256, 0, s, rowptr, colidx, (const double *)vals, pos, nblk,
                         bk, rows, (const double *)V, ldv, k, nslices, (double *)Z, ldz);
    LSPCA_HIP(hipGetLastError());
  }
  return LSPCA_OK;
}

// ---- Ut[c * ldt + i] = Y[i * ldy + c] (rows x k in, k x rows out; the
// SPCA sketch transposed for the tall-skinny QR), through 64 x 64 LDS tiles
template <typename T>
__global__ __launch_bounds__(256) void k_rows_to_cols(const T *__restrict__ Y, int64_t rows, int k,
                                                      int64_t ldy, T *__restrict__ Ut, int64_t ldt) {
  __shared__ T tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r;
    const int c = c0 + tx;
    tile[r][tx] = (i < rows && c < k) ? Y[i * ldy + c] : T(0);
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int c = c0 + r;
    const int64_t i = i0 + tx;
    if (c < k && i < rows) Ut[(int64_t)c * ldt + i] = tile[tx][r];
  }
}

int launch_rows_to_cols(lspca_dtype vdt, const void *Y, int64_t rows, int k, int64_t ldy, void *Ut, int64_t ldt,
                        hipStream_t s) {
  if (rows <= 0) return LSPCA_OK;
  const dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((k + 63) / 64));
  if (vdt == LSPCA_F32)
    hipLaunchKernelGGL(k_rows_to_cols<float>, grid, 256, 0, s, (const float *)Y, rows, k, ldy, (float *)Ut, ldt);
  else
    hipLaunchKernelGGL(k_rows_to_cols<double>, grid, 256, 0, s, (const double *)Y, rows, k, ldy, (double *)Ut,
                       ldt);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// ---- F[c][j] += Ft[j][c] (k x n FP64 from n x k), through 64 x 64 LDS tiles
__global__ __launch_bounds__(256) void k_add_transposed(const double *__restrict__ Ft, int64_t n, int k,
                                                        double *__restrict__ F) {
  __shared__ double tile[64][65];
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int64_t j = j0 + r;
    const int c = c0 + tx;
    tile[r][tx] = (j < n && c < k) ? Ft[j * k + c] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int c = c0 + r;
    const int64_t j = j0 + tx;
    if (c < k && j < n) F[(int64_t)c * n + j] += tile[tx][r];
  }
}

int launch_add_transposed(const double *Ft, int64_t n, int k, double *F, hipStream_t s) {
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((k + 63) / 64));
  hipLaunchKernelGGL(k_add_transposed, grid, 256, 0, s, Ft, n, k, F);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

}  // namespace lspca
