// Sparse X in CSR form (the paper's own data are sparse feature matrices,
// Sec. IV-A and V-A; Proposition 4 prices both products of the pass at
// O(nnz(X) l)): rows are samples; row i's entries are colidx[e], values[e]
// for e in [rowptr[i], rowptr[i + 1]). The pass of Algorithm 4 and the
// projection with such an X:
//
//  * k_csr_spmm: Y = X B for a dense row-major B (n x k; Omega for the
//    sketch, V for the projection). One wave per row, lanes over the k
//    columns, the row's entries taken in storage order (deterministic), B's
//    rows read contiguously.
//  * the CSC form of a stripe of rows, built on the device: a stable radix
//    sort of (column, entry) pairs keeps each column's entries in row order,
//    so every sum below has a fixed order.
//  * k_csc_factor: F += Y^T X column by column, F[c][j] = sum over column j's
//    entries of x * Y[row][c], FP64 accumulation; columns are cut into
//    segments of equal length (one wave each) so that a dense column does
//    not serialise the launch, and the segments' partial sums are added in
//    segment order.
//
// G = Y^T Y uses the dense products. The inputs are checked on the device
// (rowptr[0] >= 0, nondecreasing, rowptr[m] = nnz; 0 <= colidx < n) before
// any kernel indexes with them.
#include "common.h"

#include <hipcub/device/device_radix_sort.hpp>
#include <hipcub/device/device_scan.hpp>

namespace lspca {

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

int csr_check(const int64_t *rowptr, const int32_t *colidx, int64_t m, int64_t n, int64_t nnz,
              int *dflag, hipStream_t s) {
  LSPCA_TRY(zero_i32(dflag, 1, s));
  const int64_t work = (m + 1 > nnz ? m + 1 : nnz);
  const unsigned grid = (unsigned)std::min<int64_t>((work + 255) / 256, 4096);
  hipLaunchKernelGGL(k_csr_check, grid > 0 ? grid : 1, 256, 0, s, rowptr, colidx, m, n, nnz, dflag);
  LSPCA_HIP(hipGetLastError());
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
  return LSPCA_OK;
}

// acc[q] += v[t] * B[idx[t] * ldb + cb + lane + 64 q] for t in [t0, t1), in
// order of t (ACC: the accumulator type); four entries' loads in flight.
template <typename T, typename ACC, int KQ>
__device__ __forceinline__ void gather_acc(const int32_t *__restrict__ idx, const T *__restrict__ v,
                                           int64_t t0, int64_t t1, const T *__restrict__ B, int64_t ldb,
                                           int cb, int k, int lane, ACC (&acc)[KQ]) {
  bool on[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) on[q] = cb + lane + 64 * q < k;
  const T *Bc = B + cb + lane;
  int64_t t = t0;
  for (; t + 4 <= t1; t += 4) {
    int64_t r[4];
    ACC w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      r[u] = (int64_t)idx[t + u] * ldb;
      w[u] = (ACC)v[t + u];
    }
    T b[4][KQ];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < KQ; ++q) b[u][q] = on[q] ? Bc[r[u] + 64 * q] : T(0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < KQ; ++q) acc[q] = fma(w[u], (ACC)b[u][q], acc[q]);
  }
  for (; t < t1; ++t) {
    const int64_t r = (int64_t)idx[t] * ldb;
    const ACC w = (ACC)v[t];
#pragma unroll
    for (int q = 0; q < KQ; ++q)
      if (on[q]) acc[q] = fma(w, (ACC)Bc[r + 64 * q], acc[q]);
  }
}

// ---- Y[i][c] = sum_e v_e B[col_e][c] for rows r0 + i, i < rows (one wave
// per row; 64 KQ columns per pass over the row's entries)
template <typename T, int KQ>
__global__ __launch_bounds__(256) void k_csr_spmm(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colidx,
                                                  const T *__restrict__ vals, int64_t r0, int64_t rows,
                                                  const T *__restrict__ B, int k, T *__restrict__ Y,
                                                  int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= rows) return;
  const int64_t e0 = rowptr[r0 + i], e1 = rowptr[r0 + i + 1];
  for (int cb = 0; cb < k; cb += 64 * KQ) {
    T acc[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) acc[q] = T(0);
    gather_acc<T, T, KQ>(colidx, vals, e0, e1, B, k, cb, k, lane, acc);
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int c = cb + lane + 64 * q;
      if (c < k) Y[i * ldy + c] = acc[q];
    }
  }
}

int launch_csr_spmm(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals,
                    int64_t r0, int64_t rows, const void *B, int k, void *Y, int64_t ldy, hipStream_t s) {
  if (vdt != LSPCA_F32 && vdt != LSPCA_F64) {
    set_error("CSR values must be FP32 or FP64 (dtype %d)", (int)vdt);
    return LSPCA_ENOTSUP;
  }
  const size_t es = dtype_size(vdt);
  for (int64_t c0 = 0; c0 < rows; c0 += kCsrMaxRows) {      // grid size limit
    const int64_t cr = rows - c0 < kCsrMaxRows ? rows - c0 : kCsrMaxRows;
    const unsigned grid = (unsigned)((cr + 3) / 4);
    void *Yc = (char *)Y + (size_t)c0 * ldy * es;
    if (vdt == LSPCA_F32) {
      if (k <= 64)
        hipLaunchKernelGGL((k_csr_spmm<float, 1>), grid, 256, 0, s, rowptr, colidx, (const float *)vals,
                           r0 + c0, cr, (const float *)B, k, (float *)Yc, ldy);
      else if (k <= 128)
        hipLaunchKernelGGL((k_csr_spmm<float, 2>), grid, 256, 0, s, rowptr, colidx, (const float *)vals,
                           r0 + c0, cr, (const float *)B, k, (float *)Yc, ldy);
      else
        hipLaunchKernelGGL((k_csr_spmm<float, 4>), grid, 256, 0, s, rowptr, colidx, (const float *)vals,
                           r0 + c0, cr, (const float *)B, k, (float *)Yc, ldy);
    } else {
      if (k <= 64)
        hipLaunchKernelGGL((k_csr_spmm<double, 1>), grid, 256, 0, s, rowptr, colidx, (const double *)vals,
                           r0 + c0, cr, (const double *)B, k, (double *)Yc, ldy);
      else if (k <= 128)
        hipLaunchKernelGGL((k_csr_spmm<double, 2>), grid, 256, 0, s, rowptr, colidx, (const double *)vals,
                           r0 + c0, cr, (const double *)B, k, (double *)Yc, ldy);
      else
        hipLaunchKernelGGL((k_csr_spmm<double, 4>), grid, 256, 0, s, rowptr, colidx, (const double *)vals,
                           r0 + c0, cr, (const double *)B, k, (double *)Yc, ldy);
    }
    LSPCA_HIP(hipGetLastError());
  }
  return LSPCA_OK;
}

// ---- CSC of the stripe of rows [r0, r0 + rows), entries [e0, e1)
// one wave per row, lanes over its entries
__global__ __launch_bounds__(256) void k_csr_expand(const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ colidx, int64_t r0,
                                                    int64_t rows, int64_t e0, int32_t *__restrict__ keys,
                                                    uint32_t *__restrict__ idx, int32_t *__restrict__ rowof) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= rows) return;
  const int64_t a = rowptr[r0 + i], b = rowptr[r0 + i + 1];
  for (int64_t e = a + (threadIdx.x & 63); e < b; e += 64) {
    keys[e - e0] = colidx[e];
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

__global__ void k_f64_to_f32(const double *__restrict__ v, int64_t count, float *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride)
    out[t] = (float)v[t];
}

int launch_f64_to_f32(const double *V, int64_t count, float *out, hipStream_t s) {
  if (count <= 0) return LSPCA_OK;
  const unsigned grid = (unsigned)std::min<int64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(k_f64_to_f32, grid, 256, 0, s, V, count, out);
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

// colptr[j] = first position of a key >= j in the sorted keys (j <= n)
__global__ void k_colptr(const int32_t *__restrict__ skeys, int64_t cnt, int64_t n, int64_t *__restrict__ colptr) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > n) return;
  int64_t lo = 0, hi = cnt;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)skeys[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  colptr[j] = lo;
}

static int key_bits(int64_t n) {
  int b = 1;
  while ((int64_t)1 << b < n) ++b;
  return b;
}

// Work split of the column sums: segments of at most S entries; column j
// owns the segments [segoff[j], segoff[j + 1]), segcol maps a segment to its
// column.
__global__ void k_seg_count(const int64_t *__restrict__ colptr, int64_t n, int64_t S,
                            int64_t *__restrict__ segcnt) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) segcnt[j] = (colptr[j + 1] - colptr[j] + S - 1) / S;
  else if (j == n) segcnt[n] = 0;
}

__global__ void k_seg_fill(const int64_t *__restrict__ segoff, int64_t n, int32_t *__restrict__ segcol) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int64_t w = segoff[j]; w < segoff[j + 1]; ++w) segcol[w] = (int32_t)j;
}

int64_t csc_segment(int64_t cnt, int k) {
  int64_t S = (cnt * (int64_t)k * 8 + ((int64_t)1 << 31) - 1) >> 31;  // partials <= 2 GiB + n k
  return S < 256 ? 256 : S;
}

int64_t csc_segments_max(int64_t cnt, int64_t n, int k) {
  return n + (cnt + csc_segment(cnt, k) - 1) / csc_segment(cnt, k);
}

size_t csc_temp_bytes(int64_t cnt, int64_t n) {
  size_t sort = 0, scan = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort, (const int32_t *)nullptr, (int32_t *)nullptr,
                                           (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)cnt, 0,
                                           key_bits(n));
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (const int64_t *)nullptr, (int64_t *)nullptr,
                                         (int)(n + 1));
  return sort > scan ? sort : scan;
}

int build_csc(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals, int64_t r0,
              int64_t rows, int64_t e0, int64_t cnt, int64_t n, int k, CscBuffers &b, hipStream_t s) {
  if (cnt > 0) {
    hipLaunchKernelGGL(k_csr_expand, (unsigned)((rows + 3) / 4), 256, 0, s, rowptr, colidx, r0, rows, e0,
                       b.keys, b.idx, b.rowof);
    LSPCA_HIP(hipGetLastError());
    size_t tb = b.temp_bytes;
    LSPCA_HIP(hipcub::DeviceRadixSort::SortPairs(b.temp, tb, b.keys, b.skeys, b.idx, b.sidx, (int)cnt, 0,
                                                 key_bits(n), s));
    const unsigned g = (unsigned)((cnt + 255) / 256);
    if (vdt == LSPCA_F32)
      hipLaunchKernelGGL(k_csc_gather<float>, g, 256, 0, s, b.sidx, b.rowof, (const float *)vals, e0, cnt,
                         b.crow, (float *)b.cval);
    else
      hipLaunchKernelGGL(k_csc_gather<double>, g, 256, 0, s, b.sidx, b.rowof, (const double *)vals, e0, cnt,
                         b.crow, (double *)b.cval);
    LSPCA_HIP(hipGetLastError());
  }
  const unsigned gn = (unsigned)((n + 1 + 255) / 256);
  hipLaunchKernelGGL(k_colptr, gn, 256, 0, s, b.skeys, cnt, n, b.colptr);
  LSPCA_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_seg_count, gn, 256, 0, s, b.colptr, n, b.seg, b.segcnt);
  LSPCA_HIP(hipGetLastError());
  size_t tb = b.temp_bytes;
  LSPCA_HIP(hipcub::DeviceScan::ExclusiveSum(b.temp, tb, b.segcnt, b.segoff, (int)(n + 1), s));
  hipLaunchKernelGGL(k_seg_fill, (unsigned)((n + 255) / 256), 256, 0, s, b.segoff, n, b.segcol);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// ---- column sums F[c][j] += sum over column j of cval[t] * Y[crow[t]][c]
// (FP64). One wave per segment (grid-stride; the segment count is read on
// the device), lanes over c. A column of one segment adds into F directly;
// longer columns leave one partial row per segment in P, summed in segment
// order by k_seg_reduce.
template <typename T, int KQ>
__global__ __launch_bounds__(256) void k_csc_factor(const int64_t *__restrict__ colptr,
                                                    const int64_t *__restrict__ segoff,
                                                    const int32_t *__restrict__ segcol,
                                                    const int32_t *__restrict__ crow,
                                                    const T *__restrict__ cval, int64_t n, int64_t S,
                                                    const T *__restrict__ Y, int k, int64_t ldy,
                                                    double *__restrict__ F, double *__restrict__ P) {
  const int lane = threadIdx.x & 63;
  const int64_t nseg_all = segoff[n];
  for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < nseg_all; w += (int64_t)gridDim.x * 4) {
    const int64_t j = segcol[w];
    const int64_t first = segoff[j], nseg = segoff[j + 1] - first;
    const int64_t t0 = colptr[j] + (w - first) * S;
    const int64_t t1 = t0 + S < colptr[j + 1] ? t0 + S : colptr[j + 1];
    for (int cb = 0; cb < k; cb += 64 * KQ) {
      double acc[KQ];
#pragma unroll
      for (int q = 0; q < KQ; ++q) acc[q] = 0.0;
      gather_acc<T, double, KQ>(crow, cval, t0, t1, Y, ldy, cb, k, lane, acc);
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const int c = cb + lane + 64 * q;
        if (c >= k) continue;
        if (nseg == 1) F[(int64_t)c * n + j] += acc[q];
        else P[w * k + c] = acc[q];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_seg_reduce(const int64_t *__restrict__ segoff, int64_t n,
                                                    const double *__restrict__ P, int k,
                                                    double *__restrict__ F) {
  const int lane = threadIdx.x & 63;
  for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < n; j += (int64_t)gridDim.x * 4) {
    const int64_t w0 = segoff[j], w1 = segoff[j + 1];
    if (w1 - w0 < 2) continue;
    for (int c = lane; c < k; c += 64) {
      double sum = P[w0 * k + c];
      for (int64_t w = w0 + 1; w < w1; ++w) sum += P[w * k + c];
      F[(int64_t)c * n + j] += sum;
    }
  }
}

template <typename T>
static void factor_kq(const CscBuffers &b, int64_t n, const T *Y, int k, int64_t ldy, double *F,
                      unsigned grid, hipStream_t s) {
  if (k <= 64)
    hipLaunchKernelGGL((k_csc_factor<T, 1>), grid, 256, 0, s, b.colptr, b.segoff, b.segcol, b.crow,
                       (const T *)b.cval, n, b.seg, Y, k, ldy, F, b.P);
  else if (k <= 128)
    hipLaunchKernelGGL((k_csc_factor<T, 2>), grid, 256, 0, s, b.colptr, b.segoff, b.segcol, b.crow,
                       (const T *)b.cval, n, b.seg, Y, k, ldy, F, b.P);
  else
    hipLaunchKernelGGL((k_csc_factor<T, 4>), grid, 256, 0, s, b.colptr, b.segoff, b.segcol, b.crow,
                       (const T *)b.cval, n, b.seg, Y, k, ldy, F, b.P);
}

int launch_csc_factor(lspca_dtype vdt, const CscBuffers &b, int64_t n, int64_t cnt, const void *Y, int k,
                      int64_t ldy, double *F, hipStream_t s) {
  const int64_t segs = n + (cnt + b.seg - 1) / b.seg;
  const unsigned grid = (unsigned)std::min<int64_t>((segs + 3) / 4, 1 << 20);
  if (vdt == LSPCA_F32) factor_kq<float>(b, n, (const float *)Y, k, ldy, F, grid, s);
  else factor_kq<double>(b, n, (const double *)Y, k, ldy, F, grid, s);
  LSPCA_HIP(hipGetLastError());
  const unsigned gr = (unsigned)std::min<int64_t>((n + 3) / 4, 1 << 20);
  hipLaunchKernelGGL(k_seg_reduce, gr, 256, 0, s, b.segoff, n, b.P, k, F);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

}  // namespace lspca
