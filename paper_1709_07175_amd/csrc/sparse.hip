// Sketch Y = X Omega for the very sparse Omega of Sec. I-A (entries -1, 0, +1
// with probabilities 1/(2p), 1 - 1/p, 1/(2p)), without matrix cores and
// without Omega in HBM.
//
// Each workgroup regenerates Omega's nonzeros from the seed (Philox4x32-10,
// the mapping of include/lspca.h) into LDS as column lists: for output
// column c, the feature indices j with Omega[j][c] != 0 (15 bits) and the
// sign (bit 15), sorted by j so that every output is summed in the same
// order on every run. It then walks tiles of 4 rows of X: the tile is
// staged in LDS feature-major (the 4 rows of one feature in 8 bytes), and
// the thread that owns column c adds +-X[r][j] for the j in its list into 4
// FP32 accumulators (one per row): n/p signed adds per output.
#include "philox.h"

#include <cmath>
#include <cstdlib>

namespace lspca {

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

constexpr int kSpRows = 4;              // rows per tile
constexpr int kSpThreads = 256;

template <int DT> __device__ inline float h2f(uint16_t b);
template <> __device__ inline float h2f<LSPCA_BF16>(uint16_t b) { return bf16_bits_to_f32(b); }
template <> __device__ inline float h2f<LSPCA_F16>(uint16_t b) { return f16_bits_to_f32(b); }
template <int DT> __device__ inline uint16_t f2h(float f);
template <> __device__ inline uint16_t f2h<LSPCA_BF16>(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
template <> __device__ inline uint16_t f2h<LSPCA_F16>(float f) { return f32_to_f16_bits(f); }

// Dynamic LDS: [ X tile: n * 4 x 16-bit | start: k+1 ints | fill: k ints |
//                entries: cap x 16-bit ]
template <int DT>
__global__ __launch_bounds__(kSpThreads) void k_sparse_sketch(
    const uint16_t *__restrict__ X, int64_t m, int n, int64_t ldx, int k, uint32_t key0,
    uint32_t key1, uint32_t t_plus, uint64_t t_minus, int cap, float *__restrict__ Y, int64_t ldy,
    unsigned *__restrict__ colmax, uint16_t *__restrict__ Yh, uint16_t *__restrict__ Yl,
    int *__restrict__ overflow) {
  extern __shared__ __align__(16) unsigned char lds[];
  uint16_t *xt = (uint16_t *)lds;                                   // n * 4
  int *start = (int *)(lds + (((size_t)n * kSpRows * 2 + 15) & ~(size_t)15));
  int *fill = start + (k + 1);
  uint16_t *ent = (uint16_t *)(fill + k);
  const int tid = threadIdx.x;
  const int qk = (k + 3) / 4;

  // ---- column lists of Omega's nonzeros (counts, scan, scatter, sort)
  for (int c = tid; c < k; c += kSpThreads) fill[c] = 0;
  __syncthreads();
  const int64_t calls = (int64_t)n * qk;
  for (int64_t idx = tid; idx < calls; idx += kSpThreads) {
    const int j = (int)(idx / qk), q = (int)(idx % qk);
    uint32_t x[4];
    philox4x32_10(q, (uint32_t)j, 0u, kTagSparse, key0, key1, x);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 4 * q + t;
      if (c < k && (uint64_t)x[t] < t_minus) atomicAdd(&fill[c], 1);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int c = 0; c < k; ++c) {
      start[c] = acc;
      acc += fill[c];
    }
    start[k] = acc;
  }
  __syncthreads();
  // A list longer than the LDS capacity (a far tail event for the sizes the
  // host admits) switches this workgroup to regenerating each column's
  // entries on the fly: slower, same result.
  const bool fits = start[k] <= cap;
  if (!fits && tid == 0) atomicOr(overflow, 1);
  for (int c = tid; c < k; c += kSpThreads) fill[c] = 0;
  __syncthreads();
  for (int64_t idx = tid; fits && idx < calls; idx += kSpThreads) {
    const int j = (int)(idx / qk), q = (int)(idx % qk);
    uint32_t x[4];
    philox4x32_10(q, (uint32_t)j, 0u, kTagSparse, key0, key1, x);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 4 * q + t;
      if (c < k && (uint64_t)x[t] < t_minus) {
        const int pos = start[c] + atomicAdd(&fill[c], 1);
        ent[pos] = (uint16_t)(j | (x[t] < t_plus ? 0 : 0x8000));
      }
    }
  }
  __syncthreads();
  for (int c = tid; fits && c < k; c += kSpThreads) {          // insertion sort by j
    const int b = start[c], e = start[c + 1];
    for (int i = b + 1; i < e; ++i) {
      const uint16_t v = ent[i];
      int t = i - 1;
      while (t >= b && (ent[t] & 0x7fff) > (v & 0x7fff)) {
        ent[t + 1] = ent[t];
        --t;
      }
      ent[t + 1] = v;
    }
  }
  __syncthreads();

  // ---- row tiles
  const int64_t ntiles = (m + kSpRows - 1) / kSpRows;
  const int ngroups = (n + 7) / 8;
  const bool vec = (ldx % 8) == 0 && ((uintptr_t)X % 16) == 0;
  float cmax[4] = {0.f, 0.f, 0.f, 0.f};
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * kSpRows;
    for (int g = tid; g < ngroups; g += kSpThreads) {
      u16x8 v[kSpRows];
#pragma unroll
      for (int r = 0; r < kSpRows; ++r) {
        const int64_t gr = r0 + r;
        u16x8 x = {};
        if (gr < m) {
          const uint16_t *src = X + gr * ldx + 8 * g;
          if (vec && 8 * g + 7 < n) {
            x = *(const u16x8 *)src;
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = 8 * g + e < n ? src[e] : (uint16_t)0;
          }
        }
        v[r] = x;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (8 * g + e < n) {
          u16x4 w = {v[0][e], v[1][e], v[2][e], v[3][e]};
          *(u16x4 *)&xt[(8 * g + e) * kSpRows] = w;
        }
      }
    }
    __syncthreads();
    for (int cb = 0; cb < k; cb += kSpThreads) {
      const int c = cb + tid;
      if (c < k) {
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        if (fits) {
          const int b = start[c], e = start[c + 1];
          for (int i = b; i < e; ++i) {
            const uint16_t w = ent[i];
            const u16x4 xv = *(const u16x4 *)&xt[(w & 0x7fff) * kSpRows];
            const float s = (w & 0x8000) ? -1.f : 1.f;
            a0 += s * h2f<DT>(xv[0]);
            a1 += s * h2f<DT>(xv[1]);
            a2 += s * h2f<DT>(xv[2]);
            a3 += s * h2f<DT>(xv[3]);
          }
        } else {
          for (int j = 0; j < n; ++j) {               // same order: ascending j
            uint32_t x[4];
            philox4x32_10((uint32_t)(c >> 2), (uint32_t)j, 0u, kTagSparse, key0, key1, x);
            const uint32_t w = x[c & 3];
            if ((uint64_t)w < t_minus) {
              const u16x4 xv = *(const u16x4 *)&xt[j * kSpRows];
              const float s = w < t_plus ? 1.f : -1.f;
              a0 += s * h2f<DT>(xv[0]);
              a1 += s * h2f<DT>(xv[1]);
              a2 += s * h2f<DT>(xv[2]);
              a3 += s * h2f<DT>(xv[3]);
            }
          }
        }
        // Y is written transposed (ldy = rows of the stripe): as FP32 Yt[c][r]
        // (Y != NULL), or split into 16-bit parts Yh[c][r], Yl[c][r]
        const f32x4 a = {a0, a1, a2, a3};
        const bool full = r0 + 3 < m && (ldy & 3) == 0;
        if (Y) {
          float *dst = Y + (int64_t)c * ldy + r0;
          if (full) {
            *(f32x4 *)dst = a;
          } else {
#pragma unroll
            for (int r = 0; r < kSpRows; ++r)
              if (r0 + r < m) dst[r] = a[r];
          }
        } else {
          u16x4 hv, lv;
#pragma unroll
          for (int r = 0; r < kSpRows; ++r) {
            hv[r] = f2h<DT>(a[r]);
            lv[r] = f2h<DT>(a[r] - h2f<DT>(hv[r]));
          }
          uint16_t *dh = Yh + (int64_t)c * ldy + r0;
          uint16_t *dl = Yl ? Yl + (int64_t)c * ldy + r0 : nullptr;
          if (full) {
            *(u16x4 *)dh = hv;
            if (dl) *(u16x4 *)dl = lv;
          } else {
#pragma unroll
            for (int r = 0; r < kSpRows; ++r)
              if (r0 + r < m) {
                dh[r] = hv[r];
                if (dl) dl[r] = lv[r];
              }
          }
        }
        float amax = 0.f;
#pragma unroll
        for (int r = 0; r < kSpRows; ++r)
          if (r0 + r < m) amax = fmaxf(amax, fabsf(a[r]));
        cmax[cb >> 8] = fmaxf(cmax[cb >> 8], amax);
      }
    }
    __syncthreads();
  }
  if (colmax) {
    for (int cb = 0, i = 0; cb < k && i < 4; cb += kSpThreads, ++i) {
      const int c = cb + tid;
      if (c < k) atomicMax(colmax + c, __float_as_uint(cmax[i]));
    }
  }
}

// LDS needed for n features and a list capacity of cap entries.
static size_t sparse_lds_bytes(int n, int k, int cap) {
  return (((size_t)n * kSpRows * 2 + 15) & ~(size_t)15) + (size_t)(2 * k + 1) * 4 + (size_t)cap * 2;
}

// Whether the gather path applies: 16-bit X, n < 2^15, k <= 1024, and the
// expected number of nonzeros n k / p with a 10-sigma margin fits the list.
bool sparse_sketch_ok(lspca_dtype dt, int64_t n, int k, uint32_t p, int *cap_out) {
  if (dt != LSPCA_BF16 && dt != LSPCA_F16) return false;
  if (n >= 32768 || k > 1024) return false;
  const size_t budget = 160 * 1024;
  const size_t fixed = sparse_lds_bytes((int)n, k, 0);
  if (fixed >= budget) return false;
  const double mu = (double)n * k / p;                 // expected nonzeros
  const double want = mu + 10.0 * sqrt(mu) + 64;       // 10 sigma margin
  const double room = (double)(budget - fixed) / 2;
  if (want > room) return false;
  *cap_out = ((int)want + 63) & ~63;
  // test hook: a smaller capacity forces the on-the-fly fallback
  if (const char *e = getenv("LSPCA_SPARSE_CAP")) *cap_out = atoi(e);
  return true;
}

int launch_sparse_sketch(lspca_dtype dt, const void *X, int64_t m, int64_t n, int64_t ldx, int k,
                         uint64_t seed, uint32_t p, int cap, float *Y, int64_t ldy,
                         unsigned *colmax, void *Yh, void *Yl, int *overflow, hipStream_t s) {
  const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
  const uint32_t t_plus = (uint32_t)((1ull << 32) / (2ull * p));
  const uint64_t t_minus = (1ull << 32) / (uint64_t)p;
  const size_t lds = sparse_lds_bytes((int)n, k, cap);
  const int64_t ntiles = (m + kSpRows - 1) / kSpRows;
  int dev = 0, cus = 256;
  LSPCA_HIP(hipGetDevice(&dev));
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  const int64_t want = (int64_t)cus * (lds <= 80 * 1024 ? 2 : 1);
  const unsigned grid = (unsigned)(ntiles < want ? ntiles : want);
  if (dt == LSPCA_BF16) {
    LSPCA_HIP(hipFuncSetAttribute((const void *)k_sparse_sketch<LSPCA_BF16>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_sparse_sketch<LSPCA_BF16>, grid, kSpThreads, lds, s, (const uint16_t *)X, m,
                       (int)n, ldx, k, key0, key1, t_plus, t_minus, cap, Y, ldy, colmax, (uint16_t *)Yh, (uint16_t *)Yl, overflow);
  } else {
    LSPCA_HIP(hipFuncSetAttribute((const void *)k_sparse_sketch<LSPCA_F16>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_sparse_sketch<LSPCA_F16>, grid, kSpThreads, lds, s, (const uint16_t *)X, m,
                       (int)n, ldx, k, key0, key1, t_plus, t_minus, cap, Y, ldy, colmax, (uint16_t *)Yh, (uint16_t *)Yl, overflow);
  }
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

}  // namespace lspca
