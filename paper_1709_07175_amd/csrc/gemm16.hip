// Matrix-core products for 16-bit data (BF16 or FP16) with FP32 accumulation:
// v_mfma_f32_32x32x16_bf16 / v_mfma_f32_32x32x16_f16 (gfx950). Lane l holds
// A[l%32][8*(l/32) .. +7] and B[8*(l/32) .. +7][l%32]; result element v of
// lane l is D[8*(v/4) + 4*(l/32) + v%4][l%32] (checked on gfx950).
//
//  k_nt16: C[M x N] (FP32) = A[M x K] * (B_hi + B_lo)[N x K]^T, 16-bit
//          operands, both K-contiguous. Sketch Y = X Omega (no B_lo) and the
//          projection Z = X V with V split in two 16-bit parts.
//          Optionally records max |C| per column (for FP16 scaling).
//  k_tn16: P[s][M x N] (FP32) = sum over rows r of chunk s of
//          (Y_hi + Y_lo)[r][i] * X[r][j]: F = Y^T X with the FP32 sketch Y
//          split on load into 16-bit parts, Y = Y_hi + Y_lo (refinement) or
//          Y_hi alone; each column i of Y scaled by an exact power of two
//          first (FP16 range). Both operands are transposed into LDS so that
//          every fragment is one 16-byte read.
#include "common.h"

namespace lspca {

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

template <int DT> struct H16;
template <> struct H16<LSPCA_BF16> {
  __device__ static inline uint16_t from_f32(float f) { return f32_to_bf16_bits(f); }
  __device__ static inline float to_f32(uint16_t b) { return bf16_bits_to_f32(b); }
  __device__ static inline f32x16 mfma(u16x8 a, u16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
};
template <> struct H16<LSPCA_F16> {
  __device__ static inline uint16_t from_f32(float f) { return f32_to_f16_bits(f); }
  __device__ static inline float to_f32(uint16_t b) { return f16_bits_to_f32(b); }
  __device__ static inline f32x16 mfma(u16x8 a, u16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  }
};

__device__ inline int mrow(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// ------------------------------------------------------------------- NT16 --
// Tile BM x BN x 32, 4 waves as 2 x 2. VEC: 16-byte global loads (K % 8 == 0,
// 16-byte aligned rows); otherwise element loads.
template <int DT, int BM, int BN, bool SPLITB, bool VEC>
__global__ __launch_bounds__(256) void k_nt16(const uint16_t *__restrict__ A, int64_t lda,
                                              const uint16_t *__restrict__ Bh,
                                              const uint16_t *__restrict__ Bl, int64_t ldb,
                                              float *__restrict__ C, int64_t ldc, int64_t M, int N,
                                              int K, unsigned *__restrict__ colmax) {
  constexpr int BK = 32, LD = BK + 8;                 // +16 bytes per row of a tile
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 32, TN = WN / 32;
  constexpr int AV = BM * BK / 8 / 256, BV = BN * BK / 8 / 256;
  static_assert(AV >= 1 && BV >= 1, "tile too small");
  __shared__ uint16_t As[2][BM * LD];
  __shared__ uint16_t Bs[2][(SPLITB ? 2 : 1) * BN * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;

  u16x8 ra[AV], rbh[BV], rbl[SPLITB ? BV : 1];
  auto ld8 = [&](const uint16_t *p, bool ok, int kleft) -> u16x8 {
    u16x8 x = {};
    if (ok) {
      if constexpr (VEC) {
        x = *(const u16x8 *)p;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = e < kleft ? p[e] : (uint16_t)0;
      }
    }
    return x;
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int idx = tid + v * 256, r = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
      const int64_t gr = m0 + r;
      ra[v] = ld8(A + gr * lda + k0 + kc, gr < M && k0 + kc < K, K - k0 - kc);
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int idx = tid + v * 256, r = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
      const int gn = n0 + r;
      const bool ok = gn < N && k0 + kc < K;
      rbh[v] = ld8(Bh + (int64_t)gn * ldb + k0 + kc, ok, K - k0 - kc);
      if constexpr (SPLITB) rbl[v] = ld8(Bl + (int64_t)gn * ldb + k0 + kc, ok, K - k0 - kc);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int idx = tid + v * 256, r = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
      *(u16x8 *)&As[buf][r * LD + kc] = ra[v];
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int idx = tid + v * 256, r = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
      *(u16x8 *)&Bs[buf][r * LD + kc] = rbh[v];
      if constexpr (SPLITB) *(u16x8 *)&Bs[buf][(BN + r) * LD + kc] = rbl[v];
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = {};

  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int ko = kk + 8 * (lane >> 5);
      u16x8 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = *(const u16x8 *)&As[cur][(wm0 + i * 32 + (lane & 31)) * LD + ko];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = *(const u16x8 *)&Bs[cur][(wn0 + j * 32 + (lane & 31)) * LD + ko];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = H16<DT>::mfma(a[i], b[j], acc[i][j]);
      if constexpr (SPLITB) {
#pragma unroll
        for (int j = 0; j < TN; ++j)
          b[j] = *(const u16x8 *)&Bs[cur][(BN + wn0 + j * 32 + (lane & 31)) * LD + ko];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = H16<DT>::mfma(a[i], b[j], acc[i][j]);
      }
    }
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int c = n0 + wn0 + j * 32 + (lane & 31);
    float cmax = 0.f;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t r = m0 + wm0 + i * 32 + mrow(lane, v);
        if (r < M && c < N) {
          C[r * ldc + c] = acc[i][j][v];
          cmax = fmaxf(cmax, fabsf(acc[i][j][v]));
        }
      }
    if (colmax && c < N) atomicMax(colmax + c, __float_as_uint(cmax));
  }
}

// ------------------------------------------------------------------- TN16 --
// Tile: BM (columns of Y) x 128 (columns of X) x 32 rows; 4 waves as 2 x 2.
// Y: FP32 rows with leading dimension ldy, column i scaled by scale[i]
// (powers of two; NULL = 1). X: 16-bit rows, leading dimension ldx.
template <int DT, int BM, bool REFINE>
__global__ __launch_bounds__(256) void k_tn16(const float *__restrict__ Y, int64_t ldy,
                                              const uint16_t *__restrict__ X, int64_t ldx,
                                              float *__restrict__ P, int64_t rows, int Mi, int Nj,
                                              int64_t chunk, const float *__restrict__ scale) {
  constexpr int BN = 128, BK = 32, LD = BK + 8;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 32, TN = WN / 32;
  constexpr int NPART = REFINE ? 2 : 1;
  constexpr int AV = BM * BK / 4 / 256;               // float4 loads of Y per thread
  constexpr int BV = BN * BK / 8 / 256;               // 8 x 16-bit loads of X per thread
  __shared__ uint16_t As[2][NPART * BM * LD];
  __shared__ uint16_t Bs[2][BN * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  const int j0 = blockIdx.x * BN, i0 = blockIdx.y * BM;
  const int64_t rbeg = (int64_t)blockIdx.z * chunk;
  const int64_t rend = rbeg + chunk < rows ? rbeg + chunk : rows;

  f32x4 ra[AV];
  u16x8 rb[BV];
  float sc[AV][4];
#pragma unroll
  for (int v = 0; v < AV; ++v) {
    const int idx = tid + v * 256, c = (idx % (BM / 4)) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) sc[v][e] = (scale && i0 + c + e < Mi) ? scale[i0 + c + e] : 1.f;
  }
  auto load = [&](int64_t r0) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int idx = tid + v * 256, kr = idx / (BM / 4), c = (idx % (BM / 4)) * 4;
      const int64_t gr = r0 + kr;
      f32x4 x = {};
      if (gr < rend) {
        if (i0 + c + 3 < Mi && (ldy & 3) == 0) {
          x = *(const f32x4 *)(Y + gr * ldy + i0 + c);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) x[e] = i0 + c + e < Mi ? Y[gr * ldy + i0 + c + e] : 0.f;
        }
      }
      ra[v] = x;
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int idx = tid + v * 256, kr = idx / (BN / 8), c = (idx % (BN / 8)) * 8;
      const int64_t gr = r0 + kr;
      u16x8 x = {};
      if (gr < rend) {
        if (j0 + c + 7 < Nj && (ldx & 7) == 0) {
          x = *(const u16x8 *)(X + gr * ldx + j0 + c);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = j0 + c + e < Nj ? X[gr * ldx + j0 + c + e] : (uint16_t)0;
        }
      }
      rb[v] = x;
    }
  };
  // transposed stores: As[part][i][r], Bs[j][r]
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int idx = tid + v * 256, kr = idx / (BM / 4), c = (idx % (BM / 4)) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float y = ra[v][e] * sc[v][e];
        const uint16_t hi = H16<DT>::from_f32(y);
        As[buf][(c + e) * LD + kr] = hi;
        if constexpr (REFINE) As[buf][(BM + c + e) * LD + kr] = H16<DT>::from_f32(y - H16<DT>::to_f32(hi));
      }
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int idx = tid + v * 256, kr = idx / (BN / 8), c = (idx % (BN / 8)) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][(c + e) * LD + kr] = rb[v][e];
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = {};

  const int64_t nt = rend > rbeg ? (rend - rbeg + BK - 1) / BK : 0;
  if (nt > 0) {
    load(rbeg);
    store(0);
  }
  __syncthreads();
  for (int64_t t = 0; t < nt; ++t) {
    const int cur = (int)(t & 1);
    if (t + 1 < nt) load(rbeg + (t + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int ko = kk + 8 * (lane >> 5);
      u16x8 b[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = *(const u16x8 *)&Bs[cur][(wn0 + j * 32 + (lane & 31)) * LD + ko];
#pragma unroll
      for (int part = 0; part < NPART; ++part) {
        u16x8 a[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          a[i] = *(const u16x8 *)&As[cur][(part * BM + wm0 + i * 32 + (lane & 31)) * LD + ko];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = H16<DT>::mfma(a[i], b[j], acc[i][j]);
      }
    }
    if (t + 1 < nt) store(cur ^ 1);
    __syncthreads();
  }

  float *Pz = P + (int64_t)blockIdx.z * Mi * Nj;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = i0 + wm0 + i * 32 + mrow(lane, v);
        const int c = j0 + wn0 + j * 32 + (lane & 31);
        if (r < Mi && c < Nj) Pz[(int64_t)r * Nj + c] = acc[i][j][v];
      }
}

// ------------------------------------------------------------- launchers --
template <int DT, int BM, int BN, bool SPLITB>
static int nt16_typed(const uint16_t *A, int64_t lda, const uint16_t *Bh, const uint16_t *Bl,
                      int64_t ldb, float *C, int64_t ldc, int64_t M, int N, int K,
                      unsigned *colmax, hipStream_t s) {
  dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN));
  const bool vec = (lda % 8 == 0) && (ldb % 8 == 0) && (K % 8 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)Bh % 16 == 0) && (!SPLITB || (uintptr_t)Bl % 16 == 0);
  if (vec)
    hipLaunchKernelGGL((k_nt16<DT, BM, BN, SPLITB, true>), grid, dim3(256), 0, s, A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax);
  else
    hipLaunchKernelGGL((k_nt16<DT, BM, BN, SPLITB, false>), grid, dim3(256), 0, s, A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

template <int DT>
static int nt16_dt(const uint16_t *A, int64_t lda, const uint16_t *Bh, const uint16_t *Bl,
                   int64_t ldb, float *C, int64_t ldc, int64_t M, int N, int K, unsigned *colmax,
                   hipStream_t s) {
  if (Bl) {
    if (N > 128) return nt16_typed<DT, 128, 256, true>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, s);
    return nt16_typed<DT, 128, 128, true>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, s);
  }
  if (N > 128) return nt16_typed<DT, 128, 256, false>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, s);
  return nt16_typed<DT, 128, 128, false>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, s);
}

int launch_nt16(lspca_dtype dt, const void *A, int64_t lda, const void *Bh, const void *Bl,
                int64_t ldb, float *C, int64_t ldc, int64_t M, int N, int K, unsigned *colmax,
                hipStream_t s) {
  if (M <= 0 || N <= 0) return LSPCA_OK;
  if ((M + 127) / 128 > 0x7fffffff) {
    set_error("nt16 product: too many row tiles");
    return LSPCA_EINVAL;
  }
  if (dt == LSPCA_BF16)
    return nt16_dt<LSPCA_BF16>((const uint16_t *)A, lda, (const uint16_t *)Bh, (const uint16_t *)Bl, ldb, C, ldc, M, N, K, colmax, s);
  if (dt == LSPCA_F16)
    return nt16_dt<LSPCA_F16>((const uint16_t *)A, lda, (const uint16_t *)Bh, (const uint16_t *)Bl, ldb, C, ldc, M, N, K, colmax, s);
  set_error("nt16 product: dtype %d", (int)dt);
  return LSPCA_ENOTSUP;
}

template <int DT, int BM, bool REFINE>
static int tn16_typed(const float *Y, int64_t ldy, const uint16_t *X, int64_t ldx, float *P,
                      int64_t rows, int Mi, int Nj, int splits, const float *scale,
                      hipStream_t s) {
  int64_t chunk = (rows + splits - 1) / splits;
  chunk = (chunk + 31) / 32 * 32;
  dim3 grid((unsigned)((Nj + 127) / 128), (unsigned)((Mi + BM - 1) / BM), (unsigned)splits);
  hipLaunchKernelGGL((k_tn16<DT, BM, REFINE>), grid, dim3(256), 0, s, Y, ldy, X, ldx, P, rows, Mi, Nj, chunk, scale);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

template <int DT>
static int tn16_dt(const float *Y, int64_t ldy, const uint16_t *X, int64_t ldx, float *P,
                   int64_t rows, int Mi, int Nj, int splits, bool refine, const float *scale,
                   hipStream_t s) {
  if (Mi > 128) {
    if (refine) return tn16_typed<DT, 256, true>(Y, ldy, X, ldx, P, rows, Mi, Nj, splits, scale, s);
    return tn16_typed<DT, 256, false>(Y, ldy, X, ldx, P, rows, Mi, Nj, splits, scale, s);
  }
  if (refine) return tn16_typed<DT, 128, true>(Y, ldy, X, ldx, P, rows, Mi, Nj, splits, scale, s);
  return tn16_typed<DT, 128, false>(Y, ldy, X, ldx, P, rows, Mi, Nj, splits, scale, s);
}

int launch_tn16(lspca_dtype dt, const float *Y, int64_t ldy, const void *X, int64_t ldx, float *P,
                int64_t rows, int Mi, int Nj, int splits, bool refine, const float *scale,
                hipStream_t s) {
  if (Mi <= 0 || Nj <= 0 || splits <= 0) return LSPCA_OK;
  if (dt == LSPCA_BF16)
    return tn16_dt<LSPCA_BF16>(Y, ldy, (const uint16_t *)X, ldx, P, rows, Mi, Nj, splits, refine, scale, s);
  if (dt == LSPCA_F16)
    return tn16_dt<LSPCA_F16>(Y, ldy, (const uint16_t *)X, ldx, P, rows, Mi, Nj, splits, refine, scale, s);
  set_error("tn16 product: dtype %d", (int)dt);
  return LSPCA_ENOTSUP;
}

// Per-column power-of-two scales for FP16 operands: scale[c] = 2^e with
// colmax[c] * 2^e in [2^13, 2^14) (exact; no effect on the rounding of the
// mantissa), inv[c] = 2^-e. Columns that are all zero get scale 1.
__global__ void k_col_scales(const unsigned *colmax, int k, float *scale, double *inv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  const float mx = __uint_as_float(colmax[c]);
  int e = 0;
  if (mx > 0.f && isfinite(mx)) {
    int ex;
    frexpf(mx, &ex);             // mx in [2^(ex-1), 2^ex)
    e = 14 - ex;
    e = e > 100 ? 100 : (e < -100 ? -100 : e);
  }
  scale[c] = ldexpf(1.f, e);
  inv[c] = ldexp(1.0, -e);
}

int launch_col_scales(const unsigned *colmax, int k, float *scale, double *inv, hipStream_t s) {
  hipLaunchKernelGGL(k_col_scales, (k + 255) / 256, 256, 0, s, colmax, k, scale, inv);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

}  // namespace lspca
