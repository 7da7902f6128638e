// Matrix-core products for 16-bit data (BF16 or FP16) with FP32 accumulation:
// v_mfma_f32_32x32x16_bf16 / v_mfma_f32_32x32x16_f16 (gfx950). Lane l holds
// A[l%32][8*(l/32) .. +7] and B[8*(l/32) .. +7][l%32]; result element v of
// lane l is D[8*(v/4) + 4*(l/32) + v%4][l%32] (checked on gfx950).
//
//  k_nt16: C[M x N] (FP32) = A[M x K] * (B_hi + B_lo)[N x K]^T, 16-bit
//          operands, both K-contiguous. Sketch Y = X Omega (no B_lo) and the
//          projection Z = X V with V split in two 16-bit parts. The sketch
//          writes Y transposed (Yt, rows contiguous) for k_tn16, and can
//          record max |C| per column (for FP16 scaling).
//  k_tn16: P[s][M x N] (FP32) = sum over rows r of chunk s of
//          (Y_hi + Y_lo)[r][i] * X[r][j]: F = Y^T X with the sketch in
//          16-bit parts, Y = Y_hi + Y_lo (refinement) or Y_hi alone, either
//          given split (BF16) or split from the FP32 sketch as its tiles are
//          loaded, each column i scaled by an exact power of two first (FP16
//          range). Both LDS tiles are row-index contiguous, so every MFMA
//          fragment is one 16-byte read.
#include "common.h"

#include <atomic>
#include <cstdlib>
#include <type_traits>

namespace lspca {

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

template <int DT> struct H16;
template <> struct H16<LSPCA_BF16> {
  // (__bf16)f rounds to nearest even (v_cvt_pk_bf16_f32 on gfx950)
  __device__ static inline uint16_t from_f32(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
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

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4i16 lds_v4i16_t;


// ------------------------------------------------------------------- NT16 --
// Tile BM x BN x BK, WR x WC waves (2 x 2 unless chosen). VEC: 16-byte global loads (K % 8 == 0,
// 16-byte aligned rows); otherwise element loads.
// Output modes: OUT_ROWS: C row-major FP32 (ldc); OUT_T32: C transposed,
// C[c*ldc + r], FP32, with max |C| per column of each BM-row tile in
// colmax[tile][c] (bit patterns; NULL skips it); OUT_TSPLIT: the
// transposed result split into 16-bit parts Ch = rn(C), Cl = rn(C - Ch)
// (Cl may be NULL), each [c*ldc + r].
enum { OUT_ROWS = 0, OUT_T32 = 1, OUT_TSPLIT = 2 };

// Register stages of the K-tile prefetch in the 16-bit NT product, and the
// K depth of its tiles.
#ifndef LSPCA_NT16_STAGES
#define LSPCA_NT16_STAGES 3
#endif
#ifndef LSPCA_NT16_BK
#define LSPCA_NT16_BK 64
#endif
#ifndef LSPCA_NT16_SMALL_STAGES
#define LSPCA_NT16_SMALL_STAGES 3
#endif
// Row tile of the products whose B side is one column tile: the split-B
// product with N > 128 (projection with k > 128) and with N <= 128, and the
// unsplit product with N <= 128 (sketch). Larger row tiles cut the L2 reads
// of the B side per byte of A.
#ifndef LSPCA_NT16_PROJ_BM
#define LSPCA_NT16_PROJ_BM 256
#endif
#ifndef LSPCA_NT16_PROJ_BM_NARROW
#define LSPCA_NT16_PROJ_BM_NARROW 256
#endif
#ifndef LSPCA_NT16_SKETCH_BM
#define LSPCA_NT16_SKETCH_BM 256
#endif
// Waves per workgroup of the unsplit product with N <= 128 (sketch; 4, or 8
// as 4 x 2). With the 256-row tile, eight waves measured 5% faster than the
// 128 x 128 tile of four waves (which fits two workgroups per CU); four
// waves on the 256-row tile were slower.
#ifndef LSPCA_NT16_SKETCH_WAVES
#define LSPCA_NT16_SKETCH_WAVES 8
#endif
// Waves per workgroup of the split-B product (4 or 8). Eight waves (two per
// SIMD) keep more loads and LDS reads in flight next to the matrix cores:
// 10-15% faster projections with the large tiles above.
#ifndef LSPCA_NT16_PROJ_WAVES
#define LSPCA_NT16_PROJ_WAVES 8
#endif

// Stores one BM x BN tile of accumulators at (m0, n0) in the output mode
// OUT; red: WR x BN floats of LDS for the column maxima (OUT_T32). LDSSYNC:
// barriers that wait for LDS operations only (copies into LDS may stay in
// flight), else __syncthreads.
template <bool LDSSYNC> __device__ __forceinline__ void nt16_sync() {
  if constexpr (LDSSYNC) lds_barrier();
  else __syncthreads();
}

template <int DT, int BM, int BN, int OUT, int WR, int WC, bool LDSSYNC, int TM = BM / WR / 32, int TN = BN / WC / 32>
__device__ __forceinline__ void nt16_epilogue(const f32x16 (&acc)[TM][TN], float *__restrict__ C, int64_t ldc,
                                              int64_t M, int N, unsigned *__restrict__ colmax,
                                              uint16_t *__restrict__ Ch, uint16_t *__restrict__ Cl,
                                              const int64_t m0, const int n0, float *red) {
  constexpr int NT = 64 * WR * WC;
  constexpr int WM = BM / WR, WN = BN / WC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WC) * WM, wn0 = (wave % WC) * WN;
  float cm[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int c = n0 + wn0 + j * 32 + (lane & 31);
    float cmax = 0.f;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      if constexpr (OUT != OUT_ROWS) {
        // elements v = 4q .. 4q+3 of a lane are 4 consecutive rows
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t r = m0 + wm0 + i * 32 + mrow(lane, 4 * q);
          const f32x4 w = {acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2],
                           acc[i][j][4 * q + 3]};
          if (c < N) {
            const bool full = r + 3 < M && (ldc & 3) == 0;
            if constexpr (OUT == OUT_T32) {
              if (full) {
                *(f32x4 *)(C + (int64_t)c * ldc + r) = w;
              } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                  if (r + e < M) C[(int64_t)c * ldc + r + e] = w[e];
              }
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (r + e < M) cmax = fmaxf(cmax, fabsf(w[e]));
            } else {
              u16x4 hv, lv;
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                hv[e] = H16<DT>::from_f32(w[e]);
                lv[e] = H16<DT>::from_f32(w[e] - H16<DT>::to_f32(hv[e]));
              }
              if (full) {
                *(u16x4 *)(Ch + (int64_t)c * ldc + r) = hv;
                if (Cl) *(u16x4 *)(Cl + (int64_t)c * ldc + r) = lv;
              } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                  if (r + e < M) {
                    Ch[(int64_t)c * ldc + r + e] = hv[e];
                    if (Cl) Cl[(int64_t)c * ldc + r + e] = lv[e];
                  }
              }
            }
          }
        }
      } else {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t r = m0 + wm0 + i * 32 + mrow(lane, v);
          if (r < M && c < N) C[r * ldc + c] = acc[i][j][v];
        }
      }
    }
    if constexpr (OUT == OUT_T32) cm[j] = cmax;
  }
  if constexpr (OUT == OUT_T32) {
    // this tile's column maxima: lanes l and l + 32 hold one column, the two
    // waves of a column half meet in LDS; one plain store per column into
    // the partial row of this row tile (no atomics)
    if (colmax) {
      nt16_sync<LDSSYNC>();
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const float mj = fmaxf(cm[j], __shfl_xor(cm[j], 32));
        if (lane < 32) red[(wave / WC) * BN + wn0 + j * 32 + lane] = mj;
      }
      nt16_sync<LDSSYNC>();
      // one row per 128 rows of A (nt16_row_tiles), the same maximum in each
      // row this tile covers
      for (int t = tid; t < BN; t += NT)
        if (n0 + t < N) {
          float m = red[t];
#pragma unroll
          for (int w = 1; w < WR; ++w) m = fmaxf(m, red[w * BN + t]);
          const unsigned mv = __float_as_uint(m);
#pragma unroll
          for (int h = 0; h < BM / 128; ++h)
            if (m0 + 128 * h < M) colmax[(m0 / 128 + h) * (int64_t)N + n0 + t] = mv;
        }
    }
  }
}

// One BM x BN tile of C at (m0, n0); the LDS it stages through is free
// again on return, so a workgroup may call it for several tiles in turn.
template <int DT, int BM, int BN, bool SPLITB, bool VEC, int OUT, int WR = 2, int WC = 2>
__device__ __forceinline__ void nt16_tile(const uint16_t *__restrict__ A, int64_t lda,
                                          const uint16_t *__restrict__ Bh,
                                          const uint16_t *__restrict__ Bl, int64_t ldb,
                                          float *__restrict__ C, int64_t ldc, int64_t M, int N,
                                          int K, unsigned *__restrict__ colmax,
                                          uint16_t *__restrict__ Ch, uint16_t *__restrict__ Cl,
                                          const int64_t m0, const int n0) {
  // K depth of a tile: LSPCA_NT16_BK where two LDS buffers fit, else 32
  constexpr int BKW = LSPCA_NT16_BK;
  constexpr int BK = (BM + (SPLITB ? 2 : 1) * BN) * (BKW + 8) * 2 * 2 <= 160 * 1024 ? BKW : 32;
  constexpr int LD = BK + 8;                          // +16 bytes per row of a tile
  constexpr int NT = 64 * WR * WC;                   // WR x WC waves
  constexpr int WM = BM / WR, WN = BN / WC, TM = WM / 32, TN = WN / 32;
  constexpr int AV = BM * BK / 8 / NT, BV = BN * BK / 8 / NT;
  static_assert(AV >= 1 && BV >= 1, "tile too small");
  __shared__ uint16_t As[2][BM * LD];
  __shared__ uint16_t Bs[2][(SPLITB ? 2 : 1) * BN * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WC) * WM, wn0 = (wave % WC) * WN;

  // R register stages: the loads of K tile t + R are issued while tile t is
  // multiplied, so each load has R tile steps to arrive
  // the small projection tiles (one 32 x 32 block per wave, little work per
  // K tile) keep more tiles in flight
  constexpr int R = (BM == kProjSmallBM && BN == kProjSmallBN) ? LSPCA_NT16_SMALL_STAGES : LSPCA_NT16_STAGES;
  u16x8 ra[R][AV], rbh[R][BV], rbl[R][SPLITB ? BV : 1];
  // VEC: loads are issued unconditionally from clamped addresses (a row
  // past M or N only feeds outputs that are never written), so nothing
  // consumes a load before its stage is stored to LDS and the loads of
  // later stages stay in flight; pieces past K are zeroed at the store.
  const int64_t mlast = M - 1;
  const int nlast = N - 1;
  auto ld8 = [&](const uint16_t *p, bool ok, int kleft) -> u16x8 {
    u16x8 x = {};
    if (ok) {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = e < kleft ? p[e] : (uint16_t)0;
    }
    return x;
  };
  auto load = [&](int sl, int k0) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int idx = tid + v * NT, r = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
      const int64_t gr = m0 + r;
      if constexpr (VEC) {
        const int kk = k0 + kc < K ? k0 + kc : K - 8;
        ra[sl][v] = *(const u16x8 *)(A + (gr < M ? gr : mlast) * lda + kk);
      } else {
        ra[sl][v] = ld8(A + gr * lda + k0 + kc, gr < M && k0 + kc < K, K - k0 - kc);
      }
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int idx = tid + v * NT, r = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
      const int gn = n0 + r;
      if constexpr (VEC) {
        const int kk = k0 + kc < K ? k0 + kc : K - 8;
        const int64_t off = (int64_t)(gn < N ? gn : nlast) * ldb + kk;
        rbh[sl][v] = *(const u16x8 *)(Bh + off);
        if constexpr (SPLITB) rbl[sl][v] = *(const u16x8 *)(Bl + off);
      } else {
        const bool ok = gn < N && k0 + kc < K;
        rbh[sl][v] = ld8(Bh + (int64_t)gn * ldb + k0 + kc, ok, K - k0 - kc);
        if constexpr (SPLITB) rbl[sl][v] = ld8(Bl + (int64_t)gn * ldb + k0 + kc, ok, K - k0 - kc);
      }
    }
  };
  auto store = [&](int sl, int buf, int k0) {
    const u16x8 z = {};
    const bool tail = VEC && k0 + BK > K;          // uniform: the last, partial K tile
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int idx = tid + v * NT, r = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
      *(u16x8 *)&As[buf][r * LD + kc] = (tail && k0 + kc >= K) ? z : ra[sl][v];
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int idx = tid + v * NT, r = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
      const bool zero = tail && k0 + kc >= K;
      *(u16x8 *)&Bs[buf][r * LD + kc] = zero ? z : rbh[sl][v];
      if constexpr (SPLITB) *(u16x8 *)&Bs[buf][(BN + r) * LD + kc] = zero ? z : rbl[sl][v];
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = {};

  auto mma = [&](int cur) {
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
  };

  // Tile t lives in stage t % R. Steady state (groups of R steps) is
  // branch-free: the refill index is clamped to the last tile and the store
  // of the next tile always happens (a store past the end is never read),
  // so the compiler can count outstanding loads exactly.
  const int nk = (K + BK - 1) / BK;
#pragma unroll
  for (int sl = 0; sl < R; ++sl) load(sl, (sl < nk ? sl : nk - 1) * BK);
  store(0, 0, 0);
  __syncthreads();
  int kt0 = 0;
  for (; kt0 + R <= nk; kt0 += R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int kt = kt0 + u, cur = kt & 1;
      const int refill = kt + R < nk ? kt + R : nk - 1;
      load(u, refill * BK);                       // stage u's tile kt is already in LDS
      mma(cur);
      store((u + 1) % R, cur ^ 1, (kt + 1) * BK);
      __syncthreads();
    }
  }
  // the last nk % R tiles are already loaded
#pragma unroll
  for (int u = 0; u < R - 1; ++u) {
    const int kt = kt0 + u;
    if (kt >= nk) break;
    mma(kt & 1);
    if (kt + 1 < nk) store((u + 1) % R, (kt & 1) ^ 1, (kt + 1) * BK);
    __syncthreads();
  }

  nt16_epilogue<DT, BM, BN, OUT, WR, WC, false>(acc, C, ldc, M, N, colmax, Ch, Cl, m0, n0,
                                              reinterpret_cast<float *>(&As[0][0]));
}

template <int DT, int BM, int BN, bool SPLITB, bool VEC, int OUT, int WR = 2, int WC = 2>
__global__ __launch_bounds__(64 * WR * WC) void k_nt16(const uint16_t *__restrict__ A, int64_t lda,
                                              const uint16_t *__restrict__ Bh,
                                              const uint16_t *__restrict__ Bl, int64_t ldb,
                                              float *__restrict__ C, int64_t ldc, int64_t M, int N,
                                              int K, unsigned *__restrict__ colmax,
                                              uint16_t *__restrict__ Ch, uint16_t *__restrict__ Cl) {
  nt16_tile<DT, BM, BN, SPLITB, VEC, OUT, WR, WC>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl,
                                                  (int64_t)blockIdx.x * BM, (int)blockIdx.y * BN);
}

// FP16 split of the transposed FP32 sketch: column c (row of Yt) is scaled
// by scale[c] (a power of two) and split, Yh = rn(s y), Yl = rn(s y - Yh).
// VEC (ld a multiple of 8, 16-byte aligned rows): 8 elements of one column
// per thread, two 16-byte loads and one 16-byte store per part.
template <int DT, bool VEC>
__global__ void k_split16(const float *__restrict__ Yt, int64_t count, int64_t ld,
                          const float *__restrict__ scale, uint16_t *__restrict__ Yh,
                          uint16_t *__restrict__ Yl) {
  if constexpr (VEC) {
    const int64_t e8 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
    if (e8 >= count) return;
    const float sc = scale ? scale[e8 / ld] : 1.f;
    const f32x4 a = *(const f32x4 *)(Yt + e8), b = *(const f32x4 *)(Yt + e8 + 4);
    u16x8 h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float y = (e < 4 ? a[e & 3] : b[e & 3]) * sc;
      h[e] = H16<DT>::from_f32(y);
      l[e] = H16<DT>::from_f32(y - H16<DT>::to_f32(h[e]));
    }
    *(u16x8 *)(Yh + e8) = h;
    if (Yl) *(u16x8 *)(Yl + e8) = l;
  } else {
    const int64_t e4 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (e4 >= count) return;
    for (int e = 0; e < 4 && e4 + e < count; ++e) {
      const int64_t idx = e4 + e;
      const float y = Yt[idx] * (scale ? scale[idx / ld] : 1.f);
      const uint16_t h = H16<DT>::from_f32(y);
      Yh[idx] = h;
      if (Yl) Yl[idx] = H16<DT>::from_f32(y - H16<DT>::to_f32(h));
    }
  }
}

// ------------------------------------------------------------------- TN16 --
// Tile: BM (columns of Y) x BN (columns of X) x BK rows; WR x WC waves.
// Y arrives transposed and already split into 16-bit parts Yh, Yl (Yl NULL
// without refinement), 8 consecutive rows of one column contiguous: element
// (i, r) at (r / 8) * ysb + i * ysc + r % 8 (transposed: ysb = 8, ysc = the
// leading dimension; blocked in 8-row blocks: ysb = 8 * columns, ysc = 8),
// rows valid up to ylim, so its tiles go to LDS with 16-byte copies; or (YF)
// as the FP32 sketch Yf in the same indexing, each 8-row piece scaled by
// yscale[i] (NULL: 1) and split into the two parts on its way to LDS (the
// arithmetic of k_split16). X (16-bit rows,
// leading dimension ldx): each thread loads pieces of 2 rows x 8 columns
// and transposes them in registers into eight 2-row pieces of the
// column-major LDS tile Bs[j][r]. Both LDS tiles are row-index contiguous,
// so every MFMA fragment is one 16-byte read.
// VEC (16-byte aligned rows, ysc, ylim, ldx and Nj multiples of 8): loads are
// issued unconditionally from clamped addresses and rows past the chunk are
// zeroed at the LDS store, so the steady-state loop is branch-free and
// LSPCA_TN16_STAGES register stages of K tiles stay in flight.
#ifndef LSPCA_TN16_STAGES
#define LSPCA_TN16_STAGES 3
#endif
#ifndef LSPCA_TN16_BK
#define LSPCA_TN16_BK 64
#endif

template <int DT, int BM, int BN, bool REFINE, bool VEC, bool YF, int WR = 2, int WC = 2>
__global__ __launch_bounds__(64 * WR * WC) void k_tn16(const uint16_t *__restrict__ Yh,
                                              const uint16_t *__restrict__ Yl, int64_t ysb, int64_t ysc,
                                              int64_t ylim,
                                              const uint16_t *__restrict__ X, int64_t ldx,
                                              float *__restrict__ P, int64_t rows, int Mi, int Nj,
                                              int64_t chunk, const float *__restrict__ Yf,
                                              const float *__restrict__ yscale) {
  constexpr int NPART = REFINE ? 2 : 1;
  constexpr int BKW = LSPCA_TN16_BK;
  constexpr int BK = (NPART * BM + BN) * (BKW + 8) * 2 * 2 <= 160 * 1024 ? BKW : 32;
  constexpr int LD = BK + 8;
  constexpr int NT = 64 * WR * WC;                   // WR x WC waves
  constexpr int WM = BM / WR, WN = BN / WC, TM = WM / 32, TN = WN / 32;
  constexpr int AV = BM * BK / 8 / NT;                // u16x8 loads per part per thread
  constexpr int XP = BN * BK / 16 / NT;               // 2 x 8 pieces of X per thread
  // register stages: one fewer for the wide refined tile and for 256
  // accumulators per lane (the ring would not fit the register file next to
  // the accumulators)
#ifdef LSPCA_TN16_R
  constexpr int R = LSPCA_TN16_R;
#else
  constexpr int R = (((BN > 128 && REFINE) || TM * TN >= 16) && LSPCA_TN16_STAGES > 2) ? 2 : LSPCA_TN16_STAGES;
#endif
  static_assert(XP >= 1 && AV >= 1, "tile too small");
  __shared__ uint16_t As[2][NPART * BM * LD];
  __shared__ uint16_t Bs[2][BN * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WC) * WM, wn0 = (wave % WC) * WN;
  int bx, by, bz;
  xcd_map(bx, by, bz);
  const int j0 = bx * BN, i0 = by * BM;
  const int64_t rbeg = (int64_t)bz * chunk;
  const int64_t rend = rbeg + chunk < rows ? rbeg + chunk : rows;

  u16x8 ra[R][YF ? 1 : NPART][AV];
  f32x4 rf[R][YF ? AV : 1][2];                        // YF: 8 FP32 rows of one column
  u16x8 rb[R][XP][2];
  float scv[YF ? AV : 1];                             // YF: the scale of each loaded column
  if constexpr (YF) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int i = (tid + v * NT) / (BK / 8);
      scv[v] = yscale ? yscale[i0 + i < Mi ? i0 + i : Mi - 1] : 1.f;
    }
  }
  auto load = [&](int sl, int64_t r0) {
    if constexpr (YF) {
#pragma unroll
      for (int v = 0; v < AV; ++v) {
        const int idx = tid + v * NT, i = idx / (BK / 8), kr = (idx % (BK / 8)) * 8;
        const int64_t gr = r0 + kr;
        if constexpr (VEC) {
          const int ii = i0 + i < Mi ? i0 + i : Mi - 1;
          const int64_t rr = gr + 8 <= ylim ? gr : ylim - 8;      // gr, ylim: multiples of 8
          const float *src = Yf + (rr >> 3) * ysb + (int64_t)ii * ysc;
          rf[sl][v][0] = *(const f32x4 *)src;
          rf[sl][v][1] = *(const f32x4 *)(src + 4);
        } else {
          f32x4 a = {}, b = {};
          if (i0 + i < Mi) {
            const float *src = Yf + (gr >> 3) * ysb + (int64_t)(i0 + i) * ysc;   // gr % 8 == 0
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              a[e] = gr + e < rend ? src[e] : 0.f;
              b[e] = gr + 4 + e < rend ? src[4 + e] : 0.f;
            }
          }
          rf[sl][v][0] = a;
          rf[sl][v][1] = b;
        }
      }
    }
#pragma unroll
    for (int part = 0; part < (YF ? 0 : NPART); ++part) {
      const uint16_t *Ysrc = part ? Yl : Yh;
#pragma unroll
      for (int v = 0; v < AV; ++v) {
        const int idx = tid + v * NT, i = idx / (BK / 8), kr = (idx % (BK / 8)) * 8;
        const int64_t gr = r0 + kr;
        if constexpr (VEC) {
          const int ii = i0 + i < Mi ? i0 + i : Mi - 1;
          const int64_t rr = gr + 8 <= ylim ? gr : ylim - 8;      // gr, ylim: multiples of 8
          ra[sl][part][v] = *(const u16x8 *)(Ysrc + (rr >> 3) * ysb + (int64_t)ii * ysc);
        } else {
          u16x8 x = {};
          if (i0 + i < Mi) {
            const uint16_t *src = Ysrc + (gr >> 3) * ysb + (int64_t)(i0 + i) * ysc;   // gr % 8 == 0
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = gr + e < rend ? src[e] : (uint16_t)0;
          }
          ra[sl][part][v] = x;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < XP; ++p) {
      const int pidx = tid + p * NT, xp = pidx % (BK / 2), xg = pidx / (BK / 2);
      const int c = j0 + 8 * xg;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t gr = r0 + 2 * xp + h;
        if constexpr (VEC) {
          const int64_t rr = gr < rows ? gr : rows - 1;
          const int cc = c < Nj ? c : Nj - 8;
          rb[sl][p][h] = *(const u16x8 *)(X + rr * ldx + cc);
        } else {
          u16x8 x = {};
          if (gr < rend) {
            const uint16_t *src = X + gr * ldx + c;
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = c + e < Nj ? src[e] : (uint16_t)0;
          }
          rb[sl][p][h] = x;
        }
      }
    }
  };
  auto store = [&](int sl, int buf, int64_t r0) {
    const bool tail = VEC && r0 + BK > rend;            // uniform: the chunk's last K tile
    if constexpr (YF) {
      // scale and split on the way to LDS: Yh = rn(s y), Yl = rn(s y - Yh)
#pragma unroll
      for (int v = 0; v < AV; ++v) {
        const int idx = tid + v * NT, i = idx / (BK / 8), kr = (idx % (BK / 8)) * 8;
        u16x8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          float y = e < 4 ? rf[sl][v][0][e & 3] : rf[sl][v][1][e & 3];
          if (tail && r0 + kr + e >= rend) y = 0.f;
          y *= scv[v];
          h[e] = H16<DT>::from_f32(y);
          l[e] = H16<DT>::from_f32(y - H16<DT>::to_f32(h[e]));
        }
        *(u16x8 *)&As[buf][i * LD + kr] = h;
        if constexpr (REFINE) *(u16x8 *)&As[buf][(BM + i) * LD + kr] = l;
      }
    }
#pragma unroll
    for (int part = 0; part < (YF ? 0 : NPART); ++part)
#pragma unroll
      for (int v = 0; v < AV; ++v) {
        const int idx = tid + v * NT, i = idx / (BK / 8), kr = (idx % (BK / 8)) * 8;
        u16x8 x = ra[sl][part][v];
        if (tail) {
          const int64_t gr = r0 + kr;
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = gr + e < rend ? x[e] : (uint16_t)0;
        }
        *(u16x8 *)&As[buf][(part * BM + i) * LD + kr] = x;
      }
#pragma unroll
    for (int p = 0; p < XP; ++p) {
      const int pidx = tid + p * NT, xp = pidx % (BK / 2), xg = pidx / (BK / 2);
      u16x8 lo = rb[sl][p][0], hi = rb[sl][p][1];
      if (tail) {
        const int64_t gr = r0 + 2 * xp;
        const u16x8 z = {};
        lo = gr < rend ? lo : z;
        hi = gr + 1 < rend ? hi : z;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t w = (uint32_t)lo[e] | ((uint32_t)hi[e] << 16);
        *(uint32_t *)&Bs[buf][(8 * xg + e) * LD + 2 * xp] = w;
      }
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = {};

  auto mma = [&](int cur) {
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
  };

  const int64_t nt = rend > rbeg ? (rend - rbeg + BK - 1) / BK : 0;
  if (nt > 0) {
    // tile t lives in stage t % R; steady state branch-free (refill index
    // clamped to the last tile, the next tile's store always made)
#pragma unroll
    for (int sl = 0; sl < R; ++sl) load(sl, rbeg + (sl < nt ? sl : nt - 1) * BK);
    store(0, 0, rbeg);
    __syncthreads();
    int64_t t0 = 0;
    for (; t0 + R <= nt; t0 += R) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int64_t t = t0 + u;
        const int cur = (int)(t & 1);
        const int64_t refill = t + R < nt ? t + R : nt - 1;
        load(u, rbeg + refill * BK);
        mma(cur);
        store((u + 1) % R, cur ^ 1, rbeg + (t + 1) * BK);
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u < R - 1; ++u) {
      const int64_t t = t0 + u;
      if (t >= nt) break;
      mma((int)(t & 1));
      if (t + 1 < nt) store((u + 1) % R, (int)(t & 1) ^ 1, rbeg + (t + 1) * BK);
      __syncthreads();
    }
  }

  float *Pz = P + (int64_t)bz * Mi * Nj;
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

// ------------------------------------------------------------------ NT16 v2 --
// C = A (B_hi + B_lo)^T as k_nt16, for large M: persistent workgroups, each
// taking row tiles blockIdx.x, + gridDim.x, ... of one column tile, the K
// tiles of all its row tiles forming one stream through SX LDS stages. Both
// operands are copied from global memory straight into LDS (global_load_lds),
// one barrier per K tile; the MFMA fragments of a k step are read into
// registers while the previous step's products run, and the first step of
// the next K tile (of this or the next row tile) before the last products of
// this one. The accumulation order per element of C is that of nt16_tile
// (k steps of 16 in order; B_hi, then B_lo), so the two give the same bits.
// A and B rows are K-contiguous in LDS, BK / 8 chunks of 16 bytes per row,
// chunk c of row i at position c ^ ((i / rows-per-256-bytes) % chunks-per-
// row): the 16-byte fragment reads of 16 consecutive rows cover the 64 banks
// once. Needs 16-byte aligned rows, lda, ldb multiples of 8 and K a multiple
// of BK; rows past M and columns past N read clamped rows and are not stored.
template <int DT, int BM, int BN, bool SPLITB, int OUT, int WR, int WC, int BK, int SX>
__global__ __launch_bounds__(64 * WR * WC) void k_nt16v2(const uint16_t *__restrict__ A, int64_t lda,
                                                const uint16_t *__restrict__ Bh,
                                                const uint16_t *__restrict__ Bl, int64_t ldb,
                                                float *__restrict__ C, int64_t ldc, int64_t M, int N, int K,
                                                unsigned *__restrict__ colmax, uint16_t *__restrict__ Ch,
                                                uint16_t *__restrict__ Cl) {
  constexpr int NB = SPLITB ? 2 : 1;
  constexpr int NW = WR * WC;
  constexpr int WM = BM / WR, WN = BN / WC, TM = WM / 32, TN = WN / 32;
  constexpr int KS = BK / 16;                      // MFMA k steps per K tile
  constexpr int CPR = BK / 8;                      // 16-byte chunks per row
  constexpr int RPB = 16 / CPR;                    // rows per 256 bytes
  constexpr int ABYTES = BM * BK * 2, BBYTES = NB * BN * BK * 2;
  constexpr int STAGE = ABYTES + BBYTES;
  constexpr int AI = ABYTES / 1024, BI = BBYTES / 1024;   // 1 KB copy instructions per stage
  static_assert(AI % NW == 0 && BI % NW == 0, "copies split evenly over the waves");
  static_assert(KS % 2 == 0 && CPR <= 16, "tile shape");
  constexpr int AIW = AI / NW, BIW = BI / NW, LPW = AIW + BIW;
  static_assert((SX - 1) * LPW < 64 && SX >= 2, "copies in flight");
  __shared__ __align__(16) char lds[SX * STAGE];
  __shared__ float red[OUT == OUT_T32 ? WR * BN : 1];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave / WC) * WM, wn0 = (wave % WC) * WN;
  const int n0 = blockIdx.y * BN;
  const int64_t ntiles = (M + BM - 1) / BM;
  const int64_t G = gridDim.x;
  if ((int64_t)blockIdx.x >= ntiles) return;
  const int64_t T = (ntiles - blockIdx.x + G - 1) / G;    // row tiles of this workgroup
  const int nk = K / BK;
  const int64_t S = T * nk;                                // K tiles of this workgroup
  const uint32_t lds0 = lds_addr(lds);
  const int64_t mlast = M - 1;
  const int nlast = N - 1;

  // copy cursor: the next K tile to copy (row tile crt, K tile ckt); it stops
  // at the last one, so the copies past the end repeat it (never read; the
  // count of copies per K tile stays uniform)
  int64_t cs = 0, crt = blockIdx.x;
  int ckt = 0;
  auto issue = [&](int sl) {
    const uint32_t st = lds0 + sl * STAGE;
    const int64_t m0 = crt * BM;
    const int k0 = ckt * BK;
#pragma unroll
    for (int q = 0; q < AIW; ++q) {
      const int ins = wave + q * NW;
      const int c = ins * 64 + lane;
      const int i = c / CPR, pos = c % CPR;
      const int kc = pos ^ ((i / RPB) % CPR);
      const int64_t gr = m0 + i < M ? m0 + i : mlast;
      copy16_to_lds(A + gr * lda + k0 + 8 * kc, st + ins * 1024);
    }
#pragma unroll
    for (int q = 0; q < BIW; ++q) {
      const int ins = wave + q * NW;
      const int c = ins * 64 + lane;
      const int part = c / (BN * CPR), cc = c % (BN * CPR);
      const int n = cc / CPR, pos = cc % CPR;
      const int kc = pos ^ ((n / RPB) % CPR);
      const int gn = n0 + n < N ? n0 + n : nlast;
      copy16_to_lds((part ? Bl : Bh) + (int64_t)gn * ldb + k0 + 8 * kc, st + ABYTES + ins * 1024);
    }
    if (cs + 1 < S) {
      ++cs;
      if (++ckt == nk) {
        ckt = 0;
        crt += G;
      }
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = {};

  const int frow = lane & 31, fkh = lane >> 5;
  u16x8 fa[2][TM], fb[2][NB][TN];
  auto load_frag = [&](int set, int sl, int kk) {
    const char *st = lds + sl * STAGE;
    const int kc = (kk >> 3) + fkh;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int row = wm0 + i * 32 + frow;
      fa[set][i] = *(const u16x8 *)(st + row * (BK * 2) + 16 * (kc ^ ((row / RPB) % CPR)));
    }
#pragma unroll
    for (int part = 0; part < NB; ++part)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn0 + j * 32 + frow;
        fb[set][part][j] =
            *(const u16x8 *)(st + ABYTES + part * (BN * BK * 2) + n * (BK * 2) + 16 * (kc ^ ((n / RPB) % CPR)));
      }
  };
  auto mma = [&](int set) {
#pragma unroll
    for (int part = 0; part < NB; ++part)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = H16<DT>::mfma(fa[set][i], fb[set][part][j], acc[i][j]);
  };

#pragma unroll
  for (int sl = 0; sl < SX; ++sl) issue(sl);
  wait_vmcnt<(SX - 1) * LPW>();                    // K tile 0 landed (this wave's copies)
  lds_barrier();                                    // (every wave's)
  load_frag(0, 0, 0);
  int64_t rt = blockIdx.x;                          // row tile being multiplied
  int kt = 0;
  for (int64_t s = 0; s < S; ++s) {
    const int sl = (int)(s % SX);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int cur = ks & 1;                       // KS is even: step 0 of each K tile in set 0
      if (ks + 1 < KS) {
        load_frag(cur ^ 1, sl, 16 * (ks + 1));
      } else if (s + 1 < S) {
        // K tile s read into registers: tile s + 1 must have landed; then
        // stage sl is free for tile s + SX
        wait_vmcnt<(SX - 2) * LPW>();
        lds_barrier();
        issue(sl);
        load_frag(cur ^ 1, (int)((s + 1) % SX), 0);
      }
      mma(cur);
    }
    if (++kt == nk) {
      nt16_epilogue<DT, BM, BN, OUT, WR, WC, true>(acc, C, ldc, M, N, colmax, Ch, Cl, rt * BM, n0, red);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = {};
      kt = 0;
      rt += G;
    }
  }
  wait_vmcnt<0>();                                  // no copy may land after the workgroup ends
}

// ------------------------------------------------------------------ TN16 v2 --
// F = Y^T X as k_tn16 (split Y, no FP32 sketch), with both operands copied
// from global memory straight into LDS (global_load_lds, 16 bytes per lane: a
// wave instruction fills 1 KB of LDS, lane l the bytes 16 l .. 16 l + 15
// after the instruction's base) through SX LDS stages: no register staging,
// no LDS stores by the waves, one barrier per K tile. The MFMA fragments of a
// k step are read into registers while the previous step's products run, and
// the first step of tile t + 1 is read before the last products of tile t,
// so the barrier and the LDS latency sit behind matrix-core work. The
// accumulation order per output element is that of k_tn16 (k steps of 16 in
// order; high part, then low part), so the two give the same bits.
// X stays row-major in LDS; its B fragments (8 rows of one X column) come
// from ds_read_b64_tr_b16: within each 16-lane group, source lane s gives the
// address of 4 consecutive 16-bit elements and lane 4 a + e receives element
// e of source lanes a, a + 4, a + 8, a + 12 (checked on gfx950); so source
// lane s points at row s / 4 of a 4-row block, columns 4 (s % 4) .. + 3, and
// lane j gets column j's 4 rows. Bank conflicts: 16-byte chunks are swizzled
// within a row (X: chunk c of row r at position c ^ 4 (r % 4); Y: chunk c of
// row i at c ^ ((i / rows-per-256-bytes) % chunks-per-row)), so each
// half-wave's fragment reads cover the 64 banks once; the copies pick the
// source chunk for the position they fill, so the swizzle costs nothing.
// Rows past the chunk: the copies read clamped rows, and in the chunk's last
// tile the k rows at or past its end are zeroed in both fragments.
#ifndef LSPCA_TN16V2_BK
#define LSPCA_TN16V2_BK 32
#endif
#ifndef LSPCA_TN16V2_STAGES
#define LSPCA_TN16V2_STAGES 3
#endif

template <int DT, int BM, int BN, bool REFINE, int WR, int WC>
__global__ __launch_bounds__(64 * WR * WC) void k_tn16v2(const uint16_t *__restrict__ Yh,
                                                const uint16_t *__restrict__ Yl, int64_t ysb, int64_t ysc,
                                                int64_t ylim, const uint16_t *__restrict__ X, int64_t ldx,
                                                float *__restrict__ P, int64_t rows, int Mi, int Nj,
                                                int64_t chunk) {
  constexpr int NPART = REFINE ? 2 : 1;
  constexpr int BK = LSPCA_TN16V2_BK, SX = LSPCA_TN16V2_STAGES;
  constexpr int NW = WR * WC;
  constexpr int WM = BM / WR, WN = BN / WC, TM = WM / 32, TN = WN / 32;
  constexpr int KS = BK / 16;                      // MFMA k steps per tile
  constexpr int CPR = BK / 8;                      // 16-byte chunks per Y row (k runs)
  constexpr int RPB = 16 / CPR;                    // Y rows per 256 bytes
  constexpr int CPX = BN / 8;                      // 16-byte chunks per X row
  constexpr int YBYTES = NPART * BM * BK * 2, XBYTES = BK * BN * 2;
  constexpr int STAGE = YBYTES + XBYTES;
  constexpr int YI = YBYTES / 1024, XI = XBYTES / 1024;  // 1 KB copy instructions per stage
  static_assert(YI % NW == 0 && XI % NW == 0, "copies split evenly over the waves");
  static_assert(CPX >= 16 && BK % 32 == 0 && BK <= 64 && SX >= 2, "tile shape");
  constexpr int YIW = YI / NW, XIW = XI / NW, LPW = YIW + XIW;
  static_assert((SX - 1) * LPW < 64, "copies in flight");
  __shared__ __align__(16) char lds[SX * STAGE];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave / WC) * WM, wn0 = (wave % WC) * WN;
  int bx, by, bz;
  xcd_map(bx, by, bz);
  const int j0 = bx * BN, i0 = by * BM;
  const int64_t rbeg = (int64_t)bz * chunk;
  const int64_t rend = rbeg + chunk < rows ? rbeg + chunk : rows;
  const int64_t nt = rend > rbeg ? (rend - rbeg + BK - 1) / BK : 0;
  const uint32_t lds0 = lds_addr(lds);

  // copies of K tile t (rows rbeg + t BK ..) into stage sl
  auto issue = [&](int sl, int64_t t) {
    const uint32_t st = lds0 + sl * STAGE;
    const int64_t r0 = rbeg + t * BK;
#pragma unroll
    for (int q = 0; q < YIW; ++q) {
      const int ins = wave + q * NW;               // which KB of the stage's Y part
      const int c = ins * 64 + lane;               // chunk index within the Y tiles
      const int part = c / (BM * CPR), cc = c % (BM * CPR);
      const int i = cc / CPR, pos = cc % CPR;
      const int kc = pos ^ ((i / RPB) % CPR);
      const int ii = i0 + i < Mi ? i0 + i : Mi - 1;
      const int64_t gr = r0 + 8 * kc;
      const int64_t rr = gr + 8 <= ylim ? gr : ylim - 8;
      const uint16_t *src = (part ? Yl : Yh) + (rr >> 3) * ysb + (int64_t)ii * ysc;
      copy16_to_lds(src, st + ins * 1024);
    }
#pragma unroll
    for (int q = 0; q < XIW; ++q) {
      const int ins = wave + q * NW;
      const int c = ins * 64 + lane;
      const int r = c / CPX, pos = c % CPX;
      const int cx = pos ^ (4 * (r & 3));
      const int64_t gr = r0 + r < rows ? r0 + r : rows - 1;
      const int col = j0 + 8 * cx < Nj ? j0 + 8 * cx : Nj - 8;
      copy16_to_lds(X + gr * ldx + col, st + YBYTES + ins * 1024);
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = {};

  // per-lane parts of the fragment addresses
  const int arow = lane & 31, akh = lane >> 5;     // A: row in a 32-row block, k half
  const int g = lane >> 4, s = lane & 15;          // B: 16-lane group, source lane
  const int brow = 8 * (g >> 1) + (s >> 2);        // B: row within a 16-row k step (+ 4 h)
  const int bcol = 16 * (g & 1) + 4 * (s & 3);     // B: column within a 32-column block
  const int bk0 = 8 * (lane >> 5);                 // B: first k row this lane receives (+ 4 h)

  // Fragments of one k step, in two register sets (the step being multiplied
  // and the next one).
  u16x8 fa[2][NPART][TM], fb[2][TN];
  auto load_frag = [&](int set, int sl, int kk) {
    const char *st = lds + sl * STAGE;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = wn0 + j * 32 + bcol;
      v4i16 h2[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = kk + brow + 4 * h;
        const int pos = (col >> 3) ^ (4 * (r & 3));
        h2[h] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (lds_v4i16_t *)(st + YBYTES + r * (2 * BN) + 16 * pos + 2 * (col & 7)));
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        fb[set][j][e] = (uint16_t)h2[0][e];
        fb[set][j][4 + e] = (uint16_t)h2[1][e];
      }
    }
#pragma unroll
    for (int part = 0; part < NPART; ++part)
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int row = wm0 + i * 32 + arow;
        const int kc = (kk >> 3) + akh;
        const int pos = kc ^ ((row / RPB) % CPR);
        fa[set][part][i] = *(const u16x8 *)(st + part * (BM * BK * 2) + row * (BK * 2) + 16 * pos);
      }
  };
  // The products of one k step. TAIL (the chunk's last tile, first row r0):
  // the k rows at or past the chunk's end are zeroed in both operands first.
  auto mma = [&](int set, auto tailc, int kk, int64_t r0) {
    constexpr bool TAIL = decltype(tailc)::value;
    if constexpr (TAIL) {
      const int64_t lim = rend - r0 - kk;           // k rows of this step below lim are kept
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool za = 8 * akh + e >= lim, zb = bk0 + 4 * (e >> 2) + (e & 3) >= lim;
#pragma unroll
        for (int part = 0; part < NPART; ++part)
#pragma unroll
          for (int i = 0; i < TM; ++i) fa[set][part][i][e] = za ? 0 : fa[set][part][i][e];
#pragma unroll
        for (int j = 0; j < TN; ++j) fb[set][j][e] = zb ? 0 : fb[set][j][e];
      }
    }
#pragma unroll
    for (int part = 0; part < NPART; ++part)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = H16<DT>::mfma(fa[set][part][i], fb[set][j], acc[i][j]);
  };
  // one K tile: KS steps; the last step's loads are those of the next tile's
  // first step, after the wait for that tile and the refill of this stage
  auto tile = [&](int64_t t, auto tailc) {
    constexpr bool TAIL = decltype(tailc)::value;
    const int sl = (int)(t % SX);
    const int64_t r0 = rbeg + t * BK;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int cur = ks & 1;                       // KS is even: step 0 of each tile in set 0
      if (ks + 1 < KS) {
        load_frag(cur ^ 1, sl, 16 * (ks + 1));
      } else if constexpr (!TAIL) {
        // tile t read into registers: tile t + 1 must have landed; then
        // stage sl is free for tile t + SX
        wait_vmcnt<(SX - 2) * LPW>();
        lds_barrier();
        issue(sl, t + SX < nt ? t + SX : nt - 1);
        load_frag(cur ^ 1, (int)((t + 1) % SX), 0);
      }
      mma(cur, tailc, 16 * ks, r0);
    }
  };

  if (nt > 0) {
    // every stage filled first (tiles past the last are copies of the last,
    // never read: they keep the count of copies per tile uniform)
#pragma unroll
    for (int sl = 0; sl < SX; ++sl) issue(sl, sl < nt ? sl : nt - 1);
    wait_vmcnt<(SX - 1) * LPW>();                  // tile 0 landed (this wave's copies)
    lds_barrier();                                  // (every wave's)
    load_frag(0, 0, 0);
    for (int64_t t = 0; t + 1 < nt; ++t) tile(t, std::false_type{});
    tile(nt - 1, std::true_type{});
  }
  wait_vmcnt<0>();                                  // no copy may land after the workgroup ends

  float *Pz = P + (int64_t)bz * Mi * Nj;
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
// The direct-to-LDS form of the NT16 sketch (k_nt16v2) for the large tiles:
// the default; LSPCA_NT16_DIRECT=0 in the environment selects the
// register-staged k_nt16 instead (same bits), read per call.
#ifndef LSPCA_NT16_DIRECT_DEFAULT
#define LSPCA_NT16_DIRECT_DEFAULT 1
#endif
static bool nt16_direct() {
  const char *e = getenv("LSPCA_NT16_DIRECT");
  return e && *e ? atoi(e) != 0 : LSPCA_NT16_DIRECT_DEFAULT != 0;
}

// K depth and LDS stages of k_nt16v2 for a tile: 64-deep K tiles where three
// stages fit in 144 KB, else 32-deep; up to four stages.
template <int BM, int BN, bool SPLITB> struct Nt16v2Shape {
  static constexpr int NB = SPLITB ? 2 : 1;
  static constexpr int BK = 3 * (BM + NB * BN) * 64 * 2 <= 147456 ? 64 : 32;
  static constexpr int STAGE = (BM + NB * BN) * BK * 2;
  static constexpr int SX = 147456 / STAGE > 4 ? 4 : 147456 / STAGE;
};

template <int DT, int BM, int BN, bool SPLITB, int OUT, int WR, int WC>
static int nt16_direct_launch(const uint16_t *A, int64_t lda, const uint16_t *Bh, const uint16_t *Bl,
                              int64_t ldb, float *C, int64_t ldc, int64_t M, int N, int K, unsigned *colmax,
                              uint16_t *Ch, uint16_t *Cl, hipStream_t s) {
  using Sh = Nt16v2Shape<BM, BN, SPLITB>;
  auto kern = k_nt16v2<DT, BM, BN, SPLITB, OUT, WR, WC, Sh::BK, Sh::SX>;
  static std::atomic<int> per_cu[64];              // resident workgroups per CU, by device
  int dev = 0;
  LSPCA_HIP(hipGetDevice(&dev));
  int per = dev < 64 ? per_cu[dev].load(std::memory_order_relaxed) : 0;
  if (per <= 0) {
    int cus = 0, occ = 0;
    LSPCA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LSPCA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * WR * WC, 0));
    per = cus * (occ > 0 ? occ : 1);
    if (dev < 64) per_cu[dev].store(per, std::memory_order_relaxed);
  }
  const int64_t ntiles = (M + BM - 1) / BM;
  const int gy = (N + BN - 1) / BN;
  int64_t gx = (per + gy - 1) / gy;
  gx = gx < ntiles ? gx : ntiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)gx, (unsigned)gy), dim3(64 * WR * WC), 0, s, A, lda, Bh, Bl, ldb, C,
                     ldc, M, N, K, colmax, Ch, Cl);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

template <int DT, int BM, int BN, bool SPLITB, int OUT, int WR = 2, int WC = 2>
static int nt16_typed(const uint16_t *A, int64_t lda, const uint16_t *Bh, const uint16_t *Bl,
                      int64_t ldb, float *C, int64_t ldc, int64_t M, int N, int K,
                      unsigned *colmax, uint16_t *Ch, uint16_t *Cl, hipStream_t s) {
  dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN));
  const bool vec = (lda % 8 == 0) && (ldb % 8 == 0) && (K % 8 == 0) && ((uintptr_t)A % 16 == 0) &&
                   ((uintptr_t)Bh % 16 == 0) && (!SPLITB || (uintptr_t)Bl % 16 == 0);
  // the direct form for the sketch (one B part); the projection with split
  // B measured slower in it (5% with the 128-wide B tile, and the 256 x 256
  // tile needs more registers than eight waves have)
  if constexpr (BM >= 128 && !SPLITB) {
    if (vec && K >= Nt16v2Shape<BM, BN, SPLITB>::BK && K % Nt16v2Shape<BM, BN, SPLITB>::BK == 0 && nt16_direct())
      return nt16_direct_launch<DT, BM, BN, SPLITB, OUT, WR, WC>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax,
                                                                 Ch, Cl, s);
  }
  if (vec)
    hipLaunchKernelGGL((k_nt16<DT, BM, BN, SPLITB, true, OUT, WR, WC>), grid, dim3(64 * WR * WC), 0, s, A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl);
  else
    hipLaunchKernelGGL((k_nt16<DT, BM, BN, SPLITB, false, OUT, WR, WC>), grid, dim3(64 * WR * WC), 0, s, A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

template <int DT, bool SPLITB, int OUT>
static int nt16_n(const uint16_t *A, int64_t lda, const uint16_t *Bh, const uint16_t *Bl,
                  int64_t ldb, float *C, int64_t ldc, int64_t M, int N, int K, unsigned *colmax,
                  uint16_t *Ch, uint16_t *Cl, hipStream_t s) {
  // projections of few rows: the small tiles (same bits per row, lower
  // latency: many workgroups share the walk over K)
  if constexpr (SPLITB && OUT == OUT_ROWS)
    if (M <= proj_small_rows((lspca_dtype)DT))
      return nt16_typed<DT, kProjSmallBM, kProjSmallBN, true, OUT, 1, 2>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K,
                                                                       colmax, Ch, Cl, s);
  constexpr int BMW = SPLITB ? LSPCA_NT16_PROJ_BM : 128;
  constexpr int BMN = SPLITB ? LSPCA_NT16_PROJ_BM_NARROW : LSPCA_NT16_SKETCH_BM;
  // waves of the split-B (projection) product: 2 x 2, or eight as 2 x 4
  // for the 256-wide B tile and 4 x 2 for the 128-wide one
  constexpr bool W8 = SPLITB && LSPCA_NT16_PROJ_WAVES == 8;
  if (N > 128)
    return nt16_typed<DT, BMW, 256, SPLITB, OUT, 2, W8 ? 4 : 2>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl, s);
  constexpr bool S8 = W8 || (!SPLITB && LSPCA_NT16_SKETCH_WAVES == 8);
  return nt16_typed<DT, BMN, 128, SPLITB, OUT, S8 ? 4 : 2, 2>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl, s);
}

template <int DT>
static int nt16_dt(const uint16_t *A, int64_t lda, const uint16_t *Bh, const uint16_t *Bl,
                   int64_t ldb, float *C, int64_t ldc, int64_t M, int N, int K, unsigned *colmax,
                   uint16_t *Ch, uint16_t *Cl, int mode, hipStream_t s) {
  if (Bl) return nt16_n<DT, true, OUT_ROWS>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl, s);
  if (mode == OUT_T32) return nt16_n<DT, false, OUT_T32>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl, s);
  if (mode == OUT_TSPLIT) return nt16_n<DT, false, OUT_TSPLIT>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl, s);
  return nt16_n<DT, false, OUT_ROWS>(A, lda, Bh, Bl, ldb, C, ldc, M, N, K, colmax, Ch, Cl, s);
}

int launch_nt16(lspca_dtype dt, const void *A, int64_t lda, const void *Bh, const void *Bl,
                int64_t ldb, float *C, int64_t ldc, int64_t M, int N, int K, unsigned *colmax,
                void *Ch, void *Cl, int mode, hipStream_t s) {
  if (M <= 0 || N <= 0) return LSPCA_OK;
  if ((M + 127) / 128 > 0x7fffffff / 2) {
    set_error("nt16 product: too many row tiles");
    return LSPCA_EINVAL;
  }
  if (dt == LSPCA_BF16)
    return nt16_dt<LSPCA_BF16>((const uint16_t *)A, lda, (const uint16_t *)Bh, (const uint16_t *)Bl, ldb, C, ldc, M, N, K, colmax, (uint16_t *)Ch, (uint16_t *)Cl, mode, s);
  if (dt == LSPCA_F16)
    return nt16_dt<LSPCA_F16>((const uint16_t *)A, lda, (const uint16_t *)Bh, (const uint16_t *)Bl, ldb, C, ldc, M, N, K, colmax, (uint16_t *)Ch, (uint16_t *)Cl, mode, s);
  set_error("nt16 product: dtype %d", (int)dt);
  return LSPCA_ENOTSUP;
}

// ------------------------------------------------------ batched projection --
// Persistent: workgroup b takes tiles b, b + grid, ... of the table (passed
// by value: it lives in the launch's kernel arguments, so no upload precedes
// the kernel); the request of a tile is found by binary search over the
// tiles' first numbers. Eight waves per workgroup, as the projection of lspca_transform (2 x 4 for
// the 256-wide V tile, else 4 x 2): the same accumulation order per element.
constexpr int kProjThreads = 512;
template <int BN> constexpr int proj_wr() { return BN >= 256 ? 2 : 4; }

template <int DT, int BM, int BN, bool VEC>
__global__ __launch_bounds__(kProjThreads) void k_proj_batch16(const ProjTable tab,
                                                      const uint16_t *__restrict__ Vh,
                                                      const uint16_t *__restrict__ Vl, int64_t ldv,
                                                      int N, int K) {
  const int ntiles = tab.ntiles, nreq = tab.nreq, ntn = tab.ntn;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int lo = tab.nreq_s, hi = nreq - 1;             // the standard-tile requests
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab.req[mid].tile0 <= t) lo = mid;
      else hi = mid - 1;
    }
    const ProjReq &rq = tab.req[lo];
    const int local = t - rq.tile0, mt = local / ntn;
    nt16_tile<DT, BM, BN, true, VEC, OUT_ROWS, proj_wr<BN>(), 8 / proj_wr<BN>()>(
        (const uint16_t *)rq.X, rq.ldx, Vh, Vl, ldv, (float *)rq.Z, rq.ldz, rq.rows, N, K, nullptr, nullptr,
        nullptr, (int64_t)mt * BM, (local - mt * ntn) * BN);
  }
}

// The small-tile class: requests [0, nreq_s) of the table, 32 x 64 tiles of
// two waves each (the same per-element chain as every other tile shape).
constexpr int kProjSmallThreads = 128;
template <int DT, bool VEC>
__global__ __launch_bounds__(kProjSmallThreads) void k_proj_batch16s(const ProjTable tab,
                                                            const uint16_t *__restrict__ Vh,
                                                            const uint16_t *__restrict__ Vl,
                                                            int64_t ldv, int N, int K) {
  const int ntiles = tab.ntiles_s, nreq = tab.nreq_s, ntn = tab.ntn_s;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab.req[mid].tile0 <= t) lo = mid;
      else hi = mid - 1;
    }
    const ProjReq &rq = tab.req[lo];
    const int local = t - rq.tile0, mt = local / ntn;
    nt16_tile<DT, kProjSmallBM, kProjSmallBN, true, VEC, OUT_ROWS, 1, 2>(
        (const uint16_t *)rq.X, rq.ldx, Vh, Vl, ldv, (float *)rq.Z, rq.ldz, rq.rows, N, K, nullptr, nullptr,
        nullptr, (int64_t)mt * kProjSmallBM, (local - mt * ntn) * kProjSmallBN);
  }
}

static const void *proj16s_kernel(lspca_dtype dt, bool vec) {
  if (dt == LSPCA_BF16)
    return vec ? (const void *)&k_proj_batch16s<LSPCA_BF16, true> : (const void *)&k_proj_batch16s<LSPCA_BF16, false>;
  return vec ? (const void *)&k_proj_batch16s<LSPCA_F16, true> : (const void *)&k_proj_batch16s<LSPCA_F16, false>;
}

// Rows up to which the 16-bit projection uses the small tiles: below it the
// latency of one standard tile (one workgroup walking all of K for a
// 256-column block) dominates; above it the standard tiles read V fewer
// times. LSPCA_PROJ_SMALL_ROWS overrides it (a tuning and test knob).
#ifndef LSPCA_PROJ_SMALL_ROWS
#define LSPCA_PROJ_SMALL_ROWS 8192
#endif
int64_t proj_small_rows(lspca_dtype dt) {
  if (dt != LSPCA_BF16 && dt != LSPCA_F16) return 0;
  if (const char *e = getenv("LSPCA_PROJ_SMALL_ROWS")) {
    const long long x = atoll(e);
    return x > 0 ? (int64_t)x : 0;
  }
  return LSPCA_PROJ_SMALL_ROWS;
}

int proj_small_grid(lspca_dtype dt, bool vec, int *grid) {
  int dev = 0, cus = 0, per = 0;
  LSPCA_HIP(hipGetDevice(&dev));
  LSPCA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  LSPCA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, proj16s_kernel(dt, vec), kProjSmallThreads, 0));
  *grid = cus * (per > 0 ? per : 1);
  return LSPCA_OK;
}

int launch_proj_batch_small(lspca_dtype dt, const ProjTable *tab, const void *VTh, const void *VTl,
                            int64_t ldv, int k, int n, bool vec, int grid, hipStream_t s) {
  if (dt != LSPCA_BF16 && dt != LSPCA_F16) {
    set_error("small projection tiles: dtype %d (16-bit only)", (int)dt);
    return LSPCA_ENOTSUP;
  }
  void *args[] = {(void *)tab, (void *)&VTh, (void *)&VTl, (void *)&ldv, (void *)&k, (void *)&n};
  LSPCA_HIP(hipLaunchKernel(proj16s_kernel(dt, vec), dim3(grid), dim3(kProjSmallThreads), args, 0, s));
  return LSPCA_OK;
}

template <int DT, int BN, bool VEC> static const void *proj16_fn() {
  return (const void *)&k_proj_batch16<DT, 128, BN, VEC>;
}
static const void *proj16_kernel(lspca_dtype dt, int k, bool vec) {
  const bool wide = k > 128;
  if (dt == LSPCA_BF16) {
    if (wide) return vec ? proj16_fn<LSPCA_BF16, 256, true>() : proj16_fn<LSPCA_BF16, 256, false>();
    return vec ? proj16_fn<LSPCA_BF16, 128, true>() : proj16_fn<LSPCA_BF16, 128, false>();
  }
  if (wide) return vec ? proj16_fn<LSPCA_F16, 256, true>() : proj16_fn<LSPCA_F16, 256, false>();
  return vec ? proj16_fn<LSPCA_F16, 128, true>() : proj16_fn<LSPCA_F16, 128, false>();
}

int proj16_grid(lspca_dtype dt, int k, bool vec, int *grid) {
  int dev = 0, cus = 0, per = 0;
  LSPCA_HIP(hipGetDevice(&dev));
  LSPCA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  LSPCA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, proj16_kernel(dt, k, vec), kProjThreads, 0));
  *grid = cus * (per > 0 ? per : 1);
  return LSPCA_OK;
}

int launch_proj_batch16(lspca_dtype dt, const ProjTable *tab, const void *VTh, const void *VTl, int64_t ldv,
                        int k, int n, bool vec, int grid, hipStream_t s) {
  void *args[] = {(void *)tab, (void *)&VTh, (void *)&VTl, (void *)&ldv, (void *)&k, (void *)&n};
  LSPCA_HIP(hipLaunchKernel(proj16_kernel(dt, k, vec), dim3(grid), dim3(kProjThreads), args, 0, s));
  return LSPCA_OK;
}

int launch_split16(lspca_dtype dt, const float *Yt, int64_t rows_k, int64_t ld, const float *scale,
                   void *Yh, void *Yl, hipStream_t s) {
  const int64_t count = rows_k * ld;
  const bool vec = ld % 8 == 0 && (uintptr_t)Yt % 16 == 0 && (uintptr_t)Yh % 16 == 0 &&
                   (uintptr_t)Yl % 16 == 0;
  const unsigned grid = vec ? (unsigned)((count / 8 + 255) / 256) : (unsigned)((count / 4 + 256) / 256);
  if (dt == LSPCA_BF16) {
    if (vec) hipLaunchKernelGGL((k_split16<LSPCA_BF16, true>), grid, 256, 0, s, Yt, count, ld, scale, (uint16_t *)Yh, (uint16_t *)Yl);
    else hipLaunchKernelGGL((k_split16<LSPCA_BF16, false>), grid, 256, 0, s, Yt, count, ld, scale, (uint16_t *)Yh, (uint16_t *)Yl);
  } else {
    if (vec) hipLaunchKernelGGL((k_split16<LSPCA_F16, true>), grid, 256, 0, s, Yt, count, ld, scale, (uint16_t *)Yh, (uint16_t *)Yl);
    else hipLaunchKernelGGL((k_split16<LSPCA_F16, false>), grid, 256, 0, s, Yt, count, ld, scale, (uint16_t *)Yh, (uint16_t *)Yl);
  }
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// X-column tile when the Y side is one 128-column tile (k <= 128): 512, so
// the L2 reads of Y per byte of X are a quarter of a 128-wide tile's.
#ifndef LSPCA_TN16_WIDE_BN
#define LSPCA_TN16_WIDE_BN 512
#endif
#ifndef LSPCA_TN16_WIDE_ALL
#define LSPCA_TN16_WIDE_ALL 0
#endif
// X-column tile when the Y side is one 256-column tile
#ifndef LSPCA_TN16_BN256
#define LSPCA_TN16_BN256 256
#endif
// Waves per workgroup of the F product (4 as 2 x 2, or 8: 4 x 2 when the
// tile is at least as tall as wide, else 2 x 4). Eight (two per SIMD, 128
// accumulators each) measured 14-15% faster than four.
#ifndef LSPCA_TN16_WAVES
#define LSPCA_TN16_WAVES 8
#endif

// The direct-to-LDS form of F = Y^T X (k_tn16v2) for split Y, vector-aligned
// operands: the default; LSPCA_TN16_DIRECT=0 in the environment selects the
// register-staged k_tn16 instead (same bits: the same MFMA chain per output
// element), read per call.
#ifndef LSPCA_TN16_DIRECT_DEFAULT
#define LSPCA_TN16_DIRECT_DEFAULT 1
#endif
static bool tn16_direct() {
  const char *e = getenv("LSPCA_TN16_DIRECT");
  return e && *e ? atoi(e) != 0 : LSPCA_TN16_DIRECT_DEFAULT != 0;
}

template <int DT, int BM, bool REFINE, bool YF>
static int tn16_typed(const uint16_t *Yh, const uint16_t *Yl, int64_t ysb, int64_t ysc, int64_t ylim,
                      const uint16_t *X, int64_t ldx, float *P, int64_t rows, int Mi, int Nj, int splits,
                      hipStream_t s, const float *Yf = nullptr, const float *yscale = nullptr) {
  constexpr int BN = (BM <= 128 || LSPCA_TN16_WIDE_ALL) ? LSPCA_TN16_WIDE_BN : LSPCA_TN16_BN256;
  constexpr int WR = LSPCA_TN16_WAVES == 8 ? (BM >= BN ? 4 : 2) : 2;
  constexpr int WC = LSPCA_TN16_WAVES == 8 ? 8 / WR : 2;
  int64_t chunk = (rows + splits - 1) / splits;
  chunk = (chunk + 63) / 64 * 64;                 // a multiple of every K-tile depth
  dim3 grid((unsigned)((Nj + BN - 1) / BN), (unsigned)((Mi + BM - 1) / BM), (unsigned)splits);
  const bool yvec = YF ? (uintptr_t)Yf % 16 == 0
                       : (uintptr_t)Yh % 16 == 0 && (!REFINE || (uintptr_t)Yl % 16 == 0);
  const bool vec = (ysc % 8 == 0) && (ylim % 8 == 0) && yvec && (ldx % 8 == 0) && ((uintptr_t)X % 16 == 0) &&
                   (Nj % 8 == 0) && Nj >= 8 && ylim >= 8;
  if constexpr (!YF) {
    if (vec && tn16_direct()) {
      hipLaunchKernelGGL((k_tn16v2<DT, BM, BN, REFINE, WR, WC>), grid, dim3(64 * WR * WC), 0, s, Yh, Yl, ysb, ysc,
                         ylim, X, ldx, P, rows, Mi, Nj, chunk);
      LSPCA_HIP(hipGetLastError());
      return LSPCA_OK;
    }
  }
  if (vec)
    hipLaunchKernelGGL((k_tn16<DT, BM, BN, REFINE, true, YF, WR, WC>), grid, dim3(64 * WR * WC), 0, s, Yh, Yl, ysb,
                       ysc, ylim, X, ldx, P, rows, Mi, Nj, chunk, Yf, yscale);
  else
    hipLaunchKernelGGL((k_tn16<DT, BM, BN, REFINE, false, YF, WR, WC>), grid, dim3(64 * WR * WC), 0, s, Yh, Yl, ysb,
                       ysc, ylim, X, ldx, P, rows, Mi, Nj, chunk, Yf, yscale);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

template <int DT>
static int tn16_dt(const uint16_t *Yh, const uint16_t *Yl, int64_t ysb, int64_t ysc, int64_t ylim,
                   const uint16_t *X, int64_t ldx, float *P, int64_t rows, int Mi, int Nj, int splits,
                   hipStream_t s) {
  if (Mi > 128) {
    if (Yl) return tn16_typed<DT, 256, true, false>(Yh, Yl, ysb, ysc, ylim, X, ldx, P, rows, Mi, Nj, splits, s);
    return tn16_typed<DT, 256, false, false>(Yh, Yl, ysb, ysc, ylim, X, ldx, P, rows, Mi, Nj, splits, s);
  }
  if (Yl) return tn16_typed<DT, 128, true, false>(Yh, Yl, ysb, ysc, ylim, X, ldx, P, rows, Mi, Nj, splits, s);
  return tn16_typed<DT, 128, false, false>(Yh, Yl, ysb, ysc, ylim, X, ldx, P, rows, Mi, Nj, splits, s);
}

int launch_tn16(lspca_dtype dt, const void *Yh, const void *Yl, int64_t ldyt, const void *X,
                int64_t ldx, float *P, int64_t rows, int Mi, int Nj, int splits, hipStream_t s,
                bool yblocked) {
  if (Mi <= 0 || Nj <= 0 || splits <= 0) return LSPCA_OK;
  // transposed: (i, r) at i * ldyt + r; blocked: 8-row blocks of Mi columns
  const int64_t ysb = yblocked ? 8 * (int64_t)Mi : 8, ysc = yblocked ? 8 : ldyt;
  const int64_t ylim = yblocked ? (rows + 7) / 8 * 8 : ldyt;
  if (dt == LSPCA_BF16)
    return tn16_dt<LSPCA_BF16>((const uint16_t *)Yh, (const uint16_t *)Yl, ysb, ysc, ylim, (const uint16_t *)X,
                               ldx, P, rows, Mi, Nj, splits, s);
  if (dt == LSPCA_F16)
    return tn16_dt<LSPCA_F16>((const uint16_t *)Yh, (const uint16_t *)Yl, ysb, ysc, ylim, (const uint16_t *)X,
                              ldx, P, rows, Mi, Nj, splits, s);
  set_error("tn16 product: dtype %d", (int)dt);
  return LSPCA_ENOTSUP;
}

int launch_tn16_f32y(lspca_dtype dt, const float *Yt, const float *scale, int64_t ldyt, bool refine,
                     const void *X, int64_t ldx, float *P, int64_t rows, int Mi, int Nj, int splits,
                     hipStream_t s) {
  if (Mi <= 0 || Nj <= 0 || splits <= 0) return LSPCA_OK;
  if (dt != LSPCA_F16) {
    set_error("tn16 product from an FP32 sketch: dtype %d (FP16 only)", (int)dt);
    return LSPCA_ENOTSUP;
  }
  const uint16_t *Xh = (const uint16_t *)X;
  if (Mi > 128) {
    if (refine) return tn16_typed<LSPCA_F16, 256, true, true>(nullptr, nullptr, 8, ldyt, ldyt, Xh, ldx, P, rows, Mi, Nj, splits, s, Yt, scale);
    return tn16_typed<LSPCA_F16, 256, false, true>(nullptr, nullptr, 8, ldyt, ldyt, Xh, ldx, P, rows, Mi, Nj, splits, s, Yt, scale);
  }
  if (refine) return tn16_typed<LSPCA_F16, 128, true, true>(nullptr, nullptr, 8, ldyt, ldyt, Xh, ldx, P, rows, Mi, Nj, splits, s, Yt, scale);
  return tn16_typed<LSPCA_F16, 128, false, true>(nullptr, nullptr, 8, ldyt, ldyt, Xh, ldx, P, rows, Mi, Nj, splits, s, Yt, scale);
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

// colmax[c] = max over row tiles t of part[t][c] (bit patterns of
// non-negative floats compare as unsigned integers); colmax zeroed first.
__global__ void k_colmax_reduce(const unsigned *__restrict__ part, int64_t tiles, int N,
                                unsigned *__restrict__ colmax) {
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    unsigned m = 0;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) m = max(m, part[t * N + c]);
    atomicMax(colmax + c, m);
  }
}

int nt16_row_tiles(int64_t M) { return (int)((M + 127) / 128); }

int launch_colmax_reduce(const unsigned *part, int64_t tiles, int N, unsigned *colmax, hipStream_t s) {
  const unsigned grid = (unsigned)(tiles < 512 ? tiles : 512);
  if (grid == 0) return LSPCA_OK;
  hipLaunchKernelGGL(k_colmax_reduce, grid, 256, 0, s, part, tiles, N, colmax);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

int launch_col_scales(const unsigned *colmax, int k, float *scale, double *inv, hipStream_t s) {
  hipLaunchKernelGGL(k_col_scales, (k + 255) / 256, 256, 0, s, colmax, k, scale, inv);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

}  // namespace lspca
