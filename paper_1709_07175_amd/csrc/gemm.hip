// Dense matrix-core products for FP32 and FP64 data on gfx950.
//
//  k_nt: C[M x N] = A[M x K] * B[N x K]^T, both operands K-contiguous.
//        Used for the sketch Y = X Omega (B = Omega^T, Algorithm 2 step 1),
//        the projection Z = X V (eq. (dim_reduction_maps)) and the n x k by
//        k x k products of the small stage.
//  k_tn: P[s][M x N] = sum over rows r of chunk s of A[r][i] * B[r][j],
//        a split over the long row dimension with one partial per split.
//        Used for F = Y^T X and G = Y^T Y (Algorithm 2 step 2 / Algorithm 4
//        step 2a-2b: each split is a horizontal slice X_s), and for Gram
//        matrices in the small stage.
//
// Both stage K-tiles of A and B through LDS (double buffered, one barrier
// per tile) and run v_mfma_f32_16x16x4f32 (FP32) or v_mfma_f64_16x16x4f64
// (FP64) on fragments read from LDS. 256 threads = 4 waves of 64 lanes.
#include "common.h"

#include <atomic>
#include <cstdlib>
#include <type_traits>

// K depth and register prefetch stages of the FP32 NT product tiles.
#ifndef LSPCA_NT32_BK
#define LSPCA_NT32_BK 32
#endif
#ifndef LSPCA_NT32_STAGES
#define LSPCA_NT32_STAGES 2
#endif

namespace lspca {

template <typename T> struct Mfma;

// v_mfma_f32_16x16x4f32: lane l holds A[l%16][l/16] and B[l/16][l%16];
// result element v of lane l is D[4*(l/16) + v][l%16] (checked on gfx950).
// On gfx950 it runs at the FP32 matrix peak, 1.25x the rate measured for
// v_mfma_f32_32x32x2f32 (about 154 against 124 TFLOP/s of independent
// chains over all CUs).
template <> struct Mfma<float> {
  static constexpr int MB = 16, KB = 4, NV = 4;
  typedef f32x4 acc_t;
  __device__ static inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16] and B[l/16][l%16];
// result element v of lane l is D[l/16 + 4*v][l%16] (checked on gfx950).
template <> struct Mfma<double> {
  static constexpr int MB = 16, KB = 4, NV = 4;
  typedef f64x4 acc_t;
  __device__ static inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef f32x4 type; static constexpr int W = 4; };
template <> struct Vec16<double> { typedef f64x2 type; static constexpr int W = 2; };

// --------------------------------------------------------------------- NT --
// One BM x BN tile of C at (m0, n0); the LDS it stages through is free
// again on return, so a workgroup may call it for several tiles in turn.
template <typename T, int BM, int BN, int BK, int WGM, int WGN, bool VEC, int R = 1>
__device__ __forceinline__ void nt_tile(const T *__restrict__ A, int64_t lda,
                                        const T *__restrict__ B, int64_t ldb,
                                        T *__restrict__ C, int64_t ldc,
                                        int64_t M, int N, int K, T alpha, T beta,
                                        const int64_t m0, const int n0) {
  typedef Mfma<T> MF;
  constexpr int MB = MF::MB, KB = MF::KB;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / MB, TN = WN / MB;
  // padded row of a tile. FP32: rows of BK + 4 floats (16-byte aligned, an
  // odd number of 16-byte units apart), so the 16-byte fragment reads of 16
  // rows fall on distinct banks; FP64: BK + 1.
  constexpr int LD = BK + (sizeof(T) == 4 ? 4 : 1);
  static_assert(sizeof(T) != 4 || BK % 16 == 0, "FP32 tiles: K depth a multiple of 16");
  constexpr int VW = VEC ? Vec16<T>::W : 1;
  constexpr int AV = BM * BK / VW / 256, BV = BN * BK / VW / 256;
  static_assert(WGM * WGN == 4, "4 waves");
  static_assert(AV * VW * 256 == BM * BK && BV * VW * 256 == BN * BK, "tile/threads");

  __shared__ __align__(16) T As[2][BM * LD];
  __shared__ __align__(16) T Bs[2][BN * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;

  // R register stages: the loads of K tile t + R are issued while tile t is
  // multiplied (R = 1: the next tile only)
  T ra[R][AV * VW], rb[R][BV * VW];
  auto load = [&](int sl, int k0) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      int idx = tid + v * 256;
      int r = idx / (BK / VW), kc = (idx % (BK / VW)) * VW;
      int64_t gr = m0 + r;
      if constexpr (VEC) {
        // unconditional load from a clamped address (a row past M only feeds
        // outputs that are never written; pieces past K are zeroed at the
        // store), so the compiler can count the loads in flight exactly
        const int64_t rr = gr < M ? gr : M - 1;
        const int kk = k0 + kc < K ? k0 + kc : K - VW;
        const typename Vec16<T>::type x = *(const typename Vec16<T>::type *)(A + rr * lda + kk);
#pragma unroll
        for (int e = 0; e < VW; ++e) ra[sl][v * VW + e] = x[e];
      } else {
        ra[sl][v] = (gr < M && k0 + kc < K) ? A[gr * lda + k0 + kc] : (T)0;
      }
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      int idx = tid + v * 256;
      int r = idx / (BK / VW), kc = (idx % (BK / VW)) * VW;
      int gn = n0 + r;
      if constexpr (VEC) {
        const int nn = gn < N ? gn : N - 1;
        const int kk = k0 + kc < K ? k0 + kc : K - VW;
        const typename Vec16<T>::type x = *(const typename Vec16<T>::type *)(B + (int64_t)nn * ldb + kk);
#pragma unroll
        for (int e = 0; e < VW; ++e) rb[sl][v * VW + e] = x[e];
      } else {
        rb[sl][v] = (gn < N && k0 + kc < K) ? B[(int64_t)gn * ldb + k0 + kc] : (T)0;
      }
    }
  };
  // store of the tile at k0; VEC: pieces past K (the last tile's) are zeroed
  auto store = [&](int sl, int buf, int k0) {
    const bool tail = VEC && k0 + BK > K;          // uniform
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      int idx = tid + v * 256;
      int r = idx / (BK / VW), kc = (idx % (BK / VW)) * VW;
      const bool z = tail && k0 + kc >= K;
#pragma unroll
      for (int e = 0; e < VW; ++e) As[buf][r * LD + kc + e] = z ? (T)0 : ra[sl][v * VW + e];
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      int idx = tid + v * 256;
      int r = idx / (BK / VW), kc = (idx % (BK / VW)) * VW;
      const bool z = tail && k0 + kc >= K;
#pragma unroll
      for (int e = 0; e < VW; ++e) Bs[buf][r * LD + kc + e] = z ? (T)0 : rb[sl][v * VW + e];
    }
  };

  typename MF::acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = {};

  auto mma = [&](int cur) {
    if constexpr (sizeof(T) == 4) {
      // FP32: a lane reads 4 consecutive k of its row (16 bytes) and element
      // e of every lane's 4-vector goes to the e-th of four MFMAs, which sums
      // k = kk + 4 g + e over the 16-lane groups g (A and B under the same
      // map): the order of k_nt32s, so the two give the same bits
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        f32x4 a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          a[i] = *(const f32x4 *)&As[cur][(wm0 + i * MB + lane % MB) * LD + kk + 4 * (lane / MB)];
#pragma unroll
        for (int j = 0; j < TN; ++j)
          b[j] = *(const f32x4 *)&Bs[cur][(wn0 + j * MB + lane % MB) * LD + kk + 4 * (lane / MB)];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = MF::op(a[i][e], b[j][e], acc[i][j]);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += KB) {
        T a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[cur][(wm0 + i * MB + lane % MB) * LD + kk + lane / MB];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[cur][(wn0 + j * MB + lane % MB) * LD + kk + lane / MB];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = MF::op(a[i], b[j], acc[i][j]);
      }
    }
  };

  const int nk = (K + BK - 1) / BK;
  if constexpr (R == 1) {
    load(0, 0);
    store(0, 0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      if (kt + 1 < nk) load(0, (kt + 1) * BK);
      mma(cur);
      if (kt + 1 < nk) store(0, cur ^ 1, (kt + 1) * BK);
      __syncthreads();
    }
  } else {
    // tile t lives in stage t % R; the refill index is clamped to the last
    // tile (a load past it is never stored), so the steady state has no
    // branch around loads
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
        load(u, refill * BK);
        mma(cur);
        store((u + 1) % R, cur ^ 1, (kt + 1) * BK);   // past the end: never read
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u < R - 1; ++u) {
      const int kt = kt0 + u;
      if (kt >= nk) break;
      mma(kt & 1);
      if (kt + 1 < nk) store((u + 1) % R, (kt & 1) ^ 1, (kt + 1) * BK);
      __syncthreads();
    }
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < MF::NV; ++v) {
        int64_t r = m0 + wm0 + i * MB + MF::row(lane, v);
        int c = n0 + wn0 + j * MB + lane % MB;
        if (r < M && c < N) {
          T val = alpha * acc[i][j][v];
          if (beta != (T)0) val += beta * C[r * ldc + c];
          C[r * ldc + c] = val;
        }
      }
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN, bool VEC, int R = 1>
__global__ __launch_bounds__(256, 2) void k_nt(const T *__restrict__ A, int64_t lda,
                                            const T *__restrict__ B, int64_t ldb,
                                            T *__restrict__ C, int64_t ldc,
                                            int64_t M, int N, int K, T alpha, T beta) {
  // the side with fewer tiles is the short operand, kept in L2: its tiles
  // go fastest so that each block of the long operand is read once
  const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  int64_t tm, tn;
  int f;
  if (tiles_n <= tiles_m) {
    xcd_linear(tiles_m * tiles_n, (int)tiles_n, tm, f);
    tn = f;
  } else {
    xcd_linear(tiles_m * tiles_n, (int)tiles_m, tn, f);
    tm = f;
  }
  nt_tile<T, BM, BN, BK, WGM, WGN, VEC, R>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, tm * BM, (int)tn * BN);
}

// ------------------------------------------------------------ NT32 stream --
// C = A B^T in FP32 for the sketch Y = X Omega of a large stripe: persistent
// workgroups (one per CU) walk row tiles blockIdx.x, + gridDim.x, ...; the K
// tiles of all their row tiles form one stream through SX LDS stages filled
// by copies straight from global memory (global_load_lds, 16 bytes per lane,
// one barrier per K tile, no register staging). Rows of both tiles are
// K-contiguous in LDS, 16-byte chunk c of row r at position c ^ ((r / RPB) %
// CPR) (RPB rows per 256 bytes, CPR chunks per row), so the 16-byte
// fragment reads of 16 consecutive rows cover the 64 banks once. A lane reads
// 4 consecutive k of its row at once and feeds them to 4 successive
// v_mfma_f32_16x16x4f32 (element e of every lane's 4-vector in the e-th):
// the e-th instruction sums k = kk + 4 g + e over the 16-lane groups g, and
// the four together all 16 k of the step, with A and B under the same map.
// Fragments of the next k step are read while the current one's products
// run, and the next K tile's first step before the current tile's last
// products. Needs 16-byte aligned rows, lda, ldb multiples of 4 and K a
// multiple of BK; rows past M and N read clamped rows and are not stored.
template <int BM, int BN, int WR, int WC, int BK, int SX>
__global__ __launch_bounds__(64 * WR * WC) void k_nt32s(const float *__restrict__ A, int64_t lda,
                                               const float *__restrict__ B, int64_t ldb,
                                               float *__restrict__ C, int64_t ldc, int64_t M, int N,
                                               int K) {
  constexpr int NW = WR * WC;
  constexpr int WM = BM / WR, WN = BN / WC, TM = WM / 16, TN = WN / 16;
  constexpr int KS = BK / 16;                      // k steps of 16 per K tile
  constexpr int CPR = BK / 4;                      // 16-byte chunks per row
  constexpr int RPB = 256 / (BK * 4);              // rows per 256 bytes
  constexpr int ABYTES = BM * BK * 4, BBYTES = BN * BK * 4;
  constexpr int STAGE = ABYTES + BBYTES;
  constexpr int AI = ABYTES / 1024, BI = BBYTES / 1024;
  static_assert(AI % NW == 0 && BI % NW == 0, "copies split evenly over the waves");
  static_assert(KS % 2 == 0 && RPB >= 1 && CPR <= 16, "tile shape");
  constexpr int AIW = AI / NW, BIW = BI / NW, LPW = AIW + BIW;
  static_assert((SX - 1) * LPW < 64 && SX >= 2, "copies in flight");
  __shared__ __align__(16) char lds[SX * STAGE];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave / WC) * WM, wn0 = (wave % WC) * WN;
  const int n0 = blockIdx.y * BN;
  const int64_t ntiles = (M + BM - 1) / BM;
  const int64_t G = gridDim.x;
  if ((int64_t)blockIdx.x >= ntiles) return;
  const int64_t T = (ntiles - blockIdx.x + G - 1) / G;
  const int nk = K / BK;
  const int64_t S = T * nk;
  const uint32_t lds0 = lds_addr(lds);
  const int64_t mlast = M - 1;
  const int nlast = N - 1;

  // copy cursor (row tile crt, K tile ckt); stops at the last K tile, so the
  // copies past the end repeat it (never read; uniform count per K tile)
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
      const int r = c / CPR, pos = c % CPR;
      const int kc = pos ^ ((r / RPB) % CPR);
      const int64_t gr = m0 + r < M ? m0 + r : mlast;
      copy16_to_lds(A + gr * lda + k0 + 4 * kc, st + ins * 1024);
    }
#pragma unroll
    for (int q = 0; q < BIW; ++q) {
      const int ins = wave + q * NW;
      const int c = ins * 64 + lane;
      const int r = c / CPR, pos = c % CPR;
      const int kc = pos ^ ((r / RPB) % CPR);
      const int gn = n0 + r < N ? n0 + r : nlast;
      copy16_to_lds(B + (int64_t)gn * ldb + k0 + 4 * kc, st + ABYTES + ins * 1024);
    }
    if (cs + 1 < S) {
      ++cs;
      if (++ckt == nk) {
        ckt = 0;
        crt += G;
      }
    }
  };

  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = {};

  const int frow = lane & 15, fg = lane >> 4;
  f32x4 fa[2][TM], fb[2][TN];
  auto load_frag = [&](int set, int sl, int kk) {
    const char *st = lds + sl * STAGE;
    const int kc = (kk >> 2) + fg;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm0 + i * 16 + frow;
      fa[set][i] = *(const f32x4 *)(st + r * (BK * 4) + 16 * (kc ^ ((r / RPB) % CPR)));
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int r = wn0 + j * 16 + frow;
      fb[set][j] = *(const f32x4 *)(st + ABYTES + r * (BK * 4) + 16 * (kc ^ ((r / RPB) % CPR)));
    }
  };
  auto mma = [&](int set) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[set][i][e], fb[set][j][e], acc[i][j], 0, 0, 0);
  };

#pragma unroll
  for (int sl = 0; sl < SX; ++sl) issue(sl);
  wait_vmcnt<(SX - 1) * LPW>();
  lds_barrier();
  load_frag(0, 0, 0);
  int64_t rt = blockIdx.x;
  int kt = 0;
  for (int64_t s = 0; s < S; ++s) {
    const int sl = (int)(s % SX);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int cur = ks & 1;
      if (ks + 1 < KS) {
        load_frag(cur ^ 1, sl, 16 * (ks + 1));
      } else if (s + 1 < S) {
        wait_vmcnt<(SX - 2) * LPW>();              // K tile s + 1 landed (this wave's copies)
        lds_barrier();                              // (every wave's); stage sl is free
        issue(sl);
        load_frag(cur ^ 1, (int)((s + 1) % SX), 0);
      }
      mma(cur);
    }
    if (++kt == nk) {
      const int64_t m0 = rt * BM;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int c = n0 + wn0 + j * 16 + frow;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = m0 + wm0 + i * 16 + 4 * fg + v;
            if (r < M && c < N) C[r * ldc + c] = acc[i][j][v];
          }
          acc[i][j] = {};
        }
      kt = 0;
      rt += G;
    }
  }
  wait_vmcnt<0>();                                  // no copy may land after the workgroup ends
}

// The streamed FP32 sketch for a tile width: BN = 256 (eight waves as 2 x 4)
// above 128 columns, else 128 (four waves, 2 x 2); 32-deep K tiles, stages
// in 144 KB.
template <int BM, int BN, int WR, int WC>
static int nt32s_launch(const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc,
                        int64_t M, int N, int K, hipStream_t s) {
  constexpr int BK = 32, STAGE = (BM + BN) * BK * 4;
  constexpr int SX = 147456 / STAGE > 4 ? 4 : 147456 / STAGE;
  auto kern = k_nt32s<BM, BN, WR, WC, BK, SX>;
  static std::atomic<int> per_dev[64];
  int dev = 0;
  LSPCA_HIP(hipGetDevice(&dev));
  int per = dev < 64 ? per_dev[dev].load(std::memory_order_relaxed) : 0;
  if (per <= 0) {
    int cus = 0, occ = 0;
    LSPCA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LSPCA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * WR * WC, 0));
    per = cus * (occ > 0 ? occ : 1);
    if (dev < 64) per_dev[dev].store(per, std::memory_order_relaxed);
  }
  const int64_t ntiles = (M + BM - 1) / BM;
  const int gy = (N + BN - 1) / BN;
  int64_t gx = (per + gy - 1) / gy;
  gx = gx < ntiles ? gx : ntiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)gx, (unsigned)gy), dim3(64 * WR * WC), 0, s, A, lda, B, ldb, C, ldc, M,
                     N, K);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// Environment switch of the streamed FP32 product: LSPCA_NT32_STREAM=0 keeps
// the tiled k_nt (the same order of the k sums, so the same bits), read per
// call.
static bool nt32_stream_on() {
  const char *e = getenv("LSPCA_NT32_STREAM");
  return !(e && *e && atoi(e) == 0);
}

int launch_nt_tall(lspca_dtype dt, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                     int64_t ldc, int64_t M, int N, int K, hipStream_t s) {
  if (dt == LSPCA_F32 && M >= 4096 && K >= 32 && K % 32 == 0 && lda % 4 == 0 && ldb % 4 == 0 &&
      (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0 && nt32_stream_on()) {
    if (N > 128)
      return nt32s_launch<128, 256, 2, 4>((const float *)A, lda, (const float *)B, ldb, (float *)C, ldc, M, N, K,
                                          s);
    return nt32s_launch<128, 128, 2, 2>((const float *)A, lda, (const float *)B, ldb, (float *)C, ldc, M, N, K, s);
  }
  return launch_nt(dt, A, lda, B, ldb, C, ldc, M, N, K, s);
}

// --------------------------------------------------------------------- TN --
template <typename T, int BM, int BN, int BK, int WGM, int WGN, bool VEC>
__global__ __launch_bounds__(256) void k_tn(const T *__restrict__ A, int64_t lda,
                                            const T *__restrict__ B, int64_t ldb,
                                            T *__restrict__ P, int64_t ldp, int64_t rows,
                                            int Mi, int Nj, int64_t chunk, T alpha, T beta) {
  typedef Mfma<T> MF;
  constexpr int MB = MF::MB, KB = MF::KB;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / MB, TN = WN / MB;
  constexpr int VW = VEC ? Vec16<T>::W : 1;
  constexpr int AV = BM * BK / VW / 256, BV = BN * BK / VW / 256;
  static_assert(WGM * WGN == 4, "4 waves");
  static_assert(AV * VW * 256 == BM * BK && BV * VW * 256 == BN * BK, "tile/threads");

  // FP32: k-rows padded by 16 floats, so the 4 k-rows of a fragment read
  // start on different banks
  constexpr int PA = BM + (sizeof(T) == 4 ? 16 : 0), PB = BN + (sizeof(T) == 4 ? 16 : 0);
  __shared__ T As[2][BK * PA];
  __shared__ T Bs[2][BK * PB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;
  int bx, by, bz;
  xcd_map(bx, by, bz);
  const int j0 = bx * BN, i0 = by * BM;
  const int64_t rbeg = (int64_t)bz * chunk;
  const int64_t rend = rbeg + chunk < rows ? rbeg + chunk : rows;

  T ra[AV * VW], rb[BV * VW];
  auto load = [&](int64_t r0) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      int idx = tid + v * 256;
      int kr = idx / (BM / VW), c = (idx % (BM / VW)) * VW;
      int64_t gr = r0 + kr;
      if constexpr (VEC) {
        typename Vec16<T>::type x = {};
        if (gr < rend && i0 + c < Mi) x = *(const typename Vec16<T>::type *)(A + gr * lda + i0 + c);
#pragma unroll
        for (int e = 0; e < VW; ++e) ra[v * VW + e] = x[e];
      } else {
        ra[v] = (gr < rend && i0 + c < Mi) ? A[gr * lda + i0 + c] : (T)0;
      }
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      int idx = tid + v * 256;
      int kr = idx / (BN / VW), c = (idx % (BN / VW)) * VW;
      int64_t gr = r0 + kr;
      if constexpr (VEC) {
        typename Vec16<T>::type x = {};
        if (gr < rend && j0 + c < Nj) x = *(const typename Vec16<T>::type *)(B + gr * ldb + j0 + c);
#pragma unroll
        for (int e = 0; e < VW; ++e) rb[v * VW + e] = x[e];
      } else {
        rb[v] = (gr < rend && j0 + c < Nj) ? B[gr * ldb + j0 + c] : (T)0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      int idx = tid + v * 256;
      int kr = idx / (BM / VW), c = (idx % (BM / VW)) * VW;
#pragma unroll
      for (int e = 0; e < VW; ++e) As[buf][kr * PA + c + e] = ra[v * VW + e];
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      int idx = tid + v * 256;
      int kr = idx / (BN / VW), c = (idx % (BN / VW)) * VW;
#pragma unroll
      for (int e = 0; e < VW; ++e) Bs[buf][kr * PB + c + e] = rb[v * VW + e];
    }
  };

  typename MF::acc_t acc[TM][TN];
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
    for (int kk = 0; kk < BK; kk += KB) {
      T a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[cur][(kk + lane / MB) * PA + wm0 + i * MB + lane % MB];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[cur][(kk + lane / MB) * PB + wn0 + j * MB + lane % MB];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MF::op(a[i], b[j], acc[i][j]);
    }
    if (t + 1 < nt) store(cur ^ 1);
    __syncthreads();
  }

  T *Pz = P + (int64_t)bz * Mi * ldp;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < MF::NV; ++v) {
        int r = i0 + wm0 + i * MB + MF::row(lane, v);
        int c = j0 + wn0 + j * MB + lane % MB;
        if (r < Mi && c < Nj) {
          T val = alpha * acc[i][j][v];
          if (beta != (T)0) val += beta * Pz[(int64_t)r * ldp + c];
          Pz[(int64_t)r * ldp + c] = val;
        }
      }
}

// ---------------------------------------------------------------- launch --
template <typename T> static bool vec_ok(const void *p, int64_t ld, int64_t extent) {
  constexpr int W = Vec16<T>::W;
  return ((uintptr_t)p % 16 == 0) && (ld % W == 0) && (extent % W == 0);
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN, int R = 1>
static int nt_typed(const T *A, int64_t lda, const T *B, int64_t ldb, T *C, int64_t ldc,
                    int64_t M, int N, int K, T alpha, T beta, hipStream_t s) {
  const int64_t tiles = (M + BM - 1) / BM * ((N + BN - 1) / BN);
  dim3 grid((unsigned)tiles);
  if (tiles == 0) return LSPCA_OK;
  if (tiles > 0x7fffffff) {
    set_error("nt product: too many row tiles");
    return LSPCA_EINVAL;
  }
  if (vec_ok<T>(A, lda, K) && vec_ok<T>(B, ldb, K))
    hipLaunchKernelGGL((k_nt<T, BM, BN, BK, WGM, WGN, true, R>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, alpha, beta);
  else
    hipLaunchKernelGGL((k_nt<T, BM, BN, BK, WGM, WGN, false, R>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, alpha, beta);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

int launch_nt(lspca_dtype dt, const void *A, int64_t lda, const void *B, int64_t ldb,
              void *C, int64_t ldc, int64_t M, int N, int K, hipStream_t s, double alpha,
              double beta) {
  if (M <= 0 || N <= 0) return LSPCA_OK;
  switch (dt) {
    case LSPCA_F32:
      return nt_typed<float, 128, 128, LSPCA_NT32_BK, 2, 2, LSPCA_NT32_STAGES>(
          (const float *)A, lda, (const float *)B, ldb, (float *)C, ldc, M, N, K, (float)alpha,
          (float)beta, s);
    case LSPCA_F64:
      // narrow products with few 64-row tiles (a 20,000-row sketch with
      // k = 50: 313 tiles for 256 CUs) balance better with 32-row tiles (the
      // same 16 x 16 blocks and K order per output element)
      if (N <= 64 && (M + 63) / 64 < 512 && M > 4096)
        return nt_typed<double, 32, 64, 16, 2, 2>((const double *)A, lda, (const double *)B, ldb,
                                                  (double *)C, ldc, M, N, K, alpha, beta, s);
      return nt_typed<double, 64, 64, 16, 2, 2>((const double *)A, lda, (const double *)B, ldb,
                                                (double *)C, ldc, M, N, K, alpha, beta, s);
    default:
      set_error("nt product: dtype %d not handled here", (int)dt);
      return LSPCA_ENOTSUP;
  }
}

// Split count: enough blocks to fill 256 CUs several times over, at least
// 128 rows per split.
int tn_pick_splits(int64_t rows, int Mi, int Nj) {
  const int BM = 128, BN = 128;
  int64_t tiles = (int64_t)((Mi + BM - 1) / BM) * ((Nj + BN - 1) / BN);
  int64_t want = (2048 + tiles - 1) / tiles;
  int64_t maxs = (rows + 127) / 128;
  int64_t s = want < maxs ? want : maxs;
  // the partials (Mi Nj per split) written and reduced again stay within
  // 1/16 of the operands' bytes (rows (Mi + Nj)) once the launch has a
  // workgroup per CU: short and wide products (20,000 x 1,000 with k = 50)
  // otherwise move more partial bytes than they compute with
  const int64_t lean = std::max<int64_t>((256 + tiles - 1) / tiles,
                                         rows * (int64_t)(Mi + Nj) / (16 * (int64_t)Mi * Nj));
  if (s > lean) s = lean;
  if (s >= 8) s = s / 8 * 8;                 // multiple of 8 for the XCD map
  // accuracy contract: each FP32 partial sums at most kTnMaxDepth rows (the
  // launchers round the chunk up to a multiple of 64 at most, which keeps it
  // within 65,536); the partials are then added in FP64
  const int64_t deep = (rows + kTnMaxDepth - 1) / kTnMaxDepth;
  if (s < deep) s = (deep + 7) / 8 * 8;
  if (s < 1) s = 1;
  if (s > kTnMaxSplits) s = kTnMaxSplits;
  return (int)s;
}

size_t tn_partial_elems(int Mi, int Nj, int splits) {
  return (size_t)Mi * Nj * splits;
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN>
static int tn_typed(const T *A, int64_t lda, const T *B, int64_t ldb, T *P, int64_t ldp,
                    int64_t rows, int Mi, int Nj, int splits, T alpha, T beta, hipStream_t s) {
  int64_t chunk = (rows + splits - 1) / splits;
  chunk = (chunk + BK - 1) / BK * BK;
  dim3 grid((unsigned)((Nj + BN - 1) / BN), (unsigned)((Mi + BM - 1) / BM), (unsigned)splits);
  if (vec_ok<T>(A, lda, Mi) && vec_ok<T>(B, ldb, Nj))
    hipLaunchKernelGGL((k_tn<T, BM, BN, BK, WGM, WGN, true>), grid, dim3(256), 0, s, A, lda, B, ldb, P, ldp, rows, Mi, Nj, chunk, alpha, beta);
  else
    hipLaunchKernelGGL((k_tn<T, BM, BN, BK, WGM, WGN, false>), grid, dim3(256), 0, s, A, lda, B, ldb, P, ldp, rows, Mi, Nj, chunk, alpha, beta);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

int launch_tn(lspca_dtype dt, const void *A, int64_t lda, const void *B, int64_t ldb,
              void *P, int64_t rows, int Mi, int Nj, int splits, hipStream_t s, int64_t ldp,
              double alpha, double beta) {
  if (Mi <= 0 || Nj <= 0 || splits <= 0) return LSPCA_OK;
  if (ldp <= 0) ldp = Nj;
  if (splits > 1 && (ldp != Nj || beta != 0.0)) {
    set_error("tn product: ldp/beta need splits == 1");
    return LSPCA_EINVAL;
  }
  switch (dt) {
    case LSPCA_F32:
      return tn_typed<float, 128, 128, 16, 2, 2>((const float *)A, lda, (const float *)B, ldb,
                                                 (float *)P, ldp, rows, Mi, Nj, splits,
                                                 (float)alpha, (float)beta, s);
    case LSPCA_F64:
      return tn_typed<double, 64, 64, 16, 2, 2>((const double *)A, lda, (const double *)B, ldb,
                                                (double *)P, ldp, rows, Mi, Nj, splits, alpha,
                                                beta, s);
    default:
      set_error("tn product: dtype %d not handled here", (int)dt);
      return LSPCA_ENOTSUP;
  }
}

// ------------------------------------------------------------ TN32 stream --
// F = Y^T X in FP32 as k_tn (split over row chunks, one FP32 partial per
// split), with both operands copied straight into LDS (global_load_lds): a
// K tile of BK rows is BK rows of Y's BM columns and X's BN columns, row
// after row, through SX stages, one barrier per tile. A lane of 16-lane
// group g reads 4 consecutive columns of row kk + g of each tile (one 16-byte
// read) and feeds them to 4 v_mfma_f32_16x16x4f32, so MFMA row m of the e-th
// product is tile column 4 m + e: the wave's outputs are 4 x 4 interleaved
// 16 x 16 blocks, stored back as 16-byte pieces. Every output element gets
// the same chain as in k_tn (per 4 rows one MFMA, rows in order), so with
// the same chunks the two give the same bits. Fragments of the next 4 rows
// are read while the current products run. Rows past the chunk: the copies
// read clamped rows and the last tile's fragments are zeroed there. Needs
// 16-byte aligned rows, lda, ldb, Mi and Nj multiples of 4.
template <int BM, int BN, int WR, int WC, int BK, int SX>
__global__ __launch_bounds__(64 * WR * WC) void k_tn32s(const float *__restrict__ A, int64_t lda,
                                               const float *__restrict__ B, int64_t ldb,
                                               float *__restrict__ P, int64_t rows, int Mi, int Nj,
                                               int64_t chunk) {
  constexpr int NW = WR * WC;
  constexpr int WM = BM / WR, WN = BN / WC, TA = WM / 64, TB = WN / 64;
  constexpr int KS = BK / 4;                       // steps of 4 rows per K tile
  constexpr int ABYTES = BK * BM * 4, BBYTES = BK * BN * 4, STAGE = ABYTES + BBYTES;
  constexpr int AI = ABYTES / 1024, BI = BBYTES / 1024;
  static_assert(WM % 64 == 0 && WN % 64 == 0 && KS % 2 == 0, "tile shape");
  static_assert(AI % NW == 0 && BI % NW == 0, "copies split evenly over the waves");
  constexpr int AIW = AI / NW, BIW = BI / NW, LPW = AIW + BIW;
  static_assert((SX - 1) * LPW < 64 && SX >= 2, "copies in flight");
  constexpr int CA = BM / 4, CB = BN / 4;          // 16-byte chunks per tile row
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

  auto issue = [&](int sl, int64_t t) {
    const uint32_t st = lds0 + sl * STAGE;
    const int64_t r0 = rbeg + t * BK;
#pragma unroll
    for (int q = 0; q < AIW; ++q) {
      const int ins = wave + q * NW;
      const int c = ins * 64 + lane;
      const int r = c / CA, cc = c % CA;
      const int64_t gr = r0 + r < rows ? r0 + r : rows - 1;
      const int col = i0 + 4 * cc < Mi ? i0 + 4 * cc : Mi - 4;
      copy16_to_lds(A + gr * lda + col, st + ins * 1024);
    }
#pragma unroll
    for (int q = 0; q < BIW; ++q) {
      const int ins = wave + q * NW;
      const int c = ins * 64 + lane;
      const int r = c / CB, cc = c % CB;
      const int64_t gr = r0 + r < rows ? r0 + r : rows - 1;
      const int col = j0 + 4 * cc < Nj ? j0 + 4 * cc : Nj - 4;
      copy16_to_lds(B + gr * ldb + col, st + ABYTES + ins * 1024);
    }
  };

  f32x4 acc[TA * 4][TB * 4];
#pragma unroll
  for (int i = 0; i < TA * 4; ++i)
#pragma unroll
    for (int j = 0; j < TB * 4; ++j) acc[i][j] = {};

  const int fc = lane & 15, fg = lane >> 4;
  f32x4 fa[2][TA], fb[2][TB];
  auto load_frag = [&](int set, int sl, int kk) {
    const char *st = lds + sl * STAGE;
#pragma unroll
    for (int a = 0; a < TA; ++a)
      fa[set][a] = *(const f32x4 *)(st + (kk + fg) * (BM * 4) + (wm0 + 64 * a + 4 * fc) * 4);
#pragma unroll
    for (int b = 0; b < TB; ++b)
      fb[set][b] = *(const f32x4 *)(st + ABYTES + (kk + fg) * (BN * 4) + (wn0 + 64 * b + 4 * fc) * 4);
  };
  // TAIL: the chunk's last tile; this lane's row kk + fg zeroed in both
  // fragments when it is at or past the chunk's end
  auto mma = [&](int set, auto tailc, int kk, int64_t r0) {
    constexpr bool TAIL = decltype(tailc)::value;
    if constexpr (TAIL) {
      if (r0 + kk + fg >= rend) {
#pragma unroll
        for (int a = 0; a < TA; ++a) fa[set][a] = {};
#pragma unroll
        for (int b = 0; b < TB; ++b) fb[set][b] = {};
      }
    }
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
      for (int ea = 0; ea < 4; ++ea)
#pragma unroll
        for (int b = 0; b < TB; ++b)
#pragma unroll
          for (int eb = 0; eb < 4; ++eb)
            acc[4 * a + ea][4 * b + eb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                fa[set][a][ea], fb[set][b][eb], acc[4 * a + ea][4 * b + eb], 0, 0, 0);
  };
  auto tile = [&](int64_t t, auto tailc) {
    constexpr bool TAIL = decltype(tailc)::value;
    const int sl = (int)(t % SX);
    const int64_t r0 = rbeg + t * BK;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int cur = ks & 1;
      if (ks + 1 < KS) {
        load_frag(cur ^ 1, sl, 4 * (ks + 1));
      } else if constexpr (!TAIL) {
        wait_vmcnt<(SX - 2) * LPW>();              // tile t + 1 landed (this wave's copies)
        lds_barrier();                              // (every wave's); stage sl is free
        issue(sl, t + SX < nt ? t + SX : nt - 1);
        load_frag(cur ^ 1, (int)((t + 1) % SX), 0);
      }
      mma(cur, tailc, 4 * ks, r0);
    }
  };

  if (nt > 0) {
#pragma unroll
    for (int sl = 0; sl < SX; ++sl) issue(sl, sl < nt ? sl : nt - 1);
    wait_vmcnt<(SX - 1) * LPW>();
    lds_barrier();
    load_frag(0, 0, 0);
    for (int64_t t = 0; t + 1 < nt; ++t) tile(t, std::false_type{});
    tile(nt - 1, std::true_type{});
  }
  wait_vmcnt<0>();                                  // no copy may land after the workgroup ends

  // acc[4a + ea][4b + eb][v] of lane (fg, fc) is output row
  // wm0 + 64 a + 4 (4 fg + v) + ea, column wn0 + 64 b + 4 fc + eb: for fixed
  // (a, ea, b, v) the four eb are 4 consecutive columns
  float *Pz = P + (int64_t)bz * Mi * Nj;
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int ea = 0; ea < 4; ++ea)
#pragma unroll
      for (int b = 0; b < TB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = i0 + wm0 + 64 * a + 4 * (4 * fg + v) + ea;
          const int c = j0 + wn0 + 64 * b + 4 * fc;
          if (r < Mi && c < Nj) {
            const f32x4 w = {acc[4 * a + ea][4 * b][v], acc[4 * a + ea][4 * b + 1][v],
                             acc[4 * a + ea][4 * b + 2][v], acc[4 * a + ea][4 * b + 3][v]};
            *(f32x4 *)(Pz + (int64_t)r * Nj + c) = w;
          }
        }
}

template <int BM, int BN, int WR, int WC>
static int tn32s_launch(const float *A, int64_t lda, const float *B, int64_t ldb, float *P, int64_t rows, int Mi,
                        int Nj, int splits, hipStream_t s) {
  constexpr int BK = 32, STAGE = (BM + BN) * BK * 4;
  constexpr int SX = 147456 / STAGE > 4 ? 4 : 147456 / STAGE;
  // the chunks of k_tn (its K depth is 16), so the two give the same bits
  int64_t chunk = (rows + splits - 1) / splits;
  chunk = (chunk + 15) / 16 * 16;
  dim3 grid((unsigned)((Nj + BN - 1) / BN), (unsigned)((Mi + BM - 1) / BM), (unsigned)splits);
  hipLaunchKernelGGL((k_tn32s<BM, BN, WR, WC, BK, SX>), grid, dim3(64 * WR * WC), 0, s, A, lda, B, ldb, P, rows,
                     Mi, Nj, chunk);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// Environment switch of the streamed FP32 F: LSPCA_TN32_STREAM=0 keeps k_tn
// (same bits), read per call.
static bool tn32_stream_on() {
  const char *e = getenv("LSPCA_TN32_STREAM");
  return !(e && *e && atoi(e) == 0);
}

int launch_tn_factor(lspca_dtype dt, const void *A, int64_t lda, const void *B, int64_t ldb, void *P,
                     int64_t rows, int Mi, int Nj, int splits, hipStream_t s) {
  if (dt == LSPCA_F32 && Mi % 4 == 0 && Nj % 4 == 0 && lda % 4 == 0 && ldb % 4 == 0 && (uintptr_t)A % 16 == 0 &&
      (uintptr_t)B % 16 == 0 && Mi > 0 && Nj > 0 && splits > 0 && tn32_stream_on()) {
    if (Mi > 128)
      return tn32s_launch<256, 256, 4, 2>((const float *)A, lda, (const float *)B, ldb, (float *)P, rows, Mi, Nj,
                                          splits, s);
    return tn32s_launch<128, 256, 2, 4>((const float *)A, lda, (const float *)B, ldb, (float *)P, rows, Mi, Nj,
                                        splits, s);
  }
  return launch_tn(dt, A, lda, B, ldb, P, rows, Mi, Nj, splits, s);
}

// ------------------------------------------------------ batched projection --
// Persistent: workgroup b takes tiles b, b + grid, ... of the table (passed
// by value in the kernel arguments); the request of a tile is found by
// binary search over the tiles' first numbers.
template <typename T, int BM, int BN, bool VEC>
__global__ __launch_bounds__(256) void k_proj_batch(const ProjTable tab,
                                                    const T *__restrict__ VT, int64_t ldv, int N, int K) {
  const int ntiles = tab.ntiles, nreq = tab.nreq, ntn = tab.ntn;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab.req[mid].tile0 <= t) lo = mid;
      else hi = mid - 1;
    }
    const ProjReq &rq = tab.req[lo];
    const int local = t - rq.tile0, mt = local / ntn;
    nt_tile<T, BM, BN, 16, 2, 2, VEC>((const T *)rq.X, rq.ldx, VT, ldv, (T *)rq.Z, rq.ldz, rq.rows, N, K,
                                      (T)1, (T)0, (int64_t)mt * BM, (local - mt * ntn) * BN);
  }
}

static const void *projf_kernel(lspca_dtype dt, bool vec) {
  if (dt == LSPCA_F64)
    return vec ? (const void *)&k_proj_batch<double, 64, 64, true> : (const void *)&k_proj_batch<double, 64, 64, false>;
  return vec ? (const void *)&k_proj_batch<float, 128, 128, true> : (const void *)&k_proj_batch<float, 128, 128, false>;
}

int proj16_grid(lspca_dtype dt, int k, bool vec, int *grid);
int launch_proj_batch16(lspca_dtype dt, const ProjTable *tab, const void *VTh, const void *VTl, int64_t ldv,
                        int k, int n, bool vec, int grid, hipStream_t s);

void proj_tile_shape(lspca_dtype dt, int k, int *BM, int *BN) {
  switch (dt) {
    case LSPCA_F64: *BM = 64; *BN = 64; break;
    case LSPCA_F32: *BM = 128; *BN = 128; break;
    default: *BM = 128; *BN = k > 128 ? 256 : 128; break;
  }
}

int proj_batch_grid(lspca_dtype dt, int k, bool vec, int *grid) {
  if (dt == LSPCA_BF16 || dt == LSPCA_F16) return proj16_grid(dt, k, vec, grid);
  int dev = 0, cus = 0, per = 0;
  LSPCA_HIP(hipGetDevice(&dev));
  LSPCA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  LSPCA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, projf_kernel(dt, vec), 256, 0));
  *grid = cus * (per > 0 ? per : 1);
  return LSPCA_OK;
}

int launch_proj_batch(lspca_dtype dt, const ProjTable *tab, const void *VTh, const void *VTl, int64_t ldv,
                      int k, int n, bool vec, int grid, hipStream_t s) {
  if (dt == LSPCA_BF16 || dt == LSPCA_F16) return launch_proj_batch16(dt, tab, VTh, VTl, ldv, k, n, vec, grid, s);
  void *args[] = {(void *)tab, (void *)&VTh, (void *)&ldv, (void *)&k, (void *)&n};
  LSPCA_HIP(hipLaunchKernel(projf_kernel(dt, vec), dim3(grid), dim3(256), args, 0, s));
  return LSPCA_OK;
}

}  // namespace lspca
