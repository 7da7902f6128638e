// Small FP64 stage: the truncated SVD of the k x n factor F (final step of
// Algorithms 2 and 4), plus the k x k route to Sigma^s, all on the GPU.
//
// Route (own design; the paper only asks for a truncated SVD of F, or its
// eigensolution route via F F^T in the note of the algorithm table):
//   1. F^T = Q R by Cholesky QR on the n x k matrix F^T, repeated until Q is
//      orthonormal to working precision (two passes; a shifted first pass is
//      added when the first Cholesky factorisation fails).
//   2. One-sided (Hestenes) Jacobi on the k x k factor R: R W = U_R Sigma.
//      Then F = R^T Q^T = W Sigma (Q U_R)^T, so V = Q U_R and D = Sigma.
//      The subspace span(V) = span(Q) = span(F^T) is fixed by step 1 alone,
//      and the rotations of step 2 keep V orthonormal to rounding.
//   3. sigma_x: with G = R_G^T R_G (Cholesky), R_G^-T F = (R R_G^-1)^T Q^T,
//      so Sigma^s are the singular values of the k x k matrix R R_G^-1 (the
//      Q^T X of eq. (approx_svd) without a tall QR).
#include "common.h"

#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace lspca {

// 16-lane all-reduce of a double with DPP moves inside one row of a wave:
// quad_perm xor 1, quad_perm xor 2, row_half_mirror, row_mirror.
typedef int i32x2 __attribute__((ext_vector_type(2)));
template <int CTRL> __device__ inline double dpp_move(double v) {
  i32x2 p = __builtin_bit_cast(i32x2, v);
  p.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xF, 0xF, false);
  p.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, p);
}
__device__ inline double sum16(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return v;
}

// 8-lane all-reduce inside a DPP row (quad xor 1, quad xor 2, half mirror).
__device__ inline double sum8(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  return v;
}


// ----------------------------------------------------------- reductions ----
template <typename PT>
__global__ void k_reduce_add(const PT *__restrict__ P, int splits, int64_t count,
                             double *__restrict__ out, int accumulate,
                             const double *__restrict__ rowscale, int ncols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double s = accumulate ? out[e] : 0.0;
  double part = 0.0;
  for (int z = 0; z < splits; ++z) part += (double)P[(int64_t)z * count + e];
  if (rowscale) part *= rowscale[e / ncols];
  out[e] = s + part;
}

int launch_reduce_add(lspca_dtype pdt, const void *P, int splits, int64_t count, double *out,
                      int accumulate, hipStream_t s, const double *rowscale, int ncols) {
  if (count <= 0) return LSPCA_OK;
  const unsigned grid = (unsigned)((count + 255) / 256);
  if (pdt == LSPCA_F64)
    hipLaunchKernelGGL(k_reduce_add<double>, grid, 256, 0, s, (const double *)P, splits, count, out, accumulate, rowscale, ncols);
  else
    hipLaunchKernelGGL(k_reduce_add<float>, grid, 256, 0, s, (const float *)P, splits, count, out, accumulate, rowscale, ncols);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

__global__ void k_transpose_f64(const double *__restrict__ src, int64_t rows, int cols,
                                double *__restrict__ dst) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32;
  const int c0 = blockIdx.x * 32;
  for (int i = threadIdx.y; i < 32; i += 8) {
    int64_t r = r0 + i;
    int c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[i][threadIdx.x] = src[r * cols + c];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    int c = c0 + i;
    int64_t r = r0 + threadIdx.x;
    if (r < rows && c < cols) dst[(int64_t)c * rows + r] = tile[threadIdx.x][i];
  }
}

int launch_transpose_f64(const double *src, int64_t rows, int cols, double *dst, hipStream_t s) {
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(k_transpose_f64, grid, dim3(32, 8), 0, s, src, rows, cols, dst);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// ------------------------------------------------------- k x k kernels -----
// Add shift * I to the k x k matrix M, where shift = c * trace(M).
__global__ void k_shift_diag(double *M, int k, double c) {
  __shared__ double tr;
  if (threadIdx.x == 0) {
    double t = 0;
    for (int i = 0; i < k; ++i) t += M[(int64_t)i * k + i];
    tr = t;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += blockDim.x) M[(int64_t)i * k + i] += c * tr;
}

// Cholesky factor (upper triangular R, M = R^T R) of an n x n block (n <=
// 128) in LDS, right-looking on the upper triangle with the pivot row kept
// unscaled: every thread reads the pivot d_j itself and subtracts
// M[j][a] M[j][b] / d_j from the trailing entries (j < a <= b), one barrier
// per step; rows are scaled by 1/sqrt(d_j) when R is written. A pivot that
// is not positive and finite sets fail[0] (the same value is seen by all
// threads, so they leave the loop together).
__global__ __launch_bounds__(1024) void k_chol_lds(double *Mg, int n, int64_t ld, int *fail) {
  __shared__ double M[128 * 129];
  const int tid = threadIdx.x, nt = blockDim.x, s = n + 1;
  const int tx = tid & 31, ty = tid >> 5;
  for (int e = tid; e < n * n; e += nt) M[(e / n) * s + e % n] = Mg[(int64_t)(e / n) * ld + e % n];
  __syncthreads();
  bool bad = false;
  for (int j = 0; j < n; ++j) {
    const double d = M[j * s + j];
    if (!(d > 0.0) || !isfinite(d)) {
      bad = true;
      break;
    }
    const double inv = 1.0 / d;
    for (int a = j + 1 + ty; a < n; a += 32) {
      const double ra = M[j * s + a] * inv;
      for (int b = a + tx; b < n; b += 32) M[a * s + b] -= ra * M[j * s + b];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) fail[0] = 1;
    return;
  }
  for (int e = tid; e < n * n; e += nt) {
    const int a = e / n, b = e % n;
    double v = 0.0;
    if (b >= a) {
      const double r = sqrt(M[a * s + a]);
      v = b == a ? r : M[a * s + b] / r;
    }
    Mg[(int64_t)a * ld + b] = v;
  }
}

// Inverse X = R^-1 of an upper triangular n x n block (n <= 128) in LDS,
// column by column: X[j][j] = 1/R[j][j] and, for i < j,
// X[i][j] = -(sum_{p=i}^{j-1} X[i][p] R[p][j]) / R[j][j], 8 lanes per
// row i. Writes XT[c][i] = X[i][c] (ld ldxt) and, if X != NULL, X itself
// (ld ldx).
__device__ void trinv_block(const double *R, int n, int64_t ldr, double *XT, int64_t ldxt, double *X,
                            int64_t ldx) {
  __shared__ double A[128 * 129];
  const int tid = threadIdx.x, nt = blockDim.x, s = n + 1;
  const int i = tid >> 3, sub = tid & 7;
  for (int e = tid; e < n * n; e += nt) {
    const int a = e / n, b = e % n;
    A[a * s + b] = b < a ? 0.0 : R[(int64_t)a * ldr + b];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double d = 1.0 / A[j * s + j];
    double t = 0.0;
    if (i < j)
      for (int p = i + sub; p < j; p += 8) t += A[i * s + p] * A[p * s + j];
    t = sum8(t);
    __syncthreads();
    if (i < j && sub == 0) A[i * s + j] = -t * d;
    if (tid == 0) A[j * s + j] = d;
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += nt) {
    const int a = e / n, b = e % n;
    XT[(int64_t)b * ldxt + a] = A[a * s + b];
    if (X) X[(int64_t)a * ldx + b] = A[a * s + b];
  }
}

__global__ __launch_bounds__(1024) void k_trinv_lds(const double *R, int n, int64_t ldr, double *XT,
                                                    int64_t ldxt, double *X, int64_t ldx) {
  trinv_block(R, n, ldr, XT, ldxt, X, ldx);
}

// The diagonal 128-blocks of XT = (R^-1)^T (R k x k), one workgroup each:
// they are independent, so all of them in one launch.
__global__ __launch_bounds__(1024) void k_trinv_blocks(const double *R, int k, double *XT) {
  const int j0 = blockIdx.x * 128, jb = k - j0 < 128 ? k - j0 : 128;
  trinv_block(R + (int64_t)j0 * k + j0, jb, k, XT + (int64_t)j0 * k + j0, k, nullptr, 0);
}

__global__ void k_zero_lower(double *M, int k) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * k) return;
  if (e % k < e / k) M[e] = 0.0;
}

// Copy the k x k row-major matrix A into column storage Wc[c][i] = A[i][c].
__global__ void k_to_cols(const double *__restrict__ A, int k, double *__restrict__ Wc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * k) return;
  const int i = (int)(e / k), c = (int)(e % k);
  Wc[(int64_t)c * k + i] = A[e];
}



// ------------------------------------------------ one-sided Jacobi ------
// Columns live in LDS with a padded stride (len + 1 doubles) so that the
// groups of one wave, each reading a different column, hit different banks.
constexpr int kLdsAlloc = 16640;     // allocation incl. padding (130 KB)
// Block Jacobi: 2b columns of stride jacobi_ld(k) in LDS (136 KB). Up to
// k = 256 (16 lanes per column, 128 bytes per lane group) the stride is k
// rounded up to 16 mod 32 doubles, so the columns of a wave's four lane
// groups (consecutive columns) alternate between the two halves of the 64
// banks (8% faster at k = 256 than stride k + 1); beyond, one group of 32
// or 64 lanes spans all banks and the stride is k + 1.
constexpr int kBlockLdsAlloc = 17408;
__host__ __device__ inline int jacobi_ld(int k) { return k <= 256 ? k + ((16 - k) & 31) : k + 1; }
constexpr int kJacobiMaxSweeps = 40;
// dflag slots of small_factor: non-convergence flags of its two Jacobi runs
// (the SVD of F, then Sigma^s), clear of the sweep counters at dflag + 8
// and dflag + 64 (kJacobiMaxSweeps + 1 ints each).
constexpr int kNoConv = 120;
// dflag slots of small_factor's final status: an int, a spare int, then two
// doubles (D_k, D_1) at an 8-byte aligned offset.
constexpr int kStatus = 122;
// dflag slot of the skip flag of the speculative attempt; kRedo: the
// attempt's internal result asking for the run with host decisions.
constexpr int kSkip = 4;
constexpr int kRedo = 1;
// out[0] = any of a, b, c set; out[1..3] = a, b, c.
__global__ void k_any3(const int *a, const int *b, const int *c, int *out) {
  out[1] = *a;
  out[2] = *b;
  out[3] = *c;
  out[0] = (*a | *b | *c) != 0;
}
namespace cg = cooperative_groups;

// Sum over G lanes (16: one DPP row; 32, 64: rows combined by lane
// exchanges). Every lane receives the same bits (each step adds the same
// two values in either order).
template <int G> __device__ inline double sum_lanes(double v) {
  v = sum16(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16);
  if constexpr (G >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Rotation of a column pair from its Gram entries al = |a_p|^2,
// be = |a_q|^2, ga = a_p.a_q: false (no rotation) when |ga| <= tol |a_p|
// |a_q|; otherwise Rutishauser's formulas give c, s with
// (c a_p - s a_q).(s a_p + c a_q) = 0, and t = s / c, with the square roots
// and reciprocals from the hardware estimates and one Newton step each
// (relative error a few ulps; c^2 + s^2 = 1 to a few ulps, which is what
// keeps the rotation orthogonal).
__device__ inline double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ inline double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ inline bool jacobi_cst(double al, double be, double ga, double tol, double &c, double &sn,
                                  double &t) {
  if (!(ga != 0.0 && ga * ga > (tol * tol) * (al * be))) return false;
  const double d = be - al, h2 = fma(d, d, 4.0 * ga * ga);
  const double h = h2 * rsqrt_nr(h2);                         // sqrt(d^2 + 4 ga^2) > 0
  t = (d >= 0 ? 2.0 * ga : -2.0 * ga) * rcp_nr(fabs(d) + h);
  c = rsqrt_nr(fma(t, t, 1.0));
  sn = c * t;
  return true;
}

// G lanes per pair (rows gl + G i) with the squared norms kept in LDS (np,
// nq): only ga = a_p.a_q is summed over lanes, and the norms are updated with
// the identities |c a_p - s a_q|^2 = al - t ga, |s a_p + c a_q|^2 = be + t ga
// (t = s / c, which makes the new pair orthogonal); lane 0 of the group
// writes them. The caller recomputes the norms from the columns whenever it
// loads them. ROWS = 0: any length, two passes over LDS. Returns 0 (no
// rotation), 1 (a rotation of a pair with |a_p.a_q| <= sqrt(big2) |a_p|
// |a_q|) or 3 (a rotation of a pair above that).
template <int G, int ROWS>
__device__ inline int rotate_nrm(double *ap, double *aq, double *np, double *nq, int len, int gl,
                                 double tol, double big2) {
  const double al = *np, be = *nq;
  double c, sn, t, ga = 0;
  double x[ROWS > 0 ? ROWS : 1], y[ROWS > 0 ? ROWS : 1];
  if constexpr (ROWS > 0) {
    double gb = 0;                                  // two chains of fmas
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = gl + G * i;
      x[i] = r < len ? ap[r] : 0.0;
      y[i] = r < len ? aq[r] : 0.0;
      if (i & 1) gb = fma(x[i], y[i], gb);
      else ga = fma(x[i], y[i], ga);
    }
    ga += gb;
  } else {
    for (int r = gl; r < len; r += G) ga = fma(ap[r], aq[r], ga);
  }
  ga = sum_lanes<G>(ga);
  if (!jacobi_cst(al, be, ga, tol, c, sn, t)) return 0;
  const int code = ga * ga > big2 * (al * be) ? 3 : 1;
  if constexpr (ROWS > 0) {
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = gl + G * i;
      if (r < len) {
        ap[r] = c * x[i] - sn * y[i];
        aq[r] = sn * x[i] + c * y[i];
      }
    }
  } else {
    for (int r = gl; r < len; r += G) {
      const double xv = ap[r], yv = aq[r];
      ap[r] = c * xv - sn * yv;
      aq[r] = sn * xv + c * yv;
    }
  }
  if (gl == 0) {
    *np = fmax(fma(-t, ga, al), 0.0);
    *nq = fma(t, ga, be);
  }
  return code;
}

// Round-robin pair (i-th of round s) over nc' = even(nc) columns:
// column L = nc'-1 meets s, (s+i) mod L meets (s-i) mod L.
__device__ inline void rr_pair(int s, int i, int L, int &p, int &q) {
  if (i == 0) {
    p = s;
    q = L;
  } else {           // s, i < L: both sums lie in [0, 2L)
    p = s + i;
    p -= p >= L ? L : 0;
    q = s - i + L;
    q -= q >= L ? L : 0;
  }
}

__device__ inline int rotate_nrm_any(double *ap, double *aq, double *np, double *nq, int len, int gl,
                                     double tol, double big2) {
  if (len <= 32) return rotate_nrm<16, 2>(ap, aq, np, nq, len, gl, tol, big2);
  if (len <= 64) return rotate_nrm<16, 4>(ap, aq, np, nq, len, gl, tol, big2);
  if (len <= 128) return rotate_nrm<16, 8>(ap, aq, np, nq, len, gl, tol, big2);
  return rotate_nrm<16, 0>(ap, aq, np, nq, len, gl, tol, big2);
}

// One cyclic sweep over all pairs of the nc columns in LDS (column c at
// cols + c * ld, squared norm nrm[c]). Every pair of a round runs at once,
// 16 lanes per pair, with the norms updated by the rotation identities (as
// the block kernel). Adds the number of rotations to counter[0] and sets
// counter[1] when a rotated pair was above sqrt(big2) (rotate_nrm).
__device__ void lds_sweep_all(double *cols, double *nrm, int nc, int len, int ld, double tol, double big2,
                              int *counter) {
  const int ncp = (nc + 1) & ~1, L = ncp - 1, npairs = ncp / 2;
  const int g = threadIdx.x >> 4, gl = threadIdx.x & 15, ng = blockDim.x >> 4;
  int rot = 0, big = 0;
  for (int s = 0; s < L; ++s) {
    for (int i = g; i < npairs; i += ng) {
      int p, q;
      rr_pair(s, i, L, p, q);
      if (p < nc && q < nc) {
        const int a = min(p, q), b = max(p, q);
        const int r = rotate_nrm_any(cols + (int64_t)a * ld, cols + (int64_t)b * ld, nrm + a, nrm + b, len, gl,
                                     tol, big2);
        rot += r & 1;
        big |= r >> 1;
      }
    }
    __syncthreads();
  }
  if (gl == 0 && rot) atomicAdd(counter, rot);
  if (gl == 0 && big) atomicOr(counter + 1, 1);
}

// Whole k x k problem in one workgroup (k (k + 1) <= kLdsAlloc): Wc (column
// storage, global) is loaded into LDS, swept to convergence, written back.
__global__ __launch_bounds__(1024) void k_jacobi_lds(double *Wc, int k, double tol, double big2,
                                                     int max_sweeps, int *sweeps_out, int *noconv,
                                                     const int *skip) {
  if (skip && *skip) return;                        // a speculative run that is redone
  __shared__ double cols[kLdsAlloc];
  __shared__ double nrm[128];
  __shared__ int counter[2];
  const int ld = k + 1;
  const int64_t kk = (int64_t)k * k;
  const int g = threadIdx.x >> 4, gl = threadIdx.x & 15, ng = blockDim.x >> 4;
  for (int64_t e = threadIdx.x; e < kk; e += blockDim.x) cols[(e / k) * ld + e % k] = Wc[e];
  int sweep = 0;
  bool conv = false;
  for (; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) counter[0] = counter[1] = 0;
    __syncthreads();
    // squared column norms from the columns themselves at every sweep (the
    // rotation identities then carry them through the sweep)
    for (int c = g; c < k; c += ng) {
      double v = 0.0;
      for (int r = gl; r < k; r += 16) v = fma(cols[c * ld + r], cols[c * ld + r], v);
      v = sum_lanes<16>(v);
      if (gl == 0) nrm[c] = v;
    }
    __syncthreads();
    lds_sweep_all(cols, nrm, k, k, ld, tol, big2, counter);
    __syncthreads();
    const int n = counter[0], nbig = counter[1];
    __syncthreads();
    if (n == 0 || nbig == 0) {                      // converged (the next sweep would not rotate)
      sweep += n != 0;
      conv = true;
      break;
    }
  }
  for (int64_t e = threadIdx.x; e < kk; e += blockDim.x) Wc[e] = cols[(e / k) * ld + e % k];
  if (threadIdx.x == 0 && sweeps_out) *sweeps_out = sweep;
  // every sweep up to the limit still rotated: not converged
  if (threadIdx.x == 0 && !conv) *noconv = 1;
}

// Block one-sided Jacobi step for k too large for one workgroup: the k
// columns form nb (even) blocks of b; in outer round `round` the blocks pair
// up in round-robin order and workgroup w takes pair (I, J), loads its
// columns into LDS and rotates every pair (p in I, q in J) once (b rounds
// of b disjoint pairs: p = i, q = (i + s) mod b). In round 0 it first
// rotates the pairs inside I and inside J, so one outer sweep (nb - 1
// rounds) visits every column pair exactly once. Rotations set flag[0].
// One outer round for workgroup `wg` (G lanes per column or column pair, b
// groups): returns (in every thread) the number of rotations it made, plus
// kBigBit if a rotated pair was above sqrt(big2) (rotate_nrm). cols: LDS for
// 2b columns of stride jacobi_ld(k); nrm: their squared norms; counter: two
// LDS ints.
constexpr int kBigBit = 1 << 30;
template <int G, int ROWS>
__device__ int jacobi_block_round(double *Wc, int k, int b, int nb, int round, int wg, double tol,
                                  double big2, double *cols, double *nrm, int *counter) {
  const int L = nb - 1, ld = jacobi_ld(k);
  int I, J;
  rr_pair(round, wg, L, I, J);
  const int i0 = I * b, j0 = J * b;
  const int ni = max(0, min(k, i0 + b) - i0), nj = max(0, min(k, j0 + b) - j0);
  const int nc = ni + nj;
  // one group per column: load it (contiguous) and its squared norm; then
  // one group per column pair
  const int g = threadIdx.x / G, gl = threadIdx.x % G, ng = blockDim.x / G;
  if (threadIdx.x == 0) counter[0] = counter[1] = 0;
  for (int c = g; c < nc; c += ng) {
    const double *src = Wc + (int64_t)(c < ni ? i0 + c : j0 + (c - ni)) * k;
    double v = 0;
    if constexpr (ROWS > 0) {
      double x[ROWS];                               // all loads in flight at once
#pragma unroll
      for (int i = 0; i < ROWS; ++i) x[i] = gl + G * i < k ? src[gl + G * i] : 0.0;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        if (gl + G * i < k) cols[c * ld + gl + G * i] = x[i];
        v = fma(x[i], x[i], v);
      }
    } else {
      for (int r = gl; r < k; r += G) {
        const double x = src[r];
        cols[c * ld + r] = x;
        v = fma(x, x, v);
      }
    }
    v = sum_lanes<G>(v);
    if (gl == 0) nrm[c] = v;
  }
  __syncthreads();
  int rot = 0, big = 0;
  if (round == 0) {
    // pairs inside I and inside J: two interleaved round-robins
    const int bp = (max(ni, nj) + 1) & ~1, Lb = bp - 1, half = bp / 2;
    for (int s = 0; s < Lb; ++s) {
      for (int x = g; x < 2 * half; x += ng) {
        const int side = x >= half, i = x - (side ? half : 0);
        const int nside = side ? nj : ni, base = side ? ni : 0;
        int p, q;
        rr_pair(s, i, Lb, p, q);
        if (p < nside && q < nside) {
          const int a = base + min(p, q), bq = base + max(p, q);
          const int r = rotate_nrm<G, ROWS>(cols + a * ld, cols + bq * ld, nrm + a, nrm + bq, k, gl, tol, big2);
          rot += r & 1;
          big |= r >> 1;
        }
      }
      __syncthreads();
    }
  }
  const int bb = max(ni, nj);
  for (int s = 0; s < bb; ++s) {
    for (int i = g; i < bb; i += ng) {
      const int j = i + s - (i + s >= bb ? bb : 0);
      if (i < ni && j < nj) {
        const int r = rotate_nrm<G, ROWS>(cols + i * ld, cols + (ni + j) * ld, nrm + i, nrm + ni + j, k, gl, tol,
                                          big2);
        rot += r & 1;
        big |= r >> 1;
      }
    }
    __syncthreads();
  }
  for (int c = g; c < nc; c += ng) {
    double *dst = Wc + (int64_t)(c < ni ? i0 + c : j0 + (c - ni)) * k;
    for (int r = gl; r < k; r += G) dst[r] = cols[c * ld + r];
  }
  if (gl == 0 && rot) atomicAdd(counter, rot);
  if (gl == 0 && big) atomicOr(counter + 1, 1);
  __syncthreads();
  return counter[0] | (counter[1] ? kBigBit : 0);
}

// flag[0]: bit 0 set by a rotation, bit 1 by a rotation above sqrt(big2).
template <int G, int ROWS>
__global__ __launch_bounds__(1024) void k_jacobi_block(double *Wc, int k, int b, int nb, int round,
                                                       double tol, double big2, int *flag, const int *skip) {
  if (skip && *skip) return;
  __shared__ double cols[kBlockLdsAlloc];
  __shared__ double nrm[64];
  __shared__ int counter[2];
  const int n = jacobi_block_round<G, ROWS>(Wc, k, b, nb, round, blockIdx.x, tol, big2, cols, nrm, counter);
  if (threadIdx.x == 0 && n) atomicOr(flag, (n & kBigBit) ? 3 : 1);
}

// All sweeps in one cooperative launch (every workgroup resident): outer
// rounds separated by grid barriers (device-scope release and acquire, so
// the columns stored in one round are seen by the next round's loads).
// counts[sweep] (zeroed by the caller) sums the sweep's rotations, with
// kBigBit set by a rotation above sqrt(big2); every workgroup reads it after
// the sweep's last barrier, so all stop together.
template <int G, int ROWS>
__global__ __launch_bounds__(1024) void k_jacobi_coop(double *Wc, int k, int b, int nb, double tol,
                                                      double big2, int max_sweeps, int *counts,
                                                      int *sweeps_out, int *noconv, const int *skip) {
  if (skip && *skip) return;                        // every workgroup, before any grid barrier
  __shared__ double cols[kBlockLdsAlloc];
  __shared__ double nrm[64];
  __shared__ int counter[2], total;
  cg::grid_group grid = cg::this_grid();
  int sweep = 0;
  bool conv = false;
  while (sweep < max_sweeps) {
    for (int round = 0; round < nb - 1; ++round) {
      const int n = jacobi_block_round<G, ROWS>(Wc, k, b, nb, round, blockIdx.x, tol, big2, cols, nrm, counter);
      if (threadIdx.x == 0 && (n & ~kBigBit)) atomicAdd(counts + sweep, n & ~kBigBit);
      if (threadIdx.x == 0 && (n & kBigBit)) atomicOr(counts + sweep, kBigBit);
      __threadfence();
      grid.sync();
    }
    if (threadIdx.x == 0) total = atomicAdd(counts + sweep, 0);
    __syncthreads();
    ++sweep;
    // converged: no rotation, or none above sqrt(big2) (the next sweep
    // would not rotate)
    if ((total & ~kBigBit) == 0 || !(total & kBigBit)) {
      conv = true;
      break;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *sweeps_out = sweep;
    if (!conv) *noconv = 1;                  // the last sweep allowed still rotated
  }
}

// Column norms sigma_c = |Wc[c]|, ranks by decreasing sigma (ties: lower c
// first), and the sorted, normalised columns written as rows of UT:
// UT[pos][i] = Wc[c][i] / sigma_c (so UT = U_R^T with sorted columns).
// UT may be NULL (values only).
__global__ __launch_bounds__(1024) void k_jacobi_finish(const double *Wc, int k, double *UT,
                                                        double *sigma) {
  extern __shared__ double sm[];  // 2k doubles: norms, then positions
  double *nrm = sm;
  int *pos = (int *)(sm + k);
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double s = 0;
    for (int i = 0; i < k; ++i) {
      const double x = Wc[(int64_t)c * k + i];
      s += x * x;
    }
    nrm[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    int r = 0;
    for (int d = 0; d < k; ++d) r += (nrm[d] > nrm[c]) || (nrm[d] == nrm[c] && d < c);
    pos[c] = r;
    sigma[r] = nrm[c];
  }
  __syncthreads();
  if (UT) {
    for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += blockDim.x) {
      const int c = (int)(e / k), i = (int)(e % k);
      const double s = nrm[c];
      UT[(int64_t)pos[c] * k + i] = s > 0 ? Wc[e] / s : 0.0;
    }
  }
}

// Sign convention: the largest-magnitude entry of each column of V (n x k)
// is made positive; the lowest row index wins ties. One block per column.
__global__ void k_sqrt_vec(double *v, int k) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) v[i] = sqrt(v[i]);
}

// V[r][c] /= d[c] (V n x k row-major)
__global__ void k_scale_cols_inv(double *V, int64_t n, int k, const double *d) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * k) V[e] /= d[e % k];
}

// Sign of each column of V (n x k): its entry of largest magnitude made
// positive, the first row on ties. Column maxima per chunk of kSignRows rows
// (threads over columns, coalesced, eight independent loads in flight), then
// across chunks by one workgroup per column (a tree over the chunks with the
// same tie rule), then the flip.
constexpr int kSignRows = 32;
__global__ __launch_bounds__(256) void k_colmax_part(const double *__restrict__ V, int64_t n, int k,
                                                     double *__restrict__ pv, int64_t *__restrict__ pi) {
  const int64_t r0 = (int64_t)blockIdx.x * kSignRows;
  const int64_t r1 = r0 + kSignRows < n ? r0 + kSignRows : n;
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double best = -1.0;
    int64_t bi = r0;
    for (int64_t i0 = r0; i0 < r1; i0 += 8) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = i0 + u < r1 ? fabs(V[(i0 + u) * k + c]) : -1.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (a[u] > best) {
          best = a[u];
          bi = i0 + u;
        }
    }
    pv[(int64_t)blockIdx.x * k + c] = best;
    pi[(int64_t)blockIdx.x * k + c] = bi;
  }
}

// (v, i) beats (w, j): larger magnitude, or equal and the earlier row.
__device__ inline bool colmax_beats(double v, int64_t i, double w, int64_t j) {
  return v > w || (v == w && i < j);
}

// One workgroup of 256 threads per column c.
__global__ __launch_bounds__(256) void k_colmax_sign(const double *__restrict__ V, const double *__restrict__ pv,
                                                     const int64_t *__restrict__ pi, int64_t chunks, int k,
                                                     double *__restrict__ sgn) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t b = t; b < chunks; b += 256) {
    const double v = pv[b * k + c];
    const int64_t i = pi[b * k + c];
    if (colmax_beats(v, i, best, bi)) {
      best = v;
      bi = i;
    }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w && colmax_beats(sv[t + w], si[t + w], sv[t], si[t])) {
      sv[t] = sv[t + w];
      si[t] = si[t + w];
    }
    __syncthreads();
  }
  if (t == 0) sgn[c] = V[si[0] * k + c] < 0.0 ? -1.0 : 1.0;
}

// The checks of the small stage and, when they pass, its outputs, in one
// launch (no host round trip between them): status = 5 if skip is set (the
// speculative plain attempt must be redone), else 1 if the Cholesky of G
// failed (gflag, when Sigma^s is asked), else 2 / 3 if the Jacobi of the SVD
// of F / of Sigma^s stopped at its sweep limit, else 4 if D_k <= thr D_1
// (rank deficient), else 0; then, only for 0, V = Vw with the column signs
// sgn applied, sigma = sw and sigma_x = sx. stat[0] receives the status and
// the doubles after stat[2] (8-byte aligned) D_k and D_1.
__global__ void k_commit(const double *__restrict__ Vw, const double *__restrict__ sgn, int64_t n, int k,
                         const double *__restrict__ sw, const double *__restrict__ sx, const int *__restrict__ skip,
                         const int *__restrict__ gflag,
                         const int *__restrict__ noconv, double thr, double *__restrict__ V,
                         double *__restrict__ sigma, double *__restrict__ sigma_x, int *__restrict__ stat) {
  const double dk = sw[k - 1], d1 = sw[0];
  int status = 0;
  if (skip && skip[0]) status = 5;
  else if (gflag && gflag[0]) status = 1;
  else if (noconv[0]) status = 2;
  else if (noconv[1]) status = 3;
  else if (!(dk > thr * d1)) status = 4;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) {
    stat[0] = status;
    double *dd = (double *)(stat + 2);
    dd[0] = dk;
    dd[1] = d1;
  }
  if (status) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = tid; e < n * k; e += stride) V[e] = sgn[e % k] < 0.0 ? -Vw[e] : Vw[e];
  for (int64_t e = tid; e < k; e += stride) {
    sigma[e] = sw[e];
    if (sigma_x) sigma_x[e] = sx[e];
  }
}

size_t sign_fix_bytes(int64_t n, int k) {
  const int64_t chunks = (n + kSignRows - 1) / kSignRows;
  return ws_bytes<double>((size_t)chunks * k) + ws_bytes<int64_t>((size_t)chunks * k) + ws_bytes<double>(k);
}

// Column signs of V (n x k): sgn[c] = -1 where the column's entry of largest
// magnitude is negative (the flip itself is applied by k_commit).
static int sign_of_cols(const double *V, int64_t n, int k, double **sgn_out, Workspace &ws, hipStream_t s) {
  const int64_t chunks = (n + kSignRows - 1) / kSignRows;
  double *pv = ws.take<double>((size_t)chunks * k);
  int64_t *pi = ws.take<int64_t>((size_t)chunks * k);
  double *sgn = ws.take<double>(k);
  hipLaunchKernelGGL(k_colmax_part, (unsigned)chunks, 256, 0, s, V, n, k, pv, pi);
  LSPCA_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_colmax_sign, (unsigned)k, 256, 0, s, V, pv, pi, chunks, k, sgn);
  LSPCA_HIP(hipGetLastError());
  *sgn_out = sgn;
  return LSPCA_OK;
}

// ------------------------------------------------------------- driver ------
__global__ void k_zero_i32(int *p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

int zero_i32(int *p, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i32, (count + 255) / 256, 256, 0, s, p, count);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

__global__ void k_set_i32(int *p, int v) { *p = v; }

static int set_i32(int *p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i32, 1, 1, 0, s, p, v);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

namespace {

// M (k x k) = A^T A for A (rows x k, row-major), FP64.
int gram(const double *A, int64_t rows, int k, double *M, double *part, int splits,
         hipStream_t s) {
  LSPCA_TRY(launch_tn(LSPCA_F64, A, k, A, k, part, rows, k, k, splits, s));
  return launch_reduce_add(LSPCA_F64, part, splits, (int64_t)k * k, M, 0, s);
}

constexpr int kBlk = 128;   // diagonal block size of the blocked k x k kernels

// Cholesky M = R^T R (k x k, symmetric, full storage), R left in the upper
// triangle. k <= 128: one LDS kernel. Larger k: right-looking blocked form
// with 128-blocks: R_JJ = chol(M_JJ); R_J,rest = R_JJ^-T M_J,rest;
// M_rest,rest -= R_J,rest^T R_J,rest. scratch: 2 * 128 * 128 doubles.
int chol(double *M, int k, int *dflag, double *scratch, hipStream_t s) {
  if (k <= kBlk) {
    hipLaunchKernelGGL(k_chol_lds, 1, 1024, 0, s, M, k, (int64_t)k, dflag);
    LSPCA_HIP(hipGetLastError());
    return LSPCA_OK;
  }
  double *XT = scratch;
  for (int j0 = 0; j0 < k; j0 += kBlk) {
    const int jb = std::min(kBlk, k - j0);
    double *Mjj = M + (int64_t)j0 * k + j0;
    hipLaunchKernelGGL(k_chol_lds, 1, 1024, 0, s, Mjj, jb, (int64_t)k, dflag);
    LSPCA_HIP(hipGetLastError());
    const int r0 = j0 + jb, rn = k - r0;
    if (rn <= 0) break;
    hipLaunchKernelGGL(k_trinv_lds, 1, 1024, 0, s, Mjj, jb, (int64_t)k, XT, (int64_t)jb, nullptr, (int64_t)0);
    LSPCA_HIP(hipGetLastError());
    // R_J,rest[r][c] = sum_p XT[r][p] M[r0+c][j0+p]  (M symmetric)
    LSPCA_TRY(launch_nt(LSPCA_F64, XT, jb, M + (int64_t)r0 * k + j0, k, M + (int64_t)j0 * k + r0, k,
                        jb, rn, jb, s));
    // M_rest,rest -= R_J,rest^T R_J,rest
    LSPCA_TRY(launch_tn(LSPCA_F64, M + (int64_t)j0 * k + r0, k, M + (int64_t)j0 * k + r0, k,
                        M + (int64_t)r0 * k + r0, jb, rn, rn, 1, s, k, -1.0, 1.0));
  }
  hipLaunchKernelGGL(k_zero_lower, (unsigned)(((int64_t)k * k + 255) / 256), 256, 0, s, M, k);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// XT = (R^-1)^T for upper triangular R (k x k). k <= 128: one LDS kernel.
// Larger k: the diagonal blocks XT_JJ in LDS (one launch for all), then for
// each block column J and I < J, XT_JI = -XT_JJ S^T with
// S^T = sum_{P=I}^{J-1} XT_PI^T R_PJ (two products). scratch: 128 * 128
// doubles (at least).
int trinv_t(const double *R, int k, double *XT, double *scratch, hipStream_t s) {
  if (k <= kBlk) {
    hipLaunchKernelGGL(k_trinv_lds, 1, 1024, 0, s, R, k, (int64_t)k, XT, (int64_t)k, nullptr, (int64_t)0);
    LSPCA_HIP(hipGetLastError());
    return LSPCA_OK;
  }
  const int nb = (k + kBlk - 1) / kBlk;
  double *St = scratch;
  hipLaunchKernelGGL(k_zero_i32, (unsigned)(((int64_t)k * k * 2 + 255) / 256), 256, 0, s, (int *)XT, k * k * 2);
  LSPCA_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_trinv_blocks, nb, 1024, 0, s, R, k, XT);
  LSPCA_HIP(hipGetLastError());
  for (int J = 1; J < nb; ++J) {
    const int j0 = J * kBlk, jb = std::min(kBlk, k - j0);
    for (int I = 0; I < J; ++I) {
      const int i0 = I * kBlk, ib = std::min(kBlk, k - i0);
      // St[c][r] = sum over rows p in [i0, j0) of XT[p][i0+c] R[p][j0+r]  (ib x jb)
      LSPCA_TRY(launch_tn(LSPCA_F64, XT + (int64_t)i0 * k + i0, k, R + (int64_t)i0 * k + j0, k, St,
                          j0 - i0, ib, jb, 1, s, jb, 1.0, 0.0));
      // XT_JI[r][c] = -sum_p XT_JJ[r][p] St[c][p]
      LSPCA_TRY(launch_nt(LSPCA_F64, XT + (int64_t)j0 * k + j0, k, St, jb, XT + (int64_t)j0 * k + i0, k, jb,
                          ib, jb, s, -1.0, 0.0));
    }
  }
  return LSPCA_OK;
}

// The preconditioner of the small SVD (Cholesky QR of R^T) is applied when
// R is graded: max |R_ii| >= kPrecondRatio min |R_ii|. The ratio of R's
// extreme diagonal entries follows the spread of F's singular values; on
// flat or slowly decaying spectra (ratio below 4) one-sided Jacobi on R
// takes the same number of sweeps, or one more, without it, so its two
// Cholesky QR passes would only cost time; on graded ones it saves 3 to 15
// sweeps (measured on k = 128 with spectra from flat to 1e6).
constexpr double kPrecondRatio = 4.0;

// flag[0] = 1 when max_i |R_ii| >= ratio * min_i |R_ii| (R row-major k x k);
// one workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_diag_graded(const double *__restrict__ R, int k, double ratio,
                                                     int *__restrict__ flag) {
  __shared__ double smax[256], smin[256];
  const int t = threadIdx.x;
  double mx = 0.0, mn = INFINITY;
  for (int i = t; i < k; i += 256) {
    const double d = fabs(R[(int64_t)i * k + i]);
    mx = fmax(mx, d);
    mn = fmin(mn, d);
  }
  smax[t] = mx;
  smin[t] = mn;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      smax[t] = fmax(smax[t], smax[t + w]);
      smin[t] = fmin(smin[t], smin[t + w]);
    }
    __syncthreads();
  }
  if (t == 0) flag[0] = smax[0] >= ratio * smin[0] ? 1 : 0;
}

static bool debug_on() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("LSPCA_DEBUG");
    v = (e && *e && *e != '0') ? 1 : 0;
  }
  return v == 1;
}

// Threads for one round of n_pairs pairs at 16 lanes each (whole waves).
static int round_threads(int n_pairs) {
  int t = ((16 * n_pairs + 63) / 64) * 64;
  return t < 64 ? 64 : (t > 1024 ? 1024 : t);
}

// Early stop of the one-sided Jacobi: a sweep whose rotated pairs all had
// |a_p.a_q| <= d |a_p| |a_q| ends the iteration. The next sweep would meet
// off-diagonal terms of order d^2 = 1e-16 (quadratic convergence), below the
// rotation threshold 8 max(k, 16) 2^-53 >= 1.4e-14, and rotate nothing; it
// only confirmed convergence (measured: the same bits with and without the
// early stop at k = 64 to 500, flat and graded spectra, one sweep fewer).
// Returns d^2; d = LSPCA_JACOBI_EARLY when set (0 turns the early stop off),
// else kJacobiEarly.
constexpr double kJacobiEarly = 1e-8;
static double jacobi_early2() {
  double d = kJacobiEarly;
  if (const char *e = getenv("LSPCA_JACOBI_EARLY")) d = atof(e);
  return d > 0 ? d * d : 0.0;
}

// Sweep limit of the one-sided Jacobi: `dflt`, or LSPCA_JACOBI_SWEEPS when
// it is smaller (a test knob that forces the non-convergence error).
static int jacobi_sweep_limit(int dflt) {
  if (const char *e = getenv("LSPCA_JACOBI_SWEEPS")) {
    const int v = atoi(e);
    if (v >= 1 && v < dflt) return v;
  }
  return dflt;
}

// One-sided Jacobi SVD of a k x k matrix A (singular values and left
// singular vectors). A is row-major, or already in column storage
// (Wc[c][i] = A[i][c]) when `cols_given`. Writes the sorted singular
// values to sigma and, if UT != NULL, U^T (sorted rows). Sets the device
// int *noconv (zeroed by the caller) when the sweep limit was reached with
// rotations still made in the last sweep.
int jacobi_svd(const double *A, bool cols_given, int k, double *Wc, double *UT, double *sigma,
               int *dflag, int *noconv, hipStream_t s, const int *skip = nullptr) {
  const int64_t kk = (int64_t)k * k;
  if (cols_given)
    LSPCA_HIP(hipMemcpyAsync(Wc, A, kk * sizeof(double), hipMemcpyDeviceToDevice, s));
  else {
    hipLaunchKernelGGL(k_to_cols, (unsigned)((kk + 255) / 256), 256, 0, s, A, k, Wc);
    LSPCA_HIP(hipGetLastError());
  }
  const double tol = 8.0 * (double)std::max(k, 16) * 0x1p-53;
  const double big2 = jacobi_early2();
  int sweeps = 0;
  // one workgroup holding the whole matrix in LDS below k = 128; from
  // k = 128 on the block kernel's parallel rounds are faster (2.3 against
  // 2.5 ms for the small stage at k = 128, n = 2048)
  if ((int64_t)k * (k + 1) <= kLdsAlloc && k < 128) {
    hipLaunchKernelGGL(k_jacobi_lds, 1, round_threads((k + 1) / 2), 0, s, Wc, k, tol, big2,
                       jacobi_sweep_limit(60), dflag, noconv, skip);
    LSPCA_HIP(hipGetLastError());
    if (debug_on()) {
      LSPCA_HIP(hipMemcpyAsync(&sweeps, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
      LSPCA_HIP(hipStreamSynchronize(s));
    }
  } else {
    // blocks of b <= 32 columns, nb even, 2b padded columns of length k fit
    // in LDS; b groups of G lanes per workgroup, G = 16 (one DPP row, up to
    // 16 rows each) up to k = 256, 32 up to 512, else 64 looping over rows
    const int G = k <= 256 ? 16 : (k <= 512 ? 32 : 64);
    const int bmax = std::min(std::min((k <= 256 ? kBlockLdsAlloc : kLdsAlloc) / (2 * jacobi_ld(k)), 1024 / G), 32);
    if (bmax < 1) {
      set_error("jacobi: k = %d too large for the block kernel", k);
      return LSPCA_ENOTSUP;
    }
    const int nb = 2 * ((k + 2 * bmax - 1) / (2 * bmax));
    const int b = (k + nb - 1) / nb;
    // one cooperative launch for all sweeps (no host round trip per sweep);
    // LSPCA_JACOBI=launches keeps one launch per round (a test knob)
    const char *knob = getenv("LSPCA_JACOBI");
    bool done = false;
    if (!(knob && !strcmp(knob, "launches"))) {
      LSPCA_TRY(zero_i32(dflag, kJacobiMaxSweeps, s));
      int *counts = dflag, *swo = dflag + kJacobiMaxSweeps;
      double *wc = Wc;
      int kk2 = k, bb = b, nbb = nb, ms = jacobi_sweep_limit(kJacobiMaxSweeps);
      double tl = tol, bg = big2;
      int *nc = noconv;
      const int *sk = skip;
      void *args[] = {&wc, &kk2, &bb, &nbb, &tl, &bg, &ms, &counts, &swo, &nc, &sk};
      const void *fn = G == 16 ? (const void *)k_jacobi_coop<16, 16>
                               : G == 32 ? (const void *)k_jacobi_coop<32, 16> : (const void *)k_jacobi_coop<64, 0>;
      const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(nb / 2), dim3(G * b), args, 0, s);
      if (e == hipSuccess) {
        done = true;
        if (debug_on()) {
          LSPCA_HIP(hipMemcpyAsync(&sweeps, swo, sizeof(int), hipMemcpyDeviceToHost, s));
          LSPCA_HIP(hipStreamSynchronize(s));
        }
      } else {
        (void)hipGetLastError();                 // not co-resident: per-round launches
      }
    }
    int hflag = 0;
    bool conv = false;
    const int lim = jacobi_sweep_limit(kJacobiMaxSweeps);
    for (int sweep = 0; !done && sweep < lim; ++sweep) {
      LSPCA_TRY(zero_i32(dflag, 1, s));
      for (int round = 0; round < nb - 1; ++round) {
        if (G == 16)
          hipLaunchKernelGGL((k_jacobi_block<16, 16>), nb / 2, G * b, 0, s, Wc, k, b, nb, round, tol, big2, dflag,
                             skip);
        else if (G == 32)
          hipLaunchKernelGGL((k_jacobi_block<32, 16>), nb / 2, G * b, 0, s, Wc, k, b, nb, round, tol, big2, dflag,
                             skip);
        else
          hipLaunchKernelGGL((k_jacobi_block<64, 0>), nb / 2, G * b, 0, s, Wc, k, b, nb, round, tol, big2, dflag,
                             skip);
        LSPCA_HIP(hipGetLastError());
      }
      LSPCA_HIP(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
      LSPCA_HIP(hipStreamSynchronize(s));
      sweeps = sweep + 1;
      if (!(hflag & 1) || !(hflag & 2)) {
        conv = true;
        break;
      }
    }
    // the last sweep allowed still rotated: not converged
    if (!done && !conv) LSPCA_TRY(set_i32(noconv, 1, s));
  }
  if (debug_on()) fprintf(stderr, "[lspca] jacobi k=%d sweeps=%d\n", k, sweeps);
  hipLaunchKernelGGL(k_jacobi_finish, 1, 1024, (size_t)k * (sizeof(double) + sizeof(int)) + 16, s,
                     Wc, k, UT, sigma);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

}  // namespace

// F <- R^-T F (k x n), R upper triangular k x k (row-major FP64): the
// "F = (R^-1)^T F" step of Algorithm 3 (Streaming SPCA).
int apply_rinv_t(const double *R, int k, double *F, int64_t n, Workspace &ws, hipStream_t s) {
  const int64_t kk = (int64_t)k * k;
  double *XT = ws.take<double>(kk), *Ri = ws.take<double>(kk);
  double *scr = ws.take<double>(3 * 128 * 128);
  double *Fo = ws.take<double>((size_t)k * n);
  LSPCA_TRY(trinv_t(R, k, XT, scr, s));                 // XT = R^-T
  LSPCA_TRY(launch_transpose_f64(XT, k, k, Ri, s));     // Ri = R^-1
  // Fo[i][j] = sum_r Ri[r][i] F[r][j]: the split-row product with one split
  LSPCA_TRY(launch_tn(LSPCA_F64, Ri, k, F, n, Fo, k, k, (int)n, 1, s));
  LSPCA_HIP(hipMemcpyAsync(F, Fo, (size_t)k * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return LSPCA_OK;
}

int small_factor(const double *F, const double *G, int k, int64_t n, double *V, double *sigma,
                 double *sigma_x, Workspace &ws, hipStream_t s, int *rank_flag, int route) {
  const int64_t kk = (int64_t)k * k;
  const int splits = tn_pick_splits(n, k, k);
  double *Ft = ws.take<double>((size_t)n * k);
  double *Qa = ws.take<double>((size_t)n * k);
  double *Qb = ws.take<double>((size_t)n * k);
  double *part = ws.take<double>(tn_partial_elems(k, k, splits));
  double *M = ws.take<double>(kk);
  double *Rall = ws.take<double>(kk);
  double *Rtmp = ws.take<double>(kk);
  double *XT = ws.take<double>(kk);
  double *Wc = ws.take<double>(kk);
  double *UT = ws.take<double>(kk);
  double *sx = ws.take<double>(k);
  double *Vw = ws.take<double>((size_t)n * k);
  double *scr = ws.take<double>(3 * 128 * 128);
  double *prebuf = ws.take<double>(4 * kk);
  double *sw = ws.take<double>(k);
  int *dflag = ws.take<int>(kSmallFlags);
  const size_t ws_mark = ws.used;

  // Route 0 runs first as mode kSpec: the plain Cholesky QR attempt without
  // its host round trip; the Jacobi on R runs unless a Cholesky failed or R
  // is graded (a device flag the Jacobi kernels read), and the closing commit
  // reports that case. Then the stage runs again with the host decisions:
  // from the start (kFull) after a failed Cholesky, or from the
  // preconditioner with the attempt's Q and R (kGraded).
  enum { kSpec, kFull, kGraded };
  const double *q_spec = nullptr;
  auto run = [&](int mode) -> int {
  const bool spec = mode == kSpec;
  int hflag[4];
  int *skip = spec ? dflag + kSkip : nullptr;
  ws.used = ws_mark;

  LSPCA_TRY(zero_i32(dflag + kNoConv, 2, s));
  if (mode != kGraded) LSPCA_TRY(launch_transpose_f64(F, k, (int)n, Ft, s));   // F (k x n) -> F^T (n x k)

  if (route == 0) {
    // Cholesky QR passes on F^T: Q <- Q R_p^-1, R <- R_p R. Each pass's
    // Cholesky writes its own failure flag and the passes run without a host
    // round trip: after a failed factor the later steps of the attempt only
    // compute values that are then discarded. One round trip per attempt
    // reads the flags and, for the plain attempt, whether R is graded.
    const double *Qin = Ft;
    double *Qout = Qa;
    bool shifted = false;
    bool graded = mode == kGraded;
    int passes = mode == kGraded ? 2 : 0;
    if (mode == kGraded) Qin = q_spec;
    for (int attempt = 0; attempt < 2 && passes == 0; ++attempt) {
      const int npass = shifted ? 3 : 2;
      Qin = Ft;
      Qout = Qa;
      LSPCA_TRY(zero_i32(dflag, 4, s));
      for (int pss = 0; pss < npass; ++pss) {
        LSPCA_TRY(gram(Qin, n, k, M, part, splits, s));
        if (shifted && pss == 0) {
          // shift = 11 (n k + k (k + 1)) u ||F||_F^2 (shifted Cholesky QR;
          // Fukaya et al., SIAM J. Sci. Comput. 42, 2020)
          const double c = 11.0 * ((double)n * k + (double)k * (k + 1)) * 0x1p-53;
          hipLaunchKernelGGL(k_shift_diag, 1, 256, 0, s, M, k, c);
          LSPCA_HIP(hipGetLastError());
        }
        LSPCA_TRY(chol(M, k, dflag + pss, scr, s));
        LSPCA_TRY(trinv_t(M, k, XT, scr, s));
        LSPCA_TRY(launch_nt(LSPCA_F64, Qin, k, XT, k, Qout, k, n, k, k, s));
        if (pss == 0) {
          LSPCA_HIP(hipMemcpyAsync(Rall, M, kk * sizeof(double), hipMemcpyDeviceToDevice, s));
        } else {
          // Rall <- M * Rall  (nt with B = Rall^T)
          LSPCA_TRY(launch_transpose_f64(Rall, k, k, Rtmp, s));
          LSPCA_TRY(launch_nt(LSPCA_F64, M, k, Rtmp, k, Rall, k, k, k, k, s));
        }
        Qin = Qout;
        Qout = (Qout == Qa) ? Qb : Qa;
      }
      if (!shifted) {
        hipLaunchKernelGGL(k_diag_graded, 1, 256, 0, s, Rall, k, kPrecondRatio, dflag + 3);
        LSPCA_HIP(hipGetLastError());
      }
      if (spec) {
        // skip = a Cholesky of the attempt failed or R is graded (the three
        // flags kept beside it for the host)
        hipLaunchKernelGGL(k_any3, 1, 1, 0, s, dflag, dflag + 1, dflag + 3, skip);
        LSPCA_HIP(hipGetLastError());
        passes = npass;
        q_spec = Qin;
        break;
      }
      LSPCA_HIP(hipMemcpyAsync(hflag, dflag, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
      LSPCA_HIP(hipStreamSynchronize(s));
      bool failed = false;
      for (int pss = 0; pss < npass; ++pss) failed = failed || hflag[pss] != 0;
      if (!failed) {
        passes = npass;
        graded = !shifted && hflag[3] != 0;
      } else if (!shifted) {
        shifted = true;
      } else {
        break;
      }
    }
    if (passes == 0) {
      set_error("factor: Cholesky QR of F^T failed (F is numerically rank deficient)");
      *rank_flag = 1;
      return LSPCA_ERANK;
    }
    const double *Q = Qin;

    // SVD of R: R W = U_R Sigma; V = Q U_R. Preconditioning: with
    // R^T = Q2 R2 (Cholesky QR twice on the k x k matrix R^T), R2^T has the
    // same left singular vectors U_R and singular values as R, and one-sided
    // Jacobi on the columns of R2^T (= the rows of R2) needs far fewer sweeps
    // than on R when R is graded (Drmac and Veselic, SIAM J. Matrix Anal.
    // Appl. 29, 2008); applied only then (kPrecondRatio).
    bool pre = graded;
    if (debug_on()) fprintf(stderr, "[lspca] small SVD preconditioner %s\n", pre ? "on" : "off");
    if (pre) {
      double *T = prebuf;                              // 4 k x k scratch matrices
      double *S1 = T + kk, *P = T + 2 * kk, *R2 = T + 3 * kk;
      LSPCA_TRY(launch_transpose_f64(Rall, k, k, T, s));            // T = R^T
      LSPCA_TRY(zero_i32(dflag, 2, s));
      for (int pss = 0; pss < 2; ++pss) {                           // flags read once after both
        const double *Tin = pss == 0 ? T : P;
        LSPCA_TRY(gram(Tin, k, k, M, part, tn_pick_splits(k, k, k), s));
        LSPCA_TRY(chol(M, k, dflag + pss, scr, s));
        LSPCA_TRY(trinv_t(M, k, XT, scr, s));
        double *Pout = pss == 0 ? P : S1;              // P = T S^-1
        LSPCA_TRY(launch_nt(LSPCA_F64, Tin, k, XT, k, Pout, k, k, k, k, s));
        if (pss == 0) {
          LSPCA_HIP(hipMemcpyAsync(R2, M, kk * sizeof(double), hipMemcpyDeviceToDevice, s));
        } else {
          // R2 <- S2 R2  (nt with B = R2^T)
          LSPCA_TRY(launch_transpose_f64(R2, k, k, Rtmp, s));
          LSPCA_TRY(launch_nt(LSPCA_F64, M, k, Rtmp, k, R2, k, k, k, k, s));
        }
      }
      LSPCA_HIP(hipMemcpyAsync(hflag, dflag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
      LSPCA_HIP(hipStreamSynchronize(s));
      pre = hflag[0] == 0 && hflag[1] == 0;          // else Jacobi on R itself
      // the rows of R2 are the columns of R2^T: column storage as is
      if (pre) LSPCA_TRY(jacobi_svd(R2, true, k, Wc, UT, sw, dflag + 8, dflag + kNoConv, s));
    }
    if (!pre) LSPCA_TRY(jacobi_svd(Rall, false, k, Wc, UT, sw, dflag + 8, dflag + kNoConv, s, skip));
    LSPCA_TRY(launch_nt(LSPCA_F64, Q, k, UT, k, Vw, k, n, k, k, s));
  } else {
    // The route of the caption of the algorithm table: F F^T = W Lambda W^T
    // by one-sided Jacobi on the symmetric positive semidefinite F F^T (its
    // left singular vectors are W, its singular values Lambda), D =
    // Lambda^(1/2), V = F^T W D^-1, then one Cholesky QR pass on V.
    LSPCA_TRY(gram(Ft, n, k, M, part, splits, s));                 // M = F F^T
    LSPCA_HIP(hipMemcpyAsync(Rall, M, kk * sizeof(double), hipMemcpyDeviceToDevice, s));
    LSPCA_TRY(jacobi_svd(M, false, k, Wc, UT, sw, dflag + 8, dflag + kNoConv, s));   // UT = W^T, sw = Lambda
    hipLaunchKernelGGL(k_sqrt_vec, 1, 256, 0, s, sw, k);            // D
    LSPCA_HIP(hipGetLastError());
    LSPCA_TRY(launch_nt(LSPCA_F64, Ft, k, UT, k, Qa, k, n, k, k, s));      // F^T W
    hipLaunchKernelGGL(k_scale_cols_inv, (unsigned)(((int64_t)n * k + 255) / 256), 256, 0, s, Qa, n, k, sw);
    LSPCA_HIP(hipGetLastError());
    LSPCA_TRY(zero_i32(dflag, 1, s));
    LSPCA_TRY(gram(Qa, n, k, M, part, splits, s));                  // Cholesky QR: V = Qa R^-1
    LSPCA_TRY(chol(M, k, dflag, scr, s));
    if (sigma_x) LSPCA_TRY(chol(Rall, k, dflag, scr, s));         // R^T R = F F^T, for Sigma^s
    LSPCA_HIP(hipMemcpyAsync(hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    LSPCA_HIP(hipStreamSynchronize(s));
    if (hflag[0]) {
      set_error("factor: F is numerically rank deficient (the eigenvalue route resolves D_k only "
                "down to about sqrt(u) D_1)");
      *rank_flag = 1;
      return LSPCA_ERANK;
    }
    LSPCA_TRY(trinv_t(M, k, XT, scr, s));
    LSPCA_TRY(launch_nt(LSPCA_F64, Qa, k, XT, k, Vw, k, n, k, k, s));
  }
  double *sgn = nullptr;
  LSPCA_TRY(sign_of_cols(Vw, n, k, &sgn, ws, s));

  if (sigma_x) {
    // Sigma^s = singular values of R R_G^-1, G = R_G^T R_G.
    LSPCA_TRY(zero_i32(dflag, 1, s));
    LSPCA_HIP(hipMemcpyAsync(M, G, kk * sizeof(double), hipMemcpyDeviceToDevice, s));
    LSPCA_TRY(chol(M, k, dflag, scr, s));
    LSPCA_TRY(trinv_t(M, k, XT, scr, s));
    LSPCA_TRY(launch_nt(LSPCA_F64, Rall, k, XT, k, Rtmp, k, k, k, k, s));
    LSPCA_TRY(jacobi_svd(Rtmp, false, k, Wc, nullptr, sx, dflag + 64, dflag + kNoConv + 1, s));
  }

  // Checks and outputs in one launch, then one round trip for the status:
  // the outputs are written only when every check passed. Rank check on D:
  // D_k <= 64 n eps D_1 means F is numerically rank deficient (the
  // eigenvalue route squares: sqrt(64 n eps) D_1).
  const double rel = 64.0 * (double)n * 0x1p-52;
  int *stat = dflag + kStatus;
  hipLaunchKernelGGL(k_commit, (unsigned)std::max<int64_t>(1, std::min<int64_t>((n * k + 255) / 256, 65536)), 256, 0,
                     s, Vw, sgn, n, k, sw, sx, skip, sigma_x ? dflag : nullptr, dflag + kNoConv,
                     route == 0 ? rel : std::sqrt(rel), V, sigma, sigma_x, stat);
  LSPCA_HIP(hipGetLastError());
  int hstat[6] = {0, 0, 0, 0, 0, 0};
  LSPCA_HIP(hipMemcpyAsync(hstat, stat, sizeof(hstat), hipMemcpyDeviceToHost, s));
  LSPCA_HIP(hipStreamSynchronize(s));
  double dd[2];
  std::memcpy(dd, hstat + 2, sizeof(dd));
  switch (hstat[0]) {
    case 0:
      return LSPCA_OK;
    case 5:
      return kRedo;
    case 1:
      set_error("factor: Cholesky of G failed (the sketch U = X Omega is rank deficient)");
      *rank_flag = 1;
      return LSPCA_ERANK;
    case 2:
    case 3:
      set_error("factor: one-sided Jacobi did not converge within its sweep limit (%s)",
                hstat[0] == 2 ? "SVD of F" : "Sigma^s");
      return LSPCA_ENOCONV;
    default:
      set_error("factor: F is numerically rank deficient (D_k = %g, D_1 = %g)", dd[0], dd[1]);
      *rank_flag = 1;
      return LSPCA_ERANK;
  }
  };
  if (route != 0) return run(kFull);
  const int rc = run(kSpec);
  if (rc != kRedo) return rc;
  int fl[3];
  LSPCA_HIP(hipMemcpyAsync(fl, dflag + kSkip + 1, sizeof(fl), hipMemcpyDeviceToHost, s));
  LSPCA_HIP(hipStreamSynchronize(s));
  if (debug_on()) fprintf(stderr, "[lspca] small stage: plain attempt %s\n", fl[0] | fl[1] ? "failed" : "graded");
  return run(fl[0] | fl[1] ? kFull : kGraded);
}

}  // namespace lspca
