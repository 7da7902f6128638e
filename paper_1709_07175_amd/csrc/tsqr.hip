// Tall-skinny Householder QR of the sketch U = X Omega (m x k) with an
// explicit thin Q: the "Q, R = qr(U)" of Algorithm 1 (SPCA, the non-lazy
// baseline).
//
// U arrives transposed: column c of U is contiguous at U + c * ldu, with ldu
// a multiple of the block height BR (256 rows for FP32, 128 for FP64).
// Leaves: workgroup b factors rows [b*BR, (b+1)*BR) by k Householder
// reflectors H_j = I - tau_j v_j v_j^T (LAPACK's convention: v_j[j] = 1,
// H_j x = beta e_j); its k x k R goes to level 0 of a binary tree.
// Tree nodes: [R_a; R_b] -> R by reflectors whose top part is e_j and whose
// bottom part has rows 0..j only (R_b upper triangular).
// Q: top down. The root starts from C = I_k; a node maps its C to
// (C_a, C_b) = top and bottom halves of H_0 ... H_{k-1} [C; 0]; a leaf forms
// its BR x k rows of Q = H_0 ... H_{k-1} [C; 0].
//
// Register layout (1024-thread workgroups, 16 wavefronts): lane l of wave w
// holds column c = w + 16 (l / 16) + 64 q for q < NQ and rows
// r = (l % 16) + 16 i for i < NI, so the 16 lanes of one DPP row hold one
// whole column and a column sum takes four DPP steps. Columns are dealt to
// the waves cyclically, so every wave keeps work until the last reflectors.
// Reflectors, R and C are stored in the matching "slice" order: column c,
// then lane row l % 16, then i (one lane's NI entries are contiguous); a
// column occupies BR entries whatever k is.
// Reflector j touches rows >= j (leaf) or <= j (node) and columns > j only;
// with 16 reflectors per block both bounds are static, so finished rows and
// columns cost nothing.
#include "common.h"

#include <vector>

namespace lspca {

typedef int i32x2 __attribute__((ext_vector_type(2)));

template <int CTRL> __device__ inline float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ inline double dpp_f(double v) {
  i32x2 p = __builtin_bit_cast(i32x2, v);
  p.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xF, 0xF, false);
  p.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, p);
}
// Sum over a DPP row of 16 lanes, received by all 16 (bitwise equal, since
// each step adds the same two values in either order): quad_perm xor 1 and
// xor 2, then row_half_mirror and row_mirror.
template <typename T> __device__ inline T sum16(T v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  return v;
}

template <typename T> struct TsqrCfg;
template <> struct TsqrCfg<float> {
  static constexpr int BR = 256, NI = 16, NQ = 4;
  typedef float vec __attribute__((ext_vector_type(4)));
};
template <> struct TsqrCfg<double> {
  static constexpr int BR = 128, NI = 8, NQ = 2;
  typedef double vec __attribute__((ext_vector_type(2)));
};
// LDS stride of one lane slice: NI entries plus 16 bytes, so that the 16
// slices of a DPP row start on distinct bank groups for 16-byte reads.
template <typename T> constexpr int lds_stride() { return TsqrCfg<T>::NI + 16 / (int)sizeof(T); }
// Slice position of row r within a column.
template <typename T> __device__ inline int spos(int r) { return (r & 15) * TsqrCfg<T>::NI + (r >> 4); }

template <typename T> __device__ inline void put_slice(T *dst, const T (&v)[TsqrCfg<T>::NI]) {
  using V = typename TsqrCfg<T>::vec;
  constexpr int W = 16 / sizeof(T);
#pragma unroll
  for (int i = 0; i < TsqrCfg<T>::NI; i += W) {
    V x;
#pragma unroll
    for (int e = 0; e < W; ++e) x[e] = v[i + e];
    *reinterpret_cast<V *>(dst + i) = x;
  }
}
template <typename T> __device__ inline void get_slice(const T *src, T (&v)[TsqrCfg<T>::NI]) {
  using V = typename TsqrCfg<T>::vec;
  constexpr int W = 16 / sizeof(T);
#pragma unroll
  for (int i = 0; i < TsqrCfg<T>::NI; i += W) {
    const V x = *reinterpret_cast<const V *>(src + i);
#pragma unroll
    for (int e = 0; e < W; ++e) v[i + e] = x[e];
  }
}

// Householder reflector for x = (x0, rest) with ||rest||^2 = s (LAPACK
// dlarfg): beta = -sign(x0) ||x||, tau = (beta - x0) / beta, the rest of v
// is rest / (x0 - beta). s == 0 gives tau = 0 (H = I), beta = x0.
template <typename T>
__device__ inline void householder(T x0, T s, T &beta, T &tau, T &scale) {
  if (s == (T)0) {
    beta = x0;
    tau = 0;
    scale = 0;
    return;
  }
  const T norm = sqrt(x0 * x0 + s);
  beta = x0 >= (T)0 ? -norm : norm;
  tau = (beta - x0) / beta;
  scale = (T)1 / (x0 - beta);
}

// ------------------------------------------------------------------ leaf --
// Factor block b of U. Reflector j is built by the 16 lanes that hold column
// j and written three ways: v_j (slice order) over column j of the block in
// U, into the LDS buffer for the other columns (double buffered: one barrier
// per reflector), and R's column j (slice order, zeros below the diagonal)
// to R_out[b].
// RM: U row-major (row r at U + r * ldu) instead of transposed; WV: write
// the reflectors and tau (needed for Q; an R-only factorisation skips them).
template <typename T, bool RM = false, bool WV = true>
__global__ __launch_bounds__(1024) void k_tsqr_leaf(T *__restrict__ U, int64_t ldu, int64_t m, int k,
                                                    T *__restrict__ tau_out, T *__restrict__ R_out) {
  constexpr int BR = TsqrCfg<T>::BR, NI = TsqrCfg<T>::NI, NQ = TsqrCfg<T>::NQ, SP = lds_stride<T>();
  __shared__ __align__(16) T vl[2][16 * SP];
  __shared__ T tl[2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rg = lane & 15, cg = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * BR;
  const int rows_here = (int)(m - row0 < BR ? m - row0 : BR);
  T a[NQ][NI];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = w + 16 * cg + 64 * q;
    if constexpr (RM) {
      const T *src = U + (row0 + rg) * ldu + (c < k ? c : 0);
#pragma unroll
      for (int i = 0; i < NI; ++i) a[q][i] = (c < k && rg + 16 * i < rows_here) ? src[16 * i * ldu] : (T)0;
    } else {
      const T *src = U + (int64_t)(c < k ? c : 0) * ldu + row0 + rg;
#pragma unroll
      for (int i = 0; i < NI; ++i) a[q][i] = (c < k && rg + 16 * i < rows_here) ? src[16 * i] : (T)0;
    }
  }
#pragma unroll
  for (int bi = 0; bi < 4 * NQ; ++bi) {           // reflectors 16 bi .. 16 bi + 15
    const int q = bi / 4, jb = bi % 4;
    if (16 * bi >= k) break;
    for (int j16 = 0; j16 < 16; ++j16) {
      const int j = 16 * bi + j16, buf = j & 1;
      if (j >= k) break;
      if (w == j16 && cg == jb) {                 // this DPP row holds column j
        T s = 0, x0 = 0;
#pragma unroll
        for (int i = bi; i < NI; ++i) {
          const int r = rg + 16 * i;
          const T x = a[q][i];
          s += r > j ? x * x : (T)0;
          x0 += r == j ? x : (T)0;
        }
        s = sum16(s);
        x0 = sum16(x0);
        T beta, tau, scale;
        householder(x0, s, beta, tau, scale);
        T v[NI], rc[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          const int r = rg + 16 * i;
          const T x = a[q][i];
          v[i] = i < bi ? (T)0 : (r > j ? x * scale : (r == j ? (T)1 : (T)0));
          rc[i] = r < j ? x : (r == j ? beta : (T)0);
        }
        put_slice<T>(vl[buf] + rg * SP, v);
        if constexpr (WV) put_slice<T>(U + (int64_t)j * ldu + row0 + rg * NI, v);
        put_slice<T>(R_out + ((int64_t)blockIdx.x * k + j) * BR + rg * NI, rc);
        if (rg == 0) {
          tl[buf] = tau;
          if constexpr (WV) tau_out[(int64_t)blockIdx.x * k + j] = tau;
        }
      }
      __syncthreads();
      const T tau = tl[buf];
      T v[NI];
      get_slice<T>(vl[buf] + rg * SP, v);
#pragma unroll
      for (int qq = q; qq < NQ; ++qq) {
        const int c = w + 16 * cg + 64 * qq;
        if (w + 64 * qq + 48 > j) {               // wave-uniform: a column right of j
          T d0 = 0, d1 = 0;
#pragma unroll
          for (int i = bi; i < NI; ++i) {
            if ((i - bi) & 1) d1 += v[i] * a[qq][i];
            else d0 += v[i] * a[qq][i];
          }
          T d = sum16(d0 + d1);
          d = (c > j && c < k) ? d * tau : (T)0;
#pragma unroll
          for (int i = bi; i < NI; ++i) a[qq][i] -= d * v[i];
        }
      }
    }
  }
}

// ----------------------------------------------------------------- nodes --
// Node p of a level combines R_in[2p] (top, R_a) and R_in[2p+1] (bottom,
// R_b) into R_out[p]; writes the bottom parts of its reflectors to Vb[p]
// (slice order, rows 0..j, zeros elsewhere) and tau[p]. Reflector j changes
// only row j of R_a, so each lane reads its columns' entries of R_a's row j
// one step ahead and writes the final row j of R_out. A node without a
// second child copies R_in[2p].
template <typename T, bool WV = true>
__global__ __launch_bounds__(1024) void k_tsqr_node(const T *__restrict__ R_in, int nin, int k,
                                                    T *__restrict__ R_out, T *__restrict__ Vb,
                                                    T *__restrict__ tau_out) {
  constexpr int BR = TsqrCfg<T>::BR, NI = TsqrCfg<T>::NI, NQ = TsqrCfg<T>::NQ, SP = lds_stride<T>();
  __shared__ __align__(16) T vl[2][16 * SP];
  __shared__ T tl[2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rg = lane & 15, cg = lane >> 4;
  const int p = blockIdx.x;
  const int64_t kb = (int64_t)k * BR;
  const T *Ra = R_in + 2 * (int64_t)p * kb;
  T *Rn = R_out + (int64_t)p * kb;
  if (2 * p + 1 >= nin) {                         // single child: pass R through
    for (int64_t e = threadIdx.x; e < kb; e += blockDim.x) Rn[e] = Ra[e];
    if constexpr (WV)
      for (int e = threadIdx.x; e < k; e += blockDim.x) tau_out[(int64_t)p * k + e] = 0;
    return;
  }
  const T *Rb = Ra + kb;
  T *V = WV ? Vb + (int64_t)p * kb : nullptr;
  T b[NQ][NI], ra_next[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = w + 16 * cg + 64 * q;
    T t[NI];
    get_slice<T>(Rb + (int64_t)(c < k ? c : 0) * BR + rg * NI, t);
#pragma unroll
    for (int i = 0; i < NI; ++i) b[q][i] = (c < k && rg + 16 * i < k) ? t[i] : (T)0;
    ra_next[q] = c < k ? Ra[(int64_t)c * BR] : (T)0;   // row 0 sits first in every slice order
  }
#pragma unroll
  for (int bi = 0; bi < 4 * NQ; ++bi) {
    const int q = bi / 4, jb = bi % 4;
    if (16 * bi >= k) break;
    for (int j16 = 0; j16 < 16; ++j16) {
      const int j = 16 * bi + j16, buf = j & 1;
      if (j >= k) break;
      T ra[NQ];
#pragma unroll
      for (int qq = 0; qq < NQ; ++qq) {
        ra[qq] = 0;
        if (qq < q) continue;
        const int c = w + 16 * cg + 64 * qq;
        ra[qq] = ra_next[qq];
        if (c < k && j + 1 < k) ra_next[qq] = Ra[(int64_t)c * BR + spos<T>(j + 1)];
      }
      if (w == j16 && cg == jb) {
        T s = 0;
#pragma unroll
        for (int i = 0; i <= bi; ++i) {
          const T x = b[q][i];
          s += rg + 16 * i <= j ? x * x : (T)0;
        }
        s = sum16(s);
        T beta, tau, scale;
        householder(ra[q], s, beta, tau, scale);
        T v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) v[i] = (i <= bi && rg + 16 * i <= j) ? b[q][i] * scale : (T)0;
        put_slice<T>(vl[buf] + rg * SP, v);
        if constexpr (WV) put_slice<T>(V + (int64_t)j * BR + rg * NI, v);
        if (rg == 0) {
          tl[buf] = tau;
          if constexpr (WV) tau_out[(int64_t)p * k + j] = tau;
          Rn[(int64_t)j * BR + spos<T>(j)] = beta;
        }
      }
      __syncthreads();
      const T tau = tl[buf];
      T v[NI];
      get_slice<T>(vl[buf] + rg * SP, v);
#pragma unroll
      for (int qq = 0; qq < NQ; ++qq) {
        const int c = w + 16 * cg + 64 * qq;
        if (qq < q) {                             // columns left of j: zero below the diagonal
          if (rg == 0 && c < k) Rn[(int64_t)c * BR + spos<T>(j)] = (T)0;
          continue;
        }
        T wv = 0;
        if (w + 64 * qq + 48 > j) {
          T d0 = 0, d1 = 0;
#pragma unroll
          for (int i = 0; i <= bi; ++i) {
            if (i & 1) d1 += v[i] * b[qq][i];
            else d0 += v[i] * b[qq][i];
          }
          const T d = sum16(d0 + d1);
          wv = (c > j && c < k) ? (ra[qq] + d) * tau : (T)0;
#pragma unroll
          for (int i = 0; i <= bi; ++i) b[qq][i] -= wv * v[i];
        }
        if (rg == 0 && c < k && c != j) Rn[(int64_t)c * BR + spos<T>(j)] = c > j ? ra[qq] - wv : (T)0;
      }
    }
  }
}

// Staging of 16 stored reflectors (16 x BR entries, slice order) into LDS:
// thread t moves one 16-byte vector.
template <typename T> struct Stage16 {
  using V = typename TsqrCfg<T>::vec;
  static constexpr int W = 16 / sizeof(T), BR = TsqrCfg<T>::BR, NI = TsqrCfg<T>::NI, SP = lds_stride<T>();
  int jj, src, dst;
  __device__ Stage16() {
    const int e = threadIdx.x * W;
    jj = e / BR;
    src = e % BR;
    dst = jj * 16 * SP + (src / NI) * SP + src % NI;
  }
  // reflector 16 blk + jj, stored at base + j * ld
  __device__ V fetch(const T *base, int64_t ld, int blk, int k) const {
    const int j = 16 * blk + jj;
    V x = {};
    if (j < k) x = *reinterpret_cast<const V *>(base + (int64_t)j * ld + src);
    return x;
  }
};

// Q formation at a node: C_in[p] (k x k) -> C_out[2p] = top, C_out[2p+1] =
// bottom halves of H_0 ... H_{k-1} [C; 0]. Reflector j changes only row j
// of the top half, so each lane reads its columns' entries of row j of C_in
// when the descending sweep reaches it (one step ahead) and writes the final
// row j of C_out[2p]. Single child: C passes through. Reflectors come from
// Vb[p] through LDS, 16 at a time, the next 16 loaded during the current.
template <typename T>
__global__ __launch_bounds__(1024) void k_tsqr_node_q(const T *__restrict__ C_in, int nchild, int k,
                                                      const T *__restrict__ Vb,
                                                      const T *__restrict__ tau_in,
                                                      T *__restrict__ C_out) {
  constexpr int BR = TsqrCfg<T>::BR, NI = TsqrCfg<T>::NI, NQ = TsqrCfg<T>::NQ, SP = lds_stride<T>();
  using Vec = typename TsqrCfg<T>::vec;
  __shared__ __align__(16) T vs[2][16 * 16 * SP];
  __shared__ T ts[2][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rg = lane & 15, cg = lane >> 4;
  const int p = blockIdx.x;
  const int64_t kb = (int64_t)k * BR;
  const T *Cn = C_in + (int64_t)p * kb;
  T *Ca = C_out + 2 * (int64_t)p * kb;
  if (2 * p + 1 >= nchild) {
    for (int64_t e = threadIdx.x; e < kb; e += blockDim.x) Ca[e] = Cn[e];
    return;
  }
  T *Cb = Ca + kb;
  const T *V = Vb + (int64_t)p * kb;
  const T *tau = tau_in + (int64_t)p * k;
  const Stage16<T> st;
  const int nblk = (k + 15) / 16;
  Vec pre = st.fetch(V, BR, nblk - 1, k);
  T tpre = (threadIdx.x < 16 && 16 * (nblk - 1) + (int)threadIdx.x < k) ? tau[16 * (nblk - 1) + threadIdx.x] : (T)0;
  T cb[NQ][NI], cn_next[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = w + 16 * cg + 64 * q;
#pragma unroll
    for (int i = 0; i < NI; ++i) cb[q][i] = 0;
    cn_next[q] = c < k ? Cn[(int64_t)c * BR + spos<T>(k - 1)] : (T)0;
  }
#pragma unroll
  for (int bi = 4 * NQ - 1; bi >= 0; --bi) {
    if (bi >= nblk) continue;
    const int buf = bi & 1;
    *reinterpret_cast<Vec *>(&vs[buf][st.dst]) = pre;
    if (threadIdx.x < 16) ts[buf][threadIdx.x] = tpre;
    __syncthreads();
    if (bi > 0) {
      pre = st.fetch(V, BR, bi - 1, k);
      tpre = threadIdx.x < 16 ? tau[16 * (bi - 1) + threadIdx.x] : (T)0;
    }
    for (int j16 = 15; j16 >= 0; --j16) {
      const int j = 16 * bi + j16;
      if (j >= k) continue;
      T cn[NQ];
#pragma unroll
      for (int qq = 0; qq < NQ; ++qq) {
        const int c = w + 16 * cg + 64 * qq;
        cn[qq] = cn_next[qq];
        if (c < k && j > 0) cn_next[qq] = Cn[(int64_t)c * BR + spos<T>(j - 1)];
      }
      const T t = ts[buf][j16];
      T v[NI];
      get_slice<T>(&vs[buf][j16 * 16 * SP + rg * SP], v);
#pragma unroll
      for (int qq = 0; qq < NQ; ++qq) {
        const int c = w + 16 * cg + 64 * qq;
        if (w + 64 * qq < k) {                    // wave-uniform
          T d0 = 0, d1 = 0;
#pragma unroll
          for (int i = 0; i <= bi; ++i) {
            if (i & 1) d1 += v[i] * cb[qq][i];
            else d0 += v[i] * cb[qq][i];
          }
          const T d = sum16(d0 + d1);
          const T wv = (cn[qq] + d) * t;
#pragma unroll
          for (int i = 0; i <= bi; ++i) cb[qq][i] -= wv * v[i];
          if (rg == 0 && c < k) Ca[(int64_t)c * BR + spos<T>(j)] = cn[qq] - wv;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = w + 16 * cg + 64 * q;
    if (c < k) put_slice<T>(Cb + (int64_t)c * BR + rg * NI, cb[q]);
  }
}

// Q formation at a leaf: rows of Q = H_0 ... H_{k-1} [C; 0] for block b,
// reflectors read back from U (slice order) 16 at a time through LDS.
// OUT 0: Q row-major in T (ldq), written row-contiguously through an LDS
// tile; OUT 1: Q transposed and split into 16-bit parts, Qh[c*ldq + r],
// Ql[c*ldq + r] (DT the 16-bit type).
template <typename T, int OUT, int DT>
__global__ __launch_bounds__(1024) void k_tsqr_leaf_q(const T *__restrict__ U, int64_t ldu, int64_t m, int k,
                                                      const T *__restrict__ tau_in,
                                                      const T *__restrict__ C_in,
                                                      T *__restrict__ Q, int64_t ldq,
                                                      uint16_t *__restrict__ Qh,
                                                      uint16_t *__restrict__ Ql) {
  constexpr int BR = TsqrCfg<T>::BR, NI = TsqrCfg<T>::NI, NQ = TsqrCfg<T>::NQ, SP = lds_stride<T>();
  using Vec = typename TsqrCfg<T>::vec;
  __shared__ __align__(16) T vs[2][16 * 16 * SP];
  __shared__ T ts[2][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rg = lane & 15, cg = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * BR;
  const int rows_here = (int)(m - row0 < BR ? m - row0 : BR);
  const int64_t kb = (int64_t)k * BR;
  const T *C = C_in + (int64_t)blockIdx.x * kb;
  const T *Ub = U + row0;
  const T *tau = tau_in + (int64_t)blockIdx.x * k;
  const Stage16<T> st;
  const int nblk = (k + 15) / 16;
  Vec pre = st.fetch(Ub, ldu, nblk - 1, k);
  T tpre = (threadIdx.x < 16 && 16 * (nblk - 1) + (int)threadIdx.x < k) ? tau[16 * (nblk - 1) + threadIdx.x] : (T)0;
  T qv[NQ][NI];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = w + 16 * cg + 64 * q;
    T t[NI];
    get_slice<T>(C + (int64_t)(c < k ? c : 0) * BR + rg * NI, t);
#pragma unroll
    for (int i = 0; i < NI; ++i) qv[q][i] = (c < k && rg + 16 * i < k) ? t[i] : (T)0;
  }
#pragma unroll
  for (int bi = 4 * NQ - 1; bi >= 0; --bi) {
    if (bi >= nblk) continue;
    const int buf = bi & 1;
    *reinterpret_cast<Vec *>(&vs[buf][st.dst]) = pre;
    if (threadIdx.x < 16) ts[buf][threadIdx.x] = tpre;
    __syncthreads();
    if (bi > 0) {
      pre = st.fetch(Ub, ldu, bi - 1, k);
      tpre = threadIdx.x < 16 ? tau[16 * (bi - 1) + threadIdx.x] : (T)0;
    }
    for (int j16 = 15; j16 >= 0; --j16) {
      const int j = 16 * bi + j16;
      if (j >= k) continue;
      const T t = ts[buf][j16];
      T v[NI];
      get_slice<T>(&vs[buf][j16 * 16 * SP + rg * SP], v);
#pragma unroll
      for (int qq = 0; qq < NQ; ++qq) {
        if (w + 64 * qq < k) {
          T d0 = 0, d1 = 0;
#pragma unroll
          for (int i = bi; i < NI; ++i) {
            if ((i - bi) & 1) d1 += v[i] * qv[qq][i];
            else d0 += v[i] * qv[qq][i];
          }
          const T d = sum16(d0 + d1) * t;
#pragma unroll
          for (int i = bi; i < NI; ++i) qv[qq][i] -= d * v[i];
        }
      }
    }
  }
  if constexpr (OUT == 0) {
    // 16 rows at a time through an LDS tile (stride k + 1) into row-major Q
    T *tile = &vs[0][0];
    const int ts_ = k + 1;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      __syncthreads();
#pragma unroll
      for (int qq = 0; qq < NQ; ++qq) {
        const int c = w + 16 * cg + 64 * qq;
        if (c < k) tile[rg * ts_ + c] = qv[qq][i];
      }
      __syncthreads();
      for (int e = threadIdx.x; e < 16 * k; e += blockDim.x) {
        const int rr = e / k, c = e - rr * k, r = 16 * i + rr;
        if (r < rows_here) Q[(row0 + r) * ldq + c] = tile[rr * ts_ + c];
      }
    }
  } else {
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
      const int c = w + 16 * cg + 64 * qq;
      if (c >= k) continue;
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int r = rg + 16 * i;
        if (r < rows_here) {
          const float f = (float)qv[qq][i];
          uint16_t hi, lo;
          if constexpr (DT == LSPCA_BF16) {
            hi = __builtin_bit_cast(uint16_t, (__bf16)f);
            lo = __builtin_bit_cast(uint16_t, (__bf16)(f - bf16_bits_to_f32(hi)));
          } else {
            hi = f32_to_f16_bits(f);
            lo = f32_to_f16_bits(f - f16_bits_to_f32(hi));
          }
          Qh[(int64_t)c * ldq + row0 + r] = hi;
          Ql[(int64_t)c * ldq + row0 + r] = lo;
        }
      }
    }
  }
}

// C = I_k in slice order (column c: BR entries).
template <typename T> __global__ void k_eye_slices(T *C, int k) {
  constexpr int BR = TsqrCfg<T>::BR, NI = TsqrCfg<T>::NI;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * BR) return;
  const int c = (int)(e / BR), pp = (int)(e % BR);
  const int r = pp / NI + 16 * (pp % NI);
  C[e] = r == c ? (T)1 : (T)0;
}

// ---------------------------------------------------------------- driver --
static int tsqr_br(lspca_dtype ydt) { return ydt == LSPCA_F64 ? TsqrCfg<double>::BR : TsqrCfg<float>::BR; }

int tsqr_block_rows(lspca_dtype ydt) { return tsqr_br(ydt); }

int64_t tsqr_ld(int64_t m, lspca_dtype ydt) {
  const int BR = tsqr_br(ydt);
  return (m + BR - 1) / BR * BR;
}

size_t tsqr_workspace_bytes(int64_t m, int k, lspca_dtype ydt) {
  const size_t es = ydt == LSPCA_F64 ? 8 : 4;
  const int BR = tsqr_br(ydt);
  int64_t level = (m + BR - 1) / BR;
  size_t total = 0;
  bool leaf = true;
  // per level: R, C, tau; Vb above the leaves
  while (true) {
    const size_t blk = es * (size_t)level * k * BR;
    total += 2 * ws_bytes<char>(blk) + ws_bytes<char>(es * (size_t)level * k);
    if (!leaf) total += ws_bytes<char>(blk);
    if (level == 1) break;
    level = (level + 1) / 2;
    leaf = false;
  }
  return total + 4096;
}

template <typename T>
static int tsqr_typed(T *U, int64_t m, int64_t ldu, int k, Workspace &ws, int out_mode, lspca_dtype dt16,
                      T *Q, uint16_t *Qh, uint16_t *Ql, int64_t ldq, hipStream_t s) {
  constexpr int BR = TsqrCfg<T>::BR;
  if (k > BR) {
    set_error("spca_fit: k = %d exceeds the QR block height %d for this type", k, BR);
    return LSPCA_ENOTSUP;
  }
  const int64_t nb = (m + BR - 1) / BR;
  if (nb > 0x7fffffff) {
    set_error("spca_fit: too many QR blocks");
    return LSPCA_EINVAL;
  }
  if (ldu < nb * BR) {
    set_error("tsqr: leading dimension %lld below %lld", (long long)ldu, (long long)(nb * BR));
    return LSPCA_EINVAL;
  }
  const int64_t kb = (int64_t)k * BR;
  std::vector<int64_t> counts{nb};
  while (counts.back() > 1) counts.push_back((counts.back() + 1) / 2);
  const size_t L = counts.size();
  std::vector<T *> R(L), C(L), tau(L), Vb(L, nullptr);
  for (size_t l = 0; l < L; ++l) {
    R[l] = ws.take<T>((size_t)counts[l] * kb);
    C[l] = ws.take<T>((size_t)counts[l] * kb);
    tau[l] = ws.take<T>((size_t)counts[l] * k);
    if (l) Vb[l] = ws.take<T>((size_t)counts[l] * kb);
  }
  hipLaunchKernelGGL((k_tsqr_leaf<T>), (unsigned)nb, 1024, 0, s, U, ldu, m, k, tau[0], R[0]);
  LSPCA_HIP(hipGetLastError());
  for (size_t l = 1; l < L; ++l) {
    hipLaunchKernelGGL((k_tsqr_node<T>), (unsigned)counts[l], 1024, 0, s, R[l - 1], (int)counts[l - 1], k, R[l],
                       Vb[l], tau[l]);
    LSPCA_HIP(hipGetLastError());
  }
  // top-down: C at the root is the identity
  hipLaunchKernelGGL((k_eye_slices<T>), (unsigned)((kb + 255) / 256), 256, 0, s, C[L - 1], k);
  LSPCA_HIP(hipGetLastError());
  for (size_t l = L - 1; l >= 1; --l) {
    hipLaunchKernelGGL((k_tsqr_node_q<T>), (unsigned)counts[l], 1024, 0, s, C[l], (int)counts[l - 1], k, Vb[l],
                       tau[l], C[l - 1]);
    LSPCA_HIP(hipGetLastError());
  }
  if (out_mode == 0)
    hipLaunchKernelGGL((k_tsqr_leaf_q<T, 0, LSPCA_BF16>), (unsigned)nb, 1024, 0, s, U, ldu, m, k, tau[0], C[0], Q,
                       ldq, nullptr, nullptr);
  else if (dt16 == LSPCA_BF16)
    hipLaunchKernelGGL((k_tsqr_leaf_q<T, 1, LSPCA_BF16>), (unsigned)nb, 1024, 0, s, U, ldu, m, k, tau[0], C[0], Q,
                       ldq, Qh, Ql);
  else
    hipLaunchKernelGGL((k_tsqr_leaf_q<T, 1, LSPCA_F16>), (unsigned)nb, 1024, 0, s, U, ldu, m, k, tau[0], C[0], Q,
                       ldq, Qh, Ql);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// ------------------------------------------------------------- R only --
// The R factor of U (m x k) without Q: leaves and tree, no reflectors kept.
// U row-major (ldu = row stride) or transposed (column c at U + c * ldu).
// The root R (slice order, k x BR entries of the type) goes to Rroot.
size_t tsqr_r_workspace_bytes(int64_t m, int k, lspca_dtype ydt) {
  const size_t es = ydt == LSPCA_F64 ? 8 : 4;
  const int BR = tsqr_br(ydt);
  int64_t level = (m + BR - 1) / BR;
  size_t total = 0;
  while (true) {
    total += ws_bytes<char>(es * (size_t)level * k * BR);
    if (level == 1) break;
    level = (level + 1) / 2;
  }
  return total + 4096;
}

template <typename T>
static int tsqr_r_typed(const T *U, int64_t m, int64_t ldu, bool rowmajor, int k, Workspace &ws, T *Rroot,
                        hipStream_t s) {
  constexpr int BR = TsqrCfg<T>::BR;
  if (k > BR) {
    set_error("QR: k = %d exceeds the block height %d for this type", k, BR);
    return LSPCA_ENOTSUP;
  }
  const int64_t nb = (m + BR - 1) / BR, kb = (int64_t)k * BR;
  std::vector<int64_t> counts{nb};
  while (counts.back() > 1) counts.push_back((counts.back() + 1) / 2);
  std::vector<T *> R(counts.size());
  for (size_t l = 0; l < counts.size(); ++l) R[l] = ws.take<T>((size_t)counts[l] * kb);
  if (rowmajor)
    hipLaunchKernelGGL((k_tsqr_leaf<T, true, false>), (unsigned)nb, 1024, 0, s, const_cast<T *>(U), ldu, m, k,
                       nullptr, R[0]);
  else
    hipLaunchKernelGGL((k_tsqr_leaf<T, false, false>), (unsigned)nb, 1024, 0, s, const_cast<T *>(U), ldu, m, k,
                       nullptr, R[0]);
  LSPCA_HIP(hipGetLastError());
  for (size_t l = 1; l < counts.size(); ++l) {
    hipLaunchKernelGGL((k_tsqr_node<T, false>), (unsigned)counts[l], 1024, 0, s, R[l - 1], (int)counts[l - 1], k,
                       R[l], nullptr, nullptr);
    LSPCA_HIP(hipGetLastError());
  }
  LSPCA_HIP(hipMemcpyAsync(Rroot, R.back(), (size_t)kb * sizeof(T), hipMemcpyDeviceToDevice, s));
  return LSPCA_OK;
}

int tsqr_r(const void *U, lspca_dtype ydt, int64_t m, int64_t ldu, bool rowmajor, int k, Workspace &ws,
           void *Rroot, hipStream_t s) {
  if (ydt == LSPCA_F64)
    return tsqr_r_typed<double>((const double *)U, m, ldu, rowmajor, k, ws, (double *)Rroot, s);
  return tsqr_r_typed<float>((const float *)U, m, ldu, rowmajor, k, ws, (float *)Rroot, s);
}

// R of [R_a; R_b] for the two slice-order R factors stored back to back at
// Rpair; result to Rout (slice order).
int tsqr_r_merge(const void *Rpair, lspca_dtype ydt, int k, void *Rout, hipStream_t s) {
  if (ydt == LSPCA_F64)
    hipLaunchKernelGGL((k_tsqr_node<double, false>), 1, 1024, 0, s, (const double *)Rpair, 2, k, (double *)Rout,
                       nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_tsqr_node<float, false>), 1, 1024, 0, s, (const float *)Rpair, 2, k, (float *)Rout,
                       nullptr, nullptr);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

template <typename T> __global__ void k_slice_to_dense(const T *__restrict__ Rs, int k, double *__restrict__ Rd) {
  constexpr int BR = TsqrCfg<T>::BR;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * k) return;
  const int r = (int)(e / k), c = (int)(e % k);
  Rd[e] = r <= c ? (double)Rs[(int64_t)c * BR + spos<T>(r)] : 0.0;
}

// Dense k x k row-major FP64 copy of a slice-order R (zeros below).
int tsqr_r_dense(const void *Rslice, lspca_dtype ydt, int k, double *Rd, hipStream_t s) {
  const unsigned grid = (unsigned)(((int64_t)k * k + 255) / 256);
  if (ydt == LSPCA_F64)
    hipLaunchKernelGGL(k_slice_to_dense<double>, grid, 256, 0, s, (const double *)Rslice, k, Rd);
  else
    hipLaunchKernelGGL(k_slice_to_dense<float>, grid, 256, 0, s, (const float *)Rslice, k, Rd);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// Ut: U transposed (column c of U at Ut + c * ldu, ldu >= tsqr_ld(m)),
// FP32 or FP64 as ydt; overwritten by the leaves' reflectors. out_mode 0:
// Q (m x k, row-major, ydt, leading dimension ldq) in Q; out_mode 1: Q^T
// split into 16-bit parts of type dt16 in Qh, Ql (k x m, leading dimension
// ldq).
int tsqr(void *Ut, lspca_dtype ydt, int64_t m, int64_t ldu, int k, Workspace &ws, int out_mode,
         lspca_dtype dt16, void *Q, void *Qh, void *Ql, int64_t ldq, hipStream_t s) {
  if (ydt == LSPCA_F64)
    return tsqr_typed<double>((double *)Ut, m, ldu, k, ws, out_mode, dt16, (double *)Q, (uint16_t *)Qh,
                              (uint16_t *)Ql, ldq, s);
  return tsqr_typed<float>((float *)Ut, m, ldu, k, ws, out_mode, dt16, (float *)Q, (uint16_t *)Qh,
                           (uint16_t *)Ql, ldq, s);
}

}  // namespace lspca
