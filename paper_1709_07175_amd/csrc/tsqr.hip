// Tall-skinny Householder QR of the sketch U = X Omega (m x k) with an
// explicit thin Q: the "Q, R = qr(U)" of Algorithm 1 (SPCA, the non-lazy
// baseline).
//
// Leaves: workgroup b factors rows [b*BR, (b+1)*BR) of U (BR = 256 for FP32,
// 128 for FP64) by k Householder reflectors H_j = I - tau_j v_j v_j^T
// (LAPACK's convention: v_j[j] = 1, H_j x = beta e_j). Four adjacent lanes
// (a quad) own one column, each holding a quarter of its BR entries in
// registers; reflector j is built by the quad that owns column j, broadcast
// through LDS (double buffered: one barrier per reflector) and applied by
// every quad c > j.
// The block is stored back in compact form (R above, v below the
// diagonal); its k x k R goes to level 0 of a binary tree.
// Tree nodes: [R_a; R_b] -> R by reflectors whose top part is e_j and whose
// bottom part v_b has rows 0..j only (R_b upper triangular).
// Q: top down. The root starts from C = I_k; a node maps its C to
// (C_a, C_b) = top and bottom halves of H_0 ... H_{k-1} [C; 0]; a leaf forms
// its BR x k rows of Q = H_0 ... H_{k-1} [C; 0].
#include "common.h"

#include <vector>

namespace lspca {

typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Sum of a value over the four lanes of a quad (lanes 4c .. 4c+3): DPP
// quad_perm xor 1, then xor 2.
template <int CTRL> __device__ inline float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ inline double dpp_f(double v) {
  i32x2 p = __builtin_bit_cast(i32x2, v);
  p.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xF, 0xF, false);
  p.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, p);
}
template <typename T> __device__ inline T quad_sum(T v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  return v;
}

template <typename T> struct TsqrCfg;
template <> struct TsqrCfg<float> { static constexpr int BR = 256; };
template <> struct TsqrCfg<double> { static constexpr int BR = 128; };

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
// Factor one block of U in place (compact form); write tau (k) and the
// block's R (k x k, zeros below the diagonal).
template <typename T>
__global__ __launch_bounds__(1024) void k_tsqr_leaf(T *__restrict__ U, int64_t m, int k, int64_t ldu,
                                                   T *__restrict__ tau_out, T *__restrict__ R_out) {
  constexpr int BR = TsqrCfg<T>::BR, H = BR / 4;
  __shared__ T vl[2][BR];
  __shared__ T tl[2];
  const int tid = threadIdx.x, c = tid >> 2, h = tid & 3;
  const int64_t row0 = (int64_t)blockIdx.x * BR;
  const bool active = c < k;
  T a[H];
  {
    // rows row0 + h*H + i of column c; a full block loads without guards
    const T *p = U + (row0 + h * H) * ldu + c;
    const int64_t left = m - (row0 + h * H);
    if (active && left >= H) {
#pragma unroll
      for (int i = 0; i < H; ++i, p += ldu) a[i] = *p;
    } else {
#pragma unroll
      for (int i = 0; i < H; ++i, p += ldu) a[i] = (active && i < left) ? *p : (T)0;
    }
  }
  T mytau = 0;
  for (int j = 0; j < k; ++j) {
    const int buf = j & 1;
    if (c == j) {
      T s = 0, x0 = 0;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int row = h * H + i;
        s += row > j ? a[i] * a[i] : (T)0;
        x0 += row == j ? a[i] : (T)0;
      }
      s = quad_sum(s);
      x0 = quad_sum(x0);
      T beta, tau, scale;
      householder(x0, s, beta, tau, scale);
      mytau = tau;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int row = h * H + i;
        if (row > j) a[i] *= scale;
        else if (row == j) a[i] = beta;
        vl[buf][row] = row > j ? a[i] : (row == j ? (T)1 : (T)0);
      }
      if (h == 0) tl[buf] = tau;
    }
    __syncthreads();
    if (active && c > j) {
      const T tau = tl[buf];
      T d = 0;
#pragma unroll
      for (int i = 0; i < H; ++i) d += vl[buf][h * H + i] * a[i];
      d = quad_sum(d) * tau;
      asm volatile("" ::: "memory");   // re-read v from LDS: keep it out of registers
#pragma unroll
      for (int i = 0; i < H; ++i) a[i] -= d * vl[buf][h * H + i];
    }
  }
  if (!active) return;
  {
    T *p = U + (row0 + h * H) * ldu + c;
    const int64_t left = m - (row0 + h * H);
    if (left >= H) {
#pragma unroll
      for (int i = 0; i < H; ++i, p += ldu) *p = a[i];
    } else {
#pragma unroll
      for (int i = 0; i < H; ++i, p += ldu)
        if (i < left) *p = a[i];
    }
    T *rp = R_out + (int64_t)blockIdx.x * k * k + (int64_t)(h * H) * k + c;
#pragma unroll
    for (int i = 0; i < H; ++i, rp += k) {
      const int row = h * H + i;
      if (row < k) *rp = row <= c ? a[i] : (T)0;
    }
  }
  if (h == 0) tau_out[(int64_t)blockIdx.x * k + c] = mytau;
}

// ----------------------------------------------------------------- nodes --
// Node p of a level combines R_in[2p] (top) and R_in[2p+1] (bottom) into
// R_out[p]; writes the bottom parts of its reflectors to Vb[p] (column j:
// rows 0..j) and tau[p]. A node without a second child copies R_in[2p].
template <typename T>
__global__ __launch_bounds__(1024) void k_tsqr_node(const T *__restrict__ R_in, int nin, int k,
                                                   T *__restrict__ R_out, T *__restrict__ Vb,
                                                   T *__restrict__ tau_out) {
  constexpr int BR = TsqrCfg<T>::BR, H = BR / 4;
  __shared__ T vl[2][BR];
  __shared__ T tl[2];
  const int tid = threadIdx.x, c = tid >> 2, h = tid & 3;
  const int p = blockIdx.x;
  const int64_t kk = (int64_t)k * k;
  const T *Ra = R_in + (2 * (int64_t)p) * kk;
  T *Rn = R_out + (int64_t)p * kk;
  const bool active = c < k;
  if (2 * p + 1 >= nin) {                         // single child: pass R through
    for (int64_t e = tid; e < kk; e += blockDim.x) Rn[e] = Ra[e];
    for (int e = tid; e < k; e += blockDim.x) tau_out[(int64_t)p * k + e] = 0;
    return;
  }
  const T *Rb = Ra + kk;
  for (int64_t e = tid; e < kk; e += blockDim.x) Rn[e] = Ra[e];
  T b[H];
  {
    const T *p = Rb + (int64_t)(h * H) * k + c;
#pragma unroll
    for (int i = 0; i < H; ++i, p += k) b[i] = (active && h * H + i < k) ? *p : (T)0;
  }
  __syncthreads();                                // Rn complete
  for (int j = 0; j < k; ++j) {
    const int buf = j & 1;
    if (c == j) {
      T s = 0;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int row = h * H + i;
        s += row <= j ? b[i] * b[i] : (T)0;
      }
      s = quad_sum(s);
      const T x0 = Rn[(int64_t)j * k + j];
      T beta, tau, scale;
      householder(x0, s, beta, tau, scale);
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int row = h * H + i;
        const T v = row <= j ? b[i] * scale : (T)0;
        vl[buf][row] = v;
        b[i] = 0;
      }
      {
        T *vp = Vb + (int64_t)p * kk + (int64_t)(h * H) * k + j;
#pragma unroll
        for (int i = 0; i < H; ++i, vp += k)
          if (h * H + i < k) *vp = vl[buf][h * H + i];
      }
      if (h == 0) {
        tl[buf] = tau;
        tau_out[(int64_t)p * k + j] = tau;
        Rn[(int64_t)j * k + j] = beta;
      }
    }
    __syncthreads();
    if (active && c > j) {
      const T tau = tl[buf];
      T d = 0;
#pragma unroll
      for (int i = 0; i < H; ++i) d += vl[buf][h * H + i] * b[i];
      d = quad_sum(d);
      const T w = (Rn[(int64_t)j * k + c] + d) * tau;
      asm volatile("" ::: "memory");
#pragma unroll
      for (int i = 0; i < H; ++i) b[i] -= w * vl[buf][h * H + i];
      if (h == 0) Rn[(int64_t)j * k + c] -= w;
    }
  }
}

// Q formation at a node: C_in[p] (k x k) -> C_out[2p] = top, C_out[2p+1] =
// bottom halves of H_0 ... H_{k-1} [C; 0]. Single child: C passes through.
template <typename T>
__global__ __launch_bounds__(1024) void k_tsqr_node_q(const T *__restrict__ C_in, int nchild, int k,
                                                     const T *__restrict__ Vb,
                                                     const T *__restrict__ tau_in,
                                                     T *__restrict__ C_out) {
  constexpr int BR = TsqrCfg<T>::BR, H = BR / 4;
  constexpr int CH = 16;                          // reflectors per LDS chunk
  __shared__ T vl[CH][BR];
  __shared__ T tl[CH];
  const int tid = threadIdx.x, c = tid >> 2, h = tid & 3;
  const int p = blockIdx.x;
  const int64_t kk = (int64_t)k * k;
  const T *Cn = C_in + (int64_t)p * kk;
  T *Ca = C_out + (2 * (int64_t)p) * kk;
  for (int64_t e = tid; e < kk; e += blockDim.x) Ca[e] = Cn[e];
  if (2 * p + 1 >= nchild) return;
  T *Cb = Ca + kk;
  const bool active = c < k;
  T b[H];
#pragma unroll
  for (int i = 0; i < H; ++i) b[i] = 0;
  __syncthreads();                                // Ca complete
  for (int j1 = k; j1 > 0; j1 -= CH) {
    const int j0 = j1 - CH > 0 ? j1 - CH : 0;
    __syncthreads();
    for (int e = tid; e < (j1 - j0) * BR; e += blockDim.x) {
      const int jj = e / BR, row = e % BR, j = j0 + jj;
      vl[jj][row] = (row <= j && row < k) ? Vb[(int64_t)p * kk + (int64_t)row * k + j] : (T)0;
    }
    for (int e = tid; e < j1 - j0; e += blockDim.x) tl[e] = tau_in[(int64_t)p * k + j0 + e];
    __syncthreads();
    for (int j = j1 - 1; j >= j0; --j) {
      const int jj = j - j0;
      if (active) {
        T d = 0;
#pragma unroll
        for (int i = 0; i < H; ++i) d += vl[jj][h * H + i] * b[i];
        d = quad_sum(d);
        const T w = (Ca[(int64_t)j * k + c] + d) * tl[jj];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < H; ++i) b[i] -= w * vl[jj][h * H + i];
        if (h == 0) Ca[(int64_t)j * k + c] -= w;
      }
      // row j of Ca is read and written by quad c only; no barrier needed
    }
  }
  if (!active) return;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int row = h * H + i;
    if (row < k) Cb[(int64_t)row * k + c] = b[i];
  }
}

// Q formation at a leaf: rows of Q = H_0 ... H_{k-1} [C; 0] for block b.
// OUT 0: Q row-major in T (ldq); OUT 1: Q transposed and split into 16-bit
// parts, Qh[c*ldq + r], Ql[c*ldq + r] (DT the 16-bit type).
template <typename T, int OUT, int DT>
__global__ __launch_bounds__(1024) void k_tsqr_leaf_q(const T *__restrict__ U, int64_t m, int k,
                                                     int64_t ldu, const T *__restrict__ tau_in,
                                                     const T *__restrict__ C_in,
                                                     T *__restrict__ Q, int64_t ldq,
                                                     uint16_t *__restrict__ Qh,
                                                     uint16_t *__restrict__ Ql) {
  constexpr int BR = TsqrCfg<T>::BR, H = BR / 4;
  constexpr int CH = 16;
  __shared__ T vl[CH][BR];
  __shared__ T tl[CH];
  const int tid = threadIdx.x, c = tid >> 2, h = tid & 3;
  const int64_t row0 = (int64_t)blockIdx.x * BR;
  const int64_t kk = (int64_t)k * k;
  const T *C = C_in + (int64_t)blockIdx.x * kk;
  const bool active = c < k;
  T q[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int row = h * H + i;
    q[i] = (active && row < k) ? C[(int64_t)row * k + c] : (T)0;
  }
  for (int j1 = k; j1 > 0; j1 -= CH) {
    const int j0 = j1 - CH > 0 ? j1 - CH : 0;
    __syncthreads();
    // chunk of reflectors j0..j1-1: v_j[row] = 0 (row < j), 1 (row == j),
    // the stored entry below the diagonal
    for (int e = tid; e < (j1 - j0) * BR; e += blockDim.x) {
      const int jj = e / BR, row = e % BR, j = j0 + jj;
      const int64_t r = row0 + row;
      T v = 0;
      if (row == j) v = 1;
      else if (row > j && r < m) v = U[r * ldu + j];
      vl[jj][row] = v;
    }
    for (int e = tid; e < j1 - j0; e += blockDim.x) tl[e] = tau_in[(int64_t)blockIdx.x * k + j0 + e];
    __syncthreads();
    for (int j = j1 - 1; j >= j0; --j) {
      const int jj = j - j0;
      if (active) {
        T d = 0;
#pragma unroll
        for (int i = 0; i < H; ++i) d += vl[jj][h * H + i] * q[i];
        d = quad_sum(d) * tl[jj];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < H; ++i) q[i] -= d * vl[jj][h * H + i];
      }
    }
  }
  if (!active) return;
  if constexpr (OUT == 0) {
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const int64_t r = row0 + h * H + i;
      if (r < m) Q[r * ldq + c] = q[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const int64_t r = row0 + h * H + i;
      if (r < m) {
        const float f = (float)q[i];
        uint16_t hi, lo;
        if constexpr (DT == LSPCA_BF16) {
          hi = __builtin_bit_cast(uint16_t, (__bf16)f);
          lo = __builtin_bit_cast(uint16_t, (__bf16)(f - bf16_bits_to_f32(hi)));
        } else {
          hi = f32_to_f16_bits(f);
          lo = f32_to_f16_bits(f - f16_bits_to_f32(hi));
        }
        Qh[(int64_t)c * ldq + r] = hi;
        Ql[(int64_t)c * ldq + r] = lo;
      }
    }
  }
}

__global__ void k_eye(double *C, int k) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)k * k) C[e] = (e / k == e % k) ? 1.0 : 0.0;
}
__global__ void k_eye_f(float *C, int k) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)k * k) C[e] = (e / k == e % k) ? 1.f : 0.f;
}

// ---------------------------------------------------------------- driver --
static int tsqr_threads(int k) {
  int t = ((4 * k + 63) / 64) * 64;
  return t < 64 ? 64 : t;
}

size_t tsqr_workspace_bytes(int64_t m, int k, lspca_dtype ydt) {
  const size_t es = ydt == LSPCA_F64 ? 8 : 4;
  const int BR = ydt == LSPCA_F64 ? 128 : 256;
  int64_t nb = (m + BR - 1) / BR;
  size_t total = 0;
  int64_t level = nb;
  // R per level, Vb and tau per node level, C per level (top-down)
  while (true) {
    total += 3 * ws_bytes<char>(es * (size_t)level * k * k) + ws_bytes<char>(es * (size_t)level * k);
    if (level == 1) break;
    level = (level + 1) / 2;
  }
  total += ws_bytes<char>(es * (size_t)nb * k);   // leaf tau
  return total + 4096;
}

template <typename T>
static int tsqr_typed(T *U, int64_t m, int k, Workspace &ws, int out_mode, lspca_dtype dt16,
                      T *Q, uint16_t *Qh, uint16_t *Ql, int64_t ldq, hipStream_t s) {
  constexpr int BR = TsqrCfg<T>::BR;
  if (k > BR) {
    set_error("spca_fit: k = %d exceeds the QR block height %d for this type", k, BR);
    return LSPCA_ENOTSUP;
  }
  const int threads = tsqr_threads(k);
  const int64_t kk = (int64_t)k * k;
  std::vector<int64_t> counts;
  int64_t nb = (m + BR - 1) / BR;
  if (nb > 0x7fffffff) {
    set_error("spca_fit: too many QR blocks");
    return LSPCA_EINVAL;
  }
  counts.push_back(nb);
  while (counts.back() > 1) counts.push_back((counts.back() + 1) / 2);
  const size_t L = counts.size();
  std::vector<T *> R(L), Vb(L), tau(L), C(L);
  for (size_t l = 0; l < L; ++l) {
    R[l] = ws.take<T>((size_t)counts[l] * kk);
    Vb[l] = ws.take<T>((size_t)counts[l] * kk);
    tau[l] = ws.take<T>((size_t)counts[l] * k);
    C[l] = ws.take<T>((size_t)counts[l] * kk);
  }
  T *tau_leaf = tau[0];
  hipLaunchKernelGGL(k_tsqr_leaf<T>, (unsigned)nb, threads, 0, s, U, m, k, (int64_t)k, tau_leaf, R[0]);
  LSPCA_HIP(hipGetLastError());
  for (size_t l = 1; l < L; ++l) {
    hipLaunchKernelGGL(k_tsqr_node<T>, (unsigned)counts[l], threads, 0, s, R[l - 1], (int)counts[l - 1], k,
                       R[l], Vb[l], tau[l]);
    LSPCA_HIP(hipGetLastError());
  }
  // top-down: C at the root is the identity
  if constexpr (sizeof(T) == 8)
    hipLaunchKernelGGL(k_eye, (unsigned)((kk + 255) / 256), 256, 0, s, (double *)C[L - 1], k);
  else
    hipLaunchKernelGGL(k_eye_f, (unsigned)((kk + 255) / 256), 256, 0, s, (float *)C[L - 1], k);
  LSPCA_HIP(hipGetLastError());
  for (size_t l = L - 1; l >= 1; --l) {
    hipLaunchKernelGGL(k_tsqr_node_q<T>, (unsigned)counts[l], threads, 0, s, C[l], (int)counts[l - 1], k,
                       Vb[l], tau[l], C[l - 1]);
    LSPCA_HIP(hipGetLastError());
  }
  if (out_mode == 0) {
    hipLaunchKernelGGL((k_tsqr_leaf_q<T, 0, LSPCA_BF16>), (unsigned)nb, threads, 0, s, U, m, k, (int64_t)k,
                       tau_leaf, C[0], Q, ldq, nullptr, nullptr);
  } else if (dt16 == LSPCA_BF16) {
    hipLaunchKernelGGL((k_tsqr_leaf_q<T, 1, LSPCA_BF16>), (unsigned)nb, threads, 0, s, U, m, k, (int64_t)k,
                       tau_leaf, C[0], Q, ldq, Qh, Ql);
  } else {
    hipLaunchKernelGGL((k_tsqr_leaf_q<T, 1, LSPCA_F16>), (unsigned)nb, threads, 0, s, U, m, k, (int64_t)k,
                       tau_leaf, C[0], Q, ldq, Qh, Ql);
  }
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// U (m x k, row-major, FP32 or FP64 as ydt) is overwritten by its compact
// factors. out_mode 0: Q (m x k, row-major, ydt) in Q; out_mode 1: Q^T split
// into 16-bit parts of type dt16 in Qh, Ql (k x m, leading dimension ldq).
int tsqr(void *U, lspca_dtype ydt, int64_t m, int k, Workspace &ws, int out_mode,
         lspca_dtype dt16, void *Q, void *Qh, void *Ql, int64_t ldq, hipStream_t s) {
  if (ydt == LSPCA_F64)
    return tsqr_typed<double>((double *)U, m, k, ws, out_mode, dt16, (double *)Q, (uint16_t *)Qh,
                              (uint16_t *)Ql, ldq, s);
  return tsqr_typed<float>((float *)U, m, k, ws, out_mode, dt16, (float *)Q, (uint16_t *)Qh,
                           (uint16_t *)Ql, ldq, s);
}

}  // namespace lspca
