// Random test matrix Omega of eq. (rp), Sec. I-A: Gaussian N(0,1) entries or
// very sparse {-1, 0, +1} entries with probabilities {1/(2p), 1-1/p, 1/(2p)}.
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64-bit
// multiplies by M0 = 0xD2511F53 and M1 = 0xCD9E8D57 with the key bumped by
// the Weyl constants W0 = 0x9E3779B9, W1 = 0xBB67AE85 between rounds.
// The counter/key layout and the Box-Muller mapping are the ones stated in
// include/lspca.h.
#include "philox.h"

namespace lspca {

template <typename OutT> __device__ inline void put(void *out, int64_t idx, double v);
template <> __device__ inline void put<double>(void *out, int64_t idx, double v) {
  ((double *)out)[idx] = v;
}
template <> __device__ inline void put<float>(void *out, int64_t idx, double v) {
  ((float *)out)[idx] = (float)v;
}
template <> __device__ inline void put<bf16_t>(void *out, int64_t idx, double v) {
  ((uint16_t *)out)[idx] = f32_to_bf16_bits((float)v);
}
template <> __device__ inline void put<f16_t>(void *out, int64_t idx, double v) {
  ((uint16_t *)out)[idx] = f32_to_f16_bits((float)v);
}
// FP64 storage of the value the given type holds (for FP64 products with
// the exact Omega a lower-precision pass used).
struct f64_of_f32 {};
struct f64_of_bf16 {};
struct f64_of_f16 {};
template <> __device__ inline void put<f64_of_f32>(void *out, int64_t idx, double v) {
  ((double *)out)[idx] = (double)(float)v;
}
template <> __device__ inline void put<f64_of_bf16>(void *out, int64_t idx, double v) {
  ((double *)out)[idx] = (double)bf16_bits_to_f32(f32_to_bf16_bits((float)v));
}
template <> __device__ inline void put<f64_of_f16>(void *out, int64_t idx, double v) {
  ((double *)out)[idx] = (double)f16_bits_to_f32(f32_to_f16_bits((float)v));
}

// One thread per (row j, column block q): Gaussian blocks hold 2 columns,
// sparse blocks 4. out[j*ld_j + c*ld_c].
template <typename OutT>
__global__ void k_omega(int64_t n, int k, int kind, uint32_t key0, uint32_t key1,
                        uint32_t t_plus, uint64_t t_minus, void *out, int64_t ld_j,
                        int64_t ld_c) {
  const int per = kind == LSPCA_OMEGA_GAUSSIAN ? 2 : 4;
  const int64_t blocks = (k + per - 1) / per;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * blocks) return;
  const int64_t j = gid / blocks;
  const uint32_t q = (uint32_t)(gid % blocks);
  if (kind == LSPCA_OMEGA_GAUSSIAN) {
    double z0, z1;
    gaussian_pair(key0, key1, (uint64_t)j, q, z0, z1);
    int c = 2 * q;
    put<OutT>(out, j * ld_j + (int64_t)c * ld_c, z0);
    if (c + 1 < k) put<OutT>(out, j * ld_j + (int64_t)(c + 1) * ld_c, z1);
  } else {
    uint32_t x[4];
    philox4x32_10(q, (uint32_t)j, (uint32_t)((uint64_t)j >> 32), kTagSparse, key0, key1, x);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      int c = 4 * q + t;
      if (c < k) put<OutT>(out, j * ld_j + (int64_t)c * ld_c, sparse_value(x[t], t_plus, t_minus));
    }
  }
}

int launch_omega(int64_t n, int k, int kind, uint64_t seed, uint32_t p, lspca_dtype dt,
                 void *out, int64_t ld_j, int64_t ld_c, hipStream_t s, int f64_of) {
  const int per = kind == LSPCA_OMEGA_GAUSSIAN ? 2 : 4;
  const int64_t total = n * ((k + per - 1) / per);
  if (total <= 0) return LSPCA_OK;
  const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
  const uint32_t t_plus = (uint32_t)((1ull << 32) / (2ull * p));
  const uint64_t t_minus = (1ull << 32) / (uint64_t)p;
  const int threads = 256;
  const unsigned grid = (unsigned)((total + threads - 1) / threads);
  if (dt == LSPCA_F64 && f64_of != LSPCA_F64) {
    switch (f64_of) {
      case LSPCA_F32:
        hipLaunchKernelGGL(k_omega<f64_of_f32>, grid, threads, 0, s, n, k, kind, key0, key1, t_plus, t_minus, out, ld_j, ld_c);
        break;
      case LSPCA_BF16:
        hipLaunchKernelGGL(k_omega<f64_of_bf16>, grid, threads, 0, s, n, k, kind, key0, key1, t_plus, t_minus, out, ld_j, ld_c);
        break;
      default:
        hipLaunchKernelGGL(k_omega<f64_of_f16>, grid, threads, 0, s, n, k, kind, key0, key1, t_plus, t_minus, out, ld_j, ld_c);
        break;
    }
    LSPCA_HIP(hipGetLastError());
    return LSPCA_OK;
  }
  switch (dt) {
    case LSPCA_F64:
      hipLaunchKernelGGL(k_omega<double>, grid, threads, 0, s, n, k, kind, key0, key1, t_plus, t_minus, out, ld_j, ld_c);
      break;
    case LSPCA_F32:
      hipLaunchKernelGGL(k_omega<float>, grid, threads, 0, s, n, k, kind, key0, key1, t_plus, t_minus, out, ld_j, ld_c);
      break;
    case LSPCA_BF16:
      hipLaunchKernelGGL(k_omega<bf16_t>, grid, threads, 0, s, n, k, kind, key0, key1, t_plus, t_minus, out, ld_j, ld_c);
      break;
    case LSPCA_F16:
      hipLaunchKernelGGL(k_omega<f16_t>, grid, threads, 0, s, n, k, kind, key0, key1, t_plus, t_minus, out, ld_j, ld_c);
      break;
    default:
      set_error("omega: bad dtype %d", (int)dt);
      return LSPCA_EINVAL;
  }
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

}  // namespace lspca
