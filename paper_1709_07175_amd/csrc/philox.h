// Device-side Philox4x32-10 and the Omega entry mappings (see omega.hip and
// the Omega specification in include/lspca.h). Header so that the sparse
// sketch kernels can regenerate Omega's nonzeros where they need them.
#pragma once
#include "common.h"

namespace lspca {

constexpr uint32_t kTagGaussian = 0x47415553u;
constexpr uint32_t kTagSparse = 0x53505253u;

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                              uint32_t c3, uint32_t k0, uint32_t k1,
                                              uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t lo0 = M0 * c0, hi0 = __umulhi(M0, c0);
    const uint32_t lo1 = M1 * c2, hi1 = __umulhi(M1, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// Box-Muller pair for Omega[j][2q], Omega[j][2q+1] (FP64).
__device__ __forceinline__ void gaussian_pair(uint32_t key0, uint32_t key1, uint64_t j,
                                              uint32_t q, double &z0, double &z1) {
  uint32_t x[4];
  philox4x32_10(q, (uint32_t)j, (uint32_t)(j >> 32), kTagGaussian, key0, key1, x);
  const uint64_t a = (((uint64_t)x[1] << 32) | x[0]) >> 11;
  const uint64_t b = (((uint64_t)x[3] << 32) | x[2]) >> 11;
  const double u1 = (double)a * 0x1p-53 + 0x1p-54;
  const double u2 = (double)b * 0x1p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double th = 2.0 * 3.141592653589793 * u2;
  z0 = r * cos(th);
  z1 = r * sin(th);
}

// Very sparse entry from one 32-bit word: +1 below t_plus = 2^32/(2p),
// -1 below t_minus = 2^32/p, else 0.
__device__ __forceinline__ double sparse_value(uint32_t x, uint32_t t_plus, uint64_t t_minus) {
  return x < t_plus ? 1.0 : ((uint64_t)x < t_minus ? -1.0 : 0.0);
}

}  // namespace lspca
