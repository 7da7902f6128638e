// Operand preparation for the projection Z = X V (eq. (dim_reduction_maps)):
// V (n x k, FP64) is written transposed (k x n, K-contiguous for the nt
// product) in the type of X. For 16-bit X it is split into two parts,
// V = V_hi + V_lo with V_hi = rn(V) and V_lo = rn(V - V_hi), so that two
// 16-bit products into one FP32 accumulator carry about twice the bits.
#include "common.h"

namespace lspca {

template <int DT>
__global__ void k_convert_vt(const double *__restrict__ V, int64_t n, int k, void *hi, void *lo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int c = (int)(e / n);
  const int64_t j = e % n;
  const double v = V[j * k + c];
  if constexpr (DT == LSPCA_F64) {
    ((double *)hi)[e] = v;
  } else if constexpr (DT == LSPCA_F32) {
    ((float *)hi)[e] = (float)v;
  } else if constexpr (DT == LSPCA_BF16) {
    const float f = (float)v;
    const uint16_t h = f32_to_bf16_bits(f);
    ((uint16_t *)hi)[e] = h;
    if (lo) ((uint16_t *)lo)[e] = f32_to_bf16_bits(f - bf16_bits_to_f32(h));
  } else {
    const float f = (float)v;
    const uint16_t h = f32_to_f16_bits(f);
    ((uint16_t *)hi)[e] = h;
    if (lo) ((uint16_t *)lo)[e] = f32_to_f16_bits(f - f16_bits_to_f32(h));
  }
}

int launch_convert_vt(const double *V, int64_t n, int k, lspca_dtype dt, void *hi, void *lo,
                      hipStream_t s) {
  const int64_t total = n * k;
  const unsigned grid = (unsigned)((total + 255) / 256);
  switch (dt) {
    case LSPCA_F64: hipLaunchKernelGGL(k_convert_vt<LSPCA_F64>, grid, 256, 0, s, V, n, k, hi, lo); break;
    case LSPCA_F32: hipLaunchKernelGGL(k_convert_vt<LSPCA_F32>, grid, 256, 0, s, V, n, k, hi, lo); break;
    case LSPCA_BF16: hipLaunchKernelGGL(k_convert_vt<LSPCA_BF16>, grid, 256, 0, s, V, n, k, hi, lo); break;
    case LSPCA_F16: hipLaunchKernelGGL(k_convert_vt<LSPCA_F16>, grid, 256, 0, s, V, n, k, hi, lo); break;
  }
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

}  // namespace lspca
