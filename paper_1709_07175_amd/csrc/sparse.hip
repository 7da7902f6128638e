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
#include <cstring>

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
        // Y is written as FP32 transposed, Yt[c][r] (Y != NULL, ldy = rows of
        // the stripe), or split into 16-bit parts Yh, Yl in 8-row blocks
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
          // in 8-row blocks of k columns (r0 % 8 is 0 or 4)
          const int64_t ob = ((r0 >> 3) * k + c) * 8 + (r0 & 7);
          uint16_t *dh = Yh + ob;
          uint16_t *dl = Yl ? Yl + ob : nullptr;
          if (r0 + 3 < m) {
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

// ---------------------------------------------------------------------------
// Register-list variant: tiles of 8 rows, 1024 threads. Lane (c, q) owns
// output column c and one of LPC parts of its work: parts 0..LPC/2-1 take the
// column's +1 entries (ascending j, cut by position into runs of Lq entries),
// the other parts its -1 entries. A lane keeps the LDS addresses of its run in
// registers for the whole launch, so the step loop reads only X: one 16-byte
// LDS read (the 8 rows of one feature) and 8 FP32 fmas with the lane's sign.
// The parts are summed in a fixed tree (positives, negatives, then both), so
// the result does not depend on timing. The X tile is double-buffered in LDS:
// the buffers alternate every 16 slots (256 bytes, so a buffer keeps all
// banks and the second is the first plus 256), slots swizzled so that the
// staging writes spread over the banks;
// slot `zslot` holds zeros and pads every run to a whole number of steps.
// Runs longer than the register capacity (a far-tail event for the shapes the
// host admits) switch the workgroup to regenerating Omega on the fly in the
// same order.
constexpr int kGxThreads = 1024;
constexpr int kGxRows = 8;
constexpr int kGxLQ = 40;               // register run capacity, multiple of 4

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int gx_slot(int f) { return f ^ ((f >> 4) & 7); }
// LDS byte address of slot s in buffer 0; buffer 1 is 256 bytes further:
// groups of 16 slots (256 bytes, every bank once) alternate between buffers
__device__ __forceinline__ uint32_t gx_addr(int s) { return (uint32_t)(((s >> 4) * 2) * 256 + (s & 15) * 16); }

typedef __attribute__((address_space(3))) const u32x4 gx_lds_u32x4;
// 16 bytes at an LDS byte address (the kernel has no static LDS, so its
// dynamic LDS starts at address 0; the host checks this)
__device__ __forceinline__ u32x4 gx_read(uint32_t a) { return *(gx_lds_u32x4 *)(uintptr_t)a; }

template <int CTRL> __device__ __forceinline__ float gx_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum (MAX = false) or maximum over the LPC consecutive lanes of a column:
// lane xor 1, xor 2 (quad permutes), then the mirrors within 8 and 16 lanes.
// Every step combines two equal-shaped halves, so all lanes end bitwise equal.
template <int LPC, bool MAX> __device__ __forceinline__ float gx_reduce(float v) {
  auto op = [](float a, float b) { return MAX ? fmaxf(a, b) : a + b; };
  v = op(v, gx_dpp<0xB1>(v));
  v = op(v, gx_dpp<0x4E>(v));
  if (LPC >= 8) v = op(v, gx_dpp<0x141>(v));
  if (LPC >= 16) v = op(v, gx_dpp<0x140>(v));
  return v;
}

// One step: +-x for the 8 rows of a feature (4 dwords, row 2d in the low and
// row 2d+1 in the high half of dword d), each an FP32 fma with s = +-1, i.e.
// one correctly rounded addition. FP16 halves convert inside the fma
// (v_fma_mix_f32); a BF16 half is the FP32 with the same top 16 bits (one
// shift or mask). (The BF16 dot2 instruction would do both in one
// instruction but issues at under half the rate of an fma here and rounds
// its addition only faithfully.)
template <int DT>
__device__ __forceinline__ void gx_step(u32x4 xv, float s, float (&acc)[kGxRows]) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    float lo, hi;
    if (DT == LSPCA_BF16) {
      lo = __uint_as_float(xv[d] << 16);
      hi = __uint_as_float(xv[d] & 0xffff0000u);
    } else {
      lo = f16_bits_to_f32((uint16_t)xv[d]);
      hi = f16_bits_to_f32((uint16_t)(xv[d] >> 16));
    }
    acc[2 * d] = fmaf(lo, s, acc[2 * d]);
    acc[2 * d + 1] = fmaf(hi, s, acc[2 * d + 1]);
  }
}

// The run of one lane over buffer BUF in blocks of 4 steps (lq rounded up;
// the padding addresses past the run point at the zero slot): a step's
// registers are refilled with the read 4 steps ahead right after they are
// taken, so 4 reads stay in flight (reading ahead is always in bounds).
template <int DT, int BUF>
__device__ __forceinline__ void gx_run(const uint32_t (&ent)[kGxLQ], int lq, float sg, float (&acc)[kGxRows]) {
  u32x4 buf[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) buf[t] = gx_read(ent[t] + 256 * BUF);
#pragma unroll
  for (int b = 0; b < kGxLQ / 4; ++b) {
    if (4 * b >= lq) break;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const u32x4 x = buf[t];
      if (b + 1 < kGxLQ / 4) buf[t] = gx_read(ent[4 * b + 4 + t] + 256 * BUF);
      gx_step<DT>(x, sg, acc);
    }
  }
  // A use of the last read-ahead on the way out (never taken: lq >= 0) keeps
  // the compiler from sinking each block's read-ahead below its exit test.
  if (lq < 0) acc[0] = __uint_as_float(buf[0][0] ^ buf[1][1] ^ buf[2][2] ^ buf[3][3]);
}

// Sum of the LPC parts of a column, scattered: a lane keeps half of its
// values and adds its partner's copy of them (lane xor 1, xor 2, then the
// mirrors within 8 and 16 lanes). The half a lane keeps at each step is
// chosen so that the partners of the next step hold the same rows. Parts
// 0..LPC/2-1 (+1 entries) meet first, then the two signs. Afterwards lane q
// holds rows row0, row0 + 1 (LPC = 4) or row row0 (LPC = 8, 16; for 16 the
// lanes q and 15 - q both hold it).
template <int LPC>
__device__ __forceinline__ void gx_scatter(float (&v)[kGxRows], int q, int &row0) {
  const int b0 = q & 1, b1 = (q >> 1) & 1, b2 = (q >> 2) & 1, b3 = (q >> 3) & 1;
  const bool k1 = LPC == 4 ? b0 : (b0 ^ b2);
  const bool k2 = LPC == 4 ? b1 : (b1 ^ b2);
  const bool k3 = LPC == 8 ? b2 : (b2 ^ b3);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float keep = k1 ? v[i + 4] : v[i], send = k1 ? v[i] : v[i + 4];
    v[i] = keep + gx_dpp<0xB1>(send);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = k2 ? v[i + 2] : v[i], send = k2 ? v[i] : v[i + 2];
    v[i] = keep + gx_dpp<0x4E>(send);
  }
  row0 = 4 * k1 + 2 * k2;
  if (LPC >= 8) {
    const float keep = k3 ? v[1] : v[0], send = k3 ? v[0] : v[1];
    v[0] = keep + gx_dpp<0x141>(send);
    row0 += k3;
  }
  if (LPC >= 16) v[0] = v[0] + gx_dpp<0x140>(v[0]);
}

// Dynamic LDS: generation [ counts: 2k ints | max run | buckets: 2k x CAP
// 16-bit ], then reused as the two interleaved X buffers ((8 ceil(n/8) + 1)
// slots x 32 bytes). tiles_per_wg consecutive 8-row tiles per workgroup, so
// the transposed outputs of neighbouring tiles are written from one CU.
// VEC: n and ldx multiples of 8 and X 16-byte aligned (16-byte row loads).
template <int DT, int LPC, bool VEC>
__global__ __launch_bounds__(kGxThreads) void k_sparse_sketch_reg(
    const uint16_t *__restrict__ X, int64_t m, int n, int64_t ldx, int k, uint32_t key0,
    uint32_t key1, uint32_t t_plus, uint64_t t_minus, int lq_cap, int64_t tiles_per_wg,
    float *__restrict__ Y, int64_t ldy, unsigned *__restrict__ colmax, uint16_t *__restrict__ Yh,
    uint16_t *__restrict__ Yl, int *__restrict__ overflow) {
  constexpr int HALF = LPC / 2;
  constexpr int CAP = HALF * kGxLQ;                // bucket capacity per (column, sign)
  extern __shared__ __align__(16) unsigned char lds[];
  const int tid = threadIdx.x;
  const int col = tid / LPC, q = tid % LPC;
  const int sgn = q / HALF, part = q % HALF;
  const bool live = col < k;
  const int ngroups = (n + 7) >> 3;
  const int zslot = ngroups * 8;
  const int qk = (k + 3) >> 2;

  // ---- Omega's nonzeros per (column, sign): count, bucket, sort by j
  int *cnt = (int *)lds;
  int *lqmax = cnt + 2 * k;
  uint16_t *bucket = (uint16_t *)(lds + ((8 * k + 4 + 15) & ~15));
  for (int i = tid; i < 2 * k; i += kGxThreads) cnt[i] = 0;
  if (tid == 0) *lqmax = 0;
  __syncthreads();
  const int calls = n * qk;
  for (int idx = tid; idx < calls; idx += kGxThreads) {
    const int j = idx / qk, q4 = idx - j * qk;
    uint32_t x[4];
    philox4x32_10((uint32_t)q4, (uint32_t)j, 0u, kTagSparse, key0, key1, x);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 4 * q4 + t;
      if (c < k && (uint64_t)x[t] < t_minus) {
        const int b = 2 * c + (x[t] < t_plus ? 0 : 1);
        const int pos = atomicAdd(&cnt[b], 1);
        if (pos < CAP) bucket[b * CAP + pos] = (uint16_t)j;
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < 2 * k; i += kGxThreads) atomicMax(lqmax, (cnt[i] + HALF - 1) / HALF);
  __syncthreads();
  const int lq = *lqmax;
  const bool fits = lq <= kGxLQ && lq <= lq_cap;
  if (!fits && tid == 0) atomicOr(overflow, 1);
  for (int b = tid; fits && b < 2 * k; b += kGxThreads) {
    uint16_t *e = bucket + b * CAP;
    const int len = cnt[b];
    for (int i = 1; i < len; ++i) {
      const uint16_t v = e[i];
      int t = i - 1;
      while (t >= 0 && e[t] > v) {
        e[t + 1] = e[t];
        --t;
      }
      e[t + 1] = v;
    }
  }
  __syncthreads();
  uint32_t ent[kGxLQ];
  {
    const int b = 2 * col + sgn;
    const int len = live ? cnt[b] : 0;
#pragma unroll
    for (int st = 0; st < kGxLQ; ++st) {
      const int i = part * lq + st;
      int slot = zslot;
      if (fits && st < lq && i < len) slot = gx_slot(bucket[b * CAP + i]);
      ent[st] = gx_addr(slot);
      // hide the alignment of the address, so that + 256 (the second buffer)
      // stays an add and folds into the read's offset field
      asm volatile("" : "+v"(ent[st]));
    }
  }
  __syncthreads();                                 // the X buffers overwrite the buckets

  // ---- 8-row tiles
  const int64_t ntiles = (m + kGxRows - 1) / kGxRows;
  const int64_t t0 = (int64_t)blockIdx.x * tiles_per_wg;
  const int64_t t1 = t0 + tiles_per_wg < ntiles ? t0 + tiles_per_wg : ntiles;
  if (tid < 2) *(u32x4 *)(lds + gx_addr(zslot) + 256 * tid) = u32x4{0u, 0u, 0u, 0u};
  // staging: thread = feature group g (8 features) x row half h (4 rows);
  // 2 ceil(n/8) <= 1024 units (the host admits n <= 4096)
  const int ug = tid % ngroups, uh = tid / ngroups;      // uh >= 2: idle
  u16x8 v[4];
  auto load = [&](int64_t tile) {
    const int64_t r0 = tile * kGxRows;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (VEC) {
        // one unconditional 16-byte load per row, the row clamped into X:
        // rows past m only feed their own (unwritten) outputs, and a load
        // with no branch around it stays in flight through the compute
        int64_t row = r0 + 4 * (uh < 2 ? uh : 1) + r;
        row = row < m ? row : m - 1;
        v[r] = *(const u16x8 *)(X + row * ldx + 8 * ug);
      } else {
        const int64_t row = r0 + 4 * uh + r;
        u16x8 x = {};
        if (uh < 2 && row < m) {
          const uint16_t *src = X + row * ldx + 8 * ug;
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = 8 * ug + e < n ? src[e] : (uint16_t)0;
        }
        v[r] = x;
      }
    }
  };
  auto store = [&](int buf) {
    if (uh >= 2) return;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const u16x4 w = {v[0][e], v[1][e], v[2][e], v[3][e]};
      *(u16x4 *)(lds + gx_addr(gx_slot(8 * ug + e)) + 256 * buf + 8 * uh) = w;
    }
  };
  const float sg = sgn ? -1.f : 1.f;
  float amax = 0.f;
  if (t0 < t1) {
    load(t0);
    store(0);
  }
  __syncthreads();
  for (int64_t tile = t0; tile < t1; ++tile) {
    const int buf = (int)((tile - t0) & 1);
    if (tile + 1 < t1) load(tile + 1);
    float acc[kGxRows];
#pragma unroll
    for (int r = 0; r < kGxRows; ++r) acc[r] = 0.f;
    if (fits) {
      // the run length made opaque per tile (it is uniform: an SGPR), so
      // the block exit tests are made where they are used instead of being
      // hoisted out of the tile loop into spilled masks
      int lqt = lq;
      asm volatile("" : "+s"(lqt));
      if (buf == 0) gx_run<DT, 0>(ent, lqt, sg, acc);
      else gx_run<DT, 1>(ent, lqt, sg, acc);
    } else if (live) {
      // on the fly, same entries in the same order as the run
      const int lo = part * lq, hi = lo + lq;
      int rank = 0;
      for (int j = 0; j < n && rank < hi; ++j) {
        uint32_t x[4];
        philox4x32_10((uint32_t)(col >> 2), (uint32_t)j, 0u, kTagSparse, key0, key1, x);
        const uint32_t w = (col & 3) == 0 ? x[0] : (col & 3) == 1 ? x[1] : (col & 3) == 2 ? x[2] : x[3];
        if ((uint64_t)w < t_minus && (w < t_plus ? 0 : 1) == sgn) {
          if (rank >= lo) {
            const u32x4 xv = *(const u32x4 *)(lds + gx_addr(gx_slot(j)) + 256 * buf);
            gx_step<DT>(xv, sg, acc);
          }
          ++rank;
        }
      }
    }
    if (tile + 1 < t1) store(buf ^ 1);
    int row0;
    gx_scatter<LPC>(acc, q, row0);
    const int64_t r0 = tile * kGxRows;
    constexpr int RPL = LPC == 4 ? 2 : 1;
    const bool writer = live && (LPC < 16 || q < 8);
    if (Y) {
      // FP32, transposed: Y[c * ldy + r]
#pragma unroll
      for (int i = 0; i < RPL; ++i)
        if (writer && r0 + row0 + i < m) Y[(int64_t)col * ldy + r0 + row0 + i] = acc[i];
    } else if (writer) {
      // split, in 8-row blocks: the tile's block is k columns x 8 rows, so a
      // wave's stores cover 16 columns x 16 bytes contiguously
      const int64_t o = ((int64_t)tile * k + col) * kGxRows + row0;
      uint16_t hv[RPL], lv[RPL];
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        hv[i] = f2h<DT>(acc[i]);
        lv[i] = f2h<DT>(acc[i] - h2f<DT>(hv[i]));
      }
      if (RPL == 2 && r0 + row0 + 1 < m) {
        *(uint32_t *)(Yh + o) = (uint32_t)hv[0] | ((uint32_t)hv[RPL - 1] << 16);
        if (Yl) *(uint32_t *)(Yl + o) = (uint32_t)lv[0] | ((uint32_t)lv[RPL - 1] << 16);
      } else if (r0 + row0 < m) {
        Yh[o] = hv[0];
        if (Yl) Yl[o] = lv[0];
      }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i)
      if (writer && r0 + row0 + i < m) amax = fmaxf(amax, fabsf(acc[i]));
    __syncthreads();
  }
  if (colmax) {
    amax = gx_reduce<LPC, true>(amax);
    if (live && q == 0) atomicMax(colmax + col, __float_as_uint(amax));
  }
}

// LDS needed for n features and a list capacity of cap entries.
static size_t sparse_lds_bytes(int n, int k, int cap) {
  return (((size_t)n * kSpRows * 2 + 15) & ~(size_t)15) + (size_t)(2 * k + 1) * 4 + (size_t)cap * 2;
}

// Plan of the register-list kernel: lanes per column, LDS bytes.
struct GxPlan {
  int lpc = 0;
  size_t lds = 0;
};

// Chernoff bound on log P(Binomial(n, r) >= x).
static double binom_tail_log(double n, double r, double x) {
  const double a = x / n;
  if (a <= r) return 0.0;
  if (a > 1.0) return -INFINITY;
  if (a == 1.0) return n * log(r);
  return -n * (a * log(a / r) + (1 - a) * log((1 - a) / (1 - r)));
}

// Whether the register-list kernel applies: 16-bit X, n <= 4096, k <= 256,
// and every one of the 2k sign lists (each Binomial(n, 1/(2p)) long) within
// the LPC/2 runs of the registers except with probability below 1e-6 (union
// bound; an overflow costs time, not accuracy: the on-the-fly path gives the
// same bits). LSPCA_SPARSE_KERNEL=lds selects the LDS-list kernel, =reg
// requires this one (test knobs).
static bool gx_plan(lspca_dtype dt, int64_t n, int k, uint32_t p, GxPlan &g) {
  if (dt != LSPCA_BF16 && dt != LSPCA_F16) return false;
  if (n < 1 || n > 4096 || k < 1 || k > 256) return false;
  if (const char *e = getenv("LSPCA_SPARSE_KERNEL"))
    if (!strcmp(e, "lds")) return false;
  g.lpc = k > 128 ? 4 : (k > 64 ? 8 : 16);
  const int cap = g.lpc / 2 * kGxLQ;
  const int64_t ngroups = (n + 7) / 8;
  const size_t xb = (size_t)((8 * ngroups) / 16 * 2 + 2) * 256;   // through the zero slot of buffer 1
  const size_t gen = ((8 * (size_t)k + 4 + 15) & ~(size_t)15) + (size_t)2 * k * cap * 2;
  g.lds = xb > gen ? xb : gen;
  if (g.lds > 160 * 1024) return false;
  return binom_tail_log((double)n, 0.5 / p, cap + 1.0) + log(2.0 * k) <= log(1e-6);
}

// Whether a gather path applies (16-bit X): the register-list kernel, or the
// LDS-list kernel when n < 2^15, k <= 1024 and the expected number of
// nonzeros n k / p with a 10-sigma margin fits its list; *cap_out is that
// list's capacity (0 when only the register kernel applies).
bool sparse_sketch_ok(lspca_dtype dt, int64_t n, int k, uint32_t p, int *cap_out) {
  *cap_out = 0;
  GxPlan g;
  const bool reg = gx_plan(dt, n, k, p, g);
  if (dt != LSPCA_BF16 && dt != LSPCA_F16) return false;
  if (n >= 32768 || k > 1024) return reg;
  const size_t budget = 160 * 1024;
  const size_t fixed = sparse_lds_bytes((int)n, k, 0);
  if (fixed >= budget) return reg;
  const double mu = (double)n * k / p;                 // expected nonzeros
  const double want = mu + 10.0 * sqrt(mu) + 64;       // 10 sigma margin
  const double room = (double)(budget - fixed) / 2;
  if (want > room) return reg;
  *cap_out = ((int)want + 63) & ~63;
  // test hook: a smaller capacity forces the on-the-fly fallback
  if (const char *e = getenv("LSPCA_SPARSE_CAP")) *cap_out = atoi(e);
  return true;
}

template <int DT, int LPC, bool VEC>
static int launch_reg(const GxPlan &g, unsigned grid, const void *X, int64_t m, int64_t n, int64_t ldx,
                      int k, uint32_t key0, uint32_t key1, uint32_t t_plus, uint64_t t_minus, int lq_cap,
                      int64_t per, float *Y, int64_t ldy, unsigned *colmax, void *Yh, void *Yl,
                      int *overflow, hipStream_t s) {
  const void *fn = (const void *)k_sparse_sketch_reg<DT, LPC, VEC>;
  hipFuncAttributes fa;
  LSPCA_HIP(hipFuncGetAttributes(&fa, fn));
  if (fa.sharedSizeBytes != 0) {           // LDS addresses assume dynamic LDS at 0
    set_error("sparse sketch: unexpected static LDS (%zu bytes)", (size_t)fa.sharedSizeBytes);
    return LSPCA_EINVAL;
  }
  LSPCA_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds));
  hipLaunchKernelGGL((k_sparse_sketch_reg<DT, LPC, VEC>), grid, kGxThreads, g.lds, s, (const uint16_t *)X, m,
                     (int)n, ldx, k, key0, key1, t_plus, t_minus, lq_cap, per, Y, ldy, colmax,
                     (uint16_t *)Yh, (uint16_t *)Yl, overflow);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

template <int DT>
static int launch_reg_dt(const GxPlan &g, unsigned grid, const void *X, int64_t m, int64_t n, int64_t ldx,
                         int k, uint32_t key0, uint32_t key1, uint32_t t_plus, uint64_t t_minus, int lq_cap,
                         int64_t per, float *Y, int64_t ldy, unsigned *colmax, void *Yh, void *Yl,
                         int *overflow, hipStream_t s) {
  const bool vec = n % 8 == 0 && ldx % 8 == 0 && (uintptr_t)X % 16 == 0;
#define LSPCA_GX(L, V)                                                                                     \
  if (g.lpc == L && vec == V)                                                                              \
    return launch_reg<DT, L, V>(g, grid, X, m, n, ldx, k, key0, key1, t_plus, t_minus, lq_cap, per, Y, ldy, \
                                colmax, Yh, Yl, overflow, s);
  LSPCA_GX(4, true) LSPCA_GX(8, true) LSPCA_GX(16, true) LSPCA_GX(4, false) LSPCA_GX(8, false)
  LSPCA_GX(16, false)
#undef LSPCA_GX
  set_error("sparse sketch: no kernel for %d lanes per column", g.lpc);
  return LSPCA_EINVAL;
}

int launch_sparse_sketch(lspca_dtype dt, const void *X, int64_t m, int64_t n, int64_t ldx, int k,
                         uint64_t seed, uint32_t p, int cap, float *Y, int64_t ldy,
                         unsigned *colmax, void *Yh, void *Yl, int *overflow, hipStream_t s) {
  const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
  const uint32_t t_plus = (uint32_t)((1ull << 32) / (2ull * p));
  const uint64_t t_minus = (1ull << 32) / (uint64_t)p;
  if (m <= 0) return LSPCA_OK;
  int dev = 0, cus = 256;
  LSPCA_HIP(hipGetDevice(&dev));
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  GxPlan g;
  if (gx_plan(dt, n, k, p, g)) {
    // one workgroup per CU, each on a contiguous range of 8-row tiles;
    // LSPCA_SPARSE_LQ lowers the register run capacity (a test knob that
    // forces the on-the-fly fallback)
    int lq_cap = kGxLQ;
    if (const char *e = getenv("LSPCA_SPARSE_LQ")) lq_cap = atoi(e);
    const int64_t ntiles = (m + kGxRows - 1) / kGxRows;
    const int64_t g0 = ntiles < cus ? ntiles : cus;
    const int64_t per = (ntiles + g0 - 1) / g0;
    const unsigned grid = (unsigned)((ntiles + per - 1) / per);
    if (dt == LSPCA_BF16)
      return launch_reg_dt<LSPCA_BF16>(g, grid, X, m, n, ldx, k, key0, key1, t_plus, t_minus, lq_cap, per, Y,
                                       ldy, colmax, Yh, Yl, overflow, s);
    return launch_reg_dt<LSPCA_F16>(g, grid, X, m, n, ldx, k, key0, key1, t_plus, t_minus, lq_cap, per, Y, ldy,
                                    colmax, Yh, Yl, overflow, s);
  }
  const char *knob = getenv("LSPCA_SPARSE_KERNEL");
  if (cap <= 0 || (knob && !strcmp(knob, "reg"))) {
    set_error("sparse sketch: shape (n=%lld, k=%d, p=%u) not supported", (long long)n, k, p);
    return LSPCA_EINVAL;
  }
  const size_t lds = sparse_lds_bytes((int)n, k, cap);
  const int64_t ntiles = (m + kSpRows - 1) / kSpRows;
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
