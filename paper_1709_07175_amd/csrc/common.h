// Internal declarations shared by the library's translation units.
// Not part of the public ABI (that is include/lspca.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

#include "lspca.h"

namespace lspca {

// ------------------------------------------------------------ vector types --
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// 16-bit storage types are moved around as raw bits.
struct bf16_t { uint16_t bits; };
struct f16_t { uint16_t bits; };

// ------------------------------------------------------ rounding helpers --
// FP32 -> BF16, round to nearest even (finite inputs; NaN kept quiet).
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}
__device__ inline uint16_t f32_to_f16_bits(float f) {
  _Float16 h = (_Float16)f;  // v_cvt_f16_f32: round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float f16_bits_to_f32(uint16_t b) {
  return (float)__builtin_bit_cast(_Float16, b);
}

// ------------------------------------------------ direct copies into LDS --
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_cvoid_t;

// One copy instruction; lds_base is wave-uniform. Written as asm: the
// compiler's own waits for such copies are a full vmcnt(0) before every LDS
// read, which would drain the copies in flight; here the kernel waits for
// exactly the copies it needs (wait_vmcnt) before a barrier. The copy has no
// destination register, and its address registers are read at issue. One
// wait state between the M0 write and the copy. M0 is a reserved register
// (hence the silenced warning): in the kernels that use these copies no
// other instruction reads or writes M0 (checked in their assembly), so
// nothing the compiler keeps in it is lost.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void copy16_to_lds(const void *g, uint32_t lds_base) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds_base)
               : "memory", "m0");
}
#pragma clang diagnostic pop
__device__ __forceinline__ uint32_t lds_addr(const void *p) { return (uint32_t)(uintptr_t)(lds_void_t *)p; }

// Waits and barrier as asm statements that clobber memory, so that the
// compiler moves no LDS access across them; the copies into LDS are counted
// by vmcnt (complete once the data is in LDS).
template <int N> __device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ------------------------------------------------------- XCD-aware grid ----
// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with its own L2. For a split-over-rows product launched as a 3-D grid
// (x: column tiles, y: row-of-output tiles, z: row splits), this remaps the
// linear workgroup id so that all (x, y) tiles of one split z -- which read
// the same rows of the shared operand -- run on the same XCD. The map is a
// bijection of [0, X*Y*Z) whenever X*Y*Z is a multiple of 8 (the launchers
// round the split count so that it is); otherwise the identity is used.
__device__ inline void xcd_map(int &bx, int &by, int &bz) {
  const int X = gridDim.x, Y = gridDim.y, Z = gridDim.z;
  const int per = X * Y;
  const int total = per * Z;
  const int b = blockIdx.x + X * (blockIdx.y + Y * blockIdx.z);
  int logical = b;
  if ((total & 7) == 0 && (Z & 7) == 0) {
    const int xcd = b & 7, slot = b >> 3;        // slot-th workgroup on this XCD
    const int zl = slot / per, t = slot - zl * per;
    logical = (zl * 8 + xcd) * per + t;          // split zl*8+xcd, tile t
  }
  bz = logical / per;
  const int t = logical - bz * per;
  bx = t / Y;                                      // tiles sharing a column slice of B
  by = t - bx * Y;                                 // (same bx) run back to back
}

// 1-D launch of T = tiles_slow * tiles_fast output tiles: XCD x (workgroups
// b = x, x + 8, ...; the dispatcher deals workgroups to the 8 XCDs in turn)
// takes the contiguous range [x q + min(x, r), ...) of tile numbers, q = T / 8,
// r = T % 8, in order, fast index fastest. The tiles_fast tiles that share
// one block of the long operand then run back to back on one XCD and share
// its L2. A bijection of [0, T) for every T.
__device__ inline void xcd_linear(int64_t T, int tiles_fast, int64_t &slow, int &fast) {
  const int64_t b = blockIdx.x;
  const int64_t q = T / 8, r = T % 8, x = b & 7, slot = b >> 3;
  const int64_t logical = x * q + (x < r ? x : r) + slot;
  slow = logical / tiles_fast;
  fast = (int)(logical - slow * tiles_fast);
}

// ------------------------------------------------------------- errors ------
void set_error(const char *fmt, ...);
const char *get_error();

#define LSPCA_HIP(call)                                                      \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      ::lspca::set_error("%s failed: %s (%s:%d)", #call,                     \
                         hipGetErrorString(e_), __FILE__, __LINE__);         \
      return LSPCA_EHIP;                                                     \
    }                                                                        \
  } while (0)

#define LSPCA_TRY(expr)                                                      \
  do {                                                                       \
    int s_ = (expr);                                                         \
    if (s_ != LSPCA_OK) return s_;                                           \
  } while (0)

// ----------------------------------------------------------- workspace -----
// A per-device grow-only arena. Callers hold the device lock (see api.hip)
// while they use it. Slots are carved out of one allocation per call.
struct Workspace {
  char *base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  int device = -1;
  int ensure(size_t bytes);          // grows (device sync + realloc) if needed
  void reset() { used = 0; }
  template <typename T> T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    T *p = (T *)(base + used);
    used += bytes;
    return p;
  }
};
template <typename T> inline size_t ws_bytes(size_t count) {
  return (count * sizeof(T) + 255) & ~(size_t)255;
}

// ------------------------------------------------------------- timing -------
struct PhaseTimer {
  bool on = false;
  hipStream_t stream = nullptr;
  hipEvent_t ev[24];
  int slot[24];
  int n = 0;
  void begin(bool enabled, hipStream_t s);
  void mark(int phase);              // records an event ending `phase`
  int finish(lspca_timings *out);    // syncs, fills times, destroys events
  ~PhaseTimer();
};
enum Phase { PH_START = -1, PH_OMEGA = 0, PH_SKETCH, PH_FACTOR, PH_REDUCE, PH_SMALL,
             PH_QR, PH_PASS2, PH_TRANSFORM, PH_LAYOUT };

// ---------------------------------------------------------- launchers ------
// Omega generation (omega.hip). out has the layout out[j*ld_j + c*ld_c].
// f64_of: with dt == LSPCA_F64, store the value rounded to that type.
int launch_omega(int64_t n, int k, int kind, uint64_t seed, uint32_t p,
                 lspca_dtype dt, void *out, int64_t ld_j, int64_t ld_c,
                 hipStream_t s, int f64_of = LSPCA_F64);

// Dense products (gemm.hip). All matrices row-major.
//  nt: C[M x N] = A[M x K] * B[N x K]^T   (A, B: K contiguous)
//  tn: P[s][M x N] = sum_{r in chunk s} A[r][i] * B[r][j]  (split over r)
//  Epilogue: C = alpha * product + beta * C (tn: beta and ldp need splits 1).
int launch_nt(lspca_dtype dt, const void *A, int64_t lda, const void *B,
              int64_t ldb, void *C, int64_t ldc, int64_t M, int N, int K,
              hipStream_t s, double alpha = 1.0, double beta = 0.0);
// C = A B^T for a tall A (the sketch of a stripe, the projection): the
// streamed FP32 kernel where it applies (the same bits as launch_nt), else
// launch_nt.
int launch_nt_tall(lspca_dtype dt, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                     int64_t ldc, int64_t M, int N, int K, hipStream_t s);
int launch_tn(lspca_dtype dt, const void *A, int64_t lda, const void *B,
              int64_t ldb, void *P, int64_t M_rows, int Mi, int Nj, int splits,
              hipStream_t s, int64_t ldp = 0, double alpha = 1.0, double beta = 0.0);
// F = Y^T X of a stripe: the streamed FP32 kernel where it applies (the
// same bits as launch_tn), else launch_tn. splits > 1 writes one partial
// per split as launch_tn.
int launch_tn_factor(lspca_dtype dt, const void *A, int64_t lda, const void *B, int64_t ldb, void *P,
                     int64_t rows, int Mi, int Nj, int splits, hipStream_t s);
int tn_pick_splits(int64_t rows, int Mi, int Nj);
// Rows summed in FP32 by one partial of a split product (at most 65,472
// before the launchers' rounding of the chunk to 16 or 64 rows, so at most
// 65,536 after it), and the split cap (the grid's z limit, a multiple of 8),
// which keeps that depth for stripes of up to 4.29e9 rows.
constexpr int64_t kTnMaxDepth = 65472;
constexpr int64_t kTnMaxSplits = 65528;
// 16-bit products (gemm16.hip). nt16 output mode: 0 row-major FP32 C;
// 1 transposed FP32 C[c*ldc + r] with max |C| per column of each 128-row
// tile (colmax[tile][c], see nt16_row_tiles); 2
// transposed and split into 16-bit parts Ch, Cl (Cl may be NULL). B_lo
// (split second operand) only with mode 0.
int launch_nt16(lspca_dtype dt, const void *A, int64_t lda, const void *Bh,
                const void *Bl, int64_t ldb, float *C, int64_t ldc, int64_t M,
                int N, int K, unsigned *colmax, void *Ch, void *Cl, int mode,
                hipStream_t s);
// F partials from the transposed split sketch Yh/Yl[i*ldyt + r] and X, or
// (yblocked) from the sketch in 8-row blocks, (i, r) at ((r / 8) * Mi + i)
// * 8 + r % 8, rows padded to a multiple of 8 (ldyt unused).
int launch_tn16(lspca_dtype dt, const void *Yh, const void *Yl, int64_t ldyt,
                const void *X, int64_t ldx, float *P, int64_t rows, int Mi, int Nj,
                int splits, hipStream_t s, bool yblocked = false);
// The same partials from the transposed FP32 sketch Yt[i*ldyt + r] (FP16 X
// only): column i scaled by scale[i] (NULL: 1) and split into 16-bit parts
// as launch_split16 does, on the way into the product (refine: both parts).
int launch_tn16_f32y(lspca_dtype dt, const float *Yt, const float *scale, int64_t ldyt, bool refine,
                     const void *X, int64_t ldx, float *P, int64_t rows, int Mi, int Nj, int splits,
                     hipStream_t s);
// Scale row c of Yt (rows_k x ld) by scale[c] and split into 16-bit parts.
int launch_split16(lspca_dtype dt, const float *Yt, int64_t rows_k, int64_t ld,
                   const float *scale, void *Yh, void *Yl, hipStream_t s);
// Row tiles of launch_nt16 (mode 1 writes one column-max row per tile) and
// the reduction of those rows into colmax (zeroed by the caller).
int nt16_row_tiles(int64_t M);
int launch_colmax_reduce(const unsigned *part, int64_t tiles, int N, unsigned *colmax, hipStream_t s);
int launch_col_scales(const unsigned *colmax, int k, float *scale, double *inv,
                      hipStream_t s);
// Very sparse sketch by gather-adds (sparse.hip).
bool sparse_sketch_ok(lspca_dtype dt, int64_t n, int k, uint32_t p, int *cap_out);
// Output as launch_nt16 mode 1 (Y FP32 transposed + colmax), or split into
// Yh, Yl in 8-row blocks (the yblocked layout of launch_tn16; rows padded to
// a multiple of 8, the padding rows left unwritten).
int launch_sparse_sketch(lspca_dtype dt, const void *X, int64_t m, int64_t n, int64_t ldx, int k,
                         uint64_t seed, uint32_t p, int cap, float *Y, int64_t ldy,
                         unsigned *colmax, void *Yh, void *Yl, int *overflow, hipStream_t s);
size_t tn_partial_elems(int Mi, int Nj, int splits);

// Sparse X in CSR form (csr.hip). Row i's entries are colidx[e], vals[e] for
// e in [rowptr[i], rowptr[i + 1]). csr_check validates rowptr (rowptr[0] >= 0,
// nondecreasing, rowptr[m] = nnz) and colidx over [rowptr[0], nnz) on the
// device and reports the result (dflag: one device int of scratch).
int csr_check(const int64_t *rowptr, const int32_t *colidx, int64_t m, int64_t n, int64_t nnz,
              int *dflag, hipStream_t s);
// The same in two halves (other kernels may be queued between them):
// launch, then wait and report; *unsorted: some row's columns decrease
// (set by launch_row_block_pos).
int csr_check_launch(const int64_t *rowptr, const int32_t *colidx, int64_t m, int64_t n, int64_t nnz,
                     int *dflag, hipStream_t s);
int csr_check_result(const int *dflag, int64_t n, int64_t nnz, bool *unsorted, hipStream_t s);
// Z = X V by column blocks of nbc features (csr_blocks gives nbc and the
// block count): pos (rows x (nblk + 1) int32) holds each row's block
// offsets, for rows with nondecreasing columns.
int csr_blocks(int64_t n, size_t esz, int64_t *nbc);
// Sets bit 2 of *dflag when some row's columns decrease.
int launch_rows_sorted(const int64_t *rowptr, const int32_t *colidx, int64_t rows, int64_t nnz, int *dflag,
                       hipStream_t s);
int launch_row_block_pos(const int64_t *rowptr, const int32_t *colidx, int64_t rows, int64_t nnz, int64_t nbc,
                         int nblk, int32_t *pos, int *dflag, hipStream_t s);
int launch_csr_blocked(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals,
                       const int32_t *pos, int nblk, int64_t rows, const void *V, int64_t ldv, int k, void *Z,
                       int64_t ldz, hipStream_t s);
constexpr int64_t kCsrMaxRows = (int64_t)1 << 24;   // rows per row-parallel launch
// Y[i * ldy + c] = sum over row r0 + i of v * B[col * ldb + c], i < rows,
// c < k; B row-major n x k, all of the value type vdt (FP32 or FP64).
int launch_csr_spmm(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals,
                    int64_t r0, int64_t rows, const void *B, int64_t ldb, int k, void *Y, int64_t ldy,
                    hipStream_t s);
// The very sparse Omega (entries -1, 0, +1; materialised n x k row-major,
// row pitch ldo) as row lists: row j's nonzeros oc[t], t in [optr[j],
// optr[j + 1]), in column order, each the column with the sign in bit 31
// (cnt, optr: n + 1 int32, n k < 2^31; oc: room for n k codes; temp of
// om_scan_bytes). Y = X Omega from those lists (row r0 + i of X to row i
// of Y).
size_t om_scan_bytes(int64_t n);
int build_omega_lists(lspca_dtype vdt, const void *Om, int64_t ldo, int64_t n, int k, int32_t *cnt,
                      int32_t *optr, int32_t *oc, void *temp, size_t temp_bytes, hipStream_t s);
int launch_csr_sketch_lists(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals,
                            int64_t r0, int64_t rows, const int32_t *optr, const int32_t *oc, int k, void *Y,
                            int64_t ldy, hipStream_t s);
// rowptr[r0 + g * t] for t = 0 .. nb - 1 (the last clamped to rowptr[r0 +
// rows]): stripe boundaries of the CSC build.
int launch_row_bounds(const int64_t *rowptr, int64_t rows, int64_t g, int64_t nb, int64_t *out,
                      hipStream_t s);
// The column-ordered (CSC) form of a stripe of at most kCsrMaxRows rows
// (entries [e0, e0 + cnt), cnt < 2^31), in row blocks of rb rows: list
// l = b n + j holds the entries of column j in block b at [colptr[l],
// colptr[l + 1]), in row order, with the stripe-local row crow[t] and the
// value cval[t]. The column sums are cut into segments of at most `seg`
// entries (segoff: L + 1; segcol: one int per segment); lists of two or more
// segments keep partial rows in P (k FP64 each, from row moff[l] on).
struct CscShape {
  int64_t rb = 1, nblocks = 1, lists = 1, seg = 1024, segs_max = 1, partial_rows = 1;
};
CscShape csc_shape(int64_t rows, int64_t n, int64_t cnt, int k, size_t esz);
struct CscBuffers {
  int32_t *keys, *skeys, *rowof, *crow, *segcol;
  uint32_t *idx, *sidx;
  void *cval;
  int64_t *colptr, *cnt, *segoff, *moff;
  double *P;
  void *temp;
  size_t temp_bytes;
};
size_t csc_temp_bytes(int64_t cnt, int64_t lists);
int build_csc(lspca_dtype vdt, const int64_t *rowptr, const int32_t *colidx, const void *vals, int64_t r0,
              int64_t rows, int64_t e0, int64_t cnt, int64_t n, const CscShape &sh, CscBuffers &b,
              hipStream_t s);
// Ft[j * k + c] += sum over column j of the stripe of v * Y[row * ldy + c]
// (FP64 accumulation, Y of the value type; Ft is n x k).
int launch_csc_factor(lspca_dtype vdt, const CscBuffers &b, const CscShape &sh, int64_t n, int64_t cnt,
                      const void *Y, int k, int64_t ldy, double *Ft, hipStream_t s);
// Ut[c * ldt + i] = Y[i * ldy + c] for i < rows, c < k (value type vdt).
int launch_rows_to_cols(lspca_dtype vdt, const void *Y, int64_t rows, int k, int64_t ldy, void *Ut, int64_t ldt,
                        hipStream_t s);
// F[c * n + j] += Ft[j * k + c].
int launch_add_transposed(const double *Ft, int64_t n, int k, double *F, hipStream_t s);
// out[j * ldo + c] = V[j][c] (n x k FP64, row-major) in the value type (FP32:
// rounded to nearest).
int launch_v_padded(const double *V, int64_t n, int k, lspca_dtype vdt, void *out, int64_t ldo, hipStream_t s);
// Row pitch (elements) of the library's n x k or m x k row-major buffers for
// the sparse path: rows start on 128-byte boundaries.
inline int64_t csr_ld(int k, size_t esz) {
  const int64_t q = 128 / (int64_t)esz;
  return (k + q - 1) / q * q;
}

// Reductions and small FP64 stage (small.hip).
constexpr int kSmallFlags = 128;   // flag and sweep-counter ints of the small stage
// out[e] (+)= rowscale[e / ncols] * sum_s P[s][e] (rowscale may be NULL).
int launch_reduce_add(lspca_dtype pdt, const void *P, int splits, int64_t count,
                      double *out, int accumulate, hipStream_t s,
                      const double *rowscale = nullptr, int ncols = 1);
int zero_i32(int *p, int count, hipStream_t s);
// Workspace of the sign step of small_factor (part of its need).
size_t sign_fix_bytes(int64_t n, int k);
int small_factor(const double *F, const double *G, int k, int64_t n,
                 double *V, double *sigma, double *sigma_x, Workspace &ws,
                 hipStream_t s, int *rank_flag, int route = 0);
int launch_transpose_f64(const double *src, int64_t rows, int cols,
                         double *dst, hipStream_t s);
// Request table of one batched projection launch (the projection server).
// Two tile classes (16-bit data): requests [0, nreq_s) use the small tiles
// (proj_small_rows), requests [nreq_s, nreq) the standard ones. Within its
// class, request i owns tiles [req[i].tile0, req[i+1].tile0), numbered row
// tile major, ntn_s or ntn column tiles per row tile; ntiles_s and ntiles
// count each class's tiles. X rows are n-contiguous (ldx), Z rows
// k-contiguous (ldz). The kernels take the table by value (3,104 bytes of
// kernel arguments, within the 4 KiB limit).
constexpr int kProjMaxReq = 64;
struct ProjReq {
  const void *X;
  void *Z;
  int64_t ldx, ldz, rows;
  int32_t tile0, pad;
};
struct ProjTable {
  int32_t nreq, ntiles, ntn, nreq_s;
  int32_t ntiles_s, ntn_s, pad0, pad1;
  ProjReq req[kProjMaxReq];
};
static_assert(sizeof(ProjTable) + 64 <= 4096, "the table travels in the kernel arguments");
// Small tiles of the 16-bit projection Z = X (V_hi + V_lo): 32 rows x 64
// columns, two waves. Every output element is the same chain of matrix-core
// steps (K ascending, V_hi then V_lo per step) in every tile shape, so a
// row's bits do not depend on the tiles chosen. proj_small_rows: requests
// (and lspca_transform calls) of at most this many rows use them (0 for
// FP32/FP64 data, which has one tile class).
constexpr int kProjSmallBM = 32, kProjSmallBN = 64;
int64_t proj_small_rows(lspca_dtype dt);
int proj_small_grid(lspca_dtype dt, bool vec, int *grid);
int launch_proj_batch_small(lspca_dtype dt, const ProjTable *tab, const void *VTh, const void *VTl,
                            int64_t ldv, int k, int n, bool vec, int grid, hipStream_t s);
// Tile shape of the projection Z = X V for dtype dt and k columns: the one
// lspca_transform uses, so a batched result is bitwise that of a single call.
void proj_tile_shape(lspca_dtype dt, int k, int *BM, int *BN);
// Workgroups that keep every CU busy for the persistent batch kernel.
int proj_batch_grid(lspca_dtype dt, int k, bool vec, int *grid);
// Z = X V for every request of the table; the table (host memory) is copied
// into the launch's kernel arguments, so it may be reused as soon as the call
// returns. VT = V^T in the compute type (16-bit: VTh + VTl), ldv = n. vec:
// every X row and V^T row is 16-byte aligned (n a multiple of the vector
// width).
int launch_proj_batch(lspca_dtype dt, const ProjTable *tab, const void *VTh, const void *VTl,
                      int64_t ldv, int k, int n, bool vec, int grid, hipStream_t s);

int launch_convert_vt(const double *V, int64_t n, int k, lspca_dtype dt,
                      void *hi, void *lo, hipStream_t s);

// Tall-skinny Householder QR (tsqr.hip). U enters transposed, column c at
// Ut + c * ldu with ldu >= tsqr_ld(m, ydt).
int64_t tsqr_ld(int64_t m, lspca_dtype ydt);
size_t tsqr_workspace_bytes(int64_t m, int k, lspca_dtype ydt);
int tsqr(void *Ut, lspca_dtype ydt, int64_t m, int64_t ldu, int k, Workspace &ws, int out_mode,
         lspca_dtype dt16, void *Q, void *Qh, void *Ql, int64_t ldq, hipStream_t s);
// R factor only (no Q): U row-major or transposed; root R in slice order
// (k x block-height entries of ydt); merge of two such R's stored back to
// back; dense FP64 k x k copy (row-major, zeros below the diagonal).
size_t tsqr_r_workspace_bytes(int64_t m, int k, lspca_dtype ydt);
int tsqr_r(const void *U, lspca_dtype ydt, int64_t m, int64_t ldu, bool rowmajor, int k, Workspace &ws,
           void *Rroot, hipStream_t s);
int tsqr_r_merge(const void *Rpair, lspca_dtype ydt, int k, void *Rout, hipStream_t s);
int tsqr_r_dense(const void *Rslice, lspca_dtype ydt, int k, double *Rd, hipStream_t s);
int tsqr_block_rows(lspca_dtype ydt);
// F <- R^-T F for an upper triangular k x k FP64 R (row-major), F k x n.
int apply_rinv_t(const double *R, int k, double *F, int64_t n, Workspace &ws, hipStream_t s);

size_t dtype_size(lspca_dtype dt);

}  // namespace lspca
