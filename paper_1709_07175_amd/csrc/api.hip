// C ABI entry points of liblspca.so (declared in include/lspca.h).
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

#include <cstdlib>
#include <functional>

namespace lspca {

// ------------------------------------------------------------- errors ------
static thread_local char g_err[1024] = "";
static thread_local lspca_timings g_timings = {};

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char *get_error() { return g_err; }

size_t dtype_size(lspca_dtype dt) {
  switch (dt) {
    case LSPCA_F64: return 8;
    case LSPCA_F32: return 4;
    case LSPCA_BF16:
    case LSPCA_F16: return 2;
  }
  return 0;
}

// ----------------------------------------------------------- workspace -----
int Workspace::ensure(size_t bytes) {
  used = 0;
  if (bytes <= cap) return LSPCA_OK;
  if (base) {
    LSPCA_HIP(hipDeviceSynchronize());
    LSPCA_HIP(hipFree(base));
    base = nullptr;
    cap = 0;
  }
  size_t want = bytes + bytes / 8 + (1 << 20);
  if (hipMalloc(&base, want) != hipSuccess) {
    (void)hipGetLastError();
    base = nullptr;
    set_error("workspace: hipMalloc of %zu bytes failed", want);
    return LSPCA_ENOMEM;
  }
  cap = want;
  return LSPCA_OK;
}

// Copy stream and staging events of the host-streamed pass (created on
// first use; default priority).
struct HostStreaming {
  hipStream_t copy = nullptr;
  hipEvent_t loaded[2] = {}, freed[2] = {};
};

struct DeviceState {
  std::mutex mu;
  Workspace ws;
  HostStreaming hs;
  // Recorded on a call's stream after its last use of the workspace; the
  // next call's stream waits on it before writing the workspace, so calls
  // on different streams never overlap on the device in the shared slots.
  hipEvent_t ws_done = nullptr;
  bool ws_recorded = false;
};

static DeviceState &device_state(int dev) {
  static std::mutex g_mu;
  static std::map<int, DeviceState *> g_states;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_states.find(dev);
  if (it != g_states.end()) return *it->second;
  DeviceState *st = new DeviceState();  // lives until process exit
  st->ws.device = dev;
  g_states[dev] = st;
  return *st;
}

// ------------------------------------------------------------- timing -------
void PhaseTimer::begin(bool enabled, hipStream_t s) {
  on = enabled;
  stream = s;
  n = 0;
  if (!on) return;
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventRecord(ev[0], s) != hipSuccess) {
    on = false;
    return;
  }
  slot[0] = PH_START;
  n = 1;
}
void PhaseTimer::mark(int phase) {
  if (!on || n >= 24) return;
  if (hipEventCreate(&ev[n]) != hipSuccess) return;
  if (hipEventRecord(ev[n], stream) != hipSuccess) {
    (void)hipEventDestroy(ev[n]);
    return;
  }
  slot[n++] = phase;
}
int PhaseTimer::finish(lspca_timings *out) {
  if (!on) return LSPCA_OK;
  memset(out, 0, sizeof(*out));
  LSPCA_HIP(hipEventSynchronize(ev[n - 1]));
  double *fields[] = {&out->omega_ms, &out->sketch_ms, &out->factor_ms, &out->reduce_ms,
                      &out->small_ms, &out->qr_ms, &out->pass2_ms, &out->transform_ms,
                      &out->layout_ms};
  for (int i = 1; i < n; ++i) {
    float ms = 0;
    LSPCA_HIP(hipEventElapsedTime(&ms, ev[i - 1], ev[i]));
    if (slot[i] >= 0 && slot[i] < 9) *fields[slot[i]] += ms;
  }
  float tot = 0;
  LSPCA_HIP(hipEventElapsedTime(&tot, ev[0], ev[n - 1]));
  out->total_ms = tot;
  return LSPCA_OK;
}
PhaseTimer::~PhaseTimer() {
  for (int i = 0; i < n; ++i) (void)hipEventDestroy(ev[i]);
}

// ------------------------------------------------------------ helpers ------
struct Opts {
  uint32_t p = 64;
  int refine = -1;
  int timing = 0;
  hipStream_t stream = nullptr;
  int small_route = 0;
  int64_t stripe_rows = 0;
};

static int read_opts(const lspca_opts *o, Opts &out) {
  out = Opts();
  if (!o) return LSPCA_OK;
  uint32_t sz = o->struct_size;
  if (sz < offsetof(lspca_opts, sparse_p) + sizeof(uint32_t)) return LSPCA_OK;
  if (o->sparse_p) out.p = o->sparse_p;
  if (sz >= offsetof(lspca_opts, refine) + sizeof(int32_t)) out.refine = o->refine;
  if (sz >= offsetof(lspca_opts, timing) + sizeof(int32_t)) out.timing = o->timing;
  if (sz >= offsetof(lspca_opts, stream) + sizeof(void *)) out.stream = (hipStream_t)o->stream;
  if (sz >= offsetof(lspca_opts, small_route) + sizeof(int32_t)) {
    if (o->small_route != 0 && o->small_route != 1) {
      set_error("small_route must be 0 or 1 (got %d)", o->small_route);
      return LSPCA_EINVAL;
    }
    out.small_route = o->small_route;
  }
  if (sz >= offsetof(lspca_opts, stripe_rows) + sizeof(int64_t)) {
    if (o->stripe_rows < 0) {
      set_error("stripe_rows must be >= 0 (got %lld)", (long long)o->stripe_rows);
      return LSPCA_EINVAL;
    }
    out.stripe_rows = o->stripe_rows;
  }
  return LSPCA_OK;
}

static bool valid_p(uint32_t p) { return p >= 1 && p <= (1u << 30) && (p & (p - 1)) == 0; }
static bool valid_dtype(int dt) { return dt >= LSPCA_F64 && dt <= LSPCA_F16; }
static bool valid_kind(int kind) {
  return kind == LSPCA_OMEGA_GAUSSIAN || kind == LSPCA_OMEGA_VERY_SPARSE;
}

static int check_pass_args(const void *X, int dt, int64_t m, int64_t n, int64_t ldx, int k,
                           int kind, const Opts &o) {
  if (!X) { set_error("X is NULL"); return LSPCA_EINVAL; }
  if (!valid_dtype(dt)) { set_error("unknown dtype %d", dt); return LSPCA_EINVAL; }
  if (m < 1 || n < 1) { set_error("m and n must be >= 1 (m=%lld n=%lld)", (long long)m, (long long)n); return LSPCA_EINVAL; }
  if (n > (1 << 30)) { set_error("n too large"); return LSPCA_EINVAL; }
  if (ldx < n) { set_error("ldx (%lld) < n (%lld)", (long long)ldx, (long long)n); return LSPCA_EINVAL; }
  if (k < 1 || k > n) { set_error("k must satisfy 1 <= k <= n (k=%d n=%lld)", k, (long long)n); return LSPCA_EINVAL; }
  if (k > 4096) { set_error("k > 4096 is not supported"); return LSPCA_ENOTSUP; }
  if (!valid_kind(kind)) { set_error("unknown omega kind %d", kind); return LSPCA_EINVAL; }
  if (kind == LSPCA_OMEGA_VERY_SPARSE && !valid_p(o.p)) { set_error("sparse p must be a power of two in [1, 2^30] (p=%u)", o.p); return LSPCA_EINVAL; }
  return LSPCA_OK;
}

static int current_device(int *dev) {
  LSPCA_HIP(hipGetDevice(dev));
  return LSPCA_OK;
}

__global__ void k_zero_f64(double *p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}
static int zero_f64(double *p, int64_t count, hipStream_t s) {
  if (count <= 0) return LSPCA_OK;
  hipLaunchKernelGGL(k_zero_f64, (unsigned)((count + 255) / 256), 256, 0, s, p, count);
  LSPCA_HIP(hipGetLastError());
  return LSPCA_OK;
}

// --------------------------------------------------------- the pass --------
// Stripe plan for one pass: Y for a stripe of rows is kept in the workspace.
struct PassPlan {
  bool h16;             // 16-bit data: nt16/tn16 products, G = F Omega in FP64
  bool gather;          // very sparse Omega applied by gather-adds (no Omega^T)
  int cap;              // LDS list capacity of the gather kernel
  size_t esz;           // bytes per element of Y / partials (4 or 8)
  int64_t stripe;       // rows per stripe
  int splits_f, splits_g;
  size_t bytes;
};

static bool is16(lspca_dtype dt) { return dt == LSPCA_BF16 || dt == LSPCA_F16; }

static PassPlan plan_pass(lspca_dtype xdt, int64_t m, int64_t n, int k, bool want_g, int kind,
                          uint32_t sp, int64_t stripe_rows = 0) {
  PassPlan p;
  p.h16 = is16(xdt);
  p.cap = 0;
  p.gather = kind == LSPCA_OMEGA_VERY_SPARSE && sparse_sketch_ok(xdt, n, k, sp, &p.cap);
  p.esz = xdt == LSPCA_F64 ? 8 : 4;
  // Y stripe bytes: 4 GiB (under 2% of the device memory), or
  // LSPCA_STRIPE_BYTES (a tuning and test knob: small values exercise the
  // multi-stripe paths on small inputs)
  int64_t budget = (int64_t)4 << 30;
  if (const char *e = getenv("LSPCA_STRIPE_BYTES")) {
    const long long v = atoll(e);
    if (v > 0) budget = v;
  }
  int64_t rows = budget / ((int64_t)k * p.esz);
  rows = rows < 1024 ? 1024 : rows;
  if (stripe_rows > 0) rows = stripe_rows;            // the caller's slices
  p.stripe = m < rows ? m : rows;
  p.splits_f = tn_pick_splits(p.stripe, k, (int)n);
  p.splits_g = (want_g && !p.h16) ? tn_pick_splits(p.stripe, k, k) : 0;
  p.bytes = ws_bytes<char>(dtype_size(xdt) * (size_t)n * k)              // Omega^T
            + ws_bytes<char>(p.esz * (size_t)p.stripe * k)                // Y stripe
            + ws_bytes<char>(p.esz * tn_partial_elems(k, (int)n, p.splits_f))
            + (p.splits_g ? ws_bytes<char>(p.esz * tn_partial_elems(k, k, p.splits_g)) : 0);
  if (p.h16) {
    p.bytes += 2 * ws_bytes<uint16_t>((size_t)(p.stripe + 8) * k);              // Yh, Yl (+ block padding)
    p.bytes += ws_bytes<unsigned>(k) + ws_bytes<float>(k) + ws_bytes<double>(k);  // FP16 scales
    p.bytes += ws_bytes<unsigned>((size_t)nt16_row_tiles(p.stripe) * k);           // tile maxima
    p.bytes += ws_bytes<int>(4);                                                 // flags
    if (want_g)
      p.bytes += ws_bytes<double>((size_t)n * k)      // Omega^T in FP64 (the values used)
                 + ws_bytes<double>((size_t)n * k);   // this call's F
  }
  return p;
}

// Called with each stripe's sketch Y (rows x k): row-major FP32/FP64 with
// ld = k (transposed = false), or transposed FP32 with ld = rows for 16-bit
// data (transposed = true). Used by Algorithm 3 to update its R.
using StripeHook = std::function<int(const void *Y, int64_t rows, int64_t ld, bool transposed)>;

// Algorithm 4 step 2 over all rows of X (stripe by stripe): F += Y^T X,
// G += Y^T Y. Workspace must hold plan.bytes (already ensured).
static int run_pass(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx, int k,
                    int kind, uint64_t seed, const Opts &o, double *F, double *G,
                    const PassPlan &pl, Workspace &ws, PhaseTimer &tm, const StripeHook *hook = nullptr) {
  hipStream_t s = o.stream;
  const size_t xs = dtype_size(xdt);
  const bool refine = o.refine != 0;                 // default (-1) and 1: on
  void *OmT = ws.take<char>(xs * (size_t)n * k);
  void *Y = ws.take<char>(pl.esz * (size_t)pl.stripe * k);
  void *PF = ws.take<char>(pl.esz * tn_partial_elems(k, (int)n, pl.splits_f));
  void *PG = pl.splits_g ? ws.take<char>(pl.esz * tn_partial_elems(k, k, pl.splits_g)) : nullptr;
  unsigned *colmax = nullptr, *colpart = nullptr;
  float *scale = nullptr;
  double *inv = nullptr, *OmT64 = nullptr, *Fs = nullptr;
  int *flags = nullptr;
  uint16_t *Yh = nullptr, *Yl = nullptr;
  if (pl.h16) {
    Yh = ws.take<uint16_t>((size_t)(pl.stripe + 8) * k);
    Yl = ws.take<uint16_t>((size_t)(pl.stripe + 8) * k);
    colmax = ws.take<unsigned>(k);
    colpart = ws.take<unsigned>((size_t)nt16_row_tiles(pl.stripe) * k);
    scale = ws.take<float>(k);
    inv = ws.take<double>(k);
    flags = ws.take<int>(4);
    if (G) {
      OmT64 = ws.take<double>((size_t)n * k);
      Fs = ws.take<double>((size_t)n * k);
    }
  }
  const bool fp16 = xdt == LSPCA_F16;

  // Omega^T (k x n) in the compute type: OmT[c][j] = Omega[j][c]. The
  // gather path regenerates Omega inside the sketch kernel instead.
  if (!pl.gather) LSPCA_TRY(launch_omega(n, k, kind, seed, o.p, xdt, OmT, 1, n, s));
  if (OmT64) LSPCA_TRY(launch_omega(n, k, kind, seed, o.p, LSPCA_F64, OmT64, 1, n, s, xdt));
  tm.mark(PH_OMEGA);
  double *Fdst = Fs ? Fs : F;                        // 16-bit with G: this call's F first
  const int acc = Fs ? 0 : 1;
  for (int64_t r0 = 0; r0 < m; r0 += pl.stripe) {
    const int64_t rows = (m - r0) < pl.stripe ? (m - r0) : pl.stripe;
    const char *Xs = (const char *)X + (size_t)r0 * ldx * xs;
    const int sf = tn_pick_splits(rows, k, (int)n);
    if (!pl.h16) {
      // Y_s = X_s Omega (Algorithm 4 step 2a)
      LSPCA_TRY(launch_nt_tall(xdt, Xs, ldx, OmT, n, Y, k, rows, k, (int)n, s));
      tm.mark(PH_SKETCH);
      if (hook) LSPCA_TRY((*hook)(Y, rows, k, false));
      // F += Y_s^T X_s (step 2b); G += Y_s^T Y_s
      LSPCA_TRY(launch_tn_factor(xdt, Y, k, Xs, ldx, PF, rows, k, (int)n, sf, s));
      int sg = 0;
      if (G) {
        sg = tn_pick_splits(rows, k, k);
        LSPCA_TRY(launch_tn(xdt, Y, k, Y, k, PG, rows, k, k, sg, s));
      }
      tm.mark(PH_FACTOR);
      LSPCA_TRY(launch_reduce_add(xdt, PF, sf, (int64_t)k * n, F, 1, s));
      if (G) LSPCA_TRY(launch_reduce_add(xdt, PG, sg, (int64_t)k * k, G, 1, s));
      tm.mark(PH_REDUCE);
    } else {
      // sketch: BF16 directly split into Yh/Yl (transposed; in 8-row blocks
      // from the gather kernel); FP16 as FP32 transposed with column maxima,
      // then scaled and split. With a hook, BF16 also goes through FP32
      // (split without scaling).
      uint16_t *Ylo = refine ? Yl : nullptr;
      const bool y32 = fp16 || hook;
      if (fp16) LSPCA_TRY(zero_i32((int *)colmax, k, s));
      if (pl.gather) {
        LSPCA_TRY(zero_i32(flags, 1, s));
        LSPCA_TRY(launch_sparse_sketch(xdt, Xs, rows, n, ldx, k, seed, o.p, pl.cap,
                                       y32 ? (float *)Y : nullptr, rows, fp16 ? colmax : nullptr,
                                       Yh, Ylo, flags, s));
      } else {
        LSPCA_TRY(launch_nt16(xdt, Xs, ldx, OmT, nullptr, n, y32 ? (float *)Y : nullptr, rows, rows,
                              k, (int)n, fp16 ? colpart : nullptr, Yh, Ylo, y32 ? 1 : 2, s));
      }
      tm.mark(PH_SKETCH);
      // FP32 sketch -> column scales (FP16) and 16-bit parts (timed as the
      // layout phase); without a hook the FP16 split happens inside the F
      // product, as its tiles are loaded
      const bool fused = fp16 && !hook;
      if (fp16 && !pl.gather) LSPCA_TRY(launch_colmax_reduce(colpart, nt16_row_tiles(rows), k, colmax, s));
      if (fp16) LSPCA_TRY(launch_col_scales(colmax, k, scale, inv, s));
      if (y32 && !fused)
        LSPCA_TRY(launch_split16(xdt, (const float *)Y, k, rows, fp16 ? scale : nullptr, Yh, Ylo, s));
      if (y32) tm.mark(PH_LAYOUT);
      if (hook) LSPCA_TRY((*hook)(Y, rows, rows, true));
      if (fused)
        LSPCA_TRY(launch_tn16_f32y(xdt, (const float *)Y, scale, rows, refine, Xs, ldx, (float *)PF, rows, k,
                                   (int)n, sf, s));
      else  // the gather kernel writes its split sketch in 8-row blocks
        LSPCA_TRY(launch_tn16(xdt, Yh, Ylo, rows, Xs, ldx, (float *)PF, rows, k, (int)n, sf, s,
                              pl.gather && !y32));
      tm.mark(PH_FACTOR);
      const int accum = (r0 > 0) ? 1 : acc;
      LSPCA_TRY(launch_reduce_add(LSPCA_F32, PF, sf, (int64_t)k * n, Fdst, accum, s,
                                  fp16 ? inv : nullptr, (int)n));
      tm.mark(PH_REDUCE);
    }
  }
  if (Fs) {
    // G += F_s Omega (= Y^T X Omega = Y^T Y), F += F_s, both in FP64
    LSPCA_TRY(launch_nt(LSPCA_F64, Fs, n, OmT64, n, G, k, k, k, (int)n, s, 1.0, 1.0));
    LSPCA_TRY(launch_reduce_add(LSPCA_F64, Fs, 1, (int64_t)k * n, F, 1, s));
    tm.mark(PH_REDUCE);
  }
  return LSPCA_OK;
}

static size_t factor_bytes(int64_t n, int k) {
  const int splits = tn_pick_splits(n, k, k);
  const size_t kk = (size_t)k * k;
  return 4 * ws_bytes<double>((size_t)n * k) + ws_bytes<double>(tn_partial_elems(k, k, splits)) +
         6 * ws_bytes<double>(kk) + 2 * ws_bytes<double>(k) + ws_bytes<int>(kSmallFlags) +
         ws_bytes<double>(4 * kk) +
         ws_bytes<double>(3 * 128 * 128) + sign_fix_bytes(n, k);
}

// Algorithm 4 over X in host memory: stripes of `stripe` rows go through two
// device staging buffers; the copy of stripe s + 1 (copy stream) overlaps
// the pass over stripe s (the caller's stream). F and G accumulate.
static int host_pass(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx, int k, int kind,
                     uint64_t seed, const Opts &o, int64_t stripe, double *F, double *G,
                     DeviceState &st) {
  const size_t xs = dtype_size(xdt);
  HostStreaming &hs = st.hs;
  if (!hs.copy) {
    LSPCA_HIP(hipStreamCreateWithFlags(&hs.copy, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
      LSPCA_HIP(hipEventCreateWithFlags(&hs.loaded[b], hipEventDisableTiming));
      LSPCA_HIP(hipEventCreateWithFlags(&hs.freed[b], hipEventDisableTiming));
    }
  }
  const PassPlan pl = plan_pass(xdt, stripe, n, k, G != nullptr, kind, o.p);
  const size_t sbytes = ws_bytes<char>(xs * (size_t)stripe * n);
  LSPCA_TRY(st.ws.ensure(2 * sbytes + pl.bytes));
  Workspace &ws = st.ws;
  char *stage[2] = {ws.take<char>(sbytes), ws.take<char>(sbytes)};
  const size_t mark = ws.used;
  hipStream_t s = o.stream;
  PhaseTimer quiet;                                  // per-stripe phases are not recorded
  for (int b = 0; b < 2; ++b) LSPCA_HIP(hipEventRecord(hs.freed[b], s));
  int64_t it = 0;
  for (int64_t r0 = 0; r0 < m; r0 += stripe, ++it) {
    const int b = (int)(it & 1);
    const int64_t rows = m - r0 < stripe ? m - r0 : stripe;
    LSPCA_HIP(hipStreamWaitEvent(hs.copy, hs.freed[b], 0));
    LSPCA_HIP(hipMemcpy2DAsync(stage[b], (size_t)n * xs, (const char *)X + (size_t)r0 * ldx * xs,
                               (size_t)ldx * xs, (size_t)n * xs, (size_t)rows, hipMemcpyHostToDevice,
                               hs.copy));
    LSPCA_HIP(hipEventRecord(hs.loaded[b], hs.copy));
    LSPCA_HIP(hipStreamWaitEvent(s, hs.loaded[b], 0));
    ws.used = mark;
    LSPCA_TRY(run_pass(stage[b], xdt, rows, n, n, k, kind, seed, o, F, G, pl, ws, quiet));
    LSPCA_HIP(hipEventRecord(hs.freed[b], s));
  }
  // X may be released by the caller on return
  LSPCA_HIP(hipStreamSynchronize(s));
  return LSPCA_OK;
}

static int64_t host_stripe(int64_t m, int64_t n, lspca_dtype xdt, int64_t want) {
  int64_t rows = want > 0 ? want : ((int64_t)1 << 30) / (n * (int64_t)dtype_size(xdt));
  rows = (rows + 255) / 256 * 256;                   // whole tiles, vector-friendly
  return rows < m ? rows : m;
}

static int check_host_ptr(const void *X) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, X) != hipSuccess) {
    (void)hipGetLastError();
    return LSPCA_OK;                                 // pageable host memory
  }
  if (a.type == hipMemoryTypeDevice) {
    set_error("X is device memory: use lspca_accumulate / lspca_fit");
    return LSPCA_EINVAL;
  }
  return LSPCA_OK;
}

struct Locked {
  DeviceState *st = nullptr;
  std::unique_lock<std::mutex> lk;
};
static int lock_device(Locked &L) {
  int dev = 0;
  LSPCA_TRY(current_device(&dev));
  L.st = &device_state(dev);
  L.lk = std::unique_lock<std::mutex>(L.st->mu);
  return LSPCA_OK;
}

// Device-side order of the workspace across streams. begin(): the call's
// stream waits for the last use of the workspace by the previous call (on
// whatever stream it ran); the destructor records the call's own last use,
// also on an error return, so work already queued by a failed call is
// covered. Declared after the Locked guard, it runs while the lock is held.
struct WsOrder {
  DeviceState *st = nullptr;
  hipStream_t s = nullptr;
  int begin(Locked &L, hipStream_t stream) {
    DeviceState &d = *L.st;
    if (!d.ws_done) LSPCA_HIP(hipEventCreateWithFlags(&d.ws_done, hipEventDisableTiming));
    if (d.ws_recorded) LSPCA_HIP(hipStreamWaitEvent(stream, d.ws_done, 0));
    st = &d;
    s = stream;
    return LSPCA_OK;
  }
  ~WsOrder() {
    if (!st) return;
    if (hipEventRecord(st->ws_done, s) == hipSuccess)
      st->ws_recorded = true;
    else
      (void)hipGetLastError();
  }
};


// ------------------------------------------------------ sparse (CSR) X -----
static int check_csr_args(const int64_t *rowptr, const int32_t *colidx, const void *vals, int vdt,
                          int64_t m, int64_t n, int64_t nnz, int k, int kind, const Opts &o) {
  if (!rowptr) { set_error("rowptr is NULL"); return LSPCA_EINVAL; }
  if (nnz > 0 && (!colidx || !vals)) { set_error("colidx and values must not be NULL"); return LSPCA_EINVAL; }
  if (vdt != LSPCA_F32 && vdt != LSPCA_F64) {
    set_error("CSR values must be FP32 or FP64 (dtype %d)", vdt);
    return valid_dtype(vdt) ? LSPCA_ENOTSUP : LSPCA_EINVAL;
  }
  if (m < 1 || n < 1) { set_error("m and n must be >= 1 (m=%lld n=%lld)", (long long)m, (long long)n); return LSPCA_EINVAL; }
  if (n > (1 << 30)) { set_error("n too large"); return LSPCA_EINVAL; }
  if (nnz < 0) { set_error("nnz must be >= 0"); return LSPCA_EINVAL; }
  if (k < 1 || k > n) { set_error("k must satisfy 1 <= k <= n (k=%d n=%lld)", k, (long long)n); return LSPCA_EINVAL; }
  if (k > 4096) { set_error("k > 4096 is not supported"); return LSPCA_ENOTSUP; }
  if (!valid_kind(kind)) { set_error("unknown omega kind %d", kind); return LSPCA_EINVAL; }
  if (kind == LSPCA_OMEGA_VERY_SPARSE && !valid_p(o.p)) { set_error("sparse p must be a power of two in [1, 2^30] (p=%u)", o.p); return LSPCA_EINVAL; }
  return LSPCA_OK;
}

// Stripes of the CSR pass: row starts r[s] (r.back() = m) and entry starts
// e[s] = rowptr[r[s]]. A stripe holds at most `rows_cap` rows (the Y
// budget) and, where the granularity allows, at most `nnz_cap` entries (the
// CSC buffers); boundaries fall on multiples of g rows.
// The very sparse Omega goes through row lists (int32 positions: n k < 2^31).
static bool csr_lists(int kind, int64_t n, int k) {
  return kind == LSPCA_OMEGA_VERY_SPARSE && n * (int64_t)k < ((int64_t)1 << 31);
}

struct CsrPlan {
  std::vector<int64_t> r, e;
  int64_t max_rows = 0, max_cnt = 0;
  int splits_g = 0;
  int64_t ldy = 0;                                   // row pitch of Y (128-byte rows)
  int nblk = 0;                                      // Gaussian sketch by column blocks of nbc
  int64_t nbc = 0;
  CscShape shape;                                    // of the largest stripe
  size_t bytes = 0;
};



// Validates the CSR arrays on the device, then plans the stripes. Uses the
// workspace (reset on return).
static int plan_csr(const int64_t *rowptr, const int32_t *colidx, lspca_dtype vdt, int64_t m, int64_t n,
                    int64_t nnz, int k, int kind, bool want_g, const Opts &o, Workspace &ws, CsrPlan &pl) {
  hipStream_t s = o.stream;
  const size_t esz = dtype_size(vdt);
  int64_t budget = (int64_t)4 << 30;                 // Y bytes, as the dense pass
  if (const char *v = getenv("LSPCA_STRIPE_BYTES")) {
    const long long b = atoll(v);
    if (b > 0) budget = b;
  }
  int64_t nnz_cap = (int64_t)1 << 28;                // entries per CSC build
  if (const char *v = getenv("LSPCA_CSR_STRIPE_NNZ")) {
    const long long b = atoll(v);
    if (b > 0) nnz_cap = b;
  }
  int64_t rows_cap = budget / ((int64_t)k * esz);
  rows_cap = rows_cap < 64 ? 64 : rows_cap;
  rows_cap = rows_cap > kCsrMaxRows ? kCsrMaxRows : rows_cap;
  int64_t g = 64;
  if (o.stripe_rows > 0) {
    g = o.stripe_rows < kCsrMaxRows ? o.stripe_rows : kCsrMaxRows;
    rows_cap = g;
  }
  const int64_t nb = (m + g - 1) / g + 1;
  ws.reset();
  LSPCA_TRY(ws.ensure(ws_bytes<int>(1) + ws_bytes<int64_t>(nb)));
  int *flag = ws.take<int>(1);
  int64_t *bd = ws.take<int64_t>(nb);
  // a Gaussian Omega is applied by column blocks when every row's columns
  // are in order (the dense rows of Omega then stay in L2)
  const bool blocks = !csr_lists(kind, n, k);
  LSPCA_TRY(csr_check_launch(rowptr, colidx, m, n, nnz, flag, s));
  if (blocks) LSPCA_TRY(launch_rows_sorted(rowptr, colidx, m, nnz, flag, s));
  LSPCA_TRY(launch_row_bounds(rowptr, m, g, nb, bd, s));
  bool unsorted = true;
  LSPCA_TRY(csr_check_result(flag, n, nnz, &unsorted, s));
  std::vector<int64_t> hb(nb);
  LSPCA_HIP(hipMemcpyAsync(hb.data(), bd, nb * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  LSPCA_HIP(hipStreamSynchronize(s));
  ws.reset();
  pl = CsrPlan();
  pl.nblk = blocks && !unsorted ? csr_blocks(n, esz, &pl.nbc) : 0;
  int64_t b = 0;                                     // block index of the stripe start
  while (b < nb - 1) {
    int64_t t = b + 1;
    while (t < nb - 1 && (t + 1 - b) * g <= rows_cap && hb[t + 1] - hb[b] <= nnz_cap) ++t;
    const int64_t r0 = b * g, r1 = t * g < m ? t * g : m;
    pl.r.push_back(r0);
    pl.e.push_back(hb[b]);
    pl.max_rows = std::max(pl.max_rows, r1 - r0);
    pl.max_cnt = std::max(pl.max_cnt, hb[t] - hb[b]);
    b = t;
  }
  pl.r.push_back(m);
  pl.e.push_back(hb[nb - 1]);
  if (pl.max_cnt > (int64_t)INT32_MAX) {
    set_error("CSR: %lld entries in %lld rows exceed the 2^31 - 1 entries of one stripe",
              (long long)pl.max_cnt, (long long)g);
    return LSPCA_ENOTSUP;
  }
  pl.splits_g = want_g ? tn_pick_splits(pl.max_rows, k, k) : 0;
  pl.ldy = csr_ld(k, esz);
  pl.shape = csc_shape(pl.max_rows, n, pl.max_cnt, k, esz);
  const size_t E = (size_t)pl.max_cnt;
  const size_t L1 = (size_t)pl.shape.lists + 1;
  pl.bytes = ws_bytes<char>(esz * (size_t)n * pl.ldy)           // Omega, row-major
             + ws_bytes<char>(esz * (size_t)pl.max_rows * pl.ldy)  // Y stripe
             + ws_bytes<double>((size_t)n * k)                  // this call's F, transposed
             + (want_g ? ws_bytes<char>(esz * tn_partial_elems(k, k, pl.splits_g)) : 0)
             + 5 * ws_bytes<int32_t>(E)                         // keys skeys idx sidx rowof
             + ws_bytes<char>(esz * E) + 4 * ws_bytes<int64_t>(L1)
             + ws_bytes<int32_t>((size_t)pl.shape.segs_max)
             + ws_bytes<double>((size_t)pl.shape.partial_rows * k)
             + ws_bytes<char>(std::max(csc_temp_bytes(pl.max_cnt, pl.shape.lists), om_scan_bytes(n)));
  if (csr_lists(kind, n, k))                                      // Omega row lists
    pl.bytes += 2 * ws_bytes<int32_t>((size_t)n + 1) + ws_bytes<int32_t>((size_t)n * k);
  if (pl.nblk)                                                     // the stripe's block offsets
    pl.bytes += ws_bytes<int32_t>((size_t)pl.max_rows * (pl.nblk + 1)) + ws_bytes<int>(1);
  return LSPCA_OK;
}

// Algorithm 4 step 2 over a CSR X: per stripe Y = X_s Omega (row SpMM),
// F += Y^T X_s (column-ordered, from the stripe's CSC form), G += Y^T Y.
// SPCA (Algorithm 1) over a CSR X: the whole sketch U^T (column c at
// Ut + c * ldt), overwritten by the QR, and its thin Q (m x k, row pitch ldq).
struct CsrSpca {
  void *Ut;
  int64_t ldt;
  void *Q;
  int64_t ldq;
};

static int csr_pass(const int64_t *rowptr, const int32_t *colidx, const void *vals, lspca_dtype vdt,
                    int64_t n, int k, int kind, uint64_t seed, const Opts &o, const CsrPlan &pl,
                    double *F, double *G, Workspace &ws, PhaseTimer &tm, const CsrSpca *sp = nullptr) {
  hipStream_t s = o.stream;
  const size_t esz = dtype_size(vdt);
  const size_t E = (size_t)pl.max_cnt;
  const size_t L1 = (size_t)pl.shape.lists + 1;
  const int64_t ldy = pl.ldy;
  void *Om = ws.take<char>(esz * (size_t)n * ldy);
  void *Y = ws.take<char>(esz * (size_t)pl.max_rows * ldy);
  double *Ft = ws.take<double>((size_t)n * k);
  void *PG = G ? ws.take<char>(esz * tn_partial_elems(k, k, pl.splits_g)) : nullptr;
  CscBuffers b;
  b.keys = ws.take<int32_t>(E);
  b.skeys = ws.take<int32_t>(E);
  b.idx = ws.take<uint32_t>(E);
  b.sidx = ws.take<uint32_t>(E);
  b.rowof = ws.take<int32_t>(E);
  b.crow = b.keys;                                   // the unsorted keys are dead after the sort
  b.cval = ws.take<char>(esz * E);
  b.colptr = ws.take<int64_t>(L1);
  b.cnt = ws.take<int64_t>(L1);
  b.segoff = ws.take<int64_t>(L1);
  b.moff = ws.take<int64_t>(L1);
  b.segcol = ws.take<int32_t>((size_t)pl.shape.segs_max);
  b.P = ws.take<double>((size_t)pl.shape.partial_rows * k);
  b.temp_bytes = std::max(csc_temp_bytes(pl.max_cnt, pl.shape.lists), om_scan_bytes(n));
  b.temp = ws.take<char>(b.temp_bytes);
  const bool lists = csr_lists(kind, n, k);
  int32_t *optr = nullptr, *oc = nullptr;
  LSPCA_TRY(zero_f64(Ft, (int64_t)n * k, s));
  LSPCA_TRY(launch_omega(n, k, kind, seed, o.p, vdt, Om, ldy, 1, s));
  if (lists) {
    int32_t *ocnt = ws.take<int32_t>((size_t)n + 1);
    optr = ws.take<int32_t>((size_t)n + 1);
    oc = ws.take<int32_t>((size_t)n * k);
    LSPCA_TRY(build_omega_lists(vdt, Om, ldy, n, k, ocnt, optr, oc, b.temp, b.temp_bytes, s));
  }
  int32_t *pos = nullptr;
  int *pflag = nullptr;
  if (pl.nblk) {
    pos = ws.take<int32_t>((size_t)pl.max_rows * (pl.nblk + 1));
    pflag = ws.take<int>(1);
  }
  tm.mark(PH_OMEGA);
  // Y (rows x k, row pitch ldy) = rows [r0, r0 + rows) of X times Omega
  auto sketch = [&](int64_t r0, int64_t rows) -> int {
    if (lists)
      return launch_csr_sketch_lists(vdt, rowptr, colidx, vals, r0, rows, optr, oc, k, Y, ldy, s);
    if (pl.nblk) {
      LSPCA_TRY(launch_row_block_pos(rowptr + r0, colidx, rows, pl.e.back(), pl.nbc, pl.nblk, pos, pflag, s));
      return launch_csr_blocked(vdt, rowptr + r0, colidx, vals, pos, pl.nblk, rows, Om, ldy, k, Y, ldy, s);
    }
    return launch_csr_spmm(vdt, rowptr, colidx, vals, r0, rows, Om, ldy, k, Y, ldy, s);
  };
  if (sp) {
    // Algorithm 1: U = X Omega (all rows, transposed), Q R = U, F = Q^T X
    const size_t esz_ = dtype_size(vdt);
    for (size_t t = 0; t + 1 < pl.r.size(); ++t) {
      const int64_t r0 = pl.r[t], rows = pl.r[t + 1] - r0;
      LSPCA_TRY(sketch(r0, rows));
      LSPCA_TRY(launch_rows_to_cols(vdt, Y, rows, k, ldy, (char *)sp->Ut + esz_ * (size_t)r0, sp->ldt, s));
    }
    tm.mark(PH_SKETCH);
    LSPCA_TRY(tsqr(sp->Ut, vdt, pl.r.back(), sp->ldt, k, ws, 0, vdt, sp->Q, nullptr, nullptr, sp->ldq, s));
    tm.mark(PH_QR);
    for (size_t t = 0; t + 1 < pl.r.size(); ++t) {
      const int64_t r0 = pl.r[t], rows = pl.r[t + 1] - r0;
      const int64_t e0 = pl.e[t], cnt = pl.e[t + 1] - e0;
      CscShape sh = csc_shape(rows, n, pl.max_cnt, k, esz);
      LSPCA_TRY(build_csc(vdt, rowptr, colidx, vals, r0, rows, e0, cnt, n, sh, b, s));
      tm.mark(PH_LAYOUT);
      LSPCA_TRY(launch_csc_factor(vdt, b, sh, n, cnt, (const char *)sp->Q + esz_ * (size_t)r0 * sp->ldq, k,
                                  sp->ldq, Ft, s));
      tm.mark(PH_PASS2);
    }
    LSPCA_TRY(launch_add_transposed(Ft, n, k, F, s));
    tm.mark(PH_REDUCE);
    return LSPCA_OK;
  }
  for (size_t t = 0; t + 1 < pl.r.size(); ++t) {
    const int64_t r0 = pl.r[t], rows = pl.r[t + 1] - r0;
    const int64_t e0 = pl.e[t], cnt = pl.e[t + 1] - e0;
    LSPCA_TRY(sketch(r0, rows));
    tm.mark(PH_SKETCH);
    // this stripe's row blocks; the segment length of the largest stripe
    CscShape sh = csc_shape(rows, n, pl.max_cnt, k, esz);
    LSPCA_TRY(build_csc(vdt, rowptr, colidx, vals, r0, rows, e0, cnt, n, sh, b, s));
    tm.mark(PH_LAYOUT);
    LSPCA_TRY(launch_csc_factor(vdt, b, sh, n, cnt, Y, k, ldy, Ft, s));
    int sg = 0;
    if (G) {
      sg = tn_pick_splits(rows, k, k);
      LSPCA_TRY(launch_tn(vdt, Y, ldy, Y, ldy, PG, rows, k, k, sg, s));
    }
    tm.mark(PH_FACTOR);
    if (G) LSPCA_TRY(launch_reduce_add(vdt, PG, sg, (int64_t)k * k, G, 1, s));
    tm.mark(PH_REDUCE);
  }
  LSPCA_TRY(launch_add_transposed(Ft, n, k, F, s));
  tm.mark(PH_REDUCE);
  return LSPCA_OK;
}

// --------------------------------------- allocation-free projection -------
// Scratch of lspca_transform_noalloc: V^T in the compute type of X (two
// 16-bit parts for BF16/FP16 X), the only device memory that call uses
// beyond its inputs and outputs. A file-scope device array, so the call
// never allocates; every device holds its own copy until the process ends.
// The host-side name is not a device address: host code uses the address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[LSPCA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static int noalloc_scratch(char **out) {
  static std::mutex mu;
  static char *ptrs[kMaxDevices] = {};
  int dev = 0;
  LSPCA_TRY(current_device(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d: lspca_transform_noalloc supports devices 0..%d", dev, kMaxDevices - 1);
    return LSPCA_ENOTSUP;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return LSPCA_EHIP;
    }
    ptrs[dev] = (char *)p;
  }
  *out = ptrs[dev];
  return LSPCA_OK;
}

}  // namespace lspca

using namespace lspca;

// ====================================================================== ABI ==
extern "C" {

const char *lspca_version(void) { return "lspca 0.1 gfx950"; }

const char *lspca_strerror(int status) {
  switch (status) {
    case LSPCA_OK: return "ok";
    case LSPCA_EINVAL: return "invalid argument";
    case LSPCA_ENOMEM: return "out of device memory";
    case LSPCA_EHIP: return "HIP runtime error";
    case LSPCA_ERANK: return "rank deficient";
    case LSPCA_E2BIG: return "request too large";
    case LSPCA_EAGAIN: return "no capacity, retry";
    case LSPCA_ENOTSUP: return "not supported";
    case LSPCA_ETIMEDOUT: return "timed out";
    case LSPCA_ENOTFOUND: return "unknown ticket";
    case LSPCA_ENOCONV: return "Jacobi sweep limit reached";
  }
  return "unknown status";
}

const char *lspca_last_error(void) { return get_error(); }

int lspca_last_timings(lspca_timings *out) {
  if (!out) return LSPCA_EINVAL;
  *out = g_timings;
  return LSPCA_OK;
}

int lspca_omega(int64_t n, int32_t k, lspca_omega_kind kind, uint64_t seed, uint32_t p,
                lspca_dtype dtype, void *Omega, void *stream) {
  if (!Omega) { set_error("Omega is NULL"); return LSPCA_EINVAL; }
  if (n < 1 || k < 1) { set_error("n and k must be >= 1"); return LSPCA_EINVAL; }
  if (!valid_kind(kind)) { set_error("unknown omega kind %d", (int)kind); return LSPCA_EINVAL; }
  if (!valid_dtype(dtype)) { set_error("unknown dtype %d", (int)dtype); return LSPCA_EINVAL; }
  if (p == 0) p = 64;
  if (kind == LSPCA_OMEGA_VERY_SPARSE && !valid_p(p)) { set_error("bad sparse p %u", p); return LSPCA_EINVAL; }
  return launch_omega(n, k, kind, seed, p, dtype, Omega, k, 1, (hipStream_t)stream);
}

int lspca_accumulate(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx,
                     int32_t k, lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts,
                     double *F, double *G) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_pass_args(X, xdt, m, n, ldx, k, kind, o));
  if (!F) { set_error("F is NULL"); return LSPCA_EINVAL; }
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  PassPlan pl = plan_pass(xdt, m, n, k, G != nullptr, kind, o.p, o.stripe_rows);
  LSPCA_TRY(L.st->ws.ensure(pl.bytes));
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  LSPCA_TRY(run_pass(X, xdt, m, n, ldx, k, kind, seed, o, F, G, pl, L.st->ws, tm));
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int lspca_factor(const double *F, const double *G, int32_t k, int64_t n, const lspca_opts *opts,
                 double *V, double *sigma, double *sigma_x) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  if (!F || !V || !sigma) { set_error("F, V and sigma must not be NULL"); return LSPCA_EINVAL; }
  if (sigma_x && !G) { set_error("sigma_x needs G"); return LSPCA_EINVAL; }
  if (n < 1 || k < 1 || k > n) { set_error("need 1 <= k <= n (k=%d n=%lld)", k, (long long)n); return LSPCA_EINVAL; }
  if (k > 4096) { set_error("k > 4096 is not supported"); return LSPCA_ENOTSUP; }
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  LSPCA_TRY(L.st->ws.ensure(factor_bytes(n, k)));
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  int rank_flag = 0;
  LSPCA_TRY(small_factor(F, G, k, n, V, sigma, sigma_x, L.st->ws, o.stream, &rank_flag, o.small_route));
  tm.mark(PH_SMALL);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int lspca_fit(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx, int32_t k,
              lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts, double *V,
              double *sigma, double *sigma_x) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_pass_args(X, xdt, m, n, ldx, k, kind, o));
  if (!V || !sigma) { set_error("V and sigma must not be NULL"); return LSPCA_EINVAL; }
  if (k > m) { set_error("k must satisfy k <= min(m, n) (k=%d m=%lld)", k, (long long)m); return LSPCA_EINVAL; }
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  const bool want_g = sigma_x != nullptr;
  PassPlan pl = plan_pass(xdt, m, n, k, want_g, kind, o.p, o.stripe_rows);
  const size_t fg = ws_bytes<double>((size_t)k * n) + ws_bytes<double>((size_t)k * k);
  const size_t fb = factor_bytes(n, k);
  LSPCA_TRY(L.st->ws.ensure(fg + (pl.bytes > fb ? pl.bytes : fb)));
  Workspace &ws = L.st->ws;
  double *F = ws.take<double>((size_t)k * n);
  double *G = ws.take<double>((size_t)k * k);
  const size_t mark = ws.used;
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  LSPCA_TRY(zero_f64(F, (int64_t)k * n, o.stream));
  LSPCA_TRY(zero_f64(G, (int64_t)k * k, o.stream));
  LSPCA_TRY(run_pass(X, xdt, m, n, ldx, k, kind, seed, o, F, want_g ? G : nullptr, pl, ws, tm));
  ws.used = mark;                                    // the pass's slots are free again
  int rank_flag = 0;
  LSPCA_TRY(small_factor(F, want_g ? G : nullptr, k, n, V, sigma, sigma_x, ws, o.stream, &rank_flag, o.small_route));
  tm.mark(PH_SMALL);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int lspca_transform(const void *X, lspca_dtype xdt, int64_t r, int64_t n, int64_t ldx,
                    const double *V, int32_t k, void *Z, const lspca_opts *opts) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  if (!valid_dtype(xdt)) { set_error("unknown dtype %d", (int)xdt); return LSPCA_EINVAL; }
  if (r < 0 || n < 1 || k < 1 || ldx < n) { set_error("bad sizes (r=%lld n=%lld k=%d ldx=%lld)", (long long)r, (long long)n, k, (long long)ldx); return LSPCA_EINVAL; }
  if (r == 0) return LSPCA_OK;
  if (!X || !V || !Z) { set_error("X, V and Z must not be NULL"); return LSPCA_EINVAL; }
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  const size_t es = dtype_size(xdt);
  const bool h16 = is16(xdt);
  LSPCA_TRY(L.st->ws.ensure((h16 ? 2 : 1) * ws_bytes<char>(es * (size_t)n * k)));
  void *VT = L.st->ws.take<char>(es * (size_t)n * k);
  void *VTlo = h16 ? L.st->ws.take<char>(es * (size_t)n * k) : nullptr;
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  LSPCA_TRY(launch_convert_vt(V, n, k, xdt, VT, VTlo, o.stream));
  if (h16)
    LSPCA_TRY(launch_nt16(xdt, X, ldx, VT, VTlo, n, (float *)Z, k, r, k, (int)n, nullptr, nullptr,
                          nullptr, 0, o.stream));
  else
    LSPCA_TRY(launch_nt_tall(xdt, X, ldx, VT, n, Z, k, r, k, (int)n, o.stream));
  tm.mark(PH_TRANSFORM);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int lspca_transform_noalloc(const void *X, lspca_dtype xdt, int64_t r, int64_t n, int64_t ldx,
                            const double *V, int32_t k, void *Z, const lspca_opts *opts) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  if (!valid_dtype(xdt)) { set_error("unknown dtype %d", (int)xdt); return LSPCA_EINVAL; }
  if (r < 0 || n < 1 || k < 1 || ldx < n) { set_error("bad sizes (r=%lld n=%lld k=%d ldx=%lld)", (long long)r, (long long)n, k, (long long)ldx); return LSPCA_EINVAL; }
  if (r == 0) return LSPCA_OK;
  if (!X || !V || !Z) { set_error("X, V and Z must not be NULL"); return LSPCA_EINVAL; }
  const size_t es = dtype_size(xdt);
  const bool h16 = is16(xdt);
  const size_t parts = h16 ? 2 : 1;
  // V^T needs parts * es * n * k bytes (each part 256-byte aligned); checked
  // by division first so n * k cannot overflow
  const size_t cap = LSPCA_NOALLOC_SCRATCH_BYTES;
  if ((size_t)n > cap / (parts * es) / (size_t)k ||
      parts * ws_bytes<char>(es * (size_t)n * k) > cap) {
    set_error("lspca_transform_noalloc: V^T of n=%lld x k=%d in the type of X needs more than the "
              "%zu-byte scratch (n k <= %zu for this type)", (long long)n, k, cap, cap / (parts * es));
    return LSPCA_E2BIG;
  }
  char *sp = nullptr;
  LSPCA_TRY(noalloc_scratch(&sp));
  char *VT = sp;
  char *VTlo = h16 ? sp + ws_bytes<char>(es * (size_t)n * k) : nullptr;
  LSPCA_TRY(launch_convert_vt(V, n, k, xdt, VT, VTlo, o.stream));
  if (h16)
    LSPCA_TRY(launch_nt16(xdt, X, ldx, VT, VTlo, n, (float *)Z, k, r, k, (int)n, nullptr, nullptr,
                          nullptr, 0, o.stream));
  else
    LSPCA_TRY(launch_nt_tall(xdt, X, ldx, VT, n, Z, k, r, k, (int)n, o.stream));
  return LSPCA_OK;
}

int lspca_accumulate_host(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx,
                          int32_t k, lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts,
                          int64_t stripe_rows, double *F, double *G) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_pass_args(X, xdt, m, n, ldx, k, kind, o));
  if (!F) { set_error("F is NULL"); return LSPCA_EINVAL; }
  if (stripe_rows < 0) { set_error("stripe_rows must be >= 0"); return LSPCA_EINVAL; }
  LSPCA_TRY(check_host_ptr(X));
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  LSPCA_TRY(host_pass(X, xdt, m, n, ldx, k, kind, seed, o, host_stripe(m, n, xdt, stripe_rows), F, G, *L.st));
  tm.mark(PH_FACTOR);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int lspca_fit_host(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx, int32_t k,
                   lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts, int64_t stripe_rows,
                   double *V, double *sigma, double *sigma_x) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_pass_args(X, xdt, m, n, ldx, k, kind, o));
  if (!V || !sigma) { set_error("V and sigma must not be NULL"); return LSPCA_EINVAL; }
  if (k > m) { set_error("k must satisfy k <= min(m, n) (k=%d m=%lld)", k, (long long)m); return LSPCA_EINVAL; }
  if (stripe_rows < 0) { set_error("stripe_rows must be >= 0"); return LSPCA_EINVAL; }
  LSPCA_TRY(check_host_ptr(X));
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  const bool want_g = sigma_x != nullptr;
  // F and G live in their own allocation: the workspace is re-planned below
  double *FG = nullptr;
  const size_t fgn = (size_t)k * n + (size_t)k * k;
  if (hipMalloc((void **)&FG, fgn * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("fit_host: hipMalloc of F and G failed");
    return LSPCA_ENOMEM;
  }
  struct Free {
    double *p;
    ~Free() { (void)hipFree(p); }
  } guard{FG};
  double *F = FG, *G = FG + (size_t)k * n;
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  LSPCA_TRY(zero_f64(FG, (int64_t)fgn, o.stream));
  LSPCA_TRY(host_pass(X, xdt, m, n, ldx, k, kind, seed, o, host_stripe(m, n, xdt, stripe_rows), F,
                      want_g ? G : nullptr, *L.st));
  tm.mark(PH_FACTOR);
  LSPCA_TRY(L.st->ws.ensure(factor_bytes(n, k)));
  int rank_flag = 0;
  LSPCA_TRY(small_factor(F, want_g ? G : nullptr, k, n, V, sigma, sigma_x, L.st->ws, o.stream, &rank_flag, o.small_route));
  tm.mark(PH_SMALL);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int spca_fit_stream(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx, int32_t k,
                    lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts, double *V,
                    double *sigma) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_pass_args(X, xdt, m, n, ldx, k, kind, o));
  if (!V || !sigma) { set_error("V and sigma must not be NULL"); return LSPCA_EINVAL; }
  if (k > m) { set_error("k must satisfy k <= min(m, n) (k=%d m=%lld)", k, (long long)m); return LSPCA_EINVAL; }
  const lspca_dtype ydt = xdt == LSPCA_F64 ? LSPCA_F64 : LSPCA_F32;
  const int BR = tsqr_block_rows(ydt);
  if (k > BR) {
    set_error("spca_fit_stream: k = %d above the QR block height (%d)", k, BR);
    return LSPCA_ENOTSUP;
  }
  const size_t ys = dtype_size(ydt);
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  PassPlan pl = plan_pass(xdt, m, n, k, false, kind, o.p, o.stripe_rows);
  const size_t kb = (size_t)k * BR;
  const size_t keep = ws_bytes<double>((size_t)k * n) + 3 * ws_bytes<char>(ys * kb) +
                      ws_bytes<double>((size_t)k * k);
  const size_t during = pl.bytes + tsqr_r_workspace_bytes(pl.stripe, k, ydt);
  const size_t after = factor_bytes(n, k) + ws_bytes<double>((size_t)k * n) +
                       2 * ws_bytes<double>((size_t)k * k) + ws_bytes<double>(3 * 128 * 128);
  LSPCA_TRY(L.st->ws.ensure(keep + (during > after ? during : after)));
  Workspace &ws = L.st->ws;
  hipStream_t s = o.stream;
  double *F = ws.take<double>((size_t)k * n);
  char *Rpair = ws.take<char>(2 * ys * kb);          // running R, then the stripe's R
  char *Rnext = ws.take<char>(ys * kb);
  double *Rd = ws.take<double>((size_t)k * k);
  const size_t mark = ws.used;
  PhaseTimer tm;
  tm.begin(o.timing != 0, s);
  LSPCA_TRY(zero_f64(F, (int64_t)k * n, s));
  // Algorithm 3 step 2c: R <- R of qr([R; U_s]) for every stripe U_s
  bool first = true;
  StripeHook hook = [&](const void *Y, int64_t rows, int64_t ld, bool transposed) -> int {
    const size_t here = ws.used;
    LSPCA_TRY(tsqr_r(Y, ydt, rows, ld, !transposed, k, ws, first ? (void *)Rpair : (void *)(Rpair + ys * kb), s));
    if (!first) {
      LSPCA_TRY(tsqr_r_merge(Rpair, ydt, k, Rnext, s));
      LSPCA_HIP(hipMemcpyAsync(Rpair, Rnext, ys * kb, hipMemcpyDeviceToDevice, s));
    }
    first = false;
    ws.used = here;
    tm.mark(PH_QR);
    return LSPCA_OK;
  };
  // one pass: U_s = X_s Omega, F += U_s^T X_s (steps 2a-2b), R updated per stripe
  LSPCA_TRY(run_pass(X, xdt, m, n, ldx, k, kind, seed, o, F, nullptr, pl, ws, tm, &hook));
  ws.used = mark;
  // step 3: F = (R^-1)^T F; step 4: truncated SVD of F gives V^s, Sigma^s
  LSPCA_TRY(tsqr_r_dense(Rpair, ydt, k, Rd, s));
  LSPCA_TRY(apply_rinv_t(Rd, k, F, n, ws, s));
  tm.mark(PH_PASS2);
  ws.used = mark;
  int rank_flag = 0;
  LSPCA_TRY(small_factor(F, nullptr, k, n, V, sigma, nullptr, ws, s, &rank_flag, o.small_route));
  tm.mark(PH_SMALL);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int spca_fit(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx, int32_t k,
             lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts, double *V,
             double *sigma) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_pass_args(X, xdt, m, n, ldx, k, kind, o));
  if (!V || !sigma) { set_error("V and sigma must not be NULL"); return LSPCA_EINVAL; }
  if (k > m) { set_error("k must satisfy k <= min(m, n) (k=%d m=%lld)", k, (long long)m); return LSPCA_EINVAL; }
  const lspca_dtype ydt = xdt == LSPCA_F64 ? LSPCA_F64 : LSPCA_F32;
  if (k > (ydt == LSPCA_F64 ? 128 : 256)) {
    set_error("spca_fit: k = %d above the QR block height (%d)", k, ydt == LSPCA_F64 ? 128 : 256);
    return LSPCA_ENOTSUP;
  }
  const bool h16 = is16(xdt);
  const bool refine = o.refine != 0;
  const size_t xs = dtype_size(xdt), ys = dtype_size(ydt);
  const int sf = tn_pick_splits(m, k, (int)n);
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  const int64_t ldt = tsqr_ld(m, ydt);
  const size_t need = ws_bytes<char>(xs * (size_t)n * k) + ws_bytes<char>(ys * (size_t)ldt * k) +
                      (h16 ? 2 * ws_bytes<uint16_t>((size_t)m * k) : ws_bytes<char>(ys * (size_t)m * k)) +
                      tsqr_workspace_bytes(m, k, ydt) + ws_bytes<char>(ys * tn_partial_elems(k, (int)n, sf)) +
                      ws_bytes<double>((size_t)k * n) + factor_bytes(n, k);
  LSPCA_TRY(L.st->ws.ensure(need));
  Workspace &ws = L.st->ws;
  hipStream_t s = o.stream;
  void *OmT = ws.take<char>(xs * (size_t)n * k);
  void *Y = ws.take<char>(ys * (size_t)ldt * k);   // U^T: column j at Y + j * ldt
  void *Q = nullptr;
  uint16_t *Qh = nullptr, *Ql = nullptr;
  if (h16) {
    Qh = ws.take<uint16_t>((size_t)m * k);
    Ql = ws.take<uint16_t>((size_t)m * k);
  } else {
    Q = ws.take<char>(ys * (size_t)m * k);
  }
  void *PF = ws.take<char>(ys * tn_partial_elems(k, (int)n, sf));
  double *F = ws.take<double>((size_t)k * n);
  PhaseTimer tm;
  tm.begin(o.timing != 0, s);
  // Algorithm 1 step 1: U = X Omega, stored transposed (U^T = Omega^T X^T)
  LSPCA_TRY(launch_omega(n, k, kind, seed, o.p, xdt, OmT, 1, n, s));
  tm.mark(PH_OMEGA);
  if (h16) {
    LSPCA_TRY(launch_nt16(xdt, X, ldx, OmT, nullptr, n, (float *)Y, ldt, m, k, (int)n, nullptr, nullptr,
                          nullptr, 1, s));
  } else {
    const int64_t stripe = 4 << 20;               // rows per launch (grid limit on the row tiles)
    for (int64_t r0 = 0; r0 < m; r0 += stripe) {
      const int64_t rows = m - r0 < stripe ? m - r0 : stripe;
      LSPCA_TRY(launch_nt(xdt, OmT, n, (const char *)X + xs * (size_t)r0 * ldx, ldx,
                          (char *)Y + ys * (size_t)r0, ldt, k, (int)rows, (int)n, s));
    }
  }
  tm.mark(PH_SKETCH);
  // step 2: Q, R = qr(U)
  LSPCA_TRY(tsqr(Y, ydt, m, ldt, k, ws, h16 ? 1 : 0, xdt, Q, Qh, Ql, h16 ? m : k, s));
  tm.mark(PH_QR);
  // step 3: F = Q^T X (second pass over X)
  if (h16)
    LSPCA_TRY(launch_tn16(xdt, Qh, refine ? Ql : nullptr, m, X, ldx, (float *)PF, m, k, (int)n, sf, s));
  else
    LSPCA_TRY(launch_tn_factor(xdt, Q, k, X, ldx, PF, m, k, (int)n, sf, s));
  tm.mark(PH_PASS2);
  LSPCA_TRY(launch_reduce_add(ydt, PF, sf, (int64_t)k * n, F, 0, s));
  tm.mark(PH_REDUCE);
  // step 4: truncated SVD of F gives V^s, Sigma^s
  int rank_flag = 0;
  LSPCA_TRY(small_factor(F, nullptr, k, n, V, sigma, nullptr, ws, s, &rank_flag, o.small_route));
  tm.mark(PH_SMALL);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int lspca_accumulate_csr(const int64_t *rowptr, const int32_t *colidx, const void *values,
                         lspca_dtype vdt, int64_t m, int64_t n, int64_t nnz, int32_t k,
                         lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts, double *F,
                         double *G) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_csr_args(rowptr, colidx, values, vdt, m, n, nnz, k, kind, o));
  if (!F) { set_error("F is NULL"); return LSPCA_EINVAL; }
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  Workspace &ws = L.st->ws;
  CsrPlan pl;
  LSPCA_TRY(plan_csr(rowptr, colidx, vdt, m, n, nnz, k, kind, G != nullptr, o, ws, pl));
  LSPCA_TRY(ws.ensure(pl.bytes));
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  LSPCA_TRY(csr_pass(rowptr, colidx, values, vdt, n, k, kind, seed, o, pl, F, G, ws, tm));
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int lspca_fit_csr(const int64_t *rowptr, const int32_t *colidx, const void *values, lspca_dtype vdt,
                  int64_t m, int64_t n, int64_t nnz, int32_t k, lspca_omega_kind kind, uint64_t seed,
                  const lspca_opts *opts, double *V, double *sigma, double *sigma_x) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_csr_args(rowptr, colidx, values, vdt, m, n, nnz, k, kind, o));
  if (!V || !sigma) { set_error("V and sigma must not be NULL"); return LSPCA_EINVAL; }
  if (k > m) { set_error("k must satisfy k <= min(m, n) (k=%d m=%lld)", k, (long long)m); return LSPCA_EINVAL; }
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  Workspace &ws = L.st->ws;
  const bool want_g = sigma_x != nullptr;
  CsrPlan pl;
  LSPCA_TRY(plan_csr(rowptr, colidx, vdt, m, n, nnz, k, kind, want_g, o, ws, pl));
  const size_t fg = ws_bytes<double>((size_t)k * n) + ws_bytes<double>((size_t)k * k);
  const size_t fb = factor_bytes(n, k);
  LSPCA_TRY(ws.ensure(fg + (pl.bytes > fb ? pl.bytes : fb)));
  double *F = ws.take<double>((size_t)k * n);
  double *G = ws.take<double>((size_t)k * k);
  const size_t mark = ws.used;
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  LSPCA_TRY(zero_f64(F, (int64_t)k * n, o.stream));
  LSPCA_TRY(zero_f64(G, (int64_t)k * k, o.stream));
  LSPCA_TRY(csr_pass(rowptr, colidx, values, vdt, n, k, kind, seed, o, pl, F, want_g ? G : nullptr, ws, tm));
  ws.used = mark;
  int rank_flag = 0;
  LSPCA_TRY(small_factor(F, want_g ? G : nullptr, k, n, V, sigma, sigma_x, ws, o.stream, &rank_flag,
                         o.small_route));
  tm.mark(PH_SMALL);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int lspca_transform_csr(const int64_t *rowptr, const int32_t *colidx, const void *values, lspca_dtype vdt,
                        int64_t r, int64_t n, int64_t nnz, const double *V, int32_t k, void *Z,
                        const lspca_opts *opts) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  if (r < 0) { set_error("r must be >= 0"); return LSPCA_EINVAL; }
  if (r == 0) return LSPCA_OK;
  LSPCA_TRY(check_csr_args(rowptr, colidx, values, vdt, r, n, nnz, k, LSPCA_OMEGA_GAUSSIAN, o));
  if (!V || !Z) { set_error("V and Z must not be NULL"); return LSPCA_EINVAL; }
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  Workspace &ws = L.st->ws;
  const size_t esz = dtype_size(vdt);
  const int64_t ldv = csr_ld(k, esz);
  int64_t nbc = 0;
  const int nblk = csr_blocks(n, esz, &nbc);
  const bool try_blocks = r <= kCsrMaxRows;         // one launch per block over all rows
  ws.reset();
  LSPCA_TRY(ws.ensure(ws_bytes<int>(1) + ws_bytes<char>(esz * (size_t)n * ldv) +
                      (try_blocks ? ws_bytes<int32_t>((size_t)r * (nblk + 1)) : 0)));
  int *flag = ws.take<int>(1);
  void *Vp = ws.take<char>(esz * (size_t)n * ldv);  // V in the value type, 128-byte rows
  int32_t *pos = try_blocks ? ws.take<int32_t>((size_t)r * (nblk + 1)) : nullptr;
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  bool unsorted = true;
  LSPCA_TRY(csr_check_launch(rowptr, colidx, r, n, nnz, flag, o.stream));
  if (try_blocks) LSPCA_TRY(launch_row_block_pos(rowptr, colidx, r, nnz, nbc, nblk, pos, flag, o.stream));
  LSPCA_TRY(csr_check_result(flag, n, nnz, &unsorted, o.stream));
  LSPCA_TRY(launch_v_padded(V, n, k, vdt, Vp, ldv, o.stream));
  if (try_blocks && !unsorted)                       // rows with nondecreasing columns: by column blocks
    LSPCA_TRY(launch_csr_blocked(vdt, rowptr, colidx, values, pos, nblk, r, Vp, ldv, k, Z, k, o.stream));
  else
    LSPCA_TRY(launch_csr_spmm(vdt, rowptr, colidx, values, 0, r, Vp, ldv, k, Z, k, o.stream));
  tm.mark(PH_TRANSFORM);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

int spca_fit_csr(const int64_t *rowptr, const int32_t *colidx, const void *values, lspca_dtype vdt, int64_t m,
                 int64_t n, int64_t nnz, int32_t k, lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts,
                 double *V, double *sigma) {
  Opts o;
  LSPCA_TRY(read_opts(opts, o));
  LSPCA_TRY(check_csr_args(rowptr, colidx, values, vdt, m, n, nnz, k, kind, o));
  if (!V || !sigma) { set_error("V and sigma must not be NULL"); return LSPCA_EINVAL; }
  if (k > m) { set_error("k must satisfy k <= min(m, n) (k=%d m=%lld)", k, (long long)m); return LSPCA_EINVAL; }
  if (k > (vdt == LSPCA_F64 ? 128 : 256)) {
    set_error("spca_fit_csr: k = %d above the QR block height (%d)", k, vdt == LSPCA_F64 ? 128 : 256);
    return LSPCA_ENOTSUP;
  }
  Locked L;
  LSPCA_TRY(lock_device(L));
  WsOrder wo;
  LSPCA_TRY(wo.begin(L, o.stream));
  Workspace &ws = L.st->ws;
  CsrPlan pl;
  LSPCA_TRY(plan_csr(rowptr, colidx, vdt, m, n, nnz, k, kind, false, o, ws, pl));
  const size_t esz = dtype_size(vdt);
  const int64_t ldt = tsqr_ld(m, vdt), ldq = csr_ld(k, esz);
  const size_t fixed = ws_bytes<double>((size_t)k * n) + ws_bytes<char>(esz * (size_t)ldt * k) +
                       ws_bytes<char>(esz * (size_t)m * ldq);
  const size_t pass = pl.bytes + tsqr_workspace_bytes(m, k, vdt), fb = factor_bytes(n, k);
  LSPCA_TRY(ws.ensure(fixed + (pass > fb ? pass : fb)));
  double *F = ws.take<double>((size_t)k * n);
  CsrSpca sp{ws.take<char>(esz * (size_t)ldt * k), ldt, ws.take<char>(esz * (size_t)m * ldq), ldq};
  const size_t mark = ws.used;
  PhaseTimer tm;
  tm.begin(o.timing != 0, o.stream);
  LSPCA_TRY(zero_f64(F, (int64_t)k * n, o.stream));
  LSPCA_TRY(csr_pass(rowptr, colidx, values, vdt, n, k, kind, seed, o, pl, F, nullptr, ws, tm, &sp));
  ws.used = mark;
  int rank_flag = 0;
  LSPCA_TRY(small_factor(F, nullptr, k, n, V, sigma, nullptr, ws, o.stream, &rank_flag, o.small_route));
  tm.mark(PH_SMALL);
  if (o.timing) LSPCA_TRY(tm.finish(&g_timings));
  return LSPCA_OK;
}

}  // extern "C"
