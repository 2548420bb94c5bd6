// C-ABI of libmpgemm (declared in include/mpgemm.h): argument checking, the
// slice-count policy, workspace handling and the launch sequence
//   split(A rows, B columns) -> fused slice-product GEMM + accumulation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/mpgemm.h"
#include "host.h"
#include "internal.h"
#include "layout.h"

using namespace mp;

namespace mp {
namespace host {

constexpr int kNumFmt = 4;
constexpr int kMaxDim = 1 << 20;
constexpr int kMaxDFloat = 16;
constexpr int kMaxDInt8 = 40;
constexpr int kMaxNd = 14;    // longest expansion of mpgemm_nd (binary64 components)
constexpr int kMaxDNd = 112;  // most INT8 digit slices of mpgemm_nd
constexpr int kBoundBits[kNumFmt] = {100, 150, 200, 66};  // 2^-t bound per format
constexpr int kComps[kNumFmt] = {2, 3, 4, 3};
const int kCompsH[kNumFmtH] = {2, 3, 4, 3};

// Process-wide defaults of the per-thread options, read once from the
// environment: MPGEMM_MODE ("float" or "int8"; TS stays FLOAT) and
// MPGEMM_SLICES (a slice count for every format and form that allows it, or
// "data" for the binary64/binary32 form's data-chosen pairs).  Values that do
// not parse, or are out of a form's range, leave that default automatic.
struct EnvDefaults {
  int mode = MPGEMM_MODE_FLOAT;
  int slices_float = 0, slices_int8 = 0;
};
const EnvDefaults &env_defaults() {
  static const EnvDefaults d = [] {
    EnvDefaults e;
    const char *m = std::getenv("MPGEMM_MODE");
    if (m && std::strcmp(m, "int8") == 0) e.mode = MPGEMM_MODE_INT8;
    const char *s = std::getenv("MPGEMM_SLICES");
    if (s && std::strcmp(s, "data") == 0) {
      e.slices_float = MPGEMM_SLICES_DATA;
    } else if (s && *s) {
      char *end = nullptr;
      const long v = std::strtol(s, &end, 10);
      if (end && *end == '\0') {
        if (v >= 1 && v <= kMaxDFloat) e.slices_float = (int)v;
        if (v >= 1 && v <= kMaxDInt8) e.slices_int8 = (int)v;
      }
    }
    return e;
  }();
  return d;
}

struct ThreadOptions {
  ThreadOptions() {
    const EnvDefaults &e = env_defaults();
    for (int f = 0; f < kNumFmt; ++f) {
      const bool int8_ok = f != MPGEMM_TS;
      mode[f] = int8_ok ? e.mode : MPGEMM_MODE_FLOAT;
      slices[f][MPGEMM_MODE_FLOAT] = e.slices_float;
      slices[f][MPGEMM_MODE_INT8] = int8_ok ? e.slices_int8 : 0;
    }
  }
  int mode[kNumFmt] = {MPGEMM_MODE_FLOAT, MPGEMM_MODE_FLOAT, MPGEMM_MODE_FLOAT, MPGEMM_MODE_FLOAT};
  int layout[kNumFmt] = {0, 0, 0, 0};  // 0: tuned default
  int int8_tile = 0;                   // 0: automatic
  int split_kernel = 0;                // 0: fused where vectors fit, 1: pass kernels only
  int last_slice = 0;                  // 0: D extractions, 1: last slice = residual's leading component
  int slices[kNumFmt][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  int last_slices = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
};
thread_local ThreadOptions g_opt;

// Per-thread stage-timing log (mpgemm_profile_*).
struct ProfileLog {
  bool on = false;
  std::vector<hipEvent_t> pool;           // reusable events
  std::vector<std::array<hipEvent_t, 3>> marks;  // (before split, before GEMM, after GEMM)
  ~ProfileLog() {
    for (auto e : pool) (void)hipEventDestroy(e);
    for (auto &m : marks)
      for (auto e : m) (void)hipEventDestroy(e);
  }
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
thread_local ProfileLog g_prof;

int ceil_log2_int(int64_t k) {
  int r = 0;
  while ((int64_t(1) << r) < k) ++r;
  return r;
}

// The shift ceil((S + log2 k) / 2) of tau (Section 3, Algorithm 1).
int rho_of(int S, int64_t k) { return k < 1 ? 0 : (S + ceil_log2_int(k) + 1) / 2; }

// Automatic D.  FLOAT: each slice carries b = S - rho bits, so the dropped
// part falls like 2^-(D b); D is the smallest count with D b >= t + g, where
// g (guard bits) covers the gap between an element's |A||B| and the row and
// column maxima that set the slice grids for exponent spreads up to 16 bits,
// plus a margin; that gap shrinks as k grows.  INT8: 7 bits per digit slice,
// D 7 >= t + g8 with g8 = 14 guard bits below k = 2048 and 10 from there on.
int auto_slices(int fmt, int mode, int64_t k) {
  const int t = kBoundBits[fmt];
  if (mode == MPGEMM_MODE_INT8) return (t + (k < 2048 ? 14 : 10) + 6) / 7;
  const int S = fmt == MPGEMM_TS ? 24 : 53;
  const int b = S - rho_of(S, k < 1 ? 1 : k);
  int g = 22 - (11 * ceil_log2_int(k < 1 ? 1 : k)) / 10;
  if (g < 8) g = 8;
  int D = (t + g + b - 1) / b;
  if (D > kMaxDFloat) D = kMaxDFloat;
  if (D < 1) D = 1;
  return D;
}

// Tuned tables, process-wide: wave layouts per format and slice counts per
// (format, form, k range), read from the file named in MPGEMM_TUNE_FILE at
// first use, or from mpgemm_load_tune_file.  Lines:
//   "<fmt> <layout>"                   wave layout of the FLOAT-form kernel
//   "slices <fmt> <mode> <kmax> <D>"   D for k <= kmax (the smallest kmax that
//                                      covers k wins; beyond all, the formula)
// as written by paper_2301_09960_amd.tune.
struct SliceEntry {
  int fmt, mode;
  int64_t kmax;
  int D;
};
int g_layout_default[kNumFmt] = {1, 2, 2, 2};  // measured at n = 1024 and 4096 (DD, TD, QD, TS)
std::vector<SliceEntry> g_slice_table;
std::mutex g_tune_mu;
std::once_flag g_tune_once;

int fmt_index(const char *name) {
  const char *names[kNumFmt] = {"dd", "td", "qd", "ts"};
  for (int i = 0; i < kNumFmt; ++i)
    if (std::strcmp(name, names[i]) == 0) return i;
  return -1;
}

// Replaces the tables by the file's (nullptr: back to the compiled defaults).
// Returns 0, -1 if the file cannot be read, -2 for a line it does not accept
// (the tables are then left unchanged).
int load_tune_tables(const char *path) {
  int layout[kNumFmt] = {1, 2, 2, 2};
  std::vector<SliceEntry> table;
  if (path) {
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char line[256];
    int bad = 0;
    while (std::fgets(line, sizeof line, f)) {
      char a[16], b[16];
      int x = 0, D = 0;
      long long kmax = 0;
      if (line[0] == '#' || line[0] == '\n') continue;
      if (std::sscanf(line, "slices %15s %15s %lld %d", a, b, &kmax, &D) == 4) {
        const int fi = fmt_index(a);
        const int mode = std::strcmp(b, "float") == 0 ? MPGEMM_MODE_FLOAT : std::strcmp(b, "int8") == 0 ? MPGEMM_MODE_INT8 : -1;
        const int dmax = mode == MPGEMM_MODE_FLOAT ? kMaxDFloat : kMaxDInt8;
        if (fi < 0 || mode < 0 || kmax < 1 || D < 1 || D > dmax || (mode == MPGEMM_MODE_INT8 && fi == MPGEMM_TS)) {
          bad = 1;
          break;
        }
        table.push_back({fi, mode, (int64_t)kmax, D});
      } else if (std::sscanf(line, "%15s %d", a, &x) == 2 && fmt_index(a) >= 0 && x >= 1 && x <= 3) {
        layout[fmt_index(a)] = x;
      } else {
        bad = 1;
        break;
      }
    }
    std::fclose(f);
    if (bad) return -2;
  }
  std::sort(table.begin(), table.end(), [](const SliceEntry &p, const SliceEntry &q) { return p.kmax < q.kmax; });
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::copy(layout, layout + kNumFmt, g_layout_default);
  g_slice_table = std::move(table);
  return 0;
}

void load_tune_file() {
  const char *path = std::getenv("MPGEMM_TUNE_FILE");
  if (path && *path) (void)load_tune_tables(path);
}

int slices_for(int fmt, int mode, int64_t k) {
  const int s = g_opt.slices[fmt][mode];
  if (s > 0) return s;
  std::call_once(g_tune_once, load_tune_file);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const SliceEntry &e : g_slice_table)
      if (e.fmt == fmt && e.mode == mode && k <= e.kmax) return e.D;
  }
  return auto_slices(fmt, mode, k);
}
int thread_mode(int fmt) { return g_opt.mode[fmt]; }
int int8_tile_override() { return g_opt.int8_tile; }
int split_kernel_override() { return g_opt.split_kernel; }
int last_slice_option() { return g_opt.last_slice; }

// Wave layout of the binary64/binary32 slice-product kernel per format: the
// tuned table (above), replaced per thread by mpgemm_set_tile_layout.
int layout_for(int fmt) {
  if (g_opt.layout[fmt] > 0) return g_opt.layout[fmt];
  std::call_once(g_tune_once, load_tune_file);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return g_layout_default[fmt];
}
void set_last_slices(int D) { g_opt.last_slices = D; }
bool profiling() { return g_prof.on; }
void profile_mark3(hipEvent_t (&ev)[3]) {
  for (auto &x : ev) x = g_prof.on ? g_prof.take() : nullptr;
}
void profile_commit(hipEvent_t (&ev)[3]) {
  if (!g_prof.on) return;
  if (ev[0] && ev[1] && ev[2])
    g_prof.marks.push_back({ev[0], ev[1], ev[2]});
  else
    for (auto x : ev)
      if (x) g_prof.pool.push_back(x);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace carve-up for one call.
struct Plan {
  int fmt, mode, C, D, rho;
  int int8_cfg;  // INT8 GEMM tile configuration the slices are padded for
  size_t elem;  // bytes per slice element
  int64_t mbp, nbp, kbp;
  size_t off_resid_a, off_resid_b, off_pack_a, off_pack_b, off_mu_a, off_mu_b, off_exp_a, off_exp_b, off_sums, total;
};

Plan make_plan(int fmt, int mode, int64_t m, int64_t n, int64_t k, int D) {
  Plan p{};
  p.fmt = fmt;
  p.mode = mode;
  p.C = kComps[fmt];
  p.D = D;
  const bool f32 = fmt == MPGEMM_TS;
  const size_t comp = f32 ? 4 : 8;
  p.mbp = nblocks_padded(m);
  p.nbp = nblocks_padded(n);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  if (mode == MPGEMM_MODE_FLOAT) {
    p.elem = comp;
    p.rho = rho_of(f32 ? 24 : 53, k);
    p.kbp = kblocks_padded(k);
    const size_t ra = D > 1 ? (size_t)p.C * m * k * comp : 0, rb = D > 1 ? (size_t)p.C * k * n * comp : 0;
    p.off_resid_a = take(ra);
    p.off_resid_b = take(rb);
    p.off_pack_a = take((size_t)D * p.mbp * p.kbp * 256 * comp);
    p.off_pack_b = take((size_t)D * p.nbp * p.kbp * 256 * comp);
    p.off_mu_a = take((size_t)D * m * comp);
    p.off_mu_b = take((size_t)D * n * comp);
    p.off_exp_a = take((size_t)D * m * 4);
    p.off_exp_b = take((size_t)D * n * 4);
  } else {
    p.elem = 1;
    p.rho = 0;
    p.int8_cfg = int8_tile_config(m, n, g_opt.int8_tile);
    p.mbp = nblocks8_padded(m, int8_tile_blocks(p.int8_cfg));
    p.nbp = nblocks8_padded(n, int8_tile_blocks(p.int8_cfg));
    p.kbp = kblocks8_padded(k);
    p.off_resid_a = p.off_resid_b = take(0);
    p.off_pack_a = take((size_t)D * p.mbp * p.kbp * 1024);
    p.off_pack_b = take((size_t)D * p.nbp * p.kbp * 1024);
    p.off_mu_a = take((size_t)m * 8);
    p.off_mu_b = take((size_t)n * 8);
    p.off_exp_a = take((size_t)m * 4);
    p.off_exp_b = take((size_t)n * 4);
    const int64_t nchunks = ceil_div(p.kbp, int8_kblocks_per_chunk(D));
    p.off_sums = take((size_t)D * nchunks * p.mbp * p.nbp * 1024 * 4);  // blocked, padded planes
  }
  p.total = o;
  return p;
}

// Stream-ordered workspace: the thread's attached buffer, or an allocation on
// the stream that is released (to the device's pool) at the end of the call.
struct Workspace {
  char *base = nullptr;
  bool owned = false;
  hipStream_t st = nullptr;
  ~Workspace() {
    if (owned && base) (void)hipFreeAsync(base, st);
  }
};

std::mutex g_pool_mu;
bool g_pool_ready[64] = {};
int g_arch_ok[64] = {};  // 0 unknown, 1 gfx950, -1 other

void keep_pool_memory(int dev) {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  if (dev < 0 || dev >= 64 || g_pool_ready[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t threshold = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
  }
  g_pool_ready[dev] = true;
}

int acquire(Workspace &ws, size_t bytes, hipStream_t st) {
  ws.st = st;
  if (g_opt.ws) {
    if (g_opt.ws_bytes < bytes) return MPGEMM_ERR_WORKSPACE;
    ws.base = static_cast<char *>(g_opt.ws);
    return 0;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MPGEMM_ERR_HIP;
  keep_pool_memory(dev);
  void *p = nullptr;
  if (hipMallocAsync(&p, bytes > 0 ? bytes : 256, st) != hipSuccess || !p) {
    (void)hipGetLastError();
    return MPGEMM_ERR_WORKSPACE;
  }
  ws.base = static_cast<char *>(p);
  ws.owned = true;
  return 0;
}

// Called on entry by every call that launches work.  It also clears the
// thread's last-error slot: the launches below report their own failures
// through hipGetLastError, so an error left there by an earlier, unrelated
// runtime call (another library on this thread) must not be taken for theirs.
int check_device_cached() {
  (void)hipGetLastError();
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MPGEMM_ERR_HIP;
  if (dev >= 0 && dev < 64 && g_arch_ok[dev] != 0) return g_arch_ok[dev] > 0 ? 0 : MPGEMM_ERR_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MPGEMM_ERR_HIP;
  const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
  if (dev >= 0 && dev < 64) g_arch_ok[dev] = ok ? 1 : -1;
  return ok ? 0 : MPGEMM_ERR_DEVICE;
}

int hip_status(hipError_t e) { return e == hipSuccess ? 0 : MPGEMM_ERR_HIP; }

int validate(int m, int n, int k, const void *A, int lda, const void *B, int ldb, const void *C, int ldc) {
  if (m < 0) return -1;
  if (n < 0) return -2;
  if (k < 0) return -3;
  if (!A && m > 0 && k > 0) return -4;
  if (lda < (m > 1 ? m : 1)) return -5;
  if (!B && k > 0 && n > 0) return -6;
  if (ldb < (k > 1 ? k : 1)) return -7;
  if (!C && m > 0 && n > 0) return -8;
  if (ldc < (m > 1 ? m : 1)) return -9;
  if (m > kMaxDim || n > kMaxDim || k > kMaxDim) return MPGEMM_ERR_TOO_LARGE;
  return 0;
}

template <typename T>
SplitOperand<T> operand_a(const T *A, int m, int k, int lda, const Plan &p, char *base) {
  SplitOperand<T> o{};
  o.X = A;
  o.comp_stride = (int64_t)lda * k;
  o.sv = 1;
  o.sp = lda;
  o.nvec = m;
  o.len = k;
  o.orient = 0;
  o.resid = reinterpret_cast<T *>(base + p.off_resid_a);
  o.packed = base + p.off_pack_a;
  o.nbp = p.mbp;
  o.kbp = p.kbp;
  o.mu = base + p.off_mu_a;
  o.last_literal = g_opt.last_slice;
  o.exps = reinterpret_cast<int *>(base + p.off_exp_a);
  return o;
}

template <typename T>
SplitOperand<T> operand_b(const T *B, int k, int n, int ldb, const Plan &p, char *base) {
  SplitOperand<T> o{};
  o.X = B;
  o.comp_stride = (int64_t)ldb * n;
  o.sv = ldb;
  o.sp = 1;
  o.nvec = n;
  o.len = k;
  o.orient = 1;
  o.resid = reinterpret_cast<T *>(base + p.off_resid_b);
  o.packed = base + p.off_pack_b;
  o.nbp = p.nbp;
  o.kbp = p.kbp;
  o.mu = base + p.off_mu_b;
  o.last_literal = g_opt.last_slice;
  o.exps = reinterpret_cast<int *>(base + p.off_exp_b);
  return o;
}

template <typename T, int C>
hipError_t split_both(const SplitOperand<T> &a, const SplitOperand<T> &b, const Plan &p, hipStream_t st) {
  if (p.mode == MPGEMM_MODE_INT8) {
    if constexpr (sizeof(T) == 8) return launch_split_int8<C>(a, b, p.D, st);
    return hipErrorInvalidValue;
  }
  if constexpr (C <= 4) return launch_split_plain<T, C>(a, b, p.D, p.rho, g_opt.split_kernel == 0, st);
  return hipErrorInvalidValue;  // longer expansions: INT8 form only
}

template <typename T, int C>
hipError_t gemm_launch(const Plan &p, char *base, int m, int n, int k, T *Cout, int ldc, int dbg_pair, void *dbg_out,
                       int lddbg, hipStream_t st) {
  if (p.mode == MPGEMM_MODE_INT8) {
    if constexpr (sizeof(T) == 8)
      return launch_gemm_int8<C>(base + p.off_pack_a, base + p.off_pack_b,
                                 reinterpret_cast<const int *>(base + p.off_exp_a),
                                 reinterpret_cast<const int *>(base + p.off_exp_b),
                                 reinterpret_cast<int32_t *>(base + p.off_sums), p.mbp, p.nbp, p.kbp, m, n, p.D, Cout,
                                 ldc, (int64_t)ldc * n, dbg_pair, static_cast<int64_t *>(dbg_out), lddbg,
                                 p.int8_cfg, st);
    return hipErrorInvalidValue;
  }
  if constexpr (C <= 4)
    return launch_gemm_plain<T, C>(base + p.off_pack_a, base + p.off_pack_b, p.mbp, p.nbp, p.kbp, m, n, p.D, Cout,
                                   ldc, (int64_t)ldc * n, dbg_pair, static_cast<double *>(dbg_out), lddbg,
                                   layout_for(p.fmt), st);
  return hipErrorInvalidValue;
}

// The launch sequence of one product (split, then the fused slice products
// and accumulation) on the workspace at `base`, laid out by plan p.  With
// `profile`, records the thread's stage-timing events if they are enabled.
template <typename T, int C>
hipError_t launch_product(const Plan &p, char *base, int m, int n, int k, const T *A, int lda, const T *B, int ldb,
                          T *Cm, int ldc, bool profile, hipStream_t st) {
  const SplitOperand<T> a = operand_a(A, m, k, lda, p, base), b = operand_b(B, k, n, ldb, p, base);
  const bool prof = profile && g_prof.on;
  std::array<hipEvent_t, 3> ev{nullptr, nullptr, nullptr};
  if (prof) {
    for (auto &x : ev) x = g_prof.take();
    if (ev[0]) (void)hipEventRecord(ev[0], st);
  }
  hipError_t e = split_both<T, C>(a, b, p, st);
  if (ev[1]) (void)hipEventRecord(ev[1], st);
  if (e == hipSuccess) e = gemm_launch<T, C>(p, base, m, n, k, Cm, ldc, -1, nullptr, 0, st);
  if (ev[2]) (void)hipEventRecord(ev[2], st);
  if (prof) {
    if (ev[0] && ev[1] && ev[2])
      g_prof.marks.push_back(ev);
    else
      for (auto x : ev)
        if (x) g_prof.pool.push_back(x);
  }
  return e;
}

// One product in the given form with D slices (arguments already validated).
template <typename T, int C>
int run_with(int fmt, int mode, int D, int m, int n, int k, const T *A, int lda, const T *B, int ldb, T *Cm, int ldc,
             hipStream_t st) {
  int s;
  g_opt.last_slices = D;
  if (m == 0 || n == 0) return 0;
  if (k == 0) return hip_status(launch_zero_matrix(Cm, sizeof(T), C, m, n, ldc, (int64_t)ldc * n, st));
  const Plan p = make_plan(fmt, mode, m, n, k, D);
  Workspace ws;
  if ((s = acquire(ws, p.total, st))) return s;
  return hip_status(launch_product<T, C>(p, ws.base, m, n, k, A, lda, B, ldb, Cm, ldc, true, st));
}

// Slice counts chosen from the data (mpgemm_set_num_slices(fmt, FLOAT,
// MPGEMM_SLICES_DATA)): kMaxPairLim slices are made, the certificate's
// quantities (the slice exponents, the remainders after the last slice, the
// row and column sums of |A_0| and |B_0| and the product |A_0| |B_0|) are
// formed before the slice products, and each 64 x 64 tile of C takes only
// the pairs its entries need to meet 2^-t (|A||B|) (launch_tile_pairs).
constexpr int kSlicesData = -1;

bool data_mode(int fmt, int mode) { return mode == MPGEMM_MODE_FLOAT && g_opt.slices[fmt][mode] == kSlicesData; }

struct DataPlan {
  Plan p;
  size_t off_abs_a, off_abs_b, off_rs, off_cs, off_raw, off_lims, total;
  int64_t tiles_m, tiles_n;
};

DataPlan make_data_plan(int fmt, int64_t m, int64_t n, int64_t k, bool raw_outside) {
  DataPlan d{};
  d.p = make_plan(fmt, MPGEMM_MODE_FLOAT, m, n, k, kMaxPairLim);
  size_t o = d.p.total;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  const int64_t kbp = kblocks_padded(k);
  d.tiles_m = nblocks_padded(m) / kTileBlocks;
  d.tiles_n = nblocks_padded(n) / kTileBlocks;
  d.off_abs_a = take((size_t)nblocks_padded(m) * kbp * 256 * 8);
  d.off_abs_b = take((size_t)nblocks_padded(n) * kbp * 256 * 8);
  d.off_rs = take((size_t)m * 8);
  d.off_cs = take((size_t)n * 8);
  d.off_raw = take(raw_outside ? 0 : (size_t)2 * m * n * 8);
  d.off_lims = take((size_t)d.tiles_m * d.tiles_n * kMaxPairLim);
  d.total = o;
  return d;
}

// C = AB with the pairs chosen per tile; with cert (2 m n doubles) and worst,
// also the certificate of that C (its plane 0 first holds |A_0| |B_0|).
template <typename T, int C>
int run_data(int fmt, int m, int n, int k, const T *A, int lda, const T *B, int ldb, T *Cm, int ldc, double *cert,
             double *worst, hipStream_t st) {
  int s;
  const int D = kMaxPairLim;
  g_opt.last_slices = D;
  if (cert && g_opt.last_slice != 0) return MPGEMM_ERR_UNSUPPORTED;
  if (m == 0 || n == 0 || k == 0) {
    hipError_t e = hipSuccess;
    if (worst) e = launch_fill32(worst, 2, 0u, st);
    if (e == hipSuccess && cert && m > 0 && n > 0) e = launch_fill32(cert, (int64_t)4 * m * n, 0u, st);
    if (e == hipSuccess && m > 0 && n > 0) e = launch_zero_matrix(Cm, sizeof(T), C, m, n, ldc, (int64_t)ldc * n, st);
    return hip_status(e);
  }
  const DataPlan d = make_data_plan(fmt, m, n, k, cert != nullptr);
  const Plan &p = d.p;
  Workspace ws;
  if ((s = acquire(ws, d.total, st))) return s;
  char *base = ws.base;
  const SplitOperand<T> a = operand_a(A, m, k, lda, p, base), b = operand_b(B, k, n, ldb, p, base);
  double *raw = cert ? cert : reinterpret_cast<double *>(base + d.off_raw);
  double *rs = reinterpret_cast<double *>(base + d.off_rs), *cs = reinterpret_cast<double *>(base + d.off_cs);
  int8_t *lims = reinterpret_cast<int8_t *>(base + d.off_lims);
  const int S = sizeof(T) == 8 ? 53 : 24;
  const int layout = layout_for(fmt);
  std::array<hipEvent_t, 3> ev{nullptr, nullptr, nullptr};
  if (g_prof.on) {
    for (auto &x : ev) x = g_prof.take();
    if (ev[0]) (void)hipEventRecord(ev[0], st);
  }
  hipError_t e = split_both<T, C>(a, b, p, st);
  // |A_0| and |B_0| in the binary64 packed layout (the geometry of the binary64 slices)
  SplitOperand<T> ca = a, cb = b;
  ca.nbp = nblocks_padded(m);
  cb.nbp = nblocks_padded(n);
  ca.kbp = cb.kbp = kblocks_padded(k);
  if (e == hipSuccess)
    e = launch_abs_lead_product<T>(ca, cb, m, n, raw, reinterpret_cast<double *>(base + d.off_abs_a),
                                   reinterpret_cast<double *>(base + d.off_abs_b), rs, cs, layout, st);
  if (e == hipSuccess)
    e = launch_tile_pairs(m, n, k, D, p.rho, S, C, kBoundBits[fmt], a.exps, b.exps, rs, cs, raw, d.tiles_m, d.tiles_n,
                          lims, st);
  if (ev[1]) (void)hipEventRecord(ev[1], st);
  if (e == hipSuccess)
    e = launch_gemm_plain_pruned<T, C>(base + p.off_pack_a, base + p.off_pack_b, p.mbp, p.nbp, p.kbp, m, n, D, Cm,
                                       ldc, (int64_t)ldc * n, lims, layout, st);
  if (ev[2]) (void)hipEventRecord(ev[2], st);
  if (g_prof.on) {
    if (ev[0] && ev[1] && ev[2])
      g_prof.marks.push_back(ev);
    else
      for (auto x : ev)
        if (x) g_prof.pool.push_back(x);
  }
  if (e == hipSuccess && cert)
    e = launch_certify<T>(ca, cb, m, n, k, D, p.rho, C, 0, cert, worst, nullptr, nullptr, rs, cs, layout, st, lims,
                          true);
  return hip_status(e);
}

// The pair sets run_data would use: split, |A_0| |B_0| and the selection,
// then a copy of the sets (tiles_m x tiles_n x kMaxPairLim counts).
template <typename T, int C>
int debug_pair_sets_t(int fmt, int m, int n, int k, const T *A, int lda, const T *B, int ldb, int8_t *out,
                      hipStream_t st) {
  int s;
  if (m == 0 || n == 0) return 0;
  const DataPlan d = make_data_plan(fmt, m, n, k, false);
  if (k == 0) return hip_status(launch_fill32(out, (int64_t)d.tiles_m * d.tiles_n * kMaxPairLim / 4, 0u, st));
  const Plan &p = d.p;
  Workspace ws;
  if ((s = acquire(ws, d.total, st))) return s;
  char *base = ws.base;
  const SplitOperand<T> a = operand_a(A, m, k, lda, p, base), b = operand_b(B, k, n, ldb, p, base);
  double *raw = reinterpret_cast<double *>(base + d.off_raw);
  double *rs = reinterpret_cast<double *>(base + d.off_rs), *cs = reinterpret_cast<double *>(base + d.off_cs);
  int8_t *lims = reinterpret_cast<int8_t *>(base + d.off_lims);
  const int layout = layout_for(fmt);
  hipError_t e = split_both<T, C>(a, b, p, st);
  SplitOperand<T> ca = a, cb = b;
  ca.nbp = nblocks_padded(m);
  cb.nbp = nblocks_padded(n);
  ca.kbp = cb.kbp = kblocks_padded(k);
  if (e == hipSuccess)
    e = launch_abs_lead_product<T>(ca, cb, m, n, raw, reinterpret_cast<double *>(base + d.off_abs_a),
                                   reinterpret_cast<double *>(base + d.off_abs_b), rs, cs, layout, st);
  if (e == hipSuccess)
    e = launch_tile_pairs(m, n, k, kMaxPairLim, p.rho, sizeof(T) == 8 ? 53 : 24, C, kBoundBits[fmt], a.exps, b.exps,
                          rs, cs, raw, d.tiles_m, d.tiles_n, lims, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, lims, (size_t)d.tiles_m * d.tiles_n * kMaxPairLim, hipMemcpyDeviceToDevice, st);
  return hip_status(e);
}

// Simple in-format product (Section 4.4's comparison), planar formats.
int run_simple(int fmt, int staging, int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *Cm,
               int ldc, hipStream_t st) {
  if (fmt < 0 || fmt >= kNumFmt) return -1;
  if (staging != 0 && staging != 1) return -2;
  int s = validate(m, n, k, A, lda, B, ldb, Cm, ldc);
  if (s) return s < 0 ? s - 2 : s;  // shifted past (fmt, staging)
  if ((s = check_device_cached())) return s;
  if (m == 0 || n == 0) return 0;
  const int elem = fmt == MPGEMM_TS ? 4 : 8;
  if (k == 0) return hip_status(launch_zero_matrix(Cm, elem, kComps[fmt], m, n, ldc, (int64_t)ldc * n, st));
  const bool staged = staging == 1;
  switch (fmt) {
    case MPGEMM_DD: return hip_status(launch_simple<0>(m, n, k, A, lda, B, ldb, Cm, ldc, staged, st));
    case MPGEMM_TD: return hip_status(launch_simple<1>(m, n, k, A, lda, B, ldb, Cm, ldc, staged, st));
    case MPGEMM_QD: return hip_status(launch_simple<2>(m, n, k, A, lda, B, ldb, Cm, ldc, staged, st));
    default: return hip_status(launch_simple<3>(m, n, k, A, lda, B, ldb, Cm, ldc, staged, st));
  }
}

// D+S arguments: (m, n, k, Ahi, Alo, lda, Bhi, Blo, ldb, Chi, Clo, ldc) at
// positions base + 1 ...; 0 if valid.
int validate_ds(int base, int m, int n, int k, const void *Ahi, const void *Alo, int lda, const void *Bhi,
                const void *Blo, int ldb, const void *Chi, const void *Clo, int ldc) {
  if (m < 0) return -(base + 1);
  if (n < 0) return -(base + 2);
  if (k < 0) return -(base + 3);
  if (!Ahi && m > 0 && k > 0) return -(base + 4);
  if (!Alo && m > 0 && k > 0) return -(base + 5);
  if (lda < (m > 1 ? m : 1)) return -(base + 6);
  if (!Bhi && k > 0 && n > 0) return -(base + 7);
  if (!Blo && k > 0 && n > 0) return -(base + 8);
  if (ldb < (k > 1 ? k : 1)) return -(base + 9);
  if (!Chi && m > 0 && n > 0) return -(base + 10);
  if (!Clo && m > 0 && n > 0) return -(base + 11);
  if (ldc < (m > 1 ? m : 1)) return -(base + 12);
  if (m > kMaxDim || n > kMaxDim || k > kMaxDim) return MPGEMM_ERR_TOO_LARGE;
  return 0;
}

int run_simple_ds(int staging, int m, int n, int k, const double *Ahi, const float *Alo, int lda, const double *Bhi,
                  const float *Blo, int ldb, double *Chi, float *Clo, int ldc, hipStream_t st) {
  if (staging != 0 && staging != 1) return -1;
  int s = validate_ds(1, m, n, k, Ahi, Alo, lda, Bhi, Blo, ldb, Chi, Clo, ldc);
  if (s) return s;
  if ((s = check_device_cached())) return s;
  if (m == 0 || n == 0) return 0;
  if (k == 0) {
    hipError_t e = launch_zero_matrix(Chi, 8, 1, m, n, ldc, 0, st);
    if (e == hipSuccess) e = launch_zero_matrix(Clo, 4, 1, m, n, ldc, 0, st);
    return hip_status(e);
  }
  return hip_status(launch_simple_ds(m, n, k, Ahi, Alo, lda, Bhi, Blo, ldb, Chi, Clo, ldc, staging == 1, st));
}

// D+S through the DD Ozaki product: the inputs read as DD (exact), the DD
// product in the thread's DD slice form and slice count, C rounded to D+S.
int run_ds(int m, int n, int k, const double *Ahi, const float *Alo, int lda, const double *Bhi, const float *Blo,
           int ldb, double *Chi, float *Clo, int ldc, hipStream_t st) {
  int s = validate_ds(0, m, n, k, Ahi, Alo, lda, Bhi, Blo, ldb, Chi, Clo, ldc);
  if (s) return s;
  if ((s = check_device_cached())) return s;
  const int mode = g_opt.mode[MPGEMM_DD];
  const int D = slices_for(MPGEMM_DD, mode, k);
  g_opt.last_slices = D;
  if (m == 0 || n == 0) return 0;
  if (k == 0) {
    hipError_t e = launch_zero_matrix(Chi, 8, 1, m, n, ldc, 0, st);
    if (e == hipSuccess) e = launch_zero_matrix(Clo, 4, 1, m, n, ldc, 0, st);
    return hip_status(e);
  }
  const Plan p = make_plan(MPGEMM_DD, mode, m, n, k, D);
  const size_t a_bytes = align256((size_t)2 * m * k * 8), b_bytes = align256((size_t)2 * k * n * 8);
  const size_t c_bytes = align256((size_t)2 * m * n * 8);
  Workspace ws;
  if ((s = acquire(ws, p.total + a_bytes + b_bytes + c_bytes, st))) return s;
  double *Add = reinterpret_cast<double *>(ws.base + p.total);
  double *Bdd = reinterpret_cast<double *>(ws.base + p.total + a_bytes);
  double *Cdd = reinterpret_cast<double *>(ws.base + p.total + a_bytes + b_bytes);
  hipError_t e = launch_ds_to_dd(m, k, Ahi, Alo, lda, Add, st);
  if (e == hipSuccess) e = launch_ds_to_dd(k, n, Bhi, Blo, ldb, Bdd, st);
  if (e == hipSuccess) e = launch_product<double, 2>(p, ws.base, m, n, k, Add, m, Bdd, k, Cdd, m, true, st);
  if (e == hipSuccess) e = launch_dd_to_ds(m, n, Cdd, Chi, Clo, ldc, st);
  return hip_status(e);
}

// Scratch of the allocation-free DD entry point: a fixed device array, one
// copy per device, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// its device address is looked up once per device with hipGetSymbolAddress
// and that address is what the kernels receive.
constexpr size_t kScratchBytes = MPGEMM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
char *g_scratch_ptr[64] = {};

int scratch_of_current_device(char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MPGEMM_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return MPGEMM_ERR_HIP;
    }
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

// mpgemm_dd with its workspace in the device's scratch array instead of an
// allocation: the same plan and kernels, so the same result bit for bit.
int run_dd_noalloc(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *Cm, int ldc,
                   hipStream_t st) {
  int s = validate(m, n, k, A, lda, B, ldb, Cm, ldc);
  if (s) return s;
  if ((s = check_device_cached())) return s;
  const int mode = g_opt.mode[MPGEMM_DD];
  const int D = slices_for(MPGEMM_DD, mode, k);
  g_opt.last_slices = D;
  if (m == 0 || n == 0) return 0;
  if (k == 0) return hip_status(launch_zero_matrix(Cm, sizeof(double), 2, m, n, ldc, (int64_t)ldc * n, st));
  const Plan p = make_plan(MPGEMM_DD, mode, m, n, k, D);
  if (p.total > kScratchBytes) return MPGEMM_ERR_TOO_LARGE;
  char *base = nullptr;
  if ((s = scratch_of_current_device(&base))) return s;
  return hip_status(launch_product<double, 2>(p, base, m, n, k, A, lda, B, ldb, Cm, ldc, false, st));
}

template <typename T, int C>
int run(int fmt, int m, int n, int k, const T *A, int lda, const T *B, int ldb, T *Cm, int ldc, hipStream_t st) {
  int s = validate(m, n, k, A, lda, B, ldb, Cm, ldc);
  if (s) return s;
  if ((s = check_device_cached())) return s;
  const int mode = g_opt.mode[fmt];
  if (data_mode(fmt, mode)) return run_data<T, C>(fmt, m, n, k, A, lda, B, ldb, Cm, ldc, nullptr, nullptr, st);
  return run_with<T, C>(fmt, mode, slices_for(fmt, mode, k), m, n, k, A, lda, B, ldb, Cm, ldc, st);
}

// Longer binary64 expansions (c = 2 .. kMaxNd components), INT8 form: the
// policy of the INT8 form with the bound 2^-(50 c) (|A||B|) (DD / TD / QD:
// 100 / 150 / 200 bits).
int nd_auto_slices(int c, int64_t k) { return (50 * c + (k < 2048 ? 14 : 10) + 6) / 7; }

template <int C>
int run_nd(int D, int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *Cm, int ldc,
           hipStream_t st) {
  int s = validate(m, n, k, A, lda, B, ldb, Cm, ldc);
  if (s) return s < 0 ? s - 2 : s;  // shifted past (c, D)
  if ((s = check_device_cached())) return s;
  return run_with<double, C>(MPGEMM_QD, MPGEMM_MODE_INT8, D > 0 ? D : nd_auto_slices(C, k), m, n, k, A, lda, B, ldb,
                             Cm, ldc, st);
}

template <typename T, int C>
int debug_split_t(int fmt, int mode, int operand, int rows, int cols, const T *X, int ldx, int D, void *slices,
                  int *exps, hipStream_t st) {
  if (rows < 0) return -4;
  if (cols < 0) return -5;
  if (!X && rows > 0 && cols > 0) return -6;
  if (ldx < (rows > 1 ? rows : 1)) return -7;
  if (D < 0) return -8;
  if (!slices || !exps) return -9;
  int s;
  if ((s = check_device_cached())) return s;
  const int m = operand == 0 ? rows : 0, k = operand == 0 ? cols : rows, n = operand == 0 ? 0 : cols;
  if (D == 0) D = slices_for(fmt, mode, k);
  if (rows == 0 || cols == 0) return 0;
  const Plan p = make_plan(fmt, mode, m, n, k, D);
  Workspace ws;
  if ((s = acquire(ws, p.total, st))) return s;
  SplitOperand<T> a = operand_a(operand == 0 ? X : (const T *)nullptr, m, k, ldx, p, ws.base);
  SplitOperand<T> b = operand_b(operand == 1 ? X : (const T *)nullptr, k, n, ldx, p, ws.base);
  hipError_t e = split_both<T, C>(a, b, p, st);
  if (e != hipSuccess) return MPGEMM_ERR_HIP;
  const int nvec = operand == 0 ? rows : cols;
  const int64_t nbp = operand == 0 ? p.mbp : p.nbp;
  e = launch_unpack((int)p.elem, ws.base + (operand == 0 ? p.off_pack_a : p.off_pack_b), nbp, p.kbp, D, operand, rows,
                    cols, slices, st);
  if (e != hipSuccess) return MPGEMM_ERR_HIP;
  const size_t nexp = mode == MPGEMM_MODE_FLOAT ? (size_t)D * nvec : (size_t)nvec;
  e = hipMemcpyAsync(exps, ws.base + (operand == 0 ? p.off_exp_a : p.off_exp_b), nexp * sizeof(int),
                     hipMemcpyDeviceToDevice, st);
  return hip_status(e);
}

template <typename T, int C>
int debug_products_t(int fmt, int mode, int m, int n, int k, const T *A, int lda, const T *B, int ldb, int D, int a,
                     int b, void *out, int ldo, hipStream_t st) {
  int s = validate(m, n, k, A, lda, B, ldb, out, ldo);
  if (s) return s < 0 ? s - 2 : s;  // shifted past (fmt, mode)
  if ((s = check_device_cached())) return s;
  if (D == 0) D = slices_for(fmt, mode, k);
  if (mode == MPGEMM_MODE_FLOAT && (a < 1 || b < 1 || a + b > D + 1)) return -12;
  if (mode == MPGEMM_MODE_INT8 && (a < 1 || a > D)) return -12;
  if (m == 0 || n == 0 || k == 0) return 0;
  const Plan p = make_plan(fmt, mode, m, n, k, D);
  Workspace ws;
  if ((s = acquire(ws, p.total, st))) return s;
  const SplitOperand<T> sa = operand_a(A, m, k, lda, p, ws.base), sb = operand_b(B, k, n, ldb, p, ws.base);
  hipError_t e = split_both<T, C>(sa, sb, p, st);
  const int sel = mode == MPGEMM_MODE_FLOAT ? (a - 1) * D + (b - 1) : a;
  if (e == hipSuccess) e = gemm_launch<T, C>(p, ws.base, m, n, k, nullptr, m, sel, out, ldo, st);
  return hip_status(e);
}

// C = AB as run() computes it in the binary64/binary32 form, then the
// a-posteriori certificate (certify.hip) from the same split.
template <typename T, int C>
int certify_run(int fmt, int mode, int D, int m, int n, int k, const T *A, int lda, const T *B, int ldb, T *Cm,
                int ldc, double *cert, double *worst, hipStream_t st) {
  int s;
  if (mode == MPGEMM_MODE_FLOAT && g_opt.last_slice != 0) return MPGEMM_ERR_UNSUPPORTED;
  g_opt.last_slices = D;
  if (mode == MPGEMM_MODE_FLOAT && sizeof(T) == 4 && D < 2) return MPGEMM_ERR_UNSUPPORTED;  // plane 0 holds |A_0|
  if (m == 0 || n == 0 || k == 0) {
    hipError_t e = launch_fill32(worst, 2, 0u, st);
    if (e == hipSuccess && m > 0 && n > 0) e = launch_fill32(cert, (int64_t)4 * m * n, 0u, st);
    if (e == hipSuccess && m > 0 && n > 0)
      e = launch_zero_matrix(Cm, sizeof(T), C, m, n, ldc, (int64_t)ldc * n, st);
    return hip_status(e);
  }
  const Plan p = make_plan(fmt, mode, m, n, k, D);
  // |A_0| and |B_0| go into the slice buffers in the binary64 packed layout
  SplitOperand<T> ca{}, cb{};
  ca.nbp = nblocks_padded(m);
  cb.nbp = nblocks_padded(n);
  ca.kbp = cb.kbp = kblocks_padded(k);
  if (mode == MPGEMM_MODE_INT8 &&
      ((size_t)D * p.mbp * p.kbp * 1024 < (size_t)ca.nbp * ca.kbp * 256 * 8 ||
       (size_t)D * p.nbp * p.kbp * 1024 < (size_t)cb.nbp * cb.kbp * 256 * 8))
    return MPGEMM_ERR_UNSUPPORTED;  // fewer than about 8 digit planes
  Workspace ws;
  if ((s = acquire(ws, p.total, st))) return s;
  const SplitOperand<T> a = operand_a(A, m, k, lda, p, ws.base), b = operand_b(B, k, n, ldb, p, ws.base);
  hipError_t e = split_both<T, C>(a, b, p, st);
  if (e == hipSuccess) e = gemm_launch<T, C>(p, ws.base, m, n, k, Cm, ldc, -1, nullptr, 0, st);
  ca = a;
  cb = b;
  ca.nbp = nblocks_padded(m);
  cb.nbp = nblocks_padded(n);
  ca.kbp = cb.kbp = kblocks_padded(k);
  if (e == hipSuccess)
    e = launch_certify<T>(ca, cb, m, n, k, D, p.rho, C, mode == MPGEMM_MODE_INT8 ? 1 : 0, cert, worst,
                          reinterpret_cast<double *>(ws.base + p.off_pack_a),
                          reinterpret_cast<double *>(ws.base + p.off_pack_b),
                          reinterpret_cast<double *>(ws.base + p.off_mu_a),
                          reinterpret_cast<double *>(ws.base + p.off_mu_b), 1, st);
  return hip_status(e);
}

template <typename T, int C>
int certify_t(int fmt, int m, int n, int k, const T *A, int lda, const T *B, int ldb, T *Cm, int ldc, double *cert,
              double *worst, hipStream_t st) {
  int s = validate(m, n, k, A, lda, B, ldb, Cm, ldc);
  if (s) return s < 0 ? s - 1 : s;  // shifted past fmt
  if (!cert && m > 0 && n > 0) return -11;
  if (!worst) return -12;
  if ((s = check_device_cached())) return s;
  const int mode = g_opt.mode[fmt];
  if (data_mode(fmt, mode)) return run_data<T, C>(fmt, m, n, k, A, lda, B, ldb, Cm, ldc, cert, worst, st);
  return certify_run<T, C>(fmt, mode, slices_for(fmt, mode, k), m, n, k, A, lda, B, ldb, Cm, ldc, cert, worst, st);
}

// The certified product at D = d_first, d_first + 1, ... d_last, stopping at
// the first D whose certificate meets 2^-t (|A||B|): the slice count chosen
// from the data rather than from the a-priori estimate.  Reads *worst back
// after each attempt (synchronizing the stream).  A D that the certificate
// does not support (TS at D = 1, INT8 with too few digit planes) is skipped.
template <typename T, int C>
int certify_adaptive_t(int fmt, int m, int n, int k, const T *A, int lda, const T *B, int ldb, T *Cm, int ldc,
                       double *cert, double *worst, int d_first, int d_last, int *d_used, hipStream_t st) {
  int s = validate(m, n, k, A, lda, B, ldb, Cm, ldc);
  if (s) return s < 0 ? s - 1 : s;  // shifted past fmt
  if (!cert && m > 0 && n > 0) return -11;
  if (!worst) return -12;
  const int mode = g_opt.mode[fmt];
  const int dmax = mode == MPGEMM_MODE_FLOAT ? kMaxDFloat : kMaxDInt8;
  if (d_first < 1 || d_first > dmax) return -13;
  if (d_last < d_first || d_last > dmax) return -14;
  if (!d_used) return -15;
  if ((s = check_device_cached())) return s;
  const double target = std::ldexp(1.0, -kBoundBits[fmt]);
  int status = MPGEMM_ERR_UNSUPPORTED;
  for (int D = d_first; D <= d_last; ++D) {
    s = certify_run<T, C>(fmt, mode, D, m, n, k, A, lda, B, ldb, Cm, ldc, cert, worst, st);
    if (s == MPGEMM_ERR_UNSUPPORTED) continue;
    if (s) return s;
    *d_used = D;
    status = 0;
    double w = 0.0;
    if (hipMemcpyAsync(&w, worst, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      (void)hipGetLastError();
      return MPGEMM_ERR_HIP;
    }
    if (w <= target) break;
  }
  return status;
}

// Longer expansions (c components, INT8 form), as mpgemm_nd computes them.
template <int C>
int certify_nd_t(int D, int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *Cm, int ldc,
                 double *cert, double *worst, hipStream_t st) {
  int s = validate(m, n, k, A, lda, B, ldb, Cm, ldc);
  if (s) return s < 0 ? s - 2 : s;  // shifted past (c, D)
  if (!cert && m > 0 && n > 0) return -12;
  if (!worst) return -13;
  if ((s = check_device_cached())) return s;
  return certify_run<double, C>(MPGEMM_QD, MPGEMM_MODE_INT8, D > 0 ? D : nd_auto_slices(C, k), m, n, k, A, lda, B,
                                ldb, Cm, ldc, cert, worst, st);
}

// Blocked LU (Section 4.6) of a DD (C = 2) or TD (C = 3) matrix: panels on the
// LU kernels, Schur updates as products of this library in the thread's slice
// form.
template <int C>
int lu_t(int fmt, int n, double *A, int lda, int K, hipStream_t stream) {
  if (n < 0) return -1;
  if (n > 0 && !A) return -2;
  if (lda < std::max(1, n)) return -3;
  if (K < 1) return -4;
  int s = check_device_cached();
  if (s) return s;
  if (n == 0) return 0;
  const int64_t plane = (int64_t)lda * n;
  const int Kmax = std::min(K, n);
  const int rmax = n - std::min(Kmax, n);
  void *buf = nullptr;
  const size_t bytes = rmax > 0 ? (size_t)C * 8 * ((size_t)2 * rmax * Kmax + (size_t)rmax * rmax) : 0;
  if (bytes && (hipMallocAsync(&buf, bytes, stream) != hipSuccess || !buf)) {
    (void)hipGetLastError();
    return MPGEMM_ERR_WORKSPACE;
  }
  double *bl = static_cast<double *>(buf), *bu = bl + (size_t)C * rmax * Kmax, *P = bu + (size_t)C * rmax * Kmax;
  hipError_t e = hipSuccess;
  const int mode = g_opt.mode[fmt];
  for (int j0 = 0; j0 < n && e == hipSuccess && s == 0; j0 += K) {
    const int Kb = std::min(K, n - j0), r = n - j0 - Kb;
    e = launch_lu_panel(C, A, lda, plane, j0, Kb, n, stream);
    if (e != hipSuccess || r == 0) break;
    // A22 -= L21 U12, with L21 (r x Kb) and U12 (Kb x r) copied contiguous
    if ((e = launch_lu_copy(C, A, lda, plane, j0 + Kb, j0, r, Kb, bl, stream)) != hipSuccess) break;
    if ((e = launch_lu_copy(C, A, lda, plane, j0, j0 + Kb, Kb, r, bu, stream)) != hipSuccess) break;
    s = run_with<double, C>(fmt, mode, slices_for(fmt, mode, Kb), r, r, Kb, bl, r, bu, Kb, P, r, stream);
    if (s == 0) e = launch_lu_sub(C, A, lda, plane, j0 + Kb, j0 + Kb, r, r, P, stream);
  }
  if (buf) (void)hipFreeAsync(buf, stream);
  if (s) return s;
  return hip_status(e);
}

int lu_solve_t(int comps, int n, const double *LU, int lda, double *x, hipStream_t stream) {
  if (n < 0) return -1;
  if (n > 0 && !LU) return -2;
  if (lda < std::max(1, n)) return -3;
  if (n > 0 && !x) return -4;
  const int s = check_device_cached();
  if (s) return s;
  if (n == 0) return 0;
  return hip_status(launch_lu_solve(comps, LU, lda, (int64_t)lda * n, n, x, stream));
}

}  // namespace host
}  // namespace mp

using namespace mp::host;

namespace {

bool fmt_ok(int fmt) { return fmt >= 0 && fmt < kNumFmt; }
bool mode_ok(int fmt, int mode) {
  return mode == MPGEMM_MODE_FLOAT || (mode == MPGEMM_MODE_INT8 && fmt != MPGEMM_TS);
}

__global__ void k_zero_matrix(char *C, int elem_bytes, int comps, int m, int n, int ldc, int64_t c_stride) {
  const int64_t total = (int64_t)comps * m * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / ((int64_t)m * n));
    const int64_t rem = t % ((int64_t)m * n);
    const int64_t i = rem % m, j = rem / m;
    const int64_t off = (r * c_stride + i + j * ldc) * elem_bytes;
    if (elem_bytes == 8)
      *reinterpret_cast<double *>(C + off) = 0.0;
    else
      *reinterpret_cast<float *>(C + off) = 0.0f;
  }
}

}  // namespace

namespace mp {
hipError_t launch_zero_matrix(void *C, int elem_bytes, int comps, int m, int n, int ldc, int64_t c_stride,
                              hipStream_t st) {
  const int64_t total = (int64_t)comps * m * n;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = ceil_div(total, 256);
  hipLaunchKernelGGL(k_zero_matrix, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st,
                     static_cast<char *>(C), elem_bytes, comps, m, n, ldc, c_stride);
  return hipGetLastError();
}
}  // namespace mp

extern "C" {

int mpgemm_dd(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
              hipStream_t stream) {
  return run<double, 2>(MPGEMM_DD, m, n, k, A, lda, B, ldb, C, ldc, stream);
}
int mpgemm_dd_noalloc(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                      hipStream_t stream) {
  return run_dd_noalloc(m, n, k, A, lda, B, ldb, C, ldc, stream);
}
int mpgemm_td(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
              hipStream_t stream) {
  return run<double, 3>(MPGEMM_TD, m, n, k, A, lda, B, ldb, C, ldc, stream);
}
int mpgemm_qd(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
              hipStream_t stream) {
  return run<double, 4>(MPGEMM_QD, m, n, k, A, lda, B, ldb, C, ldc, stream);
}
int mpgemm_ts(int m, int n, int k, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
              hipStream_t stream) {
  return run<float, 3>(MPGEMM_TS, m, n, k, A, lda, B, ldb, C, ldc, stream);
}

int mpgemm_ds(int m, int n, int k, const double *Ahi, const float *Alo, int lda, const double *Bhi, const float *Blo,
              int ldb, double *Chi, float *Clo, int ldc, hipStream_t stream) {
  return run_ds(m, n, k, Ahi, Alo, lda, Bhi, Blo, ldb, Chi, Clo, ldc, stream);
}

int mpgemm_debug_pair_sets(int fmt, int m, int n, int k, const void *A, int lda, const void *B, int ldb,
                           int8_t *sets, hipStream_t stream) {
  if (!fmt_ok(fmt)) return -1;
  int s = validate(m, n, k, A, lda, B, ldb, sets, m > 1 ? m : 1);
  if (s) return s < 0 ? (s == -8 ? -10 : s - 1) : s;  // shifted past fmt; sets is argument 10
  if ((s = check_device_cached())) return s;
  if (fmt == MPGEMM_TS)
    return debug_pair_sets_t<float, 3>(fmt, m, n, k, (const float *)A, lda, (const float *)B, ldb, sets, stream);
  if (fmt == MPGEMM_DD)
    return debug_pair_sets_t<double, 2>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, sets, stream);
  if (fmt == MPGEMM_TD)
    return debug_pair_sets_t<double, 3>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, sets, stream);
  return debug_pair_sets_t<double, 4>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, sets, stream);
}

int mpgemm_simple(int fmt, int staging, int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *C,
                  int ldc, hipStream_t stream) {
  return run_simple(fmt, staging, m, n, k, A, lda, B, ldb, C, ldc, stream);
}

int mpgemm_ds_simple(int staging, int m, int n, int k, const double *Ahi, const float *Alo, int lda,
                     const double *Bhi, const float *Blo, int ldb, double *Chi, float *Clo, int ldc,
                     hipStream_t stream) {
  return run_simple_ds(staging, m, n, k, Ahi, Alo, lda, Bhi, Blo, ldb, Chi, Clo, ldc, stream);
}

#define MP_ND_CASES(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

int mpgemm_nd(int c, int D, int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C,
              int ldc, hipStream_t stream) {
  if (c < 2 || c > kMaxNd) return -1;
  if (D < 0 || D > kMaxDNd) return -2;
  switch (c) {
#define MP_CASE(CC) \
  case CC:          \
    return run_nd<CC>(D, m, n, k, A, lda, B, ldb, C, ldc, stream);
    MP_ND_CASES(MP_CASE)
#undef MP_CASE
  }
  return -1;
}

int mpgemm_nd_certify(int c, int D, int m, int n, int k, const double *A, int lda, const double *B, int ldb,
                      double *C, int ldc, double *cert, double *worst, hipStream_t stream) {
  if (c < 2 || c > kMaxNd) return -1;
  if (D < 0 || D > kMaxDNd) return -2;
  switch (c) {
#define MP_CASE(CC) \
  case CC:          \
    return certify_nd_t<CC>(D, m, n, k, A, lda, B, ldb, C, ldc, cert, worst, stream);
    MP_ND_CASES(MP_CASE)
#undef MP_CASE
  }
  return -1;
}

int mpgemm_nd_num_slices(int c, int k) {
  if (c < 2 || c > kMaxNd) return -1;
  if (k < 0) return -2;
  return nd_auto_slices(c, k);
}

size_t mpgemm_nd_workspace_bytes(int c, int D, int m, int n, int k) {
  if (c < 2 || c > kMaxNd || D < 0 || D > kMaxDNd || m < 0 || n < 0 || k < 0) return 0;
  if (m == 0 || n == 0 || k == 0) return 0;
  return make_plan(MPGEMM_QD, MPGEMM_MODE_INT8, m, n, k, D > 0 ? D : nd_auto_slices(c, k)).total;
}

int mpgemm_nd_debug_split(int c, int operand, int rows, int cols, const double *X, int ldx, int D, int8_t *digits,
                          int *exps, hipStream_t stream) {
  if (c < 2 || c > kMaxNd) return -1;
  if (operand != 0 && operand != 1) return -2;
  if (D < 0 || D > kMaxDNd) return -7;
  const int k = operand == 0 ? cols : rows;
  if (D == 0) D = nd_auto_slices(c, k);
  switch (c) {
#define MP_CASE(CC)                                                                                            \
  case CC: {                                                                                                   \
    const int s = debug_split_t<double, CC>(MPGEMM_QD, MPGEMM_MODE_INT8, operand, rows, cols, X, ldx, D, digits, \
                                            exps, stream);                                                     \
    return s < 0 ? s + 1 : s; /* (c, operand) in place of (fmt, mode, operand) */                              \
  }
    MP_ND_CASES(MP_CASE)
#undef MP_CASE
  }
  return -1;
}

int mpgemm_nd_debug_products(int c, int m, int n, int k, const double *A, int lda, const double *B, int ldb, int D,
                             int g, int64_t *out, int ldo, hipStream_t stream) {
  if (c < 2 || c > kMaxNd) return -1;
  if (D < 0 || D > kMaxDNd) return -9;
  if (D == 0) D = nd_auto_slices(c, k < 0 ? 0 : k);
  if (g < 1 || g > D) return -10;
  switch (c) {
#define MP_CASE(CC)                                                                                                  \
  case CC: {                                                                                                         \
    const int s = debug_products_t<double, CC>(MPGEMM_QD, MPGEMM_MODE_INT8, m, n, k, A, lda, B, ldb, D, g, 0, out, ldo, \
                                               stream);                                                              \
    return s < 0 ? s + 1 : s; /* c in place of (fmt, mode) */                                                        \
  }
    MP_ND_CASES(MP_CASE)
#undef MP_CASE
  }
  return -1;
}

int mpgemm_load_tune_file(const char *path) {
  std::call_once(g_tune_once, [] {});  // an explicit load replaces the environment's file
  return load_tune_tables(path);
}

int mpgemm_set_mode(int fmt, int mode) {
  if (!fmt_ok(fmt)) return -1;
  if (mode != MPGEMM_MODE_FLOAT && mode != MPGEMM_MODE_INT8) return -2;
  if (!mode_ok(fmt, mode)) return MPGEMM_ERR_UNSUPPORTED;
  g_opt.mode[fmt] = mode;
  return 0;
}
int mpgemm_get_mode(int fmt) { return fmt_ok(fmt) ? g_opt.mode[fmt] : -1; }

int mpgemm_set_tile_layout(int fmt, int layout) {
  if (!fmt_ok(fmt)) return -1;
  if (layout < 0 || layout > 3) return -2;
  g_opt.layout[fmt] = layout;
  return 0;
}
int mpgemm_tile_layout(int fmt) { return fmt_ok(fmt) ? layout_for(fmt) : -1; }

int mpgemm_set_int8_tile(int cfg) {
  if (cfg < 0 || cfg > 4) return -1;
  g_opt.int8_tile = cfg;
  return 0;
}

int mpgemm_set_split_kernel(int kind) {
  if (kind < 0 || kind > 1) return -1;
  g_opt.split_kernel = kind;
  return 0;
}
int mpgemm_split_kernel(void) { return g_opt.split_kernel; }

int mpgemm_set_last_slice(int kind) {
  if (kind < 0 || kind > 1) return -1;
  g_opt.last_slice = kind;
  return 0;
}
int mpgemm_last_slice(void) { return g_opt.last_slice; }

int mpgemm_set_num_slices(int fmt, int mode, int D) {
  if (!fmt_ok(fmt)) return -1;
  if (mode != MPGEMM_MODE_FLOAT && mode != MPGEMM_MODE_INT8) return -2;
  if (!mode_ok(fmt, mode)) return MPGEMM_ERR_UNSUPPORTED;
  if (D == kSlicesData) {
    if (mode != MPGEMM_MODE_FLOAT) return MPGEMM_ERR_UNSUPPORTED;
    g_opt.slices[fmt][mode] = D;
    return 0;
  }
  if (D < 0 || D > (mode == MPGEMM_MODE_FLOAT ? kMaxDFloat : kMaxDInt8)) return -3;
  g_opt.slices[fmt][mode] = D;
  return 0;
}
int mpgemm_num_slices(int fmt, int mode, int k) {
  if (!fmt_ok(fmt)) return -1;
  if (!mode_ok(fmt, mode)) return -2;
  if (k < 0) return -3;
  return slices_for(fmt, mode, k);
}
int mpgemm_last_num_slices(void) { return g_opt.last_slices; }

size_t mpgemm_workspace_bytes(int fmt, int mode, int m, int n, int k, int D) {
  if (!fmt_ok(fmt) || !mode_ok(fmt, mode) || m < 0 || n < 0 || k < 0) return 0;
  if (D == kSlicesData || (D == 0 && data_mode(fmt, mode)))
    return mode == MPGEMM_MODE_FLOAT ? make_data_plan(fmt, m, n, k, false).total : 0;
  if (D <= 0) D = slices_for(fmt, mode, k);
  return make_plan(fmt, mode, m, n, k, D).total;
}
int mpgemm_set_workspace(void *dev_ptr, size_t bytes) {
  if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) & 255)) return -1;
  g_opt.ws = dev_ptr;
  g_opt.ws_bytes = dev_ptr ? bytes : 0;
  return 0;
}

int mpgemm_debug_split(int fmt, int mode, int operand, int rows, int cols, const void *X, int ldx, int D,
                       void *slices, int *exps, hipStream_t stream) {
  if (!fmt_ok(fmt)) return -1;
  if (mode != MPGEMM_MODE_FLOAT && mode != MPGEMM_MODE_INT8) return -2;
  if (!mode_ok(fmt, mode)) return MPGEMM_ERR_UNSUPPORTED;
  if (operand != 0 && operand != 1) return -3;
  if (D > (mode == MPGEMM_MODE_FLOAT ? kMaxDFloat : kMaxDInt8)) return -8;
  switch (fmt) {
    case MPGEMM_DD:
      return debug_split_t<double, 2>(fmt, mode, operand, rows, cols, (const double *)X, ldx, D, slices, exps, stream);
    case MPGEMM_TD:
      return debug_split_t<double, 3>(fmt, mode, operand, rows, cols, (const double *)X, ldx, D, slices, exps, stream);
    case MPGEMM_QD:
      return debug_split_t<double, 4>(fmt, mode, operand, rows, cols, (const double *)X, ldx, D, slices, exps, stream);
    default:
      return debug_split_t<float, 3>(fmt, mode, operand, rows, cols, (const float *)X, ldx, D, slices, exps, stream);
  }
}

int mpgemm_debug_products(int fmt, int mode, int m, int n, int k, const void *A, int lda, const void *B, int ldb,
                          int D, int a, int b, void *out, int ldo, hipStream_t stream) {
  if (!fmt_ok(fmt)) return -1;
  if (mode != MPGEMM_MODE_FLOAT && mode != MPGEMM_MODE_INT8) return -2;
  if (!mode_ok(fmt, mode)) return MPGEMM_ERR_UNSUPPORTED;
  if (D < 0 || D > (mode == MPGEMM_MODE_FLOAT ? kMaxDFloat : kMaxDInt8)) return -10;
  switch (fmt) {
    case MPGEMM_DD:
      return debug_products_t<double, 2>(fmt, mode, m, n, k, (const double *)A, lda, (const double *)B, ldb, D, a, b,
                                         out, ldo, stream);
    case MPGEMM_TD:
      return debug_products_t<double, 3>(fmt, mode, m, n, k, (const double *)A, lda, (const double *)B, ldb, D, a, b,
                                         out, ldo, stream);
    case MPGEMM_QD:
      return debug_products_t<double, 4>(fmt, mode, m, n, k, (const double *)A, lda, (const double *)B, ldb, D, a, b,
                                         out, ldo, stream);
    default:
      return debug_products_t<float, 3>(fmt, mode, m, n, k, (const float *)A, lda, (const float *)B, ldb, D, a, b,
                                        out, ldo, stream);
  }
}

int mpgemm_dd_lu(int n, double *A, int lda, int K, hipStream_t stream) {
  return lu_t<2>(MPGEMM_DD, n, A, lda, K, stream);
}
int mpgemm_td_lu(int n, double *A, int lda, int K, hipStream_t stream) {
  return lu_t<3>(MPGEMM_TD, n, A, lda, K, stream);
}
int mpgemm_dd_lu_solve(int n, const double *LU, int lda, double *x, hipStream_t stream) {
  return lu_solve_t(2, n, LU, lda, x, stream);
}
int mpgemm_td_lu_solve(int n, const double *LU, int lda, double *x, hipStream_t stream) {
  return lu_solve_t(3, n, LU, lda, x, stream);
}

int mpgemm_certify(int fmt, int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *C, int ldc,
                   double *cert, double *worst, hipStream_t stream) {
  if (!fmt_ok(fmt)) return -1;
  switch (fmt) {
    case MPGEMM_DD:
      return certify_t<double, 2>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, (double *)C, ldc, cert,
                                  worst, stream);
    case MPGEMM_TD:
      return certify_t<double, 3>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, (double *)C, ldc, cert,
                                  worst, stream);
    case MPGEMM_QD:
      return certify_t<double, 4>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, (double *)C, ldc, cert,
                                  worst, stream);
    default:
      return certify_t<float, 3>(fmt, m, n, k, (const float *)A, lda, (const float *)B, ldb, (float *)C, ldc, cert,
                                 worst, stream);
  }
}

int mpgemm_certify_adaptive(int fmt, int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *C,
                            int ldc, double *cert, double *worst, int d_first, int d_last, int *d_used,
                            hipStream_t stream) {
  if (!fmt_ok(fmt)) return -1;
  switch (fmt) {
    case MPGEMM_DD:
      return certify_adaptive_t<double, 2>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, (double *)C,
                                           ldc, cert, worst, d_first, d_last, d_used, stream);
    case MPGEMM_TD:
      return certify_adaptive_t<double, 3>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, (double *)C,
                                           ldc, cert, worst, d_first, d_last, d_used, stream);
    case MPGEMM_QD:
      return certify_adaptive_t<double, 4>(fmt, m, n, k, (const double *)A, lda, (const double *)B, ldb, (double *)C,
                                           ldc, cert, worst, d_first, d_last, d_used, stream);
    default:
      return certify_adaptive_t<float, 3>(fmt, m, n, k, (const float *)A, lda, (const float *)B, ldb, (float *)C, ldc,
                                          cert, worst, d_first, d_last, d_used, stream);
  }
}

const char *mpgemm_status_string(int status) {
  if (status == 0) return "success";
  if (status < 0) return "invalid argument";
  switch (status) {
    case MPGEMM_ERR_HIP: return "HIP runtime error";
    case MPGEMM_ERR_WORKSPACE: return "workspace too small or allocation failed";
    case MPGEMM_ERR_DEVICE: return "device is not gfx950";
    case MPGEMM_ERR_UNSUPPORTED: return "unsupported option for this format";
    case MPGEMM_ERR_TOO_LARGE: return "size beyond library limits";
    default: return "unknown status";
  }
}

int mpgemm_check_device(void) { return check_device_cached(); }

int mpgemm_profile_enable(int on) {
  g_prof.on = on != 0;
  return 0;
}

int mpgemm_profile_read(double *split_ms, double *gemm_ms, int max_calls) {
  int done = 0;
  bool failed = false;
  while (done < max_calls && done < (int)g_prof.marks.size()) {
    auto &m = g_prof.marks[done];
    float a = 0, b = 0;
    if (hipEventSynchronize(m[2]) != hipSuccess || hipEventElapsedTime(&a, m[0], m[1]) != hipSuccess ||
        hipEventElapsedTime(&b, m[1], m[2]) != hipSuccess)
      failed = true;
    if (split_ms) split_ms[done] = a;
    if (gemm_ms) gemm_ms[done] = b;
    for (auto x : m) g_prof.pool.push_back(x);
    ++done;
  }
  g_prof.marks.erase(g_prof.marks.begin(), g_prof.marks.begin() + done);
  return failed ? -MPGEMM_ERR_HIP : done;
}

}  // extern "C"
