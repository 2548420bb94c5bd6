// Batched products: many independent products of uneven sizes in one launch
// sequence, captured once per batch shape in a HIP graph.
//
// A batch plan (per host thread, device, stream and shape: format, slice
// form, and every product's m, n, k and D) owns one device workspace holding
// every product's residuals, packed slices, maxima and exponents, plus
//   - the split descriptors of all 2 x count operands and the GEMM
//     descriptors (rewritten before every launch: they carry the caller's
//     pointers),
//   - prefix sums of the split tiles per operand and the (product, tile) work
//     items of the persistent GEMM kernel, in one list per XCD (written once).
// The graph holds: clear the maxima, one max-exponent launch and dmax pass
// launches covering all operands, clear the work counter, and one persistent
// GEMM launch.  In the INT8 form: clear the maxima, the max-exponent launch,
// one digit-split launch over all operands' blocks, clear the work counter,
// the persistent INT8 GEMM over (product, tile, k chunk, diagonal group)
// items and one combine launch over all products.  Kernels take the caller's pointers from the descriptors, so a
// cached graph is replayed with new pointers after one small host-to-device
// copy of the descriptors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/mpgemm.h"
#include "host.h"
#include "internal.h"
#include "layout.h"

namespace mp {
namespace host {
namespace {

constexpr int kMaxPlans = 6;
constexpr int kPersistentGrid = 512;  // 2 workgroups per CU on 256 CUs

// Tile configuration of one product of an INT8 batch: the one set for the
// thread (2 and 4 run as 3); else the 256 x 256 tiles unless padding to them
// exceeds 1.5 times the area padded to 128 x 128.  In batches of products of
// 64 to 1024 rows the 128 x 128 tiles run at about two thirds of the rate of
// the 256 x 256 ones per padded operation (1.03 against 1.55 POP/s), not at
// half as in one large product, whose rule takes twice the area.
int batch_int8_cfg(int64_t m, int64_t n, int cfg_override) {
  if (cfg_override >= 1) return int8_tile_config(m, n, cfg_override) == 1 ? 1 : 3;
  const int64_t area3 = ceil_div(m, 256) * ceil_div(n, 256) * 4, area1 = ceil_div(m, 128) * ceil_div(n, 128);
  return 2 * area3 <= 3 * area1 ? 3 : 1;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct ProductLayout {
  int m, n, k, D, rho;
  int64_t mbp, nbp, kbp;
  size_t resid_a, resid_b, pack_a, pack_b, mu_a, mu_b, exp_a, exp_b;
  // INT8 form: k blocks per chunk, chunks, diagonal groups, diagonal sums
  int kbc = 0, nchunks = 0, groups = 1, cfg = 1;
  size_t sums = 0;
  // binary64/binary32 slices: operand split by the fused kernel (no residual)
  bool fused_a = false, fused_b = false;
};

// The part of an operand that decides its split kernel.
struct OperandShape {
  int64_t kbp, nbp, nvec;
};

struct BatchPlan {
  int device = 0, fmt = 0, mode = 0, layout = 1, int8_tile = 0, split_kernel = 0, last_slice = 0;
  hipStream_t stream = nullptr;
  std::vector<int> m, n, k, D;
  std::vector<ProductLayout> prod;
  std::vector<int> live;  // products with m, n, k > 0
  char *ws = nullptr;
  size_t off_ops = 0, off_descs = 0, desc_bytes = 0, off_prefix0 = 0, off_prefixp = 0, off_prefixf = 0,
         off_items = 0, off_bounds = 0, off_counter = 0, off_mu = 0, mu_bytes = 0, off_prefixc = 0, total = 0;
  int nops = 0, tiles0 = 0, tilesp = 0, stripsf = 0, dmax = 0, nitems = 0, nitems3 = 0;
  int fused_nt = 1024;  // threads of the fused-split workgroups
  int64_t blocks8 = 0, blocksc = 0;  // INT8 form: split blocks, combine blocks
  void *stage = nullptr;
  hipEvent_t stage_done = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;

  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (stage_done) (void)hipEventDestroy(stage_done);
    if (stage) (void)hipHostFree(stage);
    if (ws) (void)hipFree(ws);
    exec = nullptr;
    graph = nullptr;
    stage_done = nullptr;
    stage = nullptr;
    ws = nullptr;
  }
};

struct BatchCache {
  std::vector<BatchPlan *> plans;
  hipStream_t capture[64] = {};
  uint64_t clock = 0;
};
// Owned by the thread and intentionally not destroyed at thread exit (the HIP
// runtime may already be gone then); mpgemm_batched_cache_clear frees it.
thread_local BatchCache *g_batch = nullptr;

BatchCache &cache() {
  if (!g_batch) g_batch = new BatchCache();
  return *g_batch;
}

int tiles64(int64_t a, int64_t b) { return (int)(ceil_div(a, 64) * ceil_div(b, 64)); }

// The work items of a persistent launch as kXcds per-XCD lists (take_item):
// runs of items with the same key (the tiles of one product, or of one
// product's k chunk and diagonal group) stay together in one list, so that the
// workgroups of one XCD read the same operand panels through its L2.  Runs are
// dealt out in decreasing total work, each to the list with the least work so
// far, and every list is ordered by decreasing item work (longest first).
// bounds receives the kXcds + 1 running offsets of the lists in the result.
template <typename Item, typename Key>
std::vector<Item> xcd_lists(const std::vector<Item> &items, Key key, int *bounds) {
  struct Run {
    int64_t key, item_cost, total;
    std::vector<int> idx;
  };
  std::vector<Run> runs;
  {
    std::vector<std::pair<int64_t, int>> keyed(items.size());
    for (size_t i = 0; i < items.size(); ++i) keyed[i] = {key(items[i]), (int)i};
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const std::pair<int64_t, int> &a, const std::pair<int64_t, int> &b) { return a.first < b.first; });
    for (const auto &ki : keyed) {
      if (runs.empty() || runs.back().key != ki.first) runs.push_back({ki.first, items[ki.second].cost, 0, {}});
      runs.back().idx.push_back(ki.second);
      runs.back().total += items[ki.second].cost;
    }
  }
  std::stable_sort(runs.begin(), runs.end(), [](const Run &a, const Run &b) { return a.total > b.total; });
  std::vector<std::vector<const Run *>> lists(kXcds);
  int64_t load[kXcds] = {};
  for (const Run &r : runs) {
    const int q = (int)(std::min_element(load, load + kXcds) - load);
    lists[q].push_back(&r);
    load[q] += r.total;
  }
  std::vector<Item> out;
  out.reserve(items.size());
  bounds[0] = 0;
  for (int q = 0; q < kXcds; ++q) {
    std::stable_sort(lists[q].begin(), lists[q].end(),
                     [](const Run *a, const Run *b) { return a->item_cost > b->item_cost; });
    for (const Run *r : lists[q])
      for (int i : r->idx) out.push_back(items[i]);
    bounds[q + 1] = (int)out.size();
  }
  return out;
}

template <typename T, int C>
int build_plan(BatchPlan &p, hipStream_t st) {
  const size_t w = sizeof(T);
  const int S = sizeof(T) == 8 ? 53 : 24;
  const int count = (int)p.m.size();
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  p.prod.resize(count);
  p.live.clear();
  p.dmax = 0;
  // one fused-split launch for the batch: 512-thread workgroups when every
  // product's vectors allow them, else 1024
  p.fused_nt = 512;
  for (int g = 0; g < count; ++g)
    if (p.m[g] > 0 && p.n[g] > 0 && p.k[g] > 0 && fused_threads<T, C>(kblocks_padded(p.k[g]) * kKBlk) == 1024)
      p.fused_nt = 1024;
  for (int g = 0; g < count; ++g) {
    ProductLayout &L = p.prod[g];
    L.m = p.m[g];
    L.n = p.n[g];
    L.k = p.k[g];
    L.D = p.D[g];
    if (L.m <= 0 || L.n <= 0 || L.k <= 0) continue;
    p.live.push_back(g);
    L.rho = rho_of(S, L.k);
    L.mbp = nblocks_padded(L.m);
    L.nbp = nblocks_padded(L.n);
    L.kbp = kblocks_padded(L.k);
    L.fused_a = p.split_kernel == 0 && fused_strips<T, C>(OperandShape{L.kbp, L.mbp, L.m}, p.fused_nt) >= 0;
    L.fused_b = p.split_kernel == 0 && fused_strips<T, C>(OperandShape{L.kbp, L.nbp, L.n}, p.fused_nt) >= 0;
    L.resid_a = take(L.D > 1 && !L.fused_a ? (size_t)C * L.m * L.k * w : 0);
    L.resid_b = take(L.D > 1 && !L.fused_b ? (size_t)C * L.k * L.n * w : 0);
    L.pack_a = take((size_t)L.D * L.mbp * L.kbp * 256 * w);
    L.pack_b = take((size_t)L.D * L.nbp * L.kbp * 256 * w);
    L.exp_a = take((size_t)L.D * L.m * 4);
    L.exp_b = take((size_t)L.D * L.n * 4);
    p.dmax = std::max(p.dmax, L.D);
  }
  // one region for all maxima (cleared by a single fill)
  p.off_mu = o;
  size_t mo = 0;
  for (int g : p.live) {
    ProductLayout &L = p.prod[g];
    L.mu_a = p.off_mu + mo;
    mo += (size_t)L.D * L.m * w;
    L.mu_b = p.off_mu + mo;
    mo += (size_t)L.D * L.n * w;
  }
  p.mu_bytes = (mo + 3) / 4 * 4;
  o = p.off_mu + align256(mo);
  p.nops = 2 * (int)p.live.size();
  p.off_ops = take(0);
  p.off_descs = p.off_ops + (size_t)p.nops * sizeof(SplitOperand<T>);
  p.desc_bytes = (size_t)p.nops * sizeof(SplitOperand<T>) + p.live.size() * sizeof(PlainGemmDesc);
  o = p.off_ops + align256(p.desc_bytes);
  p.off_prefix0 = take((size_t)(p.nops + 1) * 4);
  p.off_prefixp = take((size_t)(p.nops + 1) * 4);
  p.off_prefixf = take((size_t)(p.nops + 1) * 4);

  // work items: (product slot, tile)
  struct Item {
    int slot, tile;
    int64_t cost;
  };
  std::vector<Item> items;
  for (int slot = 0; slot < (int)p.live.size(); ++slot) {
    const ProductLayout &L = p.prod[p.live[slot]];
    const int ntiles = (int)((L.mbp / kTileBlocks) * (L.nbp / kTileBlocks));
    const int64_t cost = (int64_t)L.D * (L.D + 1) / 2 * L.kbp;
    for (int t = 0; t < ntiles; ++t) items.push_back({slot, t, cost});
  }
  int bounds[kXcds + 1];
  items = xcd_lists(items, [](const Item &it) { return (int64_t)it.slot; }, bounds);
  p.nitems = (int)items.size();
  p.off_items = take(items.size() * sizeof(int2));
  p.off_bounds = take(sizeof(bounds));
  p.off_counter = take(kXcds * 4);
  p.total = o;

  if (hipMalloc(&p.ws, p.total > 0 ? p.total : 256) != hipSuccess) {
    (void)hipGetLastError();
    p.ws = nullptr;
    return MPGEMM_ERR_WORKSPACE;
  }
  if (hipHostMalloc(&p.stage, p.desc_bytes > 0 ? p.desc_bytes : 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    p.stage = nullptr;
    return MPGEMM_ERR_WORKSPACE;
  }
  if (hipEventCreateWithFlags(&p.stage_done, hipEventDisableTiming) != hipSuccess) return MPGEMM_ERR_HIP;

  // static device data: prefix sums of the split work and the work list.  An
  // operand whose vectors fit a fused workgroup is split by the fused kernel
  // alone; the others by the max and pass kernels.
  std::vector<int> pre0(p.nops + 1, 0), prep(p.nops + 1, 0), pref(p.nops + 1, 0);
  int dpass = 0;
  for (int slot = 0; slot < (int)p.live.size(); ++slot) {
    const ProductLayout &L = p.prod[p.live[slot]];
    for (int side = 0; side < 2; ++side) {
      const int i = 2 * slot + side;
      const int64_t nvec = side == 0 ? L.m : L.n, nbp = side == 0 ? L.mbp : L.nbp;
      const bool fused = side == 0 ? L.fused_a : L.fused_b;
      pref[i + 1] = pref[i] + (fused ? fused_strips<T, C>(OperandShape{L.kbp, nbp, nvec}, p.fused_nt) : 0);
      pre0[i + 1] = pre0[i] + (fused ? 0 : tiles64(nvec, L.k));
      prep[i + 1] = prep[i] + (fused ? 0 : tiles64(nbp * kBlk, L.kbp * kKBlk));
      if (!fused) dpass = std::max(dpass, L.D);
    }
  }
  p.tiles0 = pre0[p.nops];
  p.tilesp = prep[p.nops];
  p.stripsf = pref[p.nops];
  std::vector<int2> it2(items.size());
  for (size_t i = 0; i < items.size(); ++i) it2[i] = make_int2(items[i].slot, items[i].tile);
  if (hipMemcpy(p.ws + p.off_prefix0, pre0.data(), pre0.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.ws + p.off_prefixp, prep.data(), prep.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.ws + p.off_prefixf, pref.data(), pref.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      (it2.size() && hipMemcpy(p.ws + p.off_items, it2.data(), it2.size() * sizeof(int2), hipMemcpyHostToDevice) !=
                         hipSuccess) ||
      hipMemcpy(p.ws + p.off_bounds, bounds, sizeof(bounds), hipMemcpyHostToDevice) != hipSuccess)
    return MPGEMM_ERR_HIP;

  // capture the launch sequence on a private stream
  BatchCache &bc = cache();
  hipStream_t &cs = bc.capture[p.device & 63];
  if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return MPGEMM_ERR_HIP;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPGEMM_ERR_HIP;
  hipError_t e = launch_split_plain_batched<T, C>(
      reinterpret_cast<const SplitOperand<T> *>(p.ws + p.off_ops), reinterpret_cast<const int *>(p.ws + p.off_prefix0),
      reinterpret_cast<const int *>(p.ws + p.off_prefixp), reinterpret_cast<const int *>(p.ws + p.off_prefixf),
      p.nops, p.tiles0, p.tilesp, p.stripsf, p.fused_nt, dpass, p.ws + p.off_mu, (int64_t)(p.mu_bytes / 4), cs);
  if (e == hipSuccess) e = launch_fill32(p.ws + p.off_counter, kXcds, 0u, cs);
  if (e == hipSuccess)
    e = launch_gemm_plain_batched<T, C>(reinterpret_cast<const PlainGemmDesc *>(p.ws + p.off_descs),
                                        reinterpret_cast<const int2 *>(p.ws + p.off_items),
                                        reinterpret_cast<const int *>(p.ws + p.off_bounds),
                                        reinterpret_cast<int *>(p.ws + p.off_counter),
                                        std::min(p.nitems, kPersistentGrid), p.layout, cs);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(cs, &graph);
  if (e != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return MPGEMM_ERR_HIP;
  }
  p.graph = graph;
  if (hipGraphInstantiate(&p.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    return MPGEMM_ERR_HIP;
  }
  (void)st;
  return 0;
}

// Descriptors carrying this call's pointers, written into the pinned stage.
template <typename T, int C>
void write_descriptors(BatchPlan &p, const T *const *A, const int *lda, const T *const *B, const int *ldb,
                       T *const *Cm, const int *ldc) {
  SplitOperand<T> *ops = static_cast<SplitOperand<T> *>(p.stage);
  PlainGemmDesc *descs = reinterpret_cast<PlainGemmDesc *>(static_cast<char *>(p.stage) +
                                                           (size_t)p.nops * sizeof(SplitOperand<T>));
  for (int slot = 0; slot < (int)p.live.size(); ++slot) {
    const int g = p.live[slot];
    const ProductLayout &L = p.prod[g];
    SplitOperand<T> a{}, b{};
    a.X = A[g];
    a.comp_stride = (int64_t)lda[g] * L.k;
    a.sv = 1;
    a.sp = lda[g];
    a.nvec = L.m;
    a.len = L.k;
    a.orient = 0;
    a.resid = reinterpret_cast<T *>(p.ws + L.resid_a);
    a.packed = p.ws + L.pack_a;
    a.nbp = L.mbp;
    a.kbp = L.kbp;
    a.mu = p.ws + L.mu_a;
    a.exps = reinterpret_cast<int *>(p.ws + L.exp_a);
    a.D = L.D;
    a.rho = L.rho;
    a.last_literal = p.last_slice;
    b.X = B[g];
    b.comp_stride = (int64_t)ldb[g] * L.n;
    b.sv = ldb[g];
    b.sp = 1;
    b.nvec = L.n;
    b.len = L.k;
    b.orient = 1;
    b.resid = reinterpret_cast<T *>(p.ws + L.resid_b);
    b.packed = p.ws + L.pack_b;
    b.nbp = L.nbp;
    b.kbp = L.kbp;
    b.mu = p.ws + L.mu_b;
    b.exps = reinterpret_cast<int *>(p.ws + L.exp_b);
    b.D = L.D;
    b.rho = L.rho;
    b.last_literal = p.last_slice;
    ops[2 * slot] = a;
    ops[2 * slot + 1] = b;
    PlainGemmDesc d{};
    d.Apk = p.ws + L.pack_a;
    d.Bpk = p.ws + L.pack_b;
    d.mbp = L.mbp;
    d.nbp = L.nbp;
    d.kbp = L.kbp;
    d.m = L.m;
    d.n = L.n;
    d.D = L.D;
    d.ldc = ldc[g];
    d.C = Cm[g];
    d.c_stride = (int64_t)ldc[g] * L.n;
    descs[slot] = d;
  }
}

// INT8-form batch: the digit split of every operand, one persistent INT8
// GEMM per tile configuration over (product, tile, k chunk, diagonal group)
// items in per-XCD lists, and one combine over every product's blocks.
template <int C>
int build_plan_int8(BatchPlan &p, int cfg_override) {
  const int count = (int)p.m.size();
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  p.prod.resize(count);
  p.live.clear();
  p.dmax = 0;
  for (int g = 0; g < count; ++g) {
    ProductLayout &L = p.prod[g];
    L.m = p.m[g];
    L.n = p.n[g];
    L.k = p.k[g];
    L.D = p.D[g];
    if (L.m <= 0 || L.n <= 0 || L.k <= 0) continue;
    p.live.push_back(g);
    L.rho = 0;
    L.cfg = batch_int8_cfg(L.m, L.n, cfg_override);
    L.mbp = nblocks8_padded(L.m, int8_tile_blocks(L.cfg));
    L.nbp = nblocks8_padded(L.n, int8_tile_blocks(L.cfg));
    L.kbp = kblocks8_padded(L.k);
    L.kbc = int8_kblocks_per_chunk(L.D);
    L.nchunks = (int)ceil_div(L.kbp, L.kbc);
    L.resid_a = L.resid_b = 0;
    L.pack_a = take((size_t)L.D * L.mbp * L.kbp * 1024);
    L.pack_b = take((size_t)L.D * L.nbp * L.kbp * 1024);
    L.exp_a = take((size_t)L.m * 4);
    L.exp_b = take((size_t)L.n * 4);
    L.sums = take((size_t)L.D * L.nchunks * L.mbp * L.nbp * 1024 * 4);
    p.dmax = std::max(p.dmax, L.D);
  }
  p.off_mu = o;
  size_t mo = 0;
  for (int g : p.live) {
    ProductLayout &L = p.prod[g];
    L.mu_a = p.off_mu + mo;
    mo += (size_t)L.m * 8;
    L.mu_b = p.off_mu + mo;
    mo += (size_t)L.n * 8;
  }
  p.mu_bytes = (mo + 3) / 4 * 4;
  o = p.off_mu + align256(mo);
  p.nops = 2 * (int)p.live.size();
  p.off_ops = take(0);
  p.off_descs = p.off_ops + (size_t)p.nops * sizeof(SplitOperand<double>);
  p.desc_bytes = (size_t)p.nops * sizeof(SplitOperand<double>) + p.live.size() * sizeof(Int8GemmDesc);
  o = p.off_ops + align256(p.desc_bytes);
  p.off_prefix0 = take((size_t)(p.nops + 1) * 4);
  p.off_prefixp = take((size_t)(p.nops + 1) * 4);
  p.off_prefixc = take((size_t)(p.live.size() + 1) * 4);

  // diagonal groups: items of about 1/4 of a persistent workgroup's fair share
  auto cum = [](int64_t g) { return g * (g + 1) / 2; };
  int64_t work = 0;
  for (int g : p.live) {
    const ProductLayout &L = p.prod[g];
    const int tb = int8_tile_blocks(L.cfg);
    work += (L.mbp / tb) * (L.nbp / tb) * (tb / 4) * (tb / 4) * cum(L.D) * L.kbp;  // in 128 x 128 tile units
  }
  const int64_t target = std::max<int64_t>(1, work / (4 * (int64_t)kPersistentGrid));
  struct Item {
    int slot, tile, chunk, group;
    int64_t cost;
  };
  std::vector<Item> items, items3;
  for (int slot = 0; slot < (int)p.live.size(); ++slot) {
    ProductLayout &L = p.prod[p.live[slot]];
    const int tb = int8_tile_blocks(L.cfg);
    const int64_t unit = (tb / 4) * (tb / 4);  // 128 x 128 tiles in one tile
    L.groups = (int)std::min<int64_t>(L.D, std::max<int64_t>(1, ceil_div(cum(L.D) * L.kbc * unit, target)));
    const int ntiles = (int)((L.mbp / tb) * (L.nbp / tb));
    std::vector<Item> &dst = L.cfg == 1 ? items : items3;
    for (int z = 0; z < L.groups; ++z) {
      // the same cut as the device: smallest g with cum(g) >= target pairs
      auto first_reaching = [&](int64_t t) {
        int64_t gg = 0;
        while (cum(gg) < t) ++gg;
        return gg;
      };
      const int64_t pairs = cum(L.D);
      const int64_t b0 = first_reaching(pairs * z / L.groups), b1 = first_reaching(pairs * (z + 1) / L.groups);
      if (b1 == b0) continue;  // empty group
      for (int c = 0; c < L.nchunks; ++c) {
        const int64_t kblocks = std::min<int64_t>(L.kbc, L.kbp - (int64_t)c * L.kbc);
        for (int t = 0; t < ntiles; ++t) dst.push_back({slot, t, c, z, (cum(b1) - cum(b0)) * kblocks});
      }
    }
  }
  // one list per XCD for each configuration; a run is one (product, k chunk,
  // diagonal group): its tiles
  auto run_key = [](const Item &it) { return ((int64_t)it.slot << 32) | ((int64_t)it.chunk << 12) | it.group; };
  int bounds[2 * (kXcds + 1)];
  items = xcd_lists(items, run_key, bounds);
  items3 = xcd_lists(items3, run_key, bounds + kXcds + 1);
  p.nitems = (int)items.size();
  p.nitems3 = (int)items3.size();
  items.insert(items.end(), items3.begin(), items3.end());
  p.off_items = take(items.size() * sizeof(int4));
  p.off_bounds = take(sizeof(bounds));
  p.off_counter = take(2 * kXcds * 4);
  p.total = o;

  if (hipMalloc(&p.ws, p.total > 0 ? p.total : 256) != hipSuccess) {
    (void)hipGetLastError();
    p.ws = nullptr;
    return MPGEMM_ERR_WORKSPACE;
  }
  if (hipHostMalloc(&p.stage, p.desc_bytes > 0 ? p.desc_bytes : 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    p.stage = nullptr;
    return MPGEMM_ERR_WORKSPACE;
  }
  if (hipEventCreateWithFlags(&p.stage_done, hipEventDisableTiming) != hipSuccess) return MPGEMM_ERR_HIP;
  // the digit split writes only blocks that hold elements: the padding blocks
  // of the packed planes are cleared here, once, and stay zero on every replay
  if (hipMemset(p.ws, 0, p.total > 0 ? p.total : 256) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess)
    return MPGEMM_ERR_HIP;

  std::vector<int> pre0(p.nops + 1, 0), preb(p.nops + 1, 0), prec(p.live.size() + 1, 0);
  for (int slot = 0; slot < (int)p.live.size(); ++slot) {
    const ProductLayout &L = p.prod[p.live[slot]];
    const int64_t kbl = ceil_div((int64_t)L.k, (int64_t)kKBlk8);
    pre0[2 * slot + 1] = pre0[2 * slot] + tiles64(L.m, L.k);
    pre0[2 * slot + 2] = pre0[2 * slot + 1] + tiles64(L.n, L.k);
    preb[2 * slot + 1] = preb[2 * slot] + (int)(ceil_div((int64_t)L.m, (int64_t)kBlk8) * kbl);
    preb[2 * slot + 2] = preb[2 * slot + 1] + (int)(ceil_div((int64_t)L.n, (int64_t)kBlk8) * kbl);
    prec[slot + 1] = prec[slot] + (int)(L.mbp * L.nbp);
  }
  p.tiles0 = pre0[p.nops];
  p.blocks8 = preb[p.nops];
  p.blocksc = prec[p.live.size()];
  std::vector<int4> it4(items.size());
  for (size_t i = 0; i < items.size(); ++i)
    it4[i] = make_int4(items[i].slot, items[i].tile, items[i].chunk, items[i].group);
  if (hipMemcpy(p.ws + p.off_prefix0, pre0.data(), pre0.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.ws + p.off_prefixp, preb.data(), preb.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.ws + p.off_prefixc, prec.data(), prec.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      (it4.size() && hipMemcpy(p.ws + p.off_items, it4.data(), it4.size() * sizeof(int4), hipMemcpyHostToDevice) !=
                         hipSuccess) ||
      hipMemcpy(p.ws + p.off_bounds, bounds, sizeof(bounds), hipMemcpyHostToDevice) != hipSuccess)
    return MPGEMM_ERR_HIP;

  BatchCache &bc = cache();
  hipStream_t &cs = bc.capture[p.device & 63];
  if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return MPGEMM_ERR_HIP;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPGEMM_ERR_HIP;
  hipError_t e = launch_split_int8_batched<C>(
      reinterpret_cast<const SplitOperand<double> *>(p.ws + p.off_ops),
      reinterpret_cast<const int *>(p.ws + p.off_prefix0), reinterpret_cast<const int *>(p.ws + p.off_prefixp),
      p.nops, p.tiles0, p.blocks8, p.dmax, p.ws + p.off_mu, (int64_t)(p.mu_bytes / 4), cs);
  if (e == hipSuccess) e = launch_fill32(p.ws + p.off_counter, 2 * kXcds, 0u, cs);
  if (e == hipSuccess)
    e = launch_int8_batched<C>(reinterpret_cast<const Int8GemmDesc *>(p.ws + p.off_descs),
                               reinterpret_cast<const int4 *>(p.ws + p.off_items), p.nitems, p.nitems3,
                               reinterpret_cast<const int *>(p.ws + p.off_bounds),
                               reinterpret_cast<int *>(p.ws + p.off_counter),
                               reinterpret_cast<const int *>(p.ws + p.off_prefixc), (int)p.live.size(), p.blocksc,
                               cs);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(cs, &graph);
  if (e != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return MPGEMM_ERR_HIP;
  }
  p.graph = graph;
  if (hipGraphInstantiate(&p.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    return MPGEMM_ERR_HIP;
  }
  return 0;
}

void write_descriptors_int8(BatchPlan &p, const double *const *A, const int *lda, const double *const *B,
                            const int *ldb, double *const *Cm, const int *ldc) {
  SplitOperand<double> *ops = static_cast<SplitOperand<double> *>(p.stage);
  Int8GemmDesc *descs = reinterpret_cast<Int8GemmDesc *>(static_cast<char *>(p.stage) +
                                                         (size_t)p.nops * sizeof(SplitOperand<double>));
  for (int slot = 0; slot < (int)p.live.size(); ++slot) {
    const int g = p.live[slot];
    const ProductLayout &L = p.prod[g];
    SplitOperand<double> a{}, b{};
    a.X = A[g];
    a.comp_stride = (int64_t)lda[g] * L.k;
    a.sv = 1;
    a.sp = lda[g];
    a.nvec = L.m;
    a.len = L.k;
    a.orient = 0;
    a.packed = p.ws + L.pack_a;
    a.nbp = L.mbp;
    a.kbp = L.kbp;
    a.mu = p.ws + L.mu_a;
    a.exps = reinterpret_cast<int *>(p.ws + L.exp_a);
    a.D = L.D;
    b.X = B[g];
    b.comp_stride = (int64_t)ldb[g] * L.n;
    b.sv = ldb[g];
    b.sp = 1;
    b.nvec = L.n;
    b.len = L.k;
    b.orient = 1;
    b.packed = p.ws + L.pack_b;
    b.nbp = L.nbp;
    b.kbp = L.kbp;
    b.mu = p.ws + L.mu_b;
    b.exps = reinterpret_cast<int *>(p.ws + L.exp_b);
    b.D = L.D;
    ops[2 * slot] = a;
    ops[2 * slot + 1] = b;
    Int8GemmDesc d{};
    d.Apk = reinterpret_cast<const int8_t *>(p.ws + L.pack_a);
    d.Bpk = reinterpret_cast<const int8_t *>(p.ws + L.pack_b);
    d.EA = reinterpret_cast<const int *>(p.ws + L.exp_a);
    d.EB = reinterpret_cast<const int *>(p.ws + L.exp_b);
    d.S = reinterpret_cast<int32_t *>(p.ws + L.sums);
    d.mbp = L.mbp;
    d.nbp = L.nbp;
    d.kbp = L.kbp;
    d.plane = L.mbp * L.nbp * 1024;
    d.kbc = L.kbc;
    d.nchunks = L.nchunks;
    d.groups = L.groups;
    d.D = L.D;
    d.m = L.m;
    d.n = L.n;
    d.ldc = ldc[g];
    d.C = Cm[g];
    d.c_stride = (int64_t)ldc[g] * L.n;
    descs[slot] = d;
  }
}

template <typename T, int C>
int run_batched(int fmt, int count, const int *m, const int *n, const int *k, const T *const *A, const int *lda,
                const T *const *B, const int *ldb, T *const *Cm, const int *ldc, hipStream_t st) {
  if (count < 0) return -1;
  if (count > 0 && (!m || !n || !k || !A || !lda || !B || !ldb || !Cm || !ldc)) {
    const void *args[] = {m, n, k, A, lda, B, ldb, Cm, ldc};
    for (int i = 0; i < 9; ++i)
      if (!args[i]) return -(i + 2);
  }
  for (int g = 0; g < count; ++g) {
    const int s = validate(m[g], n[g], k[g], A[g], lda[g], B[g], ldb[g], Cm[g], ldc[g]);
    if (s < 0) return s - 1;  // positions shifted by the leading count argument
    if (s > 0) return s;
  }
  int s;
  if ((s = check_device_cached())) return s;
  const int mode = thread_mode(fmt);
  if (mode != MPGEMM_MODE_FLOAT && (mode != MPGEMM_MODE_INT8 || sizeof(T) != 8)) return MPGEMM_ERR_UNSUPPORTED;
  const int layout = layout_for(fmt);
  if (count == 0) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MPGEMM_ERR_HIP;

  std::vector<int> Ds(count);
  for (int g = 0; g < count; ++g) Ds[g] = slices_for(fmt, mode, k[g]);
  set_last_slices(Ds.empty() ? 0 : *std::max_element(Ds.begin(), Ds.end()));

  // products with k == 0 only need C cleared
  for (int g = 0; g < count; ++g)
    if (k[g] == 0 && m[g] > 0 && n[g] > 0) {
      if (launch_zero_matrix(Cm[g], sizeof(T), C, m[g], n[g], ldc[g], (int64_t)ldc[g] * n[g], st) != hipSuccess)
        return MPGEMM_ERR_HIP;
    }

  BatchCache &bc = cache();
  BatchPlan *plan = nullptr;
  for (BatchPlan *p : bc.plans)
    if (p->device == dev && p->stream == st && p->fmt == fmt && p->mode == mode && p->layout == layout &&
        p->int8_tile == int8_tile_override() && p->split_kernel == split_kernel_override() &&
        p->last_slice == last_slice_option() &&
        (int)p->m.size() == count &&
        std::equal(p->m.begin(), p->m.end(), m) && std::equal(p->n.begin(), p->n.end(), n) &&
        std::equal(p->k.begin(), p->k.end(), k) && p->D == Ds) {
      plan = p;
      break;
    }
  if (!plan) {
    if ((int)bc.plans.size() >= kMaxPlans) {
      auto oldest = std::min_element(bc.plans.begin(), bc.plans.end(),
                                     [](const BatchPlan *a, const BatchPlan *b) { return a->last_use < b->last_use; });
      (void)hipDeviceSynchronize();  // its workspace may still be in use
      (*oldest)->release();
      delete *oldest;
      bc.plans.erase(oldest);
    }
    plan = new BatchPlan();
    plan->device = dev;
    plan->stream = st;
    plan->fmt = fmt;
    plan->mode = mode;
    plan->layout = layout;
    plan->int8_tile = int8_tile_override();
    plan->split_kernel = split_kernel_override();
    plan->last_slice = last_slice_option();
    plan->m.assign(m, m + count);
    plan->n.assign(n, n + count);
    plan->k.assign(k, k + count);
    plan->D = Ds;
    if (mode == MPGEMM_MODE_INT8) {
      if constexpr (sizeof(T) == 8) s = build_plan_int8<C>(*plan, int8_tile_override());
    } else {
      s = build_plan<T, C>(*plan, st);
    }
    if (s) {
      plan->release();
      delete plan;
      return s;
    }
    bc.plans.push_back(plan);
  }
  plan->last_use = ++bc.clock;
  if (plan->live.empty()) return 0;

  // the stage may still feed the previous launch's descriptor copy
  if (hipEventSynchronize(plan->stage_done) != hipSuccess) return MPGEMM_ERR_HIP;
  if constexpr (sizeof(T) == 8) {
    if (mode == MPGEMM_MODE_INT8)
      write_descriptors_int8(*plan, A, lda, B, ldb, Cm, ldc);
    else
      write_descriptors<T, C>(*plan, A, lda, B, ldb, Cm, ldc);
  } else {
    write_descriptors<T, C>(*plan, A, lda, B, ldb, Cm, ldc);
  }
  hipEvent_t ev[3];
  profile_mark3(ev);
  if (ev[0]) (void)hipEventRecord(ev[0], st);
  if (hipMemcpyAsync(plan->ws + plan->off_ops, plan->stage, plan->desc_bytes, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipEventRecord(plan->stage_done, st) != hipSuccess)
    return MPGEMM_ERR_HIP;
  if (ev[1]) (void)hipEventRecord(ev[1], st);
  const hipError_t e = hipGraphLaunch(plan->exec, st);
  if (ev[2]) (void)hipEventRecord(ev[2], st);
  profile_commit(ev);
  return hip_status(e);
}

}  // namespace
}  // namespace host
}  // namespace mp

using namespace mp::host;

extern "C" {

int mpgemm_dd_batched(int count, const int *m, const int *n, const int *k, const double *const *A, const int *lda,
                      const double *const *B, const int *ldb, double *const *C, const int *ldc, hipStream_t stream) {
  return run_batched<double, 2>(MPGEMM_DD, count, m, n, k, A, lda, B, ldb, C, ldc, stream);
}
int mpgemm_td_batched(int count, const int *m, const int *n, const int *k, const double *const *A, const int *lda,
                      const double *const *B, const int *ldb, double *const *C, const int *ldc, hipStream_t stream) {
  return run_batched<double, 3>(MPGEMM_TD, count, m, n, k, A, lda, B, ldb, C, ldc, stream);
}
int mpgemm_qd_batched(int count, const int *m, const int *n, const int *k, const double *const *A, const int *lda,
                      const double *const *B, const int *ldb, double *const *C, const int *ldc, hipStream_t stream) {
  return run_batched<double, 4>(MPGEMM_QD, count, m, n, k, A, lda, B, ldb, C, ldc, stream);
}
int mpgemm_ts_batched(int count, const int *m, const int *n, const int *k, const float *const *A, const int *lda,
                      const float *const *B, const int *ldb, float *const *C, const int *ldc, hipStream_t stream) {
  return run_batched<float, 3>(MPGEMM_TS, count, m, n, k, A, lda, B, ldb, C, ldc, stream);
}

int mpgemm_batched_cache_clear(void) {
  if (!g_batch) return 0;
  const hipError_t e = hipDeviceSynchronize();
  for (BatchPlan *p : g_batch->plans) {
    p->release();
    delete p;
  }
  g_batch->plans.clear();
  return e == hipSuccess ? 0 : MPGEMM_ERR_HIP;
}

}  // extern "C"
