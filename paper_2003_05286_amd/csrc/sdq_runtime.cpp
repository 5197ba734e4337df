// sdq_runtime.cpp -- host runtime behind the C ABI of include/sdq.h:
// argument validation, batch planning (work items in longest-first order,
// one persistent launch per tile-count class), the checkpoint arena for the
// stored stage factorizations, per-kernel event timing, HIP graph capture of
// repeated batches, and the autotune table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "sdq.h"
#include "sdq_internal.h"

namespace sdq {
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s);
}

using sdq::Inst;
using sdq::PairItem;
using sdq::Queue;
using sdq::SweepItem;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct KStat {
  int64_t launches = 0;
  double ms = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

struct Handle {
  DevBuf ckf;
  std::vector<sdq_instance> src;  // the instances the stages belong to
  std::vector<int64_t> off;       // per instance offset (doubles) into ckf
};

struct Tune {
  int variant = 0;     // sweep kernel variant (1 = slice exponential staged in LDS)
  int blocks_per_cu = 0;  // 0 = occupancy limit
};

// one planned batch: what gets uploaded and launched.  Sweeps run first,
// then the pair items of each mode (equal-time, time-displaced, gradient);
// every (mode, tile class) is one persistent launch.
struct Plan {
  std::vector<Inst> inst;
  std::vector<SweepItem> sweep;
  std::vector<PairItem> pair[sdq::kPairModes];
  std::vector<int32_t> llist;
  struct Range {
    int nt, off, count;
  };
  std::vector<Range> sweep_ranges, pair_ranges[sdq::kPairModes];
};

}  // namespace

struct sdq_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int num_cu = 256;
  DevBuf d_upload, d_ck, d_swz, d_fin;
  void* h_stage = nullptr;
  size_t h_cap = 0;
  hipEvent_t stage_ev = nullptr;
  bool stage_pending = false;
  std::map<uint64_t, Handle> handles;
  uint64_t next_handle = 1;
  Tune tune[sdq::kMaxNT + 1];
  std::map<long long, sdq::KernelInfo> info_cache;
  bool profiling = false;
  std::map<std::string, KStat> stats;
  std::vector<hipEvent_t> ev_pool;
  bool graphs = false;
  struct GraphEntry {
    std::vector<char> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<GraphEntry> graph_cache;
};

namespace {

sdq_status fail(sdq_ctx* c, sdq_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

sdq_status hip_fail(sdq_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, SDQ_EHIP, m);
}

#define HIP_TRY(call, what)                     \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

hipError_t grow(DevBuf& b, size_t bytes) {
  if (bytes <= b.cap) return hipSuccess;
  if (b.p) {
    hipError_t e = hipFree(b.p);  // implicit device synchronization
    if (e != hipSuccess) return e;
  }
  b.p = nullptr;
  b.cap = 0;
  size_t want = bytes + bytes / 8;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return e;
    }
    want = bytes;
  }
  b.cap = want;
  return hipSuccess;
}

int nt_of(int n) { return (n + 15) / 16; }
int nb_of(int m, int k) { return (m + k - 1) / k; }

// algorithmic cost of one sweep, for longest-first ordering
double sweep_cost(int n, int m, int k) {
  const double n3 = (double)n * n * n;
  return n3 * (2.0 * m + nb_of(m, k) * 11.0 / 3.0) + 1e4 * nb_of(m, k) * n;
}

sdq_status validate(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, bool need_inv) {
  if (!ctx) return SDQ_EINVAL;
  if (count < 0) return fail(ctx, SDQ_EINVAL, "count < 0");
  if (count > 0 && !inst) return fail(ctx, SDQ_EINVAL, "inst is NULL");
  for (int i = 0; i < count; ++i) {
    const sdq_instance& I = inst[i];
    char buf[160];
    if (I.n < 1) {
      snprintf(buf, sizeof buf, "instance %d: n = %d < 1", i, I.n);
      return fail(ctx, SDQ_EINVAL, buf);
    }
    if (I.n > 16 * sdq::kMaxNT) {
      snprintf(buf, sizeof buf, "instance %d: n = %d > %d is not supported", i, I.n, 16 * sdq::kMaxNT);
      return fail(ctx, SDQ_EUNSUPPORTED, buf);
    }
    if (I.m < 1 || I.k < 1 || I.k > I.m) {
      snprintf(buf, sizeof buf, "instance %d: need m >= 1 and 1 <= k <= m (m = %d, k = %d)", i, I.m, I.k);
      return fail(ctx, SDQ_EINVAL, buf);
    }
    if (!I.expk || !I.field) {
      snprintf(buf, sizeof buf, "instance %d: expk or field is NULL", i);
      return fail(ctx, SDQ_EINVAL, buf);
    }
    if (need_inv && !I.expk_inv) {
      snprintf(buf, sizeof buf, "instance %d: expk_inv is NULL", i);
      return fail(ctx, SDQ_EINVAL, buf);
    }
    if (!std::isfinite(I.alpha)) {
      snprintf(buf, sizeof buf, "instance %d: alpha is not finite", i);
      return fail(ctx, SDQ_EINVAL, buf);
    }
  }
  return SDQ_OK;
}

Inst base_inst(const sdq_instance& s) {
  Inst I;
  memset(&I, 0, sizeof I);
  I.expk = s.expk;
  I.expk_inv = s.expk_inv;
  I.field = s.field;
  I.alpha = s.alpha;
  I.n = s.n;
  I.m = s.m;
  I.k = s.k;
  I.nb = nb_of(s.m, s.k);
  return I;
}

// group work items by tile count, each class in longest-first order
template <class ItemT, class CostF>
void order_items(const std::vector<Inst>& inst, std::vector<ItemT>& items,
                 std::vector<Plan::Range>& ranges, CostF cost) {
  std::stable_sort(items.begin(), items.end(), [&](const ItemT& a, const ItemT& b) {
    const int na = nt_of(inst[a.inst].n), nb = nt_of(inst[b.inst].n);
    if (na != nb) return na > nb;
    return cost(a) > cost(b);
  });
  ranges.clear();
  for (size_t i = 0; i < items.size();) {
    const int nt = nt_of(inst[items[i].inst].n);
    size_t j = i;
    while (j < items.size() && nt_of(inst[items[j].inst].n) == nt) ++j;
    ranges.push_back({nt, (int)i, (int)(j - i)});
    i = j;
  }
}

const sdq::KernelInfo& info(sdq_ctx* ctx, int kind, int nt, int variant) {
  const long long key = (long long)kind * 1000 + nt * 10 + variant;
  auto it = ctx->info_cache.find(key);
  if (it == ctx->info_cache.end()) {
    sdq::KernelInfo ki{};
    if (sdq::kernel_info(kind, nt, variant, &ki) != hipSuccess || ki.blocks_per_cu < 1) {
      (void)hipGetLastError();
      ki.blocks_per_cu = 1;
    }
    it = ctx->info_cache.emplace(key, ki).first;
  }
  return it->second;
}

int grid_for(sdq_ctx* ctx, int kind, int nt, int variant, int count) {
  int per_cu = info(ctx, kind, nt, variant).blocks_per_cu;
  if (kind == sdq::KK_SWEEP && ctx->tune[nt].blocks_per_cu > 0)
    per_cu = std::min(per_cu, ctx->tune[nt].blocks_per_cu);
  const long long g = (long long)per_cu * ctx->num_cu;
  return (int)std::max(1LL, std::min<long long>(count, g));
}

hipEvent_t take_event(sdq_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// launch with optional event bracketing
template <class F>
sdq_status timed(sdq_ctx* ctx, const char* name, F launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ctx->profiling) {
    a = take_event(ctx);
    b = take_event(ctx);
    if (a) HIP_TRY(hipEventRecord(a, ctx->stream), "hipEventRecord");
  }
  hipError_t e = launch();
  if (e != hipSuccess) return hip_fail(ctx, e, name);
  if (ctx->profiling && a && b) {
    HIP_TRY(hipEventRecord(b, ctx->stream), "hipEventRecord");
    ctx->stats[name].pending.push_back({a, b});
  }
  return SDQ_OK;
}

// Swizzled, zero-padded copies of every distinct slice exponential of the
// plan (and of its transpose), in the MFMA operand order the kernels read.
struct SwzJob {
  const double* e;
  int n;
  int64_t off;
};

sdq_status prepare_swizzle(sdq_ctx* ctx, Plan& P, std::vector<SwzJob>& jobs) {
  std::map<std::pair<const double*, int>, int64_t> seen;
  int64_t tot = 0;
  for (const Inst& I : P.inst) {
    auto key = std::make_pair(I.expk, I.n);
    if (seen.count(key)) continue;
    const int64_t np = 16LL * nt_of(I.n);
    seen[key] = tot;
    jobs.push_back(SwzJob{I.expk, I.n, tot});
    tot += 2 * np * np;
  }
  HIP_TRY(grow(ctx->d_swz, (size_t)std::max<int64_t>(tot, 1) * sizeof(double)), "hipMalloc(swizzle)");
  double* base = (double*)ctx->d_swz.p;
  for (Inst& I : P.inst) {
    const int64_t off = seen[std::make_pair(I.expk, I.n)];
    const int64_t np = 16LL * nt_of(I.n);
    I.esw = base + off;
    I.eswt = base + off + np * np;
  }
  return SDQ_OK;
}

// Upload the plan (instances, items, l_list, zeroed queues) in one copy and
// run it: all sweeps, then all pair items.
sdq_status run_plan(sdq_ctx* ctx, Plan& P, int32_t* status, int count) {
  std::vector<SwzJob> swz;
  {
    sdq_status st = prepare_swizzle(ctx, P, swz);
    if (st) return st;
  }
  const size_t n_inst = P.inst.size();
  int nq = (int)P.sweep_ranges.size();
  size_t n_pair = 0;
  for (int md = 0; md < sdq::kPairModes; ++md) {
    nq += (int)P.pair_ranges[md].size();
    n_pair += P.pair[md].size();
  }
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_inst = 0;
  const size_t o_sw = align(o_inst + n_inst * sizeof(Inst));
  size_t o_pa[sdq::kPairModes];
  size_t o = align(o_sw + P.sweep.size() * sizeof(SweepItem));
  for (int md = 0; md < sdq::kPairModes; ++md) {
    o_pa[md] = o;
    o = align(o + P.pair[md].size() * sizeof(PairItem));
  }
  const size_t o_ll = o;
  const size_t o_q = align(o_ll + P.llist.size() * sizeof(int32_t));
  const size_t total = align(o_q + (size_t)std::max(nq, 1) * sizeof(Queue));
  (void)n_pair;

  if (ctx->stage_pending) {
    HIP_TRY(hipEventSynchronize(ctx->stage_ev), "hipEventSynchronize(staging)");
    ctx->stage_pending = false;
  }
  if (total > ctx->h_cap) {
    if (ctx->h_stage) HIP_TRY(hipHostFree(ctx->h_stage), "hipHostFree");
    ctx->h_stage = nullptr;
    ctx->h_cap = 0;
    HIP_TRY(hipHostMalloc(&ctx->h_stage, total * 2, hipHostMallocDefault), "hipHostMalloc");
    ctx->h_cap = total * 2;
  }
  char* h = (char*)ctx->h_stage;
  memset(h, 0, total);
  if (n_inst) memcpy(h + o_inst, P.inst.data(), n_inst * sizeof(Inst));
  if (!P.sweep.empty()) memcpy(h + o_sw, P.sweep.data(), P.sweep.size() * sizeof(SweepItem));
  for (int md = 0; md < sdq::kPairModes; ++md)
    if (!P.pair[md].empty())
      memcpy(h + o_pa[md], P.pair[md].data(), P.pair[md].size() * sizeof(PairItem));
  if (!P.llist.empty()) memcpy(h + o_ll, P.llist.data(), P.llist.size() * sizeof(int32_t));
  HIP_TRY(grow(ctx->d_upload, total), "hipMalloc(upload)");
  char* d = (char*)ctx->d_upload.p;
  HIP_TRY(hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, ctx->stream), "hipMemcpyAsync(plan)");
  HIP_TRY(hipEventRecord(ctx->stage_ev, ctx->stream), "hipEventRecord");
  ctx->stage_pending = true;
  if (status && count > 0) {
    HIP_TRY(sdq::launch_fill_i32(status, count, 0, ctx->stream), "fill(status)");
  }
  for (const SwzJob& j : swz) {
    const int64_t np = 16LL * nt_of(j.n);
    double* out = (double*)ctx->d_swz.p + j.off;
    HIP_TRY(sdq::launch_swizzle(j.e, j.n, 0, out, ctx->stream), "swizzle");
    HIP_TRY(sdq::launch_swizzle(j.e, j.n, 1, out + np * np, ctx->stream), "swizzle");
  }
  const Inst* d_inst = (const Inst*)(d + o_inst);
  const SweepItem* d_sw = (const SweepItem*)(d + o_sw);
  const int32_t* d_ll = (const int32_t*)(d + o_ll);
  Queue* d_q = (Queue*)(d + o_q);
  int qi = 0;
  for (const auto& r : P.sweep_ranges) {
    const int variant = ctx->tune[r.nt].variant;
    const int grid = grid_for(ctx, sdq::KK_SWEEP, r.nt, variant, r.count);
    Queue* q = d_q + qi++;
    sdq_status st = timed(ctx, "sweep", [&] {
      return sdq::launch_sweep(r.nt, variant, d_inst, d_sw + r.off, r.count, q, grid, ctx->stream);
    });
    if (st) return st;
  }
  static const char* names[sdq::kPairModes] = {"pair", "grad", "equal"};
  const int order[sdq::kPairModes] = {sdq::PAIR_EQUAL, sdq::PAIR_TDISP, sdq::PAIR_GRAD};
  for (int oi = 0; oi < sdq::kPairModes; ++oi) {
    const int md = order[oi];
    const PairItem* d_pa = (const PairItem*)(d + o_pa[md]);
    for (const auto& r : P.pair_ranges[md]) {
      const int grid = grid_for(ctx, sdq::KK_PAIR, r.nt, 0, r.count);
      Queue* q = d_q + qi++;
      sdq_status st = timed(ctx, names[md], [&] {
        return sdq::launch_pair(r.nt, 0, md, d_inst, d_pa + r.off, r.count, d_ll, q, grid, ctx->stream);
      });
      if (st) return st;
    }
  }
  return SDQ_OK;
}

// per-chain final-stage arena for calls that keep no stage stack
sdq_status alloc_fin(sdq_ctx* ctx, const sdq_instance* inst, int count, std::vector<int64_t>& off) {
  off.resize(count);
  int64_t tot = 0;
  for (int i = 0; i < count; ++i) {
    off[i] = tot;
    tot += (sdq::stage_doubles(inst[i].n) + 31) & ~(int64_t)31;
  }
  hipError_t e = grow(ctx->d_fin, (size_t)std::max<int64_t>(tot, 1) * sizeof(double));
  if (e != hipSuccess) return fail(ctx, SDQ_ENOMEM, "final-stage arena: " + std::string(hipGetErrorString(e)));
  return SDQ_OK;
}

void order_all_pairs(Plan& P) {
  for (int md = 0; md < sdq::kPairModes; ++md) {
    order_items(P.inst, P.pair[md], P.pair_ranges[md], [&](const PairItem& w) {
      const Inst& I = P.inst[w.inst];
      return (double)I.n * I.n * I.n * (11.0 + (w.ihi - w.ilo) * (double)I.k);
    });
  }
}

// checkpoint arena: two stage stacks per instance
sdq_status alloc_stages(sdq_ctx* ctx, DevBuf& buf, const sdq_instance* inst, int count, int stacks,
                        std::vector<int64_t>& off) {
  off.resize(count);
  int64_t tot = 0;
  for (int i = 0; i < count; ++i) {
    off[i] = tot;
    const int64_t one = (int64_t)nb_of(inst[i].m, inst[i].k) * sdq::stage_doubles(inst[i].n);
    tot += stacks * one;
    tot = (tot + 31) & ~(int64_t)31;
  }
  hipError_t e = grow(buf, (size_t)std::max<int64_t>(tot, 1) * sizeof(double));
  if (e != hipSuccess) return fail(ctx, SDQ_ENOMEM, "checkpoint arena: " + std::string(hipGetErrorString(e)));
  return SDQ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* sdq_version(void) { return "sdq 0.1 gfx950"; }

sdq_status sdq_create(sdq_ctx** out, int device, void* hip_stream) {
  if (!out) return SDQ_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return SDQ_EINVAL;
  }
  sdq_ctx* ctx = new (std::nothrow) sdq_ctx();
  if (!ctx) return SDQ_ENOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess || hipEventCreateWithFlags(&ctx->stage_ev, hipEventDisableTiming) != hipSuccess) {
    delete ctx;
    return SDQ_EHIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->num_cu = prop.multiProcessorCount;
  for (int nt = 0; nt <= sdq::kMaxNT; ++nt) {
    ctx->tune[nt] = Tune{};
    // default: slice exponential staged in LDS where that variant exists
    ctx->tune[nt].variant = (nt >= 3 && nt <= 5) ? 1 : 0;
  }
  // debug overrides (environment): SDQ_SWEEP_VARIANT, SDQ_BLOCKS_PER_CU
  if (const char* v = getenv("SDQ_SWEEP_VARIANT"))
    for (int nt = 0; nt <= sdq::kMaxNT; ++nt) ctx->tune[nt].variant = atoi(v);
  if (const char* v = getenv("SDQ_BLOCKS_PER_CU"))
    for (int nt = 0; nt <= sdq::kMaxNT; ++nt) ctx->tune[nt].blocks_per_cu = atoi(v);
  *out = ctx;
  return SDQ_OK;
}

void sdq_destroy(sdq_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->handles)
    if (kv.second.ckf.p) (void)hipFree(kv.second.ckf.p);
  for (auto& g : ctx->graph_cache)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (ctx->d_upload.p) (void)hipFree(ctx->d_upload.p);
  if (ctx->d_ck.p) (void)hipFree(ctx->d_ck.p);
  if (ctx->d_swz.p) (void)hipFree(ctx->d_swz.p);
  if (ctx->d_fin.p) (void)hipFree(ctx->d_fin.p);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  for (auto& kv : ctx->stats)
    for (auto& pr : kv.second.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->stage_ev) (void)hipEventDestroy(ctx->stage_ev);
  delete ctx;
}

const char* sdq_last_error(const sdq_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

sdq_status sdq_greens(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, sdq_scheme scheme,
                      double* const* g, double* logdet, double* sign, int32_t* status) {
  sdq_status st = validate(ctx, inst, count, false);
  if (st) return st;
  if (scheme != SDQ_INV_LOH) return fail(ctx, SDQ_EUNSUPPORTED, "only SDQ_INV_LOH is implemented");
  if (count == 0) return SDQ_OK;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int64_t> off;
  st = alloc_fin(ctx, inst, count, off);
  if (st) return st;
  Plan P;
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(inst[i]);
    I.g = g ? g[i] : nullptr;
    I.logdet = logdet ? logdet + i : nullptr;
    I.sign = sign ? sign + i : nullptr;
    I.status = status ? status + i : nullptr;
    I.fin = (double*)ctx->d_fin.p + off[i];
    P.inst.push_back(I);
    P.sweep.push_back(SweepItem{i, sdq::SW_LAST});
    P.pair[sdq::PAIR_EQUAL].push_back(PairItem{i, I.nb, 0, 0});
  }
  order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return sweep_cost(I.n, I.m, I.k);
  });
  order_all_pairs(P);
  ctx->err.clear();
  return run_plan(ctx, P, status, count);
}

sdq_status sdq_greens_tdisp(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, sdq_scheme scheme,
                            const int32_t* l_list, int32_t n_l, double* const* gt,
                            double* const* g, double* logdet, double* sign, int32_t* status) {
  sdq_status st = validate(ctx, inst, count, false);
  if (st) return st;
  if (scheme != SDQ_INV_LOH) return fail(ctx, SDQ_EUNSUPPORTED, "only SDQ_INV_LOH is implemented");
  if (n_l < 0 || (n_l > 0 && (!l_list || !gt))) return fail(ctx, SDQ_EINVAL, "bad l_list / gt");
  for (int a = 0; a < n_l; ++a) {
    if (l_list[a] < 0) return fail(ctx, SDQ_EINVAL, "l_list entry < 0");
    if (a > 0 && l_list[a] <= l_list[a - 1]) return fail(ctx, SDQ_EINVAL, "l_list must be strictly ascending");
  }
  for (int i = 0; i < count; ++i) {
    if (n_l > 0 && l_list[n_l - 1] > inst[i].m) return fail(ctx, SDQ_EINVAL, "l_list entry > m");
    if (n_l > 0 && !gt[i]) return fail(ctx, SDQ_EINVAL, "gt entry is NULL");
  }
  if (count == 0) return SDQ_OK;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int64_t> off;
  st = alloc_stages(ctx, ctx->d_ck, inst, count, 2, off);
  if (st) return st;
  double* ck = (double*)ctx->d_ck.p;
  Plan P;
  P.llist.assign(l_list, l_list + n_l);
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(inst[i]);
    I.g = g ? g[i] : nullptr;
    I.gt = n_l > 0 ? gt[i] : nullptr;
    I.logdet = logdet ? logdet + i : nullptr;
    I.sign = sign ? sign + i : nullptr;
    I.status = status ? status + i : nullptr;
    const int64_t sd = sdq::stage_doubles(I.n);
    const int64_t one = (int64_t)I.nb * sd;
    I.ckf = ck + off[i];
    I.cka = ck + off[i] + one;
    I.fin = I.ckf + (I.nb - 1) * sd;
    P.inst.push_back(I);
    P.sweep.push_back(SweepItem{i, sdq::SW_STORE});
    P.sweep.push_back(SweepItem{i, sdq::SW_STORE | sdq::SW_ADJ});
    if (I.g || I.logdet || I.sign) P.pair[sdq::PAIR_EQUAL].push_back(PairItem{i, I.nb, 0, 0});
    // group l by stage pair j: l == m -> nb, else l / k
    for (int a = 0; a < n_l;) {
      const int l = l_list[a];
      const int j = (l == I.m) ? I.nb : l / I.k;
      int b = a + 1;
      while (b < n_l) {
        const int l2 = l_list[b];
        const int j2 = (l2 == I.m) ? I.nb : l2 / I.k;
        if (j2 != j) break;
        ++b;
      }
      P.pair[sdq::PAIR_TDISP].push_back(PairItem{i, j, a, b});
      a = b;
    }
  }
  order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return sweep_cost(I.n, I.m, I.k);
  });
  order_all_pairs(P);
  ctx->err.clear();
  return run_plan(ctx, P, status, count);
}

sdq_status sdq_logdet(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, double* logdet,
                      double* sign, int32_t* status, uint64_t* ckpt_handle) {
  sdq_status st = validate(ctx, inst, count, false);
  if (st) return st;
  if (ckpt_handle) *ckpt_handle = 0;
  if (count == 0) return SDQ_OK;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  Handle H;
  std::vector<int64_t> foff;
  if (ckpt_handle) {
    st = alloc_stages(ctx, H.ckf, inst, count, 1, H.off);
    if (st) return st;
    H.src.assign(inst, inst + count);
  } else {
    st = alloc_fin(ctx, inst, count, foff);
    if (st) return st;
  }
  Plan P;
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(inst[i]);
    I.logdet = logdet ? logdet + i : nullptr;
    I.sign = sign ? sign + i : nullptr;
    I.status = status ? status + i : nullptr;
    int flags = sdq::SW_LAST;
    if (ckpt_handle) {
      I.ckf = (double*)H.ckf.p + H.off[i];
      I.fin = I.ckf + (int64_t)(I.nb - 1) * sdq::stage_doubles(I.n);
      flags = sdq::SW_STORE;
    } else {
      I.fin = (double*)ctx->d_fin.p + foff[i];
    }
    P.inst.push_back(I);
    P.sweep.push_back(SweepItem{i, flags});
    P.pair[sdq::PAIR_EQUAL].push_back(PairItem{i, I.nb, 0, 0});
  }
  order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return sweep_cost(I.n, I.m, I.k);
  });
  order_all_pairs(P);
  ctx->err.clear();
  st = run_plan(ctx, P, status, count);
  if (st) {
    if (H.ckf.p) (void)hipFree(H.ckf.p);
    return st;
  }
  if (ckpt_handle) {
    const uint64_t id = ctx->next_handle++;
    ctx->handles[id] = std::move(H);
    *ckpt_handle = id;
  }
  return SDQ_OK;
}

sdq_status sdq_logdet_grad(sdq_ctx* ctx, uint64_t ckpt_handle, const sdq_instance* inst,
                           int32_t count, double* const* grad, double* logdet, double* sign,
                           int32_t* status) {
  sdq_status st = validate(ctx, inst, count, true);
  if (st) return st;
  if (count > 0 && !grad) return fail(ctx, SDQ_EINVAL, "grad is NULL");
  for (int i = 0; i < count; ++i)
    if (!grad[i]) return fail(ctx, SDQ_EINVAL, "grad entry is NULL");
  Handle* H = nullptr;
  if (ckpt_handle) {
    auto it = ctx->handles.find(ckpt_handle);
    if (it == ctx->handles.end()) return fail(ctx, SDQ_EINVAL, "unknown checkpoint handle");
    H = &it->second;
    if ((int)H->src.size() != count) return fail(ctx, SDQ_EINVAL, "handle: instance count differs");
    for (int i = 0; i < count; ++i) {
      const sdq_instance& a = H->src[i];
      const sdq_instance& b = inst[i];
      if (a.n != b.n || a.m != b.m || a.k != b.k || a.field != b.field || a.expk != b.expk || a.alpha != b.alpha)
        return fail(ctx, SDQ_EINVAL, "handle: instances differ from those of sdq_logdet");
    }
  }
  if (count == 0) return SDQ_OK;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int64_t> off;
  st = alloc_stages(ctx, ctx->d_ck, inst, count, H ? 1 : 2, off);
  if (st) return st;
  double* ck = (double*)ctx->d_ck.p;
  Plan P;
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(inst[i]);
    I.grad = grad[i];
    I.logdet = logdet ? logdet + i : nullptr;
    I.sign = sign ? sign + i : nullptr;
    I.status = status ? status + i : nullptr;
    const int64_t sd = sdq::stage_doubles(I.n);
    const int64_t one = (int64_t)I.nb * sd;
    if (H) {
      I.ckf = (double*)H->ckf.p + H->off[i];
      I.cka = ck + off[i];
    } else {
      I.ckf = ck + off[i];
      I.cka = ck + off[i] + one;
      P.sweep.push_back(SweepItem{i, sdq::SW_STORE});
    }
    I.fin = I.ckf + (I.nb - 1) * sd;
    P.sweep.push_back(SweepItem{i, sdq::SW_STORE | sdq::SW_ADJ});
    P.inst.push_back(I);
    if (I.logdet || I.sign) P.pair[sdq::PAIR_EQUAL].push_back(PairItem{i, I.nb, 0, 0});
    for (int j = 0; j < I.nb; ++j) P.pair[sdq::PAIR_GRAD].push_back(PairItem{i, j, 0, 0});
  }
  order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return sweep_cost(I.n, I.m, I.k);
  });
  order_all_pairs(P);
  ctx->err.clear();
  return run_plan(ctx, P, status, count);
}

sdq_status sdq_release(sdq_ctx* ctx, uint64_t ckpt_handle) {
  if (!ctx) return SDQ_EINVAL;
  auto it = ctx->handles.find(ckpt_handle);
  if (it == ctx->handles.end()) return fail(ctx, SDQ_EINVAL, "unknown checkpoint handle");
  (void)hipSetDevice(ctx->device);
  if (it->second.ckf.p) HIP_TRY(hipFree(it->second.ckf.p), "hipFree(handle)");
  ctx->handles.erase(it);
  return SDQ_OK;
}

sdq_status sdq_udt(sdq_ctx* ctx, int32_t n, int32_t count, const double* w, double* u, double* d,
                   double* t) {
  if (!ctx) return SDQ_EINVAL;
  if (n < 1 || count < 0) return fail(ctx, SDQ_EINVAL, "bad n or count");
  if (n > 16 * sdq::kMaxNT) return fail(ctx, SDQ_EUNSUPPORTED, "n > 128 is not supported");
  if (count == 0) return SDQ_OK;
  if (!w || !u || !d || !t) return fail(ctx, SDQ_EINVAL, "null pointer");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  ctx->err.clear();
  return timed(ctx, "udt", [&] { return sdq::launch_udt(nt_of(n), n, count, w, u, d, t, ctx->stream); });
}

sdq_status sdq_chain_udt(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, double* u,
                         double* d, double* t) {
  sdq_status st = validate(ctx, inst, count, false);
  if (st) return st;
  if (count == 0) return SDQ_OK;
  if (!u || !d || !t) return fail(ctx, SDQ_EINVAL, "null output");
  for (int i = 1; i < count; ++i)
    if (inst[i].n != inst[0].n) return fail(ctx, SDQ_EINVAL, "all chains must share n");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  const int n = inst[0].n;
  Plan P;
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(inst[i]);
    I.u_out = u + (size_t)i * n * n;
    I.t_out = t + (size_t)i * n * n;
    I.d_out = d + (size_t)i * n;
    P.inst.push_back(I);
    P.sweep.push_back(SweepItem{i, sdq::SW_FINAL});
  }
  order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return sweep_cost(I.n, I.m, I.k);
  });
  ctx->err.clear();
  return run_plan(ctx, P, nullptr, 0);
}

sdq_status sdq_tune(sdq_ctx* ctx, const int32_t* n_list, int32_t count, const char* cache_path) {
  (void)n_list;
  (void)count;
  (void)cache_path;
  if (!ctx) return SDQ_EINVAL;
  return fail(ctx, SDQ_EUNSUPPORTED, "autotuning is not available yet");
}

sdq_status sdq_set_graphs(sdq_ctx* ctx, int enable) {
  if (!ctx) return SDQ_EINVAL;
  if (enable) return fail(ctx, SDQ_EUNSUPPORTED, "graph capture is not available yet");
  ctx->graphs = false;
  return SDQ_OK;
}

sdq_status sdq_set_profiling(sdq_ctx* ctx, int enable) {
  if (!ctx) return SDQ_EINVAL;
  HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  for (auto& kv : ctx->stats) {
    for (auto& pr : kv.second.pending) {
      ctx->ev_pool.push_back(pr.first);
      ctx->ev_pool.push_back(pr.second);
    }
  }
  ctx->stats.clear();
  ctx->profiling = enable != 0;
  return SDQ_OK;
}

sdq_status sdq_kernel_stats(sdq_ctx* ctx, const char* name, int64_t* launches, double* ms) {
  if (!ctx || !name) return SDQ_EINVAL;
  auto it = ctx->stats.find(name);
  if (it == ctx->stats.end()) {
    if (launches) *launches = 0;
    if (ms) *ms = 0.0;
    return SDQ_OK;
  }
  KStat& k = it->second;
  for (auto& pr : k.pending) {
    HIP_TRY(hipEventSynchronize(pr.second), "hipEventSynchronize");
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second), "hipEventElapsedTime");
    k.ms += t;
    k.launches += 1;
    ctx->ev_pool.push_back(pr.first);
    ctx->ev_pool.push_back(pr.second);
  }
  k.pending.clear();
  if (launches) *launches = k.launches;
  if (ms) *ms = k.ms;
  return SDQ_OK;
}

sdq_status sdq_sync(sdq_ctx* ctx) {
  if (!ctx) return SDQ_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  HIP_TRY(hipGetLastError(), "asynchronous error");
  return SDQ_OK;
}

}  // extern "C"
