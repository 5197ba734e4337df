// sdq_runtime.cpp -- host runtime behind the C ABI of include/sdq.h:
// argument validation, batch planning (work items in longest-first order,
// one persistent launch per tile-count class), the checkpoint arena for the
// stored stage factorizations, per-kernel event timing, HIP graph capture of
// repeated batches, and the autotune table.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "sdq.h"

// A roctx range around every compute entry point (host timeline of the
// call: argument checks, planning and enqueue), visible to tracing tools
// (rocprofv3 --marker-trace); without a tool attached the calls do nothing.
namespace {
struct ApiRange {
  explicit ApiRange(const char* name) { roctxRangePushA(name); }
  ~ApiRange() { roctxRangePop(); }
  ApiRange(const ApiRange&) = delete;
  ApiRange& operator=(const ApiRange&) = delete;
};
}  // namespace
#define SDQ_API_RANGE(name) ApiRange sdq_api_range_(name)
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
  bool swz_inv = false;  // also lay out expk_inv (chains of B^{-1} slices)
  // the swizzled copies are in place already: an earlier plan of the same
  // call, over the same instances, made them (the layout is a function of
  // the instances, so the pointers come out the same)
  bool swz_ready = false;
  bool dense = false;  // every instance has dense slices (sweep variant 3)
  // block products (k_prod) of the tile classes in bprod_mask (bit nt), run
  // before those classes' sweeps, which are then variant 6
  std::vector<SweepItem> prod;
  std::vector<Range> prod_ranges;
  unsigned bprod_mask = 0;
};

}  // namespace

struct sdq_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int num_cu = 256;
  DevBuf d_upload, d_ck, d_swz, d_fin;
  DevBuf d_tscr;  // per-workgroup T scratch of the variant-4/5 sweeps
  DevBuf d_gang;  // per-gang scratch of the n > 128 kernels (bars first)
  DevBuf d_ptrs;  // matrix pointer table of sdq_similarity
  DevBuf d_metro;  // sdq_metropolis: field table, proposed log|det|, signs and status
  DevBuf d_gloc;   // sdq_local_sweep: G at the block start, n x n per instance
  DevBuf d_lgrad;  // sdq_langevin: gradients of every instance, then statuses
  DevBuf d_ltab;   // sdq_langevin: chain table
  DevBuf d_hmc;    // sdq_hmc: gradients, start fields, momenta, energies, statuses
  int stab = 0;    // stabilizer of every sweep: 0 pivoted QR, 1 Jacobi SVD
  DevBuf d_htab;   // sdq_hmc: chain table
  DevBuf d_ctab;   // sdq_greens_complex: chain table
  DevBuf d_prod;   // block products of the slices (k_prod)
  // multiply the slice blocks out before the sweep (k_prod, tile classes
  // kProdMinNT .. kSweepMaxNT of sdq_greens): 0 never, 1 for every such
  // class, 2 for the class of the batch's longest chain when all its chains
  // are resident at once
  int bprod = 2;
  std::map<int, int> gang_cap;  // tile count -> gangs resident at once
  // pinned staging of plan images, a ring: the host waits for the plan
  // kStageSlots back, not the previous one, so it builds and enqueues the
  // next plans while the device runs (the device buffer they are copied to is
  // reused in stream order)
  static constexpr int kStageSlots = 4;
  struct StageSlot {
    void* h = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
  };
  StageSlot stage[kStageSlots];
  int stage_next = 0;
  std::map<uint64_t, Handle> handles;
  uint64_t next_handle = 1;
  Tune tune[sdq::kMaxNT + 1];
  std::map<long long, sdq::KernelInfo> info_cache;
  bool profiling = false;
  std::map<std::string, KStat> stats;
  std::vector<hipEvent_t> ev_pool;
  bool graphs = false;
  hipStream_t cap_stream = nullptr;  // non-null stream used only for graph capture
  // side streams of a batch whose tile classes run concurrently (created on
  // first use, default priority), with the fork event and their join events
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kSide] = {};
  struct GraphEntry {
    std::vector<char> key;
    hipGraphExec_t exec = nullptr;
    void* h = nullptr;  // pinned copy of the upload image the graph copies from
    void* d = nullptr;  // device upload buffer of the graph
  };
  std::vector<GraphEntry> graph_cache;
  // sdq_greens_noalloc: this device's fixed scratch (looked up at
  // sdq_create), the host copy of the last plan image and an event after its
  // upload (the copy is kept until that upload has completed)
  void* na_scratch = nullptr;
  std::string na_err;
  std::vector<char> na_image;
  hipEvent_t na_ev = nullptr;
  bool na_pending = false;
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
    if (I.n > sdq::kGangMaxN) {
      snprintf(buf, sizeof buf, "instance %d: n = %d > %d is not supported", i, I.n, sdq::kGangMaxN);
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
    if (ctx->stab == SDQ_STAB_SVD && I.n > 80) {
      snprintf(buf, sizeof buf, "instance %d: the Jacobi SVD stabilizer supports n <= 80 (n = %d)", i, I.n);
      return fail(ctx, SDQ_EUNSUPPORTED, buf);
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

bool is_gang(int nt) { return nt > sdq::kMaxNT; }
// the stabilized sweep runs as one workgroup up to kSweepMaxNT tiles
bool sweep_is_gang(int nt) { return nt > sdq::kSweepMaxNT; }
bool launch_is_gang(int kind, int nt) {
  return kind == sdq::KK_SWEEP || kind == sdq::KK_PROD ? sweep_is_gang(nt) : is_gang(nt);
}

// gangs of tile count nt that fit the device at once (cached)
int gang_slots(sdq_ctx* ctx, int nt) {
  auto it = ctx->gang_cap.find(nt);
  if (it != ctx->gang_cap.end()) return it->second;
  int g = 0;
  if (sdq::gang_capacity(nt, ctx->num_cu, &g) != hipSuccess) {
    (void)hipGetLastError();
    g = 0;
  }
  ctx->gang_cap[nt] = g;
  return g;
}

int grid_for(sdq_ctx* ctx, int kind, int nt, int variant, int count) {
  if (launch_is_gang(kind, nt)) {
    // a multiple of 8 gangs where the device holds them (XCD-local gangs)
    const int cap = gang_slots(ctx, nt);
    int ng = std::max(1, std::min(count, cap));
    if (ng % 8 && (ng + 7) / 8 * 8 <= cap) ng = (ng + 7) / 8 * 8;
    return ng;
  }
  int per_cu = info(ctx, kind, nt, variant).blocks_per_cu;
  if (kind == sdq::KK_SWEEP && nt <= sdq::kMaxNT && ctx->tune[nt].blocks_per_cu > 0)
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

// launch on stream s with optional event bracketing (the events are
// recorded on s, so they time this launch even when other streams run)
template <class F>
sdq_status timed_on(sdq_ctx* ctx, const std::string& name, hipStream_t s, F launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ctx->profiling) {
    a = take_event(ctx);
    b = take_event(ctx);
    if (a) HIP_TRY(hipEventRecord(a, s), "hipEventRecord");
  }
  hipError_t e = launch();
  if (e != hipSuccess) return hip_fail(ctx, e, name.c_str());
  if (ctx->profiling && a && b) {
    HIP_TRY(hipEventRecord(b, s), "hipEventRecord");
    ctx->stats[name].pending.push_back({a, b});
  }
  return SDQ_OK;
}
template <class F>
sdq_status timed(sdq_ctx* ctx, const char* name, F launch) {
  return timed_on(ctx, std::string(name), ctx->stream, launch);
}

// Swizzled, zero-padded copies of every distinct slice exponential of the
// plan (and of its transpose), in the MFMA operand order the kernels read.
struct SwzJob {
  const double* e;
  int n;
  int64_t off;
};

// `fixed`: lay the copies out there (the caller has sized it by
// swizzle_doubles) instead of in the context's growing buffer.
sdq_status prepare_swizzle(sdq_ctx* ctx, Plan& P, std::vector<SwzJob>& jobs, double*& base_out,
                           double* fixed = nullptr) {
  std::map<std::pair<const double*, int>, int64_t> seen;
  int64_t tot = 0;
  auto add = [&](const double* e, int n) {
    auto key = std::make_pair(e, n);
    if (seen.count(key)) return;
    const int64_t np = 16LL * nt_of(n);
    seen[key] = tot;
    jobs.push_back(SwzJob{e, n, tot});
    tot += 2 * np * np;
  };
  for (const Inst& I : P.inst) {
    if (!I.expk) continue;  // dense slices
    add(I.expk, I.n);
    if (P.swz_inv && I.expk_inv) add(I.expk_inv, I.n);
  }
  if (!fixed)
    HIP_TRY(grow(ctx->d_swz, (size_t)std::max<int64_t>(tot, 1) * sizeof(double)), "hipMalloc(swizzle)");
  double* base = fixed ? fixed : (double*)ctx->d_swz.p;
  base_out = base;
  for (Inst& I : P.inst) {
    if (!I.expk) continue;
    const int64_t off = seen[std::make_pair(I.expk, I.n)];
    const int64_t np = 16LL * nt_of(I.n);
    I.esw = base + off;
    I.eswt = base + off + np * np;
    if (P.swz_inv && I.expk_inv) I.eswi = base + seen[std::make_pair(I.expk_inv, I.n)];
  }
  return SDQ_OK;
}

// A planned batch turned into one upload image (instances, items, l_list,
// zeroed queue counters) and a list of launches whose pointers are offsets
// into that image once it is on the device.
struct LaunchRec {
  int kind;  // KK_SWEEP or KK_PAIR
  int nt, variant, mode, grid, count;
  size_t items_off;  // byte offset of the first item
  size_t queue_off;  // byte offset of this launch's queue counter
  size_t tscr_off;   // doubles into the T scratch (variant-4/5 sweeps)
};

struct Built {
  bool gang = false;  // has launches of the n > 128 kernels
  std::vector<char> image;
  std::vector<LaunchRec> launches;
  std::vector<SwzJob> swz;
  size_t o_inst = 0, o_ll = 0;
  size_t tscr_doubles = 0;  // T scratch of all variant-4/5 sweep launches
  double* swz_base = nullptr;   // where the swizzled operands go
  double* tscr_base = nullptr;  // T scratch (set by the caller of build_plan)
  bool fork = true;             // size classes may run on side streams
  int32_t* status = nullptr;
  int count = 0;
};

sdq_status build_plan(sdq_ctx* ctx, Plan& P, int32_t* status, int count, Built& B,
                      double* swz_fixed = nullptr) {
  {
    sdq_status st = prepare_swizzle(ctx, P, B.swz, B.swz_base, swz_fixed);
    if (st) return st;
    if (P.swz_ready) B.swz.clear();
  }
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  int nq = (int)P.sweep_ranges.size() + (int)P.prod_ranges.size();
  for (int md = 0; md < sdq::kPairModes; ++md) nq += (int)P.pair_ranges[md].size();
  const size_t o_inst = 0;
  const size_t o_sw = align(o_inst + P.inst.size() * sizeof(Inst));
  const size_t o_pr = align(o_sw + P.sweep.size() * sizeof(SweepItem));
  size_t o_pa[sdq::kPairModes];
  size_t o = align(o_pr + P.prod.size() * sizeof(SweepItem));
  for (int md = 0; md < sdq::kPairModes; ++md) {
    o_pa[md] = o;
    o = align(o + P.pair[md].size() * sizeof(PairItem));
  }
  const size_t o_ll = o;
  const size_t o_q = align(o_ll + P.llist.size() * sizeof(int32_t));
  const size_t total = align(o_q + (size_t)std::max(nq, 1) * sizeof(Queue));
  B.image.assign(total, 0);
  char* h = B.image.data();
  if (!P.inst.empty()) memcpy(h + o_inst, P.inst.data(), P.inst.size() * sizeof(Inst));
  if (!P.sweep.empty()) memcpy(h + o_sw, P.sweep.data(), P.sweep.size() * sizeof(SweepItem));
  if (!P.prod.empty()) memcpy(h + o_pr, P.prod.data(), P.prod.size() * sizeof(SweepItem));
  for (int md = 0; md < sdq::kPairModes; ++md)
    if (!P.pair[md].empty())
      memcpy(h + o_pa[md], P.pair[md].data(), P.pair[md].size() * sizeof(PairItem));
  if (!P.llist.empty()) memcpy(h + o_ll, P.llist.data(), P.llist.size() * sizeof(int32_t));
  B.o_inst = o_inst;
  B.o_ll = o_ll;
  for (const auto& r : P.sweep_ranges) B.gang |= sweep_is_gang(r.nt);
  for (int md = 0; md < sdq::kPairModes; ++md)
    for (const auto& r : P.pair_ranges[md]) B.gang |= is_gang(r.nt);
  B.status = status;
  B.count = count;
  int qi = 0;
  // the block products first: each runs before its class's sweep, in order
  // on the class's stream
  for (const auto& r : P.prod_ranges) {
    const int grid = grid_for(ctx, sdq::KK_PROD, r.nt, 0, r.count);
    B.launches.push_back(LaunchRec{sdq::KK_PROD, r.nt, 0, 0, grid, r.count, o_pr + r.off * sizeof(SweepItem),
                                   o_q + (qi++) * sizeof(Queue), 0});
  }
  for (const auto& r : P.sweep_ranges) {
    // (above kMaxNT tiles and up to kSweepMaxNT: the one-workgroup sweep with
    // T and the factor store in workgroup scratch, variant 4; over block
    // products, variant 6)
    const int variant = sweep_is_gang(r.nt) ? 0
                        : ((P.bprod_mask >> r.nt) & 1u) ? 6
                        : r.nt > sdq::kMaxNT ? 4
                        : P.dense ? 3
                        : (ctx->stab == SDQ_STAB_SVD ? 2 : ctx->tune[r.nt].variant);
    const int grid = grid_for(ctx, sdq::KK_SWEEP, r.nt, variant, r.count);
    // classes may run concurrently: each launch gets its own T scratch
    const size_t toff = B.tscr_doubles;
    if (!sweep_is_gang(r.nt)) B.tscr_doubles += (size_t)grid * (size_t)sdq::sweep_tscr_doubles(r.nt, variant);
    B.launches.push_back(LaunchRec{sdq::KK_SWEEP, r.nt, variant, 0, grid, r.count,
                                   o_sw + r.off * sizeof(SweepItem), o_q + (qi++) * sizeof(Queue), toff});
  }
  const int order[sdq::kPairModes] = {sdq::PAIR_EQUAL, sdq::PAIR_TDISP, sdq::PAIR_TDISP_PLAIN,
                                      sdq::PAIR_TDISP_DENSE, sdq::PAIR_GRAD, sdq::PAIR_BSTART,
                                      sdq::PAIR_LOCAL};
  for (int oi = 0; oi < sdq::kPairModes; ++oi) {
    const int md = order[oi];
    for (const auto& r : P.pair_ranges[md]) {
      // variant 3: the dense-slice G(tau,0) kernel (occupancy of its own)
      const int grid = grid_for(ctx, sdq::KK_PAIR, r.nt, md == sdq::PAIR_TDISP_DENSE ? 3 : 0, r.count);
      B.launches.push_back(LaunchRec{sdq::KK_PAIR, r.nt, 0, md, grid, r.count,
                                     o_pa[md] + r.off * sizeof(PairItem), o_q + (qi++) * sizeof(Queue), 0});
    }
  }
  return SDQ_OK;
}

// bytes of gang scratch a launch needs: barrier words first (256-byte
// aligned), then one scratch area per gang
size_t gang_bars_bytes(int ngangs) {
  return ((size_t)ngangs * sdq::kGangBarWords * sizeof(unsigned) + 255) & ~(size_t)255;
}
size_t gang_bytes(int nt, int ngangs) {
  const sdq::GangGeom g = sdq::gang_geom(nt);
  return gang_bars_bytes(ngangs) + (size_t)ngangs * (size_t)sdq::gang_doubles(g) * sizeof(double);
}
size_t gang_need(const Built& B) {
  size_t need = 0;
  for (const LaunchRec& L : B.launches)
    if (launch_is_gang(L.kind, L.nt)) need = std::max(need, gang_bytes(L.nt, L.grid));
  return need;
}

hipError_t launch_gang_rec(sdq_ctx* ctx, const LaunchRec& L, const Inst* d_inst, const char* d,
                           const int32_t* d_ll, hipStream_t s) {
  sdq::GangArgs a;
  a.bars = (unsigned*)ctx->d_gang.p;
  a.scratch = (double*)((char*)ctx->d_gang.p + gang_bars_bytes(L.grid));
  a.ngangs = L.grid;
  a.nt = L.nt;
  hipError_t e = sdq::launch_fill_i32((int32_t*)a.bars, L.grid * sdq::kGangBarWords, 0, s);
  if (e != hipSuccess) return e;
  if (L.kind == sdq::KK_SWEEP)
    return sdq::launch_gang_sweep(d_inst, (const SweepItem*)(d + L.items_off), L.count, a, s);
  return sdq::launch_gang_pair(L.mode, d_inst, (const PairItem*)(d + L.items_off), L.count, d_ll, a, s);
}

// Enqueue a built batch on stream s: upload h_src -> d, reset status, build
// the swizzled operands, launch.  `timing` brackets launches with events.
sdq_status enqueue_built(sdq_ctx* ctx, const Built& B, hipStream_t s, char* d, const char* h_src,
                         bool timing) {
  // (h_src null: the caller has uploaded the image already)
  if (h_src) HIP_TRY(hipMemcpyAsync(d, h_src, B.image.size(), hipMemcpyHostToDevice, s), "hipMemcpyAsync(plan)");
  if (B.status && B.count > 0) HIP_TRY(sdq::launch_fill_i32(B.status, B.count, 0, s), "fill(status)");
  for (const SwzJob& j : B.swz) {
    const int64_t np = 16LL * nt_of(j.n);
    double* out = B.swz_base + j.off;
    HIP_TRY(sdq::launch_swizzle(j.e, j.n, 0, out, s), "swizzle");
    HIP_TRY(sdq::launch_swizzle(j.e, j.n, 1, out + np * np, s), "swizzle");
  }
  const Inst* d_inst = (const Inst*)(d + B.o_inst);
  const int32_t* d_ll = (const int32_t*)(d + B.o_ll);
  static const char* names[sdq::kPairModes] = {"pair", "grad", "equal", "pair", "local", "bstart", "pair"};
  // Stream of each launch.  The items of different tile classes belong to
  // different chains, so the classes are independent: each class of the
  // one-workgroup kernels runs in order on a side stream of its own, forked
  // from s after the upload and the block products and joined back into s,
  // and the classes above kMaxNT tiles (gang kernels, which share the gang
  // scratch, and the one-workgroup sweeps whose stages the gang pair
  // kernels read) run in order on s.  A batch of one class stays on s.
  std::vector<int> cls;  // distinct one-workgroup tile classes, first-seen order
  bool any_gang = false;
  for (const LaunchRec& L : B.launches) {
    if (L.nt > sdq::kMaxNT) any_gang = true;  // runs on s
    else if (std::find(cls.begin(), cls.end(), L.nt) == cls.end()) cls.push_back(L.nt);
  }
  const bool fork = B.fork && (int)cls.size() + (any_gang ? 1 : 0) > 1;
  int nside = 0;
  auto stream_of = [&](const LaunchRec& L) -> hipStream_t {
    if (!fork || L.nt > sdq::kMaxNT) return s;
    const int c = (int)(std::find(cls.begin(), cls.end(), L.nt) - cls.begin());
    return ctx->side[c % nside];
  };
  auto launch_on = [&](const LaunchRec& L, hipStream_t ls) -> sdq_status {
    Queue* q = (Queue*)(d + L.queue_off);
    auto go = [&]() -> hipError_t {
      if (launch_is_gang(L.kind, L.nt)) return launch_gang_rec(ctx, L, d_inst, d, d_ll, ls);
      if (L.kind == sdq::KK_PROD)
        return sdq::launch_prod(L.nt, d_inst, (const SweepItem*)(d + L.items_off), L.count, q, L.grid, ls);
      if (L.kind == sdq::KK_SWEEP)
        return sdq::launch_sweep(L.nt, L.variant, d_inst, (const SweepItem*)(d + L.items_off), L.count,
                                 q, L.grid, B.tscr_base ? B.tscr_base + L.tscr_off : nullptr, ls);
      return sdq::launch_pair(L.nt, 0, L.mode, d_inst, (const PairItem*)(d + L.items_off), L.count,
                              d_ll, q, L.grid, ls);
    };
    // per-class name "<kernel>/nt<tiles>": sdq_kernel_stats("<kernel>") sums the classes
    std::string nm = std::string(L.kind == sdq::KK_SWEEP  ? "sweep"
                                 : L.kind == sdq::KK_PROD ? "prod"
                                                          : names[L.mode]) +
                     "/nt" +
                     std::to_string(L.nt);
    if (timing) return timed_on(ctx, nm, ls, go);
    hipError_t e = go();
    return e != hipSuccess ? hip_fail(ctx, e, nm.c_str()) : SDQ_OK;
  };
  // Block products first, on s and before the fork: they spread over the
  // whole device, and the classes on side streams start after them instead
  // of sharing the CUs with them (their class holds the batch's longest
  // chains, so its sweep, after them, is the step's critical path).
  for (const LaunchRec& L : B.launches)
    if (L.kind == sdq::KK_PROD) {
      sdq_status st = launch_on(L, s);
      if (st) return st;
    }
  if (fork) {
    nside = std::min((int)cls.size(), (int)sdq_ctx::kSide);
    for (int i = 0; i < nside; ++i) {
      if (!ctx->side[i])
        HIP_TRY(hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking), "hipStreamCreate(side)");
      if (!ctx->ev_join[i])
        HIP_TRY(hipEventCreateWithFlags(&ctx->ev_join[i], hipEventDisableTiming), "hipEventCreate(join)");
    }
    if (!ctx->ev_fork) HIP_TRY(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming), "hipEventCreate");
    HIP_TRY(hipEventRecord(ctx->ev_fork, s), "hipEventRecord(fork)");
    for (int i = 0; i < nside; ++i) HIP_TRY(hipStreamWaitEvent(ctx->side[i], ctx->ev_fork, 0), "hipStreamWaitEvent");
  }
  for (const LaunchRec& L : B.launches) {
    if (L.kind == sdq::KK_PROD) continue;
    sdq_status st = launch_on(L, stream_of(L));
    if (st) return st;
  }
  if (fork) {
    for (int i = 0; i < nside; ++i) {
      HIP_TRY(hipEventRecord(ctx->ev_join[i], ctx->side[i]), "hipEventRecord(join)");
      HIP_TRY(hipStreamWaitEvent(s, ctx->ev_join[i], 0), "hipStreamWaitEvent(join)");
    }
  }
  return SDQ_OK;
}

// graph cache key: the upload image, the launch list, the status target and
// the swizzle jobs (all pointers included, so any reallocation misses)
std::vector<char> graph_key(const Built& B) {
  std::vector<char> k(B.image);
  auto put = [&](const void* p, size_t n) {
    const char* c = (const char*)p;
    k.insert(k.end(), c, c + n);
  };
  for (const LaunchRec& L : B.launches) put(&L, sizeof L);
  put(&B.status, sizeof B.status);
  put(&B.count, sizeof B.count);
  for (const SwzJob& j : B.swz) put(&j, sizeof j);
  return k;
}

// Upload the plan and run it: all sweeps, then all pair items.  In graph
// mode a batch seen before (same key) replays its captured graph.
sdq_status run_plan(sdq_ctx* ctx, Plan& P, int32_t* status, int count) {
  Built B;
  sdq_status st = build_plan(ctx, P, status, count, B);
  if (st) return st;
  if (B.gang) {
    const size_t need = gang_need(B);
    hipError_t e = grow(ctx->d_gang, need);
    if (e != hipSuccess) return fail(ctx, SDQ_ENOMEM, "gang scratch: " + std::string(hipGetErrorString(e)));
  }
  if (B.tscr_doubles) {
    hipError_t e = grow(ctx->d_tscr, B.tscr_doubles * sizeof(double));
    if (e != hipSuccess) return fail(ctx, SDQ_ENOMEM, "T scratch: " + std::string(hipGetErrorString(e)));
    B.tscr_base = (double*)ctx->d_tscr.p;
  }
  if (ctx->graphs) {
    std::vector<char> key = graph_key(B);
    // the gang and T scratch areas are not part of the image: their addresses are
    const void* gp[2] = {B.gang ? ctx->d_gang.p : nullptr, B.tscr_doubles ? ctx->d_tscr.p : nullptr};
    key.insert(key.end(), (const char*)gp, (const char*)gp + sizeof gp);
    sdq_ctx::GraphEntry* hit = nullptr;
    for (auto& g : ctx->graph_cache)
      if (g.key == key) hit = &g;
    if (!hit) {
      if (ctx->graph_cache.size() >= 16) {
        auto& old = ctx->graph_cache.front();
        HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        if (old.exec) (void)hipGraphExecDestroy(old.exec);
        if (old.h) (void)hipHostFree(old.h);
        if (old.d) (void)hipFree(old.d);
        ctx->graph_cache.erase(ctx->graph_cache.begin());
      }
      sdq_ctx::GraphEntry g;
      g.key = std::move(key);
      HIP_TRY(hipHostMalloc(&g.h, B.image.size(), hipHostMallocDefault), "hipHostMalloc(graph)");
      memcpy(g.h, B.image.data(), B.image.size());
      HIP_TRY(hipMalloc(&g.d, B.image.size()), "hipMalloc(graph)");
      if (!ctx->cap_stream)
        HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
      HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      st = enqueue_built(ctx, B, ctx->cap_stream, (char*)g.d, (const char*)g.h, false);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
      if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphInstantiate");
      ctx->graph_cache.push_back(std::move(g));
      hit = &ctx->graph_cache.back();
    }
    hipGraphExec_t exec = hit->exec;
    return timed(ctx, "graph", [&] { return hipGraphLaunch(exec, ctx->stream); });
  }
  sdq_ctx::StageSlot& sl = ctx->stage[ctx->stage_next];
  ctx->stage_next = (ctx->stage_next + 1) % sdq_ctx::kStageSlots;
  if (sl.pending) {
    HIP_TRY(hipEventSynchronize(sl.ev), "hipEventSynchronize(staging)");
    sl.pending = false;
  }
  const size_t total = B.image.size();
  if (total > sl.cap) {
    if (sl.h) HIP_TRY(hipHostFree(sl.h), "hipHostFree");
    sl.h = nullptr;
    sl.cap = 0;
    HIP_TRY(hipHostMalloc(&sl.h, total * 2, hipHostMallocDefault), "hipHostMalloc");
    sl.cap = total * 2;
  }
  memcpy(sl.h, B.image.data(), total);
  HIP_TRY(grow(ctx->d_upload, total), "hipMalloc(upload)");
  st = enqueue_built(ctx, B, ctx->stream, (char*)ctx->d_upload.p, (const char*)sl.h, true);
  if (st) return st;
  HIP_TRY(hipEventRecord(sl.ev, ctx->stream), "hipEventRecord");
  sl.pending = true;
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
  bool ok = hipSetDevice(device) == hipSuccess;
  for (auto& sl : ctx->stage)
    ok = ok && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    for (auto& sl : ctx->stage)
      if (sl.ev) (void)hipEventDestroy(sl.ev);
    delete ctx;
    return SDQ_EHIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->num_cu = prop.multiProcessorCount;
  // the fixed scratch of sdq_greens_noalloc on this device (device current)
  {
    void* p = nullptr;
    hipError_t e = sdq::noalloc_scratch(device, &p);
    if (e == hipSuccess) {
      ctx->na_scratch = p;
    } else {
      (void)hipGetLastError();
      ctx->na_err = std::string("device scratch lookup failed: ") + hipGetErrorString(e);
    }
    if (hipEventCreateWithFlags(&ctx->na_ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      ctx->na_ev = nullptr;
    }
  }
  for (int nt = 0; nt <= sdq::kMaxNT; ++nt) {
    ctx->tune[nt] = Tune{};
    // defaults (sdq_tune measures them): the slice exponential staged in LDS
    // where that variant exists; above 80 sites one wave per tile with T in
    // scratch (with four waves the register matrices of n > 80 spill)
    ctx->tune[nt].variant = nt >= 6 ? 4 : ((nt >= 3 && nt <= 5) ? 1 : 0);
  }
  // debug overrides (environment): SDQ_SWEEP_VARIANT, SDQ_BLOCKS_PER_CU
  if (const char* v = getenv("SDQ_SWEEP_VARIANT"))
    for (int nt = 0; nt <= sdq::kMaxNT; ++nt) ctx->tune[nt].variant = atoi(v);
  if (const char* v = getenv("SDQ_BLOCKS_PER_CU"))
    for (int nt = 0; nt <= sdq::kMaxNT; ++nt) ctx->tune[nt].blocks_per_cu = atoi(v);
  if (const char* v = getenv("SDQ_BLOCK_PRODUCTS")) ctx->bprod = std::min(2, std::max(0, atoi(v)));
  *out = ctx;
  return SDQ_OK;
}

void sdq_destroy(sdq_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->handles)
    if (kv.second.ckf.p) (void)hipFree(kv.second.ckf.p);
  for (auto& g : ctx->graph_cache) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.h) (void)hipHostFree(g.h);
    if (g.d) (void)hipFree(g.d);
  }
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (int i = 0; i < sdq_ctx::kSide; ++i) {
    if (ctx->side[i]) (void)hipStreamSynchronize(ctx->side[i]);
    if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
    if (ctx->ev_join[i]) (void)hipEventDestroy(ctx->ev_join[i]);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->d_upload.p) (void)hipFree(ctx->d_upload.p);
  if (ctx->d_ck.p) (void)hipFree(ctx->d_ck.p);
  if (ctx->d_swz.p) (void)hipFree(ctx->d_swz.p);
  if (ctx->d_fin.p) (void)hipFree(ctx->d_fin.p);
  if (ctx->d_tscr.p) (void)hipFree(ctx->d_tscr.p);
  if (ctx->d_gang.p) (void)hipFree(ctx->d_gang.p);
  if (ctx->d_ptrs.p) (void)hipFree(ctx->d_ptrs.p);
  if (ctx->d_metro.p) (void)hipFree(ctx->d_metro.p);
  if (ctx->d_gloc.p) (void)hipFree(ctx->d_gloc.p);
  if (ctx->d_lgrad.p) (void)hipFree(ctx->d_lgrad.p);
  if (ctx->d_ltab.p) (void)hipFree(ctx->d_ltab.p);
  if (ctx->d_hmc.p) (void)hipFree(ctx->d_hmc.p);
  if (ctx->d_htab.p) (void)hipFree(ctx->d_htab.p);
  if (ctx->d_ctab.p) (void)hipFree(ctx->d_ctab.p);
  if (ctx->d_prod.p) (void)hipFree(ctx->d_prod.p);
  for (auto& sl : ctx->stage)
    if (sl.h) (void)hipHostFree(sl.h);
  for (auto& kv : ctx->stats)
    for (auto& pr : kv.second.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& sl : ctx->stage)
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  if (ctx->na_ev) (void)hipEventDestroy(ctx->na_ev);
  delete ctx;
}

const char* sdq_last_error(const sdq_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

sdq_status sdq_greens(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, sdq_scheme scheme,
                      double* const* g, double* logdet, double* sign, int32_t* status) {
  SDQ_API_RANGE("sdq_greens");
  sdq_status st = validate(ctx, inst, count, false);
  if (st) return st;
  if (scheme != SDQ_INV_LOH && scheme != SDQ_INV_PLAIN) return fail(ctx, SDQ_EINVAL, "unknown scheme");
  if (count == 0) return SDQ_OK;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int64_t> off;
  st = alloc_fin(ctx, inst, count, off);
  if (st) return st;
  Plan P;
  // Block products first (k_prod: every block of k slices of every chain
  // multiplied out at once), then the sweep over them with one
  // factorization each: the same stabilized product (Sec. 4.1), with the
  // sequential part of a chain cut to its factorizations.  Automatically
  // for the tile class (kProdMinNT .. kSweepMaxNT tiles) that holds the
  // batch's longest chain, when all of its chains are resident at once (then
  // that chain's sweep is the batch's critical path); for every such class
  // by the context's setting.
  if (ctx->bprod != 0 && ctx->stab == SDQ_STAB_QR) {
    int cnt_nt[sdq::kSweepMaxNT + 1] = {};
    double longest = 0.0;
    int crit = -1;
    for (int i = 0; i < count; ++i) {
      const int nt = nt_of(inst[i].n);
      if (nt >= sdq::kProdMinNT && nt <= sdq::kSweepMaxNT) cnt_nt[nt] += 1;
      const double c = sweep_cost(inst[i].n, inst[i].m, inst[i].k);
      if (c > longest) {
        longest = c;
        crit = nt;
      }
    }
    for (int nt = sdq::kProdMinNT; nt <= sdq::kSweepMaxNT; ++nt) {
      if (cnt_nt[nt] == 0) continue;
      if (ctx->bprod == 1 ||
          (nt == crit && cnt_nt[nt] <= grid_for(ctx, sdq::KK_SWEEP, nt, 6, 1 << 30)))
        P.bprod_mask |= 1u << nt;
    }
  }
  double* prod_base = nullptr;
  std::vector<int64_t> poff(count, -1);
  if (P.bprod_mask) {
    int64_t tot = 0;
    for (int i = 0; i < count; ++i) {
      const int nt = nt_of(inst[i].n);
      if (!((P.bprod_mask >> nt) & 1u)) continue;
      poff[i] = tot;
      tot += (int64_t)nb_of(inst[i].m, inst[i].k) * 256 * nt * nt;
    }
    // the products only shorten the critical path: without memory for
    // them the classes sweep over the slices as they are
    if (grow(ctx->d_prod, (size_t)tot * sizeof(double)) == hipSuccess) {
      prod_base = (double*)ctx->d_prod.p;
    } else {
      (void)hipGetLastError();
      P.bprod_mask = 0;
      std::fill(poff.begin(), poff.end(), -1);
    }
  }
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(inst[i]);
    I.scheme = scheme == SDQ_INV_PLAIN ? 1 : 0;
    I.g = g ? g[i] : nullptr;
    I.logdet = logdet ? logdet + i : nullptr;
    I.sign = sign ? sign + i : nullptr;
    I.status = status ? status + i : nullptr;
    I.fin = (double*)ctx->d_fin.p + off[i];
    if (poff[i] >= 0) {
      // the products' instance (slices as given, outputs none) and the
      // sweep's (one dense slice per block, k = 1)
      Inst Ip = base_inst(inst[i]);
      Ip.prod = prod_base + poff[i];
      const int ip = (int)P.inst.size();
      P.inst.push_back(Ip);
      for (int j = 0; j < I.nb; ++j) P.prod.push_back(SweepItem{ip, 0, j, 0});
      I.expk = nullptr;
      I.expk_inv = nullptr;
      I.field = Ip.prod;
      I.m = I.nb;
      I.k = 1;
    }
    const int id = (int)P.inst.size();
    P.inst.push_back(I);
    P.sweep.push_back(SweepItem{id, sdq::SW_LAST, 0, 0});
    P.pair[sdq::PAIR_EQUAL].push_back(PairItem{id, I.nb, 0, 0});
  }
  order_items(P.inst, P.prod, P.prod_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return (double)I.n * I.n * I.n * std::min(I.k, I.m - w.j * I.k);
  });
  order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return sweep_cost(I.n, I.m, I.k);
  });
  order_all_pairs(P);
  ctx->err.clear();
  return run_plan(ctx, P, status, count);
}

// sdq_greens without any allocation: every buffer the kernels need beyond
// the caller's (the plan image, the swizzled slice exponentials, the final
// stages, the T scratch) is carved out of this device's fixed scratch.
sdq_status sdq_greens_noalloc(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, sdq_scheme scheme,
                              double* const* g, double* logdet, double* sign, int32_t* status) {
  SDQ_API_RANGE("sdq_greens_noalloc");
  sdq_status st = validate(ctx, inst, count, false);
  if (st) return st;
  if (scheme != SDQ_INV_LOH && scheme != SDQ_INV_PLAIN) return fail(ctx, SDQ_EINVAL, "unknown scheme");
  for (int i = 0; i < count; ++i)
    if (inst[i].n > 16 * sdq::kMaxNT)
      return fail(ctx, SDQ_EUNSUPPORTED, "sdq_greens_noalloc: chains of n > 128 need the gang scratch");
  if (count == 0) return SDQ_OK;
  if (!ctx->na_scratch) return fail(ctx, SDQ_EHIP, "sdq_greens_noalloc: " + ctx->na_err);
  if (!ctx->na_ev) return fail(ctx, SDQ_EHIP, "sdq_greens_noalloc: no upload event");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  // layout: [swizzled operands | final stages | T scratch | plan image]
  size_t swz = 0;
  {
    std::vector<std::pair<const double*, int>> seen;
    for (int i = 0; i < count; ++i) {
      const auto key = std::make_pair(inst[i].expk, inst[i].n);
      if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
      seen.push_back(key);
      const size_t np = 16 * (size_t)nt_of(inst[i].n);
      swz += 2 * np * np * sizeof(double);
    }
  }
  std::vector<int64_t> off(count);
  int64_t fin = 0;
  for (int i = 0; i < count; ++i) {
    off[i] = fin;
    fin += (sdq::stage_doubles(inst[i].n) + 31) & ~(int64_t)31;
  }
  char* base = (char*)ctx->na_scratch;
  const size_t o_fin = align(swz);
  const size_t o_tscr = align(o_fin + (size_t)fin * sizeof(double));
  if (o_tscr > sdq::kNoAllocBytes)
    return fail(ctx, SDQ_EINVAL,
                "sdq_greens_noalloc: the batch needs more than the " + std::to_string(sdq::kNoAllocBytes >> 20) +
                    " MiB of fixed scratch (" + std::to_string(o_tscr) + " bytes before the plan); split it");
  Plan P;
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(inst[i]);
    I.scheme = scheme == SDQ_INV_PLAIN ? 1 : 0;
    I.g = g ? g[i] : nullptr;
    I.logdet = logdet ? logdet + i : nullptr;
    I.sign = sign ? sign + i : nullptr;
    I.status = status ? status + i : nullptr;
    I.fin = (double*)(base + o_fin) + off[i];
    P.inst.push_back(I);
    P.sweep.push_back(SweepItem{i, sdq::SW_LAST, 0, 0});
    P.pair[sdq::PAIR_EQUAL].push_back(PairItem{i, I.nb, 0, 0});
  }
  order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return sweep_cost(I.n, I.m, I.k);
  });
  order_all_pairs(P);
  ctx->err.clear();
  Built B;
  st = build_plan(ctx, P, status, count, B, (double*)base);
  if (st) return st;
  const size_t o_img = align(o_tscr + B.tscr_doubles * sizeof(double));
  if (o_img + B.image.size() > sdq::kNoAllocBytes)
    return fail(ctx, SDQ_EINVAL,
                "sdq_greens_noalloc: the batch needs " + std::to_string(o_img + B.image.size()) +
                    " bytes of fixed scratch, more than " + std::to_string(sdq::kNoAllocBytes >> 20) +
                    " MiB; split it");
  B.tscr_base = B.tscr_doubles ? (double*)(base + o_tscr) : nullptr;
  B.fork = false;  // side streams would be created on first use
  // the host copy of the previous image must outlive its upload
  if (ctx->na_pending) {
    HIP_TRY(hipEventSynchronize(ctx->na_ev), "hipEventSynchronize(noalloc)");
    ctx->na_pending = false;
  }
  ctx->na_image = B.image;
  HIP_TRY(hipMemcpyAsync(base + o_img, ctx->na_image.data(), ctx->na_image.size(), hipMemcpyHostToDevice,
                         ctx->stream),
          "hipMemcpyAsync(plan)");
  HIP_TRY(hipEventRecord(ctx->na_ev, ctx->stream), "hipEventRecord(noalloc)");
  ctx->na_pending = true;
  return enqueue_built(ctx, B, ctx->stream, base + o_img, nullptr, false);
}

namespace {
// checks of dense-slice instances; shape[i] gets their n, m, k (other fields
// zero) for the helpers that size library memory by instance
sdq_status validate_dense(sdq_ctx* ctx, const sdq_dense_instance* inst, int32_t count,
                          std::vector<sdq_instance>& shape) {
  if (count > 0 && !inst) return fail(ctx, SDQ_EINVAL, "inst is NULL");
  if (ctx->stab != SDQ_STAB_QR) return fail(ctx, SDQ_EUNSUPPORTED, "dense slices use the QR stabilizer");
  shape.assign(count, sdq_instance{});
  for (int i = 0; i < count; ++i) {
    const sdq_dense_instance& d = inst[i];
    char buf[160];
    if (d.n < 1 || d.n > 16 * sdq::kMaxNT) {
      snprintf(buf, sizeof buf, "instance %d: dense slices need 1 <= n <= 128 (n = %d)", i, d.n);
      return fail(ctx, d.n < 1 ? SDQ_EINVAL : SDQ_EUNSUPPORTED, buf);
    }
    if (d.m < 1 || d.k < 1 || d.k > d.m || !d.slices) {
      snprintf(buf, sizeof buf, "instance %d: need m >= 1, 1 <= k <= m and slices", i);
      return fail(ctx, SDQ_EINVAL, buf);
    }
    shape[i].n = d.n;
    shape[i].m = d.m;
    shape[i].k = d.k;
  }
  return SDQ_OK;
}
}  // namespace

sdq_status sdq_greens_dense(sdq_ctx* ctx, const sdq_dense_instance* inst, int32_t count, double* const* g,
                            double* logdet, double* sign, int32_t* status) {
  SDQ_API_RANGE("sdq_greens_dense");
  if (!ctx) return SDQ_EINVAL;
  if (count < 0) return fail(ctx, SDQ_EINVAL, "count < 0");
  std::vector<sdq_instance> shape;
  sdq_status st0 = validate_dense(ctx, inst, count, shape);
  if (st0) return st0;
  if (count == 0) return SDQ_OK;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int64_t> off;
  sdq_status st = alloc_fin(ctx, shape.data(), count, off);
  if (st) return st;
  Plan P;
  P.dense = true;
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(shape[i]);
    I.field = inst[i].slices;  // read as the dense slices by the dense sweep
    I.g = g ? g[i] : nullptr;
    I.logdet = logdet ? logdet + i : nullptr;
    I.sign = sign ? sign + i : nullptr;
    I.status = status ? status + i : nullptr;
    I.fin = (double*)ctx->d_fin.p + off[i];
    P.inst.push_back(I);
    P.sweep.push_back(SweepItem{i, sdq::SW_LAST, 0, 0});
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

sdq_status sdq_greens_tdisp_dense(sdq_ctx* ctx, const sdq_dense_instance* inst, int32_t count,
                                  const int32_t* l_list, int32_t n_l, double* const* gt, double* const* g,
                                  double* logdet, double* sign, int32_t* status) {
  SDQ_API_RANGE("sdq_greens_tdisp_dense");
  if (!ctx) return SDQ_EINVAL;
  if (count < 0) return fail(ctx, SDQ_EINVAL, "count < 0");
  std::vector<sdq_instance> shape;
  sdq_status st = validate_dense(ctx, inst, count, shape);
  if (st) return st;
  if (n_l < 0 || (n_l > 0 && (!l_list || !gt))) return fail(ctx, SDQ_EINVAL, "bad l_list / gt");
  for (int a = 0; a < n_l; ++a) {
    if (l_list[a] < 0) return fail(ctx, SDQ_EINVAL, "l_list entry < 0");
    if (a > 0 && l_list[a] <= l_list[a - 1]) return fail(ctx, SDQ_EINVAL, "l_list must be strictly ascending");
  }
  for (int i = 0; i < count; ++i) {
    if (n_l > 0 && l_list[n_l - 1] > shape[i].m) return fail(ctx, SDQ_EINVAL, "l_list entry > m");
    if (n_l > 0 && !gt[i]) return fail(ctx, SDQ_EINVAL, "gt entry is NULL");
  }
  if (count == 0) return SDQ_OK;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int64_t> off;
  st = alloc_stages(ctx, ctx->d_ck, shape.data(), count, 2, off);
  if (st) return st;
  double* ck = (double*)ctx->d_ck.p;
  Plan P;
  P.dense = true;
  P.llist.assign(l_list, l_list + n_l);
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(shape[i]);
    I.field = inst[i].slices;  // read as the dense slices by the dense sweeps
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
    P.sweep.push_back(SweepItem{i, sdq::SW_STORE, 0, 0});
    P.sweep.push_back(SweepItem{i, sdq::SW_STORE | sdq::SW_ADJ, 0, 0});
    if (I.g || I.logdet || I.sign) P.pair[sdq::PAIR_EQUAL].push_back(PairItem{i, I.nb, 0, 0});
    // group l by stage pair j (l == m -> nb, else l / k); the l inside a
    // block are reached from its start by multiplying with the dense slices
    for (int a = 0; a < n_l;) {
      const int l = l_list[a];
      const int j = (l == I.m) ? I.nb : l / I.k;
      int b = a + 1;
      while (b < n_l) {
        const int l2 = l_list[b];
        if (((l2 == I.m) ? I.nb : l2 / I.k) != j) break;
        ++b;
      }
      P.pair[sdq::PAIR_TDISP_DENSE].push_back(PairItem{i, j, a, b});
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

sdq_status sdq_greens_tdisp(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, sdq_scheme scheme,
                            const int32_t* l_list, int32_t n_l, double* const* gt,
                            double* const* g, double* logdet, double* sign, int32_t* status) {
  SDQ_API_RANGE("sdq_greens_tdisp");
  sdq_status st = validate(ctx, inst, count, false);
  if (st) return st;
  if (scheme != SDQ_INV_LOH && scheme != SDQ_INV_PLAIN) return fail(ctx, SDQ_EINVAL, "unknown scheme");
  if (n_l < 0 || (n_l > 0 && (!l_list || !gt))) return fail(ctx, SDQ_EINVAL, "bad l_list / gt");
  for (int a = 0; a < n_l; ++a) {
    if (l_list[a] < 0) return fail(ctx, SDQ_EINVAL, "l_list entry < 0");
    if (a > 0 && l_list[a] <= l_list[a - 1]) return fail(ctx, SDQ_EINVAL, "l_list must be strictly ascending");
  }
  for (int i = 0; i < count; ++i) {
    if (n_l > 0 && l_list[n_l - 1] > inst[i].m) return fail(ctx, SDQ_EINVAL, "l_list entry > m");
    if (n_l > 0 && !gt[i]) return fail(ctx, SDQ_EINVAL, "gt entry is NULL");
  }
  const bool plain = scheme == SDQ_INV_PLAIN;
  if (plain) {
    // the single-decomposition G(tau,0) decomposes B(tau,0)^{-1} itself
    st = validate(ctx, inst, count, true);
    if (st) return st;
    for (int i = 0; i < count; ++i)
      if (inst[i].n > 16 * sdq::kMaxNT)
        return fail(ctx, SDQ_EUNSUPPORTED,
                    "the single-decomposition G(tau,0) is implemented for n <= 128 only");
  }
  if (count == 0) return SDQ_OK;
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int64_t> off;
  // Loh: forward and backward stage stacks; plain: per-pair chains in the
  // same two stacks plus a third for the final forward stage
  st = alloc_stages(ctx, ctx->d_ck, inst, count, plain ? 3 : 2, off);
  if (st) return st;
  double* ck = (double*)ctx->d_ck.p;
  Plan P;
  P.llist.assign(l_list, l_list + n_l);
  P.swz_inv = plain;
  for (int i = 0; i < count; ++i) {
    Inst I = base_inst(inst[i]);
    I.scheme = plain ? 1 : 0;
    I.g = g ? g[i] : nullptr;
    I.gt = n_l > 0 ? gt[i] : nullptr;
    I.logdet = logdet ? logdet + i : nullptr;
    I.sign = sign ? sign + i : nullptr;
    I.status = status ? status + i : nullptr;
    const int64_t sd = sdq::stage_doubles(I.n);
    const int64_t one = (int64_t)I.nb * sd;
    I.ckf = ck + off[i];
    I.cka = ck + off[i] + one;
    I.fin = plain ? ck + off[i] + 2 * one : I.ckf + (I.nb - 1) * sd;
    P.inst.push_back(I);
    const bool eq = I.g || I.logdet || I.sign;
    if (!plain) {
      P.sweep.push_back(SweepItem{i, sdq::SW_STORE, 0, 0});
      P.sweep.push_back(SweepItem{i, sdq::SW_STORE | sdq::SW_ADJ, 0, 0});
    } else if (eq) {
      P.sweep.push_back(SweepItem{i, sdq::SW_LAST, 0, 0});
    }
    if (eq) P.pair[sdq::PAIR_EQUAL].push_back(PairItem{i, I.nb, 0, 0});
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
      if (plain) {
        if (j > 0) P.sweep.push_back(SweepItem{i, sdq::SW_LEFT, j, 0});
        if (j < I.nb) P.sweep.push_back(SweepItem{i, sdq::SW_RIGHT, j, 0});
      }
      P.pair[plain ? sdq::PAIR_TDISP_PLAIN : sdq::PAIR_TDISP].push_back(PairItem{i, j, a, b});
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
  SDQ_API_RANGE("sdq_logdet");
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
    P.sweep.push_back(SweepItem{i, flags, 0, 0});
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
  SDQ_API_RANGE("sdq_logdet_grad");
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
      P.sweep.push_back(SweepItem{i, sdq::SW_STORE, 0, 0});
    }
    I.fin = I.ckf + (I.nb - 1) * sd;
    P.sweep.push_back(SweepItem{i, sdq::SW_STORE | sdq::SW_ADJ, 0, 0});
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
  SDQ_API_RANGE("sdq_udt");
  if (!ctx) return SDQ_EINVAL;
  if (n < 1 || count < 0) return fail(ctx, SDQ_EINVAL, "bad n or count");
  if (n > sdq::kGangMaxN) return fail(ctx, SDQ_EUNSUPPORTED, "n > 1024 is not supported");
  if (count == 0) return SDQ_OK;
  if (!w || !u || !d || !t) return fail(ctx, SDQ_EINVAL, "null pointer");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  ctx->err.clear();
  const int nt = nt_of(n);
  if (is_gang(nt)) {
    const int ng = grid_for(ctx, sdq::KK_UDT, nt, 0, count);
    HIP_TRY(grow(ctx->d_gang, gang_bytes(nt, ng)), "hipMalloc(gang scratch)");
    sdq::GangArgs a;
    a.bars = (unsigned*)ctx->d_gang.p;
    a.scratch = (double*)((char*)ctx->d_gang.p + gang_bars_bytes(ng));
    a.ngangs = ng;
    a.nt = nt;
    return timed(ctx, "udt", [&] {
      hipError_t e = sdq::launch_fill_i32((int32_t*)a.bars, ng * sdq::kGangBarWords, 0, ctx->stream);
      if (e != hipSuccess) return e;
      return sdq::launch_gang_udt(n, count, w, u, d, t, a, ctx->stream);
    });
  }
  return timed(ctx, "udt", [&] { return sdq::launch_udt(nt, n, count, w, u, d, t, ctx->stream); });
}

sdq_status sdq_udt_complex(sdq_ctx* ctx, int32_t n, int32_t count, const double* w, double* u, double* d,
                           double* t) {
  SDQ_API_RANGE("sdq_udt_complex");
  if (!ctx) return SDQ_EINVAL;
  if (n < 1 || count < 0) return fail(ctx, SDQ_EINVAL, "bad n or count");
  if (n > sdq::complex_udt_max_n()) return fail(ctx, SDQ_EUNSUPPORTED, "complex UDT: n > 64 is not supported");
  if (count == 0) return SDQ_OK;
  if (!w || !u || !d || !t) return fail(ctx, SDQ_EINVAL, "null pointer");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  ctx->err.clear();
  // two workgroups per CU (73 KB of LDS each), grid-stride over the matrices
  const int grid = std::max(1, std::min(count, 2 * ctx->num_cu));
  return timed(ctx, "udt_complex",
               [&] { return sdq::launch_udt_complex(n, count, w, u, d, t, grid, ctx->stream); });
}

sdq_status sdq_greens_complex(sdq_ctx* ctx, const sdq_complex_instance* inst, int32_t count, double* const* g,
                              double* logdet, double* phase, int32_t* status) {
  SDQ_API_RANGE("sdq_greens_complex");
  if (!ctx) return SDQ_EINVAL;
  if (count < 0) return fail(ctx, SDQ_EINVAL, "count < 0");
  if (count == 0) return SDQ_OK;
  if (!inst) return fail(ctx, SDQ_EINVAL, "inst is NULL");
  std::vector<sdq::CChain> tab(count);
  for (int i = 0; i < count; ++i) {
    const sdq_complex_instance& c = inst[i];
    char buf[160];
    if (c.n < 1 || c.n > sdq::complex_udt_max_n()) {
      snprintf(buf, sizeof buf, "instance %d: complex chains need 1 <= n <= %d (n = %d)", i,
               sdq::complex_udt_max_n(), c.n);
      return fail(ctx, c.n < 1 ? SDQ_EINVAL : SDQ_EUNSUPPORTED, buf);
    }
    if (c.m < 1 || c.k < 1 || c.k > c.m || !c.slices) {
      snprintf(buf, sizeof buf, "instance %d: need m >= 1, 1 <= k <= m and slices", i);
      return fail(ctx, SDQ_EINVAL, buf);
    }
    tab[i] = sdq::CChain{c.slices, g ? g[i] : nullptr, logdet ? logdet + i : nullptr,
                         phase ? phase + 2 * i : nullptr, status ? status + i : nullptr, c.n, c.m, c.k, 0};
  }
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  ctx->err.clear();
  HIP_TRY(grow(ctx->d_ctab, (size_t)count * sizeof(sdq::CChain)), "hipMalloc(chain table)");
  // stream-ordered after any earlier launch that read the table; the source
  // is pageable, so it may be reused once this returns
  HIP_TRY(hipMemcpyAsync(ctx->d_ctab.p, tab.data(), (size_t)count * sizeof(sdq::CChain), hipMemcpyHostToDevice,
                         ctx->stream),
          "hipMemcpyAsync(chain table)");
  if (status) HIP_TRY(sdq::launch_fill_i32(status, count, 0, ctx->stream), "fill(status)");
  // one workgroup per CU (148 KB of LDS), grid-stride over the chains
  const int grid = std::max(1, std::min(count, ctx->num_cu));
  return timed(ctx, "greens_complex", [&] {
    return sdq::launch_greens_complex((const sdq::CChain*)ctx->d_ctab.p, count, grid, ctx->stream);
  });
}

sdq_status sdq_local_sweep(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, int32_t nf,
                           const double* unif, int32_t* accepted, int32_t* status) {
  SDQ_API_RANGE("sdq_local_sweep");
  if (!ctx) return SDQ_EINVAL;
  if (count < 0 || nf < 1 || nf > 2) return fail(ctx, SDQ_EINVAL, "need count >= 0 and nf in {1, 2}");
  if (count == 0) return SDQ_OK;
  if (!unif || !accepted) return fail(ctx, SDQ_EINVAL, "null pointer");
  const int total = count * nf;
  sdq_status st = validate(ctx, inst, total, true);
  if (st) return st;
  for (int c = 0; c < count; ++c) {
    const sdq_instance& a = inst[c * nf];
    if (a.n > 16 * sdq::kMaxNT)
      return fail(ctx, SDQ_EUNSUPPORTED, "local updates are implemented for n <= 128");
    for (int f = 1; f < nf; ++f) {
      const sdq_instance& b = inst[c * nf + f];
      if (b.field != a.field || b.n != a.n || b.m != a.m || b.k != a.k)
        return fail(ctx, SDQ_EINVAL, "the flavours of a chain must share field, n, m and k");
    }
  }
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  std::vector<int64_t> off;
  st = alloc_stages(ctx, ctx->d_ck, inst, total, 2, off);
  if (st) return st;
  double* ck = (double*)ctx->d_ck.p;
  size_t gdoubles = 0;
  for (int i = 0; i < total; ++i) gdoubles += (size_t)inst[i].n * inst[i].n;
  HIP_TRY(grow(ctx->d_gloc, gdoubles * sizeof(double)), "hipMalloc(local G)");
  double* gl = (double*)ctx->d_gloc.p;
  std::vector<Inst> base;
  size_t uoff = 0;
  for (int c = 0; c < count; ++c) {
    for (int f = 0; f < nf; ++f) {
      const int i = c * nf + f;
      Inst I = base_inst(inst[i]);
      const int64_t one = (int64_t)I.nb * sdq::stage_doubles(I.n);
      I.ckf = ck + off[i];
      I.cka = ck + off[i] + one;
      I.g = gl;
      gl += (size_t)I.n * I.n;
      I.status = status ? status + i : nullptr;
      I.unif = unif + uoff;
      I.nacc = accepted + c;
      base.push_back(I);
    }
    uoff += (size_t)inst[c * nf].m * inst[c * nf].n;
  }
  HIP_TRY(sdq::launch_fill_i32(accepted, count, 0, ctx->stream), "fill(accepted)");
  ctx->err.clear();
  // backward stages of the current field: the slices after each block stay
  // unchanged until the sweep reaches them
  {
    Plan P;
    P.inst = base;
    for (int i = 0; i < total; ++i) P.sweep.push_back(SweepItem{i, sdq::SW_STORE | sdq::SW_ADJ, 0, 0});
    order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
      const Inst& I = P.inst[w.inst];
      return sweep_cost(I.n, I.m, I.k);
    });
    st = run_plan(ctx, P, status, total);
    if (st) return st;
  }
  int nbmax = 0;
  for (const Inst& I : base) nbmax = std::max(nbmax, I.nb);
  for (int j = 0; j < nbmax; ++j) {
    // G at the block start, one item per flavour, then the block's sites
    Plan B;
    B.inst = base;
    B.swz_ready = true;
    for (int i = 0; i < total; ++i)
      if (j < base[i].nb) B.pair[sdq::PAIR_BSTART].push_back(PairItem{i, j, 0, 0});
    order_all_pairs(B);
    st = run_plan(ctx, B, nullptr, 0);
    if (st) return st;
    Plan P;
    P.inst = base;
    P.swz_ready = true;
    for (int c = 0; c < count; ++c)
      if (j < base[c * nf].nb) P.pair[sdq::PAIR_LOCAL].push_back(PairItem{c * nf, j, nf, 0});
    order_all_pairs(P);
    st = run_plan(ctx, P, nullptr, 0);
    if (st) return st;
    // forward stage j+1 from the updated field of block j
    Plan Q;
    Q.inst = base;
    Q.swz_ready = true;
    for (int i = 0; i < total; ++i)
      if (j + 1 < base[i].nb) Q.sweep.push_back(SweepItem{i, sdq::SW_BLOCK, j, 0});
    if (Q.sweep.empty()) continue;
    order_items(Q.inst, Q.sweep, Q.sweep_ranges, [&](const SweepItem& w) {
      const Inst& I = Q.inst[w.inst];
      return (double)I.n * I.n * I.n;
    });
    st = run_plan(ctx, Q, nullptr, 0);
    if (st) return st;
  }
  return SDQ_OK;
}

sdq_status sdq_metropolis(sdq_ctx* ctx, const sdq_instance* cur, const sdq_instance* prop,
                          int32_t count, int32_t nf, const double* dS, const double* u, double* logdet,
                          double* sign, int32_t* accept, int32_t* status) {
  SDQ_API_RANGE("sdq_metropolis");
  if (!ctx) return SDQ_EINVAL;
  if (count < 0 || nf < 1) return fail(ctx, SDQ_EINVAL, "need count >= 0 and nf >= 1");
  if (count == 0) return SDQ_OK;
  if (!cur || !prop || !dS || !u || !logdet || !sign || !accept)
    return fail(ctx, SDQ_EINVAL, "null pointer");
  const int total = count * nf;
  sdq_status st = validate(ctx, prop, total, false);
  if (st) return st;
  for (int i = 0; i < total; ++i) {
    if (!cur[i].field || cur[i].n != prop[i].n || cur[i].m != prop[i].m)
      return fail(ctx, SDQ_EINVAL, "cur and prop differ in n or m (or cur field is NULL)");
    if (cur[i].field == prop[i].field) return fail(ctx, SDQ_EINVAL, "cur and prop share a field");
  }
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  // device layout: fields [total] | ld_prop [total] | sg_prop [total] | st_prop [total]
  const size_t o_ld = ((size_t)total * sizeof(sdq::MetroField) + 255) & ~(size_t)255;
  const size_t o_sg = o_ld + (((size_t)total * sizeof(double) + 255) & ~(size_t)255);
  const size_t o_st = o_sg + (((size_t)total * sizeof(double) + 255) & ~(size_t)255);
  const size_t bytes = o_st + (size_t)total * sizeof(int32_t);
  HIP_TRY(grow(ctx->d_metro, bytes), "hipMalloc(metropolis)");
  char* base = (char*)ctx->d_metro.p;
  std::vector<sdq::MetroField> tab(total);
  for (int i = 0; i < total; ++i)
    tab[i] = sdq::MetroField{const_cast<double*>(cur[i].field), prop[i].field,
                             (int64_t)prop[i].m * prop[i].n};
  // the proposed log|det| and signs (the stabilized sweep and the equal-time
  // inversion of every proposed instance), then the decisions
  double* ld_p = (double*)(base + o_ld);
  double* sg_p = (double*)(base + o_sg);
  int32_t* st_p = status ? status : (int32_t*)(base + o_st);
  st = sdq_logdet(ctx, prop, total, ld_p, sg_p, st_p, nullptr);
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(base, tab.data(), (size_t)total * sizeof(sdq::MetroField), hipMemcpyHostToDevice,
                         ctx->stream),
          "hipMemcpyAsync(field table)");
  ctx->err.clear();
  return timed(ctx, "metropolis", [&] {
    return sdq::launch_metropolis(count, nf, (const sdq::MetroField*)base, ld_p, sg_p, st_p, dS, u,
                                  logdet, sign, accept, ctx->stream);
  });
}

sdq_status sdq_langevin(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, int32_t nf, double eps,
                        double inv_var, const double* noise, double* force, double* logdet, double* sign,
                        int32_t* status) {
  SDQ_API_RANGE("sdq_langevin");
  if (!ctx) return SDQ_EINVAL;
  if (count < 0 || nf < 1) return fail(ctx, SDQ_EINVAL, "need count >= 0 and nf >= 1");
  if (count == 0) return SDQ_OK;
  if (!noise) return fail(ctx, SDQ_EINVAL, "noise is NULL");
  if (!(eps > 0.0) || !std::isfinite(eps) || !(inv_var >= 0.0) || !std::isfinite(inv_var))
    return fail(ctx, SDQ_EINVAL, "need eps > 0 and a finite inv_var >= 0");
  const int total = count * nf;
  sdq_status st = validate(ctx, inst, total, true);
  if (st) return st;
  for (int c = 0; c < count; ++c) {
    const sdq_instance& a = inst[c * nf];
    for (int f = 1; f < nf; ++f) {
      const sdq_instance& b = inst[c * nf + f];
      if (b.field != a.field || b.n != a.n || b.m != a.m)
        return fail(ctx, SDQ_EINVAL, "the flavours of a chain must share field, n and m");
    }
  }
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  // the gradient of every instance (and the statuses, when the caller keeps
  // none) in the context's scratch, back to back
  size_t gtot = 0;
  int64_t lmax = 0;
  for (int i = 0; i < total; ++i) {
    gtot += (size_t)inst[i].m * inst[i].n;
    lmax = std::max<int64_t>(lmax, (int64_t)inst[i].m * inst[i].n);
  }
  const size_t o_st = (gtot * sizeof(double) + 255) & ~(size_t)255;
  HIP_TRY(grow(ctx->d_lgrad, o_st + (size_t)total * sizeof(int32_t)), "hipMalloc(langevin)");
  int32_t* stp = status ? status : (int32_t*)((char*)ctx->d_lgrad.p + o_st);
  std::vector<double*> gp(total);
  double* g = (double*)ctx->d_lgrad.p;
  for (int i = 0; i < total; ++i) {
    gp[i] = g;
    g += (size_t)inst[i].m * inst[i].n;
  }
  st = sdq_logdet_grad(ctx, 0, inst, total, gp.data(), logdet, sign, stp);
  if (st) return st;
  std::vector<sdq::LangevinChain> tab(count);
  size_t noff = 0;
  for (int c = 0; c < count; ++c) {
    const sdq_instance& a = inst[c * nf];
    const int64_t len = (int64_t)a.m * a.n;
    tab[c] = sdq::LangevinChain{const_cast<double*>(a.field), gp[c * nf], noise + noff,
                                force ? force + noff : nullptr, stp + c * nf, len};
    noff += (size_t)len;
  }
  HIP_TRY(grow(ctx->d_ltab, (size_t)count * sizeof(sdq::LangevinChain)), "hipMalloc(langevin table)");
  // stream-ordered after the previous step's update read the table; the
  // source is pageable, so it may be reused once this returns
  HIP_TRY(hipMemcpyAsync(ctx->d_ltab.p, tab.data(), (size_t)count * sizeof(sdq::LangevinChain),
                         hipMemcpyHostToDevice, ctx->stream),
          "hipMemcpyAsync(langevin table)");
  ctx->err.clear();
  // about four workgroups per CU over the batch, at least one per chain
  const int per = (int)std::max<int64_t>(1, std::min<int64_t>((lmax + 255) / 256,
                                                               (4LL * ctx->num_cu + count - 1) / count));
  const auto* d_tab = (const sdq::LangevinChain*)ctx->d_ltab.p;
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int cn = std::min(count - c0, 65535);
    st = timed(ctx, "langevin", [&] {
      return sdq::launch_langevin(cn, nf, d_tab + c0, eps, inv_var, per, ctx->stream);
    });
    if (st) return st;
  }
  return SDQ_OK;
}

sdq_status sdq_hmc(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, int32_t nf, double eps,
                   int32_t nsteps, double inv_var, const double* mom, const double* u, double* logdet,
                   double* sign, int32_t* accept, double* dH, int32_t* status) {
  SDQ_API_RANGE("sdq_hmc");
  if (!ctx) return SDQ_EINVAL;
  if (count < 0 || nf < 1) return fail(ctx, SDQ_EINVAL, "need count >= 0 and nf >= 1");
  if (count == 0) return SDQ_OK;
  if (!mom || !u || !accept) return fail(ctx, SDQ_EINVAL, "null pointer");
  if (!(eps > 0.0) || !std::isfinite(eps) || !(inv_var >= 0.0) || !std::isfinite(inv_var) || nsteps < 1)
    return fail(ctx, SDQ_EINVAL, "need eps > 0, nsteps >= 1 and a finite inv_var >= 0");
  const int total = count * nf;
  sdq_status st = validate(ctx, inst, total, true);
  if (st) return st;
  for (int c = 0; c < count; ++c) {
    const sdq_instance& a = inst[c * nf];
    for (int f = 1; f < nf; ++f) {
      const sdq_instance& b = inst[c * nf + f];
      if (b.field != a.field || b.n != a.n || b.m != a.m)
        return fail(ctx, SDQ_EINVAL, "the flavours of a chain must share field, n and m");
    }
  }
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  // scratch: gradients [total] | start fields [count] | momenta [count] |
  // e0 [count] | ld0, sg0, ld1, sg1 [total] | statuses [nsteps + 1][total]
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t gl = 0, cl = 0;
  int64_t lmax = 0;
  for (int i = 0; i < total; ++i) gl += (size_t)inst[i].m * inst[i].n;
  for (int c = 0; c < count; ++c) {
    const int64_t len = (int64_t)inst[c * nf].m * inst[c * nf].n;
    cl += (size_t)len;
    lmax = std::max(lmax, len);
  }
  const int n_eval = nsteps + 1;
  const size_t o_phi0 = al(gl * sizeof(double));
  const size_t o_p = o_phi0 + al(cl * sizeof(double));
  const size_t o_e0 = o_p + al(cl * sizeof(double));
  const size_t o_ld = o_e0 + al((size_t)count * sizeof(double));
  const size_t o_st = o_ld + 4 * al((size_t)total * sizeof(double));
  const size_t bytes = o_st + (size_t)n_eval * total * sizeof(int32_t);
  HIP_TRY(grow(ctx->d_hmc, bytes), "hipMalloc(hmc)");
  char* base = (char*)ctx->d_hmc.p;
  std::vector<double*> gp(total);
  {
    double* g = (double*)base;
    for (int i = 0; i < total; ++i) {
      gp[i] = g;
      g += (size_t)inst[i].m * inst[i].n;
    }
  }
  double* e0 = (double*)(base + o_e0);
  double* ld0 = (double*)(base + o_ld);
  double* sg0 = (double*)(base + o_ld + al((size_t)total * sizeof(double)));
  double* ld1 = (double*)(base + o_ld + 2 * al((size_t)total * sizeof(double)));
  double* sg1 = (double*)(base + o_ld + 3 * al((size_t)total * sizeof(double)));
  int32_t* st_all = (int32_t*)(base + o_st);
  std::vector<sdq::HmcChain> tab(count);
  {
    double* phi0 = (double*)(base + o_phi0);
    double* pm = (double*)(base + o_p);
    size_t off = 0;
    for (int c = 0; c < count; ++c) {
      const sdq_instance& a = inst[c * nf];
      const int64_t len = (int64_t)a.m * a.n;
      tab[c] = sdq::HmcChain{const_cast<double*>(a.field), phi0 + off, pm + off, mom + off, gp[c * nf], len};
      off += (size_t)len;
    }
  }
  HIP_TRY(grow(ctx->d_htab, (size_t)count * sizeof(sdq::HmcChain)), "hipMalloc(hmc table)");
  // stream-ordered after the previous trajectory's kernels read the table;
  // the source is pageable, so it may be reused once this returns
  HIP_TRY(hipMemcpyAsync(ctx->d_htab.p, tab.data(), (size_t)count * sizeof(sdq::HmcChain),
                         hipMemcpyHostToDevice, ctx->stream),
          "hipMemcpyAsync(hmc table)");
  const auto* d_tab = (const sdq::HmcChain*)ctx->d_htab.p;
  const int per = (int)std::max<int64_t>(1, std::min<int64_t>((lmax + 255) / 256,
                                                               (4LL * ctx->num_cu + count - 1) / count));
  ctx->err.clear();
  st = timed(ctx, "hmc", [&] { return sdq::launch_hmc_begin(count, d_tab, inv_var, e0, ctx->stream); });
  if (st) return st;
  // leapfrog: half kick, then (drift, kick) nsteps times with the last kick
  // halved; the force needs the gradient at every field on the way
  for (int e = 0; e < n_eval; ++e) {
    const bool first = e == 0, last = e == nsteps;
    st = sdq_logdet_grad(ctx, 0, inst, total, gp.data(), first ? ld0 : last ? ld1 : nullptr,
                         first ? sg0 : last ? sg1 : nullptr, st_all + (size_t)e * total);
    if (st) return st;
    if (last) break;
    const double kick = first ? 0.5 * eps : eps;
    for (int c0 = 0; c0 < count; c0 += 65535) {
      const int cn = std::min(count - c0, 65535);
      st = timed(ctx, "hmc", [&] {
        return sdq::launch_hmc_step(cn, nf, d_tab + c0, kick, eps, inv_var, per, ctx->stream);
      });
      if (st) return st;
    }
  }
  sdq::HmcEnd a{e0, ld0, sg0, ld1, sg1, st_all, n_eval, u, logdet, sign, accept, dH, status};
  return timed(ctx, "hmc", [&] {
    return sdq::launch_hmc_end(count, nf, d_tab, 0.5 * eps, inv_var, a, ctx->stream);
  });
}

sdq_status sdq_set_stabilizer(sdq_ctx* ctx, int32_t stab) {
  if (!ctx) return SDQ_EINVAL;
  if (stab != SDQ_STAB_QR && stab != SDQ_STAB_SVD) return fail(ctx, SDQ_EINVAL, "unknown stabilizer");
  ctx->stab = stab;
  return SDQ_OK;
}

sdq_status sdq_similarity(sdq_ctx* ctx, int32_t n, int32_t count, const double* left,
                          const double* right, double* const* mats) {
  SDQ_API_RANGE("sdq_similarity");
  if (!ctx) return SDQ_EINVAL;
  if (n < 1 || count < 0) return fail(ctx, SDQ_EINVAL, "bad n or count");
  if (n > 16 * sdq::kMaxNT) return fail(ctx, SDQ_EUNSUPPORTED, "sdq_similarity supports n <= 128");
  if (count == 0) return SDQ_OK;
  if (!left || !right || !mats) return fail(ctx, SDQ_EINVAL, "null pointer");
  for (int i = 0; i < count; ++i)
    if (!mats[i]) return fail(ctx, SDQ_EINVAL, "mats entry is NULL");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  ctx->err.clear();
  HIP_TRY(grow(ctx->d_ptrs, (size_t)count * sizeof(double*)), "hipMalloc(pointer table)");
  // stream-ordered after any earlier launch that read the table; the source
  // is pageable, so it may be reused once this returns
  HIP_TRY(hipMemcpyAsync(ctx->d_ptrs.p, mats, (size_t)count * sizeof(double*), hipMemcpyHostToDevice,
                         ctx->stream),
          "hipMemcpyAsync(pointer table)");
  const int nt = nt_of(n);
  const int grid = std::min(count, ctx->num_cu * 4);
  return timed(ctx, "similarity", [&] {
    return sdq::launch_similarity(nt, n, count, (double* const*)ctx->d_ptrs.p, left, right, grid,
                                  ctx->stream);
  });
}

sdq_status sdq_chain_udt(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, double* u,
                         double* d, double* t) {
  SDQ_API_RANGE("sdq_chain_udt");
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
    P.sweep.push_back(SweepItem{i, sdq::SW_FINAL, 0, 0});
  }
  order_items(P.inst, P.sweep, P.sweep_ranges, [&](const SweepItem& w) {
    const Inst& I = P.inst[w.inst];
    return sweep_cost(I.n, I.m, I.k);
  });
  ctx->err.clear();
  return run_plan(ctx, P, nullptr, 0);
}

// Autotuner: for each n, time sdq_logdet on a synthetic batch (two chains
// per CU, m = 40, k = 10, a periodic ring's second-order slice exponential,
// +-1 field) for every sweep variant (operand in LDS or HBM) and grid shape
// (one workgroup per CU or the occupancy limit), keep the fastest.  Results
// are cached as JSON lines {"arch", "n", "variant", "blocks_per_cu", "ms"}.
sdq_status sdq_tune(sdq_ctx* ctx, const int32_t* n_list, int32_t count, const char* cache_path) {
  SDQ_API_RANGE("sdq_tune");
  if (!ctx) return SDQ_EINVAL;
  if (count < 0 || (count > 0 && !n_list)) return fail(ctx, SDQ_EINVAL, "bad n_list");
  for (int a = 0; a < count; ++a)
    if (n_list[a] < 1 || n_list[a] > sdq::kGangMaxN) return fail(ctx, SDQ_EUNSUPPORTED, "n out of range");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, ctx->device), "hipGetDeviceProperties");
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  std::map<int, Tune> cached;
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char line[512];
      while (fgets(line, sizeof line, f)) {
        char a[64] = {0};
        int n = 0, v = 0, b = 0;
        if (sscanf(line, " {\"arch\": \"%63[^\"]\", \"n\": %d, \"variant\": %d, \"blocks_per_cu\": %d", a, &n, &v,
                   &b) == 4 &&
            arch == a)
          cached[n] = Tune{v, b};
      }
      fclose(f);
    }
  }
  const bool saved_graphs = ctx->graphs, saved_prof = ctx->profiling;
  ctx->graphs = false;
  ctx->profiling = false;
  sdq_status result = SDQ_OK;
  for (int a = 0; a < count && result == SDQ_OK; ++a) {
    const int n = n_list[a], nt = nt_of(n);
    if (is_gang(nt)) continue;  // one gang kernel per size: nothing to choose
    auto hit = cached.find(n);
    if (hit != cached.end()) {
      ctx->tune[nt] = hit->second;
      continue;
    }
    const int m = 40, k = 10, chains = 2 * ctx->num_cu;
    std::vector<double> E((size_t)n * n, 0.0), K((size_t)n * n, 0.0), F((size_t)chains * m * n);
    for (int i = 0; i < n; ++i) {
      K[(size_t)i * n + (i + 1) % n] -= 1.0;
      K[(size_t)((i + 1) % n) * n + i] -= 1.0;
    }
    const double dt = 0.1;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double k2 = 0.0;
        for (int q = 0; q < n; ++q) k2 += K[(size_t)i * n + q] * K[(size_t)q * n + j];
        E[(size_t)i * n + j] = (i == j ? 1.0 : 0.0) - dt * K[(size_t)i * n + j] + 0.5 * dt * dt * k2;
      }
    uint64_t x = 0x9E3779B97F4A7C15ull + n;
    for (double& v : F) {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      v = (x & 1) ? 1.0 : -1.0;
    }
    double *dE = nullptr, *dF = nullptr, *dL = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
      if (dE) (void)hipFree(dE);
      if (dF) (void)hipFree(dF);
      if (dL) (void)hipFree(dL);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&dE, E.size() * 8) != hipSuccess || hipMalloc(&dF, F.size() * 8) != hipSuccess ||
        hipMalloc(&dL, (size_t)chains * 16) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
      cleanup();
      result = fail(ctx, SDQ_ENOMEM, "tune: device allocation failed");
      break;
    }
    (void)hipMemcpy(dE, E.data(), E.size() * 8, hipMemcpyHostToDevice);
    (void)hipMemcpy(dF, F.data(), F.size() * 8, hipMemcpyHostToDevice);
    std::vector<sdq_instance> inst(chains);
    for (int c = 0; c < chains; ++c)
      inst[c] = sdq_instance{n, m, k, 0, dE, nullptr, dF + (size_t)c * m * n, 0.65};
    // the sweep variants (exponential in LDS or HBM; T in registers with
    // min(nt, 4) waves, or in scratch with one wave per tile) and the
    // occupancy cap (one workgroup per CU, or the kernel's limit)
    std::vector<Tune> cands;
    const bool lds = nt >= 3 && nt <= 5;
    for (int v : {0, 1, 4, 5})
      if ((v != 1 && v != 5) || lds)
        for (int b : {1, 0}) cands.push_back(Tune{v, b});
    double best = 1e300;
    Tune bt = ctx->tune[nt];
    for (const Tune& c : cands) {
      ctx->tune[nt] = c;
      double tmin = 1e300;
      for (int rep = 0; rep < 4 && result == SDQ_OK; ++rep) {
        (void)hipEventRecord(e0, ctx->stream);
        result = sdq_logdet(ctx, inst.data(), chains, dL, dL + chains, nullptr, nullptr);
        (void)hipEventRecord(e1, ctx->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) tmin = std::min(tmin, (double)ms);
      }
      if (result != SDQ_OK) break;
      if (tmin < best) {
        best = tmin;
        bt = c;
      }
    }
    cleanup();
    ctx->tune[nt] = bt;
    if (result == SDQ_OK && cache_path) {
      if (FILE* f = fopen(cache_path, "a")) {
        fprintf(f, "{\"arch\": \"%s\", \"n\": %d, \"variant\": %d, \"blocks_per_cu\": %d, \"ms\": %.4f}\n",
                arch.c_str(), n, bt.variant, bt.blocks_per_cu, best);
        fclose(f);
      }
    }
  }
  ctx->graphs = saved_graphs;
  ctx->profiling = saved_prof;
  return result;
}

sdq_status sdq_set_graphs(sdq_ctx* ctx, int enable) {
  if (!ctx) return SDQ_EINVAL;
  ctx->graphs = enable != 0;
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
  const std::string want(name), pre = want + "/";
  int64_t nl = 0;
  double tot = 0.0;
  for (auto& kv : ctx->stats) {
    if (kv.first != want && kv.first.compare(0, pre.size(), pre) != 0) continue;
    KStat& k = kv.second;
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
    nl += k.launches;
    tot += k.ms;
  }
  if (launches) *launches = nl;
  if (ms) *ms = tot;
  return SDQ_OK;
}

sdq_status sdq_kernel_names(sdq_ctx* ctx, char* buf, int32_t cap) {
  if (!ctx || !buf || cap < 1) return SDQ_EINVAL;
  std::string all;
  for (auto& kv : ctx->stats) {
    if (!all.empty()) all += ",";
    all += kv.first;
  }
  if ((int64_t)all.size() + 1 > cap) return fail(ctx, SDQ_EINVAL, "buffer too small for the kernel names");
  memcpy(buf, all.c_str(), all.size() + 1);
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
