// sdq_gang.hip -- chains with 128 < n <= 1024 on gfx950.
//
// An n x n FP64 matrix of such a chain no longer fits one CU (n = 256 is
// 512 KiB, the whole register file), so a chain is owned by a gang of G
// workgroups of 1024 threads.  Member g keeps the column slab
// [g*w, (g+1)*w) of the working matrix in LDS (column-major, leading
// dimension ldr = npad + 4); the geometry comes from gang_geom().  What the
// members must share goes through a per-gang scratch area in HBM:
//   * slice products W <- E diag(v) W (Sec. 4.1) are slab-local: each member
//     multiplies its own columns on FP64 MFMA with E read from the swizzled,
//     zero-padded copy in HBM (it stays in L2: all members and chains of one
//     size read the same copy);
//   * the column-pivoted Householder QR (Sec. 4.2.2) is distributed by
//     columns.  At every step each member publishes its live column of
//     largest downdated norm (rows below the step) with a pivot key; after
//     one gang barrier every wave of every member reads the winning column
//     and builds the same reflector from it (identical data, identical
//     reduction order: bitwise-identical results), then applies it to its
//     own live columns and downdates their norms.  Columns never move: the
//     step at which a column was chosen is remembered instead;
//   * R P^T and the reflectors are then written to HBM, and every later
//     operation that needs whole rows (T update, Q formation, Q^T
//     application, triangular solve, the time-displaced and gradient
//     products) reads them from there.
// Inside a QR step the candidates go through device-scope atomic stores and
// loads, and the published keys (tagged with the step) are the barrier:
// every wave polls the G keys until all carry the current tag.  Bulk data
// (R P^T, reflectors, G) is exchanged with normal stores behind a barrier on
// a monotonic counter in HBM with device-scope fences.  The grid never holds
// more workgroups than the device keeps resident at once (gang_capacity), so
// every member of every gang becomes resident, at the latest when kernels of
// other streams sharing the device have drained their workgroups; the launch
// is an ordinary one, so it can be captured in a HIP graph and overlap the
// one-workgroup kernels of other size classes.  A wait gives up after a few
// seconds (abort flag, status SDQ_ERANGE) instead of spinning forever.
//
// Paper passages: slice products and stage loop Sec. 4.1; pivoted QR and
// UDT Sec. 4.2.2; equal-time inversion Sec. 5.1 (Loh's split, mirror form);
// time-displaced inversion Sec. 6.1 (inv_sum_loh) and propagation Sec. 6;
// gradient App. A.1 with the wrap G_{l+1} = B_l G_l B_l^{-1} of Sec. 6.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sdq_internal.h"

namespace sdq {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = kGangThreads / 64;  // 16
constexpr int kPairs = 5;                  // MFMA output tiles per wave in a slab product
constexpr unsigned long long kSpinTicks = 400000000ull;  // 4 s of the 100 MHz wall clock
// The first rendezvous of a gang waits for all of its members to start.
// Other kernels of the same call (size classes on side streams) may hold
// the CUs a member needs until they finish, so this one wait is allowed
// far longer (60 s) than the waits inside a factorization, which only ever
// wait for members that are already running.
constexpr unsigned long long kAssembleTicks = 6000000000ull;

struct GLds {
  double S[kGangSlab];       // column slab, [col][row]
  double tau[kGangMaxN];     // reflector scalars; also a slice's exp(alpha f)
  double beta[kGangMaxN];    // diag R of the last QR (D = |beta|)
  int piv[kGangMaxN];        // piv[p] = global column chosen at step p
  double vn1[kGangMaxW], vn2[kGangMaxW];
  int posl[kGangMaxW];       // step at which a slab column was chosen; -1 live, -2 padding
  unsigned long long wkey[kWaves];
  double red[2 * kWaves];
  unsigned vis[kGangMaxN / 32];
  int ok;
};

// The workgroup's LDS block.  Declared at namespace scope (not passed by
// reference) so that every access is compiled as an LDS access.
__shared__ GLds L;

// one workgroup's view of its gang
struct GC {
  GangGeom geo;
  int n;        // matrix size of the current item
  int gang;     // gang index
  int g;        // member index
  int c0;       // first global column of the slab
  int t, w, l;  // thread, wave, lane
  double* base; // per-gang scratch
  unsigned* bar;
  unsigned epoch;
  bool ok;
};

__device__ __forceinline__ double* sc_R(const GC& c) { return c.base; }
__device__ __forceinline__ double* sc_V(const GC& c) { return c.base + gang_mat(c.geo); }
__device__ __forceinline__ double* sc_T(const GC& c) { return c.base + 2 * gang_mat(c.geo); }
__device__ __forceinline__ double* sc_U(const GC& c) { return c.base + 3 * gang_mat(c.geo); }
__device__ __forceinline__ double* sc_G(const GC& c, int b) { return c.base + (4 + b) * gang_mat(c.geo); }
__device__ __forceinline__ double* sc_X(const GC& c) { return c.base + 6 * gang_mat(c.geo); }
__device__ __forceinline__ double* sc_cand(const GC& c, int buf) {
  return c.base + 7 * gang_mat(c.geo) + (int64_t)buf * c.geo.G * gang_cand_stride(c.geo);
}

// ---- wave reductions ----------------------------------------------------------
// A butterfly in which each step combines a lane with a partner that
// combines it back (lane^1, lane^2 by quad permutation, the mirror inside 8
// and inside 16 lanes by DPP, then whole 16-lane rows with v_permlane16_swap
// and v_permlane32_swap): every lane adds the same two values, so all 64
// lanes, and every wave given the same data, get bitwise-identical results,
// which the redundant reflector computation of the gang QR relies on.  No
// LDS traffic.
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xf, 0xf, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ unsigned long long bits(double x) { return (unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ double dbl(unsigned long long b) { return __longlong_as_double((long long)b); }

// Combine 16-lane rows r and r^1 (R32 = false) or r and r^2 (R32 = true).
// v_permlane{16,32}_swap with both operands v returns the even row's value
// in its first result and the odd row's in its second, in both rows; both
// rows then apply op(even, odd) in the same order.
template <bool R32, class OP>
__device__ __forceinline__ unsigned long long pair_rows(unsigned long long v, OP op) {
  const unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  unsigned e0, e1, o0, o1;
  if constexpr (R32) {
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    e0 = a[0]; o0 = a[1]; e1 = b[0]; o1 = b[1];
  } else {
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    e0 = a[0]; o0 = a[1]; e1 = b[0]; o1 = b[1];
  }
  return op(((unsigned long long)e1 << 32) | e0, ((unsigned long long)o1 << 32) | o0);
}

template <class OP>
__device__ __forceinline__ unsigned long long wave_reduce(unsigned long long v, OP op) {
  v = op(v, dpp64<0xB1>(v));   // quad_perm [1,0,3,2]
  v = op(v, dpp64<0x4E>(v));   // quad_perm [2,3,0,1]
  v = op(v, dpp64<0x141>(v));  // row_half_mirror
  v = op(v, dpp64<0x140>(v));  // row_mirror
  v = pair_rows<false>(v, op);
  v = pair_rows<true>(v, op);
  return v;
}
// op(a, b) must be commutative in its bits: a + b, max
__device__ __forceinline__ double wave_sum(double v) {
  return dbl(wave_reduce(bits(v), [](unsigned long long a, unsigned long long b) { return bits(dbl(a) + dbl(b)); }));
}
__device__ __forceinline__ double wave_max(double v) {
  return dbl(wave_reduce(bits(v), [](unsigned long long a, unsigned long long b) { return bits(fmax(dbl(a), dbl(b))); }));
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  return wave_reduce(v, [](unsigned long long a, unsigned long long b) { return a > b ? a : b; });
}
__device__ __forceinline__ double pow2_scale(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 1.0;
  return ldexp(1.0, -ilogb(x));
}

// Pivot key: bits 63..16 the norm's top 48 bits, bits 15..11 a step tag,
// bits 10..0 2047 - column.  Among keys of one step the largest norm wins
// and, among norms equal to 2^-36 relative, the smallest column.  A member
// with no live column publishes the tag alone.
__device__ __forceinline__ unsigned long long pivot_key(double norm, int col) {
  double x = norm >= 0.0 ? norm : 0.0;  // NaN -> 0
  x = x < 1.0e300 ? x : 1.0e300;
  return ((unsigned long long)__double_as_longlong(x) & ~0xFFFFull) | (unsigned long long)(2047 - col);
}
__device__ __forceinline__ int key_col(unsigned long long k) { return 2047 - (int)(k & 0x7FF); }
__device__ __forceinline__ unsigned long long tag_key(unsigned long long k, int p) {
  return (k & ~0xF800ull) | ((unsigned long long)(p & 31) << 11);
}
__device__ __forceinline__ int key_tag(unsigned long long k) { return (int)((k >> 11) & 31); }

// Device memory seen as the global address space: accesses through these
// compile to global instructions (flat ones would also count against LDS
// waits and be ordered against the spill slots).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// ---- gang barrier ----------------------------------------------------------
__device__ bool gang_sync(GC& c) {
  __syncthreads();
  c.epoch += 1;
  if (c.t == 0) {
    __threadfence();
    const unsigned target = c.epoch * (unsigned)c.geo.G;
    __hip_atomic_fetch_add(gmem(&c.bar[0]), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    const unsigned long long t0 = wall_clock64();
    for (;;) {
      const unsigned v = __hip_atomic_load(gmem(&c.bar[0]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v >= target) break;
      if (__hip_atomic_load(gmem(&c.bar[1]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        good = 0;
        break;
      }
      if (wall_clock64() - t0 > kSpinTicks) {
        __hip_atomic_exchange(gmem(&c.bar[1]), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    L.ok = good;
  }
  __syncthreads();
  const bool good = L.ok != 0;
  c.ok = c.ok && good;
  return good;
}

// Start of a gang's work: every member counts itself in (word 2 of the
// barrier record) and waits until all G have, or until another member gave
// up, or kAssembleTicks.  After it every member is resident, so the bounded
// waits of gang_sync and wait_keys measure work, not scheduling.
__device__ void gang_assemble(GC& c) {
  if (c.t == 0) {
    __hip_atomic_fetch_add(gmem(&c.bar[2]), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    const unsigned long long t0 = wall_clock64();
    for (;;) {
      if (__hip_atomic_load(gmem(&c.bar[2]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (unsigned)c.geo.G)
        break;
      if (__hip_atomic_load(gmem(&c.bar[1]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        good = 0;
        break;
      }
      if (wall_clock64() - t0 > kAssembleTicks) {
        __hip_atomic_exchange(gmem(&c.bar[1]), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
    L.ok = good;
  }
  __syncthreads();
  c.ok = c.ok && L.ok != 0;
  __syncthreads();
}

// Data exchanged between members inside a QR step goes through device-scope
// atomic stores and loads: they are performed at the device coherence point,
// so no cache write-back or invalidation is needed (see wait_keys).
__device__ __forceinline__ void st_coh(double* p, double x) {
  __hip_atomic_store(gmem(p), x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Row p and rows lane + 64 s (s < RL) of a column published by another
// member: device-scope coherent loads (the system-coherence bit, which is
// what a relaxed device-scope atomic load is on this target) through a
// buffer resource, all issued before any is used.  As atomic loads the
// compiler waits for each one before issuing the next, which costs one
// memory round trip per row slot.  col is wave-uniform; entries past npad
// read as zero.
template <int RL>
__device__ __forceinline__ void ld_coh_col(const double* col, int npad, int l, int p, double& at_p,
                                           double (&x)[RL]) {
  constexpr int kCohSys = 16;  // cache policy: system-coherent scope
  const unsigned long long a = (unsigned long long)col;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(((unsigned long long)hi << 32) | lo), (short)0, npad * 8, 0x00020000);
  at_p = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, p * 8, 0, kCohSys));
#pragma unroll
  for (int s = 0; s < RL; ++s)
    x[s] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (l + 64 * s) * 8, 0, kCohSys));
}
__device__ __forceinline__ void st_coh_u64(double* p, unsigned long long x) {
  __hip_atomic_store(gmem((unsigned long long*)p), x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_coh_u64(const double* p) {
  return __hip_atomic_load(gmem((unsigned long long*)const_cast<double*>(p)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ---- slab products -----------------------------------------------------------
// S[:, slab] <- post(i) * sum_k A(i, k) pre(k) S[k, slab] on FP64 MFMA
// 16x16x4.  A(ti, tk, r, l) returns the left operand entry
// (16 ti + l%16, 16 tk + 4 r + l/16) for lane l.  Output tiles (ti, ct)
// are spread over the 16 waves; ends with a barrier.
template <class AF, class PRE, class POST>
__device__ void slab_gemm(GC& c_in, AF A, PRE pre, POST post) {
  // a register copy of the context (these functions are not always inlined,
  // and through the reference every field read would be a memory load)
  const GC c = c_in;
  const int nrt = c.geo.npad / 16, nct = c.geo.w / 16, np = nrt * nct, ldr = c.geo.ldr;
  int ti[kPairs], ct[kPairs];
  bool on[kPairs];
  d4 acc[kPairs];
#pragma unroll
  for (int s = 0; s < kPairs; ++s) {
    const int idx = c.w + kWaves * s;
    on[s] = idx < np;
    ct[s] = on[s] ? idx / nrt : 0;
    ti[s] = on[s] ? idx - ct[s] * nrt : 0;
    acc[s] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const int lq = c.l >> 4, lc = c.l & 15;
  if (on[0]) {
    for (int tk = 0; tk < nrt; ++tk) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kk = 16 * tk + 4 * r + lq;
        const double pk = pre(kk);
        double a = 0.0;
#pragma unroll
        for (int s = 0; s < kPairs; ++s) {
          if (!on[s]) continue;
          if (s == 0 || ti[s] != ti[s - 1]) a = A(ti[s], tk, r, c.l);
          const double b = L.S[(16 * ct[s] + lc) * ldr + kk] * pk;
          acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kPairs; ++s) {
    if (!on[s]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * ti[s] + lq + 4 * r;
      L.S[(16 * ct[s] + lc) * ldr + row] = acc[s][r] * post(row);
    }
  }
  __syncthreads();
}

struct One {
  __device__ double operator()(int) const { return 1.0; }
};

// left operands
struct ASwz {  // swizzled zero-padded copy (launch_swizzle order)
  const double* e;
  int nt;
  __device__ double operator()(int ti, int tk, int r, int l) const {
    return gmem(e)[((int64_t)(ti * nt + tk) * 4 + r) * 64 + l];
  }
};
struct AColMajor {  // A[i][k] = M[k*ld + i], buffer zero padded to ld x ld
  const double* M;
  int ld;
  __device__ double operator()(int ti, int tk, int r, int l) const {
    return gmem(M)[(int64_t)(16 * tk + 4 * r + (l >> 4)) * ld + 16 * ti + (l & 15)];
  }
};
// A[i][k] = M[i*n + k] * cs(k) (row-major n x n, M not null).  Device
// memory operands are loaded unconditionally from clamped in-range
// addresses and the padding is selected away afterwards: a load behind a
// per-entry branch would be waited for before the next one.
template <class CS>
struct ARowMajor {
  const double* M;
  int n;
  CS cs;
  __device__ double operator()(int ti, int tk, int r, int l) const {
    const int i = 16 * ti + (l & 15), k = 16 * tk + 4 * r + (l >> 4);
    const int kc = min(k, n - 1);
    const double x = gmem(M)[(int64_t)min(i, n - 1) * n + kc] * cs(kc);
    return (i < n && k < n) ? x : 0.0;
  }
};
// A[i][k] = M[k*n + i] (the transpose of a row-major n x n matrix, not null)
struct ARowMajorT {
  const double* M;
  int n;
  __device__ double operator()(int ti, int tk, int r, int l) const {
    const int i = 16 * ti + (l & 15), k = 16 * tk + 4 * r + (l >> 4);
    const double x = gmem(M)[(int64_t)min(k, n - 1) * n + min(i, n - 1)];
    return (i < n && k < n) ? x : 0.0;
  }
};
// A[i][k] = (i == k) cs(k) for i, k < n: the stand-in for a null M
template <class CS>
struct AIdent {
  int n;
  CS cs;
  __device__ double operator()(int ti, int tk, int r, int l) const {
    const int i = 16 * ti + (l & 15), k = 16 * tk + 4 * r + (l >> 4);
    return (i == k && i < n) ? cs(k) : 0.0;
  }
};
// the LDS vector L.beta as a column or row scale
struct BetaScale {
  __device__ double operator()(int k) const { return L.beta[k]; }
};

// ---- slab loads and stores ---------------------------------------------------
// Slab loads and stores end with a barrier (their thread mapping differs
// from that of the next writer of the slab).
// S[cc][i] = f(i, gc) for every slab entry (zero outside n x n); row-wise so
// that consecutive threads take consecutive columns of one row
// f is evaluated at clamped indices (i, gc < n) for every entry, eight per
// thread at a time before any is stored, so that its loads are in flight
// together; entries outside n x n are stored as zero.
template <bool ROWS, class F, class OP>
__device__ void slab_for_each(GC& c, F f, OP op) {
  const int w = c.geo.w, np = c.geo.npad, ldr = c.geo.ldr, n = c.n, tot = np * w;
  constexpr int CH = 8;
  for (int b = c.t; b < tot; b += CH * kGangThreads) {
    double x[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int idx = min(b + q * kGangThreads, tot - 1);
      const int i = ROWS ? idx / w : idx % np, cc = ROWS ? idx - i * w : idx / np;
      x[q] = f(min(i, n - 1), min(c.c0 + cc, n - 1));
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int idx = b + q * kGangThreads;
      if (idx >= tot) continue;
      const int i = ROWS ? idx / w : idx % np, cc = ROWS ? idx - i * w : idx / np;
      op(L.S[cc * ldr + i], i < n && c.c0 + cc < n, x[q]);
    }
  }
  __syncthreads();
}
struct SetOrZero {
  __device__ void operator()(double& e, bool in, double x) const { e = in ? x : 0.0; }
};
struct AddInside {
  __device__ void operator()(double& e, bool in, double x) const {
    if (in) e += x;
  }
};
struct MulInside {
  __device__ void operator()(double& e, bool in, double x) const {
    if (in) e *= x;
  }
};
struct SetInside {
  __device__ void operator()(double& e, bool in, double x) const {
    if (in) e = x;
  }
};
template <class F>
__device__ void slab_fill_rows(GC& c, F f) {
  slab_for_each<true>(c, f, SetOrZero{});
}
// the same, column-wise (consecutive threads take consecutive rows)
template <class F>
__device__ void slab_fill_cols(GC& c, F f) {
  slab_for_each<false>(c, f, SetOrZero{});
}
// dst[i*n + gc] = S[cc][i] for the leading n x n block
__device__ void slab_store_rowmajor(GC& c, double* dst) {
  const int w = c.geo.w, ldr = c.geo.ldr, n = c.n;
  for (int idx = c.t; idx < n * w; idx += kGangThreads) {
    const int i = idx / w, cc = idx - i * w, gc = c.c0 + cc;
    if (gc < n) gmem(dst)[(int64_t)i * n + gc] = L.S[cc * ldr + i];
  }
  __syncthreads();
}
// dst[piv[q]*n + gc] = S[cc][q]
__device__ void slab_store_rowmajor_perm(GC& c, double* dst) {
  const int w = c.geo.w, ldr = c.geo.ldr, n = c.n;
  for (int idx = c.t; idx < n * w; idx += kGangThreads) {
    const int q = idx / w, cc = idx - q * w, gc = c.c0 + cc;
    int row = L.piv[q];
    row = row < 0 ? 0 : (row >= n ? n - 1 : row);
    if (gc < n) gmem(dst)[(int64_t)row * n + gc] = L.S[cc * ldr + q];
  }
  __syncthreads();
}
// dst[gc*npad + i] = S[cc][i], whole padded slab
__device__ void slab_store_colmajor(GC& c, double* dst) {
  const int np = c.geo.npad, ldr = c.geo.ldr;
  for (int idx = c.t; idx < np * c.geo.w; idx += kGangThreads) {
    const int cc = idx / np, i = idx - cc * np;
    const int gc = c.c0 + cc;
    if (gc < np) gmem(dst)[(int64_t)gc * np + i] = L.S[cc * ldr + i];
  }
  __syncthreads();
}
__device__ void slab_identity(GC& c) {
  slab_fill_cols(c, [](int i, int gc) { return i == gc ? 1.0 : 0.0; });
}

// ---- column-pivoted QR of the gang's matrix --------------------------------
// Publish this member's best live column (rows p..n-1) and its key into
// candidate buffer p & 1.
template <int RL>
__device__ void publish_candidate(GC& c, int p) {
  unsigned long long best = 0;
  for (int cc = c.w; cc < c.geo.w; cc += kWaves)
    if (L.posl[cc] == -1) {
      const unsigned long long k = pivot_key(L.vn1[cc], c.c0 + cc);
      best = k > best ? k : best;
    }
  if (c.l == 0) L.wkey[c.w] = best;
  __syncthreads();
  if (c.w == 0) {
    unsigned long long k = c.l < kWaves ? L.wkey[c.l] : 0ull;
    k = wave_max_u64(k);
    double* out = sc_cand(c, p & 1) + (int64_t)c.g * gang_cand_stride(c.geo);
    if (k != 0ull) {
      int cc = key_col(k) - c.c0;
      cc = cc < 0 ? 0 : (cc >= c.geo.w ? c.geo.w - 1 : cc);
      const double* col = L.S + cc * c.geo.ldr;
      if constexpr (RL <= 4) {
        // all of the lane's rows read from LDS before any is stored (with
        // more rows per lane the registers this takes cost more than the
        // LDS waits it saves)
        double x[RL];
#pragma unroll
        for (int s = 0; s < RL; ++s) x[s] = col[min(c.l + 64 * s, c.geo.npad - 1)];
#pragma unroll
        for (int s = 0; s < RL; ++s) {
          const int i = c.l + 64 * s;
          if (i >= p && i < c.n) st_coh(out + i, x[s]);
        }
      } else {
        for (int i = p + c.l; i < c.n; i += 64) st_coh(out + i, col[i]);
      }
    }
    // the column is complete at the coherence point before its key appears
    __builtin_amdgcn_s_waitcnt(0);
    if (c.l == 0) st_coh_u64(out + c.geo.npad, tag_key(k, p));
  }
}

// Every wave waits until all G keys of step p carry its tag (the keys are
// both the data and the barrier of a QR step) and returns the largest.  On a
// timeout, or when another member has given up, the gang is marked broken
// and the (meaningless) current maximum is returned; later waits return at
// once.
__device__ unsigned long long wait_keys(GC& c, const double* cb, int p) {
  const int G = c.geo.G;
  const int64_t stride = gang_cand_stride(c.geo);
  const unsigned long long t0 = wall_clock64();
  for (;;) {
    unsigned long long k = 0ull;
    bool here = true;
    if (c.l < G) {
      k = ld_coh_u64(cb + (int64_t)c.l * stride + c.geo.npad);
      here = key_tag(k) == (p & 31);
    }
    if (__all(here) || !c.ok) return wave_max_u64(k);
    const bool abort = __hip_atomic_load(gmem(&c.bar[1]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    if (abort || wall_clock64() - t0 > kSpinTicks) {
      if (!abort && c.l == 0)
        __hip_atomic_exchange(gmem(&c.bar[1]), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      c.ok = false;
      return wave_max_u64(k);
    }
  }
}

// scaled 2-norm of rows [lo, n) of one LDS column, by one wave
__device__ double col_norm(const double* col, int lo, int n, int l) {
  double am = 0.0;
  for (int i = lo + l; i < n; i += 64) am = fmax(am, fabs(col[i]));
  am = wave_max(am);
  if (!(am > 0.0)) return 0.0;
  const double sc = pow2_scale(am);
  double ss = 0.0;
  for (int i = lo + l; i < n; i += 64) {
    const double x = col[i] * sc;
    ss += x * x;
  }
  return sqrt(wave_sum(ss)) / sc;
}

// On return: L.tau / L.beta / L.piv hold the reflector scalars, diag R and
// the pivot order; sc_R = R P^T (column gc = R column of the step at which gc
// was chosen, rows above and on that step) and sc_V = the reflectors (column
// gc = reflector of that step, rows below it, unit entry implied), both
// column-major npad x npad, visible to the whole gang.
template <int kRL>
__device__ void cpqr_gang(GC& c_io) {
  GC c = c_io;  // register copy, written back at the end
  const int n = c.n, ldr = c.geo.ldr;
  const double tol3z = 1.4901161193847656e-08;  // sqrt(2^-52)
  // Reset this member's two key slots to tag 31 (the slots may hold keys of
  // an earlier QR or launch whose tags would match steps 0 and 1; tag 31 is
  // not expected before step 31, when both slots hold this QR's keys), and
  // make the resets visible to the gang before any step's keys are polled.
  if (c.t == 0) {
    const int64_t st = gang_cand_stride(c.geo);
    st_coh_u64(sc_cand(c, 0) + (int64_t)c.g * st + c.geo.npad, tag_key(0ull, 31));
    st_coh_u64(sc_cand(c, 1) + (int64_t)c.g * st + c.geo.npad, tag_key(0ull, 31));
  }
  gang_sync(c);
  for (int cc = c.w; cc < c.geo.w; cc += kWaves) {
    const int gc = c.c0 + cc;
    const double nrm = gc < n ? col_norm(L.S + cc * ldr, 0, n, c.l) : 0.0;
    if (c.l == 0) {
      L.vn1[cc] = nrm;
      L.vn2[cc] = nrm;
      L.posl[cc] = gc < n ? -1 : -2;
    }
  }
  __syncthreads();
  publish_candidate<kRL>(c, 0);
  const int nrl = (n + 63) / 64;
  for (int p = 0; p < n; ++p) {
    const double* cb = sc_cand(c, p & 1);
    const unsigned long long key = wait_keys(c, cb, p);
    int gw = key_col(key);
    gw = gw < 0 ? 0 : (gw >= n ? n - 1 : gw);
    const int owner = gw / c.geo.w;
    const double* xs = cb + (int64_t)owner * gang_cand_stride(c.geo);
    double v[kRL];  // the winner column below row p, then the reflector
    double am = 0.0;
    double al;
    ld_coh_col<kRL>(xs, c.geo.npad, c.l, p, al, v);
#pragma unroll
    for (int s = 0; s < kRL; ++s) {
      const int i = c.l + 64 * s;
      v[s] = (s < nrl && i > p && i < n) ? v[s] : 0.0;
      am = fmax(am, fabs(v[s]));
    }
    am = wave_max(am);
    double xnorm = 0.0;
    if (am > 0.0) {
      const double sc = pow2_scale(am);
      double ss = 0.0;
#pragma unroll
      for (int s = 0; s < kRL; ++s) {
        const int i = c.l + 64 * s;
        const double y = v[s] * sc;
        ss += y * y;
      }
      xnorm = sqrt(wave_sum(ss)) / sc;
    }
    double tau, beta, vsc;
    if (xnorm == 0.0) {
      tau = 0.0;
      beta = al;
      vsc = 0.0;
    } else {
      beta = -copysign(hypot(al, xnorm), al);
      tau = (beta - al) / beta;
      vsc = 1.0 / (al - beta);
    }
#pragma unroll
    for (int s = 0; s < kRL; ++s) {
      const int i = c.l + 64 * s;
      v[s] = i > p ? v[s] * vsc : (i == p ? 1.0 : 0.0);
    }
    if (c.t == 0) {
      L.tau[p] = tau;
      L.beta[p] = beta;
      L.piv[p] = gw;
    }
    for (int cc = c.w; cc < c.geo.w; cc += kWaves) {
      double* col = L.S + cc * ldr;
      if (c.c0 + cc == gw) {
#pragma unroll
        for (int s = 0; s < kRL; ++s) {
          const int i = c.l + 64 * s;
          if (s < nrl && i >= p && i < n) col[i] = i == p ? beta : v[s];
        }
        if (c.l == 0) L.posl[cc] = p;
        continue;
      }
      if (L.posl[cc] != -1) continue;
      double y[kRL];
#pragma unroll
      for (int s = 0; s < kRL; ++s) {
        const int i = c.l + 64 * s;
        y[s] = (s < nrl && i >= p && i < n) ? col[i] : 0.0;
      }
      if (tau != 0.0) {
        double d = 0.0;
#pragma unroll
        for (int s = 0; s < kRL; ++s) d += v[s] * y[s];
        const double tv = tau * wave_sum(d);
#pragma unroll
        for (int s = 0; s < kRL; ++s) {
          const int i = c.l + 64 * s;
          if (s < nrl && i >= p && i < n) {
            y[s] -= tv * v[s];
            col[i] = y[s];
          }
        }
      }
      const double rp = col[p];  // row p after the update (same wave wrote it)
      double n1 = L.vn1[cc], n2 = L.vn2[cc];
      if (n1 != 0.0) {
        double tmp = fabs(rp) / n1;
        tmp = fmax(0.0, (1.0 + tmp) * (1.0 - tmp));
        const double q = n1 / n2;
        if (tmp * q * q <= tol3z) {
          double bm = 0.0;
#pragma unroll
          for (int s = 0; s < kRL; ++s)
            if (c.l + 64 * s > p) bm = fmax(bm, fabs(y[s]));
          bm = wave_max(bm);
          double nn = 0.0;
          if (bm > 0.0) {
            const double sc = pow2_scale(bm);
            double ss = 0.0;
#pragma unroll
            for (int s = 0; s < kRL; ++s)
              if (c.l + 64 * s > p) {
                const double z = y[s] * sc;
                ss += z * z;
              }
            nn = sqrt(wave_sum(ss)) / sc;
          }
          n1 = nn;
          n2 = nn;
        } else {
          n1 *= sqrt(tmp);
        }
      }
      if (c.l == 0) {
        L.vn1[cc] = n1;
        L.vn2[cc] = n2;
      }
    }
    if (p + 1 < n) publish_candidate<kRL>(c, p + 1);
  }
  __syncthreads();
  // R P^T and the reflectors to HBM
  {
    const int np = c.geo.npad;
    double* R = sc_R(c);
    double* V = sc_V(c);
    for (int idx = c.t; idx < np * c.geo.w; idx += kGangThreads) {
      const int cc = idx / np, i = idx - cc * np, gc = c.c0 + cc;
      if (gc >= np) continue;
      const int sc = gc < n ? L.posl[cc] : -1;
      const double x = L.S[cc * ldr + i];
      gmem(R)[(int64_t)gc * np + i] = (gc < n && i <= sc) ? x : 0.0;
      gmem(V)[(int64_t)gc * np + i] = (gc < n && i > sc && i < n) ? x : 0.0;
    }
  }
  gang_sync(c);
  c_io = c;
}

// Row q of a column distributed over the wave (row i in lane i % 64, slot
// i / 64), broadcast to every lane; q is wave-uniform.
template <int RL>
__device__ __forceinline__ double row_of_col(const double (&y)[RL], int q) {
  const int slot = q >> 6;
  double x = y[0];
#pragma unroll
  for (int r = 1; r < RL; ++r) x = slot == r ? y[r] : x;
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), q & 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), q & 63);
  return __hiloint2double(hi, lo);
}

// Apply the reflectors of the last QR to the own columns of the slab:
// ascending (Q^T) or descending (Q; with identity_cols the columns start as
// unit vectors, and reflectors beyond the largest own column leave them
// unchanged).  Each wave holds its own columns in registers (up to 16 / kRL
// of them), reads each reflector once from sc_V (the next one while the
// current one is applied) and applies it to all of them.
template <bool ASC, int kRL>
__device__ void apply_reflectors(GC& c_in, bool identity_cols) {
  const GC c = c_in;  // register copy
  constexpr int CM = 16 / kRL;
  const int n = c.n, ldr = c.geo.ldr, np = c.geo.npad;
  const double* V = sc_V(c);
  const int nrl = (n + 63) / 64;
  for (int s0 = 0; c.w + kWaves * s0 < c.geo.w; s0 += CM) {
    double y[CM][kRL];
    int jmax = -1;
#pragma unroll
    for (int s = 0; s < CM; ++s) {
      const int cc = c.w + kWaves * (s0 + s), gc = c.c0 + cc;
      const bool on = cc < c.geo.w && gc < n;
      if (on) jmax = max(jmax, identity_cols ? gc : n - 1);
#pragma unroll
      for (int r = 0; r < kRL; ++r) {
        const int i = c.l + 64 * r;
        y[s][r] = (on && r < nrl && i < n) ? L.S[cc * ldr + i] : 0.0;
      }
    }
    auto load = [&](int j, double (&v)[kRL], double& t) {
      t = L.tau[j];
      int pc = L.piv[j];
      pc = pc < 0 ? 0 : (pc >= n ? n - 1 : pc);
      const double* vc = V + (int64_t)pc * np;
#pragma unroll
      for (int r = 0; r < kRL; ++r) {
        const int i = c.l + 64 * r;
        const double x = gmem(vc)[min(i, np - 1)];
        v[r] = (r < nrl && i > j && i < n) ? x : (i == j ? 1.0 : 0.0);
      }
    };
    double vn[kRL], tn = 0.0;
    if (jmax >= 0) load(ASC ? 0 : jmax, vn, tn);
    for (int jj = 0; jj <= jmax; ++jj) {
      double v[kRL];
#pragma unroll
      for (int r = 0; r < kRL; ++r) v[r] = vn[r];
      const double tj = tn;
      if (jj < jmax) load(ASC ? jj + 1 : jmax - jj - 1, vn, tn);
      if (tj == 0.0) continue;
      double d[CM];
#pragma unroll
      for (int s = 0; s < CM; ++s) {
        double a = 0.0;
#pragma unroll
        for (int r = 0; r < kRL; ++r) a = fma(v[r], y[s][r], a);
        d[s] = a;
      }
#pragma unroll
      for (int s = 0; s < CM; ++s) d[s] = tj * wave_sum(d[s]);
#pragma unroll
      for (int s = 0; s < CM; ++s)
#pragma unroll
        for (int r = 0; r < kRL; ++r) y[s][r] = fma(-d[s], v[r], y[s][r]);
    }
#pragma unroll
    for (int s = 0; s < CM; ++s) {
      const int cc = c.w + kWaves * (s0 + s), gc = c.c0 + cc;
      if (cc >= c.geo.w || gc >= n) continue;
#pragma unroll
      for (int r = 0; r < kRL; ++r) {
        const int i = c.l + 64 * r;
        if (r < nrl && i < n) L.S[cc * ldr + i] = y[s][r];
      }
    }
  }
  __syncthreads();
}

// S <- R^{-1} S (R upper triangular in pivot order: R[i][q] = sc_R[piv[q]][i]),
// own columns in registers as above, each column of R read once per wave.
template <int kRL>
__device__ void back_subst(GC& c_in) {
  const GC c = c_in;  // register copy
  constexpr int CM = 16 / kRL;
  const int n = c.n, ldr = c.geo.ldr, np = c.geo.npad;
  const double* R = sc_R(c);
  const int nrl = (n + 63) / 64;
  for (int s0 = 0; c.w + kWaves * s0 < c.geo.w; s0 += CM) {
    double y[CM][kRL];
#pragma unroll
    for (int s = 0; s < CM; ++s) {
      const int cc = c.w + kWaves * (s0 + s), gc = c.c0 + cc;
      const bool on = cc < c.geo.w && gc < n;
#pragma unroll
      for (int r = 0; r < kRL; ++r) {
        const int i = c.l + 64 * r;
        y[s][r] = (on && r < nrl && i < n) ? L.S[cc * ldr + i] : 0.0;
      }
    }
    auto load = [&](int q, double (&rv)[kRL]) {
      int pc = L.piv[q];
      pc = pc < 0 ? 0 : (pc >= n ? n - 1 : pc);
      const double* rc = R + (int64_t)pc * np;
#pragma unroll
      for (int r = 0; r < kRL; ++r) {
        const int i = c.l + 64 * r;
        const double x = gmem(rc)[min(i, np - 1)];
        rv[r] = (r < nrl && i < q) ? x : 0.0;
      }
    };
    double rn[kRL];
    load(n - 1, rn);
    for (int q = n - 1; q >= 0; --q) {
      double rv[kRL];
#pragma unroll
      for (int r = 0; r < kRL; ++r) rv[r] = rn[r];
      if (q > 0) load(q - 1, rn);
      const double rb = 1.0 / L.beta[q];
#pragma unroll
      for (int s = 0; s < CM; ++s) {
        const double xq = row_of_col<kRL>(y[s], q) * rb;
#pragma unroll
        for (int r = 0; r < kRL; ++r) {
          const int i = c.l + 64 * r;
          y[s][r] = i == q ? xq : fma(-rv[r], xq, y[s][r]);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < CM; ++s) {
      const int cc = c.w + kWaves * (s0 + s), gc = c.c0 + cc;
      if (cc >= c.geo.w || gc >= n) continue;
#pragma unroll
      for (int r = 0; r < kRL; ++r) {
        const int i = c.l + 64 * r;
        if (r < nrl && i < n) L.S[cc * ldr + i] = y[s][r];
      }
    }
  }
  __syncthreads();
}

// sign of the permutation piv (thread 0; cycle walk over a bitmap in LDS)
__device__ double perm_sign(GC& c) {
  const int n = c.n;
  for (int a = c.t; a < kGangMaxN / 32; a += kGangThreads) L.vis[a] = 0u;
  __syncthreads();
  if (c.t == 0) {
    int cycles = 0;
    for (int s = 0; s < n; ++s) {
      if (L.vis[s >> 5] & (1u << (s & 31))) continue;
      ++cycles;
      int x = s;
      for (int guard = 0; guard <= n; ++guard) {
        if (L.vis[x >> 5] & (1u << (x & 31))) break;
        L.vis[x >> 5] |= 1u << (x & 31);
        int nx = L.piv[x];
        x = nx < 0 ? 0 : (nx >= n ? n - 1 : nx);
      }
    }
    L.red[0] = ((n - cycles) & 1) ? -1.0 : 1.0;
  }
  __syncthreads();
  const double r = L.red[0];
  __syncthreads();
  return r;
}

// (-1)^(number of nontrivial reflectors) = det Q (wave reduction, every thread)
__device__ double refl_sign(GC& c) {
  double cnt = 0.0;
  for (int j = c.l; j < c.n; j += 64) cnt += L.tau[j] != 0.0 ? 1.0 : 0.0;
  cnt = wave_sum(cnt);
  return (((long long)cnt) & 1) ? -1.0 : 1.0;
}

// ---- stage loop ----------------------------------------------------------------
__device__ void load_slice_scale(GC& c, const Inst& I, int q) {
  const double* f = I.field + (int64_t)(q - 1) * I.n;
  for (int i = c.t; i < c.geo.npad; i += kGangThreads) L.tau[i] = i < c.n ? exp(I.alpha * gmem(f)[i]) : 0.0;
  __syncthreads();
}

// Stabilized chain (Sec. 4.1) with the UDT of Sec. 4.2.2 every k slices,
// forward over B_1..B_m or, with SW_ADJ, backward over B_m^T..B_1^T; stage
// storage as in the single-workgroup kernels (U | T | D | sgn det U).
template <int kRL>
__device__ void sweep_gang(GC& c, const Inst& I, int flags) {
  const int n = I.n, m = I.m, k = I.k, nb = I.nb, np = c.geo.npad;
  const bool adj = (flags & SW_ADJ) != 0;
  const int64_t sd = stage_doubles(n);
  double* Tg = sc_T(c);  // T of the chain, row-major n x n (own columns)
  slab_identity(c);
  for (int i = c.t; i < np; i += kGangThreads) L.beta[i] = 1.0;
  __syncthreads();
  slab_store_rowmajor(c, Tg);
  double sgn_u = 1.0;
  const ASwz aop{adj ? I.eswt : I.esw, np / 16};
  auto copy_t = [&](double* dst) {
    for (int idx = c.t; idx < n * c.geo.w; idx += kGangThreads) {
      const int i = idx / c.geo.w, gc = c.c0 + (idx - i * c.geo.w);
      if (gc < n) gmem(dst)[(int64_t)i * n + gc] = gmem(Tg)[(int64_t)i * n + gc];
    }
  };
  for (int s = 0; s < nb; ++s) {
    const int b = adj ? nb - 1 - s : s;
    const int q0 = b * k + 1, q1 = (b + 1) * k < m ? (b + 1) * k : m;
    // U D (column scale), then the block of slices
    for (int idx = c.t; idx < np * c.geo.w; idx += kGangThreads) {
      const int cc = idx / np, i = idx - cc * np, gc = c.c0 + cc;
      if (gc < n) L.S[cc * c.geo.ldr + i] *= fabs(L.beta[gc]);
    }
    __syncthreads();
    for (int qq = 0; qq <= q1 - q0; ++qq) {
      const int q = adj ? q1 - qq : q0 + qq;
      load_slice_scale(c, I, q);
      if (!adj)
        slab_gemm(c, aop, [&](int kk) { return L.tau[kk]; }, One{});
      else
        slab_gemm(c, aop, One{}, [&](int row) { return L.tau[row]; });
    }
    cpqr_gang<kRL>(c);
    // T <- D^{-1} R P^T T with D = |diag R|
    slab_fill_rows(c, [&](int i, int gc) { return gmem(Tg)[(int64_t)i * n + gc]; });
    __syncthreads();
    slab_gemm(c, AColMajor{sc_R(c), np}, One{},
              [&](int row) { return row < n ? 1.0 / fabs(L.beta[row]) : 0.0; });
    slab_store_rowmajor(c, Tg);
    sgn_u = refl_sign(c);
    // U <- Q
    slab_identity(c);
    __syncthreads();
    apply_reflectors<false, kRL>(c, true);
    double* dst = nullptr;
    if (flags & SW_STORE) dst = adj ? (I.cka + (int64_t)b * sd) : (I.ckf + (int64_t)s * sd);
    else if ((flags & SW_LAST) && s == nb - 1) dst = I.fin;
    if (dst) {
      slab_store_rowmajor(c, dst);
      copy_t(dst + (int64_t)n * n);
      if (c.g == 0) {
        for (int i = c.t; i < n; i += kGangThreads) gmem(dst)[2 * (int64_t)n * n + i] = fabs(L.beta[i]);
        if (c.t == 0) gmem(dst)[2 * (int64_t)n * n + n] = sgn_u;
      }
    }
  }
  int bad = 0;
  for (int i = c.t; i < n; i += kGangThreads) {
    const double d = fabs(L.beta[i]);
    if (!isfinite(d) || !(d > 0.0)) bad = 1;
  }
  if (flags & SW_FINAL) {
    slab_store_rowmajor(c, I.u_out);
    copy_t(I.t_out);
    if (c.g == 0)
      for (int i = c.t; i < n; i += kGangThreads) I.d_out[i] = fabs(L.beta[i]);
  }
  if ((__any(bad) || !c.ok) && c.l == 0 && I.status) atomicOr(I.status, kStatusRange);
  __syncthreads();
}

// Equal-time G, log|det| and sign from the final forward stage (Sec. 5.1,
// mirror form): M = Dp^{-1} U^T + Dm T, G = M^{-1} Dp^{-1} U^T,
// det(1 + U D T) = det U prod(Dp) det M.  The single-decomposition scheme
// (inv_one_plus) is the same with Dp = 1, Dm = D.
template <int kRL>
__device__ void equal_gang(GC& c, const Inst& I) {
  const int n = I.n;
  const double* U = I.fin;
  const double* T = I.fin + (int64_t)n * n;
  const double* D = I.fin + 2 * (int64_t)n * n;
  const double sgn_u = gmem(I.fin)[2 * (int64_t)n * n + n];
  const bool loh = I.scheme == 0;
  auto dp = [&](int i) { const double d = gmem(D)[i]; return (loh && d > 1.0) ? d : 1.0; };
  auto dm = [&](int i) { const double d = gmem(D)[i]; return (loh && d > 1.0) ? 1.0 : d; };
  slab_fill_rows(c, [&](int i, int gc) { return dm(i) * gmem(T)[(int64_t)i * n + gc]; });
  __syncthreads();
  slab_for_each<false>(c, [&](int i, int gc) { return gmem(U)[(int64_t)gc * n + i] / dp(i); }, AddInside{});
  cpqr_gang<kRL>(c);
  slab_fill_cols(c, [&](int i, int gc) { return gmem(U)[(int64_t)gc * n + i] / dp(i); });
  __syncthreads();
  apply_reflectors<true, kRL>(c, false);
  back_subst<kRL>(c);
  int bad = 0;
  for (int idx = c.t; idx < c.geo.npad * c.geo.w; idx += kGangThreads) {
    const int cc = idx / c.geo.npad, i = idx - cc * c.geo.npad;
    if (i < n && c.c0 + cc < n && !isfinite(L.S[cc * c.geo.ldr + i])) bad = 1;
  }
  if (I.g) slab_store_rowmajor_perm(c, I.g);
  const double sp = perm_sign(c);
  if (c.g == 0 && c.w == 0) {
    double ls = 0.0, ng = 0.0;
    for (int i = c.l; i < n; i += 64) {
      const double d = gmem(D)[i];
      if (!isfinite(d) || !(d > 0.0)) bad = 1;
      ls += log(dp(i)) + log(fabs(L.beta[i]));  // dp = 1 without the split
      ng += L.beta[i] < 0.0 ? 1.0 : 0.0;
    }
    ls = wave_sum(ls);
    ng = wave_sum(ng);
    const double sq = refl_sign(c);
    if (!isfinite(ls)) bad = 1;
    if (c.l == 0) {
      if (I.logdet) *I.logdet = ls;
      if (I.sign) *I.sign = sgn_u * sq * sp * ((((long long)ng) & 1) ? -1.0 : 1.0);
    }
  }
  if ((__any(bad) || !c.ok) && c.l == 0 && I.status) atomicOr(I.status, kStatusRange);
  __syncthreads();
}

// Time-displaced G(tau_j, 0) from F[j] = U1 D1 T1 and A[j] = U2 D2 T2
// (Sec. 6.1 inv_sum_loh, same algebra as the single-workgroup kernel):
//   Mid = D_Lm (U1^T U2) D_Rp^{-1} + D_Lp^{-1} (T1 T2^T) D_Rm,
//   G(tau,0) = U2 D_Rp^{-1} Mid^{-1} D_Lp^{-1} T1,
// with D_L = D1^{-1}, D_R = D2; then B_l ... G(tau_j, 0) for the requested
// l of the block (Sec. 6).
template <int kRL>
__device__ void tdisp_gang(GC& c, const Inst& I, int j, int ilo, int ihi,
                           const int32_t* l_list) {
  const int n = I.n, m = I.m, k = I.k, nb = I.nb, np = c.geo.npad;
  const int64_t sd = stage_doubles(n);
  const double* F = j > 0 ? I.ckf + (int64_t)(j - 1) * sd : nullptr;
  const double* A = j < nb ? I.cka + (int64_t)j * sd : nullptr;
  const double* U1 = F;
  const double* T1 = F ? F + (int64_t)n * n : nullptr;
  const double* D1 = F ? F + 2 * (int64_t)n * n : nullptr;
  const double* U2 = A;
  const double* T2 = A ? A + (int64_t)n * n : nullptr;
  const double* D2 = A ? A + 2 * (int64_t)n * n : nullptr;
  double* Xg = sc_X(c);
  // P2 = T1 T2^T (slab columns), kept in HBM while P1 = U1^T U2 is formed
  // (a null stage is the identity; the null tests stay outside the loops
  // so that the loads inside them are unconditional)
  if (T2) slab_fill_cols(c, [&](int i, int gc) { return gmem(T2)[(int64_t)gc * n + i]; });
  else slab_identity(c);
  if (T1) slab_gemm(c, ARowMajor<One>{T1, n, One{}}, One{}, One{});
  else slab_gemm(c, AIdent<One>{n, One{}}, One{}, One{});
  slab_store_colmajor(c, Xg);
  __syncthreads();
  if (U2) slab_fill_rows(c, [&](int i, int gc) { return gmem(U2)[(int64_t)i * n + gc]; });
  else slab_identity(c);
  if (U1) slab_gemm(c, ARowMajorT{U1, n}, One{}, One{});
  else slab_gemm(c, AIdent<One>{n, One{}}, One{}, One{});
  // Mid, with D1 in L.tau and D2 in L.beta (both free until the QR)
  for (int i = c.t; i < np; i += kGangThreads) {
    L.tau[i] = (D1 && i < n) ? gmem(D1)[i] : 1.0;
    L.beta[i] = (D2 && i < n) ? gmem(D2)[i] : 1.0;
  }
  __syncthreads();
  slab_for_each<false>(c,
                       [&](int i, int gc) {
                         const double a = L.tau[i], b = L.beta[gc];
                         const double lm = 1.0 / (a > 1.0 ? a : 1.0);   // D_Lm
                         const double lpi = a < 1.0 ? a : 1.0;           // D_Lp^{-1}
                         const double rpi = 1.0 / (b > 1.0 ? b : 1.0);  // D_Rp^{-1}
                         const double rm = b < 1.0 ? b : 1.0;            // D_Rm
                         // (gc is clamped to n - 1; for a slab wholly past n the read is
                         // kept in range and its result is not stored)
                         const double e = L.S[max(gc - c.c0, 0) * c.geo.ldr + i];
                         return lm * e * rpi + lpi * gmem(Xg)[(int64_t)gc * np + i] * rm;
                       },
                       SetInside{});
  cpqr_gang<kRL>(c);
  // Y = D_Lp^{-1} T1 -> Q^T Y -> R^{-1} (pivot order)
  if (T1) {
    slab_fill_rows(c, [&](int i, int gc) {
      const double a = gmem(D1)[i];
      return gmem(T1)[(int64_t)i * n + gc] * (a < 1.0 ? a : 1.0);
    });
  } else {
    slab_identity(c);
  }
  apply_reflectors<true, kRL>(c, false);
  back_subst<kRL>(c);
  // undo the pivot order through HBM: X[piv[q]][:] = Z[q][:]
  for (int idx = c.t; idx < np * c.geo.w; idx += kGangThreads) {
    const int cc = idx / np, q = idx - cc * np, gc = c.c0 + cc;
    if (gc >= np) continue;
    if (q < n) {
      int row = L.piv[q];
      row = row < 0 ? 0 : (row >= n ? n - 1 : row);
      gmem(Xg)[(int64_t)gc * np + row] = gc < n ? L.S[cc * c.geo.ldr + q] : 0.0;
    } else {
      gmem(Xg)[(int64_t)gc * np + q] = 0.0;
    }
  }
  __syncthreads();
  slab_fill_cols(c, [&](int i, int gc) { return gmem(Xg)[(int64_t)gc * np + i]; });
  __syncthreads();
  // G = (U2 D_Rp^{-1}) X, D_Rp^{-1} in L.beta (free after the solve)
  for (int i = c.t; i < np; i += kGangThreads) {
    const double b = (D2 && i < n) ? gmem(D2)[i] : 1.0;
    L.beta[i] = 1.0 / (b > 1.0 ? b : 1.0);
  }
  __syncthreads();
  if (U2) slab_gemm(c, ARowMajor<BetaScale>{U2, n, BetaScale{}}, One{}, One{});
  else slab_gemm(c, AIdent<BetaScale>{n, BetaScale{}}, One{}, One{});
  int bad = 0;
  for (int idx = c.t; idx < np * c.geo.w; idx += kGangThreads) {
    const int cc = idx / np, i = idx - cc * np;
    if (i < n && c.c0 + cc < n && !isfinite(L.S[cc * c.geo.ldr + i])) bad = 1;
  }
  const int tj = j * k < m ? j * k : m;
  int lc = tj;
  const ASwz aop{I.esw, np / 16};
  for (int idx = ilo; idx < ihi; ++idx) {
    const int l = l_list[idx];
    for (int q = lc + 1; q <= l; ++q) {
      load_slice_scale(c, I, q);
      slab_gemm(c, aop, [&](int kk) { return L.tau[kk]; }, One{});
    }
    lc = l;
    slab_store_rowmajor(c, I.gt + (int64_t)idx * n * n);
  }
  if ((__any(bad) || !c.ok) && c.l == 0 && I.status) atomicOr(I.status, kStatusRange);
  __syncthreads();
}

// Gradient rows of the slices j*k+1 .. min((j+1)k, m) (App. A.1):
//   G_{jk+1} = [1 + U1 (D1 (T1 T2^T) D2) U2^T]^{-1}; udt(D1 T1 T2^T D2) = u d t,
//   U = U1 u, T = t U2^T, then the equal-time inversion (Sec. 5.1), and
//   G_{l+1} = E diag(v_l) G_l diag(1/v_l) Ebar,  grad[l-1][i] = alpha (1 - G_l)_ii.
template <int kRL>
__device__ void grad_gang(GC& c, const Inst& I, int j) {
  const int n = I.n, m = I.m, k = I.k, nb = I.nb, np = c.geo.npad, ldr = c.geo.ldr;
  const int64_t sd = stage_doubles(n);
  const double* F = j > 0 ? I.ckf + (int64_t)(j - 1) * sd : nullptr;
  const double* A = j < nb ? I.cka + (int64_t)j * sd : nullptr;
  const double* U1 = F;
  const double* T1 = F ? F + (int64_t)n * n : nullptr;
  const double* D1 = F ? F + 2 * (int64_t)n * n : nullptr;
  const double* U2 = A;
  const double* T2 = A ? A + (int64_t)n * n : nullptr;
  const double* D2 = A ? A + 2 * (int64_t)n * n : nullptr;
  double* Ug = sc_U(c);
  double* Tg = sc_T(c);
  // D1 (T1 T2^T) D2, with D1 in L.tau and D2 in L.beta (free until the QR)
  for (int i = c.t; i < np; i += kGangThreads) {
    L.tau[i] = (D1 && i < n) ? gmem(D1)[i] : 1.0;
    L.beta[i] = (D2 && i < n) ? gmem(D2)[i] : 1.0;
  }
  if (T2) slab_fill_cols(c, [&](int i, int gc) { return gmem(T2)[(int64_t)gc * n + i]; });
  else slab_identity(c);
  if (T1) slab_gemm(c, ARowMajor<One>{T1, n, One{}}, One{}, [&](int row) { return L.tau[row]; });
  else slab_gemm(c, AIdent<One>{n, One{}}, One{}, [&](int row) { return L.tau[row]; });
  slab_for_each<false>(c, [&](int, int gc) { return L.beta[gc]; }, MulInside{});
  cpqr_gang<kRL>(c);
  // T = d^{-1} (R P^T) U2^T  (slab columns), to HBM
  if (U2) slab_fill_cols(c, [&](int i, int gc) { return gmem(U2)[(int64_t)gc * n + i]; });
  else slab_identity(c);
  slab_gemm(c, AColMajor{sc_R(c), np}, One{},
            [&](int row) { return row < n ? 1.0 / fabs(L.beta[row]) : 0.0; });
  slab_store_colmajor(c, Tg);
  // U = U1 u
  slab_identity(c);
  __syncthreads();
  apply_reflectors<false, kRL>(c, true);
  if (U1) slab_gemm(c, ARowMajor<One>{U1, n, One{}}, One{}, One{});
  slab_store_colmajor(c, Ug);
  // D of the combined factorization: |beta| (kept in L.red-free storage: HBM)
  double* Dg = sc_X(c);
  if (c.g == 0)
    for (int i = c.t; i < n; i += kGangThreads) gmem(Dg)[i] = fabs(L.beta[i]);
  gang_sync(c);
  // M = Dp^{-1} U^T + Dm T
  auto dp = [&](int i) { const double d = gmem(Dg)[i]; return d > 1.0 ? d : 1.0; };
  auto dm = [&](int i) { const double d = gmem(Dg)[i]; return d < 1.0 ? d : 1.0; };
  slab_fill_rows(c, [&](int i, int gc) { return gmem(Ug)[(int64_t)i * np + gc] / dp(i); });
  slab_for_each<false>(c, [&](int i, int gc) { return dm(i) * gmem(Tg)[(int64_t)gc * np + i]; }, AddInside{});
  cpqr_gang<kRL>(c);
  slab_fill_rows(c, [&](int i, int gc) { return gmem(Ug)[(int64_t)i * np + gc] / dp(i); });
  __syncthreads();
  apply_reflectors<true, kRL>(c, false);
  back_subst<kRL>(c);
  // G_{jk+1} = P X into HBM buffer 0 (column-major, rows un-permuted)
  double* Gb[2] = {sc_G(c, 0), sc_G(c, 1)};
  for (int idx = c.t; idx < np * c.geo.w; idx += kGangThreads) {
    const int cc = idx / np, q = idx - cc * np, gc = c.c0 + cc;
    if (gc >= np) continue;
    if (q < n) {
      int row = L.piv[q];
      row = row < 0 ? 0 : (row >= n ? n - 1 : row);
      gmem(Gb[0])[(int64_t)gc * np + row] = gc < n ? L.S[cc * ldr + q] : 0.0;
    } else {
      gmem(Gb[0])[(int64_t)gc * np + q] = 0.0;
    }
  }
  gang_sync(c);
  const int l0 = j * k + 1, l1 = (j + 1) * k < m ? (j + 1) * k : m;
  bool bad = false;
  for (int gc = c.c0 + c.t; gc < c.c0 + c.geo.w && gc < n; gc += kGangThreads) {
    const double gii = gmem(Gb[0])[(int64_t)gc * np + gc];
    bad |= !isfinite(gii);
    gmem(I.grad)[(int64_t)(l0 - 1) * n + gc] = I.alpha * (1.0 - gii);
  }
  const ASwz aop{I.esw, np / 16};
  int cur = 0;
  for (int l = l0; l < l1; ++l) {
    // slab <- diag(1/v_l) Ebar [:, slab]; G_l diag(1/v_l) Ebar; E diag(v_l) (...)
    load_slice_scale(c, I, l);
    slab_fill_rows(c, [&](int i, int gc) { return gmem(I.expk_inv)[(int64_t)i * n + gc] / L.tau[i]; });
    __syncthreads();
    slab_gemm(c, AColMajor{Gb[cur], np}, One{}, One{});
    slab_gemm(c, aop, [&](int kk) { return L.tau[kk]; }, One{});
    slab_store_colmajor(c, Gb[cur ^ 1]);
    for (int gc = c.c0 + c.t; gc < c.c0 + c.geo.w && gc < n; gc += kGangThreads) {
      const double gii = L.S[(gc - c.c0) * ldr + gc];
      bad |= !isfinite(gii);
      gmem(I.grad)[(int64_t)l * n + gc] = I.alpha * (1.0 - gii);
    }
    cur ^= 1;
    gang_sync(c);
  }
  if ((__any(bad) || !c.ok) && c.l == 0 && I.status) atomicOr(I.status, kStatusRange);
  __syncthreads();
}

// plain UDT (Sec. 4.2.2) of one n x n row-major matrix
template <int kRL>
__device__ void udt_gang(GC& c, const double* w, double* u, double* d, double* t) {
  const int n = c.n, np = c.geo.npad;
  slab_fill_rows(c, [&](int i, int gc) { return gmem(w)[(int64_t)i * n + gc]; });
  __syncthreads();
  cpqr_gang<kRL>(c);
  // T = D^{-1} R P^T
  slab_fill_cols(c, [&](int i, int gc) { return sc_R(c)[(int64_t)gc * np + i] / fabs(L.beta[i]); });
  __syncthreads();
  slab_store_rowmajor(c, t);
  __syncthreads();
  slab_identity(c);
  __syncthreads();
  apply_reflectors<false, kRL>(c, true);
  slab_store_rowmajor(c, u);
  if (c.g == 0)
    for (int i = c.t; i < n; i += kGangThreads) d[i] = fabs(L.beta[i]);
  __syncthreads();
}

__device__ GC gang_ctx(const GangArgs& a) {
  GC c;
  c.geo = gang_geom(a.nt);
  // Workgroups are dispatched round-robin over the 8 XCDs; when the gang
  // count allows it, the members of a gang are blocks b, b + 8, ... so that
  // they share one XCD's L2.
  const int b = blockIdx.x;
  int gang;
  if (a.ngangs % 8 == 0) {
    const int x = b & 7, r = b >> 3;
    c.g = r % c.geo.G;
    gang = (r / c.geo.G) * 8 + x;
  } else {
    gang = b / c.geo.G;
    c.g = b - gang * c.geo.G;
  }
  c.gang = gang;
  c.c0 = c.g * c.geo.w;
  c.t = threadIdx.x;
  c.w = threadIdx.x >> 6;
  c.l = threadIdx.x & 63;
  c.base = a.scratch + (int64_t)gang * gang_doubles(c.geo);
  c.bar = a.bars + (int64_t)gang * kGangBarWords;
  c.epoch = 0;
  c.ok = true;
  c.n = 0;
  return c;
}

// The thread's indices in c, made opaque to the optimizer: called once per
// item of a kernel's loop, so that the addresses derived from them are
// recomputed for each item (a few integer instructions) instead of being
// hoisted out of the loop and kept, or spilled, across it.
__device__ __forceinline__ void gang_lanes_per_item(GC& c) {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  c.t = t;
  c.w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  c.l = t & 63;
}

template <int RL>
__global__ __launch_bounds__(kGangThreads, 1) void k_gang_sweep(const Inst* __restrict__ insts,
                                                                 const SweepItem* __restrict__ items,
                                                                 int count, GangArgs a) {
  GC c = gang_ctx(a);
  if (c.gang < count) gang_assemble(c);
  for (int it = c.gang; it < count; it += a.ngangs) {
    const SweepItem wi = items[it];
    const Inst I = insts[wi.inst];
    c.n = I.n;
    gang_lanes_per_item(c);
    sweep_gang<RL>(c, I, wi.flags);
  }
}

template <int MODE, int RL>
__global__ __launch_bounds__(kGangThreads, 1) void k_gang_pair(const Inst* __restrict__ insts,
                                                                const PairItem* __restrict__ items,
                                                                int count, const int32_t* __restrict__ l_list,
                                                                GangArgs a) {
  GC c = gang_ctx(a);
  if (c.gang < count) gang_assemble(c);
  for (int it = c.gang; it < count; it += a.ngangs) {
    const PairItem wi = items[it];
    const Inst I = insts[wi.inst];
    c.n = I.n;
    gang_lanes_per_item(c);
    if (MODE == PAIR_EQUAL) equal_gang<RL>(c, I);
    else if (MODE == PAIR_TDISP) tdisp_gang<RL>(c, I, wi.j, wi.ilo, wi.ihi, l_list);
    else grad_gang<RL>(c, I, wi.j);
  }
}

template <int RL>
__global__ __launch_bounds__(kGangThreads, 1) void k_gang_udt(int n, int count, const double* w, double* u,
                                                               double* d, double* t, GangArgs a) {
  GC c = gang_ctx(a);
  c.n = n;
  if (c.gang < count) gang_assemble(c);
  for (int it = c.gang; it < count; it += a.ngangs) {
    const int64_t off = (int64_t)it * n * n;
    udt_gang<RL>(c, w + off, u + off, d + (int64_t)it * n, t + off);
  }
}

template <class K, class... Args>
hipError_t coop_launch(K kern, GangArgs a, hipStream_t s, Args... args) {
  const GangGeom g = gang_geom(a.nt);
  if (g.G == 0 || a.ngangs < 1) return hipErrorInvalidValue;
  void* ptrs[] = {(void*)&args..., (void*)&a};
  return hipLaunchKernel((const void*)kern, dim3(a.ngangs * g.G), dim3(kGangThreads), ptrs, 0, s);
}

}  // namespace

// rows per lane of a column operation: 4 (n <= 256), 8 (<= 512), 16
int rl_of(int nt) { return nt <= 16 ? 4 : (nt <= 32 ? 8 : 16); }

hipError_t gang_capacity(int nt, int num_cu, int* ngangs) {
  const GangGeom g = gang_geom(nt);
  if (g.G == 0) return hipErrorInvalidValue;
  const void* ks[] = {(const void*)k_gang_sweep<16>, (const void*)k_gang_pair<PAIR_TDISP, 16>,
                      (const void*)k_gang_pair<PAIR_GRAD, 16>, (const void*)k_gang_pair<PAIR_EQUAL, 16>};
  int per_cu = 1 << 30;
  for (const void* k : ks) {
    int b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, kGangThreads, 0);
    if (e != hipSuccess) return e;
    per_cu = b < per_cu ? b : per_cu;
  }
  *ngangs = per_cu * num_cu / g.G;
  return hipSuccess;
}

#define SDQ_RL_SWITCH(CALL) \
  switch (rl_of(a.nt)) {    \
    case 4: return CALL(4); \
    case 8: return CALL(8); \
    default: return CALL(16); \
  }

hipError_t launch_gang_sweep(const Inst* inst, const SweepItem* items, int count, GangArgs a,
                             hipStream_t s) {
#define C(R) coop_launch(k_gang_sweep<R>, a, s, inst, items, count)
  SDQ_RL_SWITCH(C)
#undef C
}

hipError_t launch_gang_pair(int mode, const Inst* inst, const PairItem* items, int count,
                            const int32_t* l_list, GangArgs a, hipStream_t s) {
  if (mode != PAIR_EQUAL && mode != PAIR_TDISP && mode != PAIR_GRAD) return hipErrorInvalidValue;
#define C(R)                                                                                  \
  (mode == PAIR_EQUAL ? coop_launch(k_gang_pair<PAIR_EQUAL, R>, a, s, inst, items, count, l_list) \
   : mode == PAIR_TDISP ? coop_launch(k_gang_pair<PAIR_TDISP, R>, a, s, inst, items, count, l_list) \
                        : coop_launch(k_gang_pair<PAIR_GRAD, R>, a, s, inst, items, count, l_list))
  SDQ_RL_SWITCH(C)
#undef C
}

hipError_t launch_gang_udt(int n, int count, const double* w, double* u, double* d, double* t,
                           GangArgs a, hipStream_t s) {
#define C(R) coop_launch(k_gang_udt<R>, a, s, n, count, w, u, d, t)
  SDQ_RL_SWITCH(C)
#undef C
}

}  // namespace sdq
