// sdq_device.hpp -- gfx950 kernels of libsdq: stabilized DQMC Green's
// functions (C. Bauer, "Fast and stable determinant quantum Monte Carlo",
// arXiv:2003.05286).
//
// Execution model.  One workgroup owns one chain (or one stage pair) at a
// time and pulls work items from a queue in longest-first order (persistent
// launch).  A workgroup has P = min(NT, 4) waves, NT = ceil(n/16).  The
// working n x n matrix lives in registers, split by 16-column tiles over the
// waves; inside a wave it is held exactly in the accumulator layout of the
// FP64 MFMA 16x16x4 instruction:
//     lane l, register [c][ti][r]  <->  row 16*ti + (l/16) + 4*r,
//                                       column 16*(w + P*c) + (l%16)
// (on gfx950 the 16x16 FP64 accumulator gives lane l the rows
// l/16, l/16 + 4, l/16 + 8, l/16 + 12 of column l%16).
// Each column therefore lives in the four lanes l%16 = const of one wave,
// 16*NT/4 rows per lane.  This lets
//   * the slice products W <- E diag(v) W run back to back on MFMA with the
//     previous product as the B operand (no LDS round trip, no barrier),
//   * the pivoted Householder QR work on the same registers: column norms
//     and reflector dot products are lane-local sums plus two cross-row
//     shuffles; the pivot column is exchanged through LDS with one barrier
//     per column step,
//   * Q be formed and R P^T T be multiplied in place.
// The factor R (with the reflectors below it) is parked in LDS, column-major
// by original column index, for Q formation, the T update and the solves.
//
// Paper passages per routine:
//   slice products, stage loop ...... Sec. 4.1 (stabilized product, with the
//                                     naive/stabilized mixture every k slices)
//   cpqr / form_q / T update ........ Sec. 4.2.2 (UDT from pivoted QR)
//   inv_one_plus ..................... Sec. 5.1 (Loh's Dp/Dm split)
//   pair_tdisp ....................... Sec. 6.1 (inv_sum_loh), Sec. 6 (G(tau,0)
//                                     by propagation inside a block)
//   pair_grad ........................ App. A.1 (stack combination) and the
//                                     equal-time G at slice l of Sec. 6
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>
#include <utility>

#include "sdq_internal.h"

namespace sdq {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// geometry

// workgroups per CU the register budget of a kernel targets: two for the
// sweep and the equal-time inversion at n <= 64 (they fit 256 registers per
// lane with little or no spilling), one otherwise
constexpr int minb_for(int nt) { return nt <= 4 ? 2 : 1; }
// (the site loop of the local updates keeps both flavours' G and E^-1 in
// registers: one)
constexpr int minb_pair(int nt, int mode) { return mode == 4 ? 1 : minb_for(nt); }

template <int NT, int P_>
struct Geo {
  static constexpr int NP = 16 * NT;             // padded dimension
  static constexpr int P = P_;                   // waves per workgroup (one chain)
  static constexpr int CT = (NT + P - 1) / P;    // column tiles per wave (max)
  static constexpr int LDR = NP + 1;             // LDS column stride (odd: no bank conflicts)
  static constexpr int THREADS = 64 * P;
  static constexpr int KB = 8;                   // slices of exp(alpha f) staged at once
};

template <int NT, int P, bool ELDS>
struct Smem {
  using G = Geo<NT, P>;
  // Above 128 rows the n x n factor store (R and the reflectors) no longer
  // fits in the CU's 160 KB of LDS beside the rest: it then lives in a
  // per-workgroup area of device memory (rg), accessed through r_ld / r_st.
  static constexpr bool RG = NT > kMaxNT;
  double R[RG ? 1 : G::NP * G::LDR];         // factor store, [col][row]
  double E[ELDS ? G::NP * G::LDR : 1];       // staged operand (sweep: swizzled E; pair: [row][col])
  double cand[2][G::P][G::NP];               // pivot candidate columns
  double vbuf[G::KB][G::NP];                 // exp(alpha f) of the slices in flight
  double tau[G::NP];
  double dnew[G::NP];                        // |diag R| of the last QR
  double dcur[G::NP];                        // D of the current factorization
  double ckey[2][G::P];
  double red[2][G::P];
  int ccol[2][G::P];
  int perm[G::NP];                           // perm[j] = column pivoted at step j
  int sinv[G::NP];                           // sinv[c] = step at which c was pivoted
  int ired[2 * G::P];
  int item;
  double* rg;  // the factor store in device memory (RG)
};

// Device memory seen as the global address space: loads and stores through
// these compile to global instructions.  Through plain (flat) pointers the
// compiler must order every store against the spill slots in scratch memory
// (a wait for all earlier memory operations before each one) and counts
// loads against LDS waits.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// entry i of the factor store, [col][row] with stride LDR; within a
// workgroup the device-memory copy is coherent through the CU's L1 once a
// barrier has ordered the writes before the reads
template <class SM>
__device__ __forceinline__ double r_ld(const SM& S, int i) {
  if constexpr (SM::RG) return gmem(S.rg)[i];
  else return S.R[i];
}
template <class SM>
__device__ __forceinline__ void r_st(SM& S, int i, double v) {
  if constexpr (SM::RG) gmem(S.rg)[i] = v;
  else S.R[i] = v;
}

template <int NT, int P>
struct RM {  // register-resident n x n matrix, column split (see header)
  double v[Geo<NT, P>::CT][NT][4];
};

struct Lane {
  int t, w, l, g, cl;
};

__device__ __forceinline__ Lane lane_id() {
  Lane L;
  L.t = threadIdx.x;
  L.w = threadIdx.x >> 6;
  L.l = threadIdx.x & 63;
  L.g = L.l >> 4;
  L.cl = L.l & 15;
  return L;
}

// The same indices, opaque to the optimizer: called once per work item of a
// persistent loop, so that the addresses derived from them are recomputed
// for each item (a few integer instructions) instead of being hoisted out of
// the loop and kept, or spilled, across it.
__device__ __forceinline__ Lane lane_id_per_item() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  Lane L;
  L.t = t;
  L.w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  L.l = t & 63;
  L.g = L.l >> 4;
  L.cl = L.l & 15;
  return L;
}

template <int NT, int P>
__device__ __forceinline__ bool tile_ok(const Lane& L, int c) {
  return L.w + Geo<NT, P>::P * c < NT;
}
template <int NT, int P>
__device__ __forceinline__ int col_of(const Lane& L, int c) {
  return 16 * (L.w + Geo<NT, P>::P * c) + L.cl;
}
__device__ __forceinline__ int row_of(const Lane& L, int ti, int r) { return 16 * ti + L.g + 4 * r; }

// f(std::integral_constant<int, 0>{}), ..., f(integral_constant<N - 1>): loops
// whose tile index must be a compile-time constant (the column loops of the
// QR and of the reflector applications run tile by tile, so that "tile below,
// at or above the current one" is decided when compiling, not per element)
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// element r of a lane's 4-entry tile column, r wave-uniform
// the double held by lane src (byte address 4 * src) of the wave
__device__ __forceinline__ double lane_fetch(int src_addr, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(src_addr, (int)__double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src_addr, (int)__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double pick4(const double (&a)[4], int r) {
  return r == 0 ? a[0] : (r == 1 ? a[1] : (r == 2 ? a[2] : a[3]));
}

// ---- cross-lane primitives -------------------------------------------------
// A column lives in the four lanes l, l^16, l^32, l^48 (one lane per 16-lane
// row).  v_permlane16_swap / v_permlane32_swap exchange whole rows, so a
// sum over the four lanes is two swaps and two adds; every lane performs
// the same additions in the same order, so all four get bitwise-identical
// results (which the redundant per-wave reflector computation relies on).
__device__ __forceinline__ double pl16_pair_sum(double v) {
  const unsigned lo = __double2loint(v), hi = __double2hiint(v);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  // a[0]/b[0]: the even row of the pair, a[1]/b[1]: the odd row
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double pl32_pair_sum(double v) {
  const unsigned lo = __double2loint(v), hi = __double2hiint(v);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double pl16_pair_max(double v) {
  const unsigned lo = __double2loint(v), hi = __double2hiint(v);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return fmax(__hiloint2double((int)b[0], (int)a[0]), __hiloint2double((int)b[1], (int)a[1]));
}
__device__ __forceinline__ double pl32_pair_max(double v) {
  const unsigned lo = __double2loint(v), hi = __double2hiint(v);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return fmax(__hiloint2double((int)b[0], (int)a[0]), __hiloint2double((int)b[1], (int)a[1]));
}
// sum / max over the four lanes holding one column
__device__ __forceinline__ double sum_col(double v) { return pl32_pair_sum(pl16_pair_sum(v)); }
__device__ __forceinline__ double max_col(double v) { return pl32_pair_max(pl16_pair_max(v)); }

// rotate a double right by R lanes inside each 16-lane row (DPP row_ror;
// every lane has a source, so no old value is needed)
template <int R>
__device__ __forceinline__ double row_ror(double v) {
  const int lo = __builtin_amdgcn_mov_dpp((int)__double2loint(v), 0x120 + R, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)__double2hiint(v), 0x120 + R, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// max of two pivot keys (never NaN): one v_max_f64, without the operand
// canonicalization fmax() adds for NaN inputs
__device__ __forceinline__ double key_max(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// max of pivot keys over the 16 lanes of each row (all of them get it)
__device__ __forceinline__ double row_max16(double v) {
  v = key_max(v, row_ror<8>(v));
  v = key_max(v, row_ror<4>(v));
  v = key_max(v, row_ror<2>(v));
  v = key_max(v, row_ror<1>(v));
  return v;
}

// Pivot key: the column norm with its IB lowest mantissa bits replaced by
// 2^IB - 1 - column, so that one max over doubles picks the largest norm
// and, among norms equal to 2^-(52 - IB) relative, the smallest column
// index (IB = 7 up to 128 columns: 2^-45; IB = 8 up to 256: 2^-44).  A NaN
// or infinite norm is clamped (never loses eligibility); -1 marks "not a
// candidate".
template <int IB = 7>
__device__ __forceinline__ double pivot_key(double norm, int col) {
  constexpr unsigned long long M = (1ull << IB) - 1;
  double x = norm >= 0.0 ? norm : 0.0;  // NaN -> 0
  x = x < 1.0e300 ? x : 1.0e300;
  const unsigned long long b = (__double_as_longlong(x) & ~M) | (unsigned long long)(M - col);
  return __longlong_as_double((long long)b);
}
template <int IB = 7>
__device__ __forceinline__ int pivot_col(double key) {
  constexpr unsigned long long M = (1ull << IB) - 1;
  return (int)M - (int)(__double_as_longlong(key) & M);
}
// index bits of the pivot keys of an n x n register matrix
template <int NT>
constexpr int key_bits() { return 16 * NT > 128 ? 8 : 7; }

// sqrt(q) for q in [2^-30, 2^3] (scaled squared norms): the hardware
// reciprocal square root estimate refined by one Goldschmidt step
// (y -> sqrt(q), h -> 1/(2 sqrt(q))) and one Newton correction of the
// residual q - y^2; within about an ulp, and no special cases are needed in
// that range
__device__ __forceinline__ double sqrt_mid(double q) {
  const double r = __builtin_amdgcn_rsq(q);
  double y = q * r, h = 0.5 * r;
  const double e = fma(-h, y, 0.5);
  y = fma(y, e, y);
  h = fma(h, e, h);
  const double d = fma(-y, y, q);
  return fma(d, h, y);
}
// 1/x for x in [2^-4, 2^4]: the hardware reciprocal estimate and two Newton
// steps, within about an ulp
__device__ __forceinline__ double rcp_mid(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// exact power-of-two scale that brings x near 1 (1 for 0, inf, nan)
// its exact inverse (dividing by a power of two is a multiplication)
__device__ __forceinline__ double pow2_unscale(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 1.0;
  return ldexp(1.0, ilogb(x));
}
__device__ __forceinline__ double pow2_scale(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 1.0;
  return ldexp(1.0, -ilogb(x));
}

template <int NT, int P>
__device__ __forceinline__ void set_identity(const Lane& L, RM<NT, P>& A) {
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c)
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) A.v[c][ti][r] = (row_of(L, ti, r) == col_of<NT, P>(L, c)) ? 1.0 : 0.0;
}

// entry [tj][rj] of one lane's column slice; tj, rj are wave-uniform
template <int NT>
__device__ __forceinline__ double reg_at(const double (&a)[NT][4], int tj, int rj) {
  double t[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    t[r] = a[0][r];
#pragma unroll
    for (int ti = 1; ti < NT; ++ti)
      if (ti == tj) t[r] = a[ti][r];
  }
  return rj == 0 ? t[0] : rj == 1 ? t[1] : rj == 2 ? t[2] : t[3];
}


// ---------------------------------------------------------------------------
// C = A * B on FP64 MFMA.  A(ti, tk, r, i, k) is any callable returning the
// entry (i, k) of the left operand, i = 16 ti + l%16, k = 16 tk + l/16 + 4 r
// (i, k < NP) for the calling lane l; B and C are register matrices.  The B
// operand of one 16x16x4 step is register [c][tk][r] as is: its four k
// indices are rows 16tk + q + 4r, q = 0..3, so the A operand is fetched with
// the same row permutation of k.
template <int NT, int P, class AF>
__device__ __forceinline__ void gemm_rb(const Lane& L, AF A, const RM<NT, P>& B, RM<NT, P>& C) {
  constexpr int CT = Geo<NT, P>::CT;
  d4 acc[CT][NT];
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) acc[c][ti] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int tk = 0; tk < NT; ++tk) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kk = 16 * tk + L.g + 4 * r;
#pragma unroll
      for (int ti = 0; ti < NT; ++ti) {
        const double a = A(ti, tk, r, 16 * ti + L.cl, kk);
#pragma unroll
        for (int c = 0; c < CT; ++c)
          if (c == 0 || tile_ok<NT, P>(L, c))
            acc[c][ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B.v[c][tk][r], acc[c][ti], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) C.v[c][ti][r] = acc[c][ti][r];
}

// C = M B (trans: M^T B) for the row-major n x n matrix M in device memory,
// zero padded; a null M is the identity.  The loads are unconditional
// (clamped in-range addresses, padding selected away afterwards): a load
// behind a per-entry branch would be waited for before the next one.
template <int NT, int P>
__device__ __forceinline__ void gemm_gm(const Lane& L, const double* M, int n, bool trans, const RM<NT, P>& B,
                                        RM<NT, P>& C) {
  if (M == nullptr) {
#pragma unroll
    for (int c = 0; c < Geo<NT, P>::CT; ++c)
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) C.v[c][ti][r] = row_of(L, ti, r) < n ? B.v[c][ti][r] : 0.0;
    return;
  }
  const auto* g = gmem(M);
  gemm_rb<NT, P>(L,
                 [&](int, int, int, int i, int kk) -> double {
                   const int a = min(i, n - 1), b = min(kk, n - 1);
                   const double v = trans ? g[(size_t)b * n + a] : g[(size_t)a * n + b];
                   return (i < n && kk < n) ? v : 0.0;
                 },
                 B, C);
}
// C = M[:, perm] B: the columns of M gathered by S-resident pivot order
// (perm[s] for s < n), same conventions as gemm_gm
template <int NT, int P>
__device__ __forceinline__ void gemm_gm_perm(const Lane& L, const double* M, int n, const int* perm,
                                             const RM<NT, P>& B, RM<NT, P>& C) {
  if (M == nullptr) {
    gemm_rb<NT, P>(L,
                   [&](int, int, int, int i, int s) -> double {
                     return (i < n && s < n && perm[s] == i) ? 1.0 : 0.0;
                   },
                   B, C);
    return;
  }
  const auto* g = gmem(M);
  gemm_rb<NT, P>(L,
                 [&](int, int, int, int i, int s) -> double {
                   const int p = perm[min(s, n - 1)];
                   const double v = g[(size_t)min(i, n - 1) * n + p];
                   return (i < n && s < n) ? v : 0.0;
                 },
                 B, C);
}

// load a row-major n x n global matrix (or its transpose) into registers,
// zero padded; `src == nullptr` loads the identity.  Every entry is loaded
// unconditionally (padding positions read a clamped in-range address and
// are zeroed afterwards): a load inside a per-element branch makes the
// compiler wait for it before the next one, one memory latency per entry.
template <int NT, int P>
__device__ __forceinline__ void load_rm(const Lane& L, RM<NT, P>& A, const double* src, int n, bool trans) {
  if (src == nullptr) {
#pragma unroll
    for (int c = 0; c < Geo<NT, P>::CT; ++c)
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) A.v[c][ti][r] = row_of(L, ti, r) == col_of<NT, P>(L, c) ? 1.0 : 0.0;
    return;
  }
  const auto* g = gmem(src);
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c) {
    const int cc = min(col_of<NT, P>(L, c), n - 1);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = min(row_of(L, ti, r), n - 1);
        A.v[c][ti][r] = trans ? g[cc * n + rr] : g[rr * n + cc];
      }
  }
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c) {
    const bool cok = tile_ok<NT, P>(L, c) && col_of<NT, P>(L, c) < n;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (!(cok && row_of(L, ti, r) < n)) A.v[c][ti][r] = 0.0;
  }
}

// store the leading n x n block of a register matrix (row-major): one base
// address per lane (row L.g of its column) plus a wave-uniform row offset
// per register, so no per-element address is kept live
template <int NT, int P>
__device__ __forceinline__ void store_rm(const Lane& L, const RM<NT, P>& A, double* dst, int n) {
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c) {
    const int col = col_of<NT, P>(L, c);
    if (!tile_ok<NT, P>(L, c) || col >= n) continue;
    // rows L.g + 4k, k = 4 ti + r: the address advances by 4 rows per
    // register; the row test is wave-uniform except in a ragged last tile
    auto* p = gmem(dst) + (size_t)L.g * n + col;
    const size_t step = 4 * (size_t)n;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (16 * ti + 4 * r + 3 < n || row_of(L, ti, r) < n) *p = A.v[c][ti][r];
        p += step;
      }
  }
}

template <int NT, int P>
__device__ __forceinline__ bool all_finite(const Lane& L, const RM<NT, P>& A) {
  bool ok = true;
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c)
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) ok = ok && isfinite(A.v[c][ti][r]);
  return ok;
}

// ---------------------------------------------------------------------------
// Column-pivoted Householder QR of the register matrix A (columns >= n and
// rows >= n are padding: padded rows are zero, padded columns never pivot).
//   step j: pick the live column of largest remaining norm (ties: smallest
//   column index), build the reflector that maps its rows j.. to
//   (beta, 0, ...), beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta,
//   apply it to the other live columns and downdate their norms; recompute a
//   norm exactly when 1 - (|r|/vn1)^2 scaled by (vn1/vn2)^2 drops below
//   sqrt(eps) (Drmac & Bujanovic).
// Columns are not moved: on return S.R[c*LDR + i] holds, for every column
// c, R[i][s_c] for i <= s_c and the reflector v_{s_c} below (unit entry
// implied), with s_c = S.sinv[c] the step at which c was chosen; S.perm[j]
// is the column chosen at step j and S.tau[j] its reflector scalar.  So
// R P^T has column c = S.R column c masked to rows <= s_c.  Padded columns
// are stored as unit vectors with s_c = c.  One barrier per step; ends with
// a barrier.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void cpqr(const Lane& L, const int n, RM<NT, P>& A, Smem<NT, P, ELDS>& S) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  const double tol3z = 1.4901161193847656e-08;  // sqrt(2^-52)
  double vn1[CT], vn2[CT], sv2[CT], iv2[CT];  // sv2: exact power-of-two scale of vn2, iv2 = 1/sv2
  int ps[CT];  // -1: live, not yet chosen; else the step (padding: own index)

#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int col = col_of<NT, P>(L, c);
    const bool live = tile_ok<NT, P>(L, c) && col < n;
    ps[c] = live ? -1 : col;
    double mx = 0.0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) mx = fmax(mx, fabs(A.v[c][ti][r]));
    mx = max_col(mx);
    const double sc = pow2_scale(mx), usc = pow2_unscale(mx);
    double s = 0.0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double x = A.v[c][ti][r] * sc;
        s = fma(x, x, s);
      }
    s = sum_col(s);
    vn1[c] = sqrt(s) * usc;
    vn2[c] = vn1[c];
    sv2[c] = pow2_scale(vn2[c]);
    iv2[c] = pow2_unscale(vn2[c]);
  }

  int buf = 0;
  static_for<NT>([&](auto tjc) {
    constexpr int TJ = decltype(tjc)::value;
    const int jend = 16 * TJ + 16 < n ? 16 * TJ + 16 : n;
    for (int j = 16 * TJ; j < jend; ++j) {
      const int jj = j - 16 * TJ, gj = jj & 3, rj = jj >> 2;
      // row j of each column before this step's update, fetched from the
      // lane group holding it (read here, off the step's dependency chain)
      double ajc[CT];
      const int jsrc = ((gj << 4) | L.cl) << 2;
#pragma unroll
      for (int c = 0; c < CT; ++c) ajc[c] = lane_fetch(jsrc, pick4(A.v[c][TJ], rj));
      // ---- wave-local candidate (packed key), columns of this wave
      double key = -1.0;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const double kc = ps[c] < 0 ? pivot_key<key_bits<NT>()>(vn1[c], col_of<NT, P>(L, c)) : -1.0;
        key = c == 0 ? kc : key_max(key, kc);
      }
      key = row_max16(key);  // the four rows hold the same columns
      const int bc = pivot_col<key_bits<NT>()>(key);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        if (key >= 0.0 && ps[c] < 0 && col_of<NT, P>(L, c) == bc) {
#pragma unroll
          for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) S.cand[buf][L.w][row_of(L, ti, r)] = A.v[c][ti][r];
        }
      }
      double pk = key;
      if constexpr (P > 1) {
        if (L.l == 0) S.ckey[buf][L.w] = key;
        __syncthreads();
        // workgroup pivot: the owner wave follows from the column index
        pk = S.ckey[buf][0];
#pragma unroll
        for (int q = 1; q < P; ++q) pk = key_max(pk, S.ckey[buf][q]);
      } else {
        // one wave: its own LDS writes are visible to its later reads
        __builtin_amdgcn_wave_barrier();
      }
      const int pc = pivot_col<key_bits<NT>()>(pk);
      const int pw = (pc >> 4) % P;
      const double* xc = S.cand[buf][pw];
      const double alpha = xc[j];
      // norm estimate of the pivot column (key without the index bits)
      const double vpiv = __longlong_as_double(__double_as_longlong(pk) & ~((1ll << key_bits<NT>()) - 1));

      // ---- reflector (every wave computes the same one from the same data);
      // rows <= j masked in tile TJ only, tiles below TJ never touched.
      // v keeps y = the pivot column below row j times sc (exact: sc is a
      // power of two); the Householder vector is e_j + w y.
      const double sc = pow2_scale(vpiv), usc = pow2_unscale(vpiv);
      // Above kMaxNT tiles the register budget (three waves per SIMD) does
      // not hold y beside the matrix: it is read again from LDS for each of
      // its three uses (the compiler barriers keep the reads from merging)
      // instead of being spilled.
      constexpr bool VRELOAD = NT > kMaxNT;
      auto yv = [&](int ti, int r) -> double {
        const double x = xc[row_of(L, ti, r)];
        return (ti == TJ && L.g + 4 * r <= jj) ? 0.0 : x * sc;
      };
      double v[VRELOAD ? 1 : NT][4];
      double sp[4] = {0.0, 0.0, 0.0, 0.0};  // four independent accumulation chains
      if constexpr (VRELOAD) {
#pragma unroll
        for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double y = yv(ti, r);
            sp[r] = fma(y, y, sp[r]);
          }
      } else {
        // all LDS reads of the pivot column first, one wait for them
#pragma unroll
        for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) v[ti][r] = xc[row_of(L, ti, r)];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double x = v[ti][r];
            if (ti == TJ && L.g + 4 * r <= jj) x = 0.0;
            const double y = x * sc;
            v[ti][r] = y;
            sp[r] = fma(y, y, sp[r]);
          }
      }
      double s = sum_col((sp[0] + sp[1]) + (sp[2] + sp[3]));
      const double as = alpha * sc;
      double tau = 0.0, beta = alpha, w = 0.0;
      if (s != 0.0) {
        // with q = ||x[j:]||^2 (scaled) and r = 1/sqrt(q):  beta = -sign(alpha) q r,
        // tau = (beta - alpha)/beta = 1 + |alpha| / ||x||, 1/(alpha - beta) =
        // sign(alpha) / (|alpha| + ||x||), which is w / sc: one reciprocal
        // square root and one reciprocal on the dependency chain instead of a
        // square root and two divisions (|alpha| + ||x|| is within [2^-2, 2^3]
        // after the scaling)
        const double q = fma(as, as, s);
        const double r = rsqrt(q);
        const double hq = q * r;  // ||x[j:]|| * sc
        beta = -copysign(hq * usc, alpha);
        tau = fma(fabs(as), r, 1.0);
        w = copysign(rcp_mid(fabs(as) + hq), alpha);
      }

      // ---- apply H_j to the other live columns, downdate their norms
      bool need = false;
      bool rec[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = col_of<NT, P>(L, c);
        const bool is_piv = ps[c] < 0 && col == pc;
        const bool upd = ps[c] < 0 && !is_piv;
        rec[c] = false;
        double dp[4] = {0.0, 0.0, 0.0, 0.0};
        if constexpr (VRELOAD) asm volatile("" ::: "memory");
#pragma unroll
        for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if constexpr (VRELOAD) dp[r] = fma(yv(ti, r), A.v[c][ti][r], dp[r]);
            else dp[r] = fma(v[ti][r], A.v[c][ti][r], dp[r]);
          }
        if constexpr (VRELOAD) asm volatile("" ::: "memory");
        // (e_j + w y)^T a_c = a_jc + w (y^T a_c)
        const double d = fma(w, sum_col((dp[0] + dp[1]) + (dp[2] + dp[3])), ajc[c]) * (upd ? tau : 0.0);
        // row j after the update
        const double rjv = ajc[c] - d;
        if (is_piv) {
          // the pivot column becomes column j of R plus the reflector
#pragma unroll
          for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int q = L.g + 4 * r;
              const double y = VRELOAD ? yv(ti, r) : v[VRELOAD ? 0 : ti][r];
              if (ti > TJ || q > jj) A.v[c][ti][r] = w * y;
              else if (q == jj) A.v[c][ti][r] = beta;
            }
        } else {
          // rows below j: a -= (d w) y; row j: a_jc - d; rows above j: y = 0
          const double dw = d * w;
#pragma unroll
          for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              A.v[c][ti][r] = fma(-dw, VRELOAD ? yv(ti, r) : v[VRELOAD ? 0 : ti][r], A.v[c][ti][r]);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (L.g + 4 * r == jj) A.v[c][TJ][r] = rjv;
        }
        if (upd && vn1[c] != 0.0) {
          // vn1^2 - r^2 = vn1^2 (1 - (r/vn1)^2); recompute when that falls to
          // sqrt(eps) vn2^2 or below (same test, no division), all scaled by
          // the exact power of two of vn2
          const double a1 = fabs(rjv) * sv2[c], b1 = vn1[c] * sv2[c];
          const double q = fmax(0.0, (b1 - a1) * (b1 + a1));
          const double w2 = vn2[c] * sv2[c];
          if (q <= tol3z * (w2 * w2)) {
            need = true;
            rec[c] = true;
          } else {
            vn1[c] = sqrt_mid(q) * iv2[c];  // q in (sqrt(eps), 4]
          }
        }
      }
      if (__any(need)) {
        // exact recompute of the norm of rows j+1.. (rare)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          double mx = 0.0;
#pragma unroll
          for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (ti > TJ || L.g + 4 * r > jj) mx = fmax(mx, fabs(A.v[c][ti][r]));
          mx = max_col(mx);
          const double sc2 = pow2_scale(mx), usc2 = pow2_unscale(mx);
          double s2 = 0.0;
#pragma unroll
          for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (ti > TJ || L.g + 4 * r > jj) {
                const double y = A.v[c][ti][r] * sc2;
                s2 = fma(y, y, s2);
              }
          s2 = sum_col(s2);
          const double nn = sqrt(s2) * usc2;
          if (rec[c]) {
            vn1[c] = nn;
            vn2[c] = nn;
            sv2[c] = pow2_scale(nn);
            iv2[c] = pow2_unscale(nn);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < CT; ++c)
        if (ps[c] < 0 && col_of<NT, P>(L, c) == pc) ps[c] = j;
      if (L.t == 0) {
        S.tau[j] = tau;
        S.perm[j] = pc;
      }
      buf ^= 1;
    }
  });

  // ---- park R / reflectors in LDS
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (!tile_ok<NT, P>(L, c)) continue;
    const int col = col_of<NT, P>(L, c);
    const bool live = col < n;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(L, ti, r);
        r_st(S, col * G::LDR + row, live ? A.v[c][ti][r] : (row == col ? 1.0 : 0.0));
      }
    if (L.g == 0) S.sinv[col] = ps[c];
  }
  for (int t = n + L.t; t < G::NP; t += G::THREADS) {
    S.perm[t] = t;
    S.tau[t] = 0.0;
  }
  __syncthreads();
}

// D' = |diag R| (1 on padding) into S.dnew; ends with a barrier
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void diag_r(const Lane& L, const int n, Smem<NT, P, ELDS>& S) {
  using G = Geo<NT, P>;
  for (int t = L.t; t < G::NP; t += G::THREADS)
    S.dnew[t] = t < n ? fabs(r_ld(S, S.perm[t] * G::LDR + t)) : 1.0;
  __syncthreads();
}

// reflector j (in tile TJ) from the factor store, at this lane's rows of
// tiles TJ.. (zero above row j, unit at row j)
template <int TJ, int NT, int P, bool ELDS>
__device__ __forceinline__ void load_reflector(const Lane& L, const Smem<NT, P, ELDS>& S, int j,
                                               double (&v)[NT][4]) {
  const int jj = j - 16 * TJ;
  const int vc = S.perm[j] * Geo<NT, P>::LDR;
  // all reads first (one wait), then the masking of tile TJ
#pragma unroll
  for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) v[ti][r] = r_ld(S, vc + row_of(L, ti, r));
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = L.g + 4 * r;
    v[TJ][r] = q > jj ? v[TJ][r] : (q == jj ? 1.0 : 0.0);
  }
}

// X <- H_j X for all column blocks (tiles below TJ untouched); column
// tiles whose columns all lie left of `cmin` are skipped
template <int TJ, int NT, int P>
__device__ __forceinline__ void apply_reflector(const Lane& L, double tau, const double (&v)[NT][4],
                                                RM<NT, P>& X, int cmin = 0) {
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c) {
    if (16 * (L.w + P * c) + 15 < cmin) continue;  // wave-uniform
    double dp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) dp[r] = fma(v[ti][r], X.v[c][ti][r], dp[r]);
    const double d = sum_col((dp[0] + dp[1]) + (dp[2] + dp[3])) * tau;
#pragma unroll
    for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) X.v[c][ti][r] = fma(-d, v[ti][r], X.v[c][ti][r]);
  }
}

// Q = H_0 H_1 ... H_{n-1} into registers (reflectors applied last to first,
// tile by tile).  When H_j is applied, the columns left of j are still unit
// vectors e_c (c < j) that H_j leaves as they are, so a wave whose columns
// all lie left of j skips it.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void form_q(const Lane& L, const int n, const Smem<NT, P, ELDS>& S, RM<NT, P>& X) {
  set_identity<NT, P>(L, X);
  // rightmost column this wave holds
  const int cmax = 16 * (L.w + P * (Geo<NT, P>::CT - 1)) + 15;
  static_for<NT>([&](auto kc) {
    constexpr int TJ = NT - 1 - decltype(kc)::value;
    const int jhi = (16 * TJ + 15 < n - 1 ? 16 * TJ + 15 : n - 1);
    const int jtop = jhi < cmax ? jhi : cmax;
    for (int j = jtop; j >= 16 * TJ; --j) {
      const double tau = S.tau[j];
      if (tau == 0.0) continue;
      double v[NT][4];
      load_reflector<TJ, NT, P, ELDS>(L, S, j, v);
      apply_reflector<TJ, NT, P>(L, tau, v, X, j);
    }
  });
}

// Y <- Q^T Y = H_{n-1} ... H_0 Y.  Inside a tile the next reflector is read
// from LDS while the current one is applied.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void apply_qt(const Lane& L, const int n, const Smem<NT, P, ELDS>& S, RM<NT, P>& Y) {
  static_for<NT>([&](auto tjc) {
    constexpr int TJ = decltype(tjc)::value;
    const int jend = 16 * TJ + 16 < n ? 16 * TJ + 16 : n;
    if (jend <= 16 * TJ) return;
    double v[NT][4], vn[NT][4];
    load_reflector<TJ, NT, P, ELDS>(L, S, 16 * TJ, vn);
    double tn = S.tau[16 * TJ];
    for (int j = 16 * TJ; j < jend; ++j) {
      const double tau = tn;
#pragma unroll
      for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[ti][r] = vn[ti][r];
      if (j + 1 < jend) {
        load_reflector<TJ, NT, P, ELDS>(L, S, j + 1, vn);
        tn = S.tau[j + 1];
      }
      if (tau != 0.0) apply_reflector<TJ, NT, P>(L, tau, v, Y);
    }
  });
}

// Y <- R^{-1} Y (R in pivot order: R[i][j] = S.R[perm[j]*LDR + i], i <= j)
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void back_subst(const Lane& L, const int n, const Smem<NT, P, ELDS>& S, RM<NT, P>& Y) {
  using G = Geo<NT, P>;
  static_for<NT>([&](auto kc) {
    constexpr int TJ = NT - 1 - decltype(kc)::value;
    const int jhi = (16 * TJ + 15 < n - 1 ? 16 * TJ + 15 : n - 1);
    for (int j = jhi; j >= 16 * TJ; --j) {
      const int jj = j - 16 * TJ, gj = jj & 3, rj = jj >> 2;
      const double* rc = &S.R[S.perm[j] * G::LDR];
      const double rinv = 1.0 / rc[j];
      double rr[NT][4];
#pragma unroll
      for (int ti = 0; ti <= TJ; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) rr[ti][r] = rc[row_of(L, ti, r)];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 4; ++r) rr[TJ][r] = L.g + 4 * r < jj ? rr[TJ][r] : 0.0;
#pragma unroll
      for (int c = 0; c < G::CT; ++c) {
        const double zj = sum_col(L.g == gj ? pick4(Y.v[c][TJ], rj) : 0.0) * rinv;
#pragma unroll
        for (int ti = 0; ti <= TJ; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (ti == TJ && L.g + 4 * r == jj) Y.v[c][ti][r] = zj;
            else Y.v[c][ti][r] = fma(-rr[ti][r], zj, Y.v[c][ti][r]);
          }
      }
    }
  });
}

// Y <- A^{-1} Y for the register matrices A (n x n, padding zero) and Y, by
// Gaussian elimination with column pivoting: at step j the pivot is the
// live column of largest |A[j][c]| (ties: smallest column), its entries
// below row j divided by the pivot are the multipliers l_r, and row j times
// l_r is subtracted from every row r > j of the other live columns and of Y
// (so Y becomes L^{-1} Y on the way; L itself is not kept).  This is Gaussian
// elimination with partial pivoting applied to A^T, arranged like cpqr: the
// rows are static per tile (row j of every column is fetched from a fixed
// lane group), each wave offers its best column through LDS and one barrier
// per step settles the pivot, and columns are never moved.  Then U (U[i][j]
// = A[i][perm j], i <= j) is parked in S.R by original column, as cpqr parks
// R, and Y <- U^{-1} Y by back substitution; the rows of the result are in
// pivot order: A^{-1} Y [S.perm[s]][c] = Y[s][c].  A is destroyed.  A
// singular A leaves non-finite entries in Y.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void ge_solve(const Lane& L, const int n, RM<NT, P>& A, RM<NT, P>& Y, Smem<NT, P, ELDS>& S) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  int ps[CT];  // -1: live, not yet chosen; else the step (padding: own index)
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int col = col_of<NT, P>(L, c);
    ps[c] = (tile_ok<NT, P>(L, c) && col < n) ? -1 : col;
  }
  int buf = 0;
  static_for<NT>([&](auto tjc) {
    constexpr int TJ = decltype(tjc)::value;
    const int jend = 16 * TJ + 16 < n ? 16 * TJ + 16 : n;
    for (int j = 16 * TJ; j < jend; ++j) {
      const int jj = j - 16 * TJ, gj = jj & 3, rj = jj >> 2;
      const int jsrc = ((gj << 4) | L.cl) << 2;
      // row j of each column and of Y, from the lane group holding it
      double ajc[CT], yjc[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        ajc[c] = lane_fetch(jsrc, pick4(A.v[c][TJ], rj));
        yjc[c] = lane_fetch(jsrc, pick4(Y.v[c][TJ], rj));
      }
      // ---- wave-local candidate: largest |A[j][c]| of this wave's live columns
      double key = -1.0;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const double kc = ps[c] < 0 ? pivot_key(fabs(ajc[c]), col_of<NT, P>(L, c)) : -1.0;
        key = c == 0 ? kc : key_max(key, kc);
      }
      key = row_max16(key);
      const int bc = pivot_col(key);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        if (key >= 0.0 && ps[c] < 0 && col_of<NT, P>(L, c) == bc) {
#pragma unroll
          for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) S.cand[buf][L.w][row_of(L, ti, r)] = A.v[c][ti][r];
        }
      }
      double pk = key;
      if constexpr (P > 1) {
        if (L.l == 0) S.ckey[buf][L.w] = key;
        __syncthreads();
        pk = S.ckey[buf][0];
#pragma unroll
        for (int q = 1; q < P; ++q) pk = key_max(pk, S.ckey[buf][q]);
      } else {
        __builtin_amdgcn_wave_barrier();
      }
      const int pc = pivot_col(pk);
      const int pw = (pc >> 4) % P;
      const double* xc = S.cand[buf][pw];
      const double rinv = 1.0 / xc[j];
      // multipliers of the rows below j (zero at and above j)
      double ml[NT][4];
#pragma unroll
      for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) ml[ti][r] = xc[row_of(L, ti, r)];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ml[ti][r] = (ti > TJ || L.g + 4 * r > jj) ? ml[ti][r] * rinv : 0.0;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const bool upd = ps[c] < 0 && col_of<NT, P>(L, c) != pc;
        const double a = upd ? ajc[c] : 0.0;
#pragma unroll
        for (int ti = TJ; ti < NT; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            A.v[c][ti][r] = fma(-ml[ti][r], a, A.v[c][ti][r]);
            Y.v[c][ti][r] = fma(-ml[ti][r], yjc[c], Y.v[c][ti][r]);
          }
        if (ps[c] < 0 && col_of<NT, P>(L, c) == pc) ps[c] = j;
      }
      if (L.t == 0) S.perm[j] = pc;
      buf ^= 1;
    }
  });
  // ---- park U in LDS by original column (rows <= its step), as cpqr does
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (!tile_ok<NT, P>(L, c)) continue;
    const int col = col_of<NT, P>(L, c);
    const bool live = col < n;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(L, ti, r);
        S.R[col * G::LDR + row] = live ? A.v[c][ti][r] : (row == col ? 1.0 : 0.0);
      }
    if (L.g == 0) S.sinv[col] = ps[c];
  }
  for (int t = n + L.t; t < G::NP; t += G::THREADS) S.perm[t] = t;
  __syncthreads();
  back_subst<NT, P, ELDS>(L, n, S, Y);
}

// left operand of R P^T: column c, rows <= s_c
template <int NT, int P, bool ELDS>
struct RPtOp {
  const Smem<NT, P, ELDS>& S;
  __device__ double operator()(int, int, int, int i, int k) const {
    const double x = r_ld(S, k * Geo<NT, P>::LDR + i);  // read unconditionally, then masked
    return (i <= S.sinv[k]) ? x : 0.0;
  }
};

// T <- D'^{-1} (R P^T) T  with D' = S.dnew
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void update_t(const Lane& L, const Smem<NT, P, ELDS>& S, RM<NT, P>& T) {
  RM<NT, P> Tn;
  gemm_rb<NT, P>(L, RPtOp<NT, P, ELDS>{S}, T, Tn);
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c)
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) T.v[c][ti][r] = Tn.v[c][ti][r] / S.dnew[row_of(L, ti, r)];
}

// det Q = (-1)^(number of nonzero reflectors among steps 0..n-1).  No barrier.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ double refl_sign(const Lane& L, const int n, const Smem<NT, P, ELDS>& S) {
  int cnt = 0;
  for (int i = L.l; i < n; i += 64) cnt += (S.tau[i] != 0.0);
  const unsigned long long b = __ballot(cnt & 1);
  return (__popcll(b) & 1) ? -1.0 : 1.0;
}

// parity of the pivot permutation (inversions of S.perm) as +-1.
// Ends with a barrier.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ double perm_sign(const Lane& L, const int n, Smem<NT, P, ELDS>& S) {
  using G = Geo<NT, P>;
  int inv = 0;
  for (int i = L.t; i < n; i += G::THREADS) {
    const int pi = S.perm[i];
    for (int j = i + 1; j < n; ++j) inv += (S.perm[j] < pi);
  }
  const unsigned long long bi = __ballot(inv & 1);
  if (L.l == 0) S.ired[L.w] = __popcll(bi) & 1;
  __syncthreads();
  int p = 0;
  for (int q = 0; q < G::P; ++q) p ^= S.ired[q];
  __syncthreads();
  return p ? -1.0 : 1.0;
}

// ---------------------------------------------------------------------------
// (1 + U D T)^{-1} with Loh's split (Sec. 5.1).  We use the mirror image of
// the printed factorization, which needs U^T rather than T^{-1}:
//   1 + U Dm Dp T = U Dp (Dp^{-1} U^T + Dm T),  Dp = max(D,1), Dm = min(D,1)
//   G = M^{-1} Dp^{-1} U^T,   M = Dp^{-1} U^T + Dm T,
// M inverted through its pivoted QR, M P = Q R:  G = P R^{-1} Q^T Dp^{-1} U^T.
//   det(1 + U D T) = det U * prod(Dp) * det M.
// With loh = false the same code runs the single-decomposition scheme
// (Sec. 5.1 inv_one_plus, mirrored): Dp = 1, Dm = D, M = U^T + D T.
// U, T: register matrices (padding: identity); D: S.dcur.  Returns Z with
// G[S.perm[s]][c] = Z[s][c] (caller writes it out), and log|det|, sign.
template <int NT, int P, bool ELDS, bool LOH = true>
__device__ __forceinline__ void inv_one_plus(const Lane& L, const int n, Smem<NT, P, ELDS>& S, const RM<NT, P>& U,
                             const RM<NT, P>& T, double sgn_u, RM<NT, P>& Z, double* logdet,
                             double* sign) {
  constexpr bool loh = LOH;
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  // U^T via LDS
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (!tile_ok<NT, P>(L, c)) continue;
    const int col = col_of<NT, P>(L, c);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) S.R[col * G::LDR + row_of(L, ti, r)] = U.v[c][ti][r];
  }
  // sum of log Dp over the live rows (wave 0), reduced through LDS
  __syncthreads();
  RM<NT, P> M;
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int col = col_of<NT, P>(L, c);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(L, ti, r);
        const double dr = S.dcur[row];
        const double dp = (loh && dr > 1.0) ? dr : 1.0;
        const double dm = (loh && dr > 1.0) ? 1.0 : dr;
        const double ut = tile_ok<NT, P>(L, c) ? S.R[row * G::LDR + col] : 0.0;
        Z.v[c][ti][r] = ut / dp;
        M.v[c][ti][r] = ut / dp + dm * T.v[c][ti][r];
      }
  }
  double lsum = 0.0;
  if constexpr (loh)
    for (int t = L.t; t < n; t += G::THREADS) lsum += log(fmax(S.dcur[t], 1.0));
  cpqr<NT, P, ELDS>(L, n, M, S);  // begins with barriers before S.R is overwritten
  for (int t = L.t; t < n; t += G::THREADS) lsum += log(fabs(S.R[S.perm[t] * G::LDR + t]));
  int neg = 0;
  for (int t = L.t; t < n; t += G::THREADS) neg += (S.R[S.perm[t] * G::LDR + t] < 0.0);
  // wave sums
  for (int m = 32; m >= 1; m >>= 1) {
    lsum += __shfl_xor(lsum, m);
    neg += __shfl_xor(neg, m);
  }
  if (L.l == 0) {
    S.red[0][L.w] = lsum;
    S.ired[G::P + L.w] = neg;
  }
  const double sq = refl_sign<NT, P, ELDS>(L, n, S);
  const double sp = perm_sign<NT, P, ELDS>(L, n, S);  // its barrier makes S.red visible
  double ld = 0.0;
  int ng = 0;
  for (int q = 0; q < G::P; ++q) {
    ld += S.red[0][q];
    ng += S.ired[G::P + q];
  }
  *logdet = ld;
  *sign = sgn_u * sq * sp * ((ng & 1) ? -1.0 : 1.0);
  apply_qt<NT, P, ELDS>(L, n, S, Z);
  back_subst<NT, P, ELDS>(L, n, S, Z);
}

// write G[perm[s]][c] = Z[s][c] (leading n x n block) to global memory
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void store_perm_rows(const Lane& L, const int n, const Smem<NT, P, ELDS>& S,
                                                const RM<NT, P>& Z, double* dst) {
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c) {
    const int col = col_of<NT, P>(L, c);
    if (!tile_ok<NT, P>(L, c) || col >= n) continue;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = row_of(L, ti, r);
        if (s < n) gmem(dst)[S.perm[s] * n + col] = Z.v[c][ti][r];
      }
  }
}

// ---------------------------------------------------------------------------
// slice exponentials v_q = exp(sgn alpha f_q) for `cnt` slices into S.vbuf
// (sgn = -1: the diagonal of B_q^{-1}).  Slice of buffer row s: q0 + dir*s.
// Ends with a barrier.
// vbuf[s][i] = exp(sgn alpha f_{q,i}) for the cnt slices q = q0, q0 + dir, ...
// (1 on padding rows).  Every field value is loaded before any is used
// (clamped in-range indices, padding set afterwards): one memory latency per
// call.  All threads; barriers before the stores and after them.
template <int NT, int P>
__device__ __forceinline__ void fill_vbuf_to(const Lane& L, double (*vbuf)[Geo<NT, P>::NP], const Inst& I,
                                             int q0, int dir, int cnt, double sgn) {
  using G = Geo<NT, P>;
  constexpr int IT = (G::KB * G::NP + G::THREADS - 1) / G::THREADS;
  double f[IT];
#pragma unroll
  for (int e = 0; e < IT; ++e) {
    const int idx = L.t + e * G::THREADS;
    const int s = min(idx / G::NP, cnt - 1), row = min(idx % G::NP, I.n - 1);
    f[e] = gmem(I.field)[(size_t)(q0 + dir * s - 1) * I.n + row];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < IT; ++e) {
    const int idx = L.t + e * G::THREADS;
    const int s = idx / G::NP, row = idx % G::NP;
    if (s < cnt) vbuf[s][row] = row < I.n ? exp(sgn * I.alpha * f[e]) : 1.0;
  }
  __syncthreads();
}

template <int NT, int P, bool ELDS>
__device__ __forceinline__ void fill_vbuf(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I, int q0,
                                          int dir, int cnt, double sgn = 1.0) {
  fill_vbuf_to<NT, P>(L, S.vbuf, I, q0, dir, cnt, sgn);
}

template <int NT, int P>
__device__ __forceinline__ void scale_rows(const Lane& L, RM<NT, P>& A, const double* v) {
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double s = v[row_of(L, ti, r)];
#pragma unroll
      for (int c = 0; c < Geo<NT, P>::CT; ++c) A.v[c][ti][r] *= s;
    }
}

// left operand: the slice exponential (or its transpose) in its swizzled,
// zero-padded order, whose block ((ti*NT + tk)*4 + r) holds exactly the 64
// A-operand values of one MFMA step: read from the LDS copy (ELDS; one base
// address, immediate offsets) or from HBM (one coalesced 512-byte load).
// The HBM copy is read through a buffer resource: the block offset is a
// compile-time constant that goes into the instruction's scalar offset, so
// no per-block 64-bit address is kept in vector registers (with NT^2 * 4
// blocks such addresses would be hoisted out of the slice loop and spilled).
template <int NT, int P, bool ELDS>
struct EOp {
  // up to two tiles per side the whole operand (at most 16 values per lane)
  // is read once, when the operator is made, and kept in registers
  static constexpr bool REG = !ELDS && NT <= 2;
  const double* sE;            // staged swizzled copy in LDS (ELDS)
  __amdgpu_buffer_rsrc_t rsw;  // swizzled copy in HBM
  int lane8;                   // byte offset of this lane in a block
  double er[REG ? NT * NT * 4 : 1];
  __device__ EOp(const double* s, const double* esw, int lane) : sE(s), lane8(lane * 8) {
    // the copy's address is the same for the whole workgroup
    const unsigned long long a = (unsigned long long)esw;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    rsw = __builtin_amdgcn_make_buffer_rsrc((void*)(((unsigned long long)hi << 32) | lo), (short)0,
                                            NT * NT * 4 * 512, 0x00020000);
    if constexpr (REG) {
#pragma unroll
      for (int b = 0; b < NT * NT * 4; ++b)
        er[b] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rsw, lane8, b * 512, 0));
    }
  }
  __device__ double operator()(int ti, int tk, int r, int, int) const {
    if (ELDS) return sE[((ti * NT + tk) * 4 + r) * 64 + (lane8 >> 3)];
    if constexpr (REG) return er[(ti * NT + tk) * 4 + r];
    return __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(rsw, lane8, ((ti * NT + tk) * 4 + r) * 512, 0));
  }
};

template <int NT, int P, bool ELDS>
__device__ __forceinline__ void stage_e(const Lane& L, Smem<NT, P, ELDS>& S, const double* esw) {
  using G = Geo<NT, P>;
  if (!ELDS) return;
  for (int idx = L.t; idx < G::NP * G::NP; idx += G::THREADS) S.E[idx] = gmem(esw)[idx];
  // visibility: the next fill_vbuf begins with a barrier
}

// A register matrix kept in a workgroup's private global scratch between
// uses: register [c][ti][r] of lane l of wave w at ((c NT + ti) 4 + r) 64 P +
// 64 w + l, so every access of a wave is one contiguous 512-byte block.  Each
// lane reads back only what it wrote itself.
template <int NT, int P>
__device__ __forceinline__ void scr_store(const Lane& L, const RM<NT, P>& A, double* p) {
  auto* q = gmem(p) + L.w * 64 + L.l;
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c)
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) q[((c * NT + ti) * 4 + r) * 64 * P] = A.v[c][ti][r];
}
template <int NT, int P>
__device__ __forceinline__ void scr_load(const Lane& L, RM<NT, P>& A, const double* p) {
  const auto* q = gmem(p) + L.w * 64 + L.l;
#pragma unroll
  for (int c = 0; c < Geo<NT, P>::CT; ++c)
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) A.v[c][ti][r] = q[((c * NT + ti) * 4 + r) * 64 * P];
}

// store one stage U | T | D | extra
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void store_stage(const Lane& L, const int n, const Smem<NT, P, ELDS>& S,
                                            const RM<NT, P>& U, const RM<NT, P>& T, double sgn_u,
                                            double* dst) {
  store_rm<NT, P>(L, U, dst, n);
  store_rm<NT, P>(L, T, dst + (size_t)n * n, n);
  for (int t = L.t; t < n; t += Geo<NT, P>::THREADS) gmem(dst)[2 * (size_t)n * n + t] = S.dnew[t];
  if (L.t == 0) gmem(dst)[2 * (size_t)n * n + n] = sgn_u;
}

// ---------------------------------------------------------------------------
// One stabilized sweep over the chain (Sec. 4.1):
//   forward  (SW_ADJ clear):  B_m ... B_1,           blocks b = 0 .. nb-1
//   backward (SW_ADJ set):    B_1^T ... B_m^T,        blocks b = nb-1 .. 0
// Block b holds slices b*k+1 .. min((b+1)k, m); both directions stabilize on
// the same slice boundaries, so forward stage j and backward stage j meet at
// tau = min(jk, m).  Per block:  W = X_block U,  W <- W D,  W P = Q R,
// U <- Q,  D <- |diag R|,  T <- D^{-1} R P^T T.
// The two chains of the single-decomposition G(tau_j, 0) (Sec. 6: the left
// one is B(tau_j, 0)^{-1} decomposed as it stands, unitary factor on the left):
//   SW_RIGHT:  B_m ... B_{tau_j+1}: the forward sweep from block j on;
//   SW_LEFT:   B_1^{-1} ... B_{tau_j}^{-1}: W <- B_q^{-1} W for q = tau_j
//              down to 1, B_q^{-1} = diag(exp(-alpha f_q)) expk^{-1}, folded
//              in every k slices counted from tau_j.
// UDT of W by the one-sided Jacobi SVD (Hestenes), the stabilizer the paper
// compares with the QR (Sec. 4.2): column pairs (p, q) of A = W are rotated
// until every pair is orthogonal to working accuracy,
// |a_p . a_q| <= n eps ||a_p|| ||a_q||, with the rotation
//   zeta = (a_q.a_q - a_p.a_p) / (2 a_p.a_q),  t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//   c = 1 / sqrt(1 + t^2),  s = c t,  a_p <- c a_p - s a_q,  a_q <- s a_p + c a_q,
// and the same rotation applied to rows p, q of T (T <- V^T T).  Then
// D = column norms in descending order (S.dnew; as LAPACK's gesvj returns
// them, which keeps the single-decomposition schemes' middle matrices graded
// in order), U = A D^{-1} with its columns and T with its rows in that
// order (into W and T).  A sits in S.R by column,
// T in S.E by row; the pairs of a round follow the circle method over the
// NP columns (each column in one pair per round, NP - 1 rounds per sweep),
// one pair per group of 8 lanes, one barrier per round; at most 60 sweeps.
// Sign of det U: every slice has a positive determinant and the rotations
// have determinant one, so det U has the sign of det W (that of the
// previous U) times that of the ordering permutation, which is returned in
// *psign.  Returns 0, or 1 without convergence.
template <int NT, int P>
__device__ __forceinline__ int jsvd_udt(const Lane& L, const int n, Smem<NT, P, true>& S, RM<NT, P>& W, RM<NT, P>& T,
                        double* psign) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  constexpr int GS = 8;                      // lanes per column pair
  constexpr int NG = G::THREADS / GS;        // pair groups
  constexpr int RPL = G::NP / GS;            // rows (of A) / columns (of T) per lane
  const int grp = L.t / GS, gl = L.t % GS;
  const double tol = n * 2.220446049250313e-16;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (!tile_ok<NT, P>(L, c)) continue;
    const int col = col_of<NT, P>(L, c);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(L, ti, r);
        S.R[col * G::LDR + row] = W.v[c][ti][r];
        S.E[row * G::LDR + col] = T.v[c][ti][r];
      }
  }
  int failed = 1;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (L.t == 0) S.ired[0] = 0;
    __syncthreads();
    for (int rd = 0; rd < G::NP - 1; ++rd) {
      for (int pk = grp; pk < G::NP / 2; pk += NG) {
        int p = pk == 0 ? G::NP - 1 : (rd + pk) % (G::NP - 1);
        int q = pk == 0 ? rd : (rd - pk + G::NP - 1) % (G::NP - 1);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        if (q >= n) continue;  // padding columns are zero
        double* ap = &S.R[p * G::LDR];
        double* aq = &S.R[q * G::LDR];
        double app = 0.0, aqq = 0.0, apq = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const double x = ap[gl + GS * i], y = aq[gl + GS * i];
          app = fma(x, x, app);
          aqq = fma(y, y, aqq);
          apq = fma(x, y, apq);
        }
#pragma unroll
        for (int o = 1; o < GS; o <<= 1) {
          app += __shfl_xor(app, o);
          aqq += __shfl_xor(aqq, o);
          apq += __shfl_xor(apq, o);
        }
        if (app == 0.0 || aqq == 0.0 || fabs(apq) <= tol * sqrt(app) * sqrt(aqq)) continue;
        const double zeta = (aqq - app) / (2.0 * apq);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        double* tp = &S.E[p * G::LDR];
        double* tq = &S.E[q * G::LDR];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int e = gl + GS * i;
          const double x = ap[e], y = aq[e];
          ap[e] = cs * x - sn * y;
          aq[e] = sn * x + cs * y;
          const double u = tp[e], v = tq[e];
          tp[e] = cs * u - sn * v;
          tq[e] = sn * u + cs * v;
        }
        if (gl == 0) S.ired[0] = 1;
      }
      __syncthreads();
    }
    const int rotated = S.ired[0];
    __syncthreads();
    if (!rotated) {
      failed = 0;
      break;
    }
  }
  // column norms (S.tau, free here), their descending order (ties by
  // index: S.sinv[rank] = column), D = S.dnew in that order, then
  // U = A D^{-1} and T back to registers in that order (padding: identity)
  for (int t = L.t; t < G::NP; t += G::THREADS) {
    double ss = 0.0;
    if (t < n)
      for (int i = 0; i < G::NP; ++i) ss = fma(S.R[t * G::LDR + i], S.R[t * G::LDR + i], ss);
    S.tau[t] = t < n ? sqrt(ss) : 1.0;
  }
  __syncthreads();
  for (int t = L.t; t < G::NP; t += G::THREADS) {
    int rk = t;
    if (t < n) {
      const double st = S.tau[t];
      rk = 0;
      for (int i = 0; i < n; ++i) rk += (S.tau[i] > st || (S.tau[i] == st && i < t)) ? 1 : 0;
    }
    S.sinv[rk] = t;
    S.dnew[rk] = S.tau[t];
  }
  __syncthreads();
  // parity of the ordering: (-1)^(n - number of cycles), one thread
  if (L.t == 0) {
    unsigned long long seen[(G::NP + 63) / 64] = {};
    int cycles = 0;
    for (int a = 0; a < n; ++a) {
      if (seen[a >> 6] & (1ull << (a & 63))) continue;
      ++cycles;
      for (int b = a; !(seen[b >> 6] & (1ull << (b & 63))); b = S.sinv[b]) seen[b >> 6] |= 1ull << (b & 63);
    }
    S.red[0][0] = ((n - cycles) & 1) ? -1.0 : 1.0;
  }
  __syncthreads();
  *psign = S.red[0][0];
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int col = col_of<NT, P>(L, c);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(L, ti, r);
        const bool ok = tile_ok<NT, P>(L, c);
        W.v[c][ti][r] = (ok && col < n) ? S.R[S.sinv[col] * G::LDR + row] / S.dnew[col]
                                        : (row == col ? 1.0 : 0.0);
        T.v[c][ti][r] = ok ? S.E[S.sinv[row] * G::LDR + col] : (row == col ? 1.0 : 0.0);
      }
  }
  return failed;
}

// DENSE: the slices are the dense matrices at I.field (B_q at
// field + (q-1) n n; forward sweeps, and backward ones over B_q^T),
// staged through S.E one at a time when ELDS, else read from global memory.
// TG: T is not held in registers across the block's slice products and
// QR; it lives in the workgroup's scratch `tscr` between blocks and is in
// registers only for its update (after the QR, before Q is formed, while
// the working matrix is parked in LDS), which frees one register matrix.
struct NoT {};
template <int NT, int P, bool ELDS, bool SVD = false, bool DENSE = false, bool TG = false, bool PSW = false>
__device__ __forceinline__ void sweep_one(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I, const int flags,
                          const int jpair, double* tscr = nullptr) {
  static_assert(!PSW || (DENSE && !ELDS), "pre-swizzled slices are dense and read from device memory");
  static_assert(!(TG && SVD), "the SVD stabilizer keeps T in registers");
  using G = Geo<NT, P>;
  // the SVD stabilizer keeps T in S.E, so E is read from its global copy
  constexpr bool EST = ELDS && !SVD && !DENSE;
  constexpr int CT = G::CT;
  const int n = I.n, m = I.m, k = I.k, nb = I.nb;
  const bool left = (flags & SW_LEFT) != 0, right = (flags & SW_RIGHT) != 0;
  const bool block = (flags & SW_BLOCK) != 0;
  const bool adj = (flags & SW_ADJ) != 0;
  const int64_t sd = stage_doubles(n);
  const int tauj = jpair * k < m ? jpair * k : m;
  const int s_lo = (right || block) ? jpair : 0;
  const int s_hi = left ? (tauj + k - 1) / k : (block ? jpair + 1 : nb);
  const double* e_op = left ? I.eswi : (adj ? I.eswt : I.esw);
  if constexpr (EST) stage_e<NT, P, ELDS>(L, S, e_op);
  // W holds U between blocks and the block product inside a block
  RM<NT, P> W;
  std::conditional_t<TG, NoT, RM<NT, P>> T;
  // TG: where the next T update finds T (0 identity, 1 forward stage
  // jpair, 2 the scratch)
  int tsrc = 0;
  double dcol[CT];
  if (block && jpair > 0) {
    // continue from forward stage jpair: W = U, T, column scales D
    const double* F0 = I.ckf + (size_t)(jpair - 1) * sd;
    load_rm<NT, P>(L, W, F0, n, false);
    if constexpr (TG) tsrc = 1;
    else load_rm<NT, P>(L, T, F0 + (size_t)n * n, n, false);
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int col = col_of<NT, P>(L, c);
      dcol[c] = col < n ? gmem(F0)[2 * (size_t)n * n + col] : 1.0;
    }
  } else {
    set_identity<NT, P>(L, W);
    if constexpr (!TG) set_identity<NT, P>(L, T);
#pragma unroll
    for (int c = 0; c < CT; ++c) dcol[c] = 1.0;
  }
  const EOp<NT, P, EST> eop{S.E, e_op, L.l};
  int svd_failed = 0;
  // sign of det U of the current factorization (the SVD path carries it)
  double sgn_run = (block && jpair > 0) ? gmem(I.ckf + (size_t)(jpair - 1) * sd)[2 * (size_t)n * n + n] : 1.0;

  for (int s = s_lo; s < s_hi; ++s) {
    const Lane L = lane_id_per_item();
    const int b = adj ? nb - 1 - s : s;
    int q0 = b * k + 1, q1 = (b + 1) * k < m ? (b + 1) * k : m;
    if (left) {
      q1 = tauj - s * k;
      q0 = q1 - k + 1 > 1 ? q1 - k + 1 : 1;
    }
    const int cnt = q1 - q0 + 1;
    if constexpr (DENSE) {
      // ELDS: each slice goes through registers into S.E; the next one is
      // loaded while the current product runs
      constexpr int PER = (G::NP * G::NP + G::THREADS - 1) / G::THREADS;
      double nxt[PER];
      auto fetch = [&](int q) {
        const double* Bq = I.field + (size_t)(q - 1) * n * n;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          const int idx = L.t + e * G::THREADS;
          const int i = idx / G::NP, kk = idx - i * G::NP;
          nxt[e] = gmem(Bq)[(size_t)min(i, n - 1) * n + min(kk, n - 1)];
        }
      };
      // forward: W <- B_q W for q = q0..q1; backward: W <- B_q^T W, q = q1..q0
      const int qa = adj ? q1 : q0, qs = adj ? -1 : 1;
      if constexpr (ELDS) fetch(qa);
      for (int t = 0; t < cnt; ++t) {
        const int q = qa + t * qs;
        const double* Bq = I.field + (size_t)(q - 1) * n * n;
        if constexpr (ELDS) {
          __syncthreads();  // the previous slice's readers of S.E are done
#pragma unroll
          for (int e = 0; e < PER; ++e) {
            const int idx = L.t + e * G::THREADS;
            const int i = idx / G::NP, kk = idx - i * G::NP;
            if (idx < G::NP * G::NP) S.E[i * G::LDR + kk] = (i < n && kk < n) ? nxt[e] : 0.0;
          }
          __syncthreads();
          if (t + 1 < cnt) fetch(q + qs);
          if (adj)
            gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.E[kk * G::LDR + i]; }, W, W);
          else
            gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.E[i * G::LDR + kk]; }, W, W);
        } else if constexpr (PSW) {
          // the slice in the swizzled, zero-padded operand layout (forward only)
          const EOp<NT, P, false> bop{nullptr, I.field + (size_t)(q - 1) * G::NP * G::NP, L.l};
          gemm_rb<NT, P>(L, bop, W, W);
        } else {
          gemm_gm<NT, P>(L, Bq, n, adj, W, W);
        }
      }
    } else {
      for (int c0 = 0; c0 < cnt; c0 += G::KB) {
        const int cn = (cnt - c0) < G::KB ? (cnt - c0) : G::KB;
        if (left) fill_vbuf<NT, P, ELDS>(L, S, I, q1 - c0, -1, cn, -1.0);
        else if (adj) fill_vbuf<NT, P, ELDS>(L, S, I, q1 - c0, -1, cn);
        else fill_vbuf<NT, P, ELDS>(L, S, I, q0 + c0, +1, cn);
        for (int s2 = 0; s2 < cn; ++s2) {
          if (!adj && !left) {
            scale_rows<NT, P>(L, W, S.vbuf[s2]);
            gemm_rb<NT, P>(L, eop, W, W);
          } else {
            gemm_rb<NT, P>(L, eop, W, W);
            scale_rows<NT, P>(L, W, S.vbuf[s2]);
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) W.v[c][ti][r] *= dcol[c];
    double* dst = nullptr;
    if (flags & SW_STORE) dst = adj ? (I.cka + (size_t)b * sd) : (I.ckf + (size_t)s * sd);
    else if ((flags & SW_LAST) && s == nb - 1) dst = I.fin;
    else if (left && s == s_hi - 1) dst = I.ckf + (size_t)(jpair - 1) * sd;
    else if (right && s == nb - 1) dst = I.cka + (size_t)jpair * sd;
    else if (block) dst = I.ckf + (size_t)jpair * sd;
    double sgn_u = 1.0;
    if constexpr (SVD) {
      double ps = 1.0;
      svd_failed |= jsvd_udt<NT, P>(L, n, S, W, T, &ps);
      sgn_u = sgn_run * ps;
      sgn_run = sgn_u;
    } else if constexpr (TG) {
      cpqr<NT, P, ELDS>(L, n, W, S);
      diag_r<NT, P, ELDS>(L, n, S);
      sgn_u = refl_sign<NT, P, ELDS>(L, n, S);
      {
        // W is parked in LDS: T takes its place in registers for the update
        RM<NT, P> Tr;
        if (tsrc == 2) scr_load<NT, P>(L, Tr, tscr);
        else if (tsrc == 1) load_rm<NT, P>(L, Tr, I.ckf + (size_t)(jpair - 1) * sd + (size_t)n * n, n, false);
        else set_identity<NT, P>(L, Tr);
        update_t<NT, P, ELDS>(L, S, Tr);
        if (s + 1 < s_hi) scr_store<NT, P>(L, Tr, tscr);
        tsrc = 2;
        if (dst) store_rm<NT, P>(L, Tr, dst + (size_t)n * n, n);
        if ((flags & SW_FINAL) && s + 1 == s_hi) store_rm<NT, P>(L, Tr, I.t_out, n);
      }
      form_q<NT, P, ELDS>(L, n, S, W);
    } else {
      cpqr<NT, P, ELDS>(L, n, W, S);
      diag_r<NT, P, ELDS>(L, n, S);
      sgn_u = refl_sign<NT, P, ELDS>(L, n, S);
      form_q<NT, P, ELDS>(L, n, S, W);
      update_t<NT, P, ELDS>(L, S, T);
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) dcol[c] = S.dnew[col_of<NT, P>(L, c)];
    if (dst) {
      if constexpr (TG) {
        store_rm<NT, P>(L, W, dst, n);
        for (int t = L.t; t < n; t += G::THREADS) gmem(dst)[2 * (size_t)n * n + t] = S.dnew[t];
        if (L.t == 0) gmem(dst)[2 * (size_t)n * n + n] = sgn_u;
      } else {
        store_stage<NT, P, ELDS>(L, n, S, W, T, sgn_u, dst);
      }
    }
    __syncthreads();
  }

  int bad = 0;
  for (int t = L.t; t < n; t += G::THREADS) {
    const double d = S.dnew[t];
    if (!isfinite(d) || !(d > 0.0)) bad = 1;
  }
  if (flags & SW_FINAL) {
    store_rm<NT, P>(L, W, I.u_out, n);
    if constexpr (!TG) store_rm<NT, P>(L, T, I.t_out, n);
    for (int t = L.t; t < n; t += G::THREADS) gmem(I.d_out)[t] = S.dnew[t];
  }
  if ((__any(bad) || svd_failed) && L.l == 0 && I.status) atomicOr(I.status, kStatusRange);
}

// Equal-time G, log|det| and sign from the final forward stage (Sec. 5.1).
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void pair_equal(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I) {
  using G = Geo<NT, P>;
  const int n = I.n;
  const double* F = I.fin;
  RM<NT, P> U, T, Z;
  load_rm<NT, P>(L, U, F, n, false);
  load_rm<NT, P>(L, T, F + (size_t)n * n, n, false);
  __syncthreads();
  int bad = 0;
  for (int t = L.t; t < G::NP; t += G::THREADS) {
    const double d = t < n ? gmem(F)[2 * (size_t)n * n + t] : 1.0;
    if (!isfinite(d) || !(d > 0.0)) bad = 1;
    S.dcur[t] = d;
  }
  const double sgn_u = gmem(F)[2 * (size_t)n * n + n];
  double ld, sg;
  if (I.scheme == 0)
    inv_one_plus<NT, P, ELDS, true>(L, n, S, U, T, sgn_u, Z, &ld, &sg);
  else
    inv_one_plus<NT, P, ELDS, false>(L, n, S, U, T, sgn_u, Z, &ld, &sg);
  if (!all_finite<NT, P>(L, Z) || !isfinite(ld)) bad = 1;
  if (I.g) store_perm_rows<NT, P, ELDS>(L, n, S, Z, I.g);
  if (L.t == 0) {
    if (I.logdet) *I.logdet = ld;
    if (I.sign) *I.sign = sg;
  }
  if (__any(bad) && L.l == 0 && I.status) atomicOr(I.status, kStatusRange);
  __syncthreads();
}

// The sweep kernel's work loop: items from the queue until it is empty.
template <int NT, int P, bool ELDS, bool SVD = false, bool DENSE = false, bool TG = false, bool PSW = false>
__device__ __forceinline__ void sweep_items(const Inst* __restrict__ insts, const SweepItem* __restrict__ items,
                                            int count, Queue* q, double* tscr) {
  __shared__ Smem<NT, P, ELDS> S;
  const Lane L = lane_id();
  // this workgroup's T scratch (TG): one register matrix, lanes contiguous;
  // for sizes whose factor store is in device memory, that store follows it
  constexpr size_t tdoubles = (size_t)Geo<NT, P>::CT * P * NT * 256;
  constexpr size_t rdoubles = Smem<NT, P, ELDS>::RG ? (size_t)Geo<NT, P>::NP * Geo<NT, P>::LDR : 0;
  double* ts = TG ? tscr + (size_t)blockIdx.x * (tdoubles + rdoubles) : nullptr;
  if constexpr (Smem<NT, P, ELDS>::RG) {
    static_assert(TG, "the factor store in device memory needs the workgroup scratch");
    if (L.t == 0) S.rg = ts + tdoubles;
  }
  for (;;) {
    __syncthreads();
    if (L.t == 0) S.item = atomicAdd(&q->next, 1);
    __syncthreads();
    // the item is the same for the whole workgroup: scalar loads of the item,
    // its instance and every pointer in it
    const int it = __builtin_amdgcn_readfirstlane(S.item);
    if (it >= count) break;
    const SweepItem wi = items[it];
    const Inst I = insts[wi.inst];
    sweep_one<NT, P, ELDS, SVD, DENSE, TG, PSW>(L, S, I, wi.flags, wi.j, ts);
  }
}

template <int NT, int P, bool ELDS, bool SVD = false, bool DENSE = false, bool TG = false, bool PSW = false>
__global__ __launch_bounds__(64 * P, minb_for(NT)) void k_sweep(const Inst* __restrict__ insts,
                                                            const SweepItem* __restrict__ items,
                                                            int count, Queue* q, double* tscr) {
  sweep_items<NT, P, ELDS, SVD, DENSE, TG, PSW>(insts, items, count, q, tscr);
}


// Block products of a chain's slices, P_j = B_{q1} ... B_{q0} for the k
// slices q0 = jk + 1 .. q1 = min((j+1)k, m) of block j (the product of k
// slices that the stabilized product of Sec. 4.1 then factorizes), each
// written row-major to I.prod + j n n.  One workgroup per (chain, block)
// item: P = E diag(v_q0) is E with its columns scaled, and every further
// slice is W <- E diag(v_q) W as in the sweep (rows scaled, then the MFMA
// product with the swizzled E from device memory).  A chain whose blocks
// have been multiplied out this way runs its stabilized sweep over the P_j
// with one factorization per product (dense slices, k = 1): the blocks'
// slice products, independent of each other, then fill the device instead
// of lying on the sweep's sequential path.
template <int NT, int P>
struct ProdSmem {
  double vbuf[Geo<NT, P>::KB][Geo<NT, P>::NP];
  int item;
};

template <int NT, int P>
__global__ __launch_bounds__(64 * P, 2) void k_prod(const Inst* __restrict__ insts,
                                                    const SweepItem* __restrict__ items, int count, Queue* q) {
  using G = Geo<NT, P>;
  __shared__ ProdSmem<NT, P> S;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) S.item = atomicAdd(&q->next, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(S.item);
    if (it >= count) break;
    const SweepItem wi = items[it];
    const Inst I = insts[wi.inst];
    const Lane L = lane_id_per_item();
    const int n = I.n, j = wi.j;
    const int q0 = j * I.k + 1, q1 = (j + 1) * I.k < I.m ? (j + 1) * I.k : I.m;
    const int cnt = q1 - q0 + 1;
    RM<NT, P> W;
    load_rm<NT, P>(L, W, I.expk, n, false);
    for (int c0 = 0; c0 < cnt; c0 += G::KB) {
      const Lane L = lane_id_per_item();
      const EOp<NT, P, false> eop{nullptr, I.esw, L.l};
      const int cn = (cnt - c0) < G::KB ? (cnt - c0) : G::KB;
      fill_vbuf_to<NT, P>(L, S.vbuf, I, q0 + c0, +1, cn, 1.0);
      for (int s2 = 0; s2 < cn; ++s2) {
        if (c0 + s2 == 0) {
#pragma unroll
          for (int c = 0; c < G::CT; ++c) {
            const double v = S.vbuf[0][col_of<NT, P>(L, c)];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
              for (int r = 0; r < 4; ++r) W.v[c][ti][r] *= v;
          }
        } else {
          scale_rows<NT, P>(L, W, S.vbuf[s2]);
          gemm_rb<NT, P>(L, eop, W, W);
        }
      }
    }
    // swizzled store: entry (i, kk) goes to block ((i/16) NT + kk/16) 4 + (kk%16)/4,
    // lane (kk%4) 16 + i%16 (the lane that takes it as an MFMA A operand)
    double* dst = I.prod + (size_t)j * G::NP * G::NP;
#pragma unroll
    for (int c = 0; c < G::CT; ++c) {
      if (!tile_ok<NT, P>(L, c)) continue;
      const int tc = L.w + P * c, kk = col_of<NT, P>(L, c);
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = row_of(L, ti, r);
          const int blk = ((ti * NT + tc) * 4 + (L.cl >> 2)) * 64 + (L.cl & 3) * 16 + (L.g + 4 * r);
          gmem(dst)[blk] = (i < n && kk < n) ? W.v[c][ti][r] : 0.0;
        }
    }
  }
}

// stage the n x n row-major global matrix src (identity if null) into the
// LDS matrix dst ([NP][LDR]: S.E or S.R), [row][col], zero padded; all
// threads, no barrier.  The loads go out in batches of eight per thread
// before any is stored (clamped in-range addresses, padding zeroed after
// the load), so a batch costs one memory latency instead of eight.
template <int NT, int P>
__device__ __forceinline__ void stage_to(const Lane& L, double* dst, const double* src, int n) {
  using G = Geo<NT, P>;
  {
    constexpr int TOT = G::NP * G::NP, IT = (TOT + G::THREADS - 1) / G::THREADS, CH = 8;
    if (src == nullptr) {
      for (int idx = L.t; idx < TOT; idx += G::THREADS) {
        const int i = idx / G::NP, k = idx - i * G::NP;
        dst[i * G::LDR + k] = (i == k && i < n) ? 1.0 : 0.0;
      }
      return;
    }
    const auto* g = gmem(src);
#pragma unroll
    for (int b = 0; b < IT; b += CH) {
      double x[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        const int idx = L.t + (b + q) * G::THREADS;
        const int i = idx / G::NP, k = idx - i * G::NP;
        x[q] = (b + q < IT) ? g[min(i, n - 1) * n + min(k, n - 1)] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        const int idx = L.t + (b + q) * G::THREADS;
        const int i = idx / G::NP, k = idx - i * G::NP;
        if (b + q < IT && idx < TOT) dst[i * G::LDR + k] = (i < n && k < n) ? x[q] : 0.0;
      }
    }
  }
}
// stage_to for two matrices at once: every load of both goes out before any
// store, so the pair costs one memory latency instead of one per batch of
// eight (where the loads of both fit in 16 values per thread; else one after
// the other, as for a null source)
template <int NT, int P>
__device__ __forceinline__ void stage_to2(const Lane& L, double* dst_a, const double* src_a, double* dst_b,
                                          const double* src_b, int n) {
  using G = Geo<NT, P>;
  constexpr int TOT = G::NP * G::NP, IT = (TOT + G::THREADS - 1) / G::THREADS;
  if constexpr (IT > 16) {
    stage_to<NT, P>(L, dst_a, src_a, n);
    stage_to<NT, P>(L, dst_b, src_b, n);
  } else {
    if (src_a == nullptr || src_b == nullptr) {
      stage_to<NT, P>(L, dst_a, src_a, n);
      stage_to<NT, P>(L, dst_b, src_b, n);
      return;
    }
    const auto* ga = gmem(src_a);
    const auto* gb = gmem(src_b);
    double xa[IT], xb[IT];
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int idx = L.t + q * G::THREADS;
      const int i = idx / G::NP, k = idx - i * G::NP;
      const size_t o = (size_t)min(i, n - 1) * n + min(k, n - 1);
      xa[q] = ga[o];
      xb[q] = gb[o];
    }
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int idx = L.t + q * G::THREADS;
      const int i = idx / G::NP, k = idx - i * G::NP;
      if (idx < TOT) {
        const bool in = i < n && k < n;
        dst_a[i * G::LDR + k] = in ? xa[q] : 0.0;
        dst_b[i * G::LDR + k] = in ? xb[q] : 0.0;
      }
    }
  }
}

template <int NT, int P, bool ELDS>
__device__ __forceinline__ void stage_mat(const Lane& L, Smem<NT, P, ELDS>& S, const double* src,
                                          int n) {
  if constexpr (ELDS) stage_to<NT, P>(L, S.E, src, n);
}

// register matrix from an LDS matrix ([NP][LDR]): B[row][col] = a[row][col]
// or its transpose
template <int NT, int P>
__device__ __forceinline__ void load_lds_rm(const Lane& L, const double* a, RM<NT, P>& B, bool trans) {
  using G = Geo<NT, P>;
#pragma unroll
  for (int c = 0; c < G::CT; ++c) {
    const int col = col_of<NT, P>(L, c);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(L, ti, r);
        B.v[c][ti][r] = tile_ok<NT, P>(L, c) ? (trans ? a[col * G::LDR + row] : a[row * G::LDR + col]) : 0.0;
      }
  }
}

// B operand from the staged matrix: B[row][col] = S.E[row][col] or its transpose
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void load_rm_staged(const Lane& L, const Smem<NT, P, ELDS>& S,
                                               RM<NT, P>& B, bool trans) {
  using G = Geo<NT, P>;
#pragma unroll
  for (int c = 0; c < G::CT; ++c) {
    const int col = col_of<NT, P>(L, c);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(L, ti, r);
        B.v[c][ti][r] = tile_ok<NT, P>(L, c) ? (trans ? S.E[col * G::LDR + row] : S.E[row * G::LDR + col]) : 0.0;
      }
  }
}

template <int NT, int P, bool ELDS, bool DENSE = false>
__device__ __forceinline__ void tdisp_outputs(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I, const int j,
                              const int ilo, const int ihi, const int32_t* __restrict__ l_list,
                              RM<NT, P>& Gm);

// ---------------------------------------------------------------------------
// Time-displaced G(tau_j, 0) from forward stage gmem(F)[j] = U1 D1 T1 (of
// B(tau_j, 0)) and backward stage A[j] = U2 D2 T2 (of B(beta, tau_j)^T),
// Sec. 6.1 inv_sum_loh with
//   U_L D_L X_L = B(tau,0)^{-1} = T1^{-1} D1^{-1} U1^T,
//   U_R D_R X_R = B(beta,tau)   = T2^T D2 U2^T,
// i.e. D_L = D1^{-1}, D_R = D2, X_L X_R^{-1} = U1^T U2, U_L^{-1} U_R = T1 T2^T:
//   Mid = D_Lm (U1^T U2) D_Rp^{-1} + D_Lp^{-1} (T1 T2^T) D_Rm
//   G(tau,0) = U2 D_Rp^{-1} Mid^{-1} D_Lp^{-1} T1.
// Then, for requested l inside the block, G(tau_l, 0) = B_l ... G(tau_j, 0)
// (Sec. 6, propagation form), never across more than k-1 slices.
template <int NT, int P, bool ELDS, bool DENSE = false>
__device__ __forceinline__ void pair_tdisp(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I, const int j,
                           const int ilo, const int ihi, const int32_t* __restrict__ l_list) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  const int n = I.n, m = I.m, k = I.k, nb = I.nb;
  const int64_t sd = stage_doubles(n);
  const double* F = j > 0 ? I.ckf + (size_t)(j - 1) * sd : nullptr;
  const double* A = j < nb ? I.cka + (size_t)j * sd : nullptr;
  const double* U1 = F;
  const double* T1 = F ? F + (size_t)n * n : nullptr;
  const double* D1 = F ? F + 2 * (size_t)n * n : nullptr;
  const double* U2 = A;
  const double* T2 = A ? A + (size_t)n * n : nullptr;
  const double* D2 = A ? A + 2 * (size_t)n * n : nullptr;

  // D1 and D2 in LDS (their entries are read per row and per column below)
  for (int t = L.t; t < G::NP; t += G::THREADS) {
    S.dcur[t] = (D1 && t < n) ? gmem(D1)[t] : 1.0;
    S.dnew[t] = (D2 && t < n) ? gmem(D2)[t] : 1.0;
  }
  RM<NT, P> B, P1, P2, Y;
  if constexpr (ELDS) {
    // operands staged through LDS with coalesced loads, two matrices per
    // round (S.R is free until the solve parks its factor there)
    __syncthreads();
    stage_to2<NT, P>(L, S.R, T2, S.E, T1, n);
    __syncthreads();
    load_lds_rm<NT, P>(L, S.R, B, true);  // T2^T
    gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.E[i * G::LDR + kk]; }, B,
                   P2);
    load_lds_rm<NT, P>(L, S.E, Y, false);  // T1 (right-hand sides)
    __syncthreads();
    stage_to2<NT, P>(L, S.R, U1, S.E, U2, n);  // U2 stays in S.E for the final product
    __syncthreads();
    load_lds_rm<NT, P>(L, S.E, B, false);  // U2
    gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.R[kk * G::LDR + i]; }, B,
                   P1);
  } else {
    load_rm<NT, P>(L, B, U2, n, false);
    gemm_gm<NT, P>(L, U1, n, true, B, P1);
    load_rm<NT, P>(L, B, T2, n, true);
    gemm_gm<NT, P>(L, T1, n, false, B, P2);
    __syncthreads();  // S.dcur, S.dnew written
  }
  // Mid = D_Lm (U1^T U2) D_Rp^{-1} + D_Lp^{-1} (T1 T2^T) D_Rm
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double d1 = S.dcur[row_of(L, ti, r)];
      const double lm = 1.0 / (d1 > 1.0 ? d1 : 1.0);  // D_Lm
      const double lpi = d1 < 1.0 ? d1 : 1.0;          // D_Lp^{-1}
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const double d2 = S.dnew[col_of<NT, P>(L, c) < G::NP ? col_of<NT, P>(L, c) : 0];
        const double rpi = 1.0 / (d2 > 1.0 ? d2 : 1.0);  // D_Rp^{-1}
        const double rm = d2 < 1.0 ? d2 : 1.0;            // D_Rm
        P1.v[c][ti][r] = lm * P1.v[c][ti][r] * rpi + lpi * P2.v[c][ti][r] * rm;
      }
    }
  // Y = D_Lp^{-1} T1 (without LDS staging it is loaded here, after the
  // products, so that it is not live in registers during them)
  if constexpr (!ELDS) load_rm<NT, P>(L, Y, T1, n, false);
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double d1 = S.dcur[row_of(L, ti, r)];
      const double lpi = d1 < 1.0 ? d1 : 1.0;  // D_Lp^{-1}
#pragma unroll
      for (int c = 0; c < CT; ++c) Y.v[c][ti][r] *= lpi;
    }
  // Y <- Mid^{-1} Y by Gaussian elimination with column pivoting (any
  // backward-stable solve of the middle matrix serves, Sec. 6.1); the rows
  // of the result come out in pivot order, S.perm
  __syncthreads();
  ge_solve<NT, P, ELDS>(L, n, P1, Y, S);
  // G = U2 D_Rp^{-1} P Z: row s of Z scaled by 1 / max(D2[perm s], 1), then
  // the product with the columns of U2 gathered by perm
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double d2 = S.dnew[S.perm[row_of(L, ti, r)]];
      const double rpi = 1.0 / (d2 > 1.0 ? d2 : 1.0);
#pragma unroll
      for (int c = 0; c < CT; ++c) Y.v[c][ti][r] *= rpi;
    }
  RM<NT, P> Gm;
  if constexpr (ELDS) {
    gemm_rb<NT, P>(L,
                   [&](int, int, int, int i, int s) -> double {
                     return s < n ? S.E[i * G::LDR + S.perm[s]] : 0.0;
                   },
                   Y, Gm);
  } else {
    gemm_gm_perm<NT, P>(L, U2, n, S.perm, Y, Gm);
  }
  if (!all_finite<NT, P>(L, Gm) && L.l == 0 && I.status) atomicOr(I.status, kStatusRange);
  tdisp_outputs<NT, P, ELDS, DENSE>(L, S, I, j, ilo, ihi, l_list, Gm);
}

// Outputs of stage pair j from Gm = G(tau_j, 0): l_list[ilo..ihi), ascending,
// each in [tau_j, tau_j + k), G(tau_l, 0) = B_l ... B_{tau_j + 1} G(tau_j, 0)
// (Sec. 6, propagation form).  DENSE: B_q is the n x n row-major matrix at
// I.field + (q - 1) n^2, staged through LDS (or read from HBM without it).
template <int NT, int P, bool ELDS, bool DENSE>
__device__ __forceinline__ void tdisp_outputs(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I, const int j,
                              const int ilo, const int ihi, const int32_t* __restrict__ l_list,
                              RM<NT, P>& Gm) {
  using G = Geo<NT, P>;
  const int n = I.n, m = I.m, k = I.k;
  const int tj = j * k < m ? j * k : m;
  int lc = tj;
  if constexpr (DENSE) {
    for (int idx = ilo; idx < ihi; ++idx) {
      const int l = l_list[idx];
      for (int q = lc + 1; q <= l; ++q) {
        const double* Bq = I.field + (size_t)(q - 1) * n * n;
        if constexpr (ELDS) {
          __syncthreads();
          stage_mat<NT, P, ELDS>(L, S, Bq, n);
          __syncthreads();
          gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.E[i * G::LDR + kk]; }, Gm,
                         Gm);
        } else {
          gemm_gm<NT, P>(L, Bq, n, false, Gm, Gm);
        }
      }
      lc = l;
      store_rm<NT, P>(L, Gm, I.gt + (size_t)idx * n * n, n);
    }
    __syncthreads();
    return;
  }
  if (ELDS && ihi > ilo && l_list[ihi - 1] > tj) {
    // propagation ahead: stage the swizzled slice exponential in LDS
    __syncthreads();
    stage_e<NT, P, ELDS>(L, S, I.esw);
  }
  const EOp<NT, P, ELDS> eop{S.E, I.esw, L.l};
  for (int idx = ilo; idx < ihi; ++idx) {
    const int l = l_list[idx];
    const int steps = l - lc;
    for (int c0 = 0; c0 < steps; c0 += G::KB) {
      const int cn = (steps - c0) < G::KB ? (steps - c0) : G::KB;
      fill_vbuf<NT, P, ELDS>(L, S, I, lc + c0 + 1, +1, cn);
      for (int s2 = 0; s2 < cn; ++s2) {
        scale_rows<NT, P>(L, Gm, S.vbuf[s2]);
        gemm_rb<NT, P>(L, eop, Gm, Gm);
      }
    }
    lc = l;
    store_rm<NT, P>(L, Gm, I.gt + (size_t)idx * n * n, n);
  }
  __syncthreads();
}

// Time-displaced G(tau_j, 0) by the single-decomposition scheme (Sec. 6.1,
// inv_sum), from the two chains of stage pair j built by SW_LEFT / SW_RIGHT:
//   B(tau_j, 0)^{-1} = U_L D_L X_L   (ckf[j-1]; identity for j = 0)
//   B(beta, tau_j)   = U_R D_R X_R   (cka[j];   identity for j = nb)
//   G(tau_j, 0) = [U_L D_L X_L + U_R D_R X_R]^{-1} = X_R^{-1} Mid^{-1} U_L^T,
//   Mid = D_L (X_L X_R^{-1}) + (U_L^T U_R) D_R,
// with D_L and D_R unsplit and Mid inverted through its pivoted QR.  X_R^{-1}
// comes from the pivoted QR of X_R and is written over X_R in the stage (this
// item is the only reader of cka[j]).  Then the outputs of the pair as in
// the split scheme.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void pair_tdisp_plain(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I, const int j,
                                 const int ilo, const int ihi, const int32_t* __restrict__ l_list) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  const int n = I.n, nb = I.nb;
  const int64_t sd = stage_doubles(n);
  const double* F = j > 0 ? I.ckf + (size_t)(j - 1) * sd : nullptr;
  double* A = j < nb ? I.cka + (size_t)j * sd : nullptr;
  const double* UL = F;
  const double* XL = F ? F + (size_t)n * n : nullptr;
  const double* DL = F ? F + 2 * (size_t)n * n : nullptr;
  const double* UR = A;
  double* XRi = A ? A + (size_t)n * n : nullptr;
  const double* DR = A ? A + 2 * (size_t)n * n : nullptr;

  RM<NT, P> B, P1, P2;
  if (A) {
    // X_R P = Q R  ->  X_R^{-1} = P R^{-1} Q^T
    load_rm<NT, P>(L, P1, XRi, n, false);
    __syncthreads();
    cpqr<NT, P, ELDS>(L, n, P1, S);
    set_identity<NT, P>(L, B);
    apply_qt<NT, P, ELDS>(L, n, S, B);
    back_subst<NT, P, ELDS>(L, n, S, B);
    store_perm_rows<NT, P, ELDS>(L, n, S, B, XRi);
    __threadfence_block();
    __syncthreads();
  }
  // P1 = X_L X_R^{-1},  P2 = U_L^T U_R
  load_rm<NT, P>(L, B, XRi, n, false);
  gemm_gm<NT, P>(L, XL, n, false, B, P1);
  load_rm<NT, P>(L, B, UR, n, false);
  gemm_gm<NT, P>(L, UL, n, true, B, P2);
  double drc[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int col = col_of<NT, P>(L, c);
    drc[c] = (DR && col < n) ? gmem(DR)[col] : 1.0;
  }
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row_of(L, ti, r);
      const double dl = (DL && row < n) ? gmem(DL)[row] : 1.0;
#pragma unroll
      for (int c = 0; c < CT; ++c) P1.v[c][ti][r] = dl * P1.v[c][ti][r] + P2.v[c][ti][r] * drc[c];
    }
  __syncthreads();
  cpqr<NT, P, ELDS>(L, n, P1, S);
  // Mid^{-1} U_L^T = P Z,  Z = R^{-1} Q^T U_L^T
  RM<NT, P> Y;
  load_rm<NT, P>(L, Y, UL, n, true);
  apply_qt<NT, P, ELDS>(L, n, S, Y);
  back_subst<NT, P, ELDS>(L, n, S, Y);
  // G = X_R^{-1} P Z:  A(i, s) = X_R^{-1}[i][perm s]
  RM<NT, P> Gm;
  gemm_gm_perm<NT, P>(L, XRi, n, S.perm, Y, Gm);
  if (!all_finite<NT, P>(L, Gm) && L.l == 0 && I.status) atomicOr(I.status, kStatusRange);
  tdisp_outputs<NT, P, ELDS>(L, S, I, j, ilo, ihi, l_list, Gm);
}

// G_{jk+1} = [1 + B(tau_j,0) B(beta,tau_j)]^{-1} from forward stage j and
// backward stage j (App. A.1): udt(D1 (T1 T2^T) D2) = u d t, U = U1 u,
// T = t U2^T, then Loh's equal-time inversion; written to S.R row-major
// ([row][col], padding as identity), ends with a barrier.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void block_start_g(const Lane L, Smem<NT, P, ELDS>& S, const Inst& I, const int j) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  const int n = I.n, nb = I.nb;
  const int64_t sd = stage_doubles(n);
  const double* F = j > 0 ? I.ckf + (size_t)(j - 1) * sd : nullptr;
  const double* A = j < nb ? I.cka + (size_t)j * sd : nullptr;
  const double* U1 = F;
  const double* T1 = F ? F + (size_t)n * n : nullptr;
  const double* D1 = F ? F + 2 * (size_t)n * n : nullptr;
  const double* U2 = A;
  const double* T2 = A ? A + (size_t)n * n : nullptr;
  const double* D2 = A ? A + 2 * (size_t)n * n : nullptr;

  RM<NT, P> B, Mm;
  if constexpr (ELDS) {
    __syncthreads();
    stage_mat<NT, P, ELDS>(L, S, T2, n);
    __syncthreads();
    load_rm_staged<NT, P, ELDS>(L, S, B, true);  // T2^T
    __syncthreads();
    stage_mat<NT, P, ELDS>(L, S, T1, n);
    __syncthreads();
    gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.E[i * G::LDR + kk]; }, B,
                   Mm);
  } else {
    load_rm<NT, P>(L, B, T2, n, true);
    gemm_gm<NT, P>(L, T1, n, false, B, Mm);
  }
  // D1 (in S.tau) and D2 (in S.dcur), both free until the QR below
  __syncthreads();
  for (int t = L.t; t < G::NP; t += G::THREADS) {
    S.tau[t] = (D1 && t < n) ? gmem(D1)[t] : 1.0;
    S.dcur[t] = (D2 && t < n) ? gmem(D2)[t] : 1.0;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const double d2 = S.dcur[col_of<NT, P>(L, c) < G::NP ? col_of<NT, P>(L, c) : 0];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) Mm.v[c][ti][r] *= S.tau[row_of(L, ti, r)] * d2;
  }
  __syncthreads();
  cpqr<NT, P, ELDS>(L, n, Mm, S);
  diag_r<NT, P, ELDS>(L, n, S);
  RM<NT, P> u, Tm, Um;
  form_q<NT, P, ELDS>(L, n, S, u);
  if constexpr (ELDS) {
    __syncthreads();
    stage_mat<NT, P, ELDS>(L, S, U2, n);
    __syncthreads();
    load_rm_staged<NT, P, ELDS>(L, S, B, true);  // U2^T
    __syncthreads();
    stage_mat<NT, P, ELDS>(L, S, U1, n);
    __syncthreads();
  } else {
    load_rm<NT, P>(L, B, U2, n, true);  // U2^T
  }
  gemm_rb<NT, P>(L, RPtOp<NT, P, ELDS>{S}, B, Tm);
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) Tm.v[c][ti][r] /= S.dnew[row_of(L, ti, r)];
  if constexpr (ELDS) {
    gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.E[i * G::LDR + kk]; }, u,
                   Um);
  } else {
    gemm_gm<NT, P>(L, U1, n, false, u, Um);
  }
  for (int t = L.t; t < G::NP; t += G::THREADS) S.dcur[t] = S.dnew[t];
  RM<NT, P> Z;
  double ld, sg;
  inv_one_plus<NT, P, ELDS>(L, n, S, Um, Tm, 1.0, Z, &ld, &sg);
  // G_l into LDS, row-major [row][col]
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (!tile_ok<NT, P>(L, c)) continue;
    const int col = col_of<NT, P>(L, c);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = row_of(L, ti, r);
        const int row = s < n ? S.perm[s] : s;
        S.R[row * G::LDR + col] = (s < n && col < n) ? Z.v[c][ti][r] : (row == col ? 1.0 : 0.0);
      }
  }
  __syncthreads();
}

// Gradient rows for slices l = j*k+1 .. min((j+1)k, m): G_{jk+1} from the
// stage pair (block_start_g), then G_{l+1} = B_l G_l B_l^{-1} and
//   grad[l-1][i] = alpha (1 - G_l)_ii.
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void pair_grad(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I, const int j) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  const int n = I.n, m = I.m, k = I.k;
  block_start_g<NT, P, ELDS>(L, S, I, j);
  const int l0 = j * k + 1, l1 = (j + 1) * k < m ? (j + 1) * k : m;
  bool bad = false;
  for (int t = L.t; t < n; t += G::THREADS) {
    const double gii = S.R[t * G::LDR + t];
    bad |= !isfinite(gii);
    gmem(I.grad)[(size_t)(l0 - 1) * n + t] = I.alpha * (1.0 - gii);
  }
  // the wraps G_{l+1} = E (diag(v_l) G_l diag(1/v_l)) E^{-1}: E^{-1} in
  // registers and E staged in LDS once per item, v = exp(alpha f_l) once per
  // row; G stays in S.R (row-major) between slices
  RM<NT, P> Ei;
  if (l0 < l1) {
    load_rm<NT, P>(L, Ei, I.expk_inv, n, false);
    stage_e<NT, P, ELDS>(L, S, I.esw);  // visible after the first barrier below
  }
  for (int l = l0; l < l1; ++l) {
    const double* fl = I.field + (size_t)(l - 1) * n;
    __syncthreads();  // the previous slice's readers of S.R and S.vbuf are done
    for (int t = L.t; t < G::NP; t += G::THREADS) {
      const double e = t < n ? exp(I.alpha * gmem(fl)[t]) : 1.0;
      S.vbuf[0][t] = e;
      S.vbuf[1][t] = 1.0 / e;
    }
    __syncthreads();
    for (int idx = L.t; idx < n * n; idx += G::THREADS) {
      const int r = idx / n, c = idx - r * n;
      S.R[r * G::LDR + c] *= S.vbuf[0][r] * S.vbuf[1][c];
    }
    __syncthreads();
    RM<NT, P> Yr, Gn;
    gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.R[i * G::LDR + kk]; }, Ei, Yr);
    gemm_rb<NT, P>(L, EOp<NT, P, ELDS>{S.E, I.esw, L.l}, Yr, Gn);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      if (!tile_ok<NT, P>(L, c)) continue;
      const int col = col_of<NT, P>(L, c);
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) S.R[row_of(L, ti, r) * G::LDR + col] = Gn.v[c][ti][r];
    }
    __syncthreads();
    for (int t = L.t; t < n; t += G::THREADS) {
      const double gii = S.R[t * G::LDR + t];
      bad |= !isfinite(gii);
      gmem(I.grad)[(size_t)l * n + t] = I.alpha * (1.0 - gii);
    }
  }
  if (__any(bad) && L.l == 0 && I.status) atomicOr(I.status, kStatusRange);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Local updates (the determinant ratios of single flips, Sec. 2): block j of
// a sweep over the slices l = jk+1 .. min((j+1)k, m) and, in each, the sites
// i = 0 .. n-1 in order.  Flipping f_{l,i} -> -f_{l,i} multiplies B_l by
// 1 + Delta e_i e_i^T, Delta = exp(-2 alpha f_{l,i}) - 1, and det(1 + ...)
// of the chain whose rightmost factor is B_l by R = 1 + Delta (1 - G_l)_ii;
// the flip is accepted when u_{l,i} < |prod_flavours R| (the flavours share
// the field) and then every flavour's G_l becomes
//   G - (e_i - G e_i) (Delta / R) (e_i^T G)        (Sherman-Morrison),
// the field entry is negated, and after the last site of slice l
// G_{l+1} = B_l G_l B_l^{-1} with the updated B_l.  G_{jk+1} comes from the
// stage pair (block_start_g, in its own launch with one workgroup per
// flavour, PAIR_BSTART): forward stages rebuilt from the updated field
// (SW_BLOCK), backward stages of the slices after the block (untouched so
// far in the sweep).  Both flavours' G stay in registers; the owner of
// column i publishes that column of each through LDS, one barrier per site,
// and every wave takes the same decision from the same values.

// G <- E (diag(v) G diag(1/v)) E^{-1}: the wrap of G across one slice
// B = E diag(v), v = exp(alpha f) of the slice's field (v at vv[0..NP),
// 1/v at vv[NP..2NP), staged in LDS, 1 in the padding); G in registers is
// scaled, parked in LDS as the left operand of G E^{-1} (E^{-1} in registers,
// zero padded), and E comes from its swizzled copy, staged in S.E when
// `staged` (ELDS), else read from global memory.  Starts with a barrier (the
// caller's staging of vv and S.E, and any earlier reader of S.R).
template <int NT, int P, bool ELDS>
__device__ __forceinline__ void wrap_local(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I, const double* vv,
                           const RM<NT, P>& Einv, bool staged, RM<NT, P>& Gx) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (!tile_ok<NT, P>(L, c)) continue;
    const int col = col_of<NT, P>(L, c);
    const double sc = vv[G::NP + col];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_of(L, ti, r);
        S.R[row * G::LDR + col] = Gx.v[c][ti][r] * vv[row] * sc;
      }
  }
  __syncthreads();
  RM<NT, P> Yr;
  gemm_rb<NT, P>(L, [&](int, int, int, int i, int kk) -> double { return S.R[i * G::LDR + kk]; }, Einv, Yr);
  if (ELDS && staged)
    gemm_rb<NT, P>(L, EOp<NT, P, ELDS>{S.E, I.esw, L.l}, Yr, Gx);
  else
    gemm_rb<NT, P>(L, EOp<NT, P, false>{nullptr, I.esw, L.l}, Yr, Gx);
}

template <int NT, int P, bool ELDS>
__device__ __forceinline__ void pair_local(const Lane& L, Smem<NT, P, ELDS>& S, const Inst& I0, const Inst& I1,
                                           const int nf, const int j) {
  using G = Geo<NT, P>;
  constexpr int CT = G::CT;
  const int n = I0.n, m = I0.m, k = I0.k;
  const int l0 = j * k + 1, l1 = (j + 1) * k < m ? (j + 1) * k : m;
  // G at the block start (PAIR_BSTART, one workgroup per flavour) and E^{-1}
  // of each flavour, held in registers for the block
  RM<NT, P> Ga, Gb, Eia, Eib;
  load_rm<NT, P>(L, Ga, I0.g, n, false);
  load_rm<NT, P>(L, Eia, I0.expk_inv, n, false);
  if (nf > 1) {
    load_rm<NT, P>(L, Gb, I1.g, n, false);
    load_rm<NT, P>(L, Eib, I1.expk_inv, n, false);
  } else {
    set_identity<NT, P>(L, Gb);
    set_identity<NT, P>(L, Eib);
  }
  // E of the first flavour staged in LDS (read by the wraps after a barrier);
  // the second flavour shares it when its E is the same array
  stage_e<NT, P, ELDS>(L, S, I0.esw);
  const bool eb_staged = I1.esw == I0.esw;
  double* fld = const_cast<double*>(I0.field);
  // Delta takes two values per flavour (f = +-1 for Hirsch's field; any
  // other value falls back to the exponential)
  const double dap = exp(-2.0 * I0.alpha) - 1.0, dam = exp(2.0 * I0.alpha) - 1.0;
  const double dbp = exp(-2.0 * I1.alpha) - 1.0, dbm = exp(2.0 * I1.alpha) - 1.0;
  // the slice's field row and uniform numbers, staged in LDS (S.vbuf rows 0,
  // 1); the column of site i goes to rows 2 + 2 (i % 2) and 3 + 2 (i % 2):
  // with two buffers one barrier per site suffices (site i + 1 writes the
  // other buffer, and site i + 2 writes this one only after every wave has
  // passed the barrier of site i + 1, that is, finished reading site i).
  // Row 6 receives the field after the decisions (written by thread 0, read
  // only after the slice)
  const double* frow = S.vbuf[0];
  const double* urow = S.vbuf[1];
  double* fnew = S.vbuf[6];
  int nacc = 0;
  bool bad = false;
  for (int l = l0; l <= l1; ++l) {
    __syncthreads();
    for (int t = L.t; t < n; t += G::THREADS) {
      S.vbuf[0][t] = gmem(fld)[(size_t)(l - 1) * n + t];
      S.vbuf[1][t] = gmem(I0.unif)[(size_t)(l - 1) * n + t];
    }
    __syncthreads();
    // site i = 16 ti + 4 r + g sits in register [.][ti][r] of lane group g:
    // ti and r unrolled, so every register index below is static
    static_for<NT>([&](auto tic) {
      constexpr int ti = decltype(tic)::value;
      static_for<4>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
#pragma unroll 1
        for (int g = 0; g < 4; ++g) {
          const int i = 16 * ti + 4 * r + g;
          if (i >= n) break;
          double* ca = S.vbuf[2 + 2 * (g & 1)];
          double* cb = S.vbuf[3 + 2 * (g & 1)];
          // the lanes holding column i publish G e_i - e_i (both flavours):
          // then x = e_i - G e_i is minus the published column and 1 - G_ii
          // minus its entry i
          if (L.w == ti % P && L.cl == 4 * r + g) {
            constexpr int c = ti / P;
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
#pragma unroll
              for (int rr = 0; rr < 4; ++rr) {
                const double dg = (tt == ti && rr == r && L.g == g) ? 1.0 : 0.0;
                ca[row_of(L, tt, rr)] = Ga.v[c][tt][rr] - dg;
                cb[row_of(L, tt, rr)] = Gb.v[c][tt][rr] - dg;
              }
          }
          // row i of G on this wave's columns (y), while the column is in flight
          double ya[CT], yb[CT];
#pragma unroll
          for (int c = 0; c < CT; ++c) {
            ya[c] = sum_col(L.g == g ? Ga.v[c][ti][r] : 0.0);
            yb[c] = nf > 1 ? sum_col(L.g == g ? Gb.v[c][ti][r] : 0.0) : 0.0;
          }
          __syncthreads();
          // every LDS value of the site, read at once
          const double s = frow[i], u = urow[i], omga = -ca[i], omgb = -cb[i];
          double xa[NT][4], xb[NT][4];
#pragma unroll
          for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              xa[tt][rr] = ca[row_of(L, tt, rr)];
              xb[tt][rr] = cb[row_of(L, tt, rr)];
            }
          double da = s == 1.0 ? dap : dam, db = s == 1.0 ? dbp : dbm;
          if (s != 1.0 && s != -1.0) {  // the same branch in every lane
            da = exp(-2.0 * I0.alpha * s) - 1.0;
            db = exp(-2.0 * I1.alpha * s) - 1.0;
          }
          const double ra = 1.0 + da * omga;
          double rb = 1.0;
          if (nf > 1)
            rb = 1.0 + db * omgb;
          else
            db = 0.0;
          bad = bad || !isfinite(ra) || !isfinite(rb);
          const bool acc = u < fabs(ra * rb);
          // G <- G - x (Delta / R) y^T (Sherman-Morrison) when accepted; the
          // coefficient is an exact zero otherwise, which leaves G unchanged
          const double qa = acc ? da / ra : 0.0;
          const double qb = acc && nf > 1 ? db / rb : 0.0;
#pragma unroll
          for (int c = 0; c < CT; ++c) {
            const double ya_c = ya[c] * qa, yb_c = yb[c] * qb;
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
#pragma unroll
              for (int rr = 0; rr < 4; ++rr) {
                Ga.v[c][tt][rr] = fma(xa[tt][rr], ya_c, Ga.v[c][tt][rr]);
                Gb.v[c][tt][rr] = fma(xb[tt][rr], yb_c, Gb.v[c][tt][rr]);
              }
          }
          if (L.t == 0) {
            if (acc) gmem(fld)[(size_t)(l - 1) * n + i] = -s;
            fnew[i] = acc ? -s : s;
          }
          nacc += acc ? 1 : 0;
        }
      });
    });
    if (l < l1) {
      __syncthreads();  // fnew complete, the column buffers free
      double* va = S.vbuf[2];
      double* vb = S.vbuf[4];
      for (int t = L.t; t < G::NP; t += G::THREADS) {
        const double f = t < n ? fnew[t] : 0.0;
        const double ea = exp(I0.alpha * f), eb = exp(I1.alpha * f);
        va[t] = ea;
        va[G::NP + t] = 1.0 / ea;
        vb[t] = eb;
        vb[G::NP + t] = 1.0 / eb;
      }
      wrap_local<NT, P, ELDS>(L, S, I0, va, Eia, true, Ga);
      if (nf > 1) wrap_local<NT, P, ELDS>(L, S, I1, vb, Eib, eb_staged, Gb);
    }
  }
  if (L.t == 0 && I0.nacc) atomicAdd(I0.nacc, nacc);
  if (bad && L.t == 0 && I0.status) atomicOr(I0.status, kStatusRange);
  __syncthreads();
}

template <int NT, int P, bool ELDS, int MODE>
__global__ __launch_bounds__(64 * P, minb_pair(NT, MODE)) void k_pair(
    const Inst* __restrict__ insts, const PairItem* __restrict__ items, int count,
    const int32_t* __restrict__ l_list, Queue* q) {
  __shared__ Smem<NT, P, ELDS> S;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) S.item = atomicAdd(&q->next, 1);
    __syncthreads();
    // the item is the same for the whole workgroup: scalar loads of the item,
    // its instance and every pointer in it
    const int it = __builtin_amdgcn_readfirstlane(S.item);
    if (it >= count) break;
    const PairItem wi = items[it];
    const Inst I = insts[wi.inst];
    const Lane L = lane_id_per_item();
    if constexpr (MODE == PAIR_LOCAL) {
      const Inst I1 = wi.ilo > 1 ? insts[wi.inst + 1] : I;
      pair_local<NT, P, ELDS>(L, S, I, I1, wi.ilo, wi.j);
      continue;
    }
    if constexpr (MODE == PAIR_BSTART) {
      // G at the start of block j (row-major in S.R) -> I.g
      block_start_g<NT, P, ELDS>(L, S, I, wi.j);
      const int n = I.n;
      for (int t = L.t; t < n * n; t += Geo<NT, P>::THREADS)
        gmem(I.g)[t] = S.R[(t / n) * Geo<NT, P>::LDR + t % n];
      continue;
    }
    if constexpr (MODE == PAIR_TDISP) pair_tdisp<NT, P, ELDS>(L, S, I, wi.j, wi.ilo, wi.ihi, l_list);
    else if constexpr (MODE == PAIR_TDISP_DENSE)
      pair_tdisp<NT, P, ELDS, true>(L, S, I, wi.j, wi.ilo, wi.ihi, l_list);
    else if constexpr (MODE == PAIR_TDISP_PLAIN)
      pair_tdisp_plain<NT, P, ELDS>(L, S, I, wi.j, wi.ilo, wi.ihi, l_list);
    else if constexpr (MODE == PAIR_GRAD) pair_grad<NT, P, ELDS>(L, S, I, wi.j);
    else pair_equal<NT, P, ELDS>(L, S, I);
  }
}

// ---------------------------------------------------------------------------
// plain UDT of independent matrices (Sec. 4.2.2): W P = Q R,
// U = Q, D = |diag R|, T = D^{-1} R P^T
template <int NT, int P>
__global__ __launch_bounds__(64 * P) void k_udt(int n, int count, const double* __restrict__ w,
                                                          double* u, double* d, double* t) {
  using G = Geo<NT, P>;
  __shared__ Smem<NT, P, false> S;
  const Lane L = lane_id();
  for (int b = blockIdx.x; b < count; b += gridDim.x) {
    const size_t off = (size_t)b * n * n;
    RM<NT, P> W, Q, T;
    load_rm<NT, P>(L, W, w + off, n, false);
    __syncthreads();
    cpqr<NT, P, false>(L, n, W, S);
    diag_r<NT, P, false>(L, n, S);
    form_q<NT, P, false>(L, n, S, Q);
    store_rm<NT, P>(L, Q, u + off, n);
    set_identity<NT, P>(L, T);
    update_t<NT, P, false>(L, S, T);
    store_rm<NT, P>(L, T, t + off, n);
    for (int i = L.t; i < n; i += G::THREADS) d[(size_t)b * n + i] = S.dnew[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// M <- left * M * right for `count` n x n row-major matrices given by a
// device table of pointers (used to turn results for the slices E diag(v_l)
// into those of the symmetric slices E^{1/2} diag(v_l) E^{1/2}, Sec. 2).
// One workgroup per matrix in a grid-stride loop; `right` stays in registers
// for the whole launch.
template <int NT, int P>
__global__ __launch_bounds__(64 * P) void k_similarity(int n, int count, double* const* __restrict__ mats,
                                                       const double* __restrict__ left,
                                                       const double* __restrict__ right) {
  const Lane L = lane_id();
  RM<NT, P> R, X, Y;
  load_rm<NT, P>(L, R, right, n, false);
  for (int b = blockIdx.x; b < count; b += gridDim.x) {
    double* M = gmem(mats)[b];
    // X = M right
    gemm_gm<NT, P>(L, M, n, false, R, X);
    // every wave has read all of M before any wave writes it back
    __syncthreads();
    // Y = left X
    gemm_gm<NT, P>(L, left, n, false, X, Y);
    store_rm<NT, P>(L, Y, M, n);
  }
}

// ---------------------------------------------------------------------------
// per-tile-count launchers (instantiated once per NT in sdq_nt.hip)

// waves per chain: one per 16-column tile, at most four
constexpr int waves_for(int nt) { return nt < 4 ? nt : 4; }
// LDS-staged slice exponential: where it still leaves room for useful occupancy
constexpr bool lds_variant(int nt) { return nt >= 3 && nt <= 5; }

template <int NT>
struct Launch {
  static constexpr int P = waves_for(NT);
  static constexpr bool kLds = lds_variant(NT);
  static constexpr bool kPairLds = NT <= 5;  // operand staging buffer fits beside the factor store
  static constexpr bool kSvd = NT <= 5;  // A and T of the Jacobi SVD both fit in LDS
  // the dense-slice sweep (variant 3) is instantiated in its own translation
  // unit (sdq_nt_dense.hip), so that it leaves the code of these alone
  static constexpr bool kDenseLds = NT <= 5;  // a dense slice staged beside the factor store
  static hipError_t dense_sweep(const Inst* inst, const SweepItem* items, int count, Queue* q, int grid,
                                hipStream_t s) {
    hipLaunchKernelGGL((k_sweep<NT, P, kDenseLds, false, true>), dim3(grid), dim3(Geo<NT, P>::THREADS), 0, s,
                       inst, items, count, q, (double*)nullptr);
    return hipGetLastError();
  }
  static hipError_t dense_info(KernelInfo* out) {
    return info_of(k_sweep<NT, P, kDenseLds, false, true>, (int)sizeof(Smem<NT, P, kDenseLds>), out);
  }
  // block products (k_prod) and the sweep over them (variant 6), one wave
  // per tile, from kProdMinNT tiles up; also instantiated in sdq_nt_dense.hip
  // only
  static constexpr bool kProd = NT >= kProdMinNT;
  static hipError_t prod(const Inst* inst, const SweepItem* items, int count, Queue* q, int grid, hipStream_t s) {
    if constexpr (kProd) {
      hipLaunchKernelGGL((k_prod<NT, NT>), dim3(grid), dim3(Geo<NT, NT>::THREADS), 0, s, inst, items, count, q);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  static hipError_t prod_info(KernelInfo* out) {
    if constexpr (kProd) return info_of<NT>(k_prod<NT, NT>, (int)sizeof(ProdSmem<NT, NT>), out);
    return hipErrorInvalidValue;
  }
  static hipError_t bprod_sweep(const Inst* inst, const SweepItem* items, int count, Queue* q, int grid,
                                double* tscr, hipStream_t s) {
    if constexpr (kProd) {
      if (!tscr) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_sweep<NT, NT, false, false, true, true, true>), dim3(grid), dim3(Geo<NT, NT>::THREADS),
                         0, s, inst, items, count, q, tscr);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  static hipError_t bprod_sweep_info(KernelInfo* out) {
    if constexpr (kProd)
      return info_of<NT>(k_sweep<NT, NT, false, false, true, true, true>, (int)sizeof(Smem<NT, NT, false>), out);
    return hipErrorInvalidValue;
  }
  // G(tau,0) of dense-slice chains (propagation over the dense slices), also
  // instantiated in sdq_nt_dense.hip only
  static hipError_t dense_pair(const Inst* inst, const PairItem* items, int count, const int32_t* l_list,
                               Queue* q, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_pair<NT, P, kPairLds, PAIR_TDISP_DENSE>), dim3(grid), dim3(Geo<NT, P>::THREADS), 0, s,
                       inst, items, count, l_list, q);
    return hipGetLastError();
  }
  static hipError_t dense_pair_info(KernelInfo* out) {
    return info_of(k_pair<NT, P, kPairLds, PAIR_TDISP_DENSE>, (int)sizeof(Smem<NT, P, kPairLds>), out);
  }
  // variants 4 and 5: one wave per 16-column tile (PT = NT waves), T in the
  // per-workgroup scratch between blocks
  static constexpr int PT = NT;
  static hipError_t sweep(int variant, const Inst* inst, const SweepItem* items, int count, Queue* q,
                          int grid, double* tscr, hipStream_t s) {
    double* const none = nullptr;
    if (variant == 2) {
      if constexpr (kSvd) {
        hipLaunchKernelGGL((k_sweep<NT, P, true, true>), dim3(grid), dim3(Geo<NT, P>::THREADS), 0, s, inst,
                           items, count, q, none);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    }
    if (variant == 4 || variant == 5) {
      if (!tscr) return hipErrorInvalidValue;
      if (variant == 5 && kLds)
        hipLaunchKernelGGL((k_sweep<NT, PT, kLds, false, false, true>), dim3(grid), dim3(Geo<NT, PT>::THREADS), 0,
                           s, inst, items, count, q, tscr);
      else
        hipLaunchKernelGGL((k_sweep<NT, PT, false, false, false, true>), dim3(grid), dim3(Geo<NT, PT>::THREADS),
                           0, s, inst, items, count, q, tscr);
      return hipGetLastError();
    }
    if (variant == 1 && kLds)
      hipLaunchKernelGGL((k_sweep<NT, P, kLds>), dim3(grid), dim3(Geo<NT, P>::THREADS), 0, s, inst,
                         items, count, q, none);
    else
      hipLaunchKernelGGL((k_sweep<NT, P, false>), dim3(grid), dim3(Geo<NT, P>::THREADS), 0, s, inst,
                         items, count, q, none);
    return hipGetLastError();
  }
  static hipError_t pair(int mode, const Inst* inst, const PairItem* items, int count,
                         const int32_t* l_list, Queue* q, int grid, hipStream_t s) {
    const dim3 b(Geo<NT, P>::THREADS);
    if (mode == PAIR_TDISP)
      hipLaunchKernelGGL((k_pair<NT, P, kPairLds, PAIR_TDISP>), dim3(grid), b, 0, s, inst, items, count, l_list, q);
    else if (mode == PAIR_GRAD)
      hipLaunchKernelGGL((k_pair<NT, P, kPairLds, PAIR_GRAD>), dim3(grid), b, 0, s, inst, items, count, l_list, q);
    else if (mode == PAIR_TDISP_PLAIN)
      hipLaunchKernelGGL((k_pair<NT, P, kPairLds, PAIR_TDISP_PLAIN>), dim3(grid), b, 0, s, inst, items, count,
                         l_list, q);
    else if (mode == PAIR_LOCAL)
      hipLaunchKernelGGL((k_pair<NT, P, kPairLds, PAIR_LOCAL>), dim3(grid), b, 0, s, inst, items, count, l_list, q);
    else if (mode == PAIR_BSTART)
      hipLaunchKernelGGL((k_pair<NT, P, kPairLds, PAIR_BSTART>), dim3(grid), b, 0, s, inst, items, count, l_list, q);
    else
      hipLaunchKernelGGL((k_pair<NT, P, kPairLds, PAIR_EQUAL>), dim3(grid), b, 0, s, inst, items, count, l_list, q);
    return hipGetLastError();
  }
  static hipError_t similarity(int n, int count, double* const* mats, const double* left,
                               const double* right, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_similarity<NT, P>), dim3(grid), dim3(Geo<NT, P>::THREADS), 0, s, n, count,
                       mats, left, right);
    return hipGetLastError();
  }
  static hipError_t udt(int n, int count, const double* w, double* u, double* d, double* t,
                        hipStream_t s) {
    const int grid = count < 8192 ? count : 8192;
    hipLaunchKernelGGL((k_udt<NT, P>), dim3(grid), dim3(Geo<NT, P>::THREADS), 0, s, n, count, w, u,
                       d, t);
    return hipGetLastError();
  }
  template <int PW = P, class KF>
  static hipError_t info_of(KF kern, int lds, KernelInfo* out) {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, Geo<NT, PW>::THREADS, 0);
    out->threads = Geo<NT, PW>::THREADS;
    out->lds_bytes = lds;
    out->blocks_per_cu = nb;
    return e;
  }
  static hipError_t info(int kind, int variant, KernelInfo* out) {
    if (kind == KK_SWEEP && (variant == 4 || variant == 5)) {
      if (variant == 5 && kLds)
        return info_of<PT>(k_sweep<NT, PT, kLds, false, false, true>, (int)sizeof(Smem<NT, PT, kLds>), out);
      return info_of<PT>(k_sweep<NT, PT, false, false, false, true>, (int)sizeof(Smem<NT, PT, false>), out);
    }
    if (kind == KK_SWEEP) {
      if constexpr (kSvd)
        if (variant == 2) return info_of(k_sweep<NT, P, true, true>, (int)sizeof(Smem<NT, P, true>), out);
      if (variant == 1 && kLds)
        return info_of(k_sweep<NT, P, kLds>, (int)sizeof(Smem<NT, P, kLds>), out);
      return info_of(k_sweep<NT, P, false>, (int)sizeof(Smem<NT, P, false>), out);
    }
    if (kind == KK_PAIR)
      return info_of(k_pair<NT, P, kPairLds, PAIR_TDISP>, (int)sizeof(Smem<NT, P, kPairLds>), out);
    return info_of(k_udt<NT, P>, (int)sizeof(Smem<NT, P, false>), out);
  }
};

}  // namespace sdq
