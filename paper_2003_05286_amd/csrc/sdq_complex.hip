// sdq_complex.hip -- complex UDT of independent matrices (Sec. 4.2.2 over the
// complex numbers, as the complex slices of App. B need it):
//   W P = Q R (column-pivoted Householder QR), U = Q, D = |diag R|,
//   T = D^{-1} R P^T.
// One workgroup (four wave64s) per matrix, the matrix resident in LDS as
// interleaved (re, im) pairs, n <= 64.  Reflector convention: for x = A[i:, i]
// with alpha = x_0, beta = -sign(Re alpha) ||x|| is real, tau = (beta -
// alpha) / beta, v = x / (alpha - beta); H = I - tau v v^H, H^H x = beta e_0,
// so the diagonal of R is real.  Pivot: the first column of largest remaining
// norm, norms downdated with an exact recompute when cancellation threatens
// (Drmac & Bujanovic).  Q is formed in place from the reflectors after R has
// been written out (backward accumulation, Q = H_0 H_1 ... H_{n-1}).
#include <hip/hip_runtime.h>

#include "sdq_internal.h"

namespace sdq {
namespace {

constexpr int kCN = 64;           // largest n
constexpr int kCLD = kCN + 1;     // LDS row stride (in complex entries)
constexpr int kCThreads = 256;    // four waves: wave w takes rows w, w+4, ...

struct cplx {
  double x, y;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// conj(a) * b
__device__ __forceinline__ cplx cjmul(cplx a, cplx b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }

struct CSmem {
  cplx a[kCN * kCLD];
  cplx red[4][kCN];
  cplx tau[kCN];
  double vn1[kCN], vn2[kCN];
  int jpvt[kCN], ipiv[kCN];
};

// Cross-lane reductions over the wave on the DPP paths of the VALU (no LDS
// round trips): swap neighbours (quad_perm 1,0,3,2 and 2,3,0,1), mirror
// within 8 and 16 lanes, then broadcast lane 15 of each row into the next
// and lane 31 into the upper half; lane 63 then holds the result, which
// readlane makes uniform.  A lane outside a step's row mask keeps `old`.
constexpr int kDppSteps[6] = {0xB1, 0x4E, 0x141, 0x140, 0x142, 0x143};
constexpr int kDppRows[6] = {0xf, 0xf, 0xf, 0xf, 0xa, 0xc};

template <int S>
__device__ __forceinline__ double dpp_d(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)x, kDppSteps[S], kDppRows[S], 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), kDppSteps[S], kDppRows[S], 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int S>
__device__ __forceinline__ int dpp_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, kDppSteps[S], kDppRows[S], 0xf, false);
}
__device__ __forceinline__ double lane63(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, 63), hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int S = 0>
__device__ __forceinline__ double wave_sum_(double v) {
  if constexpr (S == 6) {
    return lane63(v);
  } else {
    return wave_sum_<S + 1>(v + dpp_d<S>(0.0, v));
  }
}
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_<0>(v); }

// for values >= 0
template <int S = 0>
__device__ __forceinline__ double wave_max_(double v) {
  if constexpr (S == 6) {
    return lane63(v);
  } else {
    return wave_max_<S + 1>(fmax(v, dpp_d<S>(0.0, v)));
  }
}
__device__ __forceinline__ double wave_max(double v) { return wave_max_<0>(v); }

// (value, index) of the largest value, the lowest index among equal ones;
// the result is the same for every reduction order
template <int S = 0>
__device__ __forceinline__ void wave_argmax_(double& v, int& p) {
  if constexpr (S < 6) {
    const double v2 = dpp_d<S>(v, v);
    const int p2 = dpp_i<S>(p, p);
    if (v2 > v || (v2 == v && p2 < p)) {
      v = v2;
      p = p2;
    }
    wave_argmax_<S + 1>(v, p);
  }
}
__device__ __forceinline__ int wave_argmax(double v, int p) {
  wave_argmax_<0>(v, p);
  return __builtin_amdgcn_readlane(p, 63);
}

// 2-norm of A[r0..n-1][c] by one lane (max-scaled, so no overflow)
template <class SM>
__device__ double col_norm(const SM& S, int r0, int n, int c) {
  double mx = 0.0;
  for (int r = r0; r < n; ++r) mx = fmax(mx, fmax(fabs(S.a[r * kCLD + c].x), fabs(S.a[r * kCLD + c].y)));
  if (mx == 0.0) return 0.0;
  const double inv = 1.0 / mx;
  double s = 0.0;
  for (int r = r0; r < n; ++r) {
    const double p = S.a[r * kCLD + c].x * inv, q = S.a[r * kCLD + c].y * inv;
    s += p * p + q * q;
  }
  return mx * sqrt(s);
}

// orders the LDS accesses of one wave's lanes around it (compiler fence)
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// 2-norm of the wave's 64 complex values: the plain sum of squares where it
// neither overflows nor underflows, else max-scaled
__device__ __forceinline__ double wave_norm(cplx x) {
  const double ss = wave_sum(x.x * x.x + x.y * x.y);
  if (ss > 1e-280 && ss < 1e280) return sqrt(ss);
  const double mx = wave_max(fmax(fabs(x.x), fabs(x.y)));
  if (mx == 0.0) return 0.0;
  const double p0 = x.x / mx, q0 = x.y / mx;
  return mx * sqrt(wave_sum(p0 * p0 + q0 * q0));
}

// norm downdate of column `lane` after step i (exact recompute when the
// downdated value has lost too many digits)
template <class SM>
__device__ __forceinline__ void downdate(SM& S, int n, int i, int lane, double tol3z) {
  if (lane > i && lane < n && S.vn1[lane] != 0.0) {
    const cplx aij = S.a[i * kCLD + lane];
    double tmp = hypot(aij.x, aij.y) / S.vn1[lane];
    tmp = 1.0 - tmp * tmp;
    if (tmp < 0.0) tmp = 0.0;
    const double ratio = S.vn1[lane] / S.vn2[lane];
    if (tmp * ratio * ratio <= tol3z) {
      S.vn1[lane] = i + 1 < n ? col_norm(S, i + 1, n, lane) : 0.0;
      S.vn2[lane] = S.vn1[lane];
    } else {
      S.vn1[lane] *= sqrt(tmp);
    }
  }
}

// A[i:, c] <- (I - t v v^H) A[i:, c] for the columns c0 <= c < n, v = A[i:, i]
// with v_i = 1 implied (row i taken by wave 0 outside the loop); four waves
// split the rows.
template <class SM>
__device__ void apply_reflector(SM& S, int n, int i, int c0, cplx t) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane;
  const int r0 = w == 0 ? i + 4 : i + w;
  cplx part = {0.0, 0.0};
  if (c >= c0 && c < n) {
    if (w == 0) part = S.a[i * kCLD + c];
    // unrolled so that the LDS loads of several rows are in flight at once
#pragma unroll 8
    for (int r = r0; r < n; r += 4) {
      const cplx p = cjmul(S.a[r * kCLD + i], S.a[r * kCLD + c]);
      part.x += p.x;
      part.y += p.y;
    }
  }
  S.red[w][c] = part;
  __syncthreads();
  if (c >= c0 && c < n) {
    cplx s = {S.red[0][c].x + S.red[1][c].x + S.red[2][c].x + S.red[3][c].x,
              S.red[0][c].y + S.red[1][c].y + S.red[2][c].y + S.red[3][c].y};
    s = cmul(t, s);
    if (w == 0) {
      S.a[i * kCLD + c].x -= s.x;
      S.a[i * kCLD + c].y -= s.y;
    }
#pragma unroll 8
    for (int r = r0; r < n; r += 4) {
      const cplx d = cmul(S.a[r * kCLD + i], s);
      S.a[r * kCLD + c].x -= d.x;
      S.a[r * kCLD + c].y -= d.y;
    }
  }
  __syncthreads();
}

// Column-pivoted Householder QR of S.a (n x n, in place, columns swapped
// physically): on return S.a holds R on and above the diagonal and the
// reflectors below it, S.tau the reflector scalars, S.jpvt the original
// column of each position.  Ends with a barrier.
template <class SM>
__device__ void cpqr_lds(SM& S, int n) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double tol3z = sqrt(2.220446049250313e-16);
  if (tid < n) {
    S.jpvt[tid] = tid;
    S.vn1[tid] = col_norm(S, 0, n, tid);
    S.vn2[tid] = S.vn1[tid];
  }
  __syncthreads();
  for (int i = 0; i < n; ++i) {
    // wave 0 alone, lane-synchronous (LDS operations of one wave complete
    // in order): the norm downdate of step i-1, the pivot, the column swap
    // and the reflector of step i; the other waves wait at the barrier
    if (wv == 0) {
      if (i > 0) downdate(S, n, i - 1, lane, tol3z);
      wave_fence();
      const int p = wave_argmax((lane >= i && lane < n) ? S.vn1[lane] : -1.0, lane);
      if (p != i) {
        if (lane < n) {
          const cplx x = S.a[lane * kCLD + i];
          S.a[lane * kCLD + i] = S.a[lane * kCLD + p];
          S.a[lane * kCLD + p] = x;
        }
        if (lane == 0) {
          const int tj = S.jpvt[i];
          S.jpvt[i] = S.jpvt[p];
          S.jpvt[p] = tj;
          S.vn1[p] = S.vn1[i];
          S.vn2[p] = S.vn2[i];
        }
      }
      wave_fence();
      // reflector of A[i:, i]; lane handles row i + 1 + lane
      const int r = i + 1 + lane;
      const cplx x = r < n ? S.a[r * kCLD + i] : cplx{0.0, 0.0};
      const double xnorm = wave_norm(x);
      const cplx al = S.a[i * kCLD + i];
      cplx ti = {0.0, 0.0};
      if (xnorm != 0.0 || al.y != 0.0) {
        const double nrm = hypot(hypot(al.x, al.y), xnorm);
        const double beta = -copysign(nrm, al.x);
        ti = {(beta - al.x) / beta, -al.y / beta};
        // s = 1 / (alpha - beta), scaled so that no square overflows
        const cplx dn = {al.x - beta, al.y};
        const double sm = fmax(fabs(dn.x), fabs(dn.y));
        const double ax = dn.x / sm, ay = dn.y / sm, den = (ax * ax + ay * ay) * sm;
        const cplx sc = {ax / den, -ay / den};
        if (r < n) S.a[r * kCLD + i] = cmul(x, sc);
        wave_fence();
        if (lane == 0) S.a[i * kCLD + i] = {beta, 0.0};
      }
      if (lane == 0) S.tau[i] = ti;
    }
    __syncthreads();
    const cplx ti = S.tau[i];
    if (ti.x != 0.0 || ti.y != 0.0) apply_reflector(S, n, i, i + 1, cplx{ti.x, -ti.y});
  }
}

// Q = H_0 H_1 ... H_{n-1} in place in S.a from the reflectors cpqr_lds left
// there (backward accumulation).  Ends with a barrier.
template <class SM>
__device__ void form_q_lds(SM& S, int n) {
  const int tid = threadIdx.x;
  // Q in place: for i = n-1 .. 0, apply H_i to columns i+1.. and turn
  // column i into H_i e_i
  for (int i = n - 1; i >= 0; --i) {
    const cplx ti = S.tau[i];
    if (i < n - 1 && (ti.x != 0.0 || ti.y != 0.0)) apply_reflector(S, n, i, i + 1, ti);
    if (tid < n) {
      if (tid > i) {
        const cplx v = S.a[tid * kCLD + i];
        S.a[tid * kCLD + i] = cplx{-(ti.x * v.x - ti.y * v.y), -(ti.x * v.y + ti.y * v.x)};
      } else if (tid == i) {
        S.a[tid * kCLD + i] = cplx{1.0 - ti.x, -ti.y};
      } else {
        S.a[tid * kCLD + i] = cplx{0.0, 0.0};
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kCThreads) void k_udt_complex(int n, int count, const double* __restrict__ w,
                                                           double* __restrict__ u, double* __restrict__ d,
                                                           double* __restrict__ t) {
  __shared__ CSmem S;
  const int tid = threadIdx.x;
  for (int b = blockIdx.x; b < count; b += gridDim.x) {
    const size_t off = (size_t)b * n * n;
    const cplx* W = reinterpret_cast<const cplx*>(w) + off;
    for (int e = tid; e < n * n; e += kCThreads) S.a[(e / n) * kCLD + e % n] = W[e];
    __syncthreads();
    cpqr_lds(S, n);
    // D = |diag R| (real), T = D^{-1} R P^T (rows with D = 0 undivided)
    if (tid < n) {
      d[(size_t)b * n + tid] = fabs(S.a[tid * kCLD + tid].x);
      S.ipiv[S.jpvt[tid]] = tid;
    }
    __syncthreads();
    cplx* T = reinterpret_cast<cplx*>(t) + off;
    for (int e = tid; e < n * n; e += kCThreads) {
      const int r = e / n, col = e % n, c = S.ipiv[col];
      cplx v = {0.0, 0.0};
      if (c >= r) {
        const double dr = fabs(S.a[r * kCLD + r].x);
        const double sc = dr > 0.0 ? 1.0 / dr : 1.0;
        v = {S.a[r * kCLD + c].x * sc, S.a[r * kCLD + c].y * sc};
      }
      T[e] = v;
    }
    __syncthreads();
    form_q_lds(S, n);
    cplx* U = reinterpret_cast<cplx*>(u) + off;
    for (int e = tid; e < n * n; e += kCThreads) U[e] = S.a[(e / n) * kCLD + e % n];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Chains of complex slices (App. B): G = (1 + B_m ... B_1)^{-1} for complex
// dense slices, with log|det(1 + B_m ... B_1)| and its phase.  One workgroup
// per chain, everything resident in LDS (n <= 64):
//   chain (Sec. 4.1): per block of k slices W <- B_q W on FP64 MFMA (a
//     complex product is four real ones), then W <- W D, the complex pivoted
//     QR of W (Sec. 4.2.2), D <- |diag R|, T <- D^{-1} R P^T T on MFMA, and
//     U = Q formed in place;
//   inversion (Sec. 5.1, Loh's split, in the mirror form of the real path):
//     1 + U D T = U D_p (D_p^{-1} U^H + D_m T), so G = M^{-1} D_p^{-1} U^H
//     with M = D_p^{-1} U^H + D_m T, solved by Gaussian elimination with
//     partial pivoting (row swaps in LDS) and back substitution;
//   determinant: det(1 + B) = det U prod(D_p) det M, det U the product of
//     det H_j = -tau_j / conj(tau_j) over the reflectors of the last QR, det M
//     the product of the pivots and the row-swap signs.
struct CCSmem {
  cplx a[kCN * kCLD];  // W, then R and the reflectors, then U = Q, then the right-hand sides / G
  cplx t[kCN * kCLD];  // T, then M
  cplx red[4][kCN];
  cplx tau[kCN];
  double vn1[kCN], vn2[kCN];
  double d[kCN];  // D of the current factorization
  int jpvt[kCN], ipiv[kCN];
  int piv;
};

typedef double cd4 __attribute__((ext_vector_type(4)));

// C = A X for the n x n (padded to 64) complex matrices A (by a callable:
// A(i, k) for the calling lane) and X in LDS (X(k, c) callable): wave w
// produces the output columns 16 w .. 16 w + 15, all four row tiles, into
// cr / ci in the FP64 MFMA 16x16x4 accumulator layout (lane l: rows
// 16 ti + l / 16 + 4 r of column 16 w + l % 16).
template <class AF, class XF>
__device__ __forceinline__ void cgemm(AF A, XF X, cd4 (&cr)[4], cd4 (&ci)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, cl = lane & 15;
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) cr[ti] = ci[ti] = cd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int tk = 0; tk < 4; ++tk) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kk = 16 * tk + g + 4 * r;
      const cplx b = X(kk, 16 * w + cl);
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const cplx a = A(16 * ti + cl, kk);
        cr[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr[ti], 0, 0, 0);
        cr[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr[ti], 0, 0, 0);
        ci[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci[ti], 0, 0, 0);
        ci[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci[ti], 0, 0, 0);
      }
    }
  }
}

// C = B X as cgemm, with B the row-major n x n complex matrix at Bq in device
// memory.  The sixteen B entries of a k tile are loaded at once, from
// clamped in-range addresses (entries outside n x n zeroed after the load),
// and the next tile's loads are in flight while the current tile's MFMAs
// run: a load behind a per-entry branch would be waited for before the
// next one.
template <class XF>
__device__ __forceinline__ void cgemm_hbm(const cplx* Bq, int n, XF X, cd4 (&cr)[4], cd4 (&ci)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, cl = lane & 15;
  const auto* gB = (const __attribute__((address_space(1))) double*)Bq;
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) cr[ti] = ci[ti] = cd4{0.0, 0.0, 0.0, 0.0};
  cplx a[2][4][4];  // [buffer][r][ti]
  auto load = [&](int tk, cplx (&dst)[4][4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const int i = 16 * ti + cl, kk = 16 * tk + g + 4 * r;
        const size_t off = 2 * ((size_t)min(i, n - 1) * n + min(kk, n - 1));
        dst[r][ti] = cplx{gB[off], gB[off + 1]};
      }
  };
  load(0, a[0]);
#pragma unroll
  for (int tk = 0; tk < 4; ++tk) {
    if (tk + 1 < 4) load(tk + 1, a[(tk + 1) & 1]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kk = 16 * tk + g + 4 * r;
      const cplx b = X(kk, 16 * w + cl);
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const bool ok = 16 * ti + cl < n && kk < n;
        const cplx av = a[tk & 1][r][ti];
        const double ax = ok ? av.x : 0.0, ay = ok ? av.y : 0.0;
        cr[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, b.x, cr[ti], 0, 0, 0);
        cr[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ay, b.y, cr[ti], 0, 0, 0);
        ci[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, b.y, ci[ti], 0, 0, 0);
        ci[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, b.x, ci[ti], 0, 0, 0);
      }
    }
  }
}

// write the accumulators of cgemm to an LDS matrix, each column scaled by
// cs(c) and each row by rs(i)
template <class CS, class RS>
__device__ __forceinline__ void cstore(cplx* M, const cd4 (&cr)[4], const cd4 (&ci)[4], CS cs, RS rs) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, c = 16 * w + (lane & 15);
  const double sc = cs(c);
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti + g + 4 * r;
      const double f = sc * rs(i);
      M[i * kCLD + c] = cplx{cr[ti][r] * f, ci[ti][r] * f};
    }
}

__global__ __launch_bounds__(kCThreads) void k_greens_complex(const CChain* __restrict__ tab, int count) {
  __shared__ CCSmem S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = blockIdx.x; b < count; b += gridDim.x) {
    const CChain C = tab[b];
    const int n = C.n, m = C.m, k = C.k;
    const cplx* Bs = reinterpret_cast<const cplx*>(C.slices);
    // W = U = 1, T = 1, D = 1; the padding of both matrices zero
    for (int e = tid; e < kCN * kCLD; e += kCThreads) {
      const int i = e / kCLD, j = e % kCLD;
      const cplx one = {(i == j && i < n) ? 1.0 : 0.0, 0.0};
      S.a[e] = one;
      S.t[e] = one;
    }
    if (tid < kCN) S.d[tid] = 1.0;
    __syncthreads();
    for (int q0 = 1; q0 <= m; q0 += k) {
      const int q1 = q0 + k - 1 < m ? q0 + k - 1 : m;
      // W <- B_q W for q = q0 .. q1; after the last, W <- W D
      for (int q = q0; q <= q1; ++q) {
        const cplx* Bq = Bs + (size_t)(q - 1) * n * n;
        cd4 cr[4], ci[4];
        cgemm_hbm(Bq, n, [&](int kk, int c) -> cplx { return S.a[kk * kCLD + c]; }, cr, ci);
        __syncthreads();
        const bool last = q == q1;
        cstore(S.a, cr, ci, [&](int c) { return last ? S.d[c] : 1.0; }, [](int) { return 1.0; });
        __syncthreads();
      }
      // pivoted QR, D <- |diag R|
      cpqr_lds(S, n);
      __syncthreads();
      if (tid < n) S.d[tid] = fabs(S.a[tid * kCLD + tid].x);
      if (tid >= n && tid < kCN) S.jpvt[tid] = tid;
      __syncthreads();
      // T <- D^{-1} R P^T T: row i of the result is sum_{j >= i} R[i][j] T[jpvt[j]][:] / D_i
      {
        cd4 cr[4], ci[4];
        cgemm([&](int i, int j) -> cplx { return (i < n && j < n && j >= i) ? S.a[i * kCLD + j] : cplx{0.0, 0.0}; },
              [&](int j, int c) -> cplx { return S.t[S.jpvt[j] * kCLD + c]; }, cr, ci);
        __syncthreads();
        cstore(S.t, cr, ci, [](int) { return 1.0; },
               [&](int i) { return (i < n && S.d[i] > 0.0) ? 1.0 / S.d[i] : 1.0; });
        __syncthreads();
      }
      // U = Q in place
      form_q_lds(S, n);
    }
    // phase of det U: the reflectors of the last QR
    if (wv == 0) {
      double pr = 1.0, pi = 0.0;
      if (lane == 0) {
        for (int j = 0; j < n; ++j) {
          const cplx t = S.tau[j];
          if (t.x == 0.0 && t.y == 0.0) continue;
          // -tau / conj(tau) = -tau^2 / |tau|^2
          const double a2 = t.x * t.x + t.y * t.y;
          const cplx h = {-(t.x * t.x - t.y * t.y) / a2, -(2.0 * t.x * t.y) / a2};
          const double nr = pr * h.x - pi * h.y, ni = pr * h.y + pi * h.x;
          pr = nr;
          pi = ni;
        }
        S.red[0][0] = cplx{pr, pi};
      }
    }
    __syncthreads();
    const cplx phu = S.red[0][0];
    // M = D_p^{-1} U^H + D_m T into S.t (reads U, writes T's own entry)
    for (int e = tid; e < n * n; e += kCThreads) {
      const int i = e / n, j = e % n;
      const double di = S.d[i], dp = di > 1.0 ? di : 1.0, dm = di > 1.0 ? 1.0 : di;
      const cplx u = S.a[j * kCLD + i];
      const cplx t = S.t[i * kCLD + j];
      S.t[i * kCLD + j] = cplx{u.x / dp + dm * t.x, -u.y / dp + dm * t.y};
    }
    __syncthreads();
    // right-hand sides D_p^{-1} U^H into S.a, in place by pairs (i, j), (j, i)
    for (int e = tid; e < n * n; e += kCThreads) {
      const int i = e / n, j = e % n;
      if (j < i) continue;
      const cplx uij = S.a[i * kCLD + j], uji = S.a[j * kCLD + i];
      const double dpi = S.d[i] > 1.0 ? S.d[i] : 1.0, dpj = S.d[j] > 1.0 ? S.d[j] : 1.0;
      S.a[i * kCLD + j] = cplx{uji.x / dpi, -uji.y / dpi};
      S.a[j * kCLD + i] = cplx{uij.x / dpj, -uij.y / dpj};
    }
    __syncthreads();
    // Gaussian elimination with partial pivoting on M, the same row
    // operations on the right-hand sides
    double ldm = 0.0, ppr = 1.0, ppi = 0.0;  // log|det M| and its phase (thread 0)
    for (int j = 0; j < n; ++j) {
      if (wv == 0) {
        const double am = (lane >= j && lane < n) ? hypot(S.t[lane * kCLD + j].x, S.t[lane * kCLD + j].y) : -1.0;
        const int p = wave_argmax(am, lane);
        if (lane == 0) S.piv = p;
      }
      __syncthreads();
      const int p = S.piv;
      if (p != j) {
        for (int e = tid; e < 2 * n; e += kCThreads) {
          cplx* Mt = e < n ? S.t : S.a;
          const int c = e < n ? e : e - n;
          const cplx x = Mt[j * kCLD + c];
          Mt[j * kCLD + c] = Mt[p * kCLD + c];
          Mt[p * kCLD + c] = x;
        }
        __syncthreads();
      }
      const cplx pv = S.t[j * kCLD + j];
      if (tid == 0) {
        const double ap = hypot(pv.x, pv.y);
        ldm += log(ap);
        const double ux = pv.x / ap, uy = pv.y / ap;
        const double nr = ppr * ux - ppi * uy, ni = ppr * uy + ppi * ux;
        ppr = p != j ? -nr : nr;
        ppi = p != j ? -ni : ni;
      }
      // 1 / pivot, scaled so that no square overflows
      const double sm = fmax(fabs(pv.x), fabs(pv.y));
      const double ax = pv.x / sm, ay = pv.y / sm, den = (ax * ax + ay * ay) * sm;
      const cplx rp = {ax / den, -ay / den};
      // rows r > j: M[r][c] -= l_r M[j][c] (c > j), rhs[r][:] -= l_r rhs[j][:]
      const int rows = n - 1 - j;
      for (int e = tid; e < rows * 2 * n; e += kCThreads) {
        const int r = j + 1 + e / (2 * n), cc = e % (2 * n);
        const cplx l = cmul(S.t[r * kCLD + j], rp);
        if (cc < n) {
          if (cc > j) {
            const cplx x = cmul(l, S.t[j * kCLD + cc]);
            S.t[r * kCLD + cc].x -= x.x;
            S.t[r * kCLD + cc].y -= x.y;
          }
        } else {
          const int c = cc - n;
          const cplx x = cmul(l, S.a[j * kCLD + c]);
          S.a[r * kCLD + c].x -= x.x;
          S.a[r * kCLD + c].y -= x.y;
        }
      }
      __syncthreads();
    }
    // back substitution: rhs <- U^{-1} rhs
    for (int j = n - 1; j >= 0; --j) {
      const cplx pv = S.t[j * kCLD + j];
      const double sm = fmax(fabs(pv.x), fabs(pv.y));
      const double ax = pv.x / sm, ay = pv.y / sm, den = (ax * ax + ay * ay) * sm;
      const cplx rp = {ax / den, -ay / den};
      if (tid < n) S.a[j * kCLD + tid] = cmul(S.a[j * kCLD + tid], rp);
      __syncthreads();
      for (int e = tid; e < j * n; e += kCThreads) {
        const int r = e / n, c = e % n;
        const cplx x = cmul(S.t[r * kCLD + j], S.a[j * kCLD + c]);
        S.a[r * kCLD + c].x -= x.x;
        S.a[r * kCLD + c].y -= x.y;
      }
      __syncthreads();
    }
    // outputs
    int bad = 0;
    if (C.g) {
      cplx* G = reinterpret_cast<cplx*>(C.g);
      for (int e = tid; e < n * n; e += kCThreads) {
        const cplx x = S.a[(e / n) * kCLD + e % n];
        G[e] = x;
        if (!isfinite(x.x) || !isfinite(x.y)) bad = 1;
      }
    }
    if (tid == 0) {
      double ldp = 0.0;
      for (int i = 0; i < n; ++i) ldp += log(S.d[i] > 1.0 ? S.d[i] : 1.0);
      const double ld = ldp + ldm;
      const double fr = phu.x * ppr - phu.y * ppi, fi = phu.x * ppi + phu.y * ppr;
      if (C.logdet) *C.logdet = ld;
      if (C.phase) {
        C.phase[0] = fr;
        C.phase[1] = fi;
      }
      if (!isfinite(ld) || !isfinite(fr) || !isfinite(fi)) bad = 1;
    }
    for (int i = tid; i < n; i += kCThreads)
      if (!isfinite(S.d[i]) || !(S.d[i] > 0.0)) bad = 1;
    if (__any(bad) && lane == 0 && C.status) atomicOr(C.status, kStatusRange);
    __syncthreads();
  }
}

}  // namespace

int complex_udt_max_n() { return kCN; }

hipError_t launch_greens_complex(const CChain* tab, int count, int grid, hipStream_t s) {
  if (count < 1 || grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_greens_complex, dim3(grid), dim3(kCThreads), 0, s, tab, count);
  return hipGetLastError();
}

hipError_t launch_udt_complex(int n, int count, const double* w, double* u, double* d, double* t, int grid,
                              hipStream_t s) {
  if (n < 1 || n > kCN || count < 1 || grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_udt_complex, dim3(grid), dim3(kCThreads), 0, s, n, count, w, u, d, t);
  return hipGetLastError();
}

}  // namespace sdq
