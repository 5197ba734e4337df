/*
 * sdq_oracle.c -- plain, slow, FP64 CPU oracle for the stabilized DQMC
 * Green's functions of C. Bauer, "Fast and stable determinant quantum Monte
 * Carlo" (SciPost Phys. 2020, arXiv:2003.05286).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the GPU library: only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load this file's shared object.  It shares no code, header, table or helper
 * with the HIP path, and it uses no BLAS/LAPACK: every product, pivoted QR,
 * LU and inverse is a plain loop written here, in the order the paper states
 * the steps, with no blocking or reordering.
 *
 * Conventions: every matrix is n x n, row-major, A[i*n + j].  Slice l
 * (1-based, 1 <= l <= m) uses field row l-1:
 *     B_l = expk * diag(exp(alpha * field[l-1][:]))          (Sec. 2, Sec. 3)
 * expk_inv must be the inverse of expk (exp(+dtau K)).
 *
 * Functions and the passages they follow:
 *   chain_udt          Sec. 4.1 (stabilized product "fact_mult", with the
 *                      naive/stabilized mixture every k slices) and
 *                      Sec. 4.2.2 (UDT from column-pivoted QR)
 *   cpqr               Sec. 4.2.2 (pivoted Householder QR, as LAPACK geqp3;
 *                      column-norm downdating after Drmac & Bujanovic 2008)
 *   inv_one_plus_loh   Sec. 5.1, scheme inv_one_plus_loh (D = Dp * Dm split)
 *   inv_one_plus       Sec. 5.1, scheme inv_one_plus (single decomposition)
 *   inv_sum_loh        Sec. 6.1, scheme inv_sum_loh (time-displaced)
 *   inv_sum            Sec. 6.1, scheme inv_sum
 *   or_greens_slice    App. A.1 (combining two stack elements into G_l),
 *                      G_l defined in Sec. 6 (equal-time G at slice l)
 *   or_greens_sym,     the same for the symmetric Trotter slice
 *   or_greens_tdisp_sym  B_l = E^{1/2} diag(v_l) E^{1/2} of Sec. 2
 *   or_logdet_grad     d log|det(1+B_M..B_1)| / d f_{l,i} = alpha (1-G_l)_ii
 *                      (Jacobi's formula; see the function comment)
 *   or_greens_naive    Sec. 3 (the unstabilized product, negative control)
 *   or_greens_dense,   the same chains and inversions for slices given as
 *   or_greens_tdisp_dense  dense matrices (generalized slices)
 *   or_udt_complex     Sec. 4.2.2 over the complex numbers (complex slices,
 *                      App. B): complex column-pivoted Householder QR
 *   or_greens_complex  Sec. 4.1, 4.2.2 and 5.1 (inv_one_plus_loh) for complex
 *                      slices (App. B), with the phase of det(1 + B)
 *   jacobi_svd,        Sec. 4.2 (the Jacobi SVD the paper compares with the
 *   or_greens_stab     QR; one-sided, Hestenes), as an independent stabilizer
 *                      of the same chain: a cross-check of the QR path
 * Readings of passages that are ambiguous or garbled in the paper are noted
 * where they are used.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "sdq_oracle.h"

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                      */

static double* mat_new(int n) { return (double*)calloc((size_t)n * n, sizeof(double)); }

static void mat_eye(int n, double* A) {
  memset(A, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; ++i) A[i * n + i] = 1.0;
}

static void mat_copy(int n, const double* A, double* B) {
  memcpy(B, A, sizeof(double) * (size_t)n * n);
}

/* C = A * B  (C must not alias A or B) */
static void mat_mul(int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < n; ++i) {
    double* c = C + (size_t)i * n;
    for (int j = 0; j < n; ++j) c[j] = 0.0;
    for (int p = 0; p < n; ++p) {
      const double a = A[(size_t)i * n + p];
      const double* b = B + (size_t)p * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
  }
}

/* C = A^T * B */
static void mat_mul_tn(int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < n * n; ++i) C[i] = 0.0;
  for (int p = 0; p < n; ++p)
    for (int i = 0; i < n; ++i) {
      const double a = A[(size_t)p * n + i];
      for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += a * B[(size_t)p * n + j];
    }
}

/* C = A * B^T */
static void mat_mul_nt(int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int p = 0; p < n; ++p) s += A[(size_t)i * n + p] * B[(size_t)j * n + p];
      C[(size_t)i * n + j] = s;
    }
}

/* A <- diag(d) * A */
static void scale_rows(int n, double* A, const double* d) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] *= d[i];
}

/* A <- A * diag(d) */
static void scale_cols(int n, double* A, const double* d) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] *= d[j];
}

/* Euclidean norm of x[0], x[inc], ... with the running scale/sum-of-squares
 * update, so that entries near 1e+-200 neither overflow nor underflow. */
static double nrm2(int len, const double* x, int inc) {
  double scale = 0.0, ssq = 1.0;
  for (int i = 0; i < len; ++i) {
    const double a = fabs(x[(size_t)i * inc]);
    if (a == 0.0) continue;
    if (scale < a) {
      ssq = 1.0 + ssq * (scale / a) * (scale / a);
      scale = a;
    } else {
      ssq += (a / scale) * (a / scale);
    }
  }
  return scale * sqrt(ssq);
}

/* ------------------------------------------------------------------------ */
/* Column-pivoted Householder QR (Businger-Golub), in place on a row-major
 * n x n matrix A.  On return the upper triangle holds R, the strict lower
 * triangle holds the Householder vectors (unit leading entry implied),
 * tau[j] their scalars, and jpvt[j] the original index of the column moved to
 * position j, so that  A_in * P = Q * R  with  P[jpvt[j]][j] = 1  and
 * Q = H_0 H_1 ... H_{n-1},  H_j = I - tau_j v_j v_j^T.
 *
 * Pivot rule: the first column (in current order) of maximal remaining norm.
 * Reflector: beta = -sign(alpha) ||x||, v = x / (alpha - beta), tau =
 * (beta - alpha) / beta (tau = 0 when the column below the diagonal is zero).
 * Norm downdating: vn1 <- vn1 sqrt(1 - (|r|/vn1)^2), with an exact recompute
 * when (1 - (|r|/vn1)^2)(vn1/vn2)^2 <= sqrt(eps) (Drmac & Bujanovic 2008). */
static void cpqr(int n, double* A, int* jpvt, double* tau) {
  double* vn1 = (double*)malloc(sizeof(double) * n);
  double* vn2 = (double*)malloc(sizeof(double) * n);
  const double tol3z = sqrt(2.220446049250313e-16);
  for (int j = 0; j < n; ++j) {
    jpvt[j] = j;
    vn1[j] = nrm2(n, A + j, n);
    vn2[j] = vn1[j];
  }
  for (int i = 0; i < n; ++i) {
    /* pivot */
    int p = i;
    for (int j = i + 1; j < n; ++j)
      if (vn1[j] > vn1[p]) p = j;
    if (p != i) {
      for (int r = 0; r < n; ++r) {
        double t = A[(size_t)r * n + i];
        A[(size_t)r * n + i] = A[(size_t)r * n + p];
        A[(size_t)r * n + p] = t;
      }
      int tj = jpvt[i]; jpvt[i] = jpvt[p]; jpvt[p] = tj;
      vn1[p] = vn1[i];
      vn2[p] = vn2[i];
    }
    /* reflector for A[i:, i] */
    const double alpha = A[(size_t)i * n + i];
    const double xnorm = (i + 1 < n) ? nrm2(n - i - 1, A + (size_t)(i + 1) * n + i, n) : 0.0;
    double t_i = 0.0;
    if (xnorm != 0.0) {
      const double beta = -copysign(hypot(alpha, xnorm), alpha);
      t_i = (beta - alpha) / beta;
      const double s = 1.0 / (alpha - beta);
      for (int r = i + 1; r < n; ++r) A[(size_t)r * n + i] *= s;
      A[(size_t)i * n + i] = beta;
    }
    tau[i] = t_i;
    /* apply H_i to the trailing columns */
    if (t_i != 0.0) {
      for (int j = i + 1; j < n; ++j) {
        double w = A[(size_t)i * n + j];
        for (int r = i + 1; r < n; ++r) w += A[(size_t)r * n + i] * A[(size_t)r * n + j];
        w *= t_i;
        A[(size_t)i * n + j] -= w;
        for (int r = i + 1; r < n; ++r) A[(size_t)r * n + j] -= w * A[(size_t)r * n + i];
      }
    }
    /* downdate the remaining column norms */
    for (int j = i + 1; j < n; ++j) {
      if (vn1[j] == 0.0) continue;
      double temp = fabs(A[(size_t)i * n + j]) / vn1[j];
      temp = 1.0 - temp * temp;
      if (temp < 0.0) temp = 0.0;
      const double ratio = vn1[j] / vn2[j];
      const double temp2 = temp * ratio * ratio;
      if (temp2 <= tol3z) {
        vn1[j] = (i + 1 < n) ? nrm2(n - i - 1, A + (size_t)(i + 1) * n + j, n) : 0.0;
        vn2[j] = vn1[j];
      } else {
        vn1[j] *= sqrt(temp);
      }
    }
  }
  free(vn1);
  free(vn2);
}

/* Q = H_0 H_1 ... H_{n-1} from the reflectors stored by cpqr. */
static void form_q(int n, const double* F, const double* tau, double* Q) {
  mat_eye(n, Q);
  for (int i = n - 1; i >= 0; --i) {
    if (tau[i] == 0.0) continue;
    for (int j = 0; j < n; ++j) {
      double w = Q[(size_t)i * n + j];
      for (int r = i + 1; r < n; ++r) w += F[(size_t)r * n + i] * Q[(size_t)r * n + j];
      w *= tau[i];
      Q[(size_t)i * n + j] -= w;
      for (int r = i + 1; r < n; ++r) Q[(size_t)r * n + j] -= w * F[(size_t)r * n + i];
    }
  }
}

/* parity of the permutation j -> jpvt[j]: +1 or -1 */
static double perm_sign(int n, const int* jpvt) {
  char* seen = (char*)calloc(n, 1);
  int cycles = 0;
  for (int i = 0; i < n; ++i) {
    if (seen[i]) continue;
    ++cycles;
    for (int j = i; !seen[j]; j = jpvt[j]) seen[j] = 1;
  }
  free(seen);
  return ((n - cycles) % 2 == 0) ? 1.0 : -1.0;
}

/* UDT decomposition (Sec. 4.2.2): W P = Q R, U = Q, D = |diag R|,
 * T = D^{-1} R P^T.  D is taken as the absolute value of diag R so that the
 * Dp/Dm split of Sec. 5.1 sees positive scales; the signs stay in T.  With
 * pivoting T is not triangular (the paper's "T upper triangular" holds for
 * R, not for R P^T). */
static void udt(int n, const double* W, double* U, double* D, double* T) {
  double* F = mat_new(n);
  double* tau = (double*)malloc(sizeof(double) * n);
  int* jpvt = (int*)malloc(sizeof(int) * n);
  mat_copy(n, W, F);
  cpqr(n, F, jpvt, tau);
  form_q(n, F, tau, U);
  for (int i = 0; i < n; ++i) D[i] = fabs(F[(size_t)i * n + i]);
  /* T[i][jpvt[j]] = R[i][j] / D[i] */
  memset(T, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) T[(size_t)i * n + jpvt[j]] = F[(size_t)i * n + j] / D[i];
  free(F);
  free(tau);
  free(jpvt);
}

/* One-sided Jacobi SVD (Hestenes; the stabilizer the paper compares with
 * the QR decomposition in Sec. 4.2 and finds accurate with either inversion
 * scheme): column pairs (p, q) of A are rotated, in cyclic order p < q,
 * until every pair is orthogonal to working accuracy,
 * |a_p . a_q| <= n eps ||a_p|| ||a_q||.  Then A_in V = A_out with V the
 * product of the rotations, the columns of A_out have norms sigma_j, and
 * A_in = U diag(sigma) V^T with U = A_out diag(1/sigma).  The rotation that
 * makes a pair orthogonal:  zeta = (a_q.a_q - a_p.a_p) / (2 a_p.a_q),
 * t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t,
 * a_p <- c a_p - s a_q, a_q <- s a_p + c a_q.  Returns the number of sweeps,
 * or -1 without convergence in 60 sweeps.  Row-major n x n A and V. */
static int jacobi_svd(int n, double* A, double* V) {
  const double tol = n * DBL_EPSILON;
  mat_eye(n, V);
  for (int sweep = 1; sweep <= 60; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double app = 0.0, aqq = 0.0, apq = 0.0;
        for (int i = 0; i < n; ++i) {
          const double x = A[(size_t)i * n + p], y = A[(size_t)i * n + q];
          app += x * x;
          aqq += y * y;
          apq += x * y;
        }
        if (app == 0.0 || aqq == 0.0) continue;
        if (fabs(apq) <= tol * sqrt(app) * sqrt(aqq)) continue;
        rotated = 1;
        const double zeta = (aqq - app) / (2.0 * apq);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < n; ++i) {
          double* a = A + (size_t)i * n;
          const double x = a[p], y = a[q];
          a[p] = c * x - sn * y;
          a[q] = sn * x + c * y;
          double* v = V + (size_t)i * n;
          const double vx = v[p], vy = v[q];
          v[p] = c * vx - sn * vy;
          v[q] = sn * vx + c * vy;
        }
      }
    if (!rotated) return sweep;
  }
  return -1;
}

/* UDT by the SVD: W = U diag(D) T with D = sigma in descending order (as
 * LAPACK's gesvj returns them), T = V^T. */
static int udt_svd(int n, const double* W, double* U, double* D, double* T) {
  double* A = mat_new(n);
  double* V = mat_new(n);
  double* sg = (double*)malloc(sizeof(double) * n);
  int* ord = (int*)malloc(sizeof(int) * n);
  mat_copy(n, W, A);
  const int sweeps = jacobi_svd(n, A, V);
  for (int j = 0; j < n; ++j) {
    sg[j] = nrm2(n, A + j, n);
    ord[j] = j;
  }
  /* insertion sort of the column order by decreasing sigma (stable) */
  for (int a = 1; a < n; ++a) {
    const int c = ord[a];
    int b = a - 1;
    while (b >= 0 && sg[ord[b]] < sg[c]) {
      ord[b + 1] = ord[b];
      --b;
    }
    ord[b + 1] = c;
  }
  for (int j = 0; j < n; ++j) {
    const int c = ord[j];
    D[j] = sg[c];
    for (int i = 0; i < n; ++i) U[(size_t)i * n + j] = sg[c] > 0.0 ? A[(size_t)i * n + c] / sg[c] : 0.0;
    for (int i = 0; i < n; ++i) T[(size_t)j * n + i] = V[(size_t)i * n + c];
  }
  free(A);
  free(V);
  free(sg);
  free(ord);
  return sweeps;
}

/* Inverse with log|det| and sign of det via Gaussian elimination with
 * partial pivoting (Gauss-Jordan on [A | I]). */
static void lu_inverse(int n, const double* A, double* Ainv, double* logabsdet, double* sgn) {
  double* W = mat_new(n);
  mat_copy(n, A, W);
  mat_eye(n, Ainv);
  double ld = 0.0, sg = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(W[(size_t)r * n + c]) > fabs(W[(size_t)p * n + c])) p = r;
    if (p != c) {
      for (int j = 0; j < n; ++j) {
        double t = W[(size_t)c * n + j]; W[(size_t)c * n + j] = W[(size_t)p * n + j]; W[(size_t)p * n + j] = t;
        t = Ainv[(size_t)c * n + j]; Ainv[(size_t)c * n + j] = Ainv[(size_t)p * n + j]; Ainv[(size_t)p * n + j] = t;
      }
      sg = -sg;
    }
    const double piv = W[(size_t)c * n + c];
    ld += log(fabs(piv));
    if (piv < 0) sg = -sg;
    const double ip = 1.0 / piv;
    for (int j = 0; j < n; ++j) { W[(size_t)c * n + j] *= ip; Ainv[(size_t)c * n + j] *= ip; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = W[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        W[(size_t)r * n + j] -= f * W[(size_t)c * n + j];
        Ainv[(size_t)r * n + j] -= f * Ainv[(size_t)c * n + j];
      }
    }
  }
  if (logabsdet) *logabsdet = ld;
  if (sgn) *sgn = sg;
  free(W);
}

/* M^{-1} through the udx (pivoted QR) of M:  M P = Q R  =>
 * M^{-1} = P R^{-1} Q^T.  Also log|det M| and sign det M
 * (det Q = (-1)^{#reflections}, det P = permutation parity). */
static void qr_inverse(int n, const double* M, double* Minv, double* logabsdet, double* sgn) {
  double* F = mat_new(n);
  double* Q = mat_new(n);
  double* Z = mat_new(n);
  double* tau = (double*)malloc(sizeof(double) * n);
  int* jpvt = (int*)malloc(sizeof(int) * n);
  mat_copy(n, M, F);
  cpqr(n, F, jpvt, tau);
  form_q(n, F, tau, Q);
  /* Z = R^{-1} Q^T by back substitution, column by column of Q^T */
  for (int c = 0; c < n; ++c) {
    for (int i = n - 1; i >= 0; --i) {
      double s = Q[(size_t)c * n + i]; /* (Q^T)[i][c] */
      for (int j = i + 1; j < n; ++j) s -= F[(size_t)i * n + j] * Z[(size_t)j * n + c];
      Z[(size_t)i * n + c] = s / F[(size_t)i * n + i];
    }
  }
  /* Minv = P Z : row j of Z goes to row jpvt[j] */
  for (int j = 0; j < n; ++j)
    memcpy(Minv + (size_t)jpvt[j] * n, Z + (size_t)j * n, sizeof(double) * n);
  double ld = 0.0, sg = perm_sign(n, jpvt);
  for (int i = 0; i < n; ++i) {
    const double r = F[(size_t)i * n + i];
    ld += log(fabs(r));
    if (r < 0) sg = -sg;
    if (tau[i] != 0.0) sg = -sg;
  }
  if (logabsdet) *logabsdet = ld;
  if (sgn) *sgn = sg;
  free(F); free(Q); free(Z); free(tau); free(jpvt);
}

/* ------------------------------------------------------------------------ */
/* slices and stabilized chains                                             */

typedef struct {
  int n, m, k;
  const double* expk;      /* E, or H = E^{1/2} when sym is set */
  const double* expk_inv;  /* E^{-1}, or H^{-1} when sym is set */
  const double* field;
  double alpha;
  int sym;                 /* 1: the symmetric Trotter slice H diag(v) H (Sec. 2) */
  int svd;                 /* 1: stabilize with the Jacobi SVD instead of the QR */
  const double* dense;     /* dense slices [m][n][n] (B_q at dense + (q-1) n n), or NULL */
} problem;

enum { SLICE_B = 0, SLICE_BINV = 1, SLICE_BT = 2, SLICE_BSYM = 3, SLICE_BSYMINV = 4, SLICE_DENSE = 5,
       SLICE_DENSEINV = 6 };

/* W <- X_q W with X_q = B_q, B_q^{-1} or B_q^T (q is 1-based). */
static void apply_slice(const problem* P, int kind, int q, double* W, double* tmp) {
  const int n = P->n;
  if (kind == SLICE_DENSE) {         /* B_q as given */
    mat_mul(n, P->dense + (size_t)(q - 1) * n * n, W, tmp);
    mat_copy(n, tmp, W);
    return;
  }
  if (kind == SLICE_DENSEINV) {      /* B_q^{-1} by Gauss-Jordan */
    double* Bi = mat_new(n);
    lu_inverse(n, P->dense + (size_t)(q - 1) * n * n, Bi, NULL, NULL);
    mat_mul(n, Bi, W, tmp);
    mat_copy(n, tmp, W);
    free(Bi);
    return;
  }
  double* v = (double*)malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i) v[i] = exp(P->alpha * P->field[(size_t)(q - 1) * n + i]);
  if (kind == SLICE_B) {             /* B_q = E diag(v) */
    scale_rows(n, W, v);
    mat_mul(n, P->expk, W, tmp);
    mat_copy(n, tmp, W);
  } else if (kind == SLICE_BINV) {   /* B_q^{-1} = diag(1/v) E^{-1} */
    mat_mul(n, P->expk_inv, W, tmp);
    for (int i = 0; i < n; ++i) v[i] = 1.0 / v[i];
    scale_rows(n, tmp, v);
    mat_copy(n, tmp, W);
  } else if (kind == SLICE_BSYM) {   /* B_q = H diag(v) H, H = E^{1/2} */
    mat_mul(n, P->expk, W, tmp);
    scale_rows(n, tmp, v);
    mat_mul(n, P->expk, tmp, W);
  } else if (kind == SLICE_BSYMINV) {  /* B_q^{-1} = H^{-1} diag(1/v) H^{-1} */
    mat_mul(n, P->expk_inv, W, tmp);
    for (int i = 0; i < n; ++i) v[i] = 1.0 / v[i];
    scale_rows(n, tmp, v);
    mat_mul(n, P->expk_inv, tmp, W);
  } else {                           /* B_q^T = diag(v) E^T */
    mat_mul_tn(n, P->expk, W, tmp);
    scale_rows(n, tmp, v);
    mat_copy(n, tmp, W);
  }
  free(v);
}

/* UDT of the product X_{q_count-1} ... X_{q_1} X_{q_0} (applied in the order
 * given by `order`), starting from U = I, D = 1, T = I.  Every k slices the
 * naively multiplied block is folded in with the stabilized product of
 * Sec. 4.1:  block * (U D T) = ((block U) D) T = (U' D' T') T, i.e.
 * U <- U', D <- D', T <- T' T. */
static void chain_udt(const problem* P, int kind, const int* order, int count,
                      double* U, double* D, double* T) {
  const int n = P->n;
  double* W = mat_new(n);
  double* tmp = mat_new(n);
  double* Tp = mat_new(n);
  double* T2 = mat_new(n);
  mat_eye(n, U);
  mat_eye(n, T);
  for (int i = 0; i < n; ++i) D[i] = 1.0;
  int pos = 0;
  while (pos < count) {
    const int end = (pos + P->k < count) ? pos + P->k : count;
    mat_copy(n, U, W);
    for (int s = pos; s < end; ++s) apply_slice(P, kind, order[s], W, tmp);
    scale_cols(n, W, D);
    if (P->svd)
      udt_svd(n, W, U, D, Tp);
    else
      udt(n, W, U, D, Tp);
    mat_mul(n, Tp, T, T2);
    mat_copy(n, T2, T);
    pos = end;
  }
  free(W); free(tmp); free(Tp); free(T2);
}

/* forward chain B_b ... B_a  (slices a..b, a <= b; empty if a > b) */
static void chain_fwd(const problem* P, int a, int b, double* U, double* D, double* T) {
  const int cnt = b >= a ? b - a + 1 : 0;
  int* order = (int*)malloc(sizeof(int) * (cnt ? cnt : 1));
  for (int s = 0; s < cnt; ++s) order[s] = a + s;
  chain_udt(P, P->dense ? SLICE_DENSE : (P->sym ? SLICE_BSYM : SLICE_B), order, cnt, U, D, T);
  free(order);
}

/* B_a^{-1} ... B_b^{-1}: applied as W <- B_q^{-1} W for q = b, b-1, ..., a */
static void chain_inv(const problem* P, int a, int b, double* U, double* D, double* T) {
  const int cnt = b >= a ? b - a + 1 : 0;
  int* order = (int*)malloc(sizeof(int) * (cnt ? cnt : 1));
  for (int s = 0; s < cnt; ++s) order[s] = b - s;
  chain_udt(P, P->dense ? SLICE_DENSEINV : (P->sym ? SLICE_BSYMINV : SLICE_BINV), order, cnt, U, D, T);
  free(order);
}

/* B_a^T ... B_b^T = (B_b ... B_a)^T: W <- B_q^T W for q = b, ..., a */
static void chain_trn(const problem* P, int a, int b, double* U, double* D, double* T) {
  const int cnt = b >= a ? b - a + 1 : 0;
  int* order = (int*)malloc(sizeof(int) * (cnt ? cnt : 1));
  for (int s = 0; s < cnt; ++s) order[s] = b - s;
  chain_udt(P, SLICE_BT, order, cnt, U, D, T);
  free(order);
}

/* ------------------------------------------------------------------------ */
/* inversion schemes                                                        */

/* Sec. 5.1, inv_one_plus_loh:  with Dp = max(D,1), Dm = min(D,1),
 *   1 + U D X = (X^{-1} Dp^{-1} + U Dm) Dp X
 *   G = X^{-1} Dp^{-1} M^{-1},   M = X^{-1} Dp^{-1} + U Dm,
 * M inverted through its udx.  det(1 + UDX) = det M * prod(Dp) * det X. */
static void inv_one_plus_loh(int n, const double* U, const double* D, const double* X,
                             double* G, double* logdet, double* sgn) {
  double* Xi = mat_new(n);
  double* Mm = mat_new(n);
  double* Mi = mat_new(n);
  double* tmp = mat_new(n);
  double* dpi = (double*)malloc(sizeof(double) * n);
  double* dm = (double*)malloc(sizeof(double) * n);
  double ldx, sx, ldm, sm, ld = 0.0;
  for (int i = 0; i < n; ++i) {
    const double dp = D[i] > 1.0 ? D[i] : 1.0;
    dpi[i] = 1.0 / dp;
    dm[i] = D[i] < 1.0 ? D[i] : 1.0;
    ld += log(dp);
  }
  lu_inverse(n, X, Xi, &ldx, &sx);
  /* M = Xi Dp^{-1} + U Dm */
  mat_copy(n, Xi, Mm);
  scale_cols(n, Mm, dpi);
  mat_copy(n, U, tmp);
  scale_cols(n, tmp, dm);
  for (int i = 0; i < n * n; ++i) Mm[i] += tmp[i];
  qr_inverse(n, Mm, Mi, &ldm, &sm);
  /* G = Xi (Dp^{-1} Mi) */
  scale_rows(n, Mi, dpi);
  mat_mul(n, Xi, Mi, G);
  if (logdet) *logdet = ld + ldm + ldx;
  if (sgn) *sgn = sm * sx;
  free(Xi); free(Mm); free(Mi); free(tmp); free(dpi); free(dm);
}

/* Sec. 5.1, inv_one_plus:  1 + U D X = U (U^T X^{-1} + D) X,
 * G = X^{-1} (U^T X^{-1} + D)^{-1} U^T. */
static void inv_one_plus(int n, const double* U, const double* D, const double* X,
                         double* G, double* logdet, double* sgn) {
  double* Xi = mat_new(n);
  double* Mm = mat_new(n);
  double* Mi = mat_new(n);
  double* tmp = mat_new(n);
  double ldx, sx, ldm, sm, ldu, su;
  lu_inverse(n, X, Xi, &ldx, &sx);
  mat_mul_tn(n, U, Xi, Mm);
  for (int i = 0; i < n; ++i) Mm[(size_t)i * n + i] += D[i];
  qr_inverse(n, Mm, Mi, &ldm, &sm);
  mat_mul_nt(n, Mi, U, tmp);   /* Mi U^T */
  mat_mul(n, Xi, tmp, G);
  lu_inverse(n, U, tmp, &ldu, &su);
  if (logdet) *logdet = ldm + ldx + ldu;
  if (sgn) *sgn = sm * sx * su;
  free(Xi); free(Mm); free(Mi); free(tmp);
}

/* Sec. 6.1, inv_sum_loh.  G = [U_L D_L X_L + U_R D_R X_R]^{-1} with
 *   Mid = D_Lm (X_L X_R^{-1}) D_Rp^{-1} + D_Lp^{-1} (U_L^T U_R) D_Rm
 *   G   = X_R^{-1} D_Rp^{-1} Mid^{-1} D_Lp^{-1} U_L^T.
 * Reading: the printed middle matrix is garbled (fractions of diagonal
 * matrices and a swapped "X_R D_Rp"); we read D_Lm/D_Rp as a left factor D_Lm
 * and a right factor D_Rp^{-1} (likewise D_Rm/D_Lp), and the tail as
 * D_Rp X_R, which is what the paper's next line requires. */
static void inv_sum_loh(int n, const double* UL, const double* DL, const double* XL,
                        const double* UR, const double* DR, const double* XR, double* G) {
  double* XRi = mat_new(n);
  double* A = mat_new(n);
  double* B = mat_new(n);
  double* Mi = mat_new(n);
  double* tmp = mat_new(n);
  double *dlm = malloc(sizeof(double) * n), *dlpi = malloc(sizeof(double) * n);
  double *drm = malloc(sizeof(double) * n), *drpi = malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i) {
    dlm[i] = DL[i] < 1.0 ? DL[i] : 1.0;
    dlpi[i] = 1.0 / (DL[i] > 1.0 ? DL[i] : 1.0);
    drm[i] = DR[i] < 1.0 ? DR[i] : 1.0;
    drpi[i] = 1.0 / (DR[i] > 1.0 ? DR[i] : 1.0);
  }
  lu_inverse(n, XR, XRi, NULL, NULL);
  mat_mul(n, XL, XRi, A);      /* X_L X_R^{-1} */
  scale_rows(n, A, dlm);
  scale_cols(n, A, drpi);
  mat_mul_tn(n, UL, UR, B);    /* U_L^T U_R */
  scale_rows(n, B, dlpi);
  scale_cols(n, B, drm);
  for (int i = 0; i < n * n; ++i) A[i] += B[i];
  qr_inverse(n, A, Mi, NULL, NULL);
  /* G = XRi (D_Rp^{-1} (Mi (D_Lp^{-1} U_L^T))) */
  scale_rows(n, Mi, drpi);
  scale_cols(n, Mi, dlpi);
  mat_mul_nt(n, Mi, UL, tmp);
  mat_mul(n, XRi, tmp, G);
  free(XRi); free(A); free(B); free(Mi); free(tmp);
  free(dlm); free(dlpi); free(drm); free(drpi);
}

/* Sec. 6.1, inv_sum:  Mid = D_L X_L X_R^{-1} + U_L^T U_R D_R,
 * G = X_R^{-1} Mid^{-1} U_L^T.  (The printed bracket carries d^{-1}; with
 * D_r = d^{-1} the bracket holds the plain udx, which is what we use.) */
static void inv_sum(int n, const double* UL, const double* DL, const double* XL,
                    const double* UR, const double* DR, const double* XR, double* G) {
  double* XRi = mat_new(n);
  double* A = mat_new(n);
  double* B = mat_new(n);
  double* Mi = mat_new(n);
  double* tmp = mat_new(n);
  lu_inverse(n, XR, XRi, NULL, NULL);
  mat_mul(n, XL, XRi, A);
  scale_rows(n, A, DL);
  mat_mul_tn(n, UL, UR, B);
  scale_cols(n, B, DR);
  for (int i = 0; i < n * n; ++i) A[i] += B[i];
  qr_inverse(n, A, Mi, NULL, NULL);
  mat_mul_nt(n, Mi, UL, tmp);
  mat_mul(n, XRi, tmp, G);
  free(XRi); free(A); free(B); free(Mi); free(tmp);
}

/* ------------------------------------------------------------------------ */
/* exported entry points                                                    */

static int check(int n, int m, int k, const double* expk, const double* field) {
  if (n <= 0 || m <= 0 || k <= 0 || !expk || !field) return OR_EINVAL;
  for (size_t i = 0; i < (size_t)m * n; ++i)
    if (!isfinite(field[i])) return OR_ERANGE;
  return OR_OK;
}

static int finite_all(int n, const double* A) {
  for (size_t i = 0; i < (size_t)n * n; ++i)
    if (!isfinite(A[i])) return 0;
  return 1;
}

int or_greens(int n, int m, int k, const double* expk, const double* field, double alpha,
              int scheme, double* G, double* logdet, double* sign) {
  int st = check(n, m, k, expk, field);
  if (st) return st;
  problem P = {n, m, k, expk, NULL, field, alpha};
  double* U = mat_new(n);
  double* T = mat_new(n);
  double* D = (double*)malloc(sizeof(double) * n);
  chain_fwd(&P, 1, m, U, D, T);
  if (scheme == OR_SCHEME_PLAIN)
    inv_one_plus(n, U, D, T, G, logdet, sign);
  else
    inv_one_plus_loh(n, U, D, T, G, logdet, sign);
  free(U); free(T); free(D);
  return finite_all(n, G) ? OR_OK : OR_ERANGE;
}

/* G(tau_l, 0) for 0 <= l <= m (Sec. 6): with tau_2 = 0,
 *   G(tau_l, 0) = [B_1^{-1} ... B_l^{-1} + B_M ... B_{l+1}]^{-1}
 * where each of the two chains is brought to UDX form on its own (left:
 * U_L D_L X_L, right: U_R D_R X_R) and the sum is inverted by inv_sum_loh
 * (scheme OR_SCHEME_LOH) or inv_sum (OR_SCHEME_PLAIN). */
int or_greens_tdisp(int n, int m, int k, const double* expk, const double* expk_inv,
                    const double* field, double alpha, int l, int scheme, double* Gt) {
  int st = check(n, m, k, expk, field);
  if (st) return st;
  if (!expk_inv || l < 0 || l > m) return OR_EINVAL;
  problem P = {n, m, k, expk, expk_inv, field, alpha};
  double *UL = mat_new(n), *XL = mat_new(n), *UR = mat_new(n), *XR = mat_new(n);
  double *DL = malloc(sizeof(double) * n), *DR = malloc(sizeof(double) * n);
  chain_inv(&P, 1, l, UL, DL, XL);
  chain_fwd(&P, l + 1, m, UR, DR, XR);
  if (scheme == OR_SCHEME_PLAIN)
    inv_sum(n, UL, DL, XL, UR, DR, XR, Gt);
  else
    inv_sum_loh(n, UL, DL, XL, UR, DR, XR, Gt);
  free(UL); free(XL); free(UR); free(XR); free(DL); free(DR);
  return finite_all(n, Gt) ? OR_OK : OR_ERANGE;
}

/* The same two quantities for the symmetric Trotter slices of Sec. 2,
 *   B_l = H diag(exp(alpha f_l)) H,  H = exp(-dtau K / 2)  (expk_half),
 * multiplied out slice by slice in that form (no similarity transform is
 * used): G and log|det|, sign by inv_one_plus_loh; G(tau_l, 0) by the two
 * chains of B^{-1} = H^{-1} diag(1/v) H^{-1} and B, and inv_sum_loh. */
int or_greens_sym(int n, int m, int k, const double* expk_half, const double* field, double alpha,
                  double* G, double* logdet, double* sign) {
  int st = check(n, m, k, expk_half, field);
  if (st) return st;
  problem P = {n, m, k, expk_half, NULL, field, alpha, 1};
  double* U = mat_new(n);
  double* T = mat_new(n);
  double* D = (double*)malloc(sizeof(double) * n);
  chain_fwd(&P, 1, m, U, D, T);
  inv_one_plus_loh(n, U, D, T, G, logdet, sign);
  free(U); free(T); free(D);
  return finite_all(n, G) ? OR_OK : OR_ERANGE;
}

int or_greens_tdisp_sym(int n, int m, int k, const double* expk_half, const double* expk_half_inv,
                        const double* field, double alpha, int l, double* Gt) {
  int st = check(n, m, k, expk_half, field);
  if (st) return st;
  if (!expk_half_inv || l < 0 || l > m) return OR_EINVAL;
  problem P = {n, m, k, expk_half, expk_half_inv, field, alpha, 1};
  double *UL = mat_new(n), *XL = mat_new(n), *UR = mat_new(n), *XR = mat_new(n);
  double *DL = malloc(sizeof(double) * n), *DR = malloc(sizeof(double) * n);
  chain_inv(&P, 1, l, UL, DL, XL);
  chain_fwd(&P, l + 1, m, UR, DR, XR);
  inv_sum_loh(n, UL, DL, XL, UR, DR, XR, Gt);
  free(UL); free(XL); free(UR); free(XR); free(DL); free(DR);
  return finite_all(n, Gt) ? OR_OK : OR_ERANGE;
}

/* Equal-time G at slice l, 1 <= l <= m (Sec. 6 definition),
 *   G_l = [1 + B_{l-1} ... B_1 B_M ... B_l]^{-1},
 * combined from two stack elements as in App. A.1:
 *   B_{l-1}...B_1 = U_L D_L T_L,   (B_M...B_l)^T = U_R D_R T_R,
 *   1 + U_L D_L T_L (U_R D_R T_R)^T = 1 + U_L [D_L (T_L T_R^T) D_R] U_R^T,
 * udt of the bracket = u d t, then U = U_L u, D = d, T = t U_R^T and the
 * equal-time scheme inv_one_plus_loh.  logdet/sign of det(1 + ...) too
 * (the same for every l: det is invariant under the cyclic shift). */
int or_greens_slice(int n, int m, int k, const double* expk, const double* field,
                    double alpha, int l, double* Gl, double* logdet, double* sign) {
  int st = check(n, m, k, expk, field);
  if (st) return st;
  if (l < 1 || l > m) return OR_EINVAL;
  problem P = {n, m, k, expk, NULL, field, alpha};
  double *UL = mat_new(n), *TL = mat_new(n), *UR = mat_new(n), *TR = mat_new(n);
  double *DL = malloc(sizeof(double) * n), *DR = malloc(sizeof(double) * n);
  double *Mm = mat_new(n), *u = mat_new(n), *t = mat_new(n), *d = malloc(sizeof(double) * n);
  double *U = mat_new(n), *T = mat_new(n);
  chain_fwd(&P, 1, l - 1, UL, DL, TL);
  chain_trn(&P, l, m, UR, DR, TR);
  mat_mul_nt(n, TL, TR, Mm);
  scale_rows(n, Mm, DL);
  scale_cols(n, Mm, DR);
  udt(n, Mm, u, d, t);
  mat_mul(n, UL, u, U);
  mat_mul_nt(n, t, UR, T);
  inv_one_plus_loh(n, U, d, T, Gl, logdet, sign);
  free(UL); free(TL); free(UR); free(TR); free(DL); free(DR);
  free(Mm); free(u); free(t); free(d); free(U); free(T);
  return finite_all(n, Gl) ? OR_OK : OR_ERANGE;
}

/* Gradient of log|det(1 + B_M ... B_1)| with respect to the field entries.
 * dB_l / df_{l,i} = alpha B_l e_i e_i^T, and with X = B_{l-1}...B_1,
 * Y = B_M...B_l Jacobi's formula gives
 *   d log|det(1 + Y X)| = tr[(1 + Y X)^{-1} alpha B_M..B_l e_i e_i^T B_{l-1}..B_1]
 *                       = alpha [X (1 + Y X)^{-1} Y]_ii = alpha (1 - G_l)_ii,
 * using X (1 + Y X)^{-1} Y = 1 - (1 + X Y)^{-1} and G_l = (1 + X Y)^{-1}.
 * Every requested G_l is computed from scratch by or_greens_slice.
 * grad is [n_l][n]: row r holds the gradient for slice l_list[r]. */
int or_logdet_grad(int n, int m, int k, const double* expk, const double* field, double alpha,
                   const int* l_list, int n_l, double* grad) {
  double* Gl = mat_new(n);
  int st = OR_OK;
  for (int r = 0; r < n_l && st == OR_OK; ++r) {
    st = or_greens_slice(n, m, k, expk, field, alpha, l_list[r], Gl, NULL, NULL);
    for (int i = 0; i < n; ++i) grad[(size_t)r * n + i] = alpha * (1.0 - Gl[(size_t)i * n + i]);
  }
  free(Gl);
  return st;
}

/* Sec. 3: the unstabilized chain product and a plain inverse of 1 + B
 * (negative control: fails once exp(bandwidth * beta) exceeds 1/eps). */
int or_greens_naive(int n, int m, int k, const double* expk, const double* field,
                    double alpha, double* G) {
  (void)k;
  int st = check(n, m, 1, expk, field);
  if (st) return st;
  problem P = {n, m, 1, expk, NULL, field, alpha};
  double *W = mat_new(n), *tmp = mat_new(n);
  mat_eye(n, W);
  for (int q = 1; q <= m; ++q) apply_slice(&P, SLICE_B, q, W, tmp);
  for (int i = 0; i < n; ++i) W[(size_t)i * n + i] += 1.0;
  lu_inverse(n, W, G, NULL, NULL);
  free(W); free(tmp);
  return OR_OK;
}

/* UDT of a stabilized chain, exposed for the tests: kind 0 = B_b..B_a,
 * 1 = B_a^{-1}..B_b^{-1}, 2 = B_a^T..B_b^T. */
int or_chain(int n, int m, int k, const double* expk, const double* expk_inv,
             const double* field, double alpha, int kind, int a, int b,
             double* U, double* D, double* T) {
  int st = check(n, m, k, expk, field);
  if (st) return st;
  problem P = {n, m, k, expk, expk_inv, field, alpha};
  if (kind == 0) chain_fwd(&P, a, b, U, D, T);
  else if (kind == 1) chain_inv(&P, a, b, U, D, T);
  else chain_trn(&P, a, b, U, D, T);
  return OR_OK;
}

/* Pivoted QR exposed for the tests: A (row-major n x n) is overwritten with
 * R in the upper triangle; Q and jpvt returned. */
/* or_greens and or_greens_tdisp with the stabilizer chosen: stab = 0 the
 * pivoted QR, 1 the one-sided Jacobi SVD. */
int or_greens_stab(int n, int m, int k, const double* expk, const double* field, double alpha,
                   int scheme, int stab, double* G, double* logdet, double* sign) {
  int st = check(n, m, k, expk, field);
  if (st) return st;
  problem P = {n, m, k, expk, NULL, field, alpha, 0, stab};
  double* U = mat_new(n);
  double* T = mat_new(n);
  double* D = (double*)malloc(sizeof(double) * n);
  chain_fwd(&P, 1, m, U, D, T);
  if (scheme == OR_SCHEME_PLAIN)
    inv_one_plus(n, U, D, T, G, logdet, sign);
  else
    inv_one_plus_loh(n, U, D, T, G, logdet, sign);
  free(U); free(T); free(D);
  return finite_all(n, G) ? OR_OK : OR_ERANGE;
}

int or_greens_tdisp_stab(int n, int m, int k, const double* expk, const double* expk_inv,
                         const double* field, double alpha, int l, int scheme, int stab, double* Gt) {
  int st = check(n, m, k, expk, field);
  if (st) return st;
  if (!expk_inv || l < 0 || l > m) return OR_EINVAL;
  problem P = {n, m, k, expk, expk_inv, field, alpha, 0, stab};
  double *UL = mat_new(n), *XL = mat_new(n), *UR = mat_new(n), *XR = mat_new(n);
  double *DL = malloc(sizeof(double) * n), *DR = malloc(sizeof(double) * n);
  chain_inv(&P, 1, l, UL, DL, XL);
  chain_fwd(&P, l + 1, m, UR, DR, XR);
  if (scheme == OR_SCHEME_PLAIN)
    inv_sum(n, UL, DL, XL, UR, DR, XR, Gt);
  else
    inv_sum_loh(n, UL, DL, XL, UR, DR, XR, Gt);
  free(UL); free(XL); free(UR); free(XR); free(DL); free(DR);
  return finite_all(n, Gt) ? OR_OK : OR_ERANGE;
}

/* Equal-time G, log|det| and sign for dense slices (B_l given as matrices;
 * generalized slices): the same chain and inv_one_plus_loh. */
int or_greens_dense(int n, int m, int k, const double* slices, double* G, double* logdet, double* sign) {
  if (n <= 0 || m <= 0 || k <= 0 || !slices) return OR_EINVAL;
  for (size_t i = 0; i < (size_t)m * n * n; ++i)
    if (!isfinite(slices[i])) return OR_EINVAL;
  problem P = {n, m, k, NULL, NULL, NULL, 0.0, 0, 0, slices};
  double* U = mat_new(n);
  double* T = mat_new(n);
  double* D = (double*)malloc(sizeof(double) * n);
  chain_fwd(&P, 1, m, U, D, T);
  inv_one_plus_loh(n, U, D, T, G, logdet, sign);
  free(U); free(T); free(D);
  return finite_all(n, G) ? OR_OK : OR_ERANGE;
}

/* G(tau_l, 0) for dense slices: the chain B_1^{-1}..B_l^{-1} (each slice
 * inverted by Gauss-Jordan) and B_M..B_{l+1}, combined by inv_sum_loh. */
int or_greens_tdisp_dense(int n, int m, int k, const double* slices, int l, double* Gt) {
  if (n <= 0 || m <= 0 || k <= 0 || !slices || l < 0 || l > m) return OR_EINVAL;
  problem P = {n, m, k, NULL, NULL, NULL, 0.0, 0, 0, slices};
  double *UL = mat_new(n), *XL = mat_new(n), *UR = mat_new(n), *XR = mat_new(n);
  double *DL = malloc(sizeof(double) * n), *DR = malloc(sizeof(double) * n);
  chain_inv(&P, 1, l, UL, DL, XL);
  chain_fwd(&P, l + 1, m, UR, DR, XR);
  inv_sum_loh(n, UL, DL, XL, UR, DR, XR, Gt);
  free(UL); free(XL); free(UR); free(XR); free(DL); free(DR);
  return finite_all(n, Gt) ? OR_OK : OR_ERANGE;
}

/* The Jacobi SVD of one matrix: W = U diag(s) V^T (s descending); returns the
 * number of sweeps (-1: no convergence). */
int or_svd(int n, const double* W, double* U, double* s, double* V) {
  double* T = mat_new(n);
  const int sweeps = udt_svd(n, W, U, s, T);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = T[(size_t)j * n + i];
  free(T);
  return sweeps;
}

int or_cpqr(int n, double* A, double* Q, int* jpvt) {
  double* tau = (double*)malloc(sizeof(double) * n);
  cpqr(n, A, jpvt, tau);
  form_q(n, A, tau, Q);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A[(size_t)i * n + j] = 0.0;
  free(tau);
  return OR_OK;
}

int or_udt(int n, const double* W, double* U, double* D, double* T) {
  udt(n, W, U, D, T);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Complex UDT (the complex slices of App. B need the decomposition of
 * Sec. 4.2.2 over the complex numbers).  Row-major n x n matrices of
 * double complex (interleaved re, im).                                      */

/* 2-norm of the m entries x[0], x[inc], ... without overflow */
static double cnrm2(int m, const double complex* x, int inc) {
  double scale = 0.0, ssq = 1.0;
  for (int i = 0; i < m; ++i) {
    const double part[2] = {creal(x[(size_t)i * inc]), cimag(x[(size_t)i * inc])};
    for (int h = 0; h < 2; ++h) {
      const double a = fabs(part[h]);
      if (a == 0.0) continue;
      if (scale < a) {
        ssq = 1.0 + ssq * (scale / a) * (scale / a);
        scale = a;
      } else {
        ssq += (a / scale) * (a / scale);
      }
    }
  }
  return scale * sqrt(ssq);
}

/* Column-pivoted Householder QR over the complex numbers, in place:
 * A_in P = Q R with Q = H_0 ... H_{n-1}, H_j = I - tau_j v_j v_j^H (unit
 * leading entry of v_j implied; v_j stored below the diagonal).  The same
 * pivot rule and norm downdating as the real cpqr.  Reflector of x = A[j:, j]
 * with alpha = x_0: beta = -sign(Re alpha) ||x|| (real), tau = (beta -
 * alpha) / beta, v = x / (alpha - beta), so that H^H x = beta e_0 and the
 * diagonal of R is real; tau = 0 when x_1.. = 0 and alpha is real.  H_j^H is
 * applied to the trailing columns: a <- a - conj(tau) v (v^H a). */
static void cpqr_c(int n, double complex* A, int* jpvt, double complex* tau) {
  double* vn1 = (double*)malloc(sizeof(double) * n);
  double* vn2 = (double*)malloc(sizeof(double) * n);
  const double tol3z = sqrt(2.220446049250313e-16);
  for (int j = 0; j < n; ++j) {
    jpvt[j] = j;
    vn1[j] = cnrm2(n, A + j, n);
    vn2[j] = vn1[j];
  }
  for (int i = 0; i < n; ++i) {
    int p = i;
    for (int j = i + 1; j < n; ++j)
      if (vn1[j] > vn1[p]) p = j;
    if (p != i) {
      for (int r = 0; r < n; ++r) {
        const double complex t = A[(size_t)r * n + i];
        A[(size_t)r * n + i] = A[(size_t)r * n + p];
        A[(size_t)r * n + p] = t;
      }
      int tj = jpvt[i]; jpvt[i] = jpvt[p]; jpvt[p] = tj;
      vn1[p] = vn1[i];
      vn2[p] = vn2[i];
    }
    const double complex alpha = A[(size_t)i * n + i];
    const double xnorm = (i + 1 < n) ? cnrm2(n - i - 1, A + (size_t)(i + 1) * n + i, n) : 0.0;
    double complex t_i = 0.0;
    if (xnorm != 0.0 || cimag(alpha) != 0.0) {
      const double beta = -copysign(hypot(hypot(creal(alpha), cimag(alpha)), xnorm), creal(alpha));
      t_i = (beta - alpha) / beta;
      const double complex s = 1.0 / (alpha - beta);
      for (int r = i + 1; r < n; ++r) A[(size_t)r * n + i] *= s;
      A[(size_t)i * n + i] = beta;
    }
    tau[i] = t_i;
    if (t_i != 0.0) {
      for (int j = i + 1; j < n; ++j) {
        double complex w = A[(size_t)i * n + j];
        for (int r = i + 1; r < n; ++r) w += conj(A[(size_t)r * n + i]) * A[(size_t)r * n + j];
        w *= conj(t_i);
        A[(size_t)i * n + j] -= w;
        for (int r = i + 1; r < n; ++r) A[(size_t)r * n + j] -= w * A[(size_t)r * n + i];
      }
    }
    for (int j = i + 1; j < n; ++j) {
      if (vn1[j] == 0.0) continue;
      double temp = cabs(A[(size_t)i * n + j]) / vn1[j];
      temp = 1.0 - temp * temp;
      if (temp < 0.0) temp = 0.0;
      const double ratio = vn1[j] / vn2[j];
      const double temp2 = temp * ratio * ratio;
      if (temp2 <= tol3z) {
        vn1[j] = (i + 1 < n) ? cnrm2(n - i - 1, A + (size_t)(i + 1) * n + j, n) : 0.0;
        vn2[j] = vn1[j];
      } else {
        vn1[j] *= sqrt(temp);
      }
    }
  }
  free(vn1);
  free(vn2);
}

/* Complex UDT: W P = Q R, U = Q (unitary), D = |diag R| (diag R is real),
 * T = D^{-1} R P^T (a row with D_i = 0 is left undivided). */
int or_udt_complex(int n, const double* Wd, double* Ud, double* D, double* Td) {
  if (n < 1 || !Wd || !Ud || !D || !Td) return OR_EINVAL;
  const double complex* W = (const double complex*)Wd;
  double complex* U = (double complex*)Ud;
  double complex* T = (double complex*)Td;
  double complex* F = (double complex*)malloc(sizeof(double complex) * (size_t)n * n);
  double complex* tau = (double complex*)malloc(sizeof(double complex) * n);
  int* jpvt = (int*)malloc(sizeof(int) * n);
  memcpy(F, W, sizeof(double complex) * (size_t)n * n);
  cpqr_c(n, F, jpvt, tau);
  /* Q = H_0 (H_1 (... H_{n-1} I)) */
  for (size_t e = 0; e < (size_t)n * n; ++e) U[e] = 0.0;
  for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
  for (int i = n - 1; i >= 0; --i) {
    if (tau[i] == 0.0) continue;
    for (int j = 0; j < n; ++j) {
      double complex w = U[(size_t)i * n + j];
      for (int r = i + 1; r < n; ++r) w += conj(F[(size_t)r * n + i]) * U[(size_t)r * n + j];
      w *= tau[i];
      U[(size_t)i * n + j] -= w;
      for (int r = i + 1; r < n; ++r) U[(size_t)r * n + j] -= w * F[(size_t)r * n + i];
    }
  }
  for (size_t e = 0; e < (size_t)n * n; ++e) T[e] = 0.0;
  for (int i = 0; i < n; ++i) {
    D[i] = fabs(creal(F[(size_t)i * n + i]));
    const double s = D[i] > 0.0 ? 1.0 / D[i] : 1.0;
    for (int j = i; j < n; ++j) T[(size_t)i * n + jpvt[j]] = F[(size_t)i * n + j] * s;
  }
  free(F);
  free(tau);
  free(jpvt);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Complex slices (App. B: the slices of the spin-fermion model are complex
 * matrices).  The chain of Sec. 4.1 with the complex UDT of Sec. 4.2.2 and
 * the equal-time G by inv_one_plus_loh (Sec. 5.1), all over the complex
 * numbers; det(1 + B_M...B_1) comes with a complex phase instead of a sign. */

/* C = A B, complex n x n (C must not alias A or B) */
static void cmat_mul(int n, const double complex* A, const double complex* B, double complex* C) {
  for (int i = 0; i < n; ++i) {
    double complex* c = C + (size_t)i * n;
    for (int j = 0; j < n; ++j) c[j] = 0.0;
    for (int p = 0; p < n; ++p) {
      const double complex a = A[(size_t)i * n + p];
      const double complex* b = B + (size_t)p * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
  }
}

/* complex UDT of W (the decomposition of or_udt_complex) */
static void udt_c(int n, const double complex* W, double complex* U, double* D, double complex* T) {
  double complex* F = (double complex*)malloc(sizeof(double complex) * (size_t)n * n);
  double complex* tau = (double complex*)malloc(sizeof(double complex) * n);
  int* jpvt = (int*)malloc(sizeof(int) * n);
  memcpy(F, W, sizeof(double complex) * (size_t)n * n);
  cpqr_c(n, F, jpvt, tau);
  /* Q = H_0 (H_1 (... H_{n-1} I)) */
  for (size_t e = 0; e < (size_t)n * n; ++e) U[e] = 0.0;
  for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
  for (int i = n - 1; i >= 0; --i) {
    if (tau[i] == 0.0) continue;
    for (int j = 0; j < n; ++j) {
      double complex w = U[(size_t)i * n + j];
      for (int r = i + 1; r < n; ++r) w += conj(F[(size_t)r * n + i]) * U[(size_t)r * n + j];
      w *= tau[i];
      U[(size_t)i * n + j] -= w;
      for (int r = i + 1; r < n; ++r) U[(size_t)r * n + j] -= w * F[(size_t)r * n + i];
    }
  }
  for (size_t e = 0; e < (size_t)n * n; ++e) T[e] = 0.0;
  for (int i = 0; i < n; ++i) {
    D[i] = fabs(creal(F[(size_t)i * n + i]));
    const double s = D[i] > 0.0 ? 1.0 / D[i] : 1.0;
    for (int j = i; j < n; ++j) T[(size_t)i * n + jpvt[j]] = F[(size_t)i * n + j] * s;
  }
  free(F);
  free(tau);
  free(jpvt);
}

/* Inverse of a complex matrix by Gauss-Jordan elimination with partial
 * pivoting on [A | I], with log|det A| and the phase det A / |det A|. */
static void lu_inverse_c(int n, const double complex* A, double complex* Ainv, double* logabsdet,
                         double complex* phase) {
  double complex* W = (double complex*)malloc(sizeof(double complex) * (size_t)n * n);
  memcpy(W, A, sizeof(double complex) * (size_t)n * n);
  for (size_t e = 0; e < (size_t)n * n; ++e) Ainv[e] = 0.0;
  for (int i = 0; i < n; ++i) Ainv[(size_t)i * n + i] = 1.0;
  double ld = 0.0;
  double complex ph = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (cabs(W[(size_t)r * n + c]) > cabs(W[(size_t)p * n + c])) p = r;
    if (p != c) {
      for (int j = 0; j < n; ++j) {
        double complex t = W[(size_t)c * n + j];
        W[(size_t)c * n + j] = W[(size_t)p * n + j];
        W[(size_t)p * n + j] = t;
        t = Ainv[(size_t)c * n + j];
        Ainv[(size_t)c * n + j] = Ainv[(size_t)p * n + j];
        Ainv[(size_t)p * n + j] = t;
      }
      ph = -ph;
    }
    const double complex piv = W[(size_t)c * n + c];
    const double ap = cabs(piv);
    ld += log(ap);
    ph *= piv / ap;
    const double complex ip = 1.0 / piv;
    for (int j = 0; j < n; ++j) {
      W[(size_t)c * n + j] *= ip;
      Ainv[(size_t)c * n + j] *= ip;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double complex f = W[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        W[(size_t)r * n + j] -= f * W[(size_t)c * n + j];
        Ainv[(size_t)r * n + j] -= f * Ainv[(size_t)c * n + j];
      }
    }
  }
  if (logabsdet) *logabsdet = ld;
  if (phase) *phase = ph / cabs(ph);
  free(W);
}

/* Equal-time G = (1 + B_M ... B_1)^{-1} of complex dense slices (B_q the
 * row-major n x n complex matrix at slices + (q-1) n n, interleaved re, im),
 * log|det(1 + B_M ... B_1)| and its phase (phase[0] + i phase[1]).
 *   chain (Sec. 4.1): U = 1, D = 1, T = 1; per block of k slices (the last
 *     one shorter), W = (B_q1 ... B_q0) U multiplied out naively, W <- W D,
 *     complex UDT W = U' D' T'' (Sec. 4.2.2), U <- U', D <- D', T <- T'' T;
 *   inversion (Sec. 5.1, inv_one_plus_loh as printed): D_p = max(D, 1),
 *     D_m = min(D, 1), M = T^{-1} D_p^{-1} + U D_m, G = T^{-1} D_p^{-1} M^{-1},
 *     with T^{-1} and M^{-1} by Gauss-Jordan;
 *   determinant: 1 + U D T = M D_p T, so log|det(1 + B)| = log|det M| +
 *     sum log D_p + log|det T| and its phase is that of det M times that of
 *     det T. */
int or_greens_complex(int n, int m, int k, const double* slices, double* Gd, double* logdet, double* phase) {
  if (n <= 0 || m <= 0 || k <= 0 || !slices || !Gd) return OR_EINVAL;
  for (size_t i = 0; i < 2 * (size_t)m * n * n; ++i)
    if (!isfinite(slices[i])) return OR_ERANGE;
  const double complex* B = (const double complex*)slices;
  double complex* G = (double complex*)Gd;
  const size_t nn = (size_t)n * n;
  double complex *U = malloc(sizeof(double complex) * nn), *T = malloc(sizeof(double complex) * nn);
  double complex *W = malloc(sizeof(double complex) * nn), *tmp = malloc(sizeof(double complex) * nn);
  double complex *U2 = malloc(sizeof(double complex) * nn), *T2 = malloc(sizeof(double complex) * nn);
  double *D = malloc(sizeof(double) * n), *D2 = malloc(sizeof(double) * n);
  for (size_t e = 0; e < nn; ++e) U[e] = T[e] = 0.0;
  for (int i = 0; i < n; ++i) {
    U[(size_t)i * n + i] = T[(size_t)i * n + i] = 1.0;
    D[i] = 1.0;
  }
  for (int q0 = 1; q0 <= m; q0 += k) {
    const int q1 = q0 + k - 1 < m ? q0 + k - 1 : m;
    memcpy(W, U, sizeof(double complex) * nn);
    for (int q = q0; q <= q1; ++q) {
      cmat_mul(n, B + (size_t)(q - 1) * nn, W, tmp);
      memcpy(W, tmp, sizeof(double complex) * nn);
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) W[(size_t)i * n + j] *= D[j];
    udt_c(n, W, U2, D2, T2);
    cmat_mul(n, T2, T, tmp);
    memcpy(T, tmp, sizeof(double complex) * nn);
    memcpy(U, U2, sizeof(double complex) * nn);
    memcpy(D, D2, sizeof(double) * n);
  }
  /* inv_one_plus_loh */
  double complex *Ti = malloc(sizeof(double complex) * nn), *X = malloc(sizeof(double complex) * nn);
  double complex *M = malloc(sizeof(double complex) * nn), *Mi = malloc(sizeof(double complex) * nn);
  double ldT = 0.0, ldM = 0.0, ldp = 0.0;
  double complex phT = 1.0, phM = 1.0;
  lu_inverse_c(n, T, Ti, &ldT, &phT);
  for (int i = 0; i < n; ++i) ldp += log(D[i] > 1.0 ? D[i] : 1.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double dpj = D[j] > 1.0 ? D[j] : 1.0, dmj = D[j] < 1.0 ? D[j] : 1.0;
      X[(size_t)i * n + j] = Ti[(size_t)i * n + j] / dpj;                    /* T^{-1} D_p^{-1} */
      M[(size_t)i * n + j] = X[(size_t)i * n + j] + U[(size_t)i * n + j] * dmj; /* + U D_m */
    }
  lu_inverse_c(n, M, Mi, &ldM, &phM);
  cmat_mul(n, X, Mi, G);
  const double complex ph = phM * phT;
  if (logdet) *logdet = ldM + ldp + ldT;
  if (phase) {
    phase[0] = creal(ph);
    phase[1] = cimag(ph);
  }
  int ok = isfinite(ldM + ldp + ldT);
  for (size_t e = 0; e < nn && ok; ++e) ok = isfinite(creal(G[e])) && isfinite(cimag(G[e]));
  free(U); free(T); free(W); free(tmp); free(U2); free(T2); free(D); free(D2);
  free(Ti); free(X); free(M); free(Mi);
  return ok ? OR_OK : OR_ERANGE;
}

/* exp(-s dtau K) for the periodic L x L square lattice with K_ij = -t on
 * nearest-neighbour bonds, from the plane-wave eigenbasis (Sec. 3 gives the
 * 1-D dispersion -2t cos k; on the square lattice it is
 * eps_k = -2t (cos kx + cos ky), k = 2 pi (nx, ny) / L):
 *   E_ij = (1/N) sum_k exp(-s dtau eps_k) cos(k . (r_i - r_j)). */
int or_expk_planewave(int L, double t, double dtau, double s, double* out) {
  if (L < 1) return OR_EINVAL;
  const int n = L * L;
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    const int xi = i % L, yi = i / L;
    for (int j = 0; j < n; ++j) {
      const int dx = xi - j % L, dy = yi - j / L;
      double acc = 0.0;
      for (int ny = 0; ny < L; ++ny)
        for (int nx = 0; nx < L; ++nx) {
          const double kx = 2.0 * pi * nx / L, ky = 2.0 * pi * ny / L;
          const double eps = -2.0 * t * (cos(kx) + cos(ky));
          acc += exp(-s * dtau * eps) * cos(kx * dx + ky * dy);
        }
      out[(size_t)i * n + j] = acc / n;
    }
  }
  return OR_OK;
}
