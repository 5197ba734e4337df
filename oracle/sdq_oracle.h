/* sdq_oracle.h -- the CPU oracle's own declarations (test infrastructure;
 * shared with nothing on the GPU side).  All matrices are row-major n x n
 * FP64; slice l (1-based) uses field row l-1: B_l = expk diag(exp(alpha f)). */
#ifndef SDQ_ORACLE_H
#define SDQ_ORACLE_H

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-4)

#define OR_SCHEME_LOH 0
#define OR_SCHEME_PLAIN 1

int or_greens(int n, int m, int k, const double* expk, const double* field, double alpha,
              int scheme, double* G, double* logdet, double* sign);
int or_greens_tdisp(int n, int m, int k, const double* expk, const double* expk_inv,
                    const double* field, double alpha, int l, int scheme, double* Gt);
int or_greens_slice(int n, int m, int k, const double* expk, const double* field,
                    double alpha, int l, double* Gl, double* logdet, double* sign);
int or_logdet_grad(int n, int m, int k, const double* expk, const double* field, double alpha,
                   const int* l_list, int n_l, double* grad);
int or_greens_naive(int n, int m, int k, const double* expk, const double* field,
                    double alpha, double* G);
int or_chain(int n, int m, int k, const double* expk, const double* expk_inv,
             const double* field, double alpha, int kind, int a, int b,
             double* U, double* D, double* T);
int or_greens_sym(int n, int m, int k, const double* expk_half, const double* field, double alpha,
                  double* G, double* logdet, double* sign);
int or_greens_tdisp_sym(int n, int m, int k, const double* expk_half, const double* expk_half_inv,
                        const double* field, double alpha, int l, double* Gt);
int or_greens_stab(int n, int m, int k, const double* expk, const double* field, double alpha,
                   int scheme, int stab, double* G, double* logdet, double* sign);
int or_greens_tdisp_stab(int n, int m, int k, const double* expk, const double* expk_inv,
                         const double* field, double alpha, int l, int scheme, int stab, double* Gt);
int or_svd(int n, const double* W, double* U, double* s, double* V);
int or_greens_dense(int n, int m, int k, const double* slices, double* G, double* logdet, double* sign);
int or_greens_tdisp_dense(int n, int m, int k, const double* slices, int l, double* Gt);
int or_cpqr(int n, double* A, double* Q, int* jpvt);
int or_udt(int n, const double* W, double* U, double* D, double* T);
/* complex UDT; W, U, T interleaved (re, im) n x n, D real n */
int or_udt_complex(int n, const double* W, double* U, double* D, double* T);
/* complex dense slices [m][n][n] interleaved: G (interleaved), log|det(1+B)|, phase[2] */
int or_greens_complex(int n, int m, int k, const double* slices, double* G, double* logdet, double* phase);
int or_expk_planewave(int L, double t, double dtau, double s, double* out);

#endif
