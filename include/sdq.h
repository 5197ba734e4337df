/*
 * sdq.h -- C ABI of libsdq, stabilized determinant-QMC Green's functions on
 * AMD MI355X (gfx950).
 *
 * The method is that of C. Bauer, "Fast and stable determinant quantum Monte
 * Carlo", SciPost Phys. (2020), arXiv:2003.05286:
 *   * slice matrices B_l = expk * diag(exp(alpha * f_l)), l = 1..m
 *     (Sec. 2; the Hubbard model with Hirsch's discrete field of Sec. 3 sets
 *     alpha = sigma*lambda, f = s in {+1,-1}; a continuous field uses
 *     alpha = dtau*g, f = phi);
 *   * the chain B(beta,0) = B_m ... B_1 is multiplied naively inside blocks of
 *     k slices and folded into a UDT factorization between blocks
 *     (stabilized product, Sec. 4.1; UDT from column-pivoted QR, Sec. 4.2.2);
 *   * G = (1 + B_m ... B_1)^{-1} is inverted with the scale-separating scheme
 *     of Loh et al. (Sec. 5.1, inv_one_plus_loh), G(tau,0) with its
 *     time-displaced analogue (Sec. 6.1, inv_sum_loh), and the equal-time G at
 *     an interior slice from two stored factorizations (App. A.1).
 *
 * Conventions for every call:
 *   * all matrices are FP64, row-major (C / torch order), n x n, dense;
 *   * every data pointer inside sdq_instance and every output pointer is a
 *     DEVICE pointer on the context's device, unless marked "host";
 *   * slice l (1-based) uses field row l-1;
 *   * calls are asynchronous and stream-ordered on the context's stream;
 *     argument errors are detected synchronously and returned as a negative
 *     sdq_status with nothing enqueued; numerical conditions are written per
 *     instance into the device array `status` (0 = ok, SDQ_ERANGE = a
 *     non-finite input or result, or a scale that left the FP64 range);
 *   * the caller owns every buffer it passes; the library never frees them
 *     and does not keep them past the call, except through a checkpoint
 *     handle (sdq_logdet) which keeps the library's own copies;
 *   * no C++ exception crosses this boundary.
 * Supported sizes: 1 <= n <= 1024, 1 <= k <= m.  n <= 128 runs one
 * workgroup per chain with its matrices in registers and LDS; 128 < n <= 1024
 * runs a gang of workgroups per chain (a column slab of the matrix in each
 * one's LDS, pivot candidates and operands exchanged through HBM), with no
 * more workgroups than the device holds at once.  n > 1024 returns
 * SDQ_EUNSUPPORTED.
 * Chains of different size classes (16-wide tile counts) in one call run
 * concurrently: each class of the one-workgroup kernels on a stream of its
 * own forked from the context's stream (after the block products of
 * sdq_greens, which run first, alone, on the context's stream), the gang
 * classes on the context's stream; all of them are joined back into the
 * context's stream before the call's work ends, so callers see ordinary
 * stream order.  Every wait of a
 * gang is bounded: its members must all be running within 60 s of the
 * first one (other classes of the call may hold the CUs until they finish)
 * and every wait inside a factorization ends after 4 s; a gang that gives
 * up reports SDQ_ERANGE for its chains instead of hanging.
 */
#ifndef SDQ_H
#define SDQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SDQ_OK = 0,
  SDQ_EINVAL = -1,      /* bad argument (null pointer, size, range)            */
  SDQ_ENOMEM = -2,      /* device allocation failed                            */
  SDQ_EHIP = -3,        /* a HIP runtime call failed (message in last_error)   */
  SDQ_ERANGE = -4,      /* per instance: non-finite data or FP64 range exceeded */
  SDQ_EUNSUPPORTED = -5 /* valid but not implemented (e.g. n > 1024)           */
} sdq_status;

typedef enum {
  SDQ_INV_LOH = 0,   /* Sec. 5.1 inv_one_plus_loh / Sec. 6.1 inv_sum_loh (default):
                        the scales of D split into max(D,1) and min(D,1)         */
  SDQ_INV_PLAIN = 1  /* Sec. 5.1 inv_one_plus / Sec. 6.1 inv_sum: one intermediate
                        decomposition with D unsplit.  Accurate for the
                        equal-time G; for G(tau,0) it loses accuracy away from
                        the ends of [0, beta] (Sec. 6.2) and is provided to show
                        that, not for production use.  sdq_greens and
                        sdq_greens_tdisp only.  In sdq_greens_tdisp it
                        decomposes B(tau,0)^{-1} and B(beta,tau) anew for every
                        stage pair (O(m^2/k) slice products per chain instead of
                        O(m)), needs expk_inv, and supports n <= 128
                        (SDQ_EUNSUPPORTED above).                                 */
} sdq_scheme;

/* Decomposition that stabilizes the slice products every k slices (Sec. 4.2). */
typedef enum {
  SDQ_STAB_QR = 0,  /* column-pivoted Householder QR (default)                    */
  SDQ_STAB_SVD = 1  /* one-sided Jacobi SVD: slower, an independent cross-check;
                       n <= 80 (SDQ_EUNSUPPORTED above)                             */
} sdq_stab;

typedef struct sdq_ctx sdq_ctx;

/* One Markov chain / spin flavour.  B_l = expk * diag(exp(alpha * field[l-1][:])). */
typedef struct {
  int32_t n;              /* sites N, 1 <= n <= 1024                                 */
  int32_t m;              /* slices M = beta / dtau, m >= 1                           */
  int32_t k;              /* stabilization interval, 1 <= k <= m (Sec. 4.1)          */
  int32_t pad_;
  const double* expk;     /* [n][n] exp(-dtau K)                                      */
  const double* expk_inv; /* [n][n] exp(+dtau K) = expk^{-1}; needed by
                             sdq_logdet_grad, may be NULL for the other calls          */
  const double* field;    /* [m][n] auxiliary field f_{l,i}                           */
  double alpha;           /* coupling: sigma*lambda (Ising) or dtau*g (continuous)    */
} sdq_instance;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Returns SDQ_OK and *out, or an
 * error with *out = NULL. */
sdq_status sdq_create(sdq_ctx** out, int device, void* hip_stream);
void sdq_destroy(sdq_ctx* ctx);
/* Message describing the last failing call on ctx (static storage owned by
 * ctx; valid until the next call).  Never NULL. */
const char* sdq_last_error(const sdq_ctx* ctx);
/* Library version string, e.g. "sdq 0.1 gfx950". */
const char* sdq_version(void);

/* Equal-time Green's function (Sec. 2, G = (1 + B_m...B_1)^{-1}) of `count`
 * chains in one batched launch, with log|det(1 + B_m...B_1)| and its sign.
 *   inst    host array [count]
 *   g       host array [count] of device pointers to [n][n] outputs (an entry
 *           may be NULL: then only logdet/sign are produced for it)
 *   logdet, sign  device arrays [count] (may be NULL)
 *   status  device array [count] (may be NULL)
 * Chains of different n, m, k may be mixed in one call.  For the size class
 * (97 <= n <= 144) of the batch's longest chain, when all of that class's
 * chains are resident on the device at once, the products of each block of
 * k slices are formed first, all at once, and the chain's stabilized product
 * is taken over them (Sec. 4.1; the same product up to rounding); this uses
 * ceil(m/k) (16 ceil(n/16))^2 doubles of library memory per such chain and
 * is skipped when that memory cannot be allocated.  The environment variable
 * SDQ_BLOCK_PRODUCTS (read by sdq_create: 0 never, 1 for every class of
 * 97 <= n <= 144, 2 the default above) overrides the choice. */
sdq_status sdq_greens(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, sdq_scheme scheme,
                      double* const* g, double* logdet, double* sign, int32_t* status);

/* sdq_greens for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, but nothing is allocated; everything the kernels
 * need beyond the caller's buffers (the plan, the swizzled slice
 * exponentials, the final stage of every chain, scratch) lives in one fixed
 * device array of 64 MiB per device, reserved when the library is loaded and
 * held until the process ends.  Arguments as in sdq_greens, with these limits:
 *   * every chain has n <= 128 (SDQ_EUNSUPPORTED otherwise: larger chains
 *     need the gang scratch);
 *   * the batch must fit the 64 MiB (about (2 n^2 + n) * 8 bytes per chain,
 *     e.g. some 900 chains of n = 64): SDQ_EINVAL with the size otherwise,
 *     nothing enqueued;
 *   * all chains of the call run on the context's stream (no side streams),
 *     and nothing is timed by sdq_set_profiling.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: calls that overlap in time on one device (other streams,
 * other contexts, other host threads) race with each other and must be
 * ordered by the caller; calls on one context's stream are ordered by it.
 * Before reusing its host-side copy of the plan the call waits for the
 * previous call's upload on the same context to complete. */
sdq_status sdq_greens_noalloc(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, sdq_scheme scheme,
                              double* const* g, double* logdet, double* sign, int32_t* status);

/* A chain whose slices are given as dense real matrices (models whose B_l
 * is not expk * diag(exp(alpha f_l))): slice l (1-based) is the row-major
 * n x n device matrix slices + (l-1) n n. */
typedef struct {
  int32_t n;              /* 1 <= n <= 128                                         */
  int32_t m;              /* slices, m >= 1                                         */
  int32_t k;              /* stabilization interval, 1 <= k <= m (Sec. 4.1)        */
  int32_t pad_;
  const double* slices;   /* [m][n][n]                                              */
} sdq_dense_instance;

/* Equal-time G = (1 + B_m ... B_1)^{-1}, log|det(1 + B_m ... B_1)| and its
 * sign for chains of dense slices: the same stabilized product (Sec. 4.1,
 * pivoted-QR UDT every k slices, Sec. 4.2.2) and Loh's split inversion
 * (Sec. 5.1) as sdq_greens, with B_l read as given.  g, logdet, sign, status
 * as in sdq_greens.  n > 128 and the SVD stabilizer return SDQ_EUNSUPPORTED. */
sdq_status sdq_greens_dense(sdq_ctx* ctx, const sdq_dense_instance* inst, int32_t count, double* const* g,
                            double* logdet, double* sign, int32_t* status);

/* G(tau_l, 0) = B_l ... B_1 G for chains of dense slices, by the
 * time-displaced scheme of sdq_greens_tdisp (Sec. 6.1, inv_sum_loh) from the
 * forward stages of B_l...B_1 and the backward stages of the transposed
 * chain, at multiples of k and at l = m; any other l is reached by at most
 * k-1 further products with the dense slices from the nearest lower multiple
 * of k (Sec. 6, propagation form).  Arguments as in sdq_greens_tdisp (l_list
 * ascending, 0 <= l <= m of every chain). */
sdq_status sdq_greens_tdisp_dense(sdq_ctx* ctx, const sdq_dense_instance* inst, int32_t count,
                                  const int32_t* l_list, int32_t n_l, double* const* gt, double* const* g,
                                  double* logdet, double* sign, int32_t* status);

/* Time-displaced Green's functions G(tau_l, 0) = B_l ... B_1 G (Sec. 6) for
 * every l of the host list l_list[n_l] (ascending, each 0 <= l <= m of every
 * chain), computed directly at multiples of k by the time-displaced scheme
 * from a forward factorization of B(tau,0) and a backward factorization of
 * B(beta,tau), and for other l by at most k-1 further slice products from
 * the nearest lower multiple of k (Sec. 6, propagation form).
 *   gt  host array [count] of device pointers to [n_l][n][n] outputs
 *   g   host array [count] of device pointers to the equal-time G (entries
 *       or the whole array may be NULL)
 *   logdet, sign, status  as in sdq_greens (may be NULL) */
sdq_status sdq_greens_tdisp(sdq_ctx* ctx, const sdq_instance* inst, int32_t count,
                            sdq_scheme scheme, const int32_t* l_list, int32_t n_l,
                            double* const* gt, double* const* g, double* logdet, double* sign,
                            int32_t* status);

/* log|det(1 + B_m...B_1)| and sign for `count` chains; if ckpt_handle is not
 * NULL the forward factorizations are kept in library memory and *ckpt_handle
 * identifies them for a later sdq_logdet_grad on the same instances
 * (released by sdq_release or sdq_destroy). */
sdq_status sdq_logdet(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, double* logdet,
                      double* sign, int32_t* status, uint64_t* ckpt_handle);

/* Gradient of log|det(1 + B_m...B_1)| with respect to every field entry:
 *   grad[l-1][i] = d log|det| / d f_{l,i} = alpha * (1 - G_l)_{ii},
 * with G_l the equal-time G at slice l (Sec. 6), obtained at every multiple
 * of k from a forward and a backward factorization combined as in App. A.1
 * and carried to the next k-1 slices by G_{l+1} = B_l G_l B_l^{-1}.
 *   ckpt_handle  0, or a handle from sdq_logdet on the same instances (then
 *                the forward sweep is not repeated)
 *   grad   host array [count] of device pointers to [m][n] outputs
 *   logdet, sign, status  may be NULL
 * Requires expk_inv in every instance. */
sdq_status sdq_logdet_grad(sdq_ctx* ctx, uint64_t ckpt_handle, const sdq_instance* inst,
                           int32_t count, double* const* grad, double* logdet, double* sign,
                           int32_t* status);

sdq_status sdq_release(sdq_ctx* ctx, uint64_t ckpt_handle);

/* UDT factorization W P = Q R, U = Q, D = |diag R|, T = D^{-1} R P^T
 * (Sec. 4.2.2) of `count` n x n matrices stored back to back in w
 * ([count][n][n], device); outputs u, t [count][n][n] and d [count][n].
 * 1 <= n <= 1024. */
sdq_status sdq_udt(sdq_ctx* ctx, int32_t n, int32_t count, const double* w, double* u,
                   double* d, double* t);

/* Complex UDT (Sec. 4.2.2 over the complex numbers, for complex slices such
 * as those of App. B): W P = Q R by column-pivoted Householder QR with real
 * diag R, U = Q (unitary), D = |diag R|, T = D^{-1} R P^T (a row with
 * D_i = 0 is left undivided), for `count` complex n x n matrices stored back
 * to back in w.  w, u, t: [count][n][n] complex, each entry two doubles
 * (re, im), row-major, device; d: [count][n] real, device.  The caller owns
 * all buffers; the call is ordered on the context's stream.  1 <= n <= 64
 * (SDQ_EUNSUPPORTED above); SDQ_EINVAL for a NULL buffer or count < 0. */
sdq_status sdq_udt_complex(sdq_ctx* ctx, int32_t n, int32_t count, const double* w, double* u,
                           double* d, double* t);

/* A chain of complex slices (e.g. the spin-fermion model of App. B, whose
 * slices are complex matrices): slice l (1-based) is the row-major n x n
 * complex device matrix at slices + 2 (l-1) n n, entries as (re, im) pairs. */
typedef struct {
  int32_t n;              /* 1 <= n <= 64                                           */
  int32_t m;              /* slices, m >= 1                                          */
  int32_t k;              /* stabilization interval, 1 <= k <= m (Sec. 4.1)         */
  int32_t pad_;
  const double* slices;   /* [m][n][n] complex                                       */
} sdq_complex_instance;

/* Equal-time G = (1 + B_m ... B_1)^{-1} of chains of complex slices, with
 * log|det(1 + B_m ... B_1)| and the phase det / |det| (App. B; for complex
 * slices the determinant is complex, not just signed):  the stabilized
 * product of Sec. 4.1 with the complex pivoted-QR UDT (Sec. 4.2.2,
 * sdq_udt_complex's decomposition) every k slices, and Loh's split inversion
 * (Sec. 5.1).  One workgroup per chain, matrices resident in LDS.
 *   g       host array [count] of device pointers to [n][n] complex outputs
 *           (entries may be NULL)
 *   logdet  device [count] or NULL
 *   phase   device [count][2] (re, im) or NULL
 *   status  device [count] or NULL (SDQ_ERANGE: non-finite data or result)
 * n > 64 returns SDQ_EUNSUPPORTED; chains of different n, m, k may be mixed. */
sdq_status sdq_greens_complex(sdq_ctx* ctx, const sdq_complex_instance* inst, int32_t count, double* const* g,
                              double* logdet, double* phase, int32_t* status);

/* Stabilized chain of one instance set (Sec. 4.1): the UDT factors of
 * B_m...B_1 for each chain, u, t [count][n][n], d [count][n] (device).
 * All chains must share n. */
sdq_status sdq_chain_udt(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, double* u,
                         double* d, double* t);

/* One sweep of local updates over the field of `count` chains of `nf`
 * flavours each (nf = 1 or 2; the flavours of a chain are consecutive in
 * inst and share its field, n, m and k; e.g. spin up and down of the Hubbard
 * model with alpha = +lambda, -lambda).  Sites are visited slice by slice,
 * l = 1..m, and within a slice i = 0..n-1; flipping f_{l,i} -> -f_{l,i}
 * changes det(1 + B_m...B_1) of flavour f by the ratio
 * R_f = 1 + (exp(-2 alpha_f f_{l,i}) - 1) (1 - G_l)_{ii} (Sec. 2: local updates
 * need only this ratio), and the flip is accepted when
 * u[c][l-1][i] < |prod_f R_f|.  G_l is kept current by rank-one updates after
 * every accepted flip and G_{l+1} = B_l G_l B_l^{-1} between slices, and is
 * recomputed from stabilized factorizations (the forward one rebuilt from the
 * updated field, Sec. 4.1 / App. A.1) at the start of every block of k
 * slices.
 *   unif      device [count][m][n] uniform numbers in [0, 1)
 *   accepted  device [count]: number of accepted flips of each chain
 *   status    device [count * nf] or NULL
 * The field arrays are updated in place.  Requires expk_inv; n <= 128. */
sdq_status sdq_local_sweep(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, int32_t nf,
                           const double* unif, int32_t* accepted, int32_t* status);

/* One Metropolis step with global proposals for `count` chains of `nf`
 * flavours each (Sec. 2: the weight of a field configuration is
 * exp(-S_B) prod_f |det(1 + B_f)|, and the step accepts with probability
 * min(1, exp(-dS) prod_f |det(1 + B'_f)| / |det(1 + B_f)|)).
 *   cur, prop  host arrays [count * nf]; flavour f of chain c at c * nf + f.
 *              cur[i].field is the current field (device, m x n, overwritten
 *              by prop[i].field when the chain accepts; flavours may share a
 *              field, which is then copied once); prop[i] is the proposal
 *              (same n and m, its own field array).  Only prop is evaluated.
 *   dS      device [count]: S_B(proposed) - S_B(current) (0 for the
 *           discrete Hirsch field of Sec. 3, whose bosonic weight is constant)
 *   u       device [count]: uniform numbers in (0, 1); the step accepts when
 *           log u < -dS + sum_f (log|det(1+B'_f)| - log|det(1+B_f)|)
 *   logdet, sign  device [count * nf]: log|det(1 + B_f)| and its sign for the
 *           current fields on entry (e.g. from sdq_logdet); replaced by the
 *           proposal's where the chain accepts
 *   accept  device [count]: 1 accepted, 0 rejected
 *   status  device [count * nf] or NULL: status of each proposal's
 *           evaluation; a chain with a nonzero one rejects
 * The sign is not part of the acceptance (|weight| is sampled; the sign is
 * returned for reweighting). */
sdq_status sdq_metropolis(sdq_ctx* ctx, const sdq_instance* cur, const sdq_instance* prop,
                          int32_t count, int32_t nf, const double* dS, const double* u, double* logdet,
                          double* sign, int32_t* accept, int32_t* status);

/* One Langevin step (Euler-Maruyama) of a continuous field, driven by the
 * gradient of sdq_logdet_grad.  The field's weight is exp(-S) with
 *   S = inv_var/2 sum_{l,i} phi_{l,i}^2 - sum_f log|det(1 + B_f)|
 * (Sec. 2: a Gaussian bosonic weight times the flavours' determinants, whose
 * absolute value is sampled), and the step is
 *   F   = dS/dphi = inv_var phi - sum_f grad_f     (grad_f as in sdq_logdet_grad)
 *   phi <- phi - eps F + sqrt(2 eps) noise.
 *   inst     host array [count * nf]; flavour f of chain c at c * nf + f, all
 *            flavours of a chain on the same field array (device, m x n,
 *            updated in place) with the same n and m; needs expk_inv
 *   eps      step size, > 0; inv_var >= 0 (0: no bosonic term)
 *   noise    device: the chains' [m][n] blocks of standard normal numbers,
 *            back to back in chain order
 *   force    device, same layout as noise, receives F; or NULL
 *   logdet, sign  device [count * nf] or NULL: of the field before the step
 *   status   device [count * nf] or NULL; a chain with a nonzero status of
 *            any flavour keeps its field
 * The gradients go through library memory (m * n doubles per instance). */
sdq_status sdq_langevin(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, int32_t nf, double eps,
                        double inv_var, const double* noise, double* force, double* logdet, double* sign,
                        int32_t* status);

/* One hybrid Monte Carlo trajectory of a continuous field per chain, on the
 * same weight exp(-S) as sdq_langevin (S = inv_var/2 sum phi^2 -
 * sum_f log|det(1 + B_f)|, Sec. 2), with momenta p and
 * H = S + 1/2 sum p^2: leapfrog steps
 *   p -= eps/2 F(phi); then nsteps times { phi += eps p; p -= eps F(phi) }
 *   with the last kick halved,   F = dS/dphi (the adjoint gradient),
 * then acceptance when log u < H(start) - H(end); a rejected chain gets its
 * start field back.  nsteps + 1 gradient evaluations per trajectory.
 *   inst     host array [count * nf]; flavour f of chain c at c * nf + f, all
 *            flavours of a chain on the same field array (device, m x n,
 *            updated in place) with the same n and m; needs expk_inv
 *   eps > 0, nsteps >= 1, inv_var >= 0
 *   mom      device: the chains' initial momenta, [m][n] blocks of standard
 *            normal numbers back to back in chain order
 *   u        device [count]: uniform numbers in (0, 1)
 *   logdet, sign  device [count * nf] or NULL: of each chain's field after
 *            the step (the end field if accepted, else the start field)
 *   accept   device [count]: 1 accepted, 0 rejected
 *   dH       device [count] or NULL: H(end) - H(start)
 *   status   device [count * nf] or NULL: the first nonzero status of the
 *            trajectory's evaluations; a chain with one rejects
 * Scratch (gradients, start fields, momenta) is library memory. */
sdq_status sdq_hmc(sdq_ctx* ctx, const sdq_instance* inst, int32_t count, int32_t nf, double eps,
                   int32_t nsteps, double inv_var, const double* mom, const double* u, double* logdet,
                   double* sign, int32_t* accept, double* dH, int32_t* status);

/* Choose the stabilizer of every later sweep of ctx (sdq_stab, Sec. 4.2):
 * the pivoted QR (default) or the one-sided Jacobi SVD, whose UDT is
 * U = A diag(1/sigma), D = sigma, T = V^T T_previous (A = W V with
 * orthogonal columns, sigma their norms; at most 60 Jacobi sweeps per
 * decomposition, SDQ_ERANGE in status without convergence).  Every result
 * (G, G(tau,0), log|det|, sign, gradient) is the same up to rounding; the
 * SVD takes several times as long.  Returns SDQ_EINVAL for another value. */
sdq_status sdq_set_stabilizer(sdq_ctx* ctx, int32_t stab);

/* M <- left * M * right for `count` n x n row-major device matrices: mats is
 * a host array [count] of device pointers (updated in place; the entries
 * must not overlap), left and right are device n x n matrices shared by the
 * batch.  1 <= n <= 128 (SDQ_EUNSUPPORTED above).
 * Use: the paper's slice is the symmetric Trotter form
 * B_l = E^{1/2} diag(exp(alpha f_l)) E^{1/2} (Sec. 2, E^{1/2} = exp(-dtau K/2));
 * its chain is E^{-1/2} (B'_M ... B'_1) E^{1/2} with the slices
 * B'_l = E diag(exp(alpha f_l)) every other call uses (expk = E).  So log|det|,
 * its sign and the field gradient are the same for both forms, and the
 * symmetric form's G and G(tau,0) are E^{-1/2} X E^{1/2} of the results X of
 * sdq_greens / sdq_greens_tdisp: call this with left = E^{-1/2},
 * right = E^{1/2} on them. */
sdq_status sdq_similarity(sdq_ctx* ctx, int32_t n, int32_t count, const double* left,
                          const double* right, double* const* mats);

/* Time every kernel variant for each n of n_list[count] (host) on the
 * device, keep the fastest per n in ctx, and if cache_path is not NULL
 * append the choices to that JSON-lines file (read back by later contexts
 * through the same call; an existing entry for (arch, n) is used without
 * re-timing).  Sizes n > 128 have a single kernel and are accepted but not
 * timed. */
sdq_status sdq_tune(sdq_ctx* ctx, const int32_t* n_list, int32_t count, const char* cache_path);

/* Capture later batched calls in HIP graphs and replay them when the same
 * batch (every pointer, shape, list and scheme) is seen again (enable = 1),
 * or launch directly (enable = 0, the default).  A replay runs on the
 * context's stream; at most 16 graphs are kept (oldest evicted).  Mixed-size
 * batches and chains of n > 128 are captured like any other. */
sdq_status sdq_set_graphs(sdq_ctx* ctx, int enable);

/* Record HIP events around every kernel launch (enable = 1), on the stream
 * the launch runs on; the per-kernel launch count and summed device
 * milliseconds are then read with sdq_kernel_stats.  Names: "sweep" for the
 * stabilized sweeps, "equal" for the equal-time inversions, "pair" for the
 * time-displaced inversions, "grad" for the gradient, "local" and "bstart"
 * for local updates, "udt", "udt_complex", and "graph" for a replayed graph.
 * The batched kernels are also kept per size class as "<name>/nt<T>" (T =
 * ceil(n/16), above 8 a gang class): sdq_kernel_stats("sweep") sums all
 * classes, sdq_kernel_stats("sweep/nt7") reads one; sdq_kernel_names lists
 * every name recorded.  Launches of different classes may overlap in time,
 * so a sum over classes is device time, not wall time.  Resets the
 * counters. */
sdq_status sdq_set_profiling(sdq_ctx* ctx, int enable);
sdq_status sdq_kernel_stats(sdq_ctx* ctx, const char* name, int64_t* launches, double* ms);
/* The names recorded since profiling was enabled, comma separated, into the
 * host buffer buf of cap bytes (NUL terminated); SDQ_EINVAL if it is too
 * small. */
sdq_status sdq_kernel_names(sdq_ctx* ctx, char* buf, int32_t cap);

/* Wait for all work enqueued by ctx and report an asynchronous HIP error. */
sdq_status sdq_sync(sdq_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SDQ_H */
