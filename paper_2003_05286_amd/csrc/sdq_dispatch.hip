// sdq_dispatch.hip -- selects the per-tile-count kernel instantiation, and
// the small queue-reset kernel.
#include "sdq_internal.h"

namespace sdq {

#define SDQ_DECL(N)                                                                              \
  hipError_t launch_sweep_nt##N(int, const Inst*, const SweepItem*, int, Queue*, int, double*, hipStream_t); \
  hipError_t launch_pair_nt##N(int, const Inst*, const PairItem*, int, const int32_t*, Queue*, int, \
                               hipStream_t);                                                     \
  hipError_t launch_udt_nt##N(int, int, const double*, double*, double*, double*, hipStream_t);  \
  hipError_t launch_sim_nt##N(int, int, double* const*, const double*, const double*, int, hipStream_t); \
  hipError_t kernel_info_nt##N(int, int, KernelInfo*);                                            \
  hipError_t launch_dense_sweep_nt##N(const Inst*, const SweepItem*, int, Queue*, int, hipStream_t); \
  hipError_t launch_bprod_sweep_nt##N(const Inst*, const SweepItem*, int, Queue*, int, double*, hipStream_t); \
  hipError_t bprod_sweep_info_nt##N(KernelInfo*);                                                \
  hipError_t dense_info_nt##N(KernelInfo*);                                                      \
  hipError_t launch_prod_nt##N(const Inst*, const SweepItem*, int, Queue*, int, hipStream_t);    \
  hipError_t prod_info_nt##N(KernelInfo*);                                                       \
  hipError_t launch_dense_pair_nt##N(const Inst*, const PairItem*, int, const int32_t*, Queue*, int, \
                                     hipStream_t);                                               \
  hipError_t dense_pair_info_nt##N(KernelInfo*);
SDQ_DECL(1) SDQ_DECL(2) SDQ_DECL(3) SDQ_DECL(4) SDQ_DECL(5) SDQ_DECL(6) SDQ_DECL(7) SDQ_DECL(8)
#undef SDQ_DECL
// 128 < n <= 144: the one-workgroup sweep only (sdq_nt9.hip)
hipError_t launch_sweep_nt9(int, const Inst*, const SweepItem*, int, Queue*, int, double*, hipStream_t);
hipError_t kernel_info_nt9(int, int, KernelInfo*);
hipError_t launch_prod_nt9(const Inst*, const SweepItem*, int, Queue*, int, hipStream_t);

#define SDQ_SWITCH(CALL)                                   \
  switch (nt) {                                            \
    case 1: return CALL(1);                                \
    case 2: return CALL(2);                                \
    case 3: return CALL(3);                                \
    case 4: return CALL(4);                                \
    case 5: return CALL(5);                                \
    case 6: return CALL(6);                                \
    case 7: return CALL(7);                                \
    case 8: return CALL(8);                                \
    default: return hipErrorInvalidValue;                  \
  }

hipError_t launch_sweep(int nt, int variant, const Inst* inst, const SweepItem* items, int count,
                        Queue* q, int grid, double* tscr, hipStream_t s) {
  if (nt == kSweepMaxNT) return launch_sweep_nt9(variant, inst, items, count, q, grid, tscr, s);
  if (variant == 3) {
#define C(N) launch_dense_sweep_nt##N(inst, items, count, q, grid, s)
    SDQ_SWITCH(C)
#undef C
  }
  if (variant == 6) {
#define C(N) launch_bprod_sweep_nt##N(inst, items, count, q, grid, tscr, s)
    SDQ_SWITCH(C)
#undef C
  }
#define C(N) launch_sweep_nt##N(variant, inst, items, count, q, grid, tscr, s)
  SDQ_SWITCH(C)
#undef C
}

hipError_t launch_prod(int nt, const Inst* inst, const SweepItem* items, int count, Queue* q, int grid,
                       hipStream_t s) {
  if (nt == kSweepMaxNT) return launch_prod_nt9(inst, items, count, q, grid, s);
#define C(N) launch_prod_nt##N(inst, items, count, q, grid, s)
  SDQ_SWITCH(C)
#undef C
}

hipError_t launch_pair(int nt, int variant, int mode, const Inst* inst, const PairItem* items,
                       int count, const int32_t* l_list, Queue* q, int grid, hipStream_t s) {
  (void)variant;
  if (mode == PAIR_TDISP_DENSE) {
#define C(N) launch_dense_pair_nt##N(inst, items, count, l_list, q, grid, s)
    SDQ_SWITCH(C)
#undef C
  }
#define C(N) launch_pair_nt##N(mode, inst, items, count, l_list, q, grid, s)
  SDQ_SWITCH(C)
#undef C
}

hipError_t launch_udt(int nt, int n, int count, const double* w, double* u, double* d, double* t,
                      hipStream_t s) {
#define C(N) launch_udt_nt##N(n, count, w, u, d, t, s)
  SDQ_SWITCH(C)
#undef C
}

hipError_t launch_similarity(int nt, int n, int count, double* const* mats, const double* left,
                             const double* right, int grid, hipStream_t s) {
#define C(N) launch_sim_nt##N(n, count, mats, left, right, grid, s)
  SDQ_SWITCH(C)
#undef C
}
hipError_t kernel_info(int kind, int nt, int variant, KernelInfo* out) {
  if (nt == kSweepMaxNT) return kernel_info_nt9(kind, variant, out);
  if (kind == KK_PROD) {
#define C(N) prod_info_nt##N(out)
    SDQ_SWITCH(C)
#undef C
  }
  if (kind == KK_SWEEP && variant == 6) {
#define C(N) bprod_sweep_info_nt##N(out)
    SDQ_SWITCH(C)
#undef C
  }
  if (kind == KK_SWEEP && variant == 3) {
#define C(N) dense_info_nt##N(out)
    SDQ_SWITCH(C)
#undef C
  }
  if (kind == KK_PAIR && variant == 3) {
#define C(N) dense_pair_info_nt##N(out)
    SDQ_SWITCH(C)
#undef C
  }
#define C(N) kernel_info_nt##N(kind, variant, out)
  SDQ_SWITCH(C)
#undef C
}

__global__ void k_reset(Queue* q, int nq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nq) q[i].next = 0;
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void k_swizzle(const double* e, int n, int nt, int trans, double* out) {
  const int np = 16 * nt;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= np * np) return;
  const int l = idx & 63, b = idx >> 6;
  const int r = b & 3, tk = (b >> 2) % nt, ti = (b >> 2) / nt;
  const int i = 16 * ti + (l & 15), k = 16 * tk + (l >> 4) + 4 * r;
  double x = 0.0;
  if (i < n && k < n) x = trans ? e[(size_t)k * n + i] : e[(size_t)i * n + k];
  out[idx] = x;
}

hipError_t launch_swizzle(const double* e, int n, int trans, double* out, hipStream_t s) {
  const int nt = (n + 15) / 16, np = 16 * nt;
  hipLaunchKernelGGL(k_swizzle, dim3((np * np + 255) / 256), dim3(256), 0, s, e, n, nt, trans, out);
  return hipGetLastError();
}

// Metropolis acceptance of a global proposal (Sec. 2): the weight of a field
// is exp(-S_B) prod_f |det(1 + B_f)|, so the step accepts when
//   log u < -dS + sum_f (log|det(1+B'_f)| - log|det(1+B_f)|),
// with u uniform in (0, 1); a proposal whose evaluation failed (nonzero
// status) is rejected.  On acceptance the proposed fields are copied over the
// current ones (a field shared by several flavours of the chain is copied
// once) and the chain's log|det| and signs replaced.
__global__ void k_metropolis(int count, int nf, const MetroField* __restrict__ fields,
                             const double* __restrict__ ld_prop, const double* __restrict__ sg_prop,
                             const int32_t* __restrict__ st_prop, const double* __restrict__ dS,
                             const double* __restrict__ u, double* logdet, double* sign,
                             int32_t* accept) {
  __shared__ int acc;
  const int c = blockIdx.x;
  if (c >= count) return;
  if (threadIdx.x == 0) {
    double delta = -dS[c];
    bool ok = true;
    for (int f = 0; f < nf; ++f) {
      const int i = c * nf + f;
      delta += ld_prop[i] - logdet[i];
      ok = ok && st_prop[i] == 0 && isfinite(ld_prop[i]);
    }
    acc = (ok && log(u[c]) < delta) ? 1 : 0;
    accept[c] = acc;
  }
  __syncthreads();
  if (!acc) return;
  for (int f = 0; f < nf; ++f) {
    const MetroField F = fields[c * nf + f];
    bool seen = false;
    for (int g = 0; g < f; ++g) seen = seen || fields[c * nf + g].cur == F.cur;
    if (seen) continue;
    for (int64_t t = threadIdx.x; t < F.len; t += blockDim.x) F.cur[t] = F.prop[t];
  }
  if (threadIdx.x < nf) {
    const int i = c * nf + threadIdx.x;
    logdet[i] = ld_prop[i];
    sign[i] = sg_prop[i];
  }
}
hipError_t launch_metropolis(int count, int nf, const MetroField* fields, const double* ld_prop,
                             const double* sg_prop, const int32_t* st_prop, const double* dS,
                             const double* u, double* logdet, double* sign, int32_t* accept,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_metropolis, dim3(count), dim3(256), 0, s, count, nf, fields, ld_prop, sg_prop,
                     st_prop, dS, u, logdet, sign, accept);
  return hipGetLastError();
}
// Euler-Maruyama step of Langevin dynamics for the field: blockIdx.y is the
// chain, the x blocks stride over its m * n entries.  The force reads the
// field before this thread overwrites the same entry, and no other thread
// touches that entry.
__global__ void k_langevin(int nf, const LangevinChain* __restrict__ chains, double eps, double inv_var) {
  const LangevinChain C = chains[blockIdx.y];
  for (int g = 0; g < nf; ++g)
    if (C.status[g] != 0) return;
  const double amp = sqrt(2.0 * eps);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < C.len;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double phi = C.phi[t];
    double f = inv_var * phi;
    for (int g = 0; g < nf; ++g) f -= C.grad[(int64_t)g * C.len + t];
    C.phi[t] = phi - eps * f + amp * C.noise[t];
    if (C.force) C.force[t] = f;
  }
}
hipError_t launch_langevin(int count, int nf, const LangevinChain* chains, double eps, double inv_var,
                           int grid_per_chain, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_langevin, dim3(grid_per_chain, count), dim3(256), 0, s, nf, chains, eps, inv_var);
  return hipGetLastError();
}
// sum over the workgroup of one double per thread (256 threads), in a fixed
// order; every thread gets the total
__device__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void k_hmc_begin(const HmcChain* __restrict__ chains, double inv_var,
                                                    double* e0) {
  __shared__ double red[256];
  const HmcChain C = chains[blockIdx.x];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < C.len; t += 256) {
    const double phi = C.phi[t], p = C.mom[t];
    C.phi0[t] = phi;
    C.p[t] = p;
    acc += 0.5 * inv_var * phi * phi + 0.5 * p * p;
  }
  const double e = block_sum256(acc, red);
  if (threadIdx.x == 0) e0[blockIdx.x] = e;
}
hipError_t launch_hmc_begin(int count, const HmcChain* chains, double inv_var, double* e0, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hmc_begin, dim3(count), dim3(256), 0, s, chains, inv_var, e0);
  return hipGetLastError();
}

// each thread owns its entries: the force reads phi before the drift writes it
__global__ void k_hmc_step(int nf, const HmcChain* __restrict__ chains, double kick, double eps,
                           double inv_var) {
  const HmcChain C = chains[blockIdx.y];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < C.len;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double phi = C.phi[t];
    double f = inv_var * phi;
    for (int g = 0; g < nf; ++g) f -= C.grad[(int64_t)g * C.len + t];
    const double p = C.p[t] - kick * f;
    C.p[t] = p;
    C.phi[t] = phi + eps * p;
  }
}
hipError_t launch_hmc_step(int count, int nf, const HmcChain* chains, double kick, double eps, double inv_var,
                           int grid_per_chain, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hmc_step, dim3(grid_per_chain, count), dim3(256), 0, s, nf, chains, kick, eps, inv_var);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_hmc_end(int nf, int total, const HmcChain* __restrict__ chains,
                                                  double half_kick, double inv_var, HmcEnd a) {
  __shared__ double red[256];
  __shared__ int acc_s;
  const int c = blockIdx.x;
  const HmcChain C = chains[c];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < C.len; t += 256) {
    const double phi = C.phi[t];
    double f = inv_var * phi;
    for (int g = 0; g < nf; ++g) f -= C.grad[(int64_t)g * C.len + t];
    const double p = C.p[t] - half_kick * f;
    acc += 0.5 * inv_var * phi * phi + 0.5 * p * p;
  }
  const double e1 = block_sum256(acc, red);
  if (threadIdx.x == 0) {
    double h0 = a.e0[c], h1 = e1;
    bool ok = true;
    for (int g = 0; g < nf; ++g) {
      const int i = c * nf + g;
      h0 -= a.ld0[i];
      h1 -= a.ld1[i];
      int32_t st = 0;
      for (int e = 0; e < a.n_eval; ++e) st = st ? st : a.st_all[(int64_t)e * total + i];
      ok = ok && st == 0;
      if (a.status) a.status[i] = st;
    }
    ok = ok && isfinite(h1);
    const int take = (ok && log(a.u[c]) < h0 - h1) ? 1 : 0;
    acc_s = take;
    a.accept[c] = take;
    if (a.dH) a.dH[c] = h1 - h0;
    for (int g = 0; g < nf; ++g) {
      const int i = c * nf + g;
      if (a.logdet) a.logdet[i] = take ? a.ld1[i] : a.ld0[i];
      if (a.sign) a.sign[i] = take ? a.sg1[i] : a.sg0[i];
    }
  }
  __syncthreads();
  if (acc_s) return;
  for (int64_t t = threadIdx.x; t < C.len; t += 256) C.phi[t] = C.phi0[t];
}
hipError_t launch_hmc_end(int count, int nf, const HmcChain* chains, double half_kick, double inv_var,
                          const HmcEnd& a, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hmc_end, dim3(count), dim3(256), 0, s, nf, count * nf, chains, half_kick, inv_var, a);
  return hipGetLastError();
}

hipError_t launch_reset(Queue* q, int nq, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reset, dim3((nq + 63) / 64), dim3(64), 0, s, q, nq);
  return hipGetLastError();
}

}  // namespace sdq
