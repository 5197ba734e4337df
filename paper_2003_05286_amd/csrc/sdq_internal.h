// sdq_internal.h -- structures shared by the host runtime and the gfx950
// kernels of libsdq (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdq {

// Largest number of 16-wide tiles per matrix dimension handled by the
// LDS-resident kernels: n <= 16 * kMaxNT = 128.
constexpr int kMaxNT = 8;
// The stabilized sweep also runs as one workgroup for n <= 16 * kSweepMaxNT
// = 144 (factor store in device memory); all other kernels of that size and
// every kernel above it are gang kernels.
constexpr int kSweepMaxNT = 9;

// One stored UDT factorization ("stage") of a chain, kept in HBM:
//   U [n*n] | T [n*n] | D [n] | extra [kStageExtra]
// extra[0] = sign of det U.
constexpr int kStageExtra = 8;
__host__ __device__ inline int64_t stage_doubles(int n) {
  return 2LL * n * n + n + kStageExtra;
}

// One chain as seen by the kernels.
struct Inst {
  const double* expk;      // [n][n]
  const double* expk_inv;  // [n][n] or null
  const double* field;     // [m][n]; dense-slice chains: the slices [m][n][n]
  double alpha;
  int32_t n, m, k, nb;     // nb = ceil(m / k) stabilization blocks
  int32_t scheme;          // 0: Loh's split scales (Sec. 5.1, 6.1), 1: single decomposition
  int32_t pad0;
  double* g;               // equal-time G [n][n] or null (local updates: G at the block start)
  double* gt;              // time-displaced outputs [n_l][n][n] or null
  double* grad;            // [m][n] or null
  double* logdet;          // scalar or null
  double* sign;            // scalar or null
  int32_t* status;         // scalar or null
  double* ckf;             // forward stages F[1..nb] (nb * stage_doubles) or null
  double* cka;             // backward stages A[0..nb-1] or null
  double* u_out;           // final U / D / T of the sweep, or null
  double* d_out;
  double* t_out;
  const double* esw;       // expk, zero padded to 16*ceil(n/16) and swizzled
  const double* eswt;      // expk^T, same layout (see launch_swizzle)
  double* fin;             // final forward stage (read by the equal-time inversion)
  const double* eswi;      // expk_inv in the layout of esw, or null
  const double* unif;      // local updates: uniform numbers [m][n] of the chain
  int32_t* nacc;           // local updates: accepted flips of the chain
  double* prod;            // block products [nb][16 nt][16 nt], swizzled (k_prod output), or null
};

enum SweepFlags : int32_t {
  SW_ADJ = 1,     // backward sweep over B_l^T from l = m down to 1
  SW_STORE = 2,   // store every stage (ckf for forward, cka for backward)
  SW_LAST = 4,    // store the last stage at fin (implied by SW_STORE forward)
  SW_FINAL = 8,   // write the final U, D, T to u_out / d_out / t_out
  // chains of one stage pair j of the single-decomposition G(tau_j, 0), each
  // started at tau_j = min(jk, m) and stabilized every k slices from there:
  SW_LEFT = 16,   // B_1^{-1} ... B_{tau_j}^{-1}, stored at ckf[j-1]   (j >= 1)
  SW_RIGHT = 32,  // B_m ... B_{tau_j+1},         stored at cka[j]     (j < nb)
  // block j of the forward chain from forward stage j (ckf[j-1], identity
  // for j = 0), stored at ckf[j]: rebuilds the stages as a local-update
  // sweep changes the field
  SW_BLOCK = 64,
};

struct SweepItem {
  int32_t inst;
  int32_t flags;
  int32_t j;  // stage pair of SW_LEFT / SW_RIGHT
  int32_t pad;
};

enum PairMode : int32_t { PAIR_TDISP = 0, PAIR_GRAD = 1, PAIR_EQUAL = 2, PAIR_TDISP_PLAIN = 3,
                          PAIR_LOCAL = 4, PAIR_BSTART = 5, PAIR_TDISP_DENSE = 6 };
constexpr int kPairModes = 7;

// tdisp: stage pair j, outputs for l_list[ilo..ihi) (PAIR_TDISP_PLAIN: the
//        same from the SW_LEFT / SW_RIGHT chains)
// grad:  stage pair j (slices j*k+1 .. min((j+1)k, m))
// local: block j of a local-update sweep; inst = the chain's first flavour,
//        ilo = number of flavours (1 or 2, consecutive instances)
// bstart: G at the start of block j of a local-update sweep -> Inst::g
// equal: the final forward stage -> G, logdet, sign
struct PairItem {
  int32_t inst;
  int32_t j;
  int32_t ilo;
  int32_t ihi;
};

struct Queue {
  int32_t next;
  int32_t pad[31];
};

// status bits accumulated per instance (any nonzero => SDQ_ERANGE)
// value OR-ed into an instance status word on a numerical failure (== SDQ_ERANGE)
constexpr int32_t kStatusRange = -4;

// ---- launchers (sdq_kernels.hip) -----------------------------------------
struct KernelInfo {
  int threads;
  int lds_bytes;
  int blocks_per_cu;  // occupancy reported by the runtime
};

hipError_t kernel_info(int kind, int nt, int variant, KernelInfo* out);
hipError_t launch_reset(Queue* q, int nq, hipStream_t s);
// One flavour of a chain in a Metropolis step: its current field (updated on
// acceptance) and the proposed one, m * n doubles each.
struct MetroField {
  double* cur;
  const double* prop;
  int64_t len;
};
// Global-update Metropolis decisions for `count` chains of nf flavours each
// (see sdq_metropolis); one workgroup per chain.
hipError_t launch_metropolis(int count, int nf, const MetroField* fields, const double* ld_prop,
                             const double* sg_prop, const int32_t* st_prop, const double* dS,
                             const double* u, double* logdet, double* sign, int32_t* accept,
                             hipStream_t s);
// One chain of a Langevin step: its field (updated in place), the gradients
// of its nf flavours (consecutive, len doubles apart), its noise block and
// the force output (or null), len = m * n doubles each.
struct LangevinChain {
  double* phi;
  const double* grad;
  const double* noise;
  double* force;
  const int32_t* status;  // the flavours' statuses (nf consecutive)
  int64_t len;
};
// phi <- phi - eps F + sqrt(2 eps) noise, F = inv_var phi - sum_f grad_f
// (see sdq_langevin), for chains whose flavours all have status 0 (the
// others keep their field); grid-stride over the chains' entries.
hipError_t launch_langevin(int count, int nf, const LangevinChain* chains, double eps, double inv_var,
                           int grid_per_chain, hipStream_t s);
// One chain of a hybrid Monte Carlo trajectory: its field (in place), the
// saved start field, the momenta (scratch) and the initial momenta (input),
// the gradients of its nf flavours (consecutive, len apart), len = m * n.
struct HmcChain {
  double* phi;
  double* phi0;
  double* p;
  const double* mom;
  const double* grad;
  int64_t len;
};
// Start of a trajectory: phi0 = phi, p = mom, e0[c] = inv_var/2 |phi|^2 +
// 1/2 |p|^2; one workgroup per chain (fixed reduction order).
hipError_t launch_hmc_begin(int count, const HmcChain* chains, double inv_var, double* e0, hipStream_t s);
// Kick and drift: p -= kick F(phi), phi += eps p, F = inv_var phi - sum_f grad_f.
hipError_t launch_hmc_step(int count, int nf, const HmcChain* chains, double kick, double eps, double inv_var,
                           int grid_per_chain, hipStream_t s);
// End of a trajectory: the last half kick, e1 = inv_var/2 |phi|^2 + 1/2 |p|^2,
// H = e - sum_f log|det|, the Metropolis test on exp(-(H1 - H0)) (status of
// every evaluation zero), outputs, and phi <- phi0 on rejection.
struct HmcEnd {
  const double* e0;
  const double* ld0;
  const double* sg0;
  const double* ld1;
  const double* sg1;
  const int32_t* st_all;  // [n_eval][count * nf]
  int n_eval;
  const double* u;
  double* logdet;  // or null
  double* sign;    // or null
  int32_t* accept;
  double* dH;        // or null
  int32_t* status;   // or null
};
hipError_t launch_hmc_end(int count, int nf, const HmcChain* chains, double half_kick, double inv_var,
                          const HmcEnd& a, hipStream_t s);
// Copy the n x n row-major matrix e (or its transpose) into the MFMA
// A-operand order used by the kernels: for NT = ceil(n/16), block
// b = (ti*NT + tk)*4 + r holds at position l the entry
// (16 ti + l%16, 16 tk + l/16 + 4 r) of the zero-padded matrix.
hipError_t launch_swizzle(const double* e, int n, int trans, double* out, hipStream_t s);
// Sweep kernel variants (per tile count nt, chosen by sdq_tune or the
// defaults of sdq_create):
//   0  slice exponential read from its swizzled HBM copy, T in registers
//   1  slice exponential staged in LDS (3 <= nt <= 5), T in registers
//   2  Jacobi SVD stabilizer          3  dense slices
//   4  one wave per 16-column tile, T kept in a per-workgroup HBM scratch
//      between blocks (frees a register matrix), exponential from HBM
//   5  as 4 with the exponential staged in LDS (3 <= nt <= 5)
constexpr int kSweepVariants = 6;
// variant 6: the sweep over block products (k_prod) with one factorization
// each, one wave per tile with T in the workgroup scratch like variant 4
__host__ __device__ constexpr bool sweep_variant_tg(int variant) {
  return variant == 4 || variant == 5 || variant == 6;
}
// doubles of T scratch per workgroup of a variant-4/5 sweep (0 otherwise):
// one 16 x 16 FP64 tile = 256 doubles per (wave, tile column, tile row)
__host__ __device__ inline int64_t sweep_tscr_doubles(int nt, int variant) {
  if (!sweep_variant_tg(variant)) return 0;
  // above kMaxNT tiles the factor store (16 nt x (16 nt + 1)) follows T
  return (int64_t)nt * nt * 256 + (nt > kMaxNT ? (int64_t)16 * nt * (16 * nt + 1) : 0);
}
hipError_t launch_sweep(int nt, int variant, const Inst* inst, const SweepItem* items, int count,
                        Queue* q, int grid, double* tscr, hipStream_t s);
hipError_t launch_pair(int nt, int variant, int mode, const Inst* inst, const PairItem* items,
                       int count, const int32_t* l_list, Queue* q, int grid, hipStream_t s);
// block products of the slices (k_prod): one item per (chain, block j),
// written to Inst::prod + j (16 nt)^2 in the swizzled, zero-padded layout of
// the slice exponential's copy (launch_swizzle); tile counts kProdMinNT ..
// kSweepMaxNT
constexpr int kProdMinNT = 7;
hipError_t launch_prod(int nt, const Inst* inst, const SweepItem* items, int count, Queue* q, int grid,
                       hipStream_t s);
// complex UDT of independent matrices (sdq_complex.hip): w, u, t interleaved
// (re, im) [count][n][n], d [count][n]; 1 <= n <= complex_udt_max_n()
int complex_udt_max_n();
hipError_t launch_udt_complex(int n, int count, const double* w, double* u, double* d, double* t, int grid,
                              hipStream_t s);
hipError_t launch_udt(int nt, int n, int count, const double* w, double* u, double* d, double* t,
                      hipStream_t s);
// One chain of complex dense slices (sdq_greens_complex): slices [m][n][n]
// and g [n][n] interleaved (re, im); logdet a scalar, phase two doubles.
struct CChain {
  const double* slices;
  double* g;
  double* logdet;
  double* phase;
  int32_t* status;
  int32_t n, m, k, pad;
};
// G, log|det(1+B)| and its phase for `count` chains, n <= complex_udt_max_n(),
// one workgroup per chain (grid-stride)
hipError_t launch_greens_complex(const CChain* tab, int count, int grid, hipStream_t s);
// M <- left M right for count n x n matrices (device pointer table), n <= 128
hipError_t launch_similarity(int nt, int n, int count, double* const* mats, const double* left,
                             const double* right, int grid, hipStream_t s);

enum KernelKind { KK_SWEEP = 0, KK_PAIR = 1, KK_UDT = 2, KK_PROD = 3 };

// ---- the fixed scratch of sdq_greens_noalloc (sdq_noalloc.hip) -------------
constexpr size_t kNoAllocBytes = 64ull << 20;  // per device
constexpr int kNoAllocMaxDevices = 64;
// Device address of that device's scratch (hipGetSymbolAddress, looked up
// once per device and cached); call with `device` current.
hipError_t noalloc_scratch(int device, void** ptr);

// ---- chains with n > 128: gang kernels (sdq_gang.hip) --------------------
// A chain is owned by a gang of G workgroups of kGangThreads threads; member
// g keeps columns [g*w, (g+1)*w) of the working matrix in LDS, column-major
// with leading dimension ldr.  Gangs exchange pivot candidates and operands
// through a per-gang scratch area in HBM and synchronize with a counter.
constexpr int kGangMaxN = 1024;
constexpr int kGangThreads = 1024;
constexpr int kGangSlab = 16640;  // doubles of the LDS column slab
constexpr int kGangMaxW = 128;
constexpr int kGangBarWords = 32;  // uint32 words per gang (barrier counter, abort flag, arrivals)

struct GangGeom {
  int npad;  // 16 * ceil(n / 16)
  int G;     // workgroups per chain
  int w;     // columns per workgroup (multiple of 16)
  int ldr;   // LDS column stride
};

__host__ __device__ inline GangGeom gang_geom(int nt) {
  GangGeom g;
  g.npad = 16 * nt;
  g.ldr = g.npad + 4;
  g.G = 0;
  g.w = 0;
  for (int G = 2; G <= 64; ++G) {
    const int w = 16 * (((g.npad + G - 1) / G + 15) / 16);
    if (w <= kGangMaxW && (long long)w * g.ldr <= kGangSlab) {
      g.G = G;
      g.w = w;
      break;
    }
  }
  return g;
}

// per-gang scratch (doubles): R, V, T, U, two G buffers, X, candidates
__host__ __device__ inline int64_t gang_mat(const GangGeom& g) { return (int64_t)g.npad * g.npad; }
__host__ __device__ inline int64_t gang_cand_stride(const GangGeom& g) { return g.npad + 8; }
__host__ __device__ inline int64_t gang_doubles(const GangGeom& g) {
  return 7 * gang_mat(g) + 2 * g.G * gang_cand_stride(g) + 64;
}

struct GangArgs {
  double* scratch;   // ngangs * gang_doubles(geo)
  unsigned* bars;    // ngangs * kGangBarWords, zero at launch
  int ngangs;
  int nt;
};

hipError_t launch_gang_sweep(const Inst* inst, const SweepItem* items, int count, GangArgs a,
                             hipStream_t s);
hipError_t launch_gang_pair(int mode, const Inst* inst, const PairItem* items, int count,
                            const int32_t* l_list, GangArgs a, hipStream_t s);
hipError_t launch_gang_udt(int n, int count, const double* w, double* u, double* d, double* t,
                           GangArgs a, hipStream_t s);
// largest number of gangs of tile count nt that can be resident at once
hipError_t gang_capacity(int nt, int num_cu, int* ngangs);

}  // namespace sdq
