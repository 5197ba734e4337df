// sdq_nt9.hip -- the stabilized sweep for 128 < n <= 144 as one workgroup:
// nine waves, one per 16-column tile, T and the factor store in a
// per-workgroup area of device memory (the factor store alone, 144 x 145
// doubles, exceeds the CU's LDS); and the block products of the slices
// (k_prod) at this size.  Every other kernel of this size runs as a gang
// (sdq_gang.hip); the stages the sweep writes have the same layout.
#include "sdq_device.hpp"

namespace sdq {

// variant 4: slices E diag(exp(alpha f)); variant 6: the block products of
// k_prod (swizzled), one factorization each
hipError_t launch_sweep_nt9(int variant, const Inst* inst, const SweepItem* items, int count, Queue* q,
                            int grid, double* tscr, hipStream_t s) {
  if ((variant != 4 && variant != 6) || !tscr) return hipErrorInvalidValue;
  if (variant == 6)
    hipLaunchKernelGGL((k_sweep<9, 9, false, false, true, true, true>), dim3(grid), dim3(Geo<9, 9>::THREADS), 0, s,
                       inst, items, count, q, tscr);
  else
    hipLaunchKernelGGL((k_sweep<9, 9, false, false, false, true>), dim3(grid), dim3(Geo<9, 9>::THREADS), 0, s,
                       inst, items, count, q, tscr);
  return hipGetLastError();
}

hipError_t launch_prod_nt9(const Inst* inst, const SweepItem* items, int count, Queue* q, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_prod<9, 9>), dim3(grid), dim3(Geo<9, 9>::THREADS), 0, s, inst, items, count, q);
  return hipGetLastError();
}

template <class KF>
static hipError_t info9(KF kern, int lds, KernelInfo* out) {
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, Geo<9, 9>::THREADS, 0);
  out->threads = Geo<9, 9>::THREADS;
  out->lds_bytes = lds;
  out->blocks_per_cu = nb;
  return e;
}

hipError_t kernel_info_nt9(int kind, int variant, KernelInfo* out) {
  if (kind == KK_PROD) return info9(k_prod<9, 9>, (int)sizeof(ProdSmem<9, 9>), out);
  if (kind != KK_SWEEP || (variant != 4 && variant != 6)) return hipErrorInvalidValue;
  if (variant == 6)
    return info9(k_sweep<9, 9, false, false, true, true, true>, (int)sizeof(Smem<9, 9, false>), out);
  return info9(k_sweep<9, 9, false, false, false, true>, (int)sizeof(Smem<9, 9, false>), out);
}

}  // namespace sdq
