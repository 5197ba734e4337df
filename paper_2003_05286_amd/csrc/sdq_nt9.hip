// sdq_nt9.hip -- the stabilized sweep for 128 < n <= 144 as one workgroup:
// nine waves, one per 16-column tile, T and the factor store in a
// per-workgroup area of device memory (the factor store alone, 144 x 145
// doubles, exceeds the CU's LDS).  Every other kernel of this size runs as
// a gang (sdq_gang.hip); the stages the sweep writes have the same layout.
#include "sdq_device.hpp"

namespace sdq {

hipError_t launch_sweep_nt9(int variant, const Inst* inst, const SweepItem* items, int count, Queue* q,
                            int grid, double* tscr, hipStream_t s) {
  if (variant != 4 || !tscr) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep<9, 9, false, false, false, true>), dim3(grid), dim3(Geo<9, 9>::THREADS), 0, s, inst,
                     items, count, q, tscr);
  return hipGetLastError();
}

hipError_t kernel_info_nt9(int kind, int variant, KernelInfo* out) {
  if (kind != KK_SWEEP || variant != 4) return hipErrorInvalidValue;
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep<9, 9, false, false, false, true>,
                                                              Geo<9, 9>::THREADS, 0);
  out->threads = Geo<9, 9>::THREADS;
  out->lds_bytes = (int)sizeof(Smem<9, 9, false>);
  out->blocks_per_cu = nb;
  return e;
}

}  // namespace sdq
