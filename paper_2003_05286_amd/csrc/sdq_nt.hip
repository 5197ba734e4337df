// sdq_nt.hip -- instantiates the kernels of sdq_device.hpp for one tile
// count SDQ_NT (the build compiles this file once per NT = 1..8, in parallel)
// and exports its launchers under NT-specific names.
#include "sdq_device.hpp"

#ifndef SDQ_NT
#error "define SDQ_NT"
#endif

#define SDQ_CAT2(a, b) a##b
#define SDQ_CAT(a, b) SDQ_CAT2(a, b)

namespace sdq {

hipError_t SDQ_CAT(launch_sweep_nt, SDQ_NT)(int variant, const Inst* inst, const SweepItem* items,
                                           int count, Queue* q, int grid, double* tscr, hipStream_t s) {
  return Launch<SDQ_NT>::sweep(variant, inst, items, count, q, grid, tscr, s);
}
hipError_t SDQ_CAT(launch_pair_nt, SDQ_NT)(int mode, const Inst* inst, const PairItem* items,
                                          int count, const int32_t* l_list, Queue* q, int grid,
                                          hipStream_t s) {
  return Launch<SDQ_NT>::pair(mode, inst, items, count, l_list, q, grid, s);
}
hipError_t SDQ_CAT(launch_udt_nt, SDQ_NT)(int n, int count, const double* w, double* u, double* d,
                                         double* t, hipStream_t s) {
  return Launch<SDQ_NT>::udt(n, count, w, u, d, t, s);
}
hipError_t SDQ_CAT(launch_sim_nt, SDQ_NT)(int n, int count, double* const* mats, const double* left,
                                         const double* right, int grid, hipStream_t s) {
  return Launch<SDQ_NT>::similarity(n, count, mats, left, right, grid, s);
}
hipError_t SDQ_CAT(kernel_info_nt, SDQ_NT)(int kind, int variant, KernelInfo* out) {
  return Launch<SDQ_NT>::info(kind, variant, out);
}

}  // namespace sdq
