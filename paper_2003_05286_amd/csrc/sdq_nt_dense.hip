// sdq_nt_dense.hip -- the dense-slice sweep and G(tau,0) of sdq_device.hpp,
// and the block products of the slices, for one tile count SDQ_NT (compiled
// once per NT = 1..8, like sdq_nt.hip, but apart from it: the other kernels'
// code does not depend on these instantiations).
#include "sdq_device.hpp"

#ifndef SDQ_NT
#error "define SDQ_NT"
#endif

#define SDQ_CAT2(a, b) a##b
#define SDQ_CAT(a, b) SDQ_CAT2(a, b)

namespace sdq {

hipError_t SDQ_CAT(launch_dense_sweep_nt, SDQ_NT)(const Inst* inst, const SweepItem* items, int count, Queue* q,
                                                 int grid, hipStream_t s) {
  return Launch<SDQ_NT>::dense_sweep(inst, items, count, q, grid, s);
}
hipError_t SDQ_CAT(launch_bprod_sweep_nt, SDQ_NT)(const Inst* inst, const SweepItem* items, int count, Queue* q,
                                                 int grid, double* tscr, hipStream_t s) {
  return Launch<SDQ_NT>::bprod_sweep(inst, items, count, q, grid, tscr, s);
}
hipError_t SDQ_CAT(bprod_sweep_info_nt, SDQ_NT)(KernelInfo* out) { return Launch<SDQ_NT>::bprod_sweep_info(out); }
hipError_t SDQ_CAT(dense_info_nt, SDQ_NT)(KernelInfo* out) { return Launch<SDQ_NT>::dense_info(out); }
hipError_t SDQ_CAT(launch_prod_nt, SDQ_NT)(const Inst* inst, const SweepItem* items, int count, Queue* q,
                                          int grid, hipStream_t s) {
  return Launch<SDQ_NT>::prod(inst, items, count, q, grid, s);
}
hipError_t SDQ_CAT(prod_info_nt, SDQ_NT)(KernelInfo* out) { return Launch<SDQ_NT>::prod_info(out); }
hipError_t SDQ_CAT(launch_dense_pair_nt, SDQ_NT)(const Inst* inst, const PairItem* items, int count,
                                                const int32_t* l_list, Queue* q, int grid, hipStream_t s) {
  return Launch<SDQ_NT>::dense_pair(inst, items, count, l_list, q, grid, s);
}
hipError_t SDQ_CAT(dense_pair_info_nt, SDQ_NT)(KernelInfo* out) { return Launch<SDQ_NT>::dense_pair_info(out); }

}  // namespace sdq
