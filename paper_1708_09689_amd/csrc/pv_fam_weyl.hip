// Sweep kernels of the weyl stencil family (one translation unit per family).
#include "pv_sweep.hpp"

namespace pv {

hipError_t launch_sweep_weyl(SweepParams& p, int num_cus, hipStream_t s) {
    return launch_family<PatWeyl>(p, num_cus, s);
}

hipError_t batch_fill_record_weyl(const SweepParams& p, int staged, void* dst, int* nblocks) {
    return batch_fill_record_fam<PatWeyl>(p, staged, dst, nblocks);
}

hipError_t launch_batch_sweep_weyl(const SweepParams& p, int staged, const void* table, const int* block_inst,
                                  const int* inst_block0, int grid, int red_step, hipStream_t s) {
    return launch_batch_sweep_fam<PatWeyl>(p, staged, table, block_inst, inst_block0, grid, red_step, s);
}

}  // namespace pv
