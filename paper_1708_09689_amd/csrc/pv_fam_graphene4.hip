// Sweep kernels of the graphene4 stencil family (one translation unit per family).
#include "pv_sweep.hpp"

namespace pv {

hipError_t launch_sweep_graphene4(SweepParams& p, int num_cus, hipStream_t s) {
    return launch_family<PatGraphene4>(p, num_cus, s);
}

hipError_t batch_fill_record_graphene4(const SweepParams& p, int staged, void* dst, int* nblocks) {
    return batch_fill_record_fam<PatGraphene4>(p, staged, dst, nblocks);
}

hipError_t launch_batch_sweep_graphene4(const SweepParams& p, int staged, const void* table, const int* block_inst,
                                  const int* inst_block0, int grid, int red_step, hipStream_t s) {
    return launch_batch_sweep_fam<PatGraphene4>(p, staged, table, block_inst, inst_block0, grid, red_step, s);
}

}  // namespace pv
