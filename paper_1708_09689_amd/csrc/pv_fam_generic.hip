// Sweep kernels of generic stencils with 1, 2 or 4 orbitals (one translation
// unit per family).
#include "pv_sweep.hpp"

namespace pv {

hipError_t launch_sweep_generic(SweepParams& p, int num_cus, hipStream_t s) {
    switch (p.n_orb) {
        case 1: return launch_family<PatGeneric<1>>(p, num_cus, s);
        case 2: return launch_family<PatGeneric<2>>(p, num_cus, s);
        case 4: return launch_family<PatGeneric<4>>(p, num_cus, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t batch_fill_record_generic(const SweepParams& p, int staged, void* dst, int* nblocks) {
    switch (p.n_orb) {
        case 1: return batch_fill_record_fam<PatGeneric<1>>(p, staged, dst, nblocks);
        case 2: return batch_fill_record_fam<PatGeneric<2>>(p, staged, dst, nblocks);
        case 4: return batch_fill_record_fam<PatGeneric<4>>(p, staged, dst, nblocks);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_sweep_generic(const SweepParams& p, int staged, const void* table, const int* block_inst,
                                      const int* inst_block0, int grid, int red_step, hipStream_t s) {
    switch (p.n_orb) {
        case 1: return launch_batch_sweep_fam<PatGeneric<1>>(p, staged, table, block_inst, inst_block0, grid, red_step,
                                                             s);
        case 2: return launch_batch_sweep_fam<PatGeneric<2>>(p, staged, table, block_inst, inst_block0, grid, red_step,
                                                             s);
        case 4: return launch_batch_sweep_fam<PatGeneric<4>>(p, staged, table, block_inst, inst_block0, grid, red_step,
                                                             s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pv
