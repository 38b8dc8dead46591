// The combined kernel of the plain envs of uneven batches (4 lanes per env
// for up to 4 agents, 8 for up to 8, 16 for up to 10, one launch).
#include "hase_device.h"

namespace hase {

hipError_t launch_combo(const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                        const JobDesc &job0, uint32_t K, uint32_t step_base, uint32_t slot_words,
                        hipStream_t stream)
{
    if (n_tiles == 0) return hipSuccess;
    // the widest slot array of the three tile widths
    const size_t lds = combo_lds_bytes(slot_words);
    hipLaunchKernelGGL((step_kernel_combo<KIND_PLAIN>), dim3(n_tiles), dim3(64), lds, stream, tiles,
                       n_tiles, jobs, job0, K, step_base, slot_words, 0u);
    return hipGetLastError();
}

}  // namespace hase
