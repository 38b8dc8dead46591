// Mixed-variant step kernel with 2 lanes per environment (per-tile variant
// switch) for plain envs.
#include "hase_device.h"

namespace hase {

hipError_t launch_mixed_lanes2(const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                               const JobDesc &job0, uint32_t K, uint32_t step_base,
                               uint32_t slot_words, uint32_t map_words, bool big, hipStream_t stream)
{
    return launch_mixed_l<2, KIND_PLAIN>(tiles, n_tiles, jobs, job0, K, step_base, slot_words,
                                         map_words, big, stream);
}

}  // namespace hase
