// Mixed-variant step kernels with 2 lanes per environment for the feature
// kinds: exploration, line of sight, and both (one kernel each).
#include "hase_device.h"

namespace hase {

hipError_t launch_feat_lanes2(int kind, const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                              const JobDesc &job0, uint32_t K, uint32_t step_base, uint32_t slot_words,
                              uint32_t map_words, bool big, hipStream_t stream)
{
    switch (kind) {
    case KIND_EXPLORE:
        return launch_mixed_l<2, KIND_EXPLORE>(tiles, n_tiles, jobs, job0, K, step_base,
                                               slot_words, map_words, big, stream);
    case KIND_LOS:
        return launch_mixed_l<2, KIND_LOS>(tiles, n_tiles, jobs, job0, K, step_base,
                                           slot_words, map_words, big, stream);
    case KIND_LOS | KIND_EXPLORE:
        return launch_mixed_l<2, KIND_LOS | KIND_EXPLORE>(tiles, n_tiles, jobs, job0, K, step_base,
                                                          slot_words, map_words, big, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hase
