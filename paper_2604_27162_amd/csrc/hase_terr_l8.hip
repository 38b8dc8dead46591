// Mixed-variant step kernels with 8 lanes per environment for the terrain
// kinds: terrain alone and with exploration (one kernel each); the kinds
// with line of sight are in hase_terrlos_l8.hip.
#include "hase_device.h"

namespace hase {

hipError_t launch_terr_lanes8(int kind, const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                              const JobDesc &job0, uint32_t K, uint32_t step_base, uint32_t slot_words,
                              uint32_t map_words, bool big, hipStream_t stream)
{
    switch (kind) {
    case KIND_TERRAIN:
        return launch_mixed_l<8, KIND_TERRAIN>(tiles, n_tiles, jobs, job0, K, step_base,
                                               slot_words, map_words, big, stream);
    case KIND_TERRAIN | KIND_EXPLORE:
        return launch_mixed_l<8, KIND_TERRAIN | KIND_EXPLORE>(tiles, n_tiles, jobs, job0, K, step_base,
                                                              slot_words, map_words, big, stream);
    case KIND_TERRAIN | KIND_LOS:
    case KIND_TERRAIN | KIND_LOS | KIND_EXPLORE:
        return launch_terrlos_lanes8(kind, tiles, n_tiles, jobs, job0, K, step_base, slot_words,
                                     map_words, big, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hase
