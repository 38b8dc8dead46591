// Mixed-variant step kernels with 2 lane(s) per environment for the radio
// kinds without terrain: radio alone, with exploration, with line of sight,
// and with both (one kernel each).
#include "hase_device.h"

namespace hase {

hipError_t launch_radio_lanes2(int kind, const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                               const JobDesc &job0, uint32_t K, uint32_t step_base, uint32_t slot_words,
                               uint32_t map_words, bool big, hipStream_t stream)
{
    switch (kind) {
#define HASE_RADIO_CASE(KD)                                                                   \
    case KD:                                                                                  \
        return launch_mixed_l<2, KD>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, \
                                      map_words, big, stream);
    HASE_RADIO_CASE(KIND_RADIO)
    HASE_RADIO_CASE(KIND_RADIO | KIND_EXPLORE)
    HASE_RADIO_CASE(KIND_RADIO | KIND_LOS)
    HASE_RADIO_CASE(KIND_RADIO | KIND_LOS | KIND_EXPLORE)
#undef HASE_RADIO_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hase
