// Single-variant step kernels with 16 lanes per environment (one translation
// unit per lanes value and kernel kind, so they compile in parallel).
#include "hase_device.h"

namespace hase {

hipError_t launch_step_lanes16(int nmax, int r, const Tile *tiles, uint32_t n_tiles,
                               const JobDesc *jobs, const JobDesc &job0, uint32_t K,
                               uint32_t step_base, uint32_t slot_words, hipStream_t stream)
{
    return launch_lanes<16>(nmax, r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
}

}  // namespace hase
