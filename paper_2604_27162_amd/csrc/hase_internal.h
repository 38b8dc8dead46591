// Internal interface between the host runtime (hase_runtime.cpp) and the
// gfx950 kernels (hase_kernels.hip). Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace hase {

// Every grid is stored on the device as a padded row bitboard (terrain envs:
// two of them, the tile-type planes, one after the other): PAD cells of
// "outside" on each side (PAD >= the largest view radius, so windows and move
// targets never leave the board), bit x' of padded row y' in word
// y' * LDS_ROW + (x' >> 5) (the words past P = ceil((W + 2 PAD) / 32) of a row
// are 0), then one slack word of ones. Cells outside the map read as
// blocking, so a move check needs no separate bounds test. The layout in HBM
// is the one the step kernel keeps in LDS, so staging a board is a plain copy.
constexpr int PAD = 4;
constexpr int MAX_AGENTS = 20;
constexpr int MAX_SIDE = 64;
constexpr int SPAWN_ATTEMPTS = 64;

// Agent-count buckets -> compile-time agent capacity of the step kernel.
constexpr int N_BUCKETS = 4;
constexpr int BUCKET_NMAX[N_BUCKETS] = {2, 4, 10, 20};
// one step-kernel variant per (agent-count bucket, view radius)
constexpr int MAX_VARIANTS = N_BUCKETS * PAD;

inline int board_words_per_row(int W) { return (W + 2 * PAD + 31) >> 5; }

// Every board row takes LDS_ROW words whatever the width (the widest padded
// row, MAX_SIDE + 2 PAD = 72 cells, needs 3), so row offsets are
// compile-time constants of the step kernel; plus one slack word so a
// two-word window read at the last row stays inside the board.
constexpr int LDS_ROW = 3;
constexpr int lds_board_words(int H) { return (H + 2 * PAD) * LDS_ROW + 1; }

// Words of an env's boards (planes of them, one after the other) rounded up
// to a multiple of 4: in HBM every env's boards start 16-byte aligned and in
// LDS every env slot does, so a lane stages 4 words per load and store.
constexpr int round4(int v) { return (v + 3) & ~3; }
constexpr int board_words(int H, int planes) { return round4(planes * lds_board_words(H)); }
static_assert(MAX_AGENTS % 4 == 0, "LDS env slots are whole 16-byte units");

// Packed per-env spec words.
//   spec0 = H | W << 8 | n << 16 | S << 24
//   spec1 = r | C << 4 | flags << 8 | L << 16
//   spec2 = wall_pct | P << 8
struct EnvTables {
    const uint32_t *perm;  // tile slot -> env index (tiles group similar envs)
    const uint32_t *spec0, *spec1, *spec2;
    const uint32_t *obs_off, *agent_off, *bb_off, *grid_off, *env_id;
    const uint32_t *map_off;  // first discovery-map word (exploring envs)
    // terrain envs, 8 words per env: stuck chance << 16 (word 0), move chances
    // (bytes of words 1..3, class * 3 + tile), agent classes (words 4, 5)
    const uint32_t *terr;
};

// Discovery map of an exploring env in HBM (state and per-step output): H
// rows of ceil(W/32) words, cell (x, y) at bit x & 31 of word
// y * ceil(W/32) + x / 32. In LDS the step kernel keeps it in the padded
// board layout (rows of LDS_ROW words, bit x + PAD of padded row y + PAD), so
// an agent's window addresses it exactly like the wall board.
inline int map_words(int H, int W) { return H * ((W + 31) >> 5); }

// One stepping job: a batch's state plus this call's output buffers. Per-step
// output strides are in elements; outputs of env e at output step s go to
// obs[s * obs_stride + obs_off[e]], rew[s * agent_stride + agent_off[e]],
// done[s * env_stride + e]; external actions are read at the same step index.
struct JobDesc {
    EnvTables tab;
    const uint64_t *seed;
    uint32_t *found, *t, *ep, *steps;
    uint16_t *pos;        // x | y << 8, unpadded
    const uint32_t *bb;   // padded bitboards
    uint32_t *obs;
    float *rew;
    uint8_t *done;
    const int8_t *act;    // may be null
    uint64_t obs_stride, agent_stride, env_stride;
    uint32_t k_limit;     // steps this job may take in one launch
    uint32_t out_step0;   // output step index of the job's first step in this launch
    uint32_t *disc;       // discovery maps (state), at tab.map_off[e]
    uint32_t *stuck;      // stuck agents per env (terrain)
    uint32_t *map;        // per-step map output, may be null
    uint64_t map_stride;  // map words per output step
    uint32_t *bel;        // per-agent hider beliefs (radio), at tab.agent_off[e]
    // the true state after each step (may be null): agent positions x | y << 8
    // per output row (agent_stride entries, the rewards' places), and per env
    // four words found, t, episode, stuck (env_stride * 4 words per row)
    uint16_t *spos;
    uint32_t *senv;
    // A resident range of an arena (resident = 1): envs [first, first + count)
    // of one spec, outputs relative to the range (env first + i writes obs
    // words from i * obs_env, rewards from i * n, done byte i, map words from
    // i * map_env), the output row of a step is the env's step count since
    // the range's reset, and the range stops after budget steps.
    uint32_t resident, first, budget, obs_env, map_env;
    // launch filter (read from the kernel's by-value job only): a wave steps
    // its tile only if the tile's group (variant >> 8) equals group;
    // 0xffffffff steps every tile
    uint32_t group;
};

// A wave's work: envs perm[env0 .. env0 + count) of job `job` (count <= 64 /
// lanes; 0: an empty tile, skipped); variant = agent-count bucket * 4 + view
// radius - 1 (read by the mixed-variant kernel), plus, for the tiles of an
// arena, the launch group (group_code) in bits 8 and up.
struct Tile {
    uint32_t job, env0, count, variant;
};
constexpr uint32_t ALL_GROUPS = 0xffffffffu;
// launch group of a tile: env kind, lanes per env, and whether its bucket is
// the one of up to 20 agents (a kernel of its own)
constexpr uint32_t group_code(int kind, int lanes, bool big)
{
    return (uint32_t)kind | ((uint32_t)lanes << 8) | (big ? 1u << 16 : 0u);
}

struct InitArgs {
    EnvTables tab;
    uint64_t *seed;
    uint32_t *found, *t, *ep, *steps;
    uint16_t *pos;
    uint8_t *walls;
    uint32_t *bb;
    uint32_t *disc;       // discovery maps, cleared at reset
    uint32_t *stuck;      // stuck agents, cleared at reset
    uint32_t *bel;        // per-agent beliefs, cleared at reset
    uint32_t *err;        // min over envs with too few free cells (reset only), minus env0
    uint64_t seed_value;
    uint32_t env0;        // block b resets env env0 + b
    uint32_t n_envs;
    uint32_t rebuild_only; // 1: walls/positions already loaded, only rebuild bitboards
};

// Setup of an arena range (one kernel, by-value arguments): the per-slot
// spec words, terrain words and env ids of slots [first, first + count),
// their tiles (tile i of the range at tile index first + i, the rest of the
// range's tile entries emptied), the range's job descriptor and error word.
// With clear = 1 only the tile entries of the slots are emptied (release).
struct RangeArgs {
    uint32_t *spec0, *spec1, *spec2, *terr, *env_id;
    Tile *tiles;
    JobDesc *jobs;
    uint32_t *job_err;
    JobDesc job;
    uint32_t job_index, first, count, clear;
    uint32_t s0, s1, s2, env_id_base, lanes, variant;
    uint32_t terr_words[8];
};
hipError_t launch_range(const RangeArgs &a, hipStream_t stream);

// Env kinds: each kind has its own step loop and its own kernels (so the
// register allocation of one never burdens another), and a tile holds envs
// of one kind only.
constexpr int KIND_PLAIN = 0;    // no line of sight, no exploration, no terrain
constexpr int KIND_EXPLORE = 1;  // bit 0: exploration
constexpr int KIND_LOS = 2;      // bit 1: line of sight
constexpr int KIND_TERRAIN = 4;  // bit 2: terrain
constexpr int KIND_RADIO = 8;    // bit 3: radio belief sharing
constexpr int N_KINDS = 16;      // kinds 0..15
inline int env_kind(uint32_t flags)
{
    return ((flags & 8u) ? KIND_LOS : 0) | ((flags & 16u) ? KIND_EXPLORE : 0) |
           ((flags & 32u) ? KIND_TERRAIN : 0) | ((flags & 64u) ? KIND_RADIO : 0);
}

// Launch the step kernel for tile range [tile0, tile0 + n_tiles) of variant
// (lanes, nmax, view radius r). K == 0 writes the observation of the current
// state only. Every env of the range is of the plain kind.
hipError_t launch_step(int lanes, int nmax, int r, const Tile *tiles, uint32_t n_tiles,
                       const JobDesc *jobs, const JobDesc &job0, uint32_t K,
                       uint32_t step_base, uint32_t slot_words, hipStream_t stream);

// One launch over tiles of several (bucket, radius) variants that share
// `lanes`, all envs of kind `kind`; slot_words is the largest board among
// them (both tile planes for terrain), map_words the LDS words of a
// discovery map per env (the largest one-plane board among the exploring
// envs, else 0).
hipError_t launch_mixed(int lanes, int kind, const Tile *tiles, uint32_t n_tiles,
                        const JobDesc *jobs, const JobDesc &job0, uint32_t K, uint32_t step_base,
                        uint32_t slot_words, uint32_t map_words, bool big, hipStream_t stream);

// The plain envs of an uneven batch whose buckets take 4 lanes per env (up
// to 4 agents) and 16 (up to 10 agents) in one launch: tiles of 16 lanes per
// env have bit 4 of their variant set; the envs of the 10-agent bucket with
// at most COMBO_MID_NMAX agents run at 8 lanes per env, one agent per lane,
// in tiles with bit 5 set (hase_combo.hip).
constexpr uint32_t COMBO_WIDE = 16u;
constexpr uint32_t COMBO_MID = 32u;
constexpr int COMBO_MID_NMAX = 8;
// LDS bytes per wave of that launch: 16 env slots for the 4-lane tiles, or 8
// slots with the two agent planes each for the 8-lane tiles (the 16-lane
// tiles' 4 such slots need less than either).
inline size_t combo_lds_bytes(uint32_t slot_words)
{
    const size_t narrow = (size_t)16 * (slot_words + MAX_AGENTS);
    const size_t mid = (size_t)8 * (3 * (size_t)slot_words + MAX_AGENTS);
    return (narrow > mid ? narrow : mid) * sizeof(uint32_t);
}
hipError_t launch_combo(const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                        const JobDesc &job0, uint32_t K, uint32_t step_base, uint32_t slot_words,
                        hipStream_t stream);

hipError_t launch_init(const InitArgs &a, hipStream_t stream);

// Bytes of the library's static device workspace (per GPU) and the device
// address of the current device's copy (looked up once per device).
constexpr size_t STATIC_WORKSPACE_BYTES = 1u << 20;
hipError_t static_workspace(void **ptr);

// Per-lanes entry points, one translation unit each: single-variant and
// mixed plain kernels (hase_step_l<L>.hip, hase_mixed_l<L>.hip), the line of
// sight and exploration kinds (hase_feat_l<L>.hip) and the terrain kinds
// (hase_terr_l<L>.hip, with line of sight hase_terrlos_l<L>.hip); the radio
// kinds without terrain (hase_radio_l<L>.hip) and with it
// (hase_radioter_l<L>.hip).
#define HASE_DECLARE_LANES(L)                                                                     \
    hipError_t launch_step_lanes##L(int nmax, int r, const Tile *tiles, uint32_t n_tiles,        \
                                    const JobDesc *jobs, const JobDesc &job0, uint32_t K,         \
                                    uint32_t step_base, uint32_t slot_words, hipStream_t stream); \
    hipError_t launch_mixed_lanes##L(const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,   \
                                     const JobDesc &job0, uint32_t K, uint32_t step_base,         \
                                     uint32_t slot_words, uint32_t map_words, bool big,                     \
                                     hipStream_t stream);                                         \
    hipError_t launch_feat_lanes##L(int kind, const Tile *tiles, uint32_t n_tiles,               \
                                    const JobDesc *jobs, const JobDesc &job0, uint32_t K,         \
                                    uint32_t step_base, uint32_t slot_words, uint32_t map_words, bool big,  \
                                    hipStream_t stream);                                          \
    hipError_t launch_terr_lanes##L(int kind, const Tile *tiles, uint32_t n_tiles,               \
                                    const JobDesc *jobs, const JobDesc &job0, uint32_t K,         \
                                    uint32_t step_base, uint32_t slot_words, uint32_t map_words, bool big,  \
                                    hipStream_t stream);                                          \
    hipError_t launch_terrlos_lanes##L(int kind, const Tile *tiles, uint32_t n_tiles,            \
                                       const JobDesc *jobs, const JobDesc &job0, uint32_t K,      \
                                       uint32_t step_base, uint32_t slot_words,                   \
                                       uint32_t map_words, bool big, hipStream_t stream);                   \
    hipError_t launch_radio_lanes##L(int kind, const Tile *tiles, uint32_t n_tiles,              \
                                     const JobDesc *jobs, const JobDesc &job0, uint32_t K,        \
                                     uint32_t step_base, uint32_t slot_words, uint32_t map_words, bool big, \
                                     hipStream_t stream);                                         \
    hipError_t launch_radioter_lanes##L(int kind, const Tile *tiles, uint32_t n_tiles,           \
                                        const JobDesc *jobs, const JobDesc &job0, uint32_t K,     \
                                        uint32_t step_base, uint32_t slot_words,                  \
                                        uint32_t map_words, bool big, hipStream_t stream);
HASE_DECLARE_LANES(1)
HASE_DECLARE_LANES(2)
HASE_DECLARE_LANES(4)
HASE_DECLARE_LANES(8)
HASE_DECLARE_LANES(16)
#undef HASE_DECLARE_LANES

bool variant_supported(int lanes, int nmax);

}  // namespace hase
