/*
 * hase.h -- C ABI of the MI355X (gfx950) vectorised hide-and-seek step.
 *
 * One call steps thousands of independent hide-and-seek gridworlds: every
 * agent's discrete action is applied under the wall and collision rules,
 * seeker/hider detection becomes rewards and termination flags, finished
 * episodes auto-reset from their unchanged grid, random actions come from a
 * counter-based generator, and every agent's bit-packed egocentric window is
 * written. This is the data-parallel environment step of the paper's engine
 * (Sec. 4.1: the step loop over environments, with rewards, termination and
 * truncation outputs; Sec. 4.2: pristine-grid resets; Sec. 3.3: desynchronised
 * initialisation and the decentralised observation mode), reduced to a
 * discrete gridworld (Sec. 3.1 problem tuple, Sec. 3.2 blocking tiles).
 *
 * Memory: the caller allocates ALL device memory (state buffer, actions,
 * observations, rewards, dones), e.g. as torch tensors; the library keeps only
 * a host handle and never frees caller memory. Pointers named d_* are device
 * pointers, h_* are host pointers.
 *
 * Asynchrony: hase_step and hase_observe only enqueue work on the handle's
 * stream (hipStream_t passed as void*); the caller synchronises. hase_reset,
 * hase_get_state and hase_set_state synchronise the stream before returning.
 *
 * Errors: every call returns HASE_OK (0) or a negative code; arguments are
 * validated before any work is enqueued. hase_last_error() gives a
 * thread-local detail string for the last failing call of the calling thread.
 *
 * Threading: one handle must not be used from two host threads at once;
 * distinct handles are independent and may share a stream.
 */
#ifndef HASE_H
#define HASE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define HASE_OK 0
#define HASE_EINVAL (-1)  /* bad spec or argument */
#define HASE_ENOMEM (-2)  /* caller's state buffer smaller than required */
#define HASE_EGRID (-3)   /* an env has too few free cells for its agents */
#define HASE_EHIP (-4)    /* HIP runtime error (detail in hase_last_error) */
#define HASE_ESTATE (-5)  /* state arrays inconsistent with the batch */
#define HASE_ENOTREADY (-6) /* step/observe before the first reset or set_state */

/* ---------------------------------------------------------------- flags */
#define HASE_COLLIDE 1u      /* a move into a cell held by another agent is rejected */
#define HASE_CAPTURE_ENDS 2u /* the episode terminates once every hider was found */
#define HASE_DESYNC 4u       /* first episode starts with t0 ~ U{0..L-1} elapsed */
/* line of sight (Sec. 3.1, observation function: a deterministic line-of-sight
 * projection): a window cell is hidden when the open segment between the
 * centres of the agent's cell and that cell passes through the inside of a
 * blocking cell (a wall or outside the map) other than the two end cells;
 * hidden cells read 0 in every channel and a seeker sees a hider only if the
 * hider's cell is visible */
#define HASE_OCCLUDE 8u
/* exploration (Sec. 3.1 intrinsic reward for undiscovered tiles; Sec. 3.3
 * centralised observation; the discovery-map layer of the observation tensor
 * table): each env keeps a discovery map of the cells its seekers have seen
 * this episode (empty at every episode start); after the moves of a step a
 * seeker earns 1/128 per cell of its window (inside the map, visible under
 * HASE_OCCLUDE) absent from the map before that step, then those cells join
 * the map; its reward is (128 * detections + new cells) / 128. The map after
 * each step is the optional output of hase_step_maps. */
#define HASE_EXPLORE 16u
/* terrain (Sec. 3.2 traversal kinetics, collision models and agent-tile move
 * speed; the tile flags W/A/F/B and the AgentState stuck / walk / fly / swim
 * bits of Fig. "Bit Packing Environment Structure"): cells are ground
 * (walkable, flyable), wall (blocking), water (aquatic, flyable) or mud
 * (walkable, flyable, sticky); agents are walkers (ground, mud), swimmers
 * (water) or flyers (all but walls). A move onto a tile the agent's class may
 * not enter is blocked; an allowed move succeeds with the (class, tile) move
 * chance; a walker entering mud gets stuck with the stuck chance; a stuck
 * agent does not move until, after the moves of a step, a teammate that is
 * not stuck stands within Chebyshev distance 1. Observation channel 0 holds
 * the tiles the agent's class may not enter. With HASE_OCCLUDE, only walls
 * and cells outside the map block sight. */
#define HASE_TERRAIN 32u
/* radio belief sharing (Sec. 3.3, radio paragraph; the 1-D belief vector of
 * the observation space, Sec. 3.1): every agent keeps a belief word, bit h
 * set when it knows of hider h this episode (empty at every episode start).
 * After the detections of a step a seeker's belief gains the hiders it sees;
 * then every agent whose radio target is another agent sends it its belief,
 * all messages formed before any is delivered, and the receiver ORs it in
 * (so the beliefs of an env together equal its found word). Targets come
 * with the actions: a drawn action also draws a target (the RADIO stream,
 * uniform over the n agents, the agent itself meaning no message); an
 * external action v >= 0 moves v mod 5 and names target v / 5 - 1 (v / 5 = 0
 * or > n: no message); other negative values than -1 stay without a message.
 * Each agent's observation ends with its belief word after the channels.
 * Radio changes no move, reward or episode end. */
#define HASE_RADIO 64u

/* step modes */
#define HASE_STEP_PERSISTENT 0u  /* all n_steps in one launch per tile variant (graph-replayed) */
#define HASE_STEP_PER_LAUNCH 1u  /* one kernel launch per step (baseline) */

/*
 * One environment's configuration.
 *   height, width  grid size, 2..64 each; cell (x, y), x = column, y = row,
 *                  y = 0 the top row
 *   n_agents       1..20 (the paper's agent bound, Sec. 3)
 *   n_seekers      0..n_agents; agents [0, n_seekers) seek, the rest hide
 *   view_radius    r in 1..4: the window is (2r+1) x (2r+1) cells, and a seeker
 *                  detects a hider at Chebyshev distance <= r
 *   n_channels     3 (blocked, teammate, opponent) or 4 (+ outside-the-map)
 *   wall_pct       0..99: each cell is an iid blocking tile with this
 *                  probability (integer threshold, see hase_reset)
 *   flags          HASE_COLLIDE | HASE_CAPTURE_ENDS | HASE_DESYNC |
 *                  HASE_OCCLUDE | HASE_EXPLORE | HASE_TERRAIN | HASE_RADIO
 *   episode_len    L in 1..65535: truncation when t reaches L
 * Terrain fields (read only with HASE_TERRAIN; 0 otherwise):
 *   water_pct, mud_pct  percent of water and mud cells, wall_pct + water_pct
 *                  + mud_pct <= 99 (the same draw per cell as the walls: wall
 *                  below floor(wall_pct 2^32 / 100), else water below the
 *                  threshold of wall_pct + water_pct, else mud below that of
 *                  the three, else ground)
 *   stuck_pct      0..100, chance that a walker entering mud gets stuck
 *   speed_pct      0..100, chance that a move onto a tile succeeds, index
 *                  class * 3 + tile (classes walker, swimmer, flyer; tiles
 *                  ground, water, mud)
 *   agent_classes  2 bits per agent (bits 2i, 2i+1 for agent i): 0 walker,
 *                  1 swimmer, 2 flyer; 0 for i >= n_agents
 * Chances: a 32-bit draw x meets p percent iff x * 100 < p * 2^32.
 */
typedef struct hase_env_spec {
    uint16_t height, width;
    uint8_t n_agents, n_seekers, view_radius, n_channels;
    uint8_t wall_pct, flags;
    uint16_t episode_len;
    uint8_t water_pct, mud_pct, stuck_pct;
    uint8_t speed_pct[9];
    uint64_t agent_classes;
} hase_env_spec;

/*
 * A batch: n_envs environments. specs points to n_specs host entries:
 * n_specs == 1 broadcasts one spec (uniform batch), n_specs == n_envs gives
 * every env its own spec (uneven batch). Env e's generator id is
 * env_id_base + e (so shards of one logical batch reproduce it exactly).
 */
typedef struct hase_batch_desc {
    uint32_t n_envs;
    const hase_env_spec *specs;
    uint32_t n_specs;
    uint32_t env_id_base;
} hase_batch_desc;

/*
 * Sizes of a batch. Per step the outputs are
 *   obs   obs_words_per_step uint32: env e's [n][C*w + b] block (w =
 *         ceil((2r+1)^2 / 32), b = 1 for HASE_RADIO envs, else 0) starts at
 *         word obs_off[e] (hase_get_offsets); for agent i, channel c the
 *         window bit k = (dy+r)(2r+1) + (dx+r) is bit (k & 31) of word
 *         i*(C*w + b) + c*w + (k >> 5); unused bits are 0; a radio env's
 *         agent i has its belief word at i*(C*w + 1) + C*w.
 *         Channels: 0 blocking tile or outside the map, 1 another agent of the
 *         same role, 2 an agent of the other role, 3 outside the map.
 *   rew   agents_total float32: env e's agents start at agent_off[e]
 *   done  n_envs uint8: bit 0 terminated, bit 1 truncated
 *   map   (hase_step_maps only) map_words_per_step uint32: the discovery map
 *         of every HASE_EXPLORE env after the step (other envs take no
 *         words), env e's at word map_off[e] (hase_get_map_offsets): H rows
 *         of ceil(W/32) words, cell (x, y) at bit x & 31 of word
 *         y * ceil(W/32) + x / 32, bits past W are 0
 * and external actions are agents_total int8 per step.
 * state_bytes is the device buffer hase_create needs; cells_total the
 * number of grid cells (walls array of the host state).
 */
typedef struct hase_layout {
    uint64_t state_bytes;
    uint64_t obs_words_per_step;
    uint64_t agents_total;
    uint64_t n_envs;
    uint64_t cells_total;
    uint64_t map_words_per_step;
} hase_layout;

/*
 * Host-side state of a batch (checkpoint / test loading). All arrays are
 * host memory owned by the caller, sized from hase_layout:
 *   walls    [cells_total] uint8, env e's H*W cells row-major: 1 = blocking,
 *            0 = open; HASE_TERRAIN envs: the tile type, 0 ground, 1 wall,
 *            2 water, 3 mud (set_state rejects other values: HASE_ESTATE)
 *   pos_x/y  [agents_total] uint8 (x < W, y < H)
 *   found    [n_envs] hiders found this episode (bit i = agent i)
 *   t        [n_envs] steps elapsed in the episode
 *   episode  [n_envs] episode index since the reset
 *   steps    [n_envs] step calls since the reset (the generator's step key)
 *   seed     [n_envs] generator seed
 *   stuck    [n_envs] bit i: agent i is stuck (HASE_TERRAIN envs); may be
 *            NULL: get_state skips it and set_state clears it
 *   discovered [map_words_per_step] discovery maps of the HASE_EXPLORE envs
 *            (the map layout above); may be NULL: get_state then skips the
 *            maps and set_state clears every map; set_state rejects a map
 *            with bits past the width (HASE_ESTATE)
 *   belief   [agents_total] radio beliefs (HASE_RADIO envs: bit h = hider h
 *            known; other envs 0); may be NULL: get_state skips it and
 *            set_state clears it; set_state rejects bits that are not hiders
 *            of a radio env (HASE_ESTATE)
 * Env ids are not part of the state: they come from the batch descriptor.
 */
typedef struct hase_host_state {
    uint8_t *walls;
    uint8_t *pos_x, *pos_y;
    uint32_t *found, *t, *episode, *steps;
    uint64_t *seed;
    uint32_t *discovered;
    uint32_t *stuck;
    uint32_t *belief;
} hase_host_state;

typedef struct hase_batch hase_batch;

/* Fill *out for the batch; validates every spec. */
int hase_query_layout(const hase_batch_desc *desc, hase_layout *out);

/*
 * Create a handle over caller memory d_state (>= layout.state_bytes device
 * bytes, 256-byte aligned) on stream (a hipStream_t, or NULL for the null
 * stream). Uploads the per-env tables (synchronously). The envs are not usable
 * until hase_reset or hase_set_state.
 */
int hase_create(const hase_batch_desc *desc, void *d_state, uint64_t state_bytes,
                void *stream, hase_batch **out);

/* Copy the per-env output offsets (words / agents) into host arrays [n_envs]. */
int hase_get_offsets(const hase_batch *b, uint64_t *h_obs_off, uint64_t *h_agent_off);

/* First map word of every env in one step's map output (hase_step_maps) and
 * in the state's discovered array; envs without HASE_EXPLORE take 0 words.
 * h_map_off: [n_envs] host array. */
int hase_get_map_offsets(const hase_batch *b, uint64_t *h_map_off);

/*
 * reset(seed) of every env (Sec. 3.3 desynchronised start, Sec. 4.2 grid):
 * walls (terrain: tile types) from the generator, free-cell check (HASE_EGRID
 * names the first env with fewer free cells than agents, or with terrain,
 * fewer than n cells some agent's class may stand on), agents spawned,
 * counters, stuck agents, discovery maps and beliefs cleared, desync offset
 * drawn;
 * writes the first observation to d_obs0
 * (obs_words_per_step words; may be NULL). Synchronises the stream.
 */
int hase_reset(hase_batch *b, uint64_t seed, uint32_t *d_obs0);

/*
 * n_steps >= 1 consecutive steps of every env (the step loop of Sec. 4.1):
 * actions, moves, detection and rewards, termination/truncation, same-step
 * auto-reset, observation of the resulting state.
 *   d_actions  NULL (every action drawn from the generator) or
 *              [n_steps][agents_total] int8; -1 = draw, 0 stay, 1 N (y-1),
 *              2 S (y+1), 3 E (x+1), 4 W (x-1), anything else = stay
 *              (HASE_RADIO envs: move and radio target packed, see there)
 *   d_obs      [n_steps][obs_words_per_step] uint32
 *   d_rew      [n_steps][agents_total] float32
 *   d_done     [n_steps][n_envs] uint8
 *   mode       HASE_STEP_PERSISTENT or HASE_STEP_PER_LAUNCH (identical results)
 * Enqueued on the stream; output buffers must not overlap the state. A
 * persistent call runs all n_steps inside one kernel launch per variant
 * group: a batch with one group launches its kernel directly; with several,
 * the call replays a captured graph whose groups sit on parallel branches
 * and run concurrently.
 */
int hase_step(hase_batch *b, uint32_t n_steps, const int8_t *d_actions, uint32_t *d_obs,
              float *d_rew, uint8_t *d_done, uint32_t mode);

/*
 * hase_step plus the centralised observation of HASE_EXPLORE envs:
 *   d_map  [n_steps][map_words_per_step] uint32 (the map layout of
 *          hase_layout), the discovery maps after each step; NULL = no map
 *          output (then identical to hase_step)
 * Same argument rules and launch behaviour as hase_step.
 */
int hase_step_maps(hase_batch *b, uint32_t n_steps, const int8_t *d_actions, uint32_t *d_obs,
                   float *d_rew, uint8_t *d_done, uint32_t *d_map, uint32_t mode);

/*
 * Every output of a step call (observability modes of Sec. 3.3: the
 * decentralised windows alone, or with the centralised discovery map, each
 * with or without the omniscient true state):
 *   obs, rew, done  as for hase_step (required)
 *   map        as for hase_step_maps, or NULL
 *   pos        [n_steps][agents_total] uint16, or NULL: every agent's cell
 *              x | y << 8 after the step (after a same-step auto-reset: the
 *              respawned cell), agent i of env e at agent_off[e] + i
 *   env_state  [n_steps][n_envs][4] uint32, or NULL: per env after the step
 *              found (bit h: hider h found this episode), t (steps elapsed in
 *              the episode), episode (episodes ended since the reset) and
 *              stuck (bit i: agent i stuck; terrain envs, else 0); the same
 *              values hase_get_state returns, row by row
 * The true state is the state the next step starts from; with the
 * observations it is what a centralised critic or the with-true-state
 * observability modes read.
 */
typedef struct hase_outputs {
    uint32_t *obs;
    float *rew;
    uint8_t *done;
    uint32_t *map;
    uint16_t *pos;
    uint32_t *env_state;
} hase_outputs;

/* hase_step with any subset of the optional outputs (same argument rules,
 * launch behaviour and results; hase_step and hase_step_maps are this call
 * with pos and env_state NULL). */
int hase_step_outputs(hase_batch *b, uint32_t n_steps, const int8_t *d_actions,
                      const hase_outputs *out, uint32_t mode);

/*
 * Capture (if not cached) the persistent step graph for exactly these
 * arguments without launching it, so a later persistent hase_step (or
 * hase_step_maps, with the same d_map) only replays it: no capture cost on
 * the critical path (a batch with one variant group needs no graph: then
 * only the arguments are checked). Same argument rules as hase_step;
 * enqueues nothing.
 */
int hase_prepare(hase_batch *b, uint32_t n_steps, const int8_t *d_actions, uint32_t *d_obs,
                 float *d_rew, uint8_t *d_done);
int hase_prepare_maps(hase_batch *b, uint32_t n_steps, const int8_t *d_actions, uint32_t *d_obs,
                      float *d_rew, uint8_t *d_done, uint32_t *d_map);
int hase_prepare_outputs(hase_batch *b, uint32_t n_steps, const int8_t *d_actions,
                         const hase_outputs *out);

/* Observation of the current state (e.g. after hase_set_state); enqueued. */
int hase_observe(hase_batch *b, uint32_t *d_obs);

/* Download / upload the full state (synchronises). set_state validates
 * positions (inside the map), tile values and, as hase_reset does for the
 * grids it draws, that every env has room for its agents (at least n cells
 * that each agent's class may stand on, else HASE_EGRID naming the first such
 * env, and nothing is uploaded), then rebuilds the device-side bitboards. */
int hase_get_state(hase_batch *b, const hase_host_state *out);
int hase_set_state(hase_batch *b, const hase_host_state *in);

/*
 * Tiling of the step kernel: lanes_per_env in {1,2,4,8,16} lanes of one
 * 64-lane wavefront cooperate on one env, so a wave steps 64/lanes_per_env
 * envs. lanes[v] applies to the envs whose agent count falls in bucket v:
 * v = 0 for n <= 2, 1 for n <= 4, 2 for n <= 10, 3 for n <= 20. 0 takes the
 * default: 4, 4, 16, 16 lanes, except that when the buckets with the widest
 * of those hold at least half of the batch's agents, every bucket present
 * takes the widest (one launch group); hase_create starts from the
 * default. Plain envs whose buckets take 4 and 16 lanes share one launch,
 * in which the envs of bucket 2 with at most 8 agents run at 8 lanes per env
 * (one agent per lane) while bucket 2 reads 16. Results never depend on the
 * tiling. Rebuilds the tile table (synchronously) and drops cached graphs.
 */
#define HASE_N_BUCKETS 4
int hase_set_tiling(hase_batch *b, const uint32_t lanes[HASE_N_BUCKETS]);
int hase_get_tiling(const hase_batch *b, uint32_t lanes[HASE_N_BUCKETS]);

/*
 * Autotuner of the tiling: coordinate descent over lanes_per_env of every
 * agent-count bucket present in the batch, timing persistent calls of
 * n_steps (HIP events on the handle's stream; the median of 5 runs per
 * candidate, which replaces the best only when more than 2% faster) into the
 * caller's scratch outputs (sized as for hase_step with n_steps). The state is snapshotted
 * and restored, so tuning does not advance the envs, and results never depend
 * on the tiling. Applies the fastest tiling found and copies it to lanes_out
 * (may be NULL). Synchronises the stream.
 */
int hase_autotune(hase_batch *b, uint32_t n_steps, uint32_t *d_obs, float *d_rew, uint8_t *d_done,
                  uint32_t lanes_out[HASE_N_BUCKETS]);

/*
 * Serving: several batches (one per request, each with its own state) stepped
 * together, one launch per lanes-per-env value across all of them. Request i
 * takes io[i].n_steps <= n_steps steps; its outputs (and optional actions)
 * are indexed by output step io[i].out_step0 + k in its own buffers, laid out
 * as for hase_step, and d_map (may be NULL) as for hase_step_maps. Handles
 * must be distinct and not in use elsewhere; the
 * work is enqueued on `stream` (a hipStream_t): with more than one lanes
 * value the launches run concurrently on side streams of io[0].batch,
 * forked from and joined back into `stream`. d_workspace is caller device
 * memory of hase_multi_workspace bytes (job and tile tables), which must stay
 * untouched until the launch completes.
 */
typedef struct hase_step_io {
    hase_batch *batch;
    uint32_t n_steps;
    uint32_t out_step0;
    const int8_t *d_actions;
    uint32_t *d_obs;
    float *d_rew;
    uint8_t *d_done;
    uint32_t *d_map;
} hase_step_io;

int hase_multi_workspace(hase_batch *const *batches, uint32_t n, uint64_t *bytes);
int hase_step_multi(const hase_step_io *io, uint32_t n, uint32_t n_steps, void *d_workspace,
                    uint64_t workspace_bytes, void *stream);

/*
 * Arena: resident env slots for serving (continuous batching). An arena of
 * n_slots slots, each with room for one env of at most max_height x
 * max_width cells and max_agents agents, lives in one caller buffer of
 * hase_query_arena bytes. A request is admitted into a range of free slots
 * with hase_reset_range, stepped with every other admitted range by
 * hase_step_resident, and leaves with hase_release_range; all three only
 * enqueue work on the arena's stream (no host synchronisation), so the
 * admission of one request overlaps the steps of the others. max_ranges
 * bounds the ranges admitted at once.
 */
typedef struct hase_arena_desc {
    uint32_t n_slots;
    uint16_t max_height, max_width;
    uint8_t max_agents;
    uint32_t max_ranges;
} hase_arena_desc;

/* A range's own output buffers (caller device memory, laid out as the
 * outputs of a uniform batch of `count` envs of the range's spec, env i of
 * the range at the place of env i):
 *   obs   [step_budget][count * n * (C * w + b)] uint32
 *   rew   [step_budget][count * n] float32
 *   done  [step_budget][count] uint8
 *   map   [step_budget][count * H * ceil(W/32)] uint32, or NULL (exploring
 *         specs only; NULL: no map output)
 *   obs0  [count * n * (C * w + b)] uint32: the observation after the
 *         reset, or NULL
 *   err   one uint32 in device or pinned host memory, or NULL: written in
 *         stream order after the reset, 0xffffffff when every env of the
 *         range had room for its agents, else the index within the range of
 *         the first env that had not (as hase_range_error, without a host
 *         synchronisation)
 *   pos, env_state  the true state after each step (hase_outputs), laid out
 *         for the range's count envs, or NULL
 * Row k of obs, rew, done, map, pos and env_state is the range's k-th step
 * since its reset. */
typedef struct hase_out_ptrs {
    uint32_t *obs;
    float *rew;
    uint8_t *done;
    uint32_t *map;
    uint32_t *obs0;
    uint32_t *err;
    uint16_t *pos;
    uint32_t *env_state;
} hase_out_ptrs;

/* Device bytes of an arena (validates the descriptor: n_slots >= 1, sides
 * 2..64, max_agents 1..20, max_ranges 1..65536). */
int hase_query_arena(const hase_arena_desc *desc, uint64_t *state_bytes);

/* Create an arena over caller memory d_state (>= hase_query_arena bytes,
 * 256-byte aligned) on stream (a hipStream_t or NULL). Uploads the slot
 * tables (synchronously); every slot starts free. */
int hase_create_arena(const hase_arena_desc *desc, void *d_state, uint64_t state_bytes,
                      void *stream, hase_batch **out);

/*
 * Admit a request into slots [first_slot, first_slot + count), which must lie
 * inside the arena and be free: every env gets `spec` (fitting the arena's
 * caps), generator seed `seed` and env id env_id_base + i for slot
 * first_slot + i, and is reset exactly as hase_reset resets a batch (walls,
 * spawn, desync; Sec. 4.2 resets, Sec. 3.3 desynchronised start), so a
 * range reproduces the batch hase_create + hase_reset would make of it. The
 * range then takes step_budget >= 1 steps through hase_step_resident,
 * writing them to *out (copied; the buffers must stay valid until the range
 * is released), and stops. Enqueued on the arena's stream; nothing
 * synchronises. An env with too few free cells for its agents (HASE_EGRID
 * at hase_reset) does not fail the call: hase_range_error reports it, and
 * the range's outputs are then meaningless. Errors (synchronous, before any
 * work): HASE_EINVAL for a bad spec, a spec beyond the caps, slots outside
 * the arena or taken, a zero budget, null output buffers, no free range.
 */
int hase_reset_range(hase_batch *arena, uint32_t first_slot, uint32_t count,
                     const hase_env_spec *spec, uint64_t seed, uint32_t env_id_base,
                     uint32_t step_budget, const hase_out_ptrs *out);

/* Every admitted range takes min(n_steps, steps left of its budget) steps
 * (the step of hase_step, persistent: one kernel launch per group of ranges
 * with the same env kind and lanes per env, groups concurrent). Enqueued. */
int hase_step_resident(hase_batch *arena, uint32_t n_steps);

/* Release the range starting at first_slot: its slots are free for another
 * hase_reset_range, and later steps leave it alone (enqueued, in stream
 * order after the steps before it). */
int hase_release_range(hase_batch *arena, uint32_t first_slot);

/* The range's reset check (synchronises the stream): *bad_env = -1 when every
 * env had room for its agents, else the first env (index within the range)
 * that had not. */
int hase_range_error(hase_batch *arena, uint32_t first_slot, int64_t *bad_env);

/*
 * hase_step_multi without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation). Same arguments, results and launch
 * behaviour as hase_step_multi; the job and tile tables go to a static
 * device array of the library, HASE_STATIC_WORKSPACE_BYTES per GPU, held by
 * every GPU the library runs on until the process ends. A call needing more
 * (hase_multi_workspace) returns HASE_ENOMEM before any work is enqueued.
 * The call allocates nothing. Every call on one GPU shares that GPU's array,
 * which keeps the last call's tables: calls that overlap on one GPU (other
 * streams, other host threads) race, so the caller serialises them (e.g.
 * one stream, or an event between them).
 */
#define HASE_STATIC_WORKSPACE_BYTES (1u << 20)
int hase_step_multi_static(const hase_step_io *io, uint32_t n, uint32_t n_steps, void *stream);

/* Release the handle (never frees caller memory). */
int hase_destroy(hase_batch *b);

const char *hase_strerror(int code);
const char *hase_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HASE_H */
