// Host runtime of the hide-and-seek step: the C ABI declared in include/hase.h.
//
// Owns no device memory: every device byte (state, inputs, outputs) comes
// from the caller. The state buffer is carved into structure-of-arrays regions
// (256-byte aligned): per-env spec words, output offsets, generator keys and
// counters, agent positions, canonical walls, padded wall bitboards, the
// discovery maps of exploring envs, the tile table and an error word. The step runs as one launch per tile variant; a
// persistent call is captured once into a hipGraph (variants as concurrent
// branches) keyed by its arguments and replayed afterwards.

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <list>
#include <map>
#include <string>
#include <vector>

#include "../../include/hase.h"
#include "hase_internal.h"

using namespace hase;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(HASE_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                                \
    do {                                                             \
        hipError_t _e = (call);                                      \
        if (_e != hipSuccess) return hip_fail(_e, #call);            \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int words_per_channel(int r)
{
    const int d = 2 * r + 1;
    return (d * d + 31) / 32;
}

int bucket_of(int n)
{
    for (int b = 0; b < N_BUCKETS; ++b)
        if (n <= BUCKET_NMAX[b]) return b;
    return N_BUCKETS - 1;
}

// Built-in lanes per env for each agent-count bucket (overridable by the tiler).
const uint32_t DEFAULT_LANES[N_BUCKETS] = {4, 4, 16, 16};

// Default tiling of a batch: the built-in lanes per bucket. A batch of plain
// envs only keeps them (its 4- and 16-lane envs share one combined launch);
// otherwise, when the buckets with the widest built-in lanes hold at least
// half of the batch's agents, every bucket takes those lanes, so the whole
// batch is one launch group (one kernel keeps all SIMDs busy to the end,
// instead of two groups finishing at different times).
void default_lanes(const std::vector<hase_env_spec> &specs, uint32_t out[N_BUCKETS])
{
    bool all_plain = true;
    for (const hase_env_spec &s : specs) all_plain = all_plain && env_kind(s.flags) == KIND_PLAIN;
    if (all_plain) {
        for (int bk = 0; bk < N_BUCKETS; ++bk) out[bk] = DEFAULT_LANES[bk];
        return;
    }
    uint64_t agents[N_BUCKETS] = {}, total = 0;
    for (const hase_env_spec &s : specs) {
        agents[bucket_of(s.n_agents)] += s.n_agents;
        total += s.n_agents;
    }
    uint32_t widest = 0;
    for (int bk = 0; bk < N_BUCKETS; ++bk)
        if (agents[bk]) widest = std::max(widest, DEFAULT_LANES[bk]);
    uint64_t in_widest = 0;
    for (int bk = 0; bk < N_BUCKETS; ++bk)
        if (agents[bk] && DEFAULT_LANES[bk] == widest) in_widest += agents[bk];
    const bool one_group = 2 * in_widest >= total;
    for (int bk = 0; bk < N_BUCKETS; ++bk)
        out[bk] = (one_group && agents[bk]) ? widest : DEFAULT_LANES[bk];
}

int check_spec(const hase_env_spec &s, uint32_t idx)
{
    if (s.height < 2 || s.height > MAX_SIDE || s.width < 2 || s.width > MAX_SIDE)
        return fail(HASE_EINVAL, "spec %u: height/width must be in 2..%d", idx, MAX_SIDE);
    if (s.n_agents < 1 || s.n_agents > MAX_AGENTS)
        return fail(HASE_EINVAL, "spec %u: n_agents must be in 1..%d", idx, MAX_AGENTS);
    if (s.n_seekers > s.n_agents)
        return fail(HASE_EINVAL, "spec %u: n_seekers > n_agents", idx);
    if (s.view_radius < 1 || s.view_radius > PAD)
        return fail(HASE_EINVAL, "spec %u: view_radius must be in 1..%d", idx, PAD);
    if (s.n_channels != 3 && s.n_channels != 4)
        return fail(HASE_EINVAL, "spec %u: n_channels must be 3 or 4", idx);
    if (s.wall_pct > 99) return fail(HASE_EINVAL, "spec %u: wall_pct must be <= 99", idx);
    if (s.flags & ~127u) return fail(HASE_EINVAL, "spec %u: unknown flag bits", idx);
    if (s.episode_len < 1) return fail(HASE_EINVAL, "spec %u: episode_len must be >= 1", idx);
    if (s.flags & HASE_TERRAIN) {
        if ((int)s.wall_pct + s.water_pct + s.mud_pct > 99)
            return fail(HASE_EINVAL, "spec %u: wall_pct + water_pct + mud_pct must be <= 99", idx);
        if (s.stuck_pct > 100) return fail(HASE_EINVAL, "spec %u: stuck_pct must be <= 100", idx);
        for (int k = 0; k < 9; ++k)
            if (s.speed_pct[k] > 100) return fail(HASE_EINVAL, "spec %u: speed_pct must be <= 100", idx);
        for (int i = 0; i < 32; ++i) {
            const uint32_t c = (uint32_t)(s.agent_classes >> (2 * i)) & 3u;
            if (c == 3u || (i >= s.n_agents && c != 0u))
                return fail(HASE_EINVAL, "spec %u: agent %d has an invalid class", idx, i);
        }
    }
    return HASE_OK;
}

struct Regions {
    size_t perm, spec0, spec1, spec2, obs_off, agent_off, bb_off, grid_off, env_id, map_off, terr;
    size_t seed, found, t, ep, steps, stuck, bel, pos, walls, bb, disc, tiles, err;
    size_t jobs, job_err;  // arenas only: the ranges' job descriptors and error words
    size_t total;
};

struct Plan {
    std::vector<hase_env_spec> specs;
    std::vector<uint32_t> obs_off, agent_off, grid_off, bb_off, map_off;
    uint64_t obs_words = 0, agents = 0, cells = 0, bb_words = 0, map_words = 0;
    size_t max_tiles = 0;
    Regions reg{};
};

int make_plan(const hase_batch_desc *d, Plan &p)
{
    if (!d) return fail(HASE_EINVAL, "null batch descriptor");
    if (d->n_envs == 0) return fail(HASE_EINVAL, "n_envs must be >= 1");
    if (!d->specs || (d->n_specs != 1 && d->n_specs != d->n_envs))
        return fail(HASE_EINVAL, "n_specs must be 1 or n_envs (got %u for %u envs)", d->n_specs,
                    d->n_envs);
    const uint32_t N = d->n_envs;
    p.specs.resize(N);
    for (uint32_t e = 0; e < N; ++e) {
        const hase_env_spec &s = d->specs[d->n_specs == 1 ? 0 : e];
        if (d->n_specs != 1 || e == 0) {
            const int rc = check_spec(s, e);
            if (rc) return rc;
        }
        p.specs[e] = s;
    }
    p.obs_off.resize(N);
    p.agent_off.resize(N);
    p.grid_off.resize(N);
    p.bb_off.resize(N);
    p.map_off.resize(N);
    for (uint32_t e = 0; e < N; ++e) {
        const hase_env_spec &s = p.specs[e];
        p.obs_off[e] = (uint32_t)p.obs_words;
        p.agent_off[e] = (uint32_t)p.agents;
        p.grid_off[e] = (uint32_t)p.cells;
        p.bb_off[e] = (uint32_t)p.bb_words;
        p.map_off[e] = (uint32_t)p.map_words;
        // radio envs: one belief word after each agent's channels
        p.obs_words += (uint64_t)s.n_agents *
                       (s.n_channels * words_per_channel(s.view_radius) + ((s.flags & HASE_RADIO) ? 1 : 0));
        p.agents += s.n_agents;
        p.cells += (uint64_t)s.height * s.width;
        // terrain envs keep two board planes (tile types)
        p.bb_words += (uint64_t)board_words(s.height, (s.flags & HASE_TERRAIN) ? 2 : 1);
        if (s.flags & HASE_EXPLORE) p.map_words += (uint64_t)map_words(s.height, s.width);
    }
    if (p.obs_words >= (1ull << 32) || p.cells >= (1ull << 32) || p.bb_words >= (1ull << 32) ||
        p.map_words >= (1ull << 32))
        return fail(HASE_EINVAL, "batch too large: per-step offsets exceed 32 bits");
    if ((uint64_t)N + 64 >= (1ull << 32)) return fail(HASE_EINVAL, "too many envs");
    p.max_tiles = (size_t)N + (size_t)MAX_VARIANTS * N_KINDS;
    Regions &r = p.reg;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    r.perm = take(4ull * N);
    r.spec0 = take(4ull * N);
    r.spec1 = take(4ull * N);
    r.spec2 = take(4ull * N);
    r.obs_off = take(4ull * N);
    r.agent_off = take(4ull * N);
    r.bb_off = take(4ull * N);
    r.grid_off = take(4ull * N);
    r.env_id = take(4ull * N);
    r.map_off = take(4ull * N);
    r.terr = take(32ull * N);
    r.seed = take(8ull * N);
    r.found = take(4ull * N);
    r.t = take(4ull * N);
    r.ep = take(4ull * N);
    r.steps = take(4ull * N);
    r.stuck = take(4ull * N);
    r.bel = take(4ull * p.agents);
    r.pos = take(2ull * p.agents);
    r.walls = take(p.cells);
    r.bb = take(4ull * p.bb_words);
    r.disc = take(4ull * p.map_words);
    r.tiles = take(sizeof(Tile) * p.max_tiles);
    r.err = take(16);
    r.total = off;
    return HASE_OK;
}

// One kernel launch of a step call: a single (bucket, radius) variant, or
// (mixed) every variant sharing `lanes`, over contiguous tiles of envs of one
// kind (plain, exploration, line of sight).
struct Variant {
    int lanes = 0, nmax = 0, r = 0, kind = KIND_PLAIN;
    // mixed: the per-tile variant switch (the feature kinds have only that
    // kernel); xpl: an env explores (LDS discovery maps of map_words); big:
    // the bucket of up to 20 agents, whose mixed kernel is its own; combo:
    // the combined launch of plain envs at 4, 8 and 16 lanes
    bool mixed = false, xpl = false, big = false, combo = false;
    uint32_t tile0 = 0, n_tiles = 0, slot_words = 0, map_words = 0;
};

// lanes x kinds x (big or not) launches at most, plus the combined one,
// each on its own stream when forked
constexpr int MAX_LAUNCHES = 5 * N_KINDS * 2 + 1;

struct GraphEntry {
    uint32_t n_steps;
    const void *act, *obs, *rew, *done, *map, *spos, *senv;
    hipGraphExec_t exec;
};

}  // namespace

struct hase_batch {
    Plan plan;
    uint32_t n_envs = 0, env_id_base = 0;
    char *d = nullptr;  // caller's state buffer
    hipStream_t stream = nullptr;
    bool ready = false;
    uint32_t lanes[N_BUCKETS];
    std::vector<Variant> variants;
    std::vector<Tile> host_tiles;  // host copy of the device tile table
    hipStream_t side[MAX_LAUNCHES] = {};
    hipEvent_t fork_ev = nullptr, join_ev[MAX_LAUNCHES] = {};
    std::list<GraphEntry> graphs;  // most recently used first

    // arena (hase_create_arena): n_envs slots of capacity cap_h x cap_w
    // cells and cap_n agents; ranges of slots admitted by hase_reset_range
    struct Range {
        uint32_t count, job, kind, lanes, n_tiles, slot_words, map_words;
        bool big, mid;  // mid: 8-lane tiles of the combined kernel
    };
    bool arena = false;
    uint32_t cap_h = 0, cap_w = 0, cap_n = 0;
    std::map<uint32_t, Range> ranges;  // by first slot
    std::vector<uint32_t> free_jobs;

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(d + off); }

    EnvTables tables() const
    {
        const Regions &r = plan.reg;
        EnvTables t;
        t.perm = at<uint32_t>(r.perm);
        t.spec0 = at<uint32_t>(r.spec0);
        t.spec1 = at<uint32_t>(r.spec1);
        t.spec2 = at<uint32_t>(r.spec2);
        t.obs_off = at<uint32_t>(r.obs_off);
        t.agent_off = at<uint32_t>(r.agent_off);
        t.bb_off = at<uint32_t>(r.bb_off);
        t.grid_off = at<uint32_t>(r.grid_off);
        t.env_id = at<uint32_t>(r.env_id);
        t.map_off = at<uint32_t>(r.map_off);
        t.terr = at<uint32_t>(r.terr);
        return t;
    }
};

namespace {

// Launch group of an arena range's tiles (bits 8 and up of their variant):
// the kernel's group code, plus bit 17 for the 8-lane tiles that the
// combined kernel runs.
uint32_t arena_group(int kind, int lanes, bool big, bool mid)
{
    return group_code(kind, lanes, big) | (mid ? 1u << 17 : 0u);
}

void drop_graphs(hase_batch *b)
{
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

// Group envs by (kind, agent-count bucket, view radius) -- one kernel variant
// each --, keep env order inside a group (neighbouring envs write neighbouring
// outputs: sorting a group by agent count and area cost 8% more HBM write
// traffic on uneven batches for no speed), and cut it into tiles of
// 64 / lanes envs. Variants that share a (lanes, kind) run as one mixed
// launch, so all buckets of an uneven batch share the chip.
int build_tiles(hase_batch *b)
{
    const Plan &p = b->plan;
    const uint32_t N = b->n_envs;
    std::vector<uint32_t> perm;
    perm.reserve(N);
    std::vector<Tile> tiles;
    std::vector<Variant> vars;
    // plain envs whose bucket takes 4 lanes (up to 4 agents) or 16 (up to 10)
    // go to one launch when both widths occur or when some of them have 5 to
    // COMBO_MID_NMAX agents: those take 8 lanes there, one agent per lane, so
    // a wave holds 8 of them instead of 4 (half the waves at equal time per
    // wave)
    auto in_combo = [&](int bk) {
        return bk < N_BUCKETS - 1 && ((b->lanes[bk] == 4 && bk <= 1) || b->lanes[bk] == 16);
    };
    auto combo_width = [&](const hase_env_spec &s) -> uint32_t {
        const int bk = bucket_of(s.n_agents);
        if (b->lanes[bk] == 4) return 4;
        return (bk == 2 && s.n_agents <= COMBO_MID_NMAX) ? 8 : 16;
    };
    bool has4 = false, has8 = false, has16 = false;
    for (const hase_env_spec &s : p.specs) {
        if (env_kind(s.flags) != KIND_PLAIN || !in_combo(bucket_of(s.n_agents))) continue;
        const uint32_t w = combo_width(s);
        (w == 4 ? has4 : w == 8 ? has8 : has16) = true;
    }
    const bool combo = has8 || (has4 && has16);
    if (combo) {
        Variant grp;
        grp.lanes = 4;  // LDS of 16 env slots per wave
        grp.kind = KIND_PLAIN;
        grp.mixed = grp.combo = true;
        grp.tile0 = (uint32_t)tiles.size();
        for (uint32_t L : {4u, 8u, 16u}) {
            for (int bk = 0; bk < N_BUCKETS; ++bk) {
                if (!in_combo(bk)) continue;
                for (int r = 1; r <= PAD; ++r) {
                    const uint32_t base = (uint32_t)perm.size();
                    for (uint32_t e = 0; e < N; ++e) {
                        const hase_env_spec &s = p.specs[e];
                        if (bucket_of(s.n_agents) == bk && s.view_radius == r &&
                            env_kind(s.flags) == KIND_PLAIN && combo_width(s) == L) {
                            perm.push_back(e);
                            grp.slot_words = std::max(grp.slot_words, (uint32_t)board_words(s.height, 1));
                        }
                    }
                    const uint32_t cnt = (uint32_t)perm.size() - base, E = 64u / L;
                    const uint32_t width_bits = L == 16 ? COMBO_WIDE : L == 8 ? COMBO_MID : 0u;
                    for (uint32_t i = 0; i < cnt; i += E) {
                        Tile t;
                        t.job = 0;
                        t.env0 = base + i;
                        t.count = std::min<uint32_t>(E, cnt - i);
                        t.variant = (uint32_t)(bk * 4 + r - 1) | width_bits;
                        tiles.push_back(t);
                    }
                }
            }
        }
        grp.n_tiles = (uint32_t)tiles.size() - grp.tile0;
        if (combo_lds_bytes(grp.slot_words) > 65536)
            return fail(HASE_EINVAL, "tiling: the combined launch needs more than 64 KiB of LDS per wave");
        vars.push_back(grp);
    }
    const uint32_t lane_order[] = {1, 2, 4, 8, 16};
    for (uint32_t L : lane_order) {
        for (int kb = 0; kb < 2 * N_KINDS; ++kb) {
            const int kind = kb >> 1;
            const bool big = (kb & 1) != 0;
            Variant grp;
            grp.lanes = (int)L;
            grp.kind = kind;
            grp.big = big;
            grp.tile0 = (uint32_t)tiles.size();
            int n_var = 0;
            for (int bk = 0; bk < N_BUCKETS; ++bk) {
                if (b->lanes[bk] != L || (bk == N_BUCKETS - 1) != big) continue;
                if (combo && kind == KIND_PLAIN && in_combo(bk)) continue;
                for (int r = 1; r <= PAD; ++r) {
                    std::vector<uint32_t> ids;
                    for (uint32_t e = 0; e < N; ++e) {
                        const hase_env_spec &s = p.specs[e];
                        if (bucket_of(s.n_agents) == bk && s.view_radius == r &&
                            env_kind(s.flags) == kind)
                            ids.push_back(e);
                    }
                    if (ids.empty()) continue;
                    const uint32_t E = 64u / L;
                    const uint32_t base = (uint32_t)perm.size();
                    for (uint32_t e : ids) {
                        perm.push_back(e);
                        // LDS slots of whole 16-byte units (boards, respawn
                        // words, discovery map)
                        if (p.specs[e].flags & HASE_EXPLORE) {
                            grp.xpl = true;
                            grp.map_words = std::max(
                                grp.map_words, (uint32_t)round4(lds_board_words(p.specs[e].height)));
                        }
                        // terrain: two tile planes
                        const int planes = (p.specs[e].flags & HASE_TERRAIN) ? 2 : 1;
                        grp.slot_words = std::max(
                            grp.slot_words, (uint32_t)board_words(p.specs[e].height, planes));
                    }
                    for (uint32_t i = 0; i < ids.size(); i += E) {
                        Tile t;
                        t.job = 0;
                        t.env0 = base + i;
                        t.count = std::min<uint32_t>(E, (uint32_t)ids.size() - i);
                        t.variant = (uint32_t)(bk * 4 + r - 1);
                        tiles.push_back(t);
                    }
                    grp.nmax = BUCKET_NMAX[bk];
                    grp.r = r;
                    ++n_var;
                }
            }
            if (n_var == 0) continue;
            grp.mixed = n_var > 1 || kind != KIND_PLAIN;
            grp.n_tiles = (uint32_t)tiles.size() - grp.tile0;
            const size_t lds_bytes =
                (size_t)(64u / L) * (grp.slot_words + MAX_AGENTS + grp.map_words) * 4;
            if (lds_bytes > 65536)
                return fail(HASE_EINVAL, "tiling: %u lanes/env needs %zu bytes of LDS per wave", L,
                            lds_bytes);
            vars.push_back(grp);
        }
    }
    if (tiles.size() > p.max_tiles) return fail(HASE_EINVAL, "tile table overflow");
    HIP_TRY(hipMemcpyAsync(b->d + p.reg.perm, perm.data(), 4 * perm.size(), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipMemcpyAsync(b->d + p.reg.tiles, tiles.data(), sizeof(Tile) * tiles.size(),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->variants = vars;
    b->host_tiles = tiles;
    drop_graphs(b);
    return HASE_OK;
}

JobDesc make_job(const hase_batch *b, const int8_t *act, uint32_t *obs, float *rew, uint8_t *done,
                 uint32_t *map = nullptr)
{
    const Regions &r = b->plan.reg;
    JobDesc j;
    j.tab = b->tables();
    j.seed = b->at<uint64_t>(r.seed);
    j.found = b->at<uint32_t>(r.found);
    j.t = b->at<uint32_t>(r.t);
    j.ep = b->at<uint32_t>(r.ep);
    j.steps = b->at<uint32_t>(r.steps);
    j.pos = b->at<uint16_t>(r.pos);
    j.bb = b->at<uint32_t>(r.bb);
    j.obs = obs;
    j.rew = rew;
    j.done = done;
    j.act = act;
    j.obs_stride = b->plan.obs_words;
    j.agent_stride = b->plan.agents;
    j.env_stride = b->n_envs;
    j.k_limit = 0xffffffffu;
    j.out_step0 = 0;
    j.disc = b->at<uint32_t>(r.disc);
    j.stuck = b->at<uint32_t>(r.stuck);
    j.bel = b->at<uint32_t>(r.bel);
    j.map = map;
    j.map_stride = b->plan.map_words;
    j.spos = nullptr;
    j.senv = nullptr;
    j.resident = 0;
    j.first = j.budget = j.obs_env = j.map_env = 0;
    j.group = ALL_GROUPS;
    return j;
}

// Enqueue every variant of one call on `stream`; with `fork`, variants after
// the first run on side streams joined back into `stream` (graph branches).
int enqueue(hase_batch *b, const JobDesc &job, uint32_t K, uint32_t step_base, hipStream_t stream,
            bool fork)
{
    const Tile *tiles = b->at<Tile>(b->plan.reg.tiles);
    // the fork point precedes every launch of the call, so no group waits for
    // another one launched before it
    if (fork && b->variants.size() > 1) HIP_TRY(hipEventRecord(b->fork_ev, stream));
    for (size_t i = 0; i < b->variants.size(); ++i) {
        const Variant &v = b->variants[i];
        hipStream_t s = stream;
        if (fork && i > 0) {
            HIP_TRY(hipStreamWaitEvent(b->side[i], b->fork_ev, 0));
            s = b->side[i];
        }
        if (v.combo)
            HIP_TRY(launch_combo(tiles + v.tile0, v.n_tiles, nullptr, job, K, step_base, v.slot_words, s));
        else if (v.mixed)
            HIP_TRY(launch_mixed(v.lanes, v.kind, tiles + v.tile0, v.n_tiles, nullptr, job, K,
                                 step_base, v.slot_words, v.map_words, v.big, s));
        else
            HIP_TRY(launch_step(v.lanes, v.nmax, v.r, tiles + v.tile0, v.n_tiles, nullptr, job, K,
                                step_base, v.slot_words, s));
        if (fork && i > 0) {
            HIP_TRY(hipEventRecord(b->join_ev[i], s));
            HIP_TRY(hipStreamWaitEvent(stream, b->join_ev[i], 0));
        }
    }
    return HASE_OK;
}

// The fork event and the first `count` side streams (created on first use;
// side stream 0 is also the graph capture stream).
int ensure_streams(hase_batch *b, size_t count)
{
    if (count > (size_t)MAX_LAUNCHES) return fail(HASE_EINVAL, "too many launches (%zu)", count);
    if (!b->fork_ev) HIP_TRY(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
    for (size_t i = 0; i < std::max<size_t>(count, 1); ++i) {
        if (b->side[i]) continue;
        HIP_TRY(hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&b->join_ev[i], hipEventDisableTiming));
    }
    return HASE_OK;
}

// The cached graph for these arguments (captured and instantiated on a miss).
int graph_for(hase_batch *b, const JobDesc &job, uint32_t n_steps, hipGraphExec_t *out)
{
    int rc = ensure_streams(b, b->variants.size());
    if (rc) return rc;
    for (auto it = b->graphs.begin(); it != b->graphs.end(); ++it) {
        if (it->n_steps == n_steps && it->act == job.act && it->obs == job.obs &&
            it->rew == job.rew && it->done == job.done && it->map == job.map &&
            it->spos == job.spos && it->senv == job.senv) {
            b->graphs.splice(b->graphs.begin(), b->graphs, it);
            *out = b->graphs.front().exec;
            return HASE_OK;
        }
    }
    // capture on a private stream (the caller's may be the null stream)
    hipStream_t cap = b->side[0];
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
    rc = enqueue(b, job, n_steps, 0, cap, true);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    GraphEntry g{n_steps, job.act, job.obs, job.rew, job.done, job.map, job.spos, job.senv, exec};
    b->graphs.push_front(g);
    while (b->graphs.size() > 8) {
        (void)hipGraphExecDestroy(b->graphs.back().exec);
        b->graphs.pop_back();
    }
    *out = exec;
    return HASE_OK;
}

// One launch of the whole call. With several variant groups: the captured
// graph (one kernel node per group, groups on parallel branches) replayed on
// the stream. With one group the kernel is launched directly: a graph of one
// node adds only the graph launch's host cost (measured under a runtime
// trace: 32.7 us per hipGraphLaunch against 11.1 us per hipLaunchKernel),
// which a call of a few steps waits for.
int persistent_step(hase_batch *b, const JobDesc &job, uint32_t n_steps)
{
    if (b->variants.size() == 1) return enqueue(b, job, n_steps, 0, b->stream, false);
    hipGraphExec_t exec = nullptr;
    const int rc = graph_for(b, job, n_steps, &exec);
    if (rc) return rc;
    HIP_TRY(hipGraphLaunch(exec, b->stream));
    return HASE_OK;
}

int check_step_args(const hase_batch *b, uint32_t n_steps, const uint32_t *d_obs, const float *d_rew,
                    const uint8_t *d_done)
{
    if (!b) return fail(HASE_EINVAL, "null handle");
    if (b->arena) return fail(HASE_EINVAL, "an arena is stepped by hase_step_resident");
    if (!b->ready) return fail(HASE_ENOTREADY, "step before reset/set_state");
    if (n_steps == 0) return fail(HASE_EINVAL, "n_steps must be >= 1");
    if (!d_obs || !d_rew || !d_done) return fail(HASE_EINVAL, "null output buffer");
    return HASE_OK;
}

InitArgs make_init(const hase_batch *b, uint64_t seed, uint32_t rebuild)
{
    const Regions &r = b->plan.reg;
    InitArgs a;
    a.tab = b->tables();
    a.seed = b->at<uint64_t>(r.seed);
    a.found = b->at<uint32_t>(r.found);
    a.t = b->at<uint32_t>(r.t);
    a.ep = b->at<uint32_t>(r.ep);
    a.steps = b->at<uint32_t>(r.steps);
    a.pos = b->at<uint16_t>(r.pos);
    a.walls = b->at<uint8_t>(r.walls);
    a.bb = b->at<uint32_t>(r.bb);
    a.disc = b->at<uint32_t>(r.disc);
    a.stuck = b->at<uint32_t>(r.stuck);
    a.bel = b->at<uint32_t>(r.bel);
    a.err = b->at<uint32_t>(r.err);
    a.seed_value = seed;
    a.env0 = 0;
    a.n_envs = b->n_envs;
    a.rebuild_only = rebuild;
    return a;
}

// Mutable per-env state (walls and bitboards never change while stepping).
struct Snapshot {
    std::vector<uint16_t> pos;
    std::vector<uint32_t> found, t, ep, steps, stuck, disc, bel;
};

int snapshot_take(hase_batch *b, Snapshot &s)
{
    const Plan &p = b->plan;
    const uint32_t N = b->n_envs;
    s.pos.resize(p.agents);
    s.found.resize(N);
    s.t.resize(N);
    s.ep.resize(N);
    s.steps.resize(N);
    s.stuck.resize(N);
    s.disc.resize(p.map_words);
    s.bel.resize(p.agents);
    auto down = [&](void *dst, size_t off, size_t bytes) {
        return hipMemcpyAsync(dst, b->d + off, bytes, hipMemcpyDeviceToHost, b->stream);
    };
    HIP_TRY(down(s.pos.data(), p.reg.pos, 2 * p.agents));
    HIP_TRY(down(s.found.data(), p.reg.found, 4ull * N));
    HIP_TRY(down(s.t.data(), p.reg.t, 4ull * N));
    HIP_TRY(down(s.ep.data(), p.reg.ep, 4ull * N));
    HIP_TRY(down(s.steps.data(), p.reg.steps, 4ull * N));
    HIP_TRY(down(s.stuck.data(), p.reg.stuck, 4ull * N));
    HIP_TRY(down(s.bel.data(), p.reg.bel, 4ull * p.agents));
    if (p.map_words) HIP_TRY(down(s.disc.data(), p.reg.disc, 4ull * p.map_words));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return HASE_OK;
}

int snapshot_restore(hase_batch *b, const Snapshot &s)
{
    const Plan &p = b->plan;
    const uint32_t N = b->n_envs;
    auto up = [&](size_t off, const void *src, size_t bytes) {
        return hipMemcpyAsync(b->d + off, src, bytes, hipMemcpyHostToDevice, b->stream);
    };
    HIP_TRY(up(p.reg.pos, s.pos.data(), 2 * p.agents));
    HIP_TRY(up(p.reg.found, s.found.data(), 4ull * N));
    HIP_TRY(up(p.reg.t, s.t.data(), 4ull * N));
    HIP_TRY(up(p.reg.ep, s.ep.data(), 4ull * N));
    HIP_TRY(up(p.reg.steps, s.steps.data(), 4ull * N));
    HIP_TRY(up(p.reg.stuck, s.stuck.data(), 4ull * N));
    HIP_TRY(up(p.reg.bel, s.bel.data(), 4ull * p.agents));
    if (p.map_words) HIP_TRY(up(p.reg.disc, s.disc.data(), 4ull * p.map_words));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return HASE_OK;
}

// Milliseconds of a persistent call of n_steps under the current tiling: the
// faster of two timed calls, after an untimed one that also captures the
// graph; the state is restored before each call and at the end.
constexpr int AUTOTUNE_REPS = 5;
constexpr float AUTOTUNE_MARGIN = 0.02f;

int time_tiling(hase_batch *b, const JobDesc &job, uint32_t n_steps, const Snapshot &snap,
                float *ms)
{
    int rc = persistent_step(b, job, n_steps);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hipError_t err = hipSuccess;
    // the median of AUTOTUNE_REPS timed runs, each from the same snapshot
    float t[AUTOTUNE_REPS] = {};
    int got = 0;
    for (int rep = 0; rep < AUTOTUNE_REPS && !rc && err == hipSuccess; ++rep) {
        rc = snapshot_restore(b, snap);
        if (rc) break;
        err = hipEventRecord(e0, b->stream);
        if (err == hipSuccess) rc = persistent_step(b, job, n_steps);
        if (err == hipSuccess && !rc) err = hipEventRecord(e1, b->stream);
        if (err == hipSuccess && !rc) err = hipEventSynchronize(e1);
        if (err == hipSuccess && !rc) err = hipEventElapsedTime(&t[got], e0, e1);
        if (err == hipSuccess && !rc) ++got;
    }
    std::sort(t, t + got);
    *ms = got ? t[got / 2] : 0.f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (err != hipSuccess) return hip_fail(err, "autotune timing");
    return snapshot_restore(b, snap);
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

int hase_query_layout(const hase_batch_desc *desc, hase_layout *out)
{
    if (!out) return fail(HASE_EINVAL, "null layout pointer");
    Plan p;
    const int rc = make_plan(desc, p);
    if (rc) return rc;
    out->state_bytes = p.reg.total;
    out->obs_words_per_step = p.obs_words;
    out->agents_total = p.agents;
    out->n_envs = desc->n_envs;
    out->cells_total = p.cells;
    out->map_words_per_step = p.map_words;
    return HASE_OK;
}

int hase_create(const hase_batch_desc *desc, void *d_state, uint64_t state_bytes, void *stream,
                hase_batch **out)
{
    if (!out) return fail(HASE_EINVAL, "null output handle pointer");
    *out = nullptr;
    hase_batch *b = new hase_batch();
    int rc = make_plan(desc, b->plan);
    if (rc) {
        delete b;
        return rc;
    }
    if (!d_state || ((uintptr_t)d_state & 255u)) {
        delete b;
        return fail(HASE_EINVAL, "state buffer must be a non-null 256-byte aligned device pointer");
    }
    if (state_bytes < b->plan.reg.total) {
        const size_t need = b->plan.reg.total;
        delete b;
        return fail(HASE_ENOMEM, "state buffer has %llu bytes, needs %zu",
                    (unsigned long long)state_bytes, need);
    }
    b->n_envs = desc->n_envs;
    b->env_id_base = desc->env_id_base;
    b->d = static_cast<char *>(d_state);
    b->stream = static_cast<hipStream_t>(stream);
    default_lanes(b->plan.specs, b->lanes);

    const uint32_t N = b->n_envs;
    const Plan &p = b->plan;
    std::vector<uint32_t> s0(N), s1(N), s2(N), id(N), terr(8ull * N, 0u);
    for (uint32_t e = 0; e < N; ++e) {
        const hase_env_spec &s = p.specs[e];
        if (s.flags & HASE_TERRAIN) {
            uint32_t *tr = &terr[8ull * e];
            tr[0] = s.water_pct | ((uint32_t)s.mud_pct << 8) | ((uint32_t)s.stuck_pct << 16);
            for (int k = 0; k < 9; ++k) tr[1 + k / 4] |= (uint32_t)s.speed_pct[k] << (8 * (k % 4));
            tr[4] = (uint32_t)s.agent_classes;
            tr[5] = (uint32_t)(s.agent_classes >> 32);
        }
        s0[e] = s.height | (s.width << 8) | ((uint32_t)s.n_agents << 16) | ((uint32_t)s.n_seekers << 24);
        s1[e] = s.view_radius | ((uint32_t)s.n_channels << 4) | ((uint32_t)s.flags << 8) |
                ((uint32_t)s.episode_len << 16);
        s2[e] = s.wall_pct | ((uint32_t)board_words_per_row(s.width) << 8);
        id[e] = desc->env_id_base + e;
    }
    auto up = [&](size_t off, const void *src, size_t bytes) {
        return hipMemcpyAsync(b->d + off, src, bytes, hipMemcpyHostToDevice, b->stream);
    };
    hipError_t e;
    if ((e = up(p.reg.spec0, s0.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.spec1, s1.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.spec2, s2.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.obs_off, p.obs_off.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.agent_off, p.agent_off.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.bb_off, p.bb_off.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.grid_off, p.grid_off.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.env_id, id.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.map_off, p.map_off.data(), 4ull * N)) != hipSuccess ||
        (e = up(p.reg.terr, terr.data(), 32ull * N)) != hipSuccess ||
        (e = hipStreamSynchronize(b->stream)) != hipSuccess) {
        delete b;
        return hip_fail(e, "hase_create upload");
    }
    rc = build_tiles(b);
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return HASE_OK;
}

int hase_get_offsets(const hase_batch *b, uint64_t *h_obs_off, uint64_t *h_agent_off)
{
    if (b && b->arena) return fail(HASE_EINVAL, "hase_get_offsets: not an operation of an arena");
    if (!b) return fail(HASE_EINVAL, "null handle");
    for (uint32_t e = 0; e < b->n_envs; ++e) {
        if (h_obs_off) h_obs_off[e] = b->plan.obs_off[e];
        if (h_agent_off) h_agent_off[e] = b->plan.agent_off[e];
    }
    return HASE_OK;
}

int hase_get_map_offsets(const hase_batch *b, uint64_t *h_map_off)
{
    if (b && b->arena) return fail(HASE_EINVAL, "hase_get_map_offsets: not an operation of an arena");
    if (!b || !h_map_off) return fail(HASE_EINVAL, "null argument");
    for (uint32_t e = 0; e < b->n_envs; ++e) h_map_off[e] = b->plan.map_off[e];
    return HASE_OK;
}

int hase_reset(hase_batch *b, uint64_t seed, uint32_t *d_obs0)
{
    if (b && b->arena) return fail(HASE_EINVAL, "hase_reset: not an operation of an arena");
    if (!b) return fail(HASE_EINVAL, "null handle");
    HIP_TRY(hipMemsetAsync(b->d + b->plan.reg.err, 0xff, 4, b->stream));
    HIP_TRY(launch_init(make_init(b, seed, 0), b->stream));
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, b->d + b->plan.reg.err, 4, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (err != 0xffffffffu) {
        b->ready = false;
        return fail(HASE_EGRID, "env %u has too few free cells for its agents", err);
    }
    b->ready = true;
    if (d_obs0) {
        const int rc = enqueue(b, make_job(b, nullptr, d_obs0, nullptr, nullptr), 0, 0, b->stream,
                               false);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(b->stream));
    }
    return HASE_OK;
}

int hase_step(hase_batch *b, uint32_t n_steps, const int8_t *d_actions, uint32_t *d_obs, float *d_rew,
              uint8_t *d_done, uint32_t mode)
{
    return hase_step_maps(b, n_steps, d_actions, d_obs, d_rew, d_done, nullptr, mode);
}

int hase_step_maps(hase_batch *b, uint32_t n_steps, const int8_t *d_actions, uint32_t *d_obs,
                   float *d_rew, uint8_t *d_done, uint32_t *d_map, uint32_t mode)
{
    const hase_outputs out{d_obs, d_rew, d_done, d_map, nullptr, nullptr};
    return hase_step_outputs(b, n_steps, d_actions, &out, mode);
}

int hase_step_outputs(hase_batch *b, uint32_t n_steps, const int8_t *d_actions,
                      const hase_outputs *out, uint32_t mode)
{
    if (!out) return fail(HASE_EINVAL, "null outputs");
    const int rc0 = check_step_args(b, n_steps, out->obs, out->rew, out->done);
    if (rc0) return rc0;
    if (mode != HASE_STEP_PERSISTENT && mode != HASE_STEP_PER_LAUNCH)
        return fail(HASE_EINVAL, "unknown step mode %u", mode);
    JobDesc job = make_job(b, d_actions, out->obs, out->rew, out->done, out->map);
    job.spos = out->pos;
    job.senv = out->env_state;
    if (mode == HASE_STEP_PERSISTENT) return persistent_step(b, job, n_steps);
    if (b->variants.size() > 1) {
        const int rc = ensure_streams(b, b->variants.size());
        if (rc) return rc;
    }
    for (uint32_t k = 0; k < n_steps; ++k) {
        const int rc = enqueue(b, job, 1, k, b->stream, b->variants.size() > 1);
        if (rc) return rc;
    }
    return HASE_OK;
}

int hase_prepare(hase_batch *b, uint32_t n_steps, const int8_t *d_actions, uint32_t *d_obs,
                 float *d_rew, uint8_t *d_done)
{
    return hase_prepare_maps(b, n_steps, d_actions, d_obs, d_rew, d_done, nullptr);
}

int hase_prepare_maps(hase_batch *b, uint32_t n_steps, const int8_t *d_actions, uint32_t *d_obs,
                      float *d_rew, uint8_t *d_done, uint32_t *d_map)
{
    const hase_outputs out{d_obs, d_rew, d_done, d_map, nullptr, nullptr};
    return hase_prepare_outputs(b, n_steps, d_actions, &out);
}

int hase_prepare_outputs(hase_batch *b, uint32_t n_steps, const int8_t *d_actions,
                         const hase_outputs *out)
{
    if (!out) return fail(HASE_EINVAL, "null outputs");
    const int rc = check_step_args(b, n_steps, out->obs, out->rew, out->done);
    if (rc) return rc;
    if (b->variants.size() == 1) return HASE_OK;  // launched directly, no graph
    JobDesc job = make_job(b, d_actions, out->obs, out->rew, out->done, out->map);
    job.spos = out->pos;
    job.senv = out->env_state;
    hipGraphExec_t exec = nullptr;
    return graph_for(b, job, n_steps, &exec);
}

int hase_observe(hase_batch *b, uint32_t *d_obs)
{
    if (b && b->arena) return fail(HASE_EINVAL, "hase_observe: not an operation of an arena");
    if (!b) return fail(HASE_EINVAL, "null handle");
    if (!b->ready) return fail(HASE_ENOTREADY, "observe before reset/set_state");
    if (!d_obs) return fail(HASE_EINVAL, "null obs buffer");
    return enqueue(b, make_job(b, nullptr, d_obs, nullptr, nullptr), 0, 0, b->stream, false);
}

int hase_get_state(hase_batch *b, const hase_host_state *out)
{
    if (b && b->arena) return fail(HASE_EINVAL, "hase_get_state: not an operation of an arena");
    if (!b || !out) return fail(HASE_EINVAL, "null argument");
    if (!out->walls || !out->pos_x || !out->pos_y || !out->found || !out->t || !out->episode ||
        !out->steps || !out->seed)
        return fail(HASE_EINVAL, "null host array in state");
    const Plan &p = b->plan;
    const uint32_t N = b->n_envs;
    std::vector<uint16_t> pos(p.agents);
    auto down = [&](void *dst, size_t off, size_t bytes) {
        return hipMemcpyAsync(dst, b->d + off, bytes, hipMemcpyDeviceToHost, b->stream);
    };
    HIP_TRY(down(out->walls, p.reg.walls, p.cells));
    HIP_TRY(down(pos.data(), p.reg.pos, 2 * p.agents));
    HIP_TRY(down(out->found, p.reg.found, 4ull * N));
    HIP_TRY(down(out->t, p.reg.t, 4ull * N));
    HIP_TRY(down(out->episode, p.reg.ep, 4ull * N));
    HIP_TRY(down(out->steps, p.reg.steps, 4ull * N));
    HIP_TRY(down(out->seed, p.reg.seed, 8ull * N));
    if (out->discovered && p.map_words)
        HIP_TRY(down(out->discovered, p.reg.disc, 4ull * p.map_words));
    if (out->stuck) HIP_TRY(down(out->stuck, p.reg.stuck, 4ull * N));
    if (out->belief) HIP_TRY(down(out->belief, p.reg.bel, 4ull * p.agents));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (uint64_t i = 0; i < p.agents; ++i) {
        out->pos_x[i] = (uint8_t)(pos[i] & 0xff);
        out->pos_y[i] = (uint8_t)(pos[i] >> 8);
    }
    return HASE_OK;
}

int hase_set_state(hase_batch *b, const hase_host_state *in)
{
    if (b && b->arena) return fail(HASE_EINVAL, "hase_set_state: not an operation of an arena");
    if (!b || !in) return fail(HASE_EINVAL, "null argument");
    if (!in->walls || !in->pos_x || !in->pos_y || !in->found || !in->t || !in->episode ||
        !in->steps || !in->seed)
        return fail(HASE_EINVAL, "null host array in state");
    const Plan &p = b->plan;
    const uint32_t N = b->n_envs;
    std::vector<uint16_t> pos(p.agents);
    for (uint32_t e = 0; e < N; ++e) {
        const hase_env_spec &s = p.specs[e];
        for (uint32_t j = 0; j < s.n_agents; ++j) {
            const uint32_t i = p.agent_off[e] + j;
            if (in->pos_x[i] >= s.width || in->pos_y[i] >= s.height)
                return fail(HASE_ESTATE, "env %u agent %u outside the %ux%u map", e, j, s.width,
                            s.height);
            pos[i] = (uint16_t)(in->pos_x[i] | (in->pos_y[i] << 8));
        }
        const uint8_t max_tile = (s.flags & HASE_TERRAIN) ? 3 : 1;
        // cells each agent class may stand on (plain envs: open cells, the
        // walker's count): an auto-reset must find room for all n agents, as
        // hase_reset demands of the grids it draws
        uint32_t room[3] = {0, 0, 0};
        for (uint32_t c = 0; c < (uint32_t)s.height * s.width; ++c) {
            const uint8_t v = in->walls[p.grid_off[e] + c];
            if (v > max_tile)
                return fail(HASE_ESTATE, "env %u cell %u: tile value %u above %u", e, c, v, max_tile);
            const bool terr = (s.flags & HASE_TERRAIN) != 0;
            room[0] += terr ? (v == 0 || v == 3) : (v == 0);  // walker: ground, mud
            room[1] += terr && v == 2;                       // swimmer: water
            room[2] += terr && v != 1;                       // flyer: all but walls
        }
        for (uint32_t j = 0; j < s.n_agents; ++j) {
            const uint32_t cls = (s.flags & HASE_TERRAIN) ? (uint32_t)(s.agent_classes >> (2 * j)) & 3u : 0u;
            if (room[cls] < s.n_agents)
                return fail(HASE_EGRID, "env %u has too few free cells for its agents", e);
        }
        if (in->stuck && in->stuck[e] != 0u &&
            (!(s.flags & HASE_TERRAIN) || (in->stuck[e] >> s.n_agents) != 0u))
            return fail(HASE_ESTATE, "env %u: stuck bits of absent agents or without terrain", e);
        if (in->belief) {
            // beliefs hold hider bits only, and only in radio envs
            const uint32_t hm = (s.flags & HASE_RADIO)
                                    ? (uint32_t)(((1ull << s.n_agents) - 1ull) & ~((1ull << s.n_seekers) - 1ull))
                                    : 0u;
            for (uint32_t j = 0; j < s.n_agents; ++j)
                if (in->belief[p.agent_off[e] + j] & ~hm)
                    return fail(HASE_ESTATE, "env %u agent %u: belief bits that are not hiders of a radio env",
                                e, j);
        }
        if (in->discovered && (s.flags & HASE_EXPLORE)) {
            // map bits past the width are not cells
            const uint32_t rw = (s.width + 31) / 32, tail = s.width & 31u;
            const uint32_t bad = tail ? ~((1u << tail) - 1u) : 0u;
            for (uint32_t y = 0; y < s.height; ++y)
                if (in->discovered[p.map_off[e] + y * rw + rw - 1] & bad)
                    return fail(HASE_ESTATE, "env %u: discovery map row %u has bits past the width",
                                e, y);
        }
    }
    auto up = [&](size_t off, const void *src, size_t bytes) {
        return hipMemcpyAsync(b->d + off, src, bytes, hipMemcpyHostToDevice, b->stream);
    };
    HIP_TRY(up(p.reg.walls, in->walls, p.cells));
    HIP_TRY(up(p.reg.pos, pos.data(), 2 * p.agents));
    HIP_TRY(up(p.reg.found, in->found, 4ull * N));
    HIP_TRY(up(p.reg.t, in->t, 4ull * N));
    HIP_TRY(up(p.reg.ep, in->episode, 4ull * N));
    HIP_TRY(up(p.reg.steps, in->steps, 4ull * N));
    HIP_TRY(up(p.reg.seed, in->seed, 8ull * N));
    if (p.map_words) {
        if (in->discovered)
            HIP_TRY(up(p.reg.disc, in->discovered, 4ull * p.map_words));
        else
            HIP_TRY(hipMemsetAsync(b->d + p.reg.disc, 0, 4ull * p.map_words, b->stream));
    }
    if (in->stuck)
        HIP_TRY(up(p.reg.stuck, in->stuck, 4ull * N));
    else
        HIP_TRY(hipMemsetAsync(b->d + p.reg.stuck, 0, 4ull * N, b->stream));
    if (in->belief)
        HIP_TRY(up(p.reg.bel, in->belief, 4ull * p.agents));
    else
        HIP_TRY(hipMemsetAsync(b->d + p.reg.bel, 0, 4ull * p.agents, b->stream));
    HIP_TRY(launch_init(make_init(b, 0, 1), b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->ready = true;
    return HASE_OK;
}

int hase_set_tiling(hase_batch *b, const uint32_t lanes[HASE_N_BUCKETS])
{
    if (b && b->arena) return fail(HASE_EINVAL, "hase_set_tiling: not an operation of an arena");
    if (!b || !lanes) return fail(HASE_EINVAL, "null argument");
    uint32_t next[N_BUCKETS], dflt[N_BUCKETS];
    default_lanes(b->plan.specs, dflt);
    for (int i = 0; i < N_BUCKETS; ++i) {
        next[i] = lanes[i] ? lanes[i] : dflt[i];
        if (!variant_supported((int)next[i], BUCKET_NMAX[i]))
            return fail(HASE_EINVAL, "bucket %d: unsupported lanes per env %u", i, next[i]);
    }
    uint32_t prev[N_BUCKETS];
    std::memcpy(prev, b->lanes, sizeof prev);
    std::memcpy(b->lanes, next, sizeof next);
    const int rc = build_tiles(b);
    if (rc) {
        std::memcpy(b->lanes, prev, sizeof prev);
        build_tiles(b);
    }
    return rc;
}

int hase_get_tiling(const hase_batch *b, uint32_t lanes[HASE_N_BUCKETS])
{
    if (b && b->arena) return fail(HASE_EINVAL, "hase_get_tiling: not an operation of an arena");
    if (!b || !lanes) return fail(HASE_EINVAL, "null argument");
    for (int i = 0; i < N_BUCKETS; ++i) lanes[i] = b->lanes[i];
    return HASE_OK;
}

int hase_autotune(hase_batch *b, uint32_t n_steps, uint32_t *d_obs, float *d_rew, uint8_t *d_done,
                  uint32_t lanes_out[HASE_N_BUCKETS])
{
    const int rc0 = check_step_args(b, n_steps, d_obs, d_rew, d_done);
    if (rc0) return rc0;
    Snapshot snap;
    int rc = snapshot_take(b, snap);
    if (rc) return rc;
    bool present[N_BUCKETS] = {};
    for (const hase_env_spec &s : b->plan.specs) present[bucket_of(s.n_agents)] = true;
    const JobDesc job = make_job(b, nullptr, d_obs, d_rew, d_done);
    uint32_t best[N_BUCKETS];
    std::memcpy(best, b->lanes, sizeof best);
    float best_ms = 0.f;
    rc = time_tiling(b, job, n_steps, snap, &best_ms);
    if (rc) return rc;
    const uint32_t cands[] = {1, 2, 4, 8, 16};
    for (int bk = 0; bk < N_BUCKETS; ++bk) {
        if (!present[bk]) continue;
        for (uint32_t L : cands) {
            if (L == best[bk] || !variant_supported((int)L, BUCKET_NMAX[bk])) continue;
            std::memcpy(b->lanes, best, sizeof best);
            b->lanes[bk] = L;
            if (build_tiles(b) != HASE_OK) continue;  // e.g. LDS too small for this shape
            float ms = 0.f;
            rc = time_tiling(b, job, n_steps, snap, &ms);
            if (rc) break;
            // a candidate must beat the best by more than the run-to-run
            // spread of the median
            if (ms < best_ms * (1.f - AUTOTUNE_MARGIN)) {
                best_ms = ms;
                best[bk] = L;
            }
        }
        if (rc) break;
    }
    std::memcpy(b->lanes, best, sizeof best);
    const int rc2 = build_tiles(b);
    const int rc3 = snapshot_restore(b, snap);
    if (rc) return rc;
    if (rc2) return rc2;
    if (rc3) return rc3;
    if (lanes_out)
        for (int i = 0; i < N_BUCKETS; ++i) lanes_out[i] = best[i];
    return HASE_OK;
}

int hase_multi_workspace(hase_batch *const *batches, uint32_t n, uint64_t *bytes)
{
    if (!bytes || (n && !batches)) return fail(HASE_EINVAL, "null argument");
    size_t tiles = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!batches[i]) return fail(HASE_EINVAL, "null handle %u", i);
        if (batches[i]->arena) return fail(HASE_EINVAL, "handle %u is an arena", i);
        tiles += batches[i]->host_tiles.size();
    }
    *bytes = align256(sizeof(JobDesc) * (size_t)(n ? n : 1)) + align256(sizeof(Tile) * (tiles ? tiles : 1));
    return HASE_OK;
}

int hase_step_multi(const hase_step_io *io, uint32_t n, uint32_t n_steps, void *d_workspace,
                    uint64_t workspace_bytes, void *stream)
{
    if (n == 0) return HASE_OK;
    if (!io || !d_workspace) return fail(HASE_EINVAL, "null argument");
    if (n_steps == 0) return fail(HASE_EINVAL, "n_steps must be >= 1");
    std::vector<hase_batch *> bs(n);
    std::vector<JobDesc> jobs(n);
    for (uint32_t i = 0; i < n; ++i) {
        hase_batch *b = io[i].batch;
        const int rc = check_step_args(b, io[i].n_steps, io[i].d_obs, io[i].d_rew, io[i].d_done);
        if (rc) return fail(rc, "request %u: %s", i, g_last_error.c_str());
        if (io[i].n_steps > n_steps)
            return fail(HASE_EINVAL, "request %u: %u steps > call's %u", i, io[i].n_steps, n_steps);
        for (uint32_t j = 0; j < i; ++j)
            if (bs[j] == b) return fail(HASE_EINVAL, "request %u repeats a batch handle", i);
        bs[i] = b;
        jobs[i] = make_job(b, io[i].d_actions, io[i].d_obs, io[i].d_rew, io[i].d_done, io[i].d_map);
        jobs[i].k_limit = io[i].n_steps;
        jobs[i].out_step0 = io[i].out_step0;
    }
    uint64_t need = 0;
    int rc = hase_multi_workspace(bs.data(), n, &need);
    if (rc) return rc;
    if (workspace_bytes < need)
        return fail(HASE_ENOMEM, "workspace has %llu bytes, needs %llu",
                    (unsigned long long)workspace_bytes, (unsigned long long)need);
    // one launch group per (lanes, kind) across all requests; a plain group
    // whose tiles carry more than one variant code runs the mixed kernel
    struct Group {
        uint32_t lanes = 0, tile0 = 0, n_tiles = 0, slot = 0, map = 0, code0 = 0;
        int kind = KIND_PLAIN;
        bool mixed = false, big = false, combo = false;
    };
    std::vector<Tile> tiles;
    std::vector<Group> groups;
    const uint32_t lane_order[] = {1, 2, 4, 8, 16};
    for (uint32_t L : lane_order) {
        for (int kb = 0; kb < 4 * N_KINDS; ++kb) {
            const int kind = (kb >> 1) % N_KINDS;
            const bool big = (kb & 1) != 0, combo = kb >= 2 * N_KINDS;
            if (combo && (L != 4 || kind != KIND_PLAIN || big)) continue;
            Group g;
            auto open_group = [&]() {
                g = Group{};
                g.lanes = L;
                g.kind = kind;
                g.big = big;
                g.combo = combo;
                // the feature kinds have only the mixed kernel
                g.mixed = kind != KIND_PLAIN || combo;
                g.tile0 = (uint32_t)tiles.size();
            };
            auto close_group = [&]() {
                g.n_tiles = (uint32_t)tiles.size() - g.tile0;
                if (g.n_tiles) groups.push_back(g);
            };
            open_group();
            for (uint32_t i = 0; i < n; ++i) {
                for (const Variant &v : bs[i]->variants) {
                    if ((uint32_t)v.lanes != L || v.kind != kind || v.big != big || v.combo != combo)
                        continue;
                    // a request whose boards would push the group past 64 KiB of
                    // LDS per wave starts a launch group of its own
                    const uint32_t slot = std::max(g.slot, v.slot_words), map = std::max(g.map, v.map_words);
                    const size_t need = combo ? combo_lds_bytes(slot)
                                              : (size_t)(64u / L) * (slot + MAX_AGENTS + map) * 4;
                    if (need > 65536 && tiles.size() > g.tile0) {
                        close_group();
                        open_group();
                    }
                    for (uint32_t t = v.tile0; t < v.tile0 + v.n_tiles; ++t) {
                        Tile tl = bs[i]->host_tiles[t];
                        tl.job = i;
                        if (tiles.size() == g.tile0)
                            g.code0 = tl.variant;
                        else if (tl.variant != g.code0)
                            g.mixed = true;
                        tiles.push_back(tl);
                    }
                    g.slot = std::max(g.slot, v.slot_words);
                    g.map = std::max(g.map, v.map_words);
                }
            }
            close_group();
        }
    }
    if (groups.size() > (size_t)MAX_LAUNCHES)
        return fail(HASE_EINVAL, "these requests need %zu launch groups, at most %d", groups.size(),
                    MAX_LAUNCHES);
    char *ws = static_cast<char *>(d_workspace);
    const size_t jobs_bytes = align256(sizeof(JobDesc) * n);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(ws, jobs.data(), sizeof(JobDesc) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ws + jobs_bytes, tiles.data(), sizeof(Tile) * tiles.size(),
                           hipMemcpyHostToDevice, st));
    const JobDesc *djobs = reinterpret_cast<const JobDesc *>(ws);
    const Tile *dtiles = reinterpret_cast<const Tile *>(ws + jobs_bytes);
    // several groups run concurrently on the first request's side streams,
    // forked after the uploads and joined back into the stream
    hase_batch *fb = bs[0];
    const bool fork = groups.size() > 1;
    if (fork) {
        rc = ensure_streams(fb, groups.size());
        if (rc) return rc;
        HIP_TRY(hipEventRecord(fb->fork_ev, st));
    }
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group &g = groups[gi];
        hipStream_t s = st;
        if (fork && gi > 0) {
            HIP_TRY(hipStreamWaitEvent(fb->side[gi], fb->fork_ev, 0));
            s = fb->side[gi];
        }
        if (g.combo)
            HIP_TRY(launch_combo(dtiles + g.tile0, g.n_tiles, djobs, jobs[0], n_steps, 0, g.slot, s));
        else if (g.mixed)
            HIP_TRY(launch_mixed((int)g.lanes, g.kind, dtiles + g.tile0, g.n_tiles, djobs, jobs[0],
                                 n_steps, 0, g.slot, g.map, g.big, s));
        else
            HIP_TRY(launch_step((int)g.lanes, BUCKET_NMAX[g.code0 >> 2], (int)(g.code0 & 3u) + 1,
                                dtiles + g.tile0, g.n_tiles, djobs, jobs[0], n_steps, 0, g.slot, s));
        if (fork && gi > 0) {
            HIP_TRY(hipEventRecord(fb->join_ev[gi], s));
            HIP_TRY(hipStreamWaitEvent(st, fb->join_ev[gi], 0));
        }
    }
    return HASE_OK;
}

// ---------------------------------------------------------------- arenas

int hase_query_arena(const hase_arena_desc *desc, uint64_t *state_bytes)
{
    if (!desc || !state_bytes) return fail(HASE_EINVAL, "null argument");
    const uint64_t N = desc->n_slots;
    if (N == 0 || N >= (1u << 26)) return fail(HASE_EINVAL, "n_slots must be in 1..2^26-1");
    if (desc->max_height < 2 || desc->max_height > MAX_SIDE || desc->max_width < 2 ||
        desc->max_width > MAX_SIDE)
        return fail(HASE_EINVAL, "max_height/max_width must be in 2..%d", MAX_SIDE);
    if (desc->max_agents < 1 || desc->max_agents > MAX_AGENTS)
        return fail(HASE_EINVAL, "max_agents must be in 1..%d", MAX_AGENTS);
    if (desc->max_ranges < 1 || desc->max_ranges > 65536)
        return fail(HASE_EINVAL, "max_ranges must be in 1..65536");
    const uint64_t A = N * desc->max_agents, cells = N * desc->max_height * desc->max_width;
    const uint64_t bbw = N * (uint64_t)board_words(desc->max_height, 2);
    const uint64_t mw = N * (uint64_t)map_words(desc->max_height, desc->max_width);
    if (A >= (1ull << 32) || cells >= (1ull << 32) || bbw >= (1ull << 32))
        return fail(HASE_EINVAL, "arena too large: offsets exceed 32 bits");
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    // the same regions as a batch (slot-indexed), plus the ranges' jobs
    for (int i = 0; i < 10; ++i) take(4 * N);  // perm .. map_off
    take(32 * N);                             // terr
    take(8 * N);                              // seed
    for (int i = 0; i < 5; ++i) take(4 * N);  // found, t, ep, steps, stuck
    take(4 * A);                              // bel
    take(2 * A);                              // pos
    take(cells);                              // walls
    take(4 * bbw);                            // bb
    take(4 * mw);                             // disc
    take(sizeof(Tile) * N);                   // tiles: tile i of a range at its slot first + i
    take(16);                                 // err
    take(sizeof(JobDesc) * desc->max_ranges); // jobs
    take(4ull * desc->max_ranges);            // job_err
    *state_bytes = off;
    return HASE_OK;
}

int hase_create_arena(const hase_arena_desc *desc, void *d_state, uint64_t state_bytes, void *stream,
                      hase_batch **out)
{
    if (!out) return fail(HASE_EINVAL, "null output handle pointer");
    *out = nullptr;
    uint64_t need = 0;
    int rc = hase_query_arena(desc, &need);
    if (rc) return rc;
    if (!d_state || ((uintptr_t)d_state & 255u))
        return fail(HASE_EINVAL, "state buffer must be a non-null 256-byte aligned device pointer");
    if (state_bytes < need)
        return fail(HASE_ENOMEM, "state buffer has %llu bytes, needs %llu",
                    (unsigned long long)state_bytes, (unsigned long long)need);
    hase_batch *b = new hase_batch();
    b->arena = true;
    b->n_envs = desc->n_slots;
    b->cap_h = desc->max_height;
    b->cap_w = desc->max_width;
    b->cap_n = desc->max_agents;
    b->d = static_cast<char *>(d_state);
    b->stream = static_cast<hipStream_t>(stream);
    for (uint32_t j = desc->max_ranges; j-- > 0;) b->free_jobs.push_back(j);
    const uint64_t N = desc->n_slots;
    Regions &r = b->plan.reg;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const uint64_t A = N * b->cap_n;
    const uint32_t bw = (uint32_t)board_words(b->cap_h, 2), mw = (uint32_t)map_words(b->cap_h, b->cap_w);
    r.perm = take(4 * N);
    r.spec0 = take(4 * N);
    r.spec1 = take(4 * N);
    r.spec2 = take(4 * N);
    r.obs_off = take(4 * N);
    r.agent_off = take(4 * N);
    r.bb_off = take(4 * N);
    r.grid_off = take(4 * N);
    r.env_id = take(4 * N);
    r.map_off = take(4 * N);
    r.terr = take(32 * N);
    r.seed = take(8 * N);
    r.found = take(4 * N);
    r.t = take(4 * N);
    r.ep = take(4 * N);
    r.steps = take(4 * N);
    r.stuck = take(4 * N);
    r.bel = take(4 * A);
    r.pos = take(2 * A);
    r.walls = take(N * b->cap_h * b->cap_w);
    r.bb = take(4 * N * bw);
    r.disc = take(4 * N * mw);
    r.tiles = take(sizeof(Tile) * N);
    r.err = take(16);
    r.jobs = take(sizeof(JobDesc) * desc->max_ranges);
    r.job_err = take(4ull * desc->max_ranges);
    r.total = off;
    // slot-indexed state offsets (every slot has the capacity of the caps);
    // the tile table starts empty
    std::vector<uint32_t> perm(N), zero(N, 0u), aoff(N), bboff(N), goff(N), moff(N);
    for (uint32_t e = 0; e < N; ++e) {
        perm[e] = e;
        aoff[e] = e * b->cap_n;
        bboff[e] = e * bw;
        goff[e] = e * b->cap_h * b->cap_w;
        moff[e] = e * mw;
    }
    std::vector<Tile> tiles(N, Tile{0u, 0u, 0u, 0u});
    auto up = [&](size_t o, const void *src, size_t bytes) {
        return hipMemcpyAsync(b->d + o, src, bytes, hipMemcpyHostToDevice, b->stream);
    };
    hipError_t e;
    if ((e = up(r.perm, perm.data(), 4 * N)) != hipSuccess ||
        (e = up(r.obs_off, zero.data(), 4 * N)) != hipSuccess ||
        (e = up(r.agent_off, aoff.data(), 4 * N)) != hipSuccess ||
        (e = up(r.bb_off, bboff.data(), 4 * N)) != hipSuccess ||
        (e = up(r.grid_off, goff.data(), 4 * N)) != hipSuccess ||
        (e = up(r.map_off, moff.data(), 4 * N)) != hipSuccess ||
        (e = up(r.tiles, tiles.data(), sizeof(Tile) * N)) != hipSuccess ||
        (e = hipStreamSynchronize(b->stream)) != hipSuccess) {
        delete b;
        return hip_fail(e, "hase_create_arena upload");
    }
    b->ready = true;
    *out = b;
    return HASE_OK;
}

int hase_reset_range(hase_batch *b, uint32_t first_slot, uint32_t count, const hase_env_spec *spec,
                     uint64_t seed, uint32_t env_id_base, uint32_t step_budget,
                     const hase_out_ptrs *out)
{
    if (!b || !spec || !out) return fail(HASE_EINVAL, "null argument");
    if (!b->arena) return fail(HASE_EINVAL, "hase_reset_range needs an arena (hase_create_arena)");
    int rc = check_spec(*spec, 0);
    if (rc) return rc;
    const hase_env_spec &s = *spec;
    if (s.height > b->cap_h || s.width > b->cap_w || s.n_agents > b->cap_n)
        return fail(HASE_EINVAL, "spec %ux%u with %u agents exceeds the arena's %ux%u, %u agents",
                    s.height, s.width, s.n_agents, b->cap_h, b->cap_w, b->cap_n);
    if (count == 0 || (uint64_t)first_slot + count > b->n_envs)
        return fail(HASE_EINVAL, "slots [%u, %u + %u) outside the arena's %u", first_slot, first_slot,
                    count, b->n_envs);
    if (step_budget == 0) return fail(HASE_EINVAL, "step_budget must be >= 1");
    if (!out->obs || !out->rew || !out->done) return fail(HASE_EINVAL, "null output buffer");
    // no overlap with an admitted range
    auto nx = b->ranges.lower_bound(first_slot);
    if (nx != b->ranges.end() && nx->first < first_slot + count)
        return fail(HASE_EINVAL, "slots from %u are taken by the range at %u", first_slot, nx->first);
    if (nx != b->ranges.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second.count > first_slot)
            return fail(HASE_EINVAL, "slot %u is taken by the range at %u", first_slot, pv->first);
    }
    if (b->free_jobs.empty()) return fail(HASE_EINVAL, "the arena holds its maximum of ranges");
    // tiling: the default lanes of the spec's bucket, widened while the
    // wave's LDS (envs per wave x cap-sized slot) would exceed 64 KiB
    const int kind = env_kind(s.flags);
    const int planes = (s.flags & HASE_TERRAIN) ? 2 : 1;
    const uint32_t slot_words = (uint32_t)board_words((int)b->cap_h, planes);
    const uint32_t mwl = (s.flags & HASE_EXPLORE) ? (uint32_t)round4(lds_board_words((int)b->cap_h)) : 0u;
    const int bk = bucket_of(s.n_agents);
    uint32_t lanes = DEFAULT_LANES[bk];
    while (lanes < 16 && (size_t)(64u / lanes) * (slot_words + MAX_AGENTS + mwl) * 4 > 65536) lanes *= 2;
    if (!variant_supported((int)lanes, BUCKET_NMAX[bk]) ||
        (size_t)(64u / lanes) * (slot_words + MAX_AGENTS + mwl) * 4 > 65536)
        return fail(HASE_EINVAL, "no tiling fits this spec in LDS");
    // plain envs of 5 to COMBO_MID_NMAX agents take the combined kernel's
    // 8-lane tiles, one agent per lane (8 envs per wave instead of 4)
    const bool mid = kind == KIND_PLAIN && bk == 2 && lanes == 16 && s.n_agents <= COMBO_MID_NMAX &&
                     combo_lds_bytes(slot_words) <= 65536;
    if (mid) lanes = 8;
    const uint32_t E = 64u / lanes;
    const uint32_t w = (uint32_t)words_per_channel(s.view_radius);
    const uint32_t obs_env = s.n_agents * (s.n_channels * w + ((s.flags & HASE_RADIO) ? 1u : 0u));
    const uint32_t map_env = (s.flags & HASE_EXPLORE) ? (uint32_t)map_words(s.height, s.width) : 0u;
    if ((uint64_t)count * obs_env >= (1ull << 32) || (uint64_t)count * s.n_agents >= (1ull << 32))
        return fail(HASE_EINVAL, "range too large: per-step output offsets exceed 32 bits");

    const uint32_t job = b->free_jobs.back();
    const Regions &r = b->plan.reg;
    JobDesc j = make_job(b, nullptr, out->obs, out->rew, out->done, out->map);
    j.spos = out->pos;
    j.senv = out->env_state;
    j.obs_stride = (uint64_t)count * obs_env;
    j.agent_stride = (uint64_t)count * s.n_agents;
    j.env_stride = count;
    j.map_stride = (uint64_t)count * map_env;
    j.resident = 1;
    j.first = first_slot;
    j.budget = step_budget;
    j.obs_env = obs_env;
    j.map_env = map_env;

    RangeArgs a{};
    a.spec0 = b->at<uint32_t>(r.spec0);
    a.spec1 = b->at<uint32_t>(r.spec1);
    a.spec2 = b->at<uint32_t>(r.spec2);
    a.terr = b->at<uint32_t>(r.terr);
    a.env_id = b->at<uint32_t>(r.env_id);
    a.tiles = b->at<Tile>(r.tiles);
    a.jobs = b->at<JobDesc>(r.jobs);
    a.job_err = b->at<uint32_t>(r.job_err);
    a.job = j;
    a.job_index = job;
    a.first = first_slot;
    a.count = count;
    a.clear = 0;
    a.s0 = s.height | (s.width << 8) | ((uint32_t)s.n_agents << 16) | ((uint32_t)s.n_seekers << 24);
    a.s1 = s.view_radius | ((uint32_t)s.n_channels << 4) | ((uint32_t)s.flags << 8) |
           ((uint32_t)s.episode_len << 16);
    a.s2 = s.wall_pct | ((uint32_t)board_words_per_row(s.width) << 8);
    a.env_id_base = env_id_base;
    a.lanes = lanes;
    const bool big = bk == N_BUCKETS - 1;
    a.variant = (uint32_t)(bk * 4 + s.view_radius - 1) | (mid ? COMBO_MID : 0u) |
                (arena_group(kind, (int)lanes, big, mid) << 8);
    if (s.flags & HASE_TERRAIN) {
        a.terr_words[0] = s.water_pct | ((uint32_t)s.mud_pct << 8) | ((uint32_t)s.stuck_pct << 16);
        for (int k = 0; k < 9; ++k) a.terr_words[1 + k / 4] |= (uint32_t)s.speed_pct[k] << (8 * (k % 4));
        a.terr_words[4] = (uint32_t)s.agent_classes;
        a.terr_words[5] = (uint32_t)(s.agent_classes >> 32);
    }
    HIP_TRY(launch_range(a, b->stream));
    InitArgs ia = make_init(b, seed, 0);
    ia.err = b->at<uint32_t>(r.job_err) + job;
    ia.env0 = first_slot;
    ia.n_envs = count;
    HIP_TRY(launch_init(ia, b->stream));
    if (out->err)
        HIP_TRY(hipMemcpyAsync(out->err, ia.err, 4, hipMemcpyDefault, b->stream));
    const uint32_t n_tiles = (count + E - 1) / E;
    if (out->obs0) {
        // the first observation: an observe-only launch over the range's tiles
        JobDesc j0 = j;
        j0.obs = out->obs0;
        j0.obs_stride = 0;
        if (mid)
            HIP_TRY(launch_combo(b->at<Tile>(r.tiles) + first_slot, n_tiles, nullptr, j0, 0, 0, slot_words,
                                 b->stream));
        else
            HIP_TRY(launch_mixed((int)lanes, kind, b->at<Tile>(r.tiles) + first_slot, n_tiles, nullptr,
                                 j0, 0, 0, slot_words, mwl, big, b->stream));
    }
    b->free_jobs.pop_back();
    b->ranges[first_slot] =
        hase_batch::Range{count, job, (uint32_t)kind, lanes, n_tiles, slot_words, mwl, big, mid};
    return HASE_OK;
}

int hase_release_range(hase_batch *b, uint32_t first_slot)
{
    if (!b) return fail(HASE_EINVAL, "null handle");
    if (!b->arena) return fail(HASE_EINVAL, "hase_release_range needs an arena");
    auto it = b->ranges.find(first_slot);
    if (it == b->ranges.end()) return fail(HASE_EINVAL, "no range starts at slot %u", first_slot);
    RangeArgs a{};
    a.tiles = b->at<Tile>(b->plan.reg.tiles);
    a.first = first_slot;
    a.count = it->second.count;
    a.clear = 1;
    HIP_TRY(launch_range(a, b->stream));
    b->free_jobs.push_back(it->second.job);
    b->ranges.erase(it);
    return HASE_OK;
}

int hase_range_error(hase_batch *b, uint32_t first_slot, int64_t *bad_env)
{
    if (!b || !bad_env) return fail(HASE_EINVAL, "null argument");
    if (!b->arena) return fail(HASE_EINVAL, "hase_range_error needs an arena");
    auto it = b->ranges.find(first_slot);
    if (it == b->ranges.end()) return fail(HASE_EINVAL, "no range starts at slot %u", first_slot);
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, b->d + b->plan.reg.job_err + 4ull * it->second.job, 4,
                           hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    *bad_env = err == 0xffffffffu ? -1 : (int64_t)err;
    return HASE_OK;
}

int hase_step_resident(hase_batch *b, uint32_t n_steps)
{
    if (!b) return fail(HASE_EINVAL, "null handle");
    if (!b->arena) return fail(HASE_EINVAL, "hase_step_resident needs an arena");
    if (n_steps == 0) return fail(HASE_EINVAL, "n_steps must be >= 1");
    // one launch per (kind, lanes) group over the tile entries up to the
    // group's last range (a wave skips entries of other groups and empty
    // ones); groups run concurrently on forked streams
    struct G {
        uint32_t kind, lanes, extent, slot, map;
        bool big, mid;
    };
    std::vector<G> groups;
    for (const auto &kv : b->ranges) {
        const hase_batch::Range &rg = kv.second;
        G *g = nullptr;
        for (G &x : groups)
            if (x.kind == rg.kind && x.lanes == rg.lanes && x.big == rg.big && x.mid == rg.mid) g = &x;
        if (!g) {
            groups.push_back(G{rg.kind, rg.lanes, 0u, rg.slot_words, rg.map_words, rg.big, rg.mid});
            g = &groups.back();
        }
        g->extent = std::max(g->extent, kv.first + rg.n_tiles);
    }
    if (groups.empty()) return HASE_OK;
    const bool fork = groups.size() > 1;
    if (fork) {
        const int rc = ensure_streams(b, groups.size());
        if (rc) return rc;
        HIP_TRY(hipEventRecord(b->fork_ev, b->stream));
    }
    const Tile *tiles = b->at<Tile>(b->plan.reg.tiles);
    const JobDesc *jobs = b->at<JobDesc>(b->plan.reg.jobs);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const G &g = groups[gi];
        JobDesc filter{};
        filter.group = arena_group((int)g.kind, (int)g.lanes, g.big, g.mid);
        hipStream_t st = b->stream;
        if (fork && gi > 0) {
            HIP_TRY(hipStreamWaitEvent(b->side[gi], b->fork_ev, 0));
            st = b->side[gi];
        }
        if (g.mid)
            HIP_TRY(launch_combo(tiles, g.extent, jobs, filter, n_steps, 0, g.slot, st));
        else
            HIP_TRY(launch_mixed((int)g.lanes, (int)g.kind, tiles, g.extent, jobs, filter, n_steps, 0,
                                 g.slot, g.map, g.big, st));
        if (fork && gi > 0) {
            HIP_TRY(hipEventRecord(b->join_ev[gi], st));
            HIP_TRY(hipStreamWaitEvent(b->stream, b->join_ev[gi], 0));
        }
    }
    return HASE_OK;
}

int hase_step_multi_static(const hase_step_io *io, uint32_t n, uint32_t n_steps, void *stream)
{
    if (n == 0) return HASE_OK;
    if (!io) return fail(HASE_EINVAL, "null argument");
    std::vector<hase_batch *> bs(n);
    for (uint32_t i = 0; i < n; ++i) bs[i] = io[i].batch;
    uint64_t need = 0;
    const int rc = hase_multi_workspace(bs.data(), n, &need);
    if (rc) return rc;
    if (need > STATIC_WORKSPACE_BYTES)
        return fail(HASE_ENOMEM,
                    "these requests need %llu bytes of job and tile tables; the static workspace "
                    "holds %zu (use hase_step_multi with a caller workspace)",
                    (unsigned long long)need, STATIC_WORKSPACE_BYTES);
    void *ws = nullptr;
    HIP_TRY(static_workspace(&ws));
    return hase_step_multi(io, n, n_steps, ws, STATIC_WORKSPACE_BYTES, stream);
}

int hase_destroy(hase_batch *b)
{
    if (!b) return HASE_OK;
    drop_graphs(b);
    for (int i = 0; i < MAX_LAUNCHES; ++i) {
        if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
        if (b->join_ev[i]) (void)hipEventDestroy(b->join_ev[i]);
    }
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    delete b;
    return HASE_OK;
}

const char *hase_strerror(int code)
{
    switch (code) {
    case HASE_OK: return "ok";
    case HASE_EINVAL: return "invalid argument";
    case HASE_ENOMEM: return "state buffer too small";
    case HASE_EGRID: return "an environment has too few free cells for its agents";
    case HASE_EHIP: return "HIP runtime error";
    case HASE_ESTATE: return "inconsistent state";
    case HASE_ENOTREADY: return "batch not reset";
    default: return "unknown error";
    }
}

const char *hase_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
