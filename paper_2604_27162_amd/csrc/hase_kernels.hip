// gfx950 kernels of the vectorised hide-and-seek step.
//
// step_kernel<LANES, NMAX>: one 64-lane wavefront steps a tile of 64/LANES
// environments; the LANES lanes of one env hold identical copies of its small
// state (agent positions, counters) in registers, resolve the sequential moves
// redundantly (no cross-lane traffic), and split the parallel work between
// them: generator blocks, reward stores and (agent, word) observation tasks.
// The env's padded wall bitboard is staged once per launch into the wave's
// LDS slot; a persistent launch (K > 1) then runs K steps with state in
// registers and only the outputs going to HBM.
//
// The rules are those of the paper's step loop (Sec. 4.1) reduced to a
// discrete gridworld: blocking tiles (Sec. 3.2), reward for locating hiders in
// a zero-sum game (Sec. 3, Sec. 3.1), Found flag (POIState F bit, Fig. "Bit
// Packing Environment Structure"), termination/truncation and reset from the
// unchanged grid (Sec. 4.1, 4.2), local-window decentralised observations
// (Sec. 3.3 mode 1). Integer work only: no MFMA.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hase_internal.h"

namespace hase {

// ------------------------------------------------------------ generator

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies with the output permutation (hi1^c1^k0, lo1, hi0^c3^k1, lo0),
// key bumped by the Weyl increments between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// Counter layout: (env id, stream << 24 | sub, a, b).
enum : uint32_t { ST_ACTION = 0u, ST_SPAWN = 1u, ST_WALL = 2u, ST_DESYNC = 3u };

// floor(x * m / 2^32)
__device__ __forceinline__ uint32_t range_map(uint32_t x, uint32_t m) { return __umulhi(x, m); }

// ------------------------------------------------------------ helpers

// Pointers read from descriptors are generic; casting them to the global
// address space lets the compiler use global_* (not flat_*) memory ops.
#define GAS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GAS T *gp(T *p)
{
    return (GAS T *)p;
}
template <class T>
__device__ __forceinline__ const GAS T *gp(const T *p)
{
    return (const GAS T *)p;
}

// OR over the LANES lanes of this env (aligned groups of LANES lanes).
template <int LANES>
__device__ __forceinline__ uint32_t group_or(uint32_t v)
{
#pragma unroll
    for (int m = 1; m < LANES; m <<= 1) v |= (uint32_t)__shfl_xor((int)v, m, 64);
    return v;
}

template <int LANES>
__device__ __forceinline__ uint64_t group_or64(uint64_t v)
{
    uint32_t lo = group_or<LANES>((uint32_t)v), hi = group_or<LANES>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Bit of the padded board at packed padded cell pc = y' << 8 | x'.
__device__ __forceinline__ uint32_t board_bit(const uint32_t *slot, int P, int pc)
{
    const int yy = pc >> 8, xx = pc & 0xff;
    return (slot[yy * P + (xx >> 5)] >> (xx & 31)) & 1u;
}

// Agent spawn for episode ep: agents in index order, up to 64 uniform draws
// each, first cell that is open and not held by an earlier agent; if every
// draw fails, the first acceptable cell scanning row-major from the cell after
// the last draw, wrapping around. Positions are packed padded cells.
template <int NMAX>
__device__ __forceinline__ void spawn_agents(int (&pp)[NMAX], int n, int H, int W,
                                             const uint32_t *slot, int P, uint32_t env,
                                             uint32_t k0, uint32_t k1, uint32_t ep)
{
    const uint32_t cells = (uint32_t)(H * W);
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
        if (i < n) {
            bool placed = false;
            uint32_t c = 0;
            for (uint32_t j = 0; j < (uint32_t)SPAWN_ATTEMPTS && !placed; ++j) {
                const U4 x = philox(env, (ST_SPAWN << 24) | (uint32_t)i, ep, j, k0, k1);
                c = range_map(x.x, cells);
                const uint32_t y = c / (uint32_t)W, xx = c - y * (uint32_t)W;
                const int pc = (int)(((y + PAD) << 8) | (xx + PAD));
                bool ok = board_bit(slot, P, pc) == 0u;
#pragma unroll
                for (int k = 0; k < i; ++k) ok = ok && (pp[k] != pc);
                if (ok) {
                    pp[i] = pc;
                    placed = true;
                }
            }
            for (uint32_t d = 1; d <= cells && !placed; ++d) {
                uint32_t cc = c + d;
                if (cc >= cells) cc -= cells;
                const uint32_t y = cc / (uint32_t)W, xx = cc - y * (uint32_t)W;
                const int pc = (int)(((y + PAD) << 8) | (xx + PAD));
                bool ok = board_bit(slot, P, pc) == 0u;
#pragma unroll
                for (int k = 0; k < i; ++k) ok = ok && (pp[k] != pc);
                if (ok) {
                    pp[i] = pc;
                    placed = true;
                }
            }
        }
    }
}

// ------------------------------------------------------------ step kernel

template <int LANES, int NMAX>
__global__ __launch_bounds__(64) void step_kernel(const Tile *__restrict__ tiles, uint32_t n_tiles,
                                                  const JobDesc *__restrict__ jobs, JobDesc job0,
                                                  uint32_t K, uint32_t step_base, uint32_t slot_words)
{
    extern __shared__ uint32_t lds[];
    const int lane = (int)threadIdx.x;
    const int q = lane / LANES;  // env slot in the tile
    const int l = lane % LANES;  // sub-lane within the env

    const uint32_t tile_id = blockIdx.x;
    if (tile_id >= n_tiles) return;
    const Tile tile = tiles[tile_id];
    const JobDesc J = jobs ? jobs[tile.job] : job0;
    const bool active = q < (int)tile.count;
    // inactive slots shadow the tile's first env and never store
    const uint32_t e = gp(J.tab.perm)[tile.env0 + (active ? (uint32_t)q : 0u)];

    const uint32_t s0 = gp(J.tab.spec0)[e], s1 = gp(J.tab.spec1)[e], s2 = gp(J.tab.spec2)[e];
    const int H = (int)(s0 & 0xffu), W = (int)((s0 >> 8) & 0xffu);
    const int n = (int)((s0 >> 16) & 0xffu), S = (int)(s0 >> 24);
    const int r = (int)(s1 & 0xfu), C = (int)((s1 >> 4) & 0xfu);
    const uint32_t flags = (s1 >> 8) & 0xffu, Lep = s1 >> 16;
    const int P = (int)((s2 >> 8) & 0xffu);
    const int D = 2 * r + 1;
    const int w = (D * D + 31) >> 5;
    const uint32_t dmask = (1u << D) - 1u;

    const uint32_t obs_off = gp(J.tab.obs_off)[e], agent_off = gp(J.tab.agent_off)[e];
    const uint32_t env = gp(J.tab.env_id)[e];
    const uint64_t seed = gp(J.seed)[e];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t found = gp(J.found)[e], t = gp(J.t)[e], ep = gp(J.ep)[e], steps = gp(J.steps)[e];

    // this env's LDS slot: padded bitboard, then per-agent positions and
    // detection counts (read by agent index, which differs between lanes)
    uint32_t *slot = lds + (uint32_t)q * (slot_words + 2 * NMAX);
    int *apos = (int *)(slot + slot_words);
    int *acnt = apos + NMAX;
    {
        const GAS uint32_t *src = gp(J.bb) + gp(J.tab.bb_off)[e];
        const int bw = (H + 2 * PAD) * P + 1;
        for (int i = l; i < bw; i += LANES) slot[i] = src[i];
    }

    // unused agent slots sit on a valid padded cell so that any speculated
    // board read of their (never applied) move target stays inside the slot
    int pp[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        int v = (PAD << 8) | PAD;
        if (j < n) {
            const uint32_t p = gp(J.pos)[agent_off + (uint32_t)j];
            v = (int)((((p >> 8) + PAD) << 8) | ((p & 0xffu) + PAD));
        }
        pp[j] = v;
    }
    __syncthreads();

    const uint32_t hmask = (uint32_t)(((1ull << n) - 1ull) & ~((1ull << S) - 1ull));
    const int ncalls = (n + 3) >> 2;
    const uint32_t Kj = K < J.k_limit ? K : J.k_limit;
    const bool obs_only = (K == 0);
    const uint32_t nsteps = obs_only ? 1u : Kj;
    // w in {1, 2, 3}: task / w for task < 64 via a multiply-shift
    const uint32_t winv = (65536u + (uint32_t)w - 1u) / (uint32_t)w;

    for (uint32_t k = 0; k < nsteps; ++k) {
        const uint64_t ostep = (uint64_t)J.out_step0 + step_base + k;

        if (!obs_only) {
            // ---- 1 actions: 3 bits per agent
            uint64_t acts = 0;
            for (int g = l; g < ncalls; g += LANES) {
                const U4 x = philox(env, (ST_ACTION << 24) | (uint32_t)g, steps, 0u, k0, k1);
                const uint32_t a4 = range_map(x.x, 5u) | (range_map(x.y, 5u) << 3) |
                                    (range_map(x.z, 5u) << 6) | (range_map(x.w, 5u) << 9);
                acts |= (uint64_t)a4 << (12 * g);
            }
            acts = group_or64<LANES>(acts);
            if (J.act) {
                const GAS int8_t *ap = gp(J.act) + ostep * J.agent_stride + agent_off;
                uint64_t ov = 0, om = 0;
                for (int j = l; j < n; j += LANES) {
                    const int v = ap[j];
                    if (v != -1) {
                        const uint32_t a = (v >= 0 && v <= 4) ? (uint32_t)v : 0u;
                        ov |= (uint64_t)a << (3 * j);
                        om |= 7ull << (3 * j);
                    }
                }
                ov = group_or64<LANES>(ov);
                om = group_or64<LANES>(om);
                acts = (acts & ~om) | ov;
            }

            // ---- 2 moves, agent-index order
            int tgt[NMAX];
            uint32_t open[NMAX];
#pragma unroll
            for (int i = 0; i < NMAX; ++i) {
                const uint32_t a = (uint32_t)(acts >> (3 * i)) & 7u;
                const int dlt = a == 1u ? -256 : a == 2u ? 256 : a == 3u ? 1 : a == 4u ? -1 : 0;
                tgt[i] = pp[i] + dlt;
                open[i] = (i < n && a != 0u) ? (board_bit(slot, P, tgt[i]) ^ 1u) : 0u;
            }
#pragma unroll
            for (int i = 0; i < NMAX; ++i) {
                bool mv = open[i] != 0u;
                if (flags & 1u) {
#pragma unroll
                    for (int j = 0; j < NMAX; ++j)
                        if (j != i) mv = mv && !(j < n && pp[j] == tgt[i]);
                }
                if (mv) pp[i] = tgt[i];
            }

            // ---- 3 detection: Chebyshev distance <= r between opposite roles
            int cnt[NMAX];
#pragma unroll
            for (int i = 0; i < NMAX; ++i) cnt[i] = 0;
#pragma unroll
            for (int i = 0; i < NMAX; ++i) {
#pragma unroll
                for (int j = i + 1; j < NMAX; ++j) {
                    const int dx = (pp[i] & 0xff) - (pp[j] & 0xff);
                    const int dy = (pp[i] >> 8) - (pp[j] >> 8);
                    const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
                    const bool seen = j < n && ((i < S) != (j < S)) && (ax > ay ? ax : ay) <= r;
                    cnt[i] += seen ? 1 : 0;
                    cnt[j] += seen ? 1 : 0;
                    // the hider of the pair is the higher index (seekers come first)
                    found |= seen ? (1u << j) : 0u;
                }
            }
#pragma unroll
            for (int j = 0; j < NMAX; ++j)
                if ((j % LANES) == l) acnt[j] = cnt[j];
            __syncthreads();
            if (active) {
                GAS float *rp = gp(J.rew) + ostep * J.agent_stride + agent_off;
                for (int a = l; a < n; a += LANES) {
                    const int c = acnt[a];
                    rp[a] = (float)(a < S ? c : -c);
                }
            }

            // ---- 4 termination / truncation
            t += 1u;
            const bool term = (flags & 2u) && n > S && (found & hmask) == hmask;
            const bool trunc = t >= Lep;
            const uint32_t d = (term ? 1u : 0u) | (trunc ? 2u : 0u);
            if (active && l == 0) gp(J.done)[ostep * J.env_stride + e] = (uint8_t)d;

            // ---- 5 same-step auto-reset from the unchanged grid
            if (d) {
                ep += 1u;
                t = 0u;
                found = 0u;
                spawn_agents<NMAX>(pp, n, H, W, slot, P, env, k0, k1, ep);
            }

            // ---- 6 generator step key
            steps += 1u;
        }

        // ---- 7 observations: task = agent * w + word
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
            if ((j % LANES) == l) apos[j] = pp[j];
        __syncthreads();
        if (active) {
            GAS uint32_t *ob = gp(J.obs) + ostep * J.obs_stride + obs_off;
            const int ntask = n * w;
            for (int task = l; task < ntask; task += LANES) {
                const int a = (int)(((uint32_t)task * winv) >> 16);
                const int wd = task - a * w;
                const int pa = apos[a];
                const int ax = pa & 0xff, ay = pa >> 8;
                const int col = ax - r;  // padded column of the window's left edge
                const int kbase = 32 * wd;
                // columns of the window outside the map
                const int lowc = PAD - col > 0 ? PAD - col : 0;
                const int hic = W + PAD - col;  // first window column right of the map
                const uint32_t colout = ((1u << lowc) - 1u) |
                                        (hic < D ? (dmask & ~((1u << hic) - 1u)) : 0u);
                uint32_t wall = 0, outside = 0, team = 0, opp = 0;
                for (int rho = 0; rho < D; ++rho) {
                    const int sh = rho * D - kbase + 32;
                    if (sh <= 32 - D || sh >= 64) continue;
                    const int row = ay - r + rho;
                    const uint32_t *rp = slot + row * P + (col >> 5);
                    const uint32_t bits = __builtin_amdgcn_alignbit(rp[1], rp[0], (uint32_t)(col & 31)) & dmask;
                    wall |= (uint32_t)(((uint64_t)bits << sh) >> 32);
                    const bool rowout = row < PAD || row >= H + PAD;
                    const uint32_t ob3 = rowout ? dmask : colout;
                    outside |= (uint32_t)(((uint64_t)ob3 << sh) >> 32);
                }
                const bool seeker = a < S;
#pragma unroll
                for (int j = 0; j < NMAX; ++j) {
                    const int dx = (pp[j] & 0xff) - ax + r;
                    const int dy = (pp[j] >> 8) - ay + r;
                    const int kk = dy * D + dx - kbase;
                    const bool in = j < n && j != a && (uint32_t)dx < (uint32_t)D &&
                                    (uint32_t)dy < (uint32_t)D && (uint32_t)kk < 32u;
                    const uint32_t bit = in ? (1u << (kk & 31)) : 0u;
                    if ((j < S) == seeker)
                        team |= bit;
                    else
                        opp |= bit;
                }
                GAS uint32_t *oa = ob + (uint32_t)(a * C * w + wd);
                oa[0] = wall;
                oa[w] = team;
                oa[2 * w] = opp;
                if (C == 4) oa[3 * w] = outside;
            }
        }
    }

    // write back the state
    if (active && !obs_only) {
        if (l == 0) {
            gp(J.found)[e] = found;
            gp(J.t)[e] = t;
            gp(J.ep)[e] = ep;
            gp(J.steps)[e] = steps;
        }
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            if (j < n && (j % LANES) == l) {
                const uint32_t x = (uint32_t)(pp[j] & 0xff) - PAD, y = (uint32_t)(pp[j] >> 8) - PAD;
                gp(J.pos)[agent_off + (uint32_t)j] = (uint16_t)(x | (y << 8));
            }
        }
    }
}

// ------------------------------------------------------------ init kernel

// One 64-lane block per env: walls from the generator (reset) or loaded
// (rebuild), padded bitboard, free-cell check, spawn of episode 0, desync.
__global__ __launch_bounds__(64) void init_kernel(InitArgs A)
{
    __shared__ uint8_t cellw[MAX_SIDE * MAX_SIDE];
    __shared__ uint32_t board[(MAX_SIDE + 2 * PAD) * 3 + 1];
    const uint32_t e = blockIdx.x;
    const int lane = (int)threadIdx.x;
    const uint32_t s0 = A.tab.spec0[e], s1 = A.tab.spec1[e], s2 = A.tab.spec2[e];
    const int H = (int)(s0 & 0xffu), W = (int)((s0 >> 8) & 0xffu);
    const int n = (int)((s0 >> 16) & 0xffu);
    const uint32_t flags = (s1 >> 8) & 0xffu, Lep = s1 >> 16;
    const uint32_t wall_pct = s2 & 0xffu;
    const int P = (int)((s2 >> 8) & 0xffu);
    const int cells = H * W;
    const uint32_t env = A.tab.env_id[e];
    uint8_t *walls = A.walls + A.tab.grid_off[e];
    const uint32_t k0 = (uint32_t)A.seed_value, k1 = (uint32_t)(A.seed_value >> 32);

    if (!A.rebuild_only) {
        // a cell is blocking iff its word is below floor(pct * 2^32 / 100)
        const uint32_t T = (uint32_t)(((uint64_t)wall_pct << 32) / 100u);
        for (int g = lane; 4 * g < cells; g += 64) {
            const U4 x = philox(env, (ST_WALL << 24) | (uint32_t)g, 0u, 0u, k0, k1);
            const uint32_t v[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int c = 4 * g + m;
                if (c < cells) {
                    const uint8_t b = v[m] < T ? 1 : 0;
                    cellw[c] = b;
                    walls[c] = b;
                }
            }
        }
    } else {
        for (int c = lane; c < cells; c += 64) cellw[c] = walls[c] ? 1 : 0;
    }
    __syncthreads();

    const int rows = H + 2 * PAD;
    const int bw = rows * P + 1;
    for (int i = lane; i < bw; i += 64) {
        uint32_t word = 0xffffffffu;  // slack word
        if (i < rows * P) {
            const int yy = i / P, j = i - (i / P) * P;
            word = 0;
            for (int b = 0; b < 32; ++b) {
                const int xx = 32 * j + b;
                const bool out = yy < PAD || yy >= H + PAD || xx < PAD || xx >= W + PAD;
                bool v = true;
                if (!out) v = cellw[(yy - PAD) * W + (xx - PAD)] != 0;
                word |= (v ? 1u : 0u) << b;
            }
        }
        board[i] = word;
        A.bb[A.tab.bb_off[e] + (uint32_t)i] = word;
    }
    __syncthreads();
    if (A.rebuild_only) return;

    int f = 0;
    for (int c = lane; c < cells; c += 64) f += cellw[c] ? 0 : 1;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) f += __shfl_xor(f, m, 64);
    if (f < n) {
        if (lane == 0) atomicMin(A.err, e);
        return;
    }
    if (lane == 0) {
        int pp[MAX_AGENTS];
#pragma unroll
        for (int j = 0; j < MAX_AGENTS; ++j) pp[j] = (PAD << 8) | PAD;
        spawn_agents<MAX_AGENTS>(pp, n, H, W, board, P, env, k0, k1, 0u);
        const uint32_t ao = A.tab.agent_off[e];
#pragma unroll
        for (int j = 0; j < MAX_AGENTS; ++j) {
            if (j < n) {
                const uint32_t x = (uint32_t)(pp[j] & 0xff) - PAD, y = (uint32_t)(pp[j] >> 8) - PAD;
                A.pos[ao + (uint32_t)j] = (uint16_t)(x | (y << 8));
            }
        }
        A.seed[e] = A.seed_value;
        A.found[e] = 0;
        A.ep[e] = 0;
        A.steps[e] = 0;
        uint32_t t0 = 0;
        if (flags & 4u) t0 = range_map(philox(env, ST_DESYNC << 24, 0u, 0u, k0, k1).x, Lep);
        A.t[e] = t0;
    }
}

// ------------------------------------------------------------ launchers

template <int LANES, int NMAX>
static hipError_t launch_variant(const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                                 const JobDesc &job0, uint32_t K, uint32_t step_base,
                                 uint32_t slot_words, hipStream_t stream)
{
    const size_t lds = (size_t)(64 / LANES) * (slot_words + 2 * NMAX) * sizeof(uint32_t);
    hipLaunchKernelGGL((step_kernel<LANES, NMAX>), dim3(n_tiles), dim3(64), lds, stream, tiles,
                       n_tiles, jobs, job0, K, step_base, slot_words);
    return hipGetLastError();
}

template <int LANES>
static hipError_t launch_lanes(int nmax, const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                               const JobDesc &job0, uint32_t K, uint32_t step_base,
                               uint32_t slot_words, hipStream_t stream)
{
    switch (nmax) {
    case 2: return launch_variant<LANES, 2>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 4: return launch_variant<LANES, 4>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 10: return launch_variant<LANES, 10>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 20: return launch_variant<LANES, 20>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    default: return hipErrorInvalidValue;
    }
}

bool variant_supported(int lanes, int nmax)
{
    const bool l_ok = lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32;
    const bool n_ok = nmax == 2 || nmax == 4 || nmax == 10 || nmax == 20;
    return l_ok && n_ok;
}

hipError_t launch_step(int lanes, int nmax, const Tile *tiles, uint32_t n_tiles,
                       const JobDesc *jobs, const JobDesc &job0, uint32_t K, uint32_t step_base,
                       uint32_t slot_words, hipStream_t stream)
{
    if (n_tiles == 0) return hipSuccess;
    switch (lanes) {
    case 1: return launch_lanes<1>(nmax, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 2: return launch_lanes<2>(nmax, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 4: return launch_lanes<4>(nmax, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 8: return launch_lanes<8>(nmax, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 16: return launch_lanes<16>(nmax, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 32: return launch_lanes<32>(nmax, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(const InitArgs &a, hipStream_t stream)
{
    if (a.n_envs == 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel, dim3(a.n_envs), dim3(64), 0, stream, a);
    return hipGetLastError();
}

}  // namespace hase
