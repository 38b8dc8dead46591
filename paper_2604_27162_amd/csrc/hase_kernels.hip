// gfx950 init kernel and the launch dispatchers of the hide-and-seek step
// (the step-kernel variants live in hase_step_l*.hip, one file per lanes
// value; their device code is in hase_device.h).

#include <mutex>

#include "hase_device.h"

namespace hase {

// ------------------------------------------------------------ static workspace

// The device workspace of hase_step_multi_static: the job and tile tables of
// a multi-batch step, for callers that cannot allocate device memory. Every
// GPU holds its own copy of this array until the process ends. In host code
// `scratch` names a host-side stand-in, not the device array: its device
// address comes from hipGetSymbolAddress, looked up once per device with
// that device current, and only that address is ever handed to HIP.
static __device__ __align__(256) unsigned char scratch[STATIC_WORKSPACE_BYTES];

hipError_t static_workspace(void **ptr)
{
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

// ------------------------------------------------------------ init kernel

// One 64-lane block per env: walls (terrain: tile types) from the generator
// (reset) or loaded (rebuild), padded board planes, free-cell check, spawn of
// episode 0, desync, empty discovery map (exploring envs), nobody stuck, no
// beliefs.
__global__ __launch_bounds__(64) void init_kernel(InitArgs A)
{
    __shared__ uint8_t cellw[MAX_SIDE * MAX_SIDE];
    __shared__ uint32_t board[2][(MAX_SIDE + 2 * PAD) * LDS_ROW + 1];
    __shared__ int spawned[MAX_AGENTS];
    const uint32_t e = A.env0 + blockIdx.x;
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
    const bool terrain = (flags & 32u) != 0u;
    // terrain word 0: water % | mud % << 8 | stuck % << 16; words 4, 5: classes
    const uint32_t tw0 = terrain ? A.tab.terr[8u * e] : 0u;
    const uint32_t clo = terrain ? A.tab.terr[8u * e + 4u] : 0u;
    const uint32_t chi = terrain ? A.tab.terr[8u * e + 5u] : 0u;

    if (!A.rebuild_only) {
        // a cell is blocking iff its word is below floor(pct * 2^32 / 100);
        // with terrain, water / mud below the cumulative thresholds
        const uint32_t T = (uint32_t)(((uint64_t)wall_pct << 32) / 100u);
        const uint32_t Tw = (uint32_t)(((uint64_t)(wall_pct + (tw0 & 0xffu)) << 32) / 100u);
        const uint32_t Tm =
            (uint32_t)(((uint64_t)(wall_pct + (tw0 & 0xffu) + ((tw0 >> 8) & 0xffu)) << 32) / 100u);
        for (int g = lane; 4 * g < cells; g += 64) {
            const U4 x = philox(env, (ST_WALL << 24) | (uint32_t)g, 0u, 0u, k0, k1);
            const uint32_t v[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int c = 4 * g + m;
                if (c < cells) {
                    uint8_t b = v[m] < T ? 1 : 0;
                    if (terrain && b == 0) b = v[m] < Tw ? 2 : (v[m] < Tm ? 3 : 0);
                    cellw[c] = b;
                    walls[c] = b;
                }
            }
        }
    } else {
        for (int c = lane; c < cells; c += 64)
            cellw[c] = terrain ? (uint8_t)(walls[c] & 3u) : (uint8_t)(walls[c] ? 1 : 0);
    }
    __syncthreads();

    // Board planes (plane 1 after plane 0, terrain only), rows of LDS_ROW
    // words whose words past P are 0, then a slack word of ones, in HBM and in
    // the LDS copies the spawn below reads, as in the step kernel; the HBM
    // boards end with zero words up to a multiple of 4. Plane 0: wall or mud
    // (outside: 1), plane 1: water or mud (outside: 0).
    const int rows = H + 2 * PAD;
    const int bw = rows * LDS_ROW + 1;
    const int planes = terrain ? 2 : 1;
    uint32_t *bb = A.bb + A.tab.bb_off[e];
    for (int pl = 0; pl < planes; ++pl) {
        for (int i = lane; i < bw; i += 64) {
            uint32_t word = 0xffffffffu;  // slack word
            const int yy = i / LDS_ROW, j = i - yy * LDS_ROW;
            if (i < rows * LDS_ROW) {
                word = 0;
                for (int b = 0; b < 32 && j < P; ++b) {
                    const int xx = 32 * j + b;
                    const bool out = yy < PAD || yy >= H + PAD || xx < PAD || xx >= W + PAD;
                    bool v = pl == 0;
                    if (!out) v = ((cellw[(yy - PAD) * W + (xx - PAD)] >> pl) & 1u) != 0;
                    word |= (v ? 1u : 0u) << b;
                }
            }
            board[pl][i] = word;
            bb[pl * bw + i] = word;
        }
    }
    for (int i = planes * bw + lane; i < round4(planes * bw); i += 64) bb[i] = 0u;
    if (!terrain)
        for (int i = lane; i < bw; i += 64) board[1][i] = 0u;
    __syncthreads();
    if (A.rebuild_only) return;
    if (flags & 16u) {
        uint32_t *map = A.disc + A.tab.map_off[e];
        for (int i = lane; i < H * ((W + 31) >> 5); i += 64) map[i] = 0u;
    }

    // room: free cells (plain), or the cells each class may stand on
    int f[3] = {0, 0, 0};  // walker, swimmer, flyer
    for (int c = lane; c < cells; c += 64) {
        const uint32_t ty = cellw[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) f[k] += (class_blocked((uint32_t)k, ty & 1u, ty >> 1) & 1u) ? 0 : 1;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) f[k] += __shfl_xor(f[k], m, 64);
    bool room = true;
    for (int i = 0; i < n; ++i) {
        const uint32_t c = agent_class(clo, chi, i);
        room = room && (c == 0u ? f[0] : (c == 1u ? f[1] : f[2])) >= n;
    }
    if (!room) {
        if (lane == 0) {
            atomicMin(A.err, e - A.env0);
            // a batch with such an env is refused; an arena range with one
            // is reported failed but may still be stepped until released, so
            // its agents get cells inside the map (the first cell)
            const uint32_t ao = A.tab.agent_off[e];
            for (int j = 0; j < n; ++j) A.pos[ao + (uint32_t)j] = 0;
            A.seed[e] = A.seed_value;
            A.found[e] = A.t[e] = A.ep[e] = A.steps[e] = A.stuck[e] = 0;
            for (int j = 0; j < n; ++j) A.bel[ao + (uint32_t)j] = 0u;
        }
        return;
    }
    if (lane == 0) {
        spawn_agents_if(spawned, n, H, W, env, k0, k1, 0u, [&](int i, int pc) {
            const int yy = pc >> 8, xx = pc & 0xff;
            const int wi = yy * LDS_ROW + (xx >> 5);
            const uint32_t b0 = (board[0][wi] >> (xx & 31)) & 1u, b1 = (board[1][wi] >> (xx & 31)) & 1u;
            return (class_blocked(agent_class(clo, chi, i), b0, b1) & 1u) == 0u;
        });
        const uint32_t ao = A.tab.agent_off[e];
        for (int j = 0; j < n; ++j) {
            const uint32_t x = (uint32_t)(spawned[j] & 0xff) - PAD, y = (uint32_t)(spawned[j] >> 8) - PAD;
            A.pos[ao + (uint32_t)j] = (uint16_t)(x | (y << 8));
        }
        A.seed[e] = A.seed_value;
        A.found[e] = 0;
        A.ep[e] = 0;
        A.steps[e] = 0;
        A.stuck[e] = 0;
        for (int j = 0; j < n; ++j) A.bel[ao + (uint32_t)j] = 0u;
        uint32_t t0 = 0;
        if (flags & 4u) t0 = range_map(philox(env, ST_DESYNC << 24, 0u, 0u, k0, k1).x, Lep);
        A.t[e] = t0;
    }
}

// ------------------------------------------------------------ launchers

// Variants exist for at most 4 agents per lane (larger ones would not unroll
// and would index registers dynamically).
bool variant_supported(int lanes, int nmax)
{
    const bool l_ok = lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16;
    const bool n_ok = nmax == 2 || nmax == 4 || nmax == 10 || nmax == 20;
    return l_ok && n_ok && (nmax + lanes - 1) / lanes <= 4;
}

hipError_t launch_step(int lanes, int nmax, int r, const Tile *tiles, uint32_t n_tiles,
                       const JobDesc *jobs, const JobDesc &job0, uint32_t K, uint32_t step_base,
                       uint32_t slot_words, hipStream_t stream)
{
    if (n_tiles == 0) return hipSuccess;
    switch (lanes) {
    case 1: return launch_step_lanes1(nmax, r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 2: return launch_step_lanes2(nmax, r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 4: return launch_step_lanes4(nmax, r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 8: return launch_step_lanes8(nmax, r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 16: return launch_step_lanes16(nmax, r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mixed(int lanes, int kind, const Tile *tiles, uint32_t n_tiles,
                        const JobDesc *jobs, const JobDesc &job0, uint32_t K, uint32_t step_base,
                        uint32_t slot_words, uint32_t map_words, bool big, hipStream_t stream)
{
    if (n_tiles == 0) return hipSuccess;
#define HASE_MIXED_CASE(L)                                                                          \
    case L:                                                                                         \
        if (kind == KIND_PLAIN)                                                                     \
            return launch_mixed_lanes##L(tiles, n_tiles, jobs, job0, K, step_base, slot_words,      \
                                         map_words, big, stream);                                        \
        if (kind & KIND_RADIO) {                                                                    \
            if (kind & KIND_TERRAIN)                                                                \
                return launch_radioter_lanes##L(kind, tiles, n_tiles, jobs, job0, K, step_base,     \
                                                slot_words, map_words, big, stream);                     \
            return launch_radio_lanes##L(kind, tiles, n_tiles, jobs, job0, K, step_base,            \
                                         slot_words, map_words, big, stream);                            \
        }                                                                                           \
        if (kind & KIND_TERRAIN)                                                                    \
            return launch_terr_lanes##L(kind, tiles, n_tiles, jobs, job0, K, step_base, slot_words, \
                                        map_words, big, stream);                                         \
        return launch_feat_lanes##L(kind, tiles, n_tiles, jobs, job0, K, step_base, slot_words,     \
                                    map_words, big, stream);
    switch (lanes) {
    HASE_MIXED_CASE(1)
    HASE_MIXED_CASE(2)
    HASE_MIXED_CASE(4)
    HASE_MIXED_CASE(8)
    HASE_MIXED_CASE(16)
    default: return hipErrorInvalidValue;
    }
#undef HASE_MIXED_CASE
}

hipError_t launch_init(const InitArgs &a, hipStream_t stream)
{
    if (a.n_envs == 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel, dim3(a.n_envs), dim3(64), 0, stream, a);
    return hipGetLastError();
}

// ------------------------------------------------------------ arena ranges

// One thread per slot of the range: its spec words, terrain words and env
// id, and its tile entry (slot first + i holds tile i of the range while i <
// the range's tile count, else an empty entry); thread 0 also writes the
// range's job descriptor and clears its error word. With clear, only the
// tile entries are emptied.
__global__ __launch_bounds__(256) void range_kernel(RangeArgs A)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.count) return;
    const uint32_t slot = A.first + i;
    Tile tl{0u, 0u, 0u, 0u};
    if (!A.clear) {
        A.spec0[slot] = A.s0;
        A.spec1[slot] = A.s1;
        A.spec2[slot] = A.s2;
        A.env_id[slot] = A.env_id_base + i;
        for (int k = 0; k < 8; ++k) A.terr[8u * slot + (uint32_t)k] = A.terr_words[k];
        const uint32_t E = 64u / A.lanes;  // envs per tile
        if (i * E < A.count) {
            tl.job = A.job_index;
            tl.env0 = A.first + i * E;
            tl.count = A.count - i * E < E ? A.count - i * E : E;
            tl.variant = A.variant;
        }
        if (i == 0) {
            A.jobs[A.job_index] = A.job;
            A.job_err[A.job_index] = 0xffffffffu;
        }
    }
    A.tiles[slot] = tl;
}

hipError_t launch_range(const RangeArgs &a, hipStream_t stream)
{
    if (a.count == 0) return hipSuccess;
    hipLaunchKernelGGL(range_kernel, dim3((a.count + 255) / 256), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace hase
