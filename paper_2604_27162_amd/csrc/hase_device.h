// gfx950 device code of the vectorised hide-and-seek step (included by the
// per-lanes translation units hase_step_l*.hip and by hase_kernels.hip).
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

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "hase_internal.h"

namespace hase {

// ------------------------------------------------------------ generator

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies with the output permutation (hi1^c1^k0, lo1, hi0^c3^k1, lo0),
// key bumped by the Weyl increments between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

// a ^ b ^ c in one instruction (gfx950 three-input bitwise op, truth table
// 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
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
enum : uint32_t { ST_ACTION = 0u, ST_SPAWN = 1u, ST_WALL = 2u, ST_DESYNC = 3u, ST_MOVE = 4u, ST_RADIO = 5u };

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

// Bit of the padded board in LDS (rows of LDS_ROW words) at packed padded
// cell pc = y' << 8 | x'.
__device__ __forceinline__ uint32_t board_bit(const uint32_t *slot, int pc)
{
    const int yy = pc >> 8, xx = pc & 0xff;
    return (slot[yy * LDS_ROW + (xx >> 5)] >> (xx & 31)) & 1u;
}

// Agent spawn for episode ep: agents in index order, up to 64 uniform draws
// each, first cell that agent i may stand on (ok(i, cell)) and no earlier
// agent holds; if every draw fails, the first acceptable cell scanning
// row-major from the cell after the last draw, wrapping around. Positions
// (packed padded cells) are written to out[0..n) in LDS; the loops are not
// unrolled (spawning is rare), and all lanes of an env may run it together
// since they write identical values.
template <typename OK>
__device__ __forceinline__ void spawn_agents_if(int *out, int n, int H, int W, uint32_t env,
                                                uint32_t k0, uint32_t k1, uint32_t ep, OK ok_fn)
{
    const uint32_t cells = (uint32_t)(H * W);
    for (int i = 0; i < n; ++i) {
        bool placed = false;
        uint32_t c = 0;
        for (uint32_t j = 0; j < (uint32_t)SPAWN_ATTEMPTS && !placed; ++j) {
            const U4 x = philox(env, (ST_SPAWN << 24) | (uint32_t)i, ep, j, k0, k1);
            c = range_map(x.x, cells);
            const uint32_t y = c / (uint32_t)W, xx = c - y * (uint32_t)W;
            const int pc = (int)(((y + PAD) << 8) | (xx + PAD));
            bool ok = ok_fn(i, pc);
            for (int k = 0; k < i && ok; ++k) ok = out[k] != pc;
            if (ok) {
                out[i] = pc;
                placed = true;
            }
        }
        for (uint32_t d = 1; d <= cells && !placed; ++d) {
            uint32_t cc = c + d;
            if (cc >= cells) cc -= cells;
            const uint32_t y = cc / (uint32_t)W, xx = cc - y * (uint32_t)W;
            const int pc = (int)(((y + PAD) << 8) | (xx + PAD));
            bool ok = ok_fn(i, pc);
            for (int k = 0; k < i && ok; ++k) ok = out[k] != pc;
            if (ok) {
                out[i] = pc;
                placed = true;
            }
        }
        // No room at all (only an arena range reported failed at its reset
        // gets here): the agent takes its last drawn cell, inside the map.
        if (!placed) {
            const uint32_t y = c / (uint32_t)W, xx = c - y * (uint32_t)W;
            out[i] = (int)(((y + PAD) << 8) | (xx + PAD));
        }
    }
}

// ------------------------------------------------------------ terrain

// Tile types are two board planes (plane 0 = wall or mud, plane 1 = water or
// mud; outside reads as wall: 1, 0). Agent classes: 0 walker (ground, mud),
// 1 swimmer (water), 2 flyer (anything but walls). Cells an agent of class
// cls may not enter, from plane bits b0, b1 (any width of bits at once).
__device__ __forceinline__ uint32_t class_blocked(uint32_t cls, uint32_t b0, uint32_t b1)
{
    // masks, not a conditional: the compiler turned the three-way choice on
    // a per-lane class into branches
    const uint32_t m0 = 0u - (cls == 0u ? 1u : 0u), m1 = 0u - (cls == 1u ? 1u : 0u);
    return ((b0 ^ b1) & m0) | ((b0 | ~b1) & m1) | ((b0 & ~b1) & ~(m0 | m1));
}

// Class of agent i from the two class words (2 bits per agent).
__device__ __forceinline__ uint32_t agent_class(uint32_t lo, uint32_t hi, int i)
{
    return ((i < 16 ? lo : hi) >> (2 * (i & 15))) & 3u;
}

// a or b as a value. A conditional expression over two variables is an lvalue,
// which clang may lower to a select of their addresses; with variables that
// lambdas capture by reference, that kept them (and a table of their
// addresses) in scratch memory.
__device__ __forceinline__ uint32_t pick(bool c, uint32_t a, uint32_t b) { return c ? a : b; }

// A uniform word x meets a chance of pct percent: x / 2^32 < pct / 100.
__device__ __forceinline__ bool chance(uint32_t x, uint32_t pct)
{
    return (uint64_t)x * 100u < ((uint64_t)pct << 32);
}

// ------------------------------------------------------------ step kernel

// OR over the LANES lanes of one env with DPP moves inside 16-lane rows
// (quad swaps, half-row and row mirrors); 32-lane groups add one shuffle.
template <int LANES>
__device__ __forceinline__ uint32_t group_or_dpp(uint32_t v)
{
    if constexpr (LANES >= 2) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    if constexpr (LANES >= 4) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    if constexpr (LANES >= 8) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
    if constexpr (LANES >= 16) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);
    if constexpr (LANES >= 32) v |= (uint32_t)__shfl_xor((int)v, 16, 64);
    return v;
}

// Each block is one wavefront: its lanes run in lockstep and its LDS
// operations complete in issue order, so sharing values through LDS between
// lanes needs only a compiler ordering point (a wavefront-scope fence emits
// no wait on outstanding global stores).
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Window rows of one agent into W-word bitmasks (bit k = row * D + column),
// fully unrolled for radius R: wall|outside from the padded board (TER: the
// cells the agent's class cls may not enter, from the two tile planes, plane
// 1 pw words after plane 0, and, when lw is given, the walls and outside
// alone, which block sight) and, for 4-channel envs, outside-the-map only.
template <int R, int W, bool TER = false>
__device__ __forceinline__ void window_rows(const uint32_t *slot, int H, int Wd, int ax, int ay,
                                            bool want_out, uint32_t (&wall)[W], uint32_t (&outm)[W],
                                            int pw = 0, uint32_t cls = 0u,
                                            uint32_t (*lw)[W] = nullptr)
{
    constexpr int D = 2 * R + 1;
    constexpr uint32_t DM = (1u << D) - 1u;
    const int col = ax - R;  // padded column of the window's left edge
    // one base address; the rows are at constant offsets from it
    const uint32_t *base = slot + (ay - R) * LDS_ROW + (col >> 5);
    const uint32_t sh = (uint32_t)(col & 31);
#pragma unroll
    for (int rho = 0; rho < D; ++rho) {
        const uint32_t *rp = base + rho * LDS_ROW;
        uint32_t bits = __builtin_amdgcn_alignbit(rp[1], rp[0], sh);
        const int off = rho * D, wi = off >> 5, b = off & 31;
        if constexpr (TER) {
            const uint32_t b1 = __builtin_amdgcn_alignbit(rp[pw + 1], rp[pw], sh);
            if (lw != nullptr) {
                const uint32_t wb = bits & ~b1 & DM;  // wall type (outside reads as wall)
                (*lw)[wi] |= wb << b;
                if (b + D > 32) (*lw)[wi + 1] |= wb >> (32 - b);
            }
            bits = class_blocked(cls, bits, b1);
        }
        bits &= DM;
        wall[wi] |= bits << b;
        if (b + D > 32) wall[wi + 1] |= bits >> (32 - b);
    }
    if (want_out) {
        // columns of the window left / right of the map
        const int lowc = PAD - col > 0 ? PAD - col : 0;
        const int hic = Wd + PAD - col;
        const uint32_t colout = ((1u << lowc) - 1u) | (hic < D ? (DM & ~((1u << hic) - 1u)) : 0u);
#pragma unroll
        for (int rho = 0; rho < D; ++rho) {
            const int row = ay - R + rho;
            const uint32_t ob = (uint32_t)(row - PAD) >= (uint32_t)H ? DM : colout;
            const int off = rho * D, wi = off >> 5, b = off & 31;
            outm[wi] |= ob << b;
            if (b + D > 32) outm[wi + 1] |= ob >> (32 - b);
        }
    }
}

// Windows of radius R over the env's two agent planes (seekers at pl, hiders
// pw words later; the board's padded row layout, no bits outside the map):
// bit k = row * D + column, as for the walls.
template <int R, int W>
__device__ __forceinline__ void plane_windows(const uint32_t *pl, int pw, int ax, int ay,
                                              uint32_t (&sk)[W], uint32_t (&hd)[W])
{
    constexpr int D = 2 * R + 1;
    constexpr uint32_t DM = (1u << D) - 1u;
    const int col = ax - R;
    const uint32_t *base = pl + (ay - R) * LDS_ROW + (col >> 5);
    const uint32_t sh = (uint32_t)(col & 31);
#pragma unroll
    for (int i = 0; i < W; ++i) sk[i] = hd[i] = 0u;
#pragma unroll
    for (int rho = 0; rho < D; ++rho) {
        const uint32_t *rp = base + rho * LDS_ROW;
        const uint32_t s = __builtin_amdgcn_alignbit(rp[1], rp[0], sh) & DM;
        const uint32_t h = __builtin_amdgcn_alignbit(rp[pw + 1], rp[pw], sh) & DM;
        const int off = rho * D, wi = off >> 5, b = off & 31;
        sk[wi] |= s << b;
        hd[wi] |= h << b;
        if (b + D > 32) {
            sk[wi + 1] |= s >> (32 - b);
            hd[wi + 1] |= h >> (32 - b);
        }
    }
}

// Word and bit of packed padded cell pc in a plane of the board's layout.
__device__ __forceinline__ uint32_t plane_word(int pc) { return (uint32_t)((pc >> 8) * LDS_ROW + ((pc & 0xff) >> 5)); }
__device__ __forceinline__ uint32_t plane_bit(int pc) { return 1u << (pc & 31); }

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// Every lane of a 2- or 4-lane group gets the 12-bit blocks of all lanes of
// its group, in lane order, via DPP broadcasts (quad_perm patterns).
// Value of lane k of the caller's env (its LANES consecutive lanes, 2 or 4:
// a quad permutation within the env's quad or pair of lanes).
template <int LANES>
__device__ __forceinline__ uint32_t env_lane_bcast(uint32_t v, int k)
{
    static_assert(LANES == 2 || LANES == 4, "quad broadcasts serve 2 or 4 lanes per env");
    if constexpr (LANES == 4) {
        switch (k) {
        case 0: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x00, 0xF, 0xF, false);
        case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x55, 0xF, 0xF, false);
        case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xAA, 0xF, 0xF, false);
        default: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xFF, 0xF, 0xF, false);
        }
    } else {
        // quad_perm [0, 0, 2, 2] or [1, 1, 3, 3]
        if (k == 0) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xA0, 0xF, 0xF, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xF5, 0xF, 0xF, false);
    }
}

// Value of lane k of the caller's env when the env has 8 or 16 lanes (DPP
// row broadcast of lane k of each 16-lane row; with 8 lanes per env the
// upper env of a row takes lane 8 + k).
template <int LANES>
__device__ __forceinline__ uint32_t env_bcast(uint32_t v, int k)
{
    static_assert(LANES == 8 || LANES == 16, "row broadcasts serve 8 or 16 lanes per env");
    uint32_t lo = 0u, hi = 0u;
    switch (k) {
#define HASE_BCAST(K)                                                                          \
    case K:                                                                                    \
        lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + (K), 0xF, 0xF, false);   \
        if constexpr (LANES == 8)                                                              \
            hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x158 + ((K) & 7), 0xF, 0xF, false); \
        break;
        HASE_BCAST(0) HASE_BCAST(1) HASE_BCAST(2) HASE_BCAST(3) HASE_BCAST(4) HASE_BCAST(5)
        HASE_BCAST(6) HASE_BCAST(7) HASE_BCAST(8) HASE_BCAST(9) HASE_BCAST(10) HASE_BCAST(11)
        HASE_BCAST(12) HASE_BCAST(13) HASE_BCAST(14) HASE_BCAST(15)
#undef HASE_BCAST
    default: break;
    }
    if constexpr (LANES == 8) return (threadIdx.x & 8u) ? hi : lo;
    return lo;
}

template <int LANES>
__device__ __forceinline__ uint64_t gather_window(uint32_t v)
{
    if constexpr (LANES == 4) {
        return (uint64_t)dpp_mov<0x00>(v) | ((uint64_t)dpp_mov<0x55>(v) << 12) |
               ((uint64_t)dpp_mov<0xAA>(v) << 24) | ((uint64_t)dpp_mov<0xFF>(v) << 36);
    } else {
        return (uint64_t)dpp_mov<0xA0>(v) | ((uint64_t)dpp_mov<0xF5>(v) << 12);
    }
}

// mine[m] = pp[l + m * LANES] (pp[0] when that agent does not exist) with
// compile-time register indices only (a select per candidate agent), so the
// positions never leave registers.
template <int LANES, int NMAX, int TPL>
__device__ __forceinline__ void own_positions(const int (&pp)[NMAX], int l, int n, int (&mine)[TPL])
{
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
        int a = l + m * LANES;
        // With many agents the compares a == i, hoisted out of the step loop
        // as lane masks, would not fit the scalar registers (they would be
        // spilled to vector lanes and read back every step): an empty asm
        // makes a opaque here, so each compare is redone on the vector unit.
        if constexpr (NMAX > 4) asm volatile("" : "+v"(a));
        int v = pp[0];
#pragma unroll
        for (int i = 1; i < NMAX; ++i) v = (a == i) ? pp[i] : v;
        mine[m] = a < n ? v : pp[0];
    }
}

// Positions of the agents whose indices a lane's tasks hold (aid[m] < n).
template <int NMAX, int TPL>
__device__ __forceinline__ void own_positions_ids(const int (&pp)[NMAX], const int (&aid)[TPL],
                                                  int (&mine)[TPL])
{
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
        int v = pp[0];
#pragma unroll
        for (int i = 1; i < NMAX; ++i) v = (aid[m] == i) ? pp[i] : v;
        mine[m] = v;
    }
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));

// W contiguous words in one vector store
template <int W>
__device__ __forceinline__ void store_words(GAS uint32_t *p, const uint32_t (&v)[W])
{
    if constexpr (W == 1) {
        p[0] = v[0];
    } else if constexpr (W == 2) {
        u32x2 x;
        x.x = v[0];
        x.y = v[1];
        *(GAS u32x2 *)p = x;
    } else {
        u32x3 x;
        x.x = v[0];
        x.y = v[1];
        x.z = v[2];
        *(GAS u32x3 *)p = x;
    }
}

// Parking cell of unused agent slots (packed padded coordinates): never in
// any window and never equal to a move target, so the inner loops need no
// agent-count test.
constexpr int FAR_CELL = (0xF0 << 8) | 0xF0;
// a draw the agent may not take (above every packed cell)
constexpr uint32_t NO_CELL = 0xffffu;

// Move-target offsets of actions 0..4 (stay, N, S, E, W) as packed
// (dy << 8) + dx + 257, 12 bits per action.
constexpr uint64_t MOVE_TABLE = 0x101ull | (0x001ull << 12) | (0x201ull << 24) |
                                (0x102ull << 36) | (0x100ull << 48);

// Channels of one agent at packed padded cell pa: window rows of the board
// (wall|outside and, when want_out, outside only) and the other agents by
// role. exact == false assumes agents occupy distinct cells (collisions on):
// the opponent count is then the popcount of the opponent window and the
// only agent on the centre cell is the agent itself. exact == true tests
// every other agent by index. Returns the number of other-role agents in the
// window (Chebyshev distance <= R).
template <int R, int W, int NMAX, bool EXACT, bool TER = false, bool PLN = false>
__device__ __forceinline__ int agent_masks_raw(const uint32_t *slot, int H, int Wd,
                                           const int (&pp)[NMAX], int a, int pa, int n, int S,
                                           bool want_out, uint32_t (&wall)[W], uint32_t (&outm)[W],
                                           uint32_t (&team)[W], uint32_t (&opp)[W], int pw = 0,
                                           uint32_t cls = 0u, uint32_t (*lw)[W] = nullptr,
                                           const uint32_t *planes = nullptr, int plw = 0)
{
    constexpr int D = 2 * R + 1;
    constexpr int CENTER = R * D + R;
#pragma unroll
    for (int i = 0; i < W; ++i) wall[i] = outm[i] = team[i] = opp[i] = 0u;
    if (lw != nullptr) {
#pragma unroll
        for (int i = 0; i < W; ++i) (*lw)[i] = 0u;
    }
    const int ax = pa & 0xff, ay = pa >> 8;
    window_rows<R, W, TER>(slot, H, Wd, ax, ay, want_out, wall, outm, pw, cls, lw);
    const bool sa = a < S;
    if constexpr (!EXACT && NMAX <= 4) {
        // Distinct cells: the agent itself is the centre (in no channel) and
        // the others are the NMAX - 1 agents k (k < a) or k + 1 (k >= a). One
        // packed difference u = (dy + R) << 8 | (dx + R) gives both the
        // window test and the bit index (an agent outside the window makes
        // a byte of u at least D: coordinates differ by less than 256 - D).
        const uint32_t base = (uint32_t)(R * 256 + R) - (uint32_t)pa;
        uint64_t tm = 0, op = 0;
        uint32_t tm_hi = 0, op_hi = 0;  // window bits 64.. (radius 4 only)
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < NMAX - 1; ++k) {
            const bool up = k >= a;
            const uint32_t u = (uint32_t)(up ? pp[k + 1] : pp[k]) + base;
            const bool same = ((up ? k + 1 : k) < S) == sa;
            const uint32_t lo = u & 0xffu, hi = u >> 8;
            const bool in = (lo > hi ? lo : hi) < (uint32_t)D;
            const uint32_t kk = (uint32_t)__umul24(hi, (uint32_t)D) + lo;
            if constexpr (W <= 2) {
                const uint64_t bit = in ? (1ull << (kk & 63u)) : 0ull;
                tm |= same ? bit : 0ull;
                op |= same ? 0ull : bit;
            } else {
                const uint64_t bit = (in && kk < 64u) ? (1ull << (kk & 63u)) : 0ull;
                const uint32_t bh = (in && kk >= 64u) ? (1u << (kk & 31u)) : 0u;
                tm |= same ? bit : 0ull;
                op |= same ? 0ull : bit;
                tm_hi |= same ? bh : 0u;
                op_hi |= same ? 0u : bh;
            }
            cnt += (in && !same) ? 1 : 0;
        }
        team[0] = (uint32_t)tm;
        opp[0] = (uint32_t)op;
        if constexpr (W >= 2) {
            team[1] = (uint32_t)(tm >> 32);
            opp[1] = (uint32_t)(op >> 32);
        }
        if constexpr (W == 3) {
            team[2] = tm_hi;
            opp[2] = op_hi;
        }
        return cnt;
    } else if constexpr (!EXACT && PLN) {
        // Distinct cells, one agent per lane: the env's seeker and hider
        // planes (kept up to date by the agents' own lanes) read like the
        // walls; the agent's own bit is the centre of its own role's window.
        uint32_t skw[W], hdw[W];
        plane_windows<R, W>(planes, plw, pa & 0xff, pa >> 8, skw, hdw);
        const bool sa = a < S;
        int cnt = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            team[i] = sa ? skw[i] : hdw[i];
            opp[i] = sa ? hdw[i] : skw[i];
            cnt += __builtin_popcount(opp[i]);
        }
        team[CENTER >> 5] &= ~(1u << (CENTER & 31));
        return cnt;
    } else if constexpr (!EXACT) {
        // Bits of all agents in the window, and of the seekers among them,
        // from the packed difference u = (dy + R) << 8 | (dx + R) (see above);
        // a shifted 0/1 word carries the window test, and the seeker masks
        // are loop-invariant words, so no lane-mask logic is needed.
        const uint32_t base = (uint32_t)(R * 256 + R) - (uint32_t)pa;
        uint64_t all = 0, sk = 0;
        uint32_t all_hi = 0, sk_hi = 0;  // window bits 64.. (radius 4 only)
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            const uint32_t u = (uint32_t)pp[j] + base;
            const uint32_t lo = u & 0xffu, hi = u >> 8;
            const uint32_t in = (lo > hi ? lo : hi) < (uint32_t)D ? 1u : 0u;
            const uint32_t kk = (uint32_t)__umul24(hi, (uint32_t)D) + lo;
            const uint32_t skm = j < S ? 0xffffffffu : 0u;
            const uint64_t skm64 = ((uint64_t)skm << 32) | skm;
            const uint64_t bit = (uint64_t)in << (kk & 63u);
            if constexpr (W <= 2) {
                all |= bit;
                sk |= bit & skm64;
            } else {
                const bool low = kk < 64u;
                const uint64_t b01 = low ? bit : 0ull;
                const uint32_t b2 = low ? 0u : (uint32_t)bit;
                all |= b01;
                sk |= b01 & skm64;
                all_hi |= b2;
                sk_hi |= b2 & skm;
            }
        }
        const uint64_t hd = all & ~sk;
        const uint64_t tm = sa ? sk : hd, op = sa ? hd : sk;
        team[0] = (uint32_t)tm;
        opp[0] = (uint32_t)op;
        int cnt = __builtin_popcount((uint32_t)op);
        if constexpr (W >= 2) {
            team[1] = (uint32_t)(tm >> 32);
            opp[1] = (uint32_t)(op >> 32);
            cnt += __builtin_popcount((uint32_t)(op >> 32));
        }
        if constexpr (W == 3) {
            const uint32_t hd_hi = all_hi & ~sk_hi;
            team[2] = sa ? sk_hi : hd_hi;
            opp[2] = sa ? hd_hi : sk_hi;
            cnt += __builtin_popcount(opp[2]);
        }
        team[CENTER >> 5] &= ~(1u << (CENTER & 31));
        return cnt;
    } else {
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            const int dx = (pp[j] & 0xff) - ax + R;
            const int dy = (pp[j] >> 8) - ay + R;
            const bool in = j < n && j != a && (uint32_t)dx < (uint32_t)D && (uint32_t)dy < (uint32_t)D;
            const int kk = __umul24((uint32_t)dy, (uint32_t)D) + dx;
            const uint32_t bit = in ? (1u << (kk & 31)) : 0u;
            const bool same = (j < S) == sa;
            cnt += (in && !same) ? 1 : 0;
#pragma unroll
            for (int i = 0; i < W; ++i) {
                const uint32_t bi = (kk >> 5) == i ? bit : 0u;
                team[i] |= same ? bi : 0u;
                opp[i] |= same ? 0u : bi;
            }
        }
        return cnt;
    }
}

// ------------------------------------------------------------ line of sight

// Does the open segment from the centre of window cell (0,0) to the centre of
// (dx,dy) pass through the inside of the unit square of cell (ex,ey)? Both
// are open convex sets, so they meet iff no separating axis exists among the
// square's edge normals (x, y) and the segment's normal (-dy, dx): along x and
// y their open projections must overlap, along the normal the square's corners
// must lie strictly on both sides of the segment's line. Doubled coordinates
// keep every quantity an integer.
constexpr bool seg_cuts_cell(int dx, int dy, int ex, int ey)
{
    auto overlap = [](int a0, int a1, int b0, int b1) {
        return (a0 > b0 ? a0 : b0) < (a1 < b1 ? a1 : b1);
    };
    const int lx = dx < 0 ? dx : 0, hx = dx < 0 ? 0 : dx;
    const int ly = dy < 0 ? dy : 0, hy = dy < 0 ? 0 : dy;
    if (dx == 0 ? ex != 0 : !overlap(2 * lx, 2 * hx, 2 * ex - 1, 2 * ex + 1)) return false;
    if (dy == 0 ? ey != 0 : !overlap(2 * ly, 2 * hy, 2 * ey - 1, 2 * ey + 1)) return false;
    int fmin = 0x7fffffff, fmax = -0x7fffffff;
    for (int sx = -1; sx <= 1; sx += 2) {
        for (int sy = -1; sy <= 1; sy += 2) {
            const int f = -dy * (2 * ex + sx) + dx * (2 * ey + sy);
            fmin = f < fmin ? f : fmin;
            fmax = f > fmax ? f : fmax;
        }
    }
    return fmin < 0 && 0 < fmax;
}

// Shadow table of radius R: for each cell b within Chebyshev distance R - 1
// of the centre (only those can lie strictly between the centre and a window
// cell), its window bit and the window cells whose segment from the centre
// passes through b's inside (bit k = (dy + R)(2R + 1) + dx + R).
template <int R>
struct LosTable {
    static constexpr int D = 2 * R + 1;
    static constexpr int W = (D * D + 31) / 32;
    static constexpr int NB = (2 * R - 1) * (2 * R - 1) - 1;
    int bit[NB > 0 ? NB : 1];
    uint32_t shadow[NB > 0 ? NB : 1][W];
    constexpr LosTable() : bit(), shadow()
    {
        int i = 0;
        for (int ey = -(R - 1); ey <= R - 1; ++ey) {
            for (int ex = -(R - 1); ex <= R - 1; ++ex) {
                if (ex == 0 && ey == 0) continue;
                bit[i] = (ey + R) * D + ex + R;
                for (int w = 0; w < W; ++w) shadow[i][w] = 0u;
                for (int dy = -R; dy <= R; ++dy) {
                    for (int dx = -R; dx <= R; ++dx) {
                        if (dx == ex && dy == ey) continue;
                        if (seg_cuts_cell(dx, dy, ex, ey)) {
                            const int k = (dy + R) * D + dx + R;
                            shadow[i][k >> 5] |= 1u << (k & 31);
                        }
                    }
                }
                ++i;
            }
        }
    }
};

template <int R>
inline constexpr LosTable<R> LOS_TABLE{};

// occ |= shadow of blocker I when the window shows a blocking cell there. The
// table entries are constexpr locals (template indices only), so they are
// immediate constants of the kernel and zero words cost nothing.
template <int R, int W, int I, int WI>
__device__ __forceinline__ void los_word(uint32_t (&occ)[W], uint32_t m)
{
    constexpr uint32_t sh = LOS_TABLE<R>.shadow[I][WI];
    if constexpr (sh != 0u) occ[WI] |= sh & m;
}

template <int R, int W, int I, int... WI>
__device__ __forceinline__ void los_one(const uint32_t (&wall)[W], uint32_t (&occ)[W],
                                        std::integer_sequence<int, WI...>)
{
    constexpr int b = LOS_TABLE<R>.bit[I];
    const uint32_t m = 0u - ((wall[b >> 5] >> (b & 31)) & 1u);
    (los_word<R, W, I, WI>(occ, m), ...);
}

template <int R, int W, int... I>
__device__ __forceinline__ void los_all(const uint32_t (&wall)[W], uint32_t (&occ)[W],
                                        std::integer_sequence<int, I...>)
{
    (los_one<R, W, I>(wall, occ, std::make_integer_sequence<int, W>{}), ...);
}

// Visible window cells of an agent from its wall|outside window: every cell
// not in the shadow of a blocking cell.
template <int R, int W>
__device__ __forceinline__ void los_visible(const uint32_t (&wall)[W], uint32_t (&vis)[W])
{
    uint32_t occ[W];
#pragma unroll
    for (int w = 0; w < W; ++w) occ[w] = 0u;
    if constexpr (LosTable<R>::NB > 0)
        los_all<R, W>(wall, occ, std::make_integer_sequence<int, LosTable<R>::NB>{});
#pragma unroll
    for (int w = 0; w < W; ++w) vis[w] = ~occ[w];
}

// Line of sight: the channels of one agent restricted to the cells visible
// from its own (vis, from the window of sight blockers: walls and outside),
// and the count of the visible opponents.
template <int R, int W, int NMAX, bool EXACT>
__device__ __forceinline__ int occlude(const int (&pp)[NMAX], int a, int pa, int n, int S,
                                       const uint32_t (&blockers)[W], uint32_t (&wall)[W],
                                       uint32_t (&outm)[W], uint32_t (&team)[W],
                                       uint32_t (&opp)[W], uint32_t (&vis)[W])
{
    los_visible<R, W>(blockers, vis);
#pragma unroll
    for (int i = 0; i < W; ++i) {
        wall[i] &= vis[i];
        outm[i] &= vis[i];
        team[i] &= vis[i];
        opp[i] &= vis[i];
    }
    int cnt = 0;
    if constexpr (!EXACT) {
        // distinct cells: one opponent per opponent bit
#pragma unroll
        for (int i = 0; i < W; ++i) cnt += __builtin_popcount(opp[i]);
    } else {
        // agents may share cells: count visible opponents one by one
        constexpr int D = 2 * R + 1;
        const int ax = pa & 0xff, ay = pa >> 8;
        const bool sa = a < S;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            const int dx = (pp[j] & 0xff) - ax + R;
            const int dy = (pp[j] >> 8) - ay + R;
            const bool in = j < n && j != a && (uint32_t)dx < (uint32_t)D &&
                            (uint32_t)dy < (uint32_t)D && ((j < S) != sa);
            const int kk = in ? dy * D + dx : 0;
            uint32_t vw = vis[0];
#pragma unroll
            for (int i = 1; i < W; ++i) vw = (kk >> 5) == i ? vis[i] : vw;
            cnt += (in && ((vw >> (kk & 31)) & 1u)) ? 1 : 0;
        }
    }
    return cnt;
}

// Channels of one agent (agent_masks_raw). The feature loop (FEAT) adds the
// per-env options: with line of sight (occl) every channel is restricted to
// the visible cells and the opponent count to visible opponents; with
// exploration (xpl) seen gets the window cells that are visible and inside
// the map (bits past the window's D*D cells are undefined).
template <int R, int W, int NMAX, bool EXACT, bool FEAT, bool TER, bool PLN = false>
__device__ __forceinline__ int agent_masks(const uint32_t *slot, int H, int Wd,
                                           const int (&pp)[NMAX], int a, int pa, int n, int S,
                                           bool want_out, bool occl, bool xpl, uint32_t (&wall)[W],
                                           uint32_t (&outm)[W], uint32_t (&team)[W],
                                           uint32_t (&opp)[W], uint32_t (&seen)[W], int pw,
                                           uint32_t cls, const uint32_t *planes = nullptr,
                                           int plw = 0)
{
    // exploration needs the outside-the-map cells whatever the channel count
    // (outm is stored only for 4-channel envs); with terrain and line of
    // sight, only walls and outside block sight, not what the class may not
    // enter
    uint32_t lw[W];
    int cnt = agent_masks_raw<R, W, NMAX, EXACT, TER, PLN>(slot, H, Wd, pp, a, pa, n, S,
                                                           FEAT ? (want_out || xpl) : want_out, wall,
                                                           outm, team, opp, pw, cls,
                                                           (TER && occl) ? &lw : nullptr, planes, plw);
    if constexpr (FEAT) {
        uint32_t vis[W];
#pragma unroll
        for (int i = 0; i < W; ++i) vis[i] = 0xffffffffu;
        if (occl) {
            if constexpr (TER)
                cnt = occlude<R, W, NMAX, EXACT>(pp, a, pa, n, S, lw, wall, outm, team, opp, vis);
            else
                cnt = occlude<R, W, NMAX, EXACT>(pp, a, pa, n, S, wall, wall, outm, team, opp, vis);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) seen[i] = vis[i] & ~outm[i];
    }
    return cnt;
}

template <int R, int W, int NMAX, int TPL, bool EXACT, bool FEAT, bool TER = false, bool PLN = false>
__device__ __forceinline__ void all_masks(const uint32_t *slot, int H, int Wd,
                                          const int (&pp)[NMAX], int l, int lanes,
                                          const int (&mine)[TPL], int n, int S, bool want_out,
                                          bool occl, bool xpl, uint32_t (&wall)[TPL][W],
                                          uint32_t (&outm)[TPL][W], uint32_t (&team)[TPL][W],
                                          uint32_t (&opp)[TPL][W], uint32_t (&seen)[TPL][W],
                                          int (&cnt)[TPL], int pw = 0, uint32_t clo = 0u,
                                          uint32_t chi = 0u, const uint32_t *planes = nullptr,
                                          int plw = 0, const int *aids = nullptr)
{
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
        const int a = aids != nullptr ? aids[m] : l + m * lanes;
        const uint32_t cls = TER ? agent_class(clo, chi, a) : 0u;
        cnt[m] = agent_masks<R, W, NMAX, EXACT, FEAT, TER, PLN>(
            slot, H, Wd, pp, a, mine[m], n, S, want_out, occl, xpl, wall[m], outm[m], team[m],
            opp[m], seen[m], pw, cls, planes, plw);
    }
}

// ------------------------------------------------------------ exploration

// Row rho of a window mask (D bits).
template <int R, int W>
__device__ __forceinline__ uint32_t window_row(const uint32_t (&m)[W], int rho)
{
    constexpr int D = 2 * R + 1;
    const int off = rho * D, wi = off >> 5, b = off & 31;
    uint32_t v = m[wi] >> b;
    if (b + D > 32) v |= m[wi + 1] << (32 - b);
    return v & ((1u << D) - 1u);
}

// Cells of a seeker's seen window (agent at packed padded cell pa) that the
// env's discovery map (LDS, padded board layout) does not hold yet.
template <int R, int W>
__device__ __forceinline__ int explore_fresh(const uint32_t *map, int pa, const uint32_t (&seen)[W])
{
    constexpr int D = 2 * R + 1;
    const int col = (pa & 0xff) - R;
    const uint32_t *base = map + ((pa >> 8) - R) * LDS_ROW + (col >> 5);
    const uint32_t sh = (uint32_t)(col & 31);
    int f = 0;
#pragma unroll
    for (int rho = 0; rho < D; ++rho) {
        const uint32_t *rp = base + rho * LDS_ROW;
        const uint32_t old = __builtin_amdgcn_alignbit(rp[1], rp[0], sh);
        f += __builtin_popcount(window_row<R, W>(seen, rho) & ~old);
    }
    return f;
}

// Add a seeker's seen window to the discovery map. Seekers of one env share
// the map words (several lanes, or one lane's tasks), hence LDS atomics.
template <int R, int W>
__device__ __forceinline__ void explore_mark(uint32_t *map, int pa, const uint32_t (&seen)[W])
{
    constexpr int D = 2 * R + 1;
    const int col = (pa & 0xff) - R;
    uint32_t *base = map + ((pa >> 8) - R) * LDS_ROW + (col >> 5);
    const uint32_t sh = (uint32_t)(col & 31);
#pragma unroll
    for (int rho = 0; rho < D; ++rho) {
        uint32_t *rp = base + rho * LDS_ROW;
        const uint64_t v = (uint64_t)window_row<R, W>(seen, rho) << sh;
        __hip_atomic_fetch_or(rp, (uint32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_or(rp + 1, (uint32_t)(v >> 32), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// LDS discovery map (padded layout) -> HBM map of H rows of ceil(W/32) words
// (1 or 2), split over the env's lanes in chunks of 4 consecutive words (one
// 16-byte store each; the words past the map in the last chunk are read from
// padding rows and not stored).
template <int LANES>
__device__ __forceinline__ void map_store(GAS uint32_t *dst, const uint32_t *map, int H, int Wd, int l)
{
    const uint32_t rs = Wd > 32 ? 1u : 0u;  // log2 of the words per row
    const uint32_t total = (uint32_t)H << rs;
    for (uint32_t w0 = 4u * (uint32_t)l; w0 < total; w0 += 4u * LANES) {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t w = w0 + (uint32_t)k, y = w >> rs, j = w & rs;
            const uint32_t *row = map + (y + PAD) * LDS_ROW + j;
            v[k] = __builtin_amdgcn_alignbit(row[1], row[0], PAD);
        }
        if (w0 + 4u <= total) {
            u32x4_a4 x;
            x.x = v[0];
            x.y = v[1];
            x.z = v[2];
            x.w = v[3];
            *(GAS u32x4_a4 *)(dst + w0) = x;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (w0 + (uint32_t)k < total) dst[w0 + k] = v[k];
        }
    }
}

// HBM map -> LDS discovery map (all mw words of the padded layout, rows
// outside the map and the slack word 0), words split over the env's lanes.
template <int LANES>
__device__ __forceinline__ void map_load(uint32_t *map, const GAS uint32_t *src, int H, int Wd, int l)
{
    const int rw = (Wd + 31) >> 5;
    const int mw = (H + 2 * PAD) * LDS_ROW + 1;
    for (int i = l; i < mw; i += LANES) {
        const int yy = i / LDS_ROW, j = i - yy * LDS_ROW, y = yy - PAD;
        uint32_t v = 0u;
        if ((uint32_t)y < (uint32_t)H) {
            const uint32_t cur = j < rw ? src[y * rw + j] : 0u;
            const uint32_t prev = (j >= 1 && j - 1 < rw) ? src[y * rw + j - 1] : 0u;
            v = (cur << PAD) | (prev >> (32 - PAD));
        }
        map[i] = v;
    }
}

// Blocked-move field of one agent, 5 bits: bit 0 set (action 0, stay, never
// moves), bits 1..4 = the target cells of actions 1..4 (north, south, east,
// west) hold a wall or lie outside the map. From the agent's wall|outside
// window around its current cell, or from the board at cell pa.
template <int R, int W>
__device__ __forceinline__ uint32_t blocked_field(const uint32_t (&wall)[W])
{
    constexpr int D = 2 * R + 1, C = R * D + R;
    auto bit = [&](int k) { return (wall[k >> 5] >> (k & 31)) & 1u; };
    return 1u | (bit(C - D) << 1) | (bit(C + D) << 2) | (bit(C + 1) << 3) | (bit(C - 1) << 4);
}

__device__ __forceinline__ uint32_t blocked_field_board(const uint32_t *slot, int pa)
{
    return 1u | (board_bit(slot, pa - 256) << 1) | (board_bit(slot, pa + 256) << 2) |
           (board_bit(slot, pa + 1) << 3) | (board_bit(slot, pa - 1) << 4);
}

// Fields of agents 0..NMAX-1 (NMAX <= 6) at bits 5a.., gathered from the
// lanes that own them: every lane of the env gets the same word.
template <int LANES, int NMAX, int TPL, typename F>
__device__ __forceinline__ uint32_t gather_blocked(int l, F field)
{
    static_assert(NMAX * 5 <= 32, "blocked fields need NMAX <= 6");
    // when every task slot fits the word, slots of absent agents (whose
    // actions are always 0) need no test
    constexpr bool ALL_FIT = LANES * TPL * 5 <= 32;
    uint32_t v = 0;
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
        const int a = l + m * LANES;
        v |= (ALL_FIT || a < NMAX) ? field(m) << (5 * a) : 0u;
    }
    return group_or_dpp<LANES>(v);
}

// K steps of one tile: the envs perm[tile.env0 ..] of job J, LANES lanes per
// env, at most NMAX agents, view radius R, all of kind KIND. K == 0 writes
// the observation of the current state only. UNROLL unrolls the step loop
// over each action window (single-variant launches; the mixed kernels keep
// one copy per variant to bound their code size). map_words is the LDS
// discovery map per env slot (0 when no env of the launch explores).
template <int LANES, int NMAX, int R, bool UNROLL, int KIND>
__device__ __forceinline__ void step_tile(const Tile &tile, const JobDesc &J, uint32_t K,
                                          uint32_t step_base, uint32_t slot_words,
                                          uint32_t map_words, uint32_t *lds)
{
    constexpr int D = 2 * R + 1;
    constexpr int W = (D * D + 31) / 32;             // words per channel
    constexpr int TPL = (NMAX + LANES - 1) / LANES;  // agent tasks per lane
    constexpr int MAXCALLS = (NMAX + 3) / 4;         // generator blocks per step
    // actions come from a window of future steps when every block of a step
    // has its own lane; otherwise each lane draws all blocks itself
    constexpr bool WINDOWED = LANES >= MAXCALLS && LANES > 1;
    // with at most 4 agents and 2 or 4 lanes the window is gathered by DPP and
    // spans exactly LANES steps
    constexpr bool DPP_WINDOW = WINDOWED && NMAX <= 4 && (LANES == 2 || LANES == 4);
    // external actions of windowed loops are read a window ahead and merged
    // into the window's generator blocks, so no step waits for its action
    // bytes; radio targets come with the bytes, so radio envs do this only
    // where their targets are drawn for a window too (more than 2 or 4
    // lanes' DPP windows)
    constexpr bool WIN_ACT =
        WINDOWED && ((KIND & KIND_RADIO) == 0 || !(NMAX <= 4 && (LANES == 2 || LANES == 4)));
    // with at most 4 agents the wall tests of the moves come from bits kept
    // from the previous step's windows instead of board reads, and detection
    // (rewards, found bits) is a pairwise Chebyshev test in every lane of the
    // env, independent of the observation masks
    constexpr bool NBR = NMAX <= 4 && (KIND & KIND_TERRAIN) == 0;
    constexpr bool PAIRS = NMAX <= 4;
    // plain respawns of the DPP-window loops try the first LANES / NMAX draws
    // of every agent side by side before running the spawn rule
    constexpr bool FAST_SPAWN = DPP_WINDOW && (KIND & KIND_TERRAIN) == 0 && LANES >= NMAX;
    constexpr int SA = FAST_SPAWN ? LANES / NMAX : 1;
    // with 8 or 16 lanes per env each lane draws the first SL draws of its
    // own agents
    constexpr bool LANE_SPAWN = !FAST_SPAWN && LANES >= 8;
    // moves with a lane per agent, 8 or 16 lanes per env and more than 4
    // agents (no terrain): each lane decides its own agent's move (with two
    // agents per lane, the 20-agent kernels spilled registers)
    constexpr bool LANE_MOVES = LANES >= 8 && TPL == 1 && !NBR && (KIND & KIND_TERRAIN) == 0;
    constexpr bool LANE_MOVES_T = LANES >= 8 && TPL == 1 && (KIND & KIND_TERRAIN) != 0;
    // one agent per lane and more than 4 agents: the teammate / opponent
    // channels of envs with distinct cells come from two LDS planes of the
    // agents' cells (seekers, hiders), each lane keeping its own agent's bit
    // up to date, instead of a pass over all agents per lane (not for
    // terrain, which ran 7% slower with them)
    constexpr bool PLANES = LANES >= 8 && TPL == 1 && NMAX > 4 && (KIND & KIND_TERRAIN) == 0;
    // plain envs of the 2- and 4-lane window loops: a lane without an agent
    // of its own repeats agent l mod n (same cells, roles, output places), so
    // every lane stores the same words to the same places and no store sits
    // behind a branch (inactive slots repeat the tile's first env in full)
    constexpr bool DUP = KIND == KIND_PLAIN && DPP_WINDOW && TPL == 1;
    constexpr int SL = NMAX >= 20 ? 2 : 3;
    constexpr int NP = PAIRS ? NMAX * (NMAX - 1) / 2 : 1;  // agent pairs i < j

    const int lane = (int)threadIdx.x;
    const int q = lane / LANES;  // env slot in the tile
    const int l = lane % LANES;  // sub-lane within the env

    const bool active = q < (int)tile.count;
    // inactive slots shadow the tile's first env and never store
    const uint32_t e = gp(J.tab.perm)[tile.env0 + (active ? (uint32_t)q : 0u)];

    const uint32_t s0 = gp(J.tab.spec0)[e], s1 = gp(J.tab.spec1)[e];
    const int H = (int)(s0 & 0xffu), Wd = (int)((s0 >> 8) & 0xffu);
    const int n = (int)((s0 >> 16) & 0xffu), S = (int)(s0 >> 24);
    const int C = (int)((s1 >> 4) & 0xfu);
    const uint32_t flags = (s1 >> 8) & 0xffu, Lep = s1 >> 16;
    const bool collide = (flags & 1u) != 0u;
    // the agent index each task stands for (its own, or with DUP the agent
    // it repeats)
    int aid[TPL];
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
        const int a = l + m * LANES;
        aid[m] = (DUP && a >= n) ? a % n : a;
    }
    const bool want_out = C == 4;
    constexpr bool FEAT_OK = KIND != KIND_PLAIN;
    constexpr bool XPL = (KIND & KIND_EXPLORE) != 0;  // every env of the tile explores
    constexpr bool TER = (KIND & KIND_TERRAIN) != 0;  // every env of the tile has terrain
    constexpr bool RAD = (KIND & KIND_RADIO) != 0;    // every env of the tile has radio

    // agent_off: the env's agents in the state (positions, beliefs)
    const uint32_t agent_off = gp(J.tab.agent_off)[e];
    const uint32_t env = gp(J.tab.env_id)[e];
    const uint64_t seed = gp(J.seed)[e];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t found = gp(J.found)[e], t = gp(J.t)[e], ep = gp(J.ep)[e], steps = gp(J.steps)[e];
    // Output places: the job's first output row, its step limit, and the
    // env's first obs word, first reward (and action) and done byte in a
    // row. A resident range writes row = the env's step count since its
    // reset (the same for every env of the range, so for the whole tile),
    // relative to the range's first env, and stops at its budget.
    // The step count and limit stay wave-uniform (scalar registers): a
    // per-lane trip count would turn the step loop into a divergent one.
    uint32_t out_step0 = J.out_step0, k_limit = J.k_limit;
    uint32_t obs_off, out_agent = agent_off, out_env = e;
    if (J.resident) {
        const uint32_t rel = e - J.first;
        const uint32_t s_wave = __builtin_amdgcn_readfirstlane(steps);
        out_step0 = s_wave;
        k_limit = J.budget > s_wave ? J.budget - s_wave : 0u;
        obs_off = rel * J.obs_env;
        out_agent = rel * (uint32_t)n;
        out_env = rel;
        if (K != 0u && k_limit == 0u) return;  // the range has taken its budget
    } else {
        obs_off = gp(J.tab.obs_off)[e];
    }
    // terrain: the second tile plane pw words after the first, the stuck
    // chance (bits 16..23 of word 0), the move chances (bytes of words 1..3,
    // class * 3 + tile), the agent classes (words 4, 5) and the stuck agents
    const int pw = TER ? (H + 2 * PAD) * LDS_ROW + 1 : 0;
    uint32_t tch = 0u, sp_a = 0u, sp_b = 0u, sp_c = 0u, clo = 0u, chi = 0u, stuck = 0u;
    if constexpr (TER) {
        const GAS uint32_t *tr = gp(J.tab.terr) + 8u * e;
        tch = tr[0];
        sp_a = tr[1];
        sp_b = tr[2];
        sp_c = tr[3];
        clo = tr[4];
        chi = tr[5];
        stuck = gp(J.stuck)[e];
    }

    // this env's LDS slot: the padded bitboard, then MAX_AGENTS words where a
    // respawn writes the new positions, then (feature launches with an
    // exploring env) the discovery map
    uint32_t *slot = lds + (uint32_t)q * (slot_words * (PLANES ? 3u : 1u) + MAX_AGENTS + map_words);
    int *spawned = (int *)(slot + slot_words);
    uint32_t *mslot = slot + slot_words + MAX_AGENTS;
    // the agent planes (PLANES): seekers, then hiders slot_words later
    uint32_t *planes = slot + slot_words + MAX_AGENTS + map_words;
    const int plw = (int)slot_words;
    const uint32_t map_off = XPL ? gp(J.tab.map_off)[e] : 0u;
    if constexpr (XPL) {
        if (K != 0u) map_load<LANES>(mslot, gp(J.disc) + map_off, H, Wd, l);
    }
    {
        // The board planes are stored in HBM as they sit in LDS, 16-byte
        // aligned and padded to 16 bytes: the env's lanes copy them 4 words
        // per load, 8 loads in flight per lane before their stores (one
        // memory round trip per batch instead of one per word).
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const GAS u32x4 *src = (const GAS u32x4 *)(gp(J.bb) + gp(J.tab.bb_off)[e]);
        u32x4 *dst = (u32x4 *)slot;
        const int n4 = board_words(H, TER ? 2 : 1) >> 2;
        for (int base = 0; base < n4; base += 8 * LANES) {
            u32x4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = base + u * LANES + l;
                if (i < n4) v[u] = src[i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = base + u * LANES + l;
                if (i < n4) dst[i] = v[u];
            }
        }
    }
    const uint32_t last_word = slot_words - 1u;

    int pp[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        int v = FAR_CELL;
        if (j < n) {
            const uint32_t p = gp(J.pos)[agent_off + (uint32_t)j];
            v = (int)((((p >> 8) + PAD) << 8) | ((p & 0xffu) + PAD));
        }
        pp[j] = v;
    }
    // positions of this lane's own agents l + m * LANES (agent 0's position for
    // lanes without an agent), kept in registers
    int mine[TPL];
    if constexpr (DUP)
        own_positions_ids<NMAX, TPL>(pp, aid, mine);
    else
        own_positions<LANES, NMAX, TPL>(pp, l, n, mine);
    if constexpr (PLANES) {
        for (uint32_t i = (uint32_t)l; i < 2u * slot_words; i += LANES) planes[i] = 0u;
        wave_lds_fence();
        if (l < n)
            __hip_atomic_fetch_or(planes + (l < S ? 0 : plw) + plane_word(mine[0]), plane_bit(mine[0]),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        wave_lds_fence();
    }

    const uint32_t hmask = (uint32_t)(((1ull << n) - 1ull) & ~((1ull << S) - 1ull));
    const uint64_t amask = (1ull << (3 * n)) - 1ull;  // action bits of real agents
    const int ncalls = (n + 3) >> 2;
    const int kb = WINDOWED ? LANES / ncalls : 1;  // steps per action window
    // in a window, lane l draws block (step + wstep, group wgroup)
    const int wstep = WINDOWED ? l / ncalls : 0, wgroup = WINDOWED ? l - wstep * ncalls : 0;
    const uint32_t Kj = K < k_limit ? K : k_limit;
    const bool obs_only = (K == 0);
    const uint32_t nsteps = obs_only ? 1u : Kj;

    const uint64_t row = (uint64_t)out_step0 + step_base;
    GAS uint32_t *obs_p = gp(J.obs) + row * J.obs_stride + obs_off;
    GAS float *rew_p = obs_only ? nullptr : gp(J.rew) + row * J.agent_stride + out_agent;
    GAS uint8_t *done_p = obs_only ? nullptr : gp(J.done) + row * J.env_stride + out_env;
    const GAS int8_t *act_p = J.act ? gp(J.act) + row * J.agent_stride + out_agent : nullptr;
    // the true state after each step, when requested (a wave-uniform test)
    const bool want_state = J.spos != nullptr && !obs_only;
    GAS uint16_t *spos_p = (J.spos != nullptr && !obs_only) ? gp(J.spos) + row * J.agent_stride + out_agent
                                                             : nullptr;
    GAS uint32_t *senv_p = (J.senv != nullptr && !obs_only)
                               ? gp(J.senv) + (row * J.env_stride + out_env) * 4u
                               : nullptr;
    // per-step discovery maps of an active exploring env, when requested
    GAS uint32_t *map_p = nullptr;
    if constexpr (XPL) {
        if (active && J.map != nullptr && !obs_only) {
            const uint32_t map_out = J.resident ? (e - J.first) * J.map_env : map_off;
            map_p = gp(J.map) + row * J.map_stride + map_out;
        }
    }

    // Complete every load issued so far here, before the step loop: the wait
    // pass would otherwise place a vmcnt(0) wait at their first use inside the
    // loop, and on gfx9 vmcnt also counts stores, so each step would stall on
    // all of the previous step's output stores.
    __builtin_amdgcn_s_waitcnt(0);
    wave_lds_fence();

    // blocked-move fields of all agents at their current cells (NBR only)
    uint32_t nbw = 0;
    if constexpr (NBR)
        nbw = gather_blocked<LANES, NMAX, TPL>(l, [&](int m) { return blocked_field_board(slot, mine[m]); });

    const bool has_act = J.act != nullptr;
    // per-task constants: the task's agent exists (and its env is active), its
    // bit in the hider mask, its reward sign
    bool mine_live[TPL], seeker[TPL];
    uint32_t hbit[TPL];
    int rsign[TPL];
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
        const int a = l + m * LANES, ai = aid[m];
        mine_live[m] = active && a < n;
        seeker[m] = ai < S;
        hbit[m] = (ai < n && ai >= S) ? 1u << ai : 0u;
        rsign[m] = ai < S ? 1 : -1;
    }
    // radio: each task's belief (bit h: the agent knows of hider h)
    uint32_t bel[TPL];
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
        const int a = l + m * LANES;
        bel[m] = (RAD && a < n) ? gp(J.bel)[agent_off + (uint32_t)a] : 0u;
    }
    // termination needs every hider found; without capture-ends (or without
    // hiders) the test uses bit 31, which no agent sets
    const uint32_t tmask = ((flags & 2u) && n > S) ? hmask : 0x80000000u;
    const uint32_t cmask = collide ? 1u : 0u;
    // pair constants (PAIRS): pair (i, j) has opposite roles iff i < S <= j,
    // its hider is j; pinv[m] has the bits of such pairs that involve the
    // task's agent
    uint32_t pair_hb[NP], pinv[TPL];
#pragma unroll
    for (int m = 0; m < TPL; ++m) pinv[m] = 0u;
    if constexpr (PAIRS) {
        int pi = 0;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
#pragma unroll
            for (int jj = i + 1; jj < NMAX; ++jj, ++pi) {
                const bool opp_ij = i < S && S <= jj && jj < n;
                pair_hb[pi] = opp_ij ? 1u << jj : 0u;
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    const int a = aid[m];
                    pinv[m] |= (opp_ij && (a == i || a == jj)) ? 1u << pi : 0u;
                }
            }
        }
    }

    // The step loop, instantiated for channels computed assuming distinct
    // agent cells (collisions on) and for the exact per-agent test; the choice
    // is made once per env, outside the loop.
    auto run = [&](auto exact_tag, auto feat_tag) __attribute__((always_inline)) {
        constexpr bool EX = decltype(exact_tag)::value;
        // the feature loops (feat_tag = the env kind: exploration, line of
        // sight, or both) are not unrolled (bounded code size); with line of
        // sight detection goes through the counts (the pairwise test knows
        // no walls), exploration leaves it alone
        constexpr int FK = decltype(feat_tag)::value;
        constexpr bool OC = FK != KIND_PLAIN;
        constexpr bool LOS = (FK & KIND_LOS) != 0;
        constexpr bool XP = (FK & KIND_EXPLORE) != 0;
        constexpr bool USE_PAIRS = PAIRS && !LOS;
        constexpr bool PL = PLANES && !EX;
        // the lane's agent moves from cell `from` to cell `to` in the planes
        // (every clear of the wave comes before every set)
        auto plane_move = [&](int from, int to) __attribute__((always_inline)) {
            if constexpr (PL) {
                uint32_t *pl = planes + (l < S ? 0 : plw);
                if (l < n) {
                    __hip_atomic_fetch_and(pl + plane_word(from), ~plane_bit(from), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_or(pl + plane_word(to), plane_bit(to), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                wave_lds_fence();
            }
        };
        uint32_t wall[TPL][W], outm[TPL][W], team[TPL][W], opp[TPL][W], seen[TPL][W];
        int cnt[TPL];

        // this lane's output addresses of the current step, advanced per step
        GAS uint32_t *obs_l[TPL];
        GAS float *rew_l[TPL];
#pragma unroll
        for (int m = 0; m < TPL; ++m) {
            obs_l[m] = obs_p + (uint32_t)(aid[m] * (C * W + (RAD ? 1 : 0)));
            rew_l[m] = obs_only ? nullptr : rew_p + (uint32_t)aid[m];
        }
        auto store_obs = [&](int m) __attribute__((always_inline)) {
            GAS uint32_t *oa = obs_l[m];
            store_words<W>(oa, wall[m]);
            store_words<W>(oa + W, team[m]);
            store_words<W>(oa + 2 * W, opp[m]);
            if (want_out) store_words<W>(oa + 3 * W, outm[m]);
            // radio: the belief word follows the channels
            if constexpr (RAD) oa[want_out ? 4 * W : 3 * W] = bel[m];
        };

        if (obs_only) {
            all_masks<R, W, NMAX, TPL, EX, OC, TER, PL>(slot, H, Wd, pp, l, LANES, mine, n, S,
                                                        want_out, LOS, false, wall, outm, team,
                                                        opp, seen, cnt, pw, clo, chi, planes, plw, aid);
#pragma unroll
            for (int m = 0; m < TPL; ++m)
                if (DUP || mine_live[m]) store_obs(m);
            return;
        }

        // One step from the generator's actions of this step (3 bits per
        // agent); all of its stores are issued together at the end.
        // radio targets drawn for a window of steps (the windowed feature
        // loop): lane l holds the RADIO block (step + wstep, group wgroup)
        // mapped to four 5-bit targets; step rj of the window reads them
        constexpr bool RWIN = RAD && WINDOWED && !DPP_WINDOW;
        uint32_t rwin = 0u, rj = 0u;
        auto block_targets = [&](uint32_t sub, uint32_t step) __attribute__((always_inline)) {
            const U4 x = philox(env, (ST_RADIO << 24) | sub, step, 0u, k0, k1);
            const uint32_t m = (uint32_t)n;
            return range_map(x.x, m) | (range_map(x.y, m) << 5) | (range_map(x.z, m) << 10) |
                   (range_map(x.w, m) << 15);
        };

        auto step = [&](uint64_t acts) __attribute__((always_inline)) {
            // ---- 1 radio targets of this lane's tasks (own index: no
            // message): the RADIO draw, word a & 3 of block a >> 2, mapped
            // to 0..n-1, unless an external action names one
            uint32_t tgt_r[TPL];
            if constexpr (RAD) {
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    const uint32_t a = (uint32_t)(l + m * LANES);
                    if constexpr (RWIN) {
                        // block a >> 2 of this step sits in lane rj * ncalls +
                        // (a >> 2) of the env (an absent agent may read another
                        // lane's word: its target carries an empty belief)
                        const uint32_t pkd = (uint32_t)__shfl(
                            (int)rwin, q * LANES + (int)rj * ncalls + (int)(a >> 2), 64);
                        tgt_r[m] = (pkd >> (5u * (a & 3u))) & 31u;
                    } else {
                        const U4 x = philox(env, (ST_RADIO << 24) | (a >> 2), steps, 0u, k0, k1);
                        const uint32_t w = pick((a & 2u) != 0u, pick((a & 1u) != 0u, x.w, x.z),
                                                pick((a & 1u) != 0u, x.y, x.x));
                        tgt_r[m] = range_map(w, (uint32_t)n);
                    }
                    if (has_act && !WIN_ACT && (int)a < n) {
                        const int v = act_p[a];
                        if (v != -1) {
                            // v >= 0: target v div 5 - 1 (0 or past the last agent: none)
                            const uint32_t c = v >= 0 ? (uint32_t)v / 5u : 0u;
                            tgt_r[m] = (c >= 1u && c <= (uint32_t)n) ? c - 1u : a;
                        }
                    }
                }
            }
            // ---- 1 external actions override the drawn ones (-1 keeps the
            // draw); with radio a value v >= 0 moves v mod 5. The windowed
            // loops without radio merge them into the window's blocks.
            if (has_act && !WIN_ACT) {
                uint64_t ov = 0, om = 0;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    if (i < n) {
                        const int v = act_p[i];
                        if (v != -1) {
                            uint32_t a = (v >= 0 && v <= 4) ? (uint32_t)v : 0u;
                            if constexpr (RAD) a = v >= 0 ? (uint32_t)v % 5u : 0u;
                            ov |= (uint64_t)a << (3 * i);
                            om |= 7ull << (3 * i);
                        }
                    }
                }
                acts = (acts & ~om) | ov;
                act_p += J.agent_stride;
            }
            acts &= amask;

            // the lane's agent's cell before the moves (for the planes)
            const int pl_from = mine[0];
            // ---- 2 moves, agent-index order (redundant in every lane of the env)
            if constexpr (TER) {
                // Terrain: a stuck agent stays; the target must be a tile the
                // agent's class may enter and (collisions on) free; then the
                // move chance and, for a walker entering mud, the stuck chance
                // decide, from words 2(i&1) and 2(i&1)+1 of the MOVE block of
                // agent pair i>>1 at this step. Everything but the
                // occupancy test depends on the agent alone, so each lane
                // decides it for its own agents (target, "moves if the
                // target is free", "gets stuck if it moves"), the env's
                // lanes exchange those words through the env's LDS respawn
                // words, and every lane runs the sequential occupancy chain
                // (agents in index order) on them.
                uint32_t *xw = (uint32_t *)spawned;
                int own_tg = 0;
                uint32_t own_go = 0u, own_st = 0u;
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    const int a = l + m * LANES;
                    const uint32_t act = (uint32_t)(acts >> (3 * a)) & 7u;  // 0 for absent agents
                    const int tg = mine[m] + (int)((MOVE_TABLE >> (12u * act)) & 0x3ffull) - 257;
                    uint32_t widx = (uint32_t)(tg >> 8) * (uint32_t)LDS_ROW + (((uint32_t)tg >> 5) & 7u);
                    widx = widx < (uint32_t)pw - 1u ? widx : (uint32_t)pw - 1u;  // parked agents
                    const uint32_t sh = (uint32_t)tg & 31u;
                    const uint32_t b0 = (slot[widx] >> sh) & 1u, b1 = (slot[pw + widx] >> sh) & 1u;
                    const uint32_t cls = agent_class(clo, chi, a);
                    const U4 blk = philox(env, (ST_MOVE << 24) | ((uint32_t)a >> 1), steps, 0u, k0, k1);
                    const bool odd = (a & 1) != 0;
                    const uint32_t u = pick(odd, blk.z, blk.x), v = pick(odd, blk.w, blk.y);
                    const uint32_t type = b0 | (b1 << 1);  // ground, wall, water, mud
                    const uint32_t tile = (type + 1u) >> 1;  // ground 0, water 1, mud 2 (wall: blocked)
                    const uint32_t k = cls * 3u + tile;
                    const uint32_t pct = (pick(k < 4u, sp_a, pick(k < 8u, sp_b, sp_c)) >> (8u * (k & 3u))) & 0xffu;
                    // every condition evaluated, combined with bitwise ops
                    const uint32_t blocked = ((stuck >> (uint32_t)a) & 1u) | (class_blocked(cls, b0, b1) & 1u) |
                                             (act == 0u ? 1u : 0u);
                    const uint32_t go = (chance(u, pct) ? 1u : 0u) & (blocked ^ 1u);
                    const uint32_t sticks = go & (cls == 0u ? 1u : 0u) & (type == 3u ? 1u : 0u) &
                                            (chance(v, (tch >> 16) & 0xffu) ? 1u : 0u);
                    if constexpr (LANE_MOVES_T) {
                        own_tg = tg;
                        own_go = go;
                        own_st = sticks;
                    } else {
                        if (a < NMAX) xw[a] = (uint32_t)tg | (go << 16) | (sticks << 17);
                    }
                }
                if constexpr (LANE_MOVES_T) {
                    // one agent per lane: the lane's agent is tested against
                    // the old cells of later agents ahead, then agent by agent
                    // the agent's lane decides and the env's lanes learn its
                    // new cell and whether it got stuck (a row broadcast)
                    uint32_t acc = 0xffffu;  // cells are below 2^16
#pragma unroll
                    for (int jj = 0; jj < NMAX; ++jj)
                        acc = jj > l ? min(acc, (uint32_t)(own_tg ^ pp[jj])) : acc;
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) {
                        const uint32_t moved = own_go & ~(((acc - 1u) >> 31) & cmask);
                        const uint32_t w = env_bcast<LANES>(
                            (uint32_t)(moved ? own_tg : mine[0]) | ((moved & own_st) << 16), i % LANES);
                        const int nc = (int)(w & 0xffffu);
                        pp[i] = i < n ? nc : FAR_CELL;
                        stuck |= ((w >> 16) & 1u) << i;  // absent agents never move
                        acc = min(acc, (uint32_t)(own_tg ^ nc));
                    }
                } else {
                    wave_lds_fence();
                    int tgt[NMAX];
                    uint32_t gof[NMAX], stk[NMAX], mpre[NMAX];
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) {
                        const uint32_t w = xw[i];
                        tgt[i] = (int)(w & 0xffffu);
                        gof[i] = (w >> 16) & 1u;
                        stk[i] = (w >> 17) & 1u;
                    }
                    // the reads precede the radio exchange's and a respawn's
                    // writes to these words
                    wave_lds_fence();
                    // occupancy: the minimum of target ^ cell over the other
                    // agents is 0 exactly when the target is held; the part over
                    // agents that have not moved yet is taken ahead of the chain
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) {
                        uint32_t mn = 0xffffu;  // cells are below 2^16
#pragma unroll
                        for (int jj = i + 1; jj < NMAX; ++jj) mn = min(mn, (uint32_t)(tgt[i] ^ pp[jj]));
                        mpre[i] = mn;
                    }
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) {
                        uint32_t mn = mpre[i];
#pragma unroll
                        for (int jj = 0; jj < i; ++jj) mn = min(mn, (uint32_t)(tgt[i] ^ pp[jj]));
                        const uint32_t moved = gof[i] & ~(((mn - 1u) >> 31) & cmask);
                        stuck |= (moved & stk[i]) << i;
                        pp[i] = moved ? tgt[i] : pp[i];
                    }
                }
                // rescue: a stuck agent is freed by a teammate that is not
                // stuck within Chebyshev distance 1 after the moves ((dy + 1)
                // << 8 | (dx + 1) has both bytes below 3 exactly then); each
                // lane tests its own agents, the env's lanes OR the results
                const uint32_t before = stuck;
                if (before != 0u) {
                    own_positions<LANES, NMAX, TPL>(pp, l, n, mine);
                    const uint32_t smask = (1u << S) - 1u;  // seekers; hmask: hiders
                    uint32_t freed = 0u;
#pragma unroll
                    for (int m = 0; m < TPL; ++m) {
                        const int a = l + m * LANES;
                        uint32_t near = 0u;
#pragma unroll
                        for (int jj = 0; jj < NMAX; ++jj) {
                            const uint32_t du = (uint32_t)(mine[m] - pp[jj]) + 257u;
                            const uint32_t lo = du & 0xffu, hi = du >> 8;
                            near |= ((lo > hi ? lo : hi) < 3u ? 1u : 0u) << jj;
                        }
                        const uint32_t abit = a < 32 ? 1u << a : 0u;
                        const uint32_t mates = (a < S ? smask : hmask) & ~abit;
                        freed |= ((before & abit) != 0u && (near & mates & ~before) != 0u) ? abit : 0u;
                    }
                    stuck &= ~group_or_dpp<LANES>(freed);
                }
            } else if constexpr (NBR) {
                // Integer decisions only: lane-mask logic would cost a round
                // trip through the scalar unit on the step's critical path. A
                // move is blocked by its field bit or, with collisions on, by
                // an agent on the target (cells are below 2^16, so
                // ((c ^ c') - 1) >> 31 is 1 exactly when c == c').
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    const uint32_t a = (uint32_t)(acts >> (3 * i)) & 7u;
                    const int tg = pp[i] + (int)((MOVE_TABLE >> (12u * a)) & 0x3ffull) - 257;
                    uint32_t occ = 0u;
#pragma unroll
                    for (int jj = 0; jj < NMAX; ++jj)
                        if (jj != i) occ |= ((uint32_t)(tg ^ pp[jj]) - 1u) >> 31;
                    const uint32_t blk = ((nbw >> (5u * (uint32_t)i + a)) & 1u) | (occ & cmask);
                    pp[i] = blk ? pp[i] : tg;
                }
            } else if constexpr (LANE_MOVES) {
                // Each lane decides its own agents' moves. Agent i's target
                // must be free of the cells of agents < i after their moves
                // and of agents > i before theirs: the part over later agents
                // is taken ahead in each lane; then, agent by agent in index
                // order, the agent's lane decides, every lane of the env
                // learns the new cell (a row broadcast from that lane) and
                // tests its own targets against it (an agent that has decided
                // no longer looks at its test, and agents past the last one
                // decide nothing that counts). One board read per lane
                // instead of one per agent, and no chain over all pairs in
                // every lane.
                int tg[TPL];
                uint32_t wb[TPL], acc[TPL];
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    const int a = l + m * LANES;
                    const uint32_t act = a < NMAX ? (uint32_t)(acts >> (3 * a)) & 7u : 0u;
                    tg[m] = mine[m] + (int)((MOVE_TABLE >> (12u * act)) & 0x3ffull) - 257;
                    uint32_t widx = (uint32_t)(tg[m] >> 8) * (uint32_t)LDS_ROW + (((uint32_t)tg[m] >> 5) & 7u);
                    widx = widx < last_word ? widx : last_word;
                    wb[m] = (slot[widx] >> ((uint32_t)tg[m] & 31u)) & 1u;
                    uint32_t mn = 0xffffu;  // cells are below 2^16
#pragma unroll
                    for (int jj = 0; jj < NMAX; ++jj)
                        mn = jj > a ? min(mn, (uint32_t)(tg[m] ^ pp[jj])) : mn;
                    acc[m] = mn;
                }
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    const int mi = i / LANES;
                    const uint32_t blk = wb[mi] | (((acc[mi] - 1u) >> 31) & cmask);
                    const int nc = (int)env_bcast<LANES>((uint32_t)(blk ? mine[mi] : tg[mi]), i % LANES);
                    pp[i] = i < n ? nc : FAR_CELL;
#pragma unroll
                    for (int m = 0; m < TPL; ++m) acc[m] = min(acc[m], (uint32_t)(tg[m] ^ nc));
                }
            } else {
                // Board reads for every target first (one LDS round trip), then
                // the sequential decisions with integer logic only. A target is
                // occupied iff the minimum of target ^ cell over the other
                // agents is 0; the part over agents that have not moved yet is
                // taken ahead of the sequential chain. Staying needs no test:
                // its target is the agent's own cell.
                int tgt[NMAX];
                uint32_t wblk[NMAX], mpre[NMAX];
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    const uint32_t a = (uint32_t)(acts >> (3 * i)) & 7u;
                    tgt[i] = pp[i] + (int)((MOVE_TABLE >> (12u * a)) & 0x3ffull) - 257;
                    uint32_t widx = (uint32_t)(tgt[i] >> 8) * (uint32_t)LDS_ROW + (((uint32_t)tgt[i] >> 5) & 7u);
                    widx = widx < last_word ? widx : last_word;
                    wblk[i] = (slot[widx] >> ((uint32_t)tgt[i] & 31u)) & 1u;
                    uint32_t mn = 0xffffu;  // cells are below 2^16
#pragma unroll
                    for (int jj = i + 1; jj < NMAX; ++jj) mn = min(mn, (uint32_t)(tgt[i] ^ pp[jj]));
                    mpre[i] = mn;
                }
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    uint32_t mn = mpre[i];
#pragma unroll
                    for (int jj = 0; jj < i; ++jj) mn = min(mn, (uint32_t)(tgt[i] ^ pp[jj]));
                    const uint32_t blk = wblk[i] | (((mn - 1u) >> 31) & cmask);
                    pp[i] = blk ? pp[i] : tgt[i];
                }
            }
            if constexpr (DUP)
                own_positions_ids<NMAX, TPL>(pp, aid, mine);
            else
                own_positions<LANES, NMAX, TPL>(pp, l, n, mine);
            plane_move(pl_from, mine[0]);

            // ---- 3 detection at the post-move positions, and the channels
            all_masks<R, W, NMAX, TPL, EX, OC, TER, PL>(slot, H, Wd, pp, l, LANES, mine, n, S,
                                                        want_out, LOS, XP, wall, outm, team, opp,
                                                        seen, cnt, pw, clo, chi, planes, plw, aid);
            // The role channels feed only the (predicated) stores, so the
            // compiler would compute them inside the store region; using them
            // here keeps them in the step's main block, where they fill the
            // wait for the window rows' LDS reads. Measured faster for every
            // variant but the unrolled one with two-word windows.
            if constexpr (!UNROLL || W == 1) {
#pragma unroll
                for (int m = 0; m < TPL; ++m)
#pragma unroll
                    for (int i = 0; i < W; ++i) asm volatile("" ::"v"(team[m][i]), "v"(opp[m][i]));
            }
            // exploration: each seeker's new cells are counted against the map
            // of the previous step (every lane's reads precede every lane's
            // atomics: one wave, LDS in order), then all are added
            int fresh[TPL];
#pragma unroll
            for (int m = 0; m < TPL; ++m) fresh[m] = 0;
            if constexpr (XP) {
#pragma unroll
                for (int m = 0; m < TPL; ++m)
                    if (seeker[m]) fresh[m] = explore_fresh<R, W>(mslot, mine[m], seen[m]);
                wave_lds_fence();
#pragma unroll
                for (int m = 0; m < TPL; ++m)
                    if (seeker[m]) explore_mark<R, W>(mslot, mine[m], seen[m]);
                wave_lds_fence();
            }
            // reward of a task from its detection value v: (128 v + new cells)
            // / 128 with exploration (exact in float32), else v
            auto reward = [&](int m, int v) __attribute__((always_inline)) {
                if constexpr (XP)
                    return (float)(128 * v + fresh[m]) * 0.0078125f;
                else
                    return (float)v;
            };
            float rv[TPL];
            if constexpr (USE_PAIRS) {
                uint32_t near = 0u, seen_h = 0u;
                int pi = 0;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
#pragma unroll
                    for (int jj = i + 1; jj < NMAX; ++jj, ++pi) {
                        // u = (dy + R) << 8 | (dx + R) when both differences are
                        // within R; otherwise a byte of u is at least D
                        const uint32_t u = (uint32_t)(pp[i] - pp[jj]) + (uint32_t)(R * 256 + R);
                        const uint32_t lo = u & 0xffu, hi = u >> 8;
                        const bool in = (lo > hi ? lo : hi) < (uint32_t)D;
                        near |= in ? 1u << pi : 0u;
                        seen_h |= in ? pair_hb[pi] : 0u;
                    }
                }
#pragma unroll
                for (int m = 0; m < TPL; ++m)
                    rv[m] = reward(m, rsign[m] * __builtin_popcount(near & pinv[m]));
                found |= seen_h;
            } else {
                uint32_t seen_h = 0u;
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    rv[m] = reward(m, rsign[m] * cnt[m]);
                    seen_h |= cnt[m] > 0 ? hbit[m] : 0u;
                }
                found |= group_or_dpp<LANES>(seen_h);
            }

            // ---- 3c radio: a seeker's belief gains the hiders it sees (the
            // Chebyshev window test; with line of sight the opponent bit at
            // the hider's window cell, which is already masked by sight);
            // then every agent sends its belief to its target, all messages
            // formed before any is delivered
            if constexpr (RAD) {
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    uint32_t sh = 0u;
#pragma unroll
                    for (int h = 0; h < NMAX; ++h) {
                        // absent agents sit at FAR_CELL, outside every window
                        const uint32_t u = (uint32_t)(pp[h] - mine[m]) + (uint32_t)(R * 256 + R);
                        const uint32_t lo = u & 0xffu, hi = u >> 8;
                        bool hit = (lo < (uint32_t)D) & (hi < (uint32_t)D);
                        if constexpr (LOS) {
                            const uint32_t k = hit ? hi * (uint32_t)D + lo : 0u;
                            uint32_t wv = opp[m][0];
#pragma unroll
                            for (int wi = 1; wi < W; ++wi) wv = pick((k >> 5) == (uint32_t)wi, opp[m][wi], wv);
                            hit = hit & (((wv >> (k & 31u)) & 1u) != 0u);
                        }
                        sh |= hit ? 1u << h : 0u;
                    }
                    bel[m] |= seeker[m] ? (sh & hmask) : 0u;
                }
                // Each agent's belief and target (bits 0..19 and 27..31) go
                // to word i of the env's respawn words (unused until a reset
                // of this step; every word below NMAX is written by exactly
                // one lane), and every lane reads them all back: independent
                // LDS reads instead of one dependent cross-lane shuffle per
                // agent. A message to oneself ORs a belief into itself, and
                // an absent agent (empty belief, never a target) sends
                // nothing that counts, so neither needs a test.
                uint32_t *xw = (uint32_t *)spawned;
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    const int a = l + m * LANES;
                    if (a < NMAX) xw[a] = bel[m] | (tgt_r[m] << 27);
                }
                wave_lds_fence();
                uint32_t inc[TPL];
#pragma unroll
                for (int m = 0; m < TPL; ++m) inc[m] = 0u;
#pragma unroll
                for (int i = 0; i < NMAX; ++i) {
                    const uint32_t pk = xw[i];
                    const uint32_t ti = pk >> 27, bi = pk & 0x07ffffffu;
#pragma unroll
                    for (int m = 0; m < TPL; ++m)
                        inc[m] |= ti == (uint32_t)(l + m * LANES) ? bi : 0u;
                }
                // the reads precede any respawn write to these words
                wave_lds_fence();
#pragma unroll
                for (int m = 0; m < TPL; ++m) bel[m] |= inc[m];
            }

            // ---- 4 termination / truncation
            t += 1u;
            const uint32_t d = ((found & tmask) == tmask ? 1u : 0u) | (t >= Lep ? 2u : 0u);

            // ---- 5 outputs, assuming no reset: observations of this lane's
            // agents (channel-major words), their rewards, and the env's done
            // flag. Issuing them before the reset test lets the scheduler mix
            // them into the step's dependency chains.
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                if (DUP || mine_live[m]) {
                    store_obs(m);
                    *rew_l[m] = rv[m];
                    if (m == 0) *done_p = (uint8_t)d;
                }
            }
            if constexpr (NBR)
                nbw = gather_blocked<LANES, NMAX, TPL>(l, [&](int m) { return blocked_field<R, W>(wall[m]); });

            // ---- 6 same-step auto-reset from the unchanged grid; the env's
            // observation is written again (a later store to the same words
            // by the same lane) from the respawned positions. d is the same in
            // every lane of an env, so the DPP gather inside sees whole groups.
            if (d) {
                ep += 1u;
                t = 0u;
                found = 0u;
                // and with empty beliefs
                if constexpr (RAD) {
#pragma unroll
                    for (int m = 0; m < TPL; ++m) bel[m] = 0u;
                }
                // the new episode starts with an empty discovery map
                if constexpr (XP)
                    for (uint32_t i = (uint32_t)l; i < map_words; i += LANES) mslot[i] = 0u;
                // the respawn: each agent on a cell it may stand on (terrain:
                // a tile of its class), and nobody stuck
                if constexpr (TER) stuck = 0u;
                auto may_stand = [&](int i, int pc) __attribute__((always_inline)) {
                    if constexpr (TER) {
                        const int yy = pc >> 8, xx = pc & 0xff;
                        const int wi = yy * LDS_ROW + (xx >> 5);
                        const uint32_t b0 = (slot[wi] >> (xx & 31)) & 1u;
                        const uint32_t b1 = (slot[pw + wi] >> (xx & 31)) & 1u;
                        return (class_blocked(agent_class(clo, chi, i), b0, b1) & 1u) == 0u;
                    } else {
                        return board_bit(slot, pc) == 0u;
                    }
                };
                bool by_rule = true;
                // ceil(2^18 / Wd): (c * wdiv) >> 18 is c / Wd for every cell
                // index c of the map (c < 2^12, Wd <= 64: the rounding error
                // stays below 2^18)
                const uint32_t wdiv = ((1u << 18) + (uint32_t)Wd - 1u) / (uint32_t)Wd;
                if constexpr (FAST_SPAWN) {
                    // The rule's first SA draws of every agent, made side
                    // by side (draw j of agent i by lane j * NMAX + i of
                    // the env) and broadcast to the env's lanes; when
                    // each agent takes one of them, the placement is
                    // settled in registers. Otherwise the rule runs in
                    // full, from the first agent.
                    const uint32_t cells = (uint32_t)(H * Wd);
                    const U4 x = philox(env, (ST_SPAWN << 24) | (uint32_t)(l % NMAX), ep,
                                        (uint32_t)(l / NMAX), k0, k1);
                    const uint32_t mine_c = range_map(x.x, cells);
                    int cpc[SA][NMAX];
                    uint32_t cfree[SA][NMAX];
#pragma unroll
                    for (int j = 0; j < SA; ++j) {
#pragma unroll
                        for (int i = 0; i < NMAX; ++i) {
                            const uint32_t c = env_lane_bcast<LANES>(mine_c, j * NMAX + i);
                            // c / Wd, exact for c < 2^12 and Wd <= 64
                            const uint32_t y = (c * wdiv) >> 18, xx = c - y * (uint32_t)Wd;
                            cpc[j][i] = (int)(((y + PAD) << 8) | (xx + PAD));
                            cfree[j][i] = board_bit(slot, cpc[j][i]) ^ 1u;
                        }
                    }
                    int np[NMAX];
                    uint32_t all_ok = 1u;
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) {
                        uint32_t placed = 0u;
                        int p = FAR_CELL;
#pragma unroll
                        for (int j = 0; j < SA; ++j) {
                            uint32_t ok = cfree[j][i] & (placed ^ 1u);
#pragma unroll
                            for (int k = 0; k < i; ++k) ok &= cpc[j][i] != np[k] ? 1u : 0u;
                            p = ok ? cpc[j][i] : p;
                            placed |= ok;
                        }
                        np[i] = i < n ? p : FAR_CELL;
                        all_ok &= (i < n) ? placed : 1u;
                    }
                    if (all_ok) {
#pragma unroll
                        for (int jj = 0; jj < NMAX; ++jj) pp[jj] = np[jj];
                        by_rule = false;
                    }
                }
                if constexpr (LANE_SPAWN) {
                    // Each lane makes the rule's first SL draws of its own
                    // agents and keeps those the agent may stand on (as
                    // packed cells). Then, agent by agent in index order, the
                    // agent's lane offers its first kept draw, every lane of
                    // the env takes it (a broadcast from that lane) and drops
                    // that cell from its own draws. This is the rule's choice
                    // as long as each agent still has a kept draw; if one has
                    // none left, the rule runs in full, from the first agent.
                    const uint32_t cells = (uint32_t)(H * Wd);
                    uint32_t dr[TPL][SL];
#pragma unroll
                    for (int m = 0; m < TPL; ++m) {
                        const int a = l + m * LANES;
                        // draws SL-1 down to 0, shifted in (one generator
                        // block at a time: few registers)
#pragma unroll 1
                        for (int j = SL - 1; j >= 0; --j) {
                            const U4 x = philox(env, (ST_SPAWN << 24) | (uint32_t)a, ep, (uint32_t)j, k0, k1);
                            const uint32_t c = range_map(x.x, cells);
                            const uint32_t y = (c * wdiv) >> 18, xx = c - y * (uint32_t)Wd;
                            const int pc = (int)(((y + PAD) << 8) | (xx + PAD));
#pragma unroll
                            for (int jj = SL - 1; jj > 0; --jj) dr[m][jj] = dr[m][jj - 1];
                            dr[m][0] = (a < n && may_stand(a, pc)) ? (uint32_t)pc : NO_CELL;
                        }
                    }
                    uint32_t fail = 0u;
#pragma unroll
                    for (int a = 0; a < NMAX; ++a) {
                        const int m = a / LANES;
                        uint32_t f = dr[m][SL - 1];
#pragma unroll
                        for (int j = SL - 2; j >= 0; --j) f = dr[m][j] != NO_CELL ? dr[m][j] : f;
                        const uint32_t ch = env_bcast<LANES>(f, a % LANES);
                        fail |= (a < n && ch == NO_CELL) ? 1u : 0u;
                        pp[a] = a < n ? (int)ch : FAR_CELL;
#pragma unroll
                        for (int m2 = 0; m2 < TPL; ++m2)
#pragma unroll
                            for (int j = 0; j < SL; ++j) dr[m2][j] = dr[m2][j] == ch ? NO_CELL : dr[m2][j];
                    }
                    by_rule = fail != 0u;
                }
                if (by_rule) {
                    spawn_agents_if(spawned, n, H, Wd, env, k0, k1, ep, may_stand);
                    wave_lds_fence();
#pragma unroll
                    for (int jj = 0; jj < NMAX; ++jj) pp[jj] = jj < n ? spawned[jj] : FAR_CELL;
                }
                {
                    const int from = mine[0];
                    if constexpr (DUP)
                        own_positions_ids<NMAX, TPL>(pp, aid, mine);
                    else
                        own_positions<LANES, NMAX, TPL>(pp, l, n, mine);
                    plane_move(from, mine[0]);
                }
                all_masks<R, W, NMAX, TPL, EX, OC, TER, PL>(slot, H, Wd, pp, l, LANES, mine, n, S,
                                                            want_out, LOS, false, wall, outm, team,
                                                            opp, seen, cnt, pw, clo, chi, planes, plw, aid);
#pragma unroll
                for (int m = 0; m < TPL; ++m)
                    if (DUP || mine_live[m]) store_obs(m);
                if constexpr (NBR)
                    nbw = gather_blocked<LANES, NMAX, TPL>(l, [&](int m) { return blocked_field<R, W>(wall[m]); });
            }
            // ---- 7 the discovery map after the step (centralised observation)
            if constexpr (XP) {
                if (map_p != nullptr) {
                    wave_lds_fence();
                    map_store<LANES>(map_p, mslot, H, Wd, l);
                    map_p += J.map_stride;
                }
            }
            // ---- 8 the true state after the step (observability modes with
            // the true state): positions, then found / t / episode / stuck
            if (want_state) {
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    if (mine_live[m]) {
                        const uint32_t pc = (uint32_t)mine[m];
                        spos_p[l + m * LANES] = (uint16_t)(((pc & 0xffu) - PAD) | (((pc >> 8) - PAD) << 8));
                    }
                }
                if (active && l == 0) {
                    typedef uint32_t u32x4s __attribute__((ext_vector_type(4)));
                    u32x4s v;
                    v.x = found;
                    v.y = t;
                    v.z = ep;
                    v.w = stuck;
                    *(GAS u32x4s *)senv_p = v;
                }
                spos_p += J.agent_stride;
                senv_p += J.env_stride * 4u;
            }
            steps += 1u;
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                obs_l[m] += J.obs_stride;
                rew_l[m] += J.agent_stride;
            }
            done_p += J.env_stride;
        };

        // action words of this lane's generator block: 4 draws mapped to 0..4
        auto block_actions = [&](uint32_t sub, uint32_t step) __attribute__((always_inline)) {
            const U4 x = philox(env, (ST_ACTION << 24) | sub, step, 0u, k0, k1);
            return range_map(x.x, 5u) | (range_map(x.y, 5u) << 3) | (range_map(x.z, 5u) << 6) |
                   (range_map(x.w, 5u) << 9);
        };
        // External action bytes of agents 4g .. 4g+3 at step `row` of this
        // launch, as loaded (byte i for agent 4g + i), and the bytes that
        // count as draws (past the env's agents or past the launch's steps).
        // Every load reads inside the buffer (rows and agents are clamped)
        // and nothing branches per lane, so the loads of the next window are
        // in flight while the current one runs; they are only looked at
        // when merged into that window.
        struct ExtBytes {
            uint32_t b[4], draw;
        };
        const GAS int8_t *const act0 = act_p;
        auto ext_bytes = [&](uint32_t row, uint32_t g) __attribute__((always_inline)) {
            ExtBytes x;
            x.draw = 0xffffffffu;
#pragma unroll
            for (int i = 0; i < 4; ++i) x.b[i] = 0u;
            if (has_act) {
                const uint32_t rr = row < nsteps ? row : nsteps - 1u;
                const GAS int8_t *rp = act0 + (uint64_t)rr * J.agent_stride;
                x.draw = row < nsteps ? 0u : 0xffffffffu;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int a = (int)(4u * g) + i;
                    x.b[i] = (uint32_t)(uint8_t)rp[a < n ? a : n - 1];
                    x.draw |= a < n ? 0u : 0xffu << (8 * i);
                }
            }
            return x;
        };
        // a generator block's four 3-bit actions with the external bytes
        // merged in (-1 keeps the draw, 0..4 replaces it, anything else stays;
        // with radio v >= 0 moves v mod 5)
        auto merge_ext = [&](uint32_t drawn, const ExtBytes &x) __attribute__((always_inline)) {
            if (!has_act) return drawn;
            const uint32_t bytes = (x.b[0] | (x.b[1] << 8) | (x.b[2] << 16) | (x.b[3] << 24)) | x.draw;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v = (int)(int8_t)(bytes >> (8 * i));
                uint32_t a = (v >= 0 && v <= 4) ? (uint32_t)v : 0u;
                if constexpr (RAD) a = v >= 0 ? (uint32_t)v % 5u : 0u;
                drawn = v == -1 ? drawn : ((drawn & ~(7u << (3 * i))) | (a << (3 * i)));
            }
            return drawn;
        };
        // a radio block's four 5-bit targets (agents 4g .. 4g+3) with the
        // external bytes merged in: v >= 0 names agent v div 5 - 1 (0 or
        // past the last agent: no message, the agent's own index), -1
        // keeps the draw, anything else sends nothing
        auto merge_tgt = [&](uint32_t drawn, const ExtBytes &x, uint32_t g) __attribute__((always_inline)) {
            if (!has_act) return drawn;
            const uint32_t bytes = (x.b[0] | (x.b[1] << 8) | (x.b[2] << 16) | (x.b[3] << 24)) | x.draw;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v = (int)(int8_t)(bytes >> (8 * i));
                const uint32_t c = v >= 0 ? (uint32_t)v / 5u : 0u;
                const uint32_t t = (c >= 1u && c <= (uint32_t)n) ? c - 1u : 4u * g + (uint32_t)i;
                drawn = v == -1 ? drawn : ((drawn & ~(31u << (5 * i))) | (t << (5 * i)));
            }
            return drawn;
        };

        if constexpr (DPP_WINDOW) {
            // lane l draws the block of step steps + l; a window covers LANES steps
            // (the external bytes of the next window are loaded while the
            // current one runs)
            if constexpr (UNROLL && !OC) {
                // two copies of the unrolled loop, with and without external
                // actions, so the loads of the next window stay in flight
                // (with a run-time test around them, the join after it waited
                // for every outstanding load)
                auto window_loop = [&](auto with_act) __attribute__((always_inline)) {
                    constexpr bool WA = decltype(with_act)::value;
                    uint32_t k = 0;
                    ExtBytes nb{};
                    if constexpr (WA) nb = ext_bytes((uint32_t)l, 0u);
                    for (; k + LANES <= nsteps; k += LANES) {
                        const ExtBytes cb = nb;
                        uint32_t drawn = block_actions(0u, steps + (uint32_t)l);
                        if constexpr (WA) {
                            nb = ext_bytes(k + LANES + (uint32_t)l, 0u);
                            drawn = merge_ext(drawn, cb);
                        }
                        const uint64_t w = gather_window<LANES>(drawn);
#pragma unroll
                        for (int jw = 0; jw < LANES; ++jw) step((w >> (12 * jw)) & 0xfffull);
                    }
                    if (k < nsteps) {
                        uint32_t drawn = block_actions(0u, steps + (uint32_t)l);
                        if constexpr (WA) drawn = merge_ext(drawn, nb);
                        const uint64_t w = gather_window<LANES>(drawn);
                        for (uint32_t jw = 0; k < nsteps; ++k, ++jw) step((w >> (12u * jw)) & 0xfffull);
                    }
                };
                if (has_act)
                    window_loop(std::true_type{});
                else
                    window_loop(std::false_type{});
            } else if constexpr (KIND == KIND_PLAIN) {
                // one loop, the window drawn when its index wraps (measured
                // faster than the nested form below for the plain loops)
                uint64_t w = 0;
                ExtBytes nb = ext_bytes((uint32_t)l, 0u);
                for (uint32_t k = 0; k < nsteps; ++k) {
                    const uint32_t jw = k & (uint32_t)(LANES - 1);
                    if (jw == 0u) {
                        const ExtBytes cb = nb;
                        nb = ext_bytes(k + LANES + (uint32_t)l, 0u);
                        w = gather_window<LANES>(merge_ext(block_actions(0u, steps + (uint32_t)l), cb));
                    }
                    step((w >> (12u * jw)) & 0xfffull);
                }
            } else {
                // the feature loops: one window per outer iteration (with the
                // single-loop form the compiler threaded the wrap test into
                // an irreducible loop)
                ExtBytes nb = ext_bytes((uint32_t)l, 0u);
                for (uint32_t left = nsteps; left != 0u;) {
                    const ExtBytes cb = nb;
                    nb = ext_bytes(nsteps - left + LANES + (uint32_t)l, 0u);
                    const uint64_t w = gather_window<LANES>(
                        WIN_ACT ? merge_ext(block_actions(0u, steps + (uint32_t)l), cb)
                                : block_actions(0u, steps + (uint32_t)l));
                    const uint32_t nw = left < (uint32_t)LANES ? left : (uint32_t)LANES;
#pragma unroll 1
                    for (uint32_t jw = 0; jw < nw; ++jw) step((w >> (12u * jw)) & 0xfffull);
                    left -= nw;
                }
            }
        } else if constexpr (WINDOWED && KIND == KIND_PLAIN) {
            // lane l draws block (step + wstep, group wgroup) of the window
            uint32_t win = 0;
            int j = 0;
            ExtBytes nb = ext_bytes((uint32_t)wstep, (uint32_t)wgroup);
            for (uint32_t k = 0; k < nsteps; ++k) {
                if (j == 0) {
                    const ExtBytes cb = nb;
                    nb = ext_bytes(k + (uint32_t)kb + (uint32_t)wstep, (uint32_t)wgroup);
                    win = merge_ext(block_actions((uint32_t)wgroup, steps + (uint32_t)wstep), cb);
                }
                uint64_t acts = 0;
#pragma unroll
                for (int g = 0; g < MAXCALLS; ++g) {
                    if (g < ncalls) {
                        const uint32_t v = (uint32_t)__shfl((int)win, q * LANES + j * ncalls + g, 64);
                        acts |= (uint64_t)v << (12 * g);
                    }
                }
                step(acts);
                j = (j + 1 == kb) ? 0 : j + 1;
            }
        } else if constexpr (WINDOWED) {
            // the same, one window of kb steps per outer iteration; compiled
            // twice, with and without external actions (a run-time test
            // around the byte loads makes the compiler wait for every
            // outstanding store where the paths join)
            auto feature_loop = [&](auto with_act) __attribute__((always_inline)) {
                constexpr bool WA = decltype(with_act)::value && WIN_ACT;
                ExtBytes nb{};
                if constexpr (WA) nb = ext_bytes((uint32_t)wstep, (uint32_t)wgroup);
                for (uint32_t left = nsteps; left != 0u;) {
                    const ExtBytes cb = nb;
                    const uint32_t drawn = block_actions((uint32_t)wgroup, steps + (uint32_t)wstep);
                    uint32_t win = drawn;
                    if constexpr (WA) {
                        nb = ext_bytes(nsteps - left + (uint32_t)kb + (uint32_t)wstep, (uint32_t)wgroup);
                        win = merge_ext(drawn, cb);
                    }
                    if constexpr (RWIN) {
                        rwin = block_targets((uint32_t)wgroup, steps + (uint32_t)wstep);
                        if constexpr (WA) rwin = merge_tgt(rwin, cb, (uint32_t)wgroup);
                    }
                    const uint32_t nw = left < (uint32_t)kb ? left : (uint32_t)kb;
#pragma unroll 1
                    for (uint32_t j = 0; j < nw; ++j) {
                        if constexpr (RWIN) rj = j;
                        uint64_t acts = 0;
#pragma unroll
                        for (int g = 0; g < MAXCALLS; ++g) {
                            if (g < ncalls) {
                                const uint32_t v =
                                    (uint32_t)__shfl((int)win, q * LANES + (int)j * ncalls + g, 64);
                                acts |= (uint64_t)v << (12 * g);
                            }
                        }
                        step(acts);
                    }
                    left -= nw;
                }
            };
            if (has_act)
                feature_loop(std::true_type{});
            else
                feature_loop(std::false_type{});
        } else {
            for (uint32_t k = 0; k < nsteps; ++k) {
                uint64_t acts = 0;
#pragma unroll
                for (int g = 0; g < MAXCALLS; ++g)
                    if (g < ncalls) acts |= (uint64_t)block_actions((uint32_t)g, steps) << (12 * g);
                step(acts);
            }
        }
    };
    // The feature loops use the exact per-agent channels, which are right
    // whether or not agents may share a cell; the distinct-cell shortcut is
    // kept for the plain loop and the two single-feature kinds below.
    if constexpr (KIND == KIND_PLAIN) {
        if (collide)
            run(std::false_type{}, std::integral_constant<int, 0>{});
        else
            run(std::true_type{}, std::integral_constant<int, 0>{});
    } else if constexpr (KIND == KIND_TERRAIN || KIND == KIND_RADIO) {
        // terrain alone and radio alone also take the shortcut when
        // collisions keep agents on distinct cells (stuck agents stay put,
        // rescue moves nobody, radio moves nobody): the exact test of every
        // agent against every window cost terrain4k a quarter of its
        // vector instructions
        if (collide)
            run(std::false_type{}, std::integral_constant<int, KIND>{});
        else
            run(std::true_type{}, std::integral_constant<int, KIND>{});
    } else {
        run(std::true_type{}, std::integral_constant<int, KIND>{});
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
        for (int jj = 0; jj < NMAX; ++jj) {
            if (jj < n && (jj % LANES) == l) {
                const uint32_t x = (uint32_t)(pp[jj] & 0xff) - PAD, y = (uint32_t)(pp[jj] >> 8) - PAD;
                gp(J.pos)[agent_off + (uint32_t)jj] = (uint16_t)(x | (y << 8));
            }
        }
        if constexpr (XPL) {
            wave_lds_fence();
            map_store<LANES>(gp(J.disc) + map_off, mslot, H, Wd, l);
        }
        if constexpr (TER) {
            if (l == 0) gp(J.stuck)[e] = stuck;
        }
        if constexpr (RAD) {
#pragma unroll
            for (int m = 0; m < TPL; ++m)
                if (mine_live[m]) gp(J.bel)[agent_off + (uint32_t)(l + m * LANES)] = bel[m];
        }
    }
}

// One variant: every tile of the launch has the same (LANES, NMAX, R).
template <int LANES, int NMAX, int R>
__global__ __launch_bounds__(64) void step_kernel(const Tile *__restrict__ tiles, uint32_t n_tiles,
                                                  const JobDesc *__restrict__ jobs, JobDesc job0,
                                                  uint32_t K, uint32_t step_base, uint32_t slot_words)
{
    extern __shared__ uint32_t lds[];
    if (blockIdx.x >= n_tiles) return;
    const Tile tile = tiles[blockIdx.x];
    const JobDesc J = jobs ? jobs[tile.job] : job0;
    step_tile<LANES, NMAX, R, true, KIND_PLAIN>(tile, J, K, step_base, slot_words, 0u, lds);
}

// Variant code of a tile: agent-count bucket * 4 + radius - 1.
__host__ __device__ constexpr uint32_t variant_code(int bucket, int r) { return (uint32_t)(bucket * 4 + r - 1); }

template <int LANES, int NMAX, int KIND>
__device__ __forceinline__ void mixed_nmax(int r, const Tile &tile, const JobDesc &J, uint32_t K,
                                           uint32_t step_base, uint32_t slot_words,
                                           uint32_t map_words, uint32_t *lds)
{
    if constexpr ((NMAX + LANES - 1) / LANES <= 4) {
        switch (r) {
        case 1: step_tile<LANES, NMAX, 1, false, KIND>(tile, J, K, step_base, slot_words, map_words, lds); break;
        case 2: step_tile<LANES, NMAX, 2, false, KIND>(tile, J, K, step_base, slot_words, map_words, lds); break;
        case 3: step_tile<LANES, NMAX, 3, false, KIND>(tile, J, K, step_base, slot_words, map_words, lds); break;
        default: step_tile<LANES, NMAX, 4, false, KIND>(tile, J, K, step_base, slot_words, map_words, lds); break;
        }
    }
}

template <int LANES, int B, int KIND>
__device__ __forceinline__ void mixed_bucket(int r, const Tile &tile, const JobDesc &J, uint32_t K,
                                             uint32_t step_base, uint32_t slot_words,
                                             uint32_t map_words, uint32_t *lds)
{
    mixed_nmax<LANES, BUCKET_NMAX[B], KIND>(r, tile, J, K, step_base, slot_words, map_words, lds);
}

// Mixed variants in one launch (uneven batches, feature kinds): each wave
// runs the code of its own tile's (bucket, radius), chosen by a wave-uniform
// switch, so every bucket of the batch shares the chip at once. One kernel
// per env kind for the buckets of up to 10 agents and one for the bucket of
// up to 20 (BIG): the registers a kernel gets are those of its heaviest
// code, and with the 20-agent code inside, the 16-lane plain kernel needed
// 292 VGPRs (one wave per SIMD) where the others need 238 (two).
template <int LANES, int KIND, bool BIG>
__global__ __launch_bounds__(64) void step_kernel_mixed(const Tile *__restrict__ tiles,
                                                        uint32_t n_tiles,
                                                        const JobDesc *__restrict__ jobs,
                                                        JobDesc job0, uint32_t K,
                                                        uint32_t step_base, uint32_t slot_words,
                                                        uint32_t map_words)
{
    extern __shared__ uint32_t lds[];
    if (blockIdx.x >= n_tiles) return;
    const Tile tile = tiles[blockIdx.x];
    // arena launches run one group over the whole tile table, whose other
    // entries belong to other groups or are empty
    if (tile.count == 0u || (job0.group != ALL_GROUPS && (tile.variant >> 8) != job0.group)) return;
    const JobDesc J = jobs ? jobs[tile.job] : job0;
    const int bucket = (int)((tile.variant >> 2) & 3u), r = (int)(tile.variant & 3u) + 1;
    if constexpr (BIG) {
        if (bucket == 3) mixed_bucket<LANES, 3, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds);
    } else {
        switch (bucket) {
        case 0: mixed_bucket<LANES, 0, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds); break;
        case 1: mixed_bucket<LANES, 1, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds); break;
        case 2: mixed_bucket<LANES, 2, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds); break;
        default: break;
        }
    }
}

// Plain envs of an uneven batch in one launch at up to three widths: the
// buckets of up to 2 and up to 4 agents at 4 lanes per env (16 envs per
// wave), those buckets and the one of up to 10 agents at 16 lanes (bit 4 of
// a tile's variant set), except that the envs of that bucket with at most 8
// agents take 8 lanes, one agent per lane (bit 5 set): 8 envs per wave in
// place of 4, so the batch needs fewer of the heaviest waves. One grid keeps
// every SIMD busy to the end, where launch groups of different widths
// finish at different times, and small envs need not spread over 16 lanes.
template <int KIND>
__global__ __launch_bounds__(64) void step_kernel_combo(const Tile *__restrict__ tiles,
                                                        uint32_t n_tiles,
                                                        const JobDesc *__restrict__ jobs,
                                                        JobDesc job0, uint32_t K,
                                                        uint32_t step_base, uint32_t slot_words,
                                                        uint32_t map_words)
{
    extern __shared__ uint32_t lds[];
    if (blockIdx.x >= n_tiles) return;
    const Tile tile = tiles[blockIdx.x];
    if (tile.count == 0u || (job0.group != ALL_GROUPS && (tile.variant >> 8) != job0.group)) return;
    const JobDesc J = jobs ? jobs[tile.job] : job0;
    const int bucket = (int)((tile.variant >> 2) & 3u), r = (int)(tile.variant & 3u) + 1;
    if ((tile.variant >> 5) & 1u) {
        mixed_nmax<8, COMBO_MID_NMAX, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds);
    } else if ((tile.variant >> 4) & 1u) {
        switch (bucket) {
        case 0: mixed_bucket<16, 0, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds); break;
        case 1: mixed_bucket<16, 1, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds); break;
        case 2: mixed_bucket<16, 2, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds); break;
        default: break;
        }
    } else {
        switch (bucket) {
        case 0: mixed_bucket<4, 0, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds); break;
        case 1: mixed_bucket<4, 1, KIND>(r, tile, J, K, step_base, slot_words, map_words, lds); break;
        default: break;
        }
    }
}

// ------------------------------------------------------------ launch helpers

template <int LANES, int NMAX, int R>
inline hipError_t launch_variant(const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                                 const JobDesc &job0, uint32_t K, uint32_t step_base,
                                 uint32_t slot_words, hipStream_t stream)
{
    // env slots with the two agent planes where one lane holds one of more
    // than 4 agents
    constexpr bool planes = LANES >= 8 && NMAX > 4 && NMAX <= LANES;
    const size_t lds =
        (size_t)(64 / LANES) * (slot_words * (planes ? 3u : 1u) + MAX_AGENTS) * sizeof(uint32_t);
    hipLaunchKernelGGL((step_kernel<LANES, NMAX, R>), dim3(n_tiles), dim3(64), lds, stream, tiles,
                       n_tiles, jobs, job0, K, step_base, slot_words);
    return hipGetLastError();
}

template <int LANES, int NMAX>
inline hipError_t launch_radius(int r, const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                                const JobDesc &job0, uint32_t K, uint32_t step_base,
                                uint32_t slot_words, hipStream_t stream)
{
    if constexpr ((NMAX + LANES - 1) / LANES > 4) {
        return hipErrorInvalidValue;
    } else {
    switch (r) {
    case 1: return launch_variant<LANES, NMAX, 1>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 2: return launch_variant<LANES, NMAX, 2>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 3: return launch_variant<LANES, NMAX, 3>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 4: return launch_variant<LANES, NMAX, 4>(tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    default: return hipErrorInvalidValue;
    }
    }
}

template <int LANES>
inline hipError_t launch_lanes(int nmax, int r, const Tile *tiles, uint32_t n_tiles,
                               const JobDesc *jobs, const JobDesc &job0, uint32_t K,
                               uint32_t step_base, uint32_t slot_words, hipStream_t stream)
{
    switch (nmax) {
    case 2: return launch_radius<LANES, 2>(r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 4: return launch_radius<LANES, 4>(r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 10: return launch_radius<LANES, 10>(r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    case 20: return launch_radius<LANES, 20>(r, tiles, n_tiles, jobs, job0, K, step_base, slot_words, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int LANES, int KIND>
inline hipError_t launch_mixed_l(const Tile *tiles, uint32_t n_tiles, const JobDesc *jobs,
                                 const JobDesc &job0, uint32_t K, uint32_t step_base,
                                 uint32_t slot_words, uint32_t map_words, bool big,
                                 hipStream_t stream)
{
    // the 16-lane kernels without terrain hold the bucket of up to 10
    // agents, whose env slots carry the two agent planes
    constexpr bool planes = LANES >= 16 && (KIND & KIND_TERRAIN) == 0;
    const size_t lds = (size_t)(64 / LANES) *
                       (slot_words * (planes ? 3u : 1u) + MAX_AGENTS + map_words) *
                       sizeof(uint32_t);
    if (big)
        hipLaunchKernelGGL((step_kernel_mixed<LANES, KIND, true>), dim3(n_tiles), dim3(64), lds,
                           stream, tiles, n_tiles, jobs, job0, K, step_base, slot_words, map_words);
    else
        hipLaunchKernelGGL((step_kernel_mixed<LANES, KIND, false>), dim3(n_tiles), dim3(64), lds,
                           stream, tiles, n_tiles, jobs, job0, K, step_base, slot_words, map_words);
    return hipGetLastError();
}

}  // namespace hase
