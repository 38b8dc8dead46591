/*
 * HASE hide-and-seek step: CPU ORACLE.
 *
 * TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this file's library. The product
 * path (the HIP library under paper_2604_27162_amd/) never calls it, and this
 * file shares no code, header, table or helper with that path.
 *
 * It is a plain, single-threaded, slow and obviously-correct restatement of
 * one vectorised step of the hide-and-seek Dec-POMDP (paper Sec. 3.1, the
 * tuple <I,S,A,T,R,Omega,O,gamma>) reduced to a discrete gridworld:
 *   - blocking tiles stop movement (Sec. 3.2, "Collision Models");
 *   - hiders are controlled randomly (Sec. 3, first paragraph);
 *   - a seeker finding a hider sets the hider's Found flag (Fig. "Bit Packing
 *     Environment Structure", POIState F bit) and is rewarded (Sec. 3.1,
 *     Reward Function);
 *   - episodes end by termination or truncation and reset from the pristine,
 *     unchanged grid (Sec. 4.1 last paragraph, Sec. 4.2);
 *   - environments are desynchronised at initialisation (Sec. 3.3, last
 *     paragraph);
 *   - each agent receives a decentralised observation of its own local
 *     window (Sec. 3.3, observability mode 1);
 *   - optionally (OR_RADIO) agents send their beliefs about the hiders to a
 *     chosen agent by radio (Sec. 3.3, radio paragraph).
 * Readings where the paper is silent are listed in the header comment of each
 * function and in the design notes; every one binds the GPU path as well.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random
 * Numbers: As Easy as 1, 2, 3", SC'11), written here from that paper's
 * definition, keyed by (seed) with counter (env, stream|sub, a, b).
 *
 * Pins: tests/test_oracle_*.py check this file against rocRAND's independent
 * Philox4x32-10, closed forms, hand-worked grids (tests/golden/), invariants
 * and brute-force enumeration on 4x4 grids against an independently written
 * declarative checker.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define OR_COLLIDE 1u
#define OR_CAPTURE 2u
#define OR_DESYNC 4u
#define OR_OCCLUDE 8u
#define OR_EXPLORE 16u
#define OR_TERRAIN 32u
#define OR_RADIO 64u

#define OR_STREAM_ACTION 0u
#define OR_STREAM_SPAWN 1u
#define OR_STREAM_WALL 2u
#define OR_STREAM_DESYNC 3u
#define OR_STREAM_MOVE 4u
#define OR_STREAM_RADIO 5u

#define OR_SPAWN_ATTEMPTS 64

/* Field order of one row of the int32 spec table [n_envs][SP_FIELDS]. The
 * terrain fields (OR_TERRAIN): percent of water and mud cells, percent chance
 * that a walker entering mud gets stuck, percent chance that a move attempt
 * onto a tile succeeds per (agent class, tile) -- walker, swimmer, flyer x
 * ground, water, mud --, and the agent classes, 2 bits per agent (0 walker,
 * 1 swimmer, 2 flyer), agents 0..15 in CLS_LO and 16..19 in CLS_HI. */
enum {
    SP_H = 0, SP_W, SP_N, SP_S, SP_R, SP_C, SP_WALLPCT, SP_FLAGS, SP_L,
    SP_WATERPCT, SP_MUDPCT, SP_STUCKPCT, SP_SPEED, SP_CLS_LO = SP_SPEED + 9, SP_CLS_HI,
    SP_FIELDS
};

/* Tile types (cells of the walls array; without OR_TERRAIN only 0 and 1)
 * and agent classes (reading R28 of the traversal kinetics of Sec. 3.2 and
 * the tile / agent flags of Fig. "Bit Packing Environment Structure"):
 * ground is walkable and flyable, water aquatic and flyable, mud walkable
 * and flyable but sticky for walkers, walls block everyone. */
enum { OR_GROUND = 0, OR_WALL = 1, OR_WATER = 2, OR_MUD = 3 };
enum { OR_WALKER = 0, OR_SWIMMER = 1, OR_FLYER = 2 };

typedef struct {
    int32_t n_envs;
    const int32_t *spec;      /* [n_envs][SP_FIELDS] */
    const int64_t *grid_off;  /* [n_envs] first cell of env e in walls[] */
    const int64_t *agent_off; /* [n_envs] first agent of env e in px/py/rew/actions */
    const int64_t *obs_off;   /* [n_envs] first obs word of env e in one step's obs */
    int64_t agents_total;     /* sum of n over envs */
    int64_t obs_total;        /* sum of n*(C*w + radio) over envs */
    uint8_t *walls;           /* [sum H*W] 1 = blocking tile */
    uint8_t *px, *py;         /* [agents_total] */
    uint32_t *found, *t, *ep, *steps; /* [n_envs] */
    uint64_t *seed;           /* [n_envs] */
    uint32_t *env_id;         /* [n_envs] */
    const int64_t *disc_off;  /* [n_envs] first discovery-map word of env e */
    int64_t disc_total;       /* sum of map words over envs */
    uint32_t *disc;           /* [disc_total] discovery maps (OR_EXPLORE envs) */
    uint32_t *stuck;          /* [n_envs] bit i: agent i is stuck (OR_TERRAIN envs) */
    uint32_t *belief;         /* [agents_total] bit h: the agent knows of hider h (OR_RADIO) */
} or_batch;

/* ---------------------------------------------------------------- Philox */

/* One Philox4x32-10 block (Salmon et al. 2011, Sec. 5): ten rounds of
 * S-box = two 32x32->64 multiplies by the round multipliers, output
 * permutation (c0,c1,c2,c3) <- (hi1^c1^k0, lo1, hi0^c3^k1, lo0), with the key
 * bumped by the Weyl constants between rounds. */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (round < 9) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Word `word` of the block keyed by seed with counter
 * (env, stream<<24 | sub, a, b). */
static uint32_t or_draw(uint64_t seed, uint32_t env, uint32_t stream, uint32_t sub,
                        uint32_t a, uint32_t b, int word)
{
    uint32_t ctr[4] = { env, (stream << 24) | sub, a, b };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    return out[word];
}

/* Map a uniform 32-bit word to {0..m-1} by the multiply-shift method
 * (Lemire 2019, without the rejection step): floor(x*m / 2^32). */
uint32_t or_range(uint32_t x, uint32_t m)
{
    return (uint32_t)(((uint64_t)x * (uint64_t)m) >> 32);
}

/* Integer wall threshold: a cell is a wall iff its word is below
 * floor(pct * 2^32 / 100). */
uint32_t or_wall_threshold(uint32_t pct)
{
    return (uint32_t)(((uint64_t)pct << 32) / 100u);
}

/* --------------------------------------------------------------- helpers */

static int or_words(int r)
{
    int d = 2 * r + 1;
    return (d * d + 31) / 32;
}

static int or_is_seeker(int i, int S) { return i < S; }

/* Observation words of one agent: C channels of or_words(r) words, then,
 * with OR_RADIO, one belief word (reading R29). */
static int or_agent_obs_words(const int32_t *sp)
{
    return sp[SP_C] * or_words(sp[SP_R]) + (((uint32_t)sp[SP_FLAGS] & OR_RADIO) ? 1 : 0);
}

/* Discovery map of an OR_EXPLORE env: H rows of ceil(W/32) words, cell (x,y)
 * at bit x & 31 of word y * ceil(W/32) + x / 32; 0 words for other envs. */
static int or_map_row_words(int W) { return (W + 31) / 32; }

static int or_in_bounds(int x, int y, int W, int H)
{
    return x >= 0 && x < W && y >= 0 && y < H;
}

/* Class of agent i (every agent is a walker without OR_TERRAIN). */
static int or_class(const int32_t *sp, int i)
{
    if (!((uint32_t)sp[SP_FLAGS] & OR_TERRAIN)) return OR_WALKER;
    uint32_t w = (uint32_t)(i < 16 ? sp[SP_CLS_LO] : sp[SP_CLS_HI]);
    return (int)((w >> (2 * (i & 15))) & 3u);
}

/* May an agent of class cls stand on a tile of this type? */
static int or_enterable(int type, int cls)
{
    switch (type) {
    case OR_GROUND: return cls == OR_WALKER || cls == OR_FLYER;
    case OR_WATER: return cls == OR_SWIMMER || cls == OR_FLYER;
    case OR_MUD: return cls == OR_WALKER || cls == OR_FLYER;
    default: return 0;
    }
}

/* Does a uniform 32-bit word x fall below pct percent: x / 2^32 < pct / 100,
 * exactly (pct in 0..100). */
static int or_chance(uint32_t x, int pct)
{
    return (uint64_t)x * 100u < ((uint64_t)(uint32_t)pct << 32);
}

/* ----------------------------------------------------------- line of sight */

/* Does the open segment from the centre of cell (0,0) to the centre of cell
 * (dx,dy) cross the interior of the unit square of cell (ex,ey)? Cells are
 * unit squares centred on integer points. The segment is P(t) = t*(dx,dy),
 * 0 < t < 1; the open square needs |x - ex| < 1/2 and |y - ey| < 1/2. Each
 * coordinate gives an open interval of t (all of t when the direction is 0
 * and the centre lies on the line, none when it does not); the segment
 * crosses the square iff the intersection of these intervals with (0,1) is
 * not empty. Interval ends are fractions num/den with den > 0, compared by
 * cross-multiplication, so the test is exact. A segment through a corner of
 * the square, or along its edge, does not cross it. */
typedef struct { int64_t num, den; } or_frac;

static int or_frac_lt(or_frac a, or_frac b) { return a.num * b.den < b.num * a.den; }

static int or_axis_interval(int d, int e, or_frac *lo, or_frac *hi)
{
    if (d == 0) return e == 0; /* |0 - e| < 1/2 for every t, or never */
    if (d > 0) {
        lo->num = 2 * e - 1; lo->den = 2 * d;  /* t > (2e-1)/(2d) */
        hi->num = 2 * e + 1; hi->den = 2 * d;  /* t < (2e+1)/(2d) */
    } else {
        lo->num = -(2 * e + 1); lo->den = -2 * d; /* dividing by d < 0 swaps the ends */
        hi->num = -(2 * e - 1); hi->den = -2 * d;
    }
    return 1;
}

static int or_segment_crosses(int dx, int dy, int ex, int ey)
{
    or_frac lo = { 0, 1 }, hi = { 1, 1 }, a, b;
    if (!or_axis_interval(dx, ex, &a, &b)) return 0;
    if (dx != 0) {
        if (or_frac_lt(lo, a)) lo = a;
        if (or_frac_lt(b, hi)) hi = b;
    }
    if (!or_axis_interval(dy, ey, &a, &b)) return 0;
    if (dy != 0) {
        if (or_frac_lt(lo, a)) lo = a;
        if (or_frac_lt(b, hi)) hi = b;
    }
    return or_frac_lt(lo, hi);
}

/* Line of sight (reading of the observation function of Sec. 3.1, a
 * deterministic line-of-sight projection, reduced to the grid; enabled per
 * env by OR_OCCLUDE): cell (cx,cy) is visible from the agent's cell (ax,ay)
 * iff no blocking cell -- a wall, or a cell outside the map -- other than
 * the two end cells has its interior crossed by the open segment joining
 * their centres. Only cells of the bounding box of the two cells can be
 * crossed. */
static int or_visible(const int32_t *sp, const uint8_t *walls, int ax, int ay, int cx, int cy)
{
    int H = sp[SP_H], W = sp[SP_W];
    int dx = cx - ax, dy = cy - ay;
    int x0 = dx < 0 ? dx : 0, x1 = dx < 0 ? 0 : dx;
    int y0 = dy < 0 ? dy : 0, y1 = dy < 0 ? 0 : dy;
    for (int ey = y0; ey <= y1; ++ey) {
        for (int ex = x0; ex <= x1; ++ex) {
            if ((ex == 0 && ey == 0) || (ex == dx && ey == dy)) continue;
            int bx = ax + ex, by = ay + ey;
            int blocking = !or_in_bounds(bx, by, W, H) || walls[by * W + bx] == OR_WALL;
            if (blocking && or_segment_crosses(dx, dy, ex, ey)) return 0;
        }
    }
    return 1;
}

/* Agent spawn for episode `e` (reading: agents are placed one after another
 * in index order; agent i tries up to 64 uniformly drawn cells and takes the
 * first that its class may stand on (without OR_TERRAIN: not a wall) and no
 * agent < i holds; if all 64 draws fail it takes the first acceptable cell
 * scanning row-major from the cell after the last draw, wrapping around).
 * The grid itself is never touched: the pristine grid of Sec. 4.2 is the one
 * drawn at reset. */
static void or_spawn(const int32_t *sp, const uint8_t *walls, uint8_t *px, uint8_t *py,
                     uint64_t seed, uint32_t env, uint32_t e)
{
    int H = sp[SP_H], W = sp[SP_W], n = sp[SP_N];
    uint32_t cells = (uint32_t)(H * W);
    for (int i = 0; i < n; ++i) {
        int placed = 0, cls = or_class(sp, i);
        uint32_t c = 0;
        for (int j = 0; j < OR_SPAWN_ATTEMPTS && !placed; ++j) {
            c = or_range(or_draw(seed, env, OR_STREAM_SPAWN, (uint32_t)i, e, (uint32_t)j, 0), cells);
            int x = (int)(c % (uint32_t)W), y = (int)(c / (uint32_t)W);
            int ok = or_enterable(walls[c], cls);
            for (int k = 0; k < i && ok; ++k)
                if (px[k] == x && py[k] == y) ok = 0;
            if (ok) { px[i] = (uint8_t)x; py[i] = (uint8_t)y; placed = 1; }
        }
        for (uint32_t d = 1; d <= cells && !placed; ++d) {
            uint32_t cc = (c + d) % cells;
            int x = (int)(cc % (uint32_t)W), y = (int)(cc / (uint32_t)W);
            int ok = or_enterable(walls[cc], cls);
            for (int k = 0; k < i && ok; ++k)
                if (px[k] == x && py[k] == y) ok = 0;
            if (ok) { px[i] = (uint8_t)x; py[i] = (uint8_t)y; placed = 1; }
        }
    }
}

/* Decentralised observation of every agent (observability mode 1, Sec. 3.3):
 * the (2r+1)x(2r+1) window around the agent, one bit per window cell, bit
 * k = (dy+r)*(2r+1) + (dx+r), packed LSB-first into ceil((2r+1)^2/32) words
 * per channel. Channels: 0 blocking tile or outside the map (with
 * OR_TERRAIN: a tile the agent's class may not enter, or outside), 1
 * teammate (another agent of the same role), 2 opponent, 3 (only when C = 4)
 * outside the map. Layout [agent][channel][word]. With OR_OCCLUDE, a window
 * cell not visible from the agent (or_visible) reads 0 in every channel.
 * With OR_RADIO each agent's words end with its belief word (the 1-D
 * belief vector of the observation space, Sec. 3.1, reading R29). */
static void or_observe(const int32_t *sp, const uint8_t *walls, const uint8_t *px,
                       const uint8_t *py, const uint32_t *belief, uint32_t *obs)
{
    int H = sp[SP_H], W = sp[SP_W], n = sp[SP_N], S = sp[SP_S], r = sp[SP_R], C = sp[SP_C];
    int occlude = ((uint32_t)sp[SP_FLAGS] & OR_OCCLUDE) != 0;
    int d = 2 * r + 1, w = or_words(r), aw = or_agent_obs_words(sp);
    memset(obs, 0, sizeof(uint32_t) * (size_t)(n * aw));
    for (int i = 0; i < n; ++i) {
        uint32_t *oi = obs + (size_t)i * aw;
        if ((uint32_t)sp[SP_FLAGS] & OR_RADIO) oi[aw - 1] = belief[i];
        int cls = or_class(sp, i);
        for (int dy = -r; dy <= r; ++dy) {
            for (int dx = -r; dx <= r; ++dx) {
                int k = (dy + r) * d + (dx + r);
                int cx = px[i] + dx, cy = py[i] + dy;
                if (occlude && !or_visible(sp, walls, px[i], py[i], cx, cy)) continue;
                int inb = or_in_bounds(cx, cy, W, H);
                uint32_t bit = 1u << (k & 31);
                int word = k >> 5;
                if (!inb || !or_enterable(walls[cy * W + cx], cls)) oi[0 * w + word] |= bit;
                if (inb) {
                    for (int j = 0; j < n; ++j) {
                        if (j == i || px[j] != cx || py[j] != cy) continue;
                        if (or_is_seeker(j, S) == or_is_seeker(i, S))
                            oi[1 * w + word] |= bit;
                        else
                            oi[2 * w + word] |= bit;
                    }
                }
                if (C == 4 && !inb) oi[3 * w + word] |= bit;
            }
        }
    }
}

/* ---------------------------------------------------------------- reset */

/* reset(seed) of every env: draw the iid walls (with OR_TERRAIN the tile
 * types: the same word per cell is a wall below the wall threshold, else
 * water below the threshold of wall + water percent, else mud below that of
 * wall + water + mud percent, else ground), check there are enough free
 * cells (at least n; with OR_TERRAIN at least n cells that each class
 * present among the agents may stand on), clear the counters, spawn episode
 * 0, draw the desynchronising initial elapsed time t0 (reading of Sec. 3.3:
 * instead of stepping each env a random number of times, its first episode
 * starts with t0 ~ U{0..L-1} steps already elapsed), and write the episode's
 * first observation into obs0. Returns 0, or -(1 + e) for the first env e
 * without enough free cells. */
int or_reset(or_batch *b, uint64_t seed, uint32_t *obs0)
{
    for (int e = 0; e < b->n_envs; ++e) {
        const int32_t *sp = b->spec + (size_t)e * SP_FIELDS;
        int H = sp[SP_H], W = sp[SP_W], n = sp[SP_N];
        uint8_t *walls = b->walls + b->grid_off[e];
        uint8_t *px = b->px + b->agent_off[e], *py = b->py + b->agent_off[e];
        uint32_t env = b->env_id[e];
        int terrain = ((uint32_t)sp[SP_FLAGS] & OR_TERRAIN) != 0;
        uint32_t T = or_wall_threshold((uint32_t)sp[SP_WALLPCT]);
        uint32_t Tw = or_wall_threshold((uint32_t)(sp[SP_WALLPCT] + sp[SP_WATERPCT]));
        uint32_t Tm = or_wall_threshold((uint32_t)(sp[SP_WALLPCT] + sp[SP_WATERPCT] + sp[SP_MUDPCT]));
        b->seed[e] = seed;
        for (int c = 0; c < H * W; ++c) {
            uint32_t x = or_draw(seed, env, OR_STREAM_WALL, (uint32_t)(c >> 2), 0, 0, c & 3);
            uint8_t type = x < T ? OR_WALL : OR_GROUND;
            if (terrain && type == OR_GROUND) type = x < Tw ? OR_WATER : (x < Tm ? OR_MUD : OR_GROUND);
            walls[c] = type;
        }
        for (int i = 0; i < n; ++i) {
            int cls = or_class(sp, i), room = 0;
            for (int c = 0; c < H * W; ++c) room += or_enterable(walls[c], cls);
            if (room < n) return -(1 + e);
        }
        b->steps[e] = 0;
        b->ep[e] = 0;
        b->found[e] = 0;
        b->stuck[e] = 0;
        if ((uint32_t)sp[SP_FLAGS] & OR_EXPLORE)
            memset(b->disc + b->disc_off[e], 0, sizeof(uint32_t) * (size_t)(H * or_map_row_words(W)));
        or_spawn(sp, walls, px, py, seed, env, 0);
        if (sp[SP_FLAGS] & OR_DESYNC)
            b->t[e] = or_range(or_draw(seed, env, OR_STREAM_DESYNC, 0, 0, 0, 0), (uint32_t)sp[SP_L]);
        else
            b->t[e] = 0;
        for (int i = 0; i < n; ++i) b->belief[b->agent_off[e] + i] = 0;
        if (obs0) or_observe(sp, walls, px, py, b->belief + b->agent_off[e], obs0 + b->obs_off[e]);
    }
    return 0;
}

/* Observation of the current state (no step), e.g. after loading a state. */
void or_observe_all(or_batch *b, uint32_t *obs)
{
    for (int e = 0; e < b->n_envs; ++e) {
        const int32_t *sp = b->spec + (size_t)e * SP_FIELDS;
        or_observe(sp, b->walls + b->grid_off[e], b->px + b->agent_off[e],
                   b->py + b->agent_off[e], b->belief + b->agent_off[e], obs + b->obs_off[e]);
    }
}

/* ----------------------------------------------------------------- step */

static const int OR_DX[5] = { 0, 0, 0, 1, -1 }; /* stay, N, S, E, W */
static const int OR_DY[5] = { 0, -1, 1, 0, 0 };

/* One step of one env, in this order (reading of the step loop of Sec. 4.1):
 *   1 actions: external value if given and not -1, else the ACTION draw at
 *     this env's step count; values outside 0..4 mean stay; with OR_RADIO a
 *     drawn action also draws a radio target (the RADIO draw, uniform over
 *     the n agents, itself meaning no message) and an external value v >= 0
 *     is move v mod 5 plus target v div 5 - 1 (v div 5 = 0 or > n: none);
 *   2 moves in agent-index order; a move is rejected if it leaves the map,
 *     enters a blocking tile, or (collisions on) enters a cell held by any
 *     other agent at that moment (agents < i already moved, agents > i not);
 *     with OR_TERRAIN (reading R28) a stuck agent does not move, a tile its
 *     class may not enter blocks it, and an allowed move succeeds with the
 *     (class, tile) move chance; a walker that enters mud gets stuck with
 *     the stuck chance; then every stuck agent with a teammate that is not
 *     stuck within Chebyshev distance 1 is freed (rescue, Sec. 3.2);
 *   3 detection: seeker i sees hider h iff their Chebyshev distance is <= r
 *     (and, with OR_OCCLUDE, h's cell is visible from i's, or_visible);
 *     seeker reward = hiders seen, hider reward = -(seekers seeing it)
 *     (zero-sum, Sec. 3 "zero-sum adversarial control"); seen hiders get the
 *     latched Found flag;
 *   4 t += 1; terminated = capture rule on, at least one hider, every hider
 *     found; truncated = t >= L; done = terminated | truncated << 1;
 *   3b exploration reward and discovery map (OR_EXPLORE);
 *   3c radio messages (OR_RADIO);
 *   5 if done: next episode, t = 0, Found, stuck and beliefs cleared, agents
 *     respawned, grid kept, discovery map cleared;
 *   6 step count += 1;
 *   7 observation of the (possibly new) state.
 */
static void or_step_env(or_batch *b, int e, const int8_t *act, uint32_t *obs, float *rew,
                        uint8_t *done)
{
    const int32_t *sp = b->spec + (size_t)e * SP_FIELDS;
    int H = sp[SP_H], W = sp[SP_W], n = sp[SP_N], S = sp[SP_S], r = sp[SP_R];
    uint32_t flags = (uint32_t)sp[SP_FLAGS];
    uint32_t L = (uint32_t)sp[SP_L];
    const uint8_t *walls = b->walls + b->grid_off[e];
    uint8_t *px = b->px + b->agent_off[e], *py = b->py + b->agent_off[e];
    uint64_t seed = b->seed[e];
    uint32_t env = b->env_id[e];
    uint32_t *bel = b->belief + b->agent_off[e];
    int radio = (flags & OR_RADIO) != 0;
    int a[20], target[20];

    /* 1 actions (and, with OR_RADIO, radio targets; reading R29) */
    for (int i = 0; i < n; ++i) {
        int v = act ? act[i] : -1;
        target[i] = i;
        if (v == -1) {
            a[i] = (int)or_range(or_draw(seed, env, OR_STREAM_ACTION, (uint32_t)(i >> 2),
                                         b->steps[e], 0, i & 3), 5u);
            if (radio)
                target[i] = (int)or_range(or_draw(seed, env, OR_STREAM_RADIO, (uint32_t)(i >> 2),
                                                  b->steps[e], 0, i & 3), (uint32_t)n);
        } else if (radio && v >= 0) {
            /* move v mod 5; v div 5 = 0 no message, 1..n agent (v div 5) - 1 */
            a[i] = v % 5;
            if (v / 5 >= 1 && v / 5 <= n) target[i] = v / 5 - 1;
        } else {
            a[i] = (v >= 0 && v <= 4) ? v : 0;
        }
    }

    /* 2 moves */
    int terrain = (flags & OR_TERRAIN) != 0;
    for (int i = 0; i < n; ++i) {
        if (a[i] == 0) continue;
        if (terrain && (b->stuck[e] >> i) & 1u) continue;
        int tx = px[i] + OR_DX[a[i]], ty = py[i] + OR_DY[a[i]];
        if (!or_in_bounds(tx, ty, W, H)) continue;
        int type = walls[ty * W + tx], cls = or_class(sp, i);
        if (!or_enterable(type, cls)) continue;
        int blocked = 0;
        if (flags & OR_COLLIDE)
            for (int j = 0; j < n; ++j)
                if (j != i && px[j] == tx && py[j] == ty) blocked = 1;
        if (blocked) continue;
        if (terrain) {
            /* move and stuck draws: words 2(i&1) and 2(i&1)+1 of the MOVE
             * block of agent pair i>>1 at this step count */
            uint32_t u = or_draw(seed, env, OR_STREAM_MOVE, (uint32_t)(i >> 1), b->steps[e], 0,
                                 2 * (i & 1));
            int tile = type == OR_GROUND ? 0 : (type == OR_WATER ? 1 : 2);
            if (!or_chance(u, sp[SP_SPEED + 3 * cls + tile])) continue;
            if (cls == OR_WALKER && type == OR_MUD) {
                uint32_t v = or_draw(seed, env, OR_STREAM_MOVE, (uint32_t)(i >> 1), b->steps[e], 0,
                                     2 * (i & 1) + 1);
                if (or_chance(v, sp[SP_STUCKPCT])) b->stuck[e] |= 1u << i;
            }
        }
        px[i] = (uint8_t)tx;
        py[i] = (uint8_t)ty;
    }
    if (terrain) {
        /* rescue: freed by a teammate that is not stuck, at Chebyshev
         * distance <= 1, after the moves */
        uint32_t before = b->stuck[e];
        for (int i = 0; i < n; ++i) {
            if (!((before >> i) & 1u)) continue;
            for (int j = 0; j < n; ++j) {
                if (j == i || ((before >> j) & 1u)) continue;
                if (or_is_seeker(j, S) != or_is_seeker(i, S)) continue;
                int ddx = px[i] - px[j], ddy = py[i] - py[j];
                if (ddx >= -1 && ddx <= 1 && ddy >= -1 && ddy <= 1) b->stuck[e] &= ~(1u << i);
            }
        }
    }

    /* 3 detection and rewards */
    int count[20];
    for (int i = 0; i < n; ++i) count[i] = 0;
    for (int i = 0; i < S; ++i) {
        for (int h = S; h < n; ++h) {
            int ddx = px[i] - px[h], ddy = py[i] - py[h];
            if (ddx < 0) ddx = -ddx;
            if (ddy < 0) ddy = -ddy;
            int cheb = ddx > ddy ? ddx : ddy;
            int vis = !(flags & OR_OCCLUDE) || or_visible(sp, walls, px[i], py[i], px[h], py[h]);
            if (cheb <= r && vis) {
                count[i] += 1;
                count[h] += 1;
                b->found[e] |= 1u << h;
                if (radio) bel[i] |= 1u << h; /* a seeker knows the hiders it sees */
            }
        }
    }
    /* 3b exploration (reading R27, OR_EXPLORE): each seeker earns 1/128 per
     * cell of its window -- inside the map and, with OR_OCCLUDE, visible --
     * that the env's discovery map did not hold before this step (cells new
     * to several seekers count for each); then every such cell of every
     * seeker enters the map. The reward is (128 v + new) / 128, exact in
     * float32. */
    int fresh[20];
    for (int i = 0; i < n; ++i) fresh[i] = 0;
    if (flags & OR_EXPLORE) {
        uint32_t *map = b->disc + b->disc_off[e];
        int rw = or_map_row_words(W);
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = 0; i < S && i < n; ++i) {
                for (int dy = -r; dy <= r; ++dy) {
                    for (int dx = -r; dx <= r; ++dx) {
                        int cx = px[i] + dx, cy = py[i] + dy;
                        if (!or_in_bounds(cx, cy, W, H)) continue;
                        if ((flags & OR_OCCLUDE) && !or_visible(sp, walls, px[i], py[i], cx, cy))
                            continue;
                        uint32_t *word = map + (size_t)cy * rw + (cx >> 5);
                        uint32_t bit = 1u << (cx & 31);
                        if (pass == 0) {
                            if (!(*word & bit)) fresh[i] += 1; /* counted against the old map */
                        } else {
                            *word |= bit;
                        }
                    }
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        int v = or_is_seeker(i, S) ? count[i] : -count[i];
        if (flags & OR_EXPLORE)
            rew[i] = (float)(128 * v + fresh[i]) * 0.0078125f;
        else
            rew[i] = (float)v;
    }

    /* 3c radio (reading R29, OR_RADIO): every agent whose target is another
     * agent sends it its belief as it stands after this step's sightings;
     * all messages of a step are delivered together (a message received now
     * is forwarded from the next step on). Tiles are not sent: the seekers'
     * discovery map already pools every seeker's visible cells and hiders
     * keep no map. */
    if (radio) {
        uint32_t sent[20];
        for (int i = 0; i < n; ++i) sent[i] = bel[i];
        for (int i = 0; i < n; ++i)
            if (target[i] != i) bel[target[i]] |= sent[i];
    }

    /* 4 termination / truncation */
    b->t[e] += 1;
    uint32_t hider_mask = 0;
    for (int h = S; h < n; ++h) hider_mask |= 1u << h;
    int terminated = (flags & OR_CAPTURE) && n - S > 0 &&
                     (b->found[e] & hider_mask) == hider_mask;
    int truncated = b->t[e] >= L;
    uint8_t d = (uint8_t)((terminated ? 1 : 0) | (truncated ? 2 : 0));
    *done = d;

    /* 5 auto-reset (the new episode's discovery map is empty) */
    if (d) {
        b->ep[e] += 1;
        b->t[e] = 0;
        b->found[e] = 0;
        b->stuck[e] = 0;
        for (int i = 0; i < n; ++i) bel[i] = 0;
        if (flags & OR_EXPLORE)
            memset(b->disc + b->disc_off[e], 0, sizeof(uint32_t) * (size_t)(H * or_map_row_words(W)));
        or_spawn(sp, walls, px, py, seed, env, b->ep[e]);
    }

    /* 6 step counter */
    b->steps[e] += 1;

    /* 7 observation */
    or_observe(sp, walls, px, py, bel, obs);
}

/* n_steps consecutive steps of every env. actions is NULL (every action
 * drawn) or [n_steps][agents_total] int8; outputs are obs
 * [n_steps][obs_total] u32, rew [n_steps][agents_total] f32, done
 * [n_steps][n_envs] u8 and, when maps is not NULL, the discovery maps
 * [n_steps][disc_total] u32. */
void or_step(or_batch *b, int n_steps, const int8_t *actions, uint32_t *obs, float *rew,
             uint8_t *done, uint32_t *maps)
{
    for (int k = 0; k < n_steps; ++k) {
        for (int e = 0; e < b->n_envs; ++e) {
            const int8_t *act = actions ? actions + (size_t)k * b->agents_total + b->agent_off[e] : NULL;
            or_step_env(b, e, act,
                        obs + (size_t)k * b->obs_total + b->obs_off[e],
                        rew + (size_t)k * b->agents_total + b->agent_off[e],
                        done + (size_t)k * b->n_envs + e);
        }
        /* centralised observation (reading R27): every env's discovery map
         * after the step, concatenated */
        if (maps && b->disc_total)
            memcpy(maps + (size_t)k * b->disc_total, b->disc, sizeof(uint32_t) * (size_t)b->disc_total);
    }
}

/* The 4-word Philox block for a raw (counter, key), exported for the pins. */
void or_philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                     uint32_t k1, uint32_t *out)
{
    uint32_t ctr[4] = { c0, c1, c2, c3 }, key[2] = { k0, k1 };
    or_philox4x32_10(ctr, key, out);
}

/* Line of sight of one cell pair, exported so the rule can be tested alone. */
int or_los(const int32_t *sp, const uint8_t *walls, int ax, int ay, int cx, int cy)
{
    return or_visible(sp, walls, ax, ay, cx, cy);
}

/* Plain spawn of one env, exported so the spawn rule can be tested alone. */
void or_spawn_env(const int32_t *sp, const uint8_t *walls, uint8_t *px, uint8_t *py,
                  uint64_t seed, uint32_t env, uint32_t e)
{
    or_spawn(sp, walls, px, py, seed, env, e);
}
