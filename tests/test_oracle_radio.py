"""Pins of the oracle's radio belief sharing (flag 64; Sec. 3.3, radio
paragraph; reading R29): hand-worked steps, the reduction to the game
without radio (radio adds only the belief word), the radio draws rebuilt
from rocRAND's Philox, and trajectory invariants (the beliefs of an env's
agents together are exactly its Found flags)."""
import json
import os

import numpy as np

from oracle import oracle as o
from paper_2604_27162_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "radio_hand_worked.json")))


def load_case(b, case):
    st = b.get_state()
    st["walls"][:] = 0
    st["pos_x"][:] = case["start"]["pos_x"]
    st["pos_y"][:] = case["start"]["pos_y"]
    st["found"][:] = 0
    st["t"][:] = 0
    st["belief"][:] = 0
    b.set_state(st)


def check_hand_worked(libpath=None):
    for case in GOLD["cases"]:
        b = o.OracleBatch([case["spec"]], libpath=libpath)
        load_case(b, case)
        n = case["spec"]["n"]
        for a, want in zip(case["actions"], case["expected"]):
            obs, rew, done = b.step(1, actions=np.array([a], np.int8))
            s = b.get_state()
            what = f'{case["name"]}: {want["notes"]}'
            assert s["belief"].tolist() == want["belief"], what
            assert int(s["found"][0]) == want["found"], what
            assert list(rew[0]) == want["rew"], what
            assert int(done[0, 0]) == want["done"], what
            per = obs[0].reshape(n, -1)
            if "obs" in want:
                assert per.tolist() == want["obs"], what
                assert [[int(x), int(y)] for x, y in zip(s["pos_x"], s["pos_y"])] == want["pos"], what
            else:
                assert per[:, -1].tolist() == want["belief_words"], what


def test_hand_worked_steps():
    check_hand_worked()


def plain_of(specs):
    return [dict(s, flags=s["flags"] & ~wl.RADIO) for s in specs]


def radio_specs(n_envs, seed):
    """Radio versions of the uneven batch's specs, some with line of sight,
    exploration or terrain, and some with capture ending the episode."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in wl.workload_specs("uneven8k", n_envs):
        extra = int(g.choice([0, 0, wl.OCCLUDE, wl.EXPLORE]))
        sp = dict(s, flags=s["flags"] | wl.RADIO | extra, S=int(g.integers(0, s["n"] + 1)))
        if g.random() < 0.2:
            sp = wl.with_terrain(sp, 15, 10, 50, None, [wl.FLYER] * sp["n"])
        out.append(sp)
    return out


def strip_belief(specs, obs):
    """Observation words of a radio batch without each agent's belief word."""
    keep = []
    for s in specs:
        w = o.words_per_channel(s["r"]) * s["C"]
        radio = 1 if s["flags"] & wl.RADIO else 0
        keep.append(np.tile(np.r_[np.ones(w, bool), np.zeros(radio, bool)], s["n"]))
    return obs[..., np.concatenate(keep)]


def check_reduces_to_plain(libpath=None, n_envs=40, steps=150):
    """Radio changes no move, reward or episode end: with drawn and with
    external actions (moves v mod 5) the outputs equal those of the same envs
    without radio, apart from the belief word."""
    specs = radio_specs(n_envs, 3)
    a = o.OracleBatch(specs, libpath=libpath)
    b = o.OracleBatch(plain_of(specs), libpath=libpath)
    np.testing.assert_array_equal(strip_belief(specs, a.reset(8)), b.reset(8))
    ra, rb = a.step(steps), b.step(steps)
    np.testing.assert_array_equal(strip_belief(specs, ra[0]), rb[0])
    np.testing.assert_array_equal(ra[1], rb[1])
    np.testing.assert_array_equal(ra[2], rb[2])
    acts = wl.radio_actions(steps, specs, 4, draw_frac=0.2)
    pacts = np.where(acts >= 0, acts % 5, acts).astype(np.int8)
    ra, rb = a.step(steps, actions=acts), b.step(steps, actions=pacts)
    np.testing.assert_array_equal(strip_belief(specs, ra[0]), rb[0])
    np.testing.assert_array_equal(ra[1], rb[1])
    np.testing.assert_array_equal(ra[2], rb[2])
    sa, sb = a.get_state(), b.get_state()
    for k in ("pos_x", "pos_y", "found", "t", "episode", "steps"):
        np.testing.assert_array_equal(sa[k], sb[k], err_msg=k)
    assert sa["belief"].any() and not sb["belief"].any()


def test_reduces_to_plain():
    check_reduces_to_plain()


def _key(seed):
    return [seed & 0xFFFFFFFF, seed >> 32]


def check_radio_draws(rocrand_philox, libpath=None):
    """A drawn step equals the external step whose move is the ACTION draw and
    whose target is the RADIO draw: word i & 3 of block (env, 5 << 24 | i >> 2,
    step, 0) mapped to 0..n-1, both words rebuilt from rocRAND."""
    seed, env, steps = 0x5EED0123456789, 7, 40
    for sp in (wl.spec(6, 6, 6, 1, 3, 0, S=2, flags=wl.COLLIDE | wl.RADIO, L=5),
               wl.spec(5, 5, 7, 2, 4, 10, S=3, flags=wl.COLLIDE | wl.RADIO, L=4)):
        n = sp["n"]
        a = o.OracleBatch([sp], env_id_base=env, libpath=libpath)
        b = o.OracleBatch([sp], env_id_base=env, libpath=libpath)
        a.reset(seed)
        b.reset(seed)
        rows = [_key(seed) + [env, (st << 24) | g, s, 0]
                for s in range(steps) for st in (0, 5) for g in range((n + 3) // 4)]
        words = rocrand_philox(rows).reshape(steps, 2, -1, 4)
        acts = np.zeros((steps, n), np.int8)
        for s in range(steps):
            for i in range(n):
                mv = (int(words[s, 0, i >> 2, i & 3]) * 5) >> 32
                tg = (int(words[s, 1, i >> 2, i & 3]) * n) >> 32
                acts[s, i] = mv + 5 * (tg + 1)
        heard = 0
        for s in range(steps):
            oa = a.step(1)
            ob = b.step(1, actions=acts[s:s + 1])
            for x, y in zip(oa, ob):
                np.testing.assert_array_equal(x, y)
            np.testing.assert_array_equal(a.belief, b.belief)
            heard |= int(a.belief[sp["S"]:].any())
        assert heard  # a hider learned something by radio


def test_radio_draws_against_rocrand(rocrand_philox):
    check_radio_draws(rocrand_philox)


def seen_by(spec, px, py, i):
    """Hiders inside seeker i's window (Chebyshev distance <= r; no walls)."""
    m = 0
    for h in range(spec["S"], spec["n"]):
        if max(abs(int(px[i]) - int(px[h])), abs(int(py[i]) - int(py[h]))) <= spec["r"]:
            m |= 1 << h
    return m


def check_trajectory_invariants(libpath=None, n_envs=50, steps=120):
    """Per step: the OR of an env's beliefs is its Found word; beliefs hold
    only hider bits; within an episode beliefs only grow; a finished episode
    leaves every belief empty; each agent's belief word of the observation is
    its state belief; without line of sight a seeker knows every hider in its
    window."""
    specs = radio_specs(n_envs, 5)
    b = o.OracleBatch(specs, libpath=libpath)
    b.reset(17)
    aw = [s["n"] * (o.words_per_channel(s["r"]) * s["C"] + 1) for s in specs]
    offs = np.r_[0, np.cumsum(aw)]
    prev = b.belief.copy()
    grew = 0
    for _ in range(steps):
        obs, _, done = b.step(1)
        st = b.get_state()
        for e, s in enumerate(specs):
            lo, hi = b.agent_off[e], b.agent_off[e] + s["n"]
            bel = st["belief"][lo:hi]
            hm = ((1 << s["n"]) - 1) & ~((1 << s["S"]) - 1)
            assert int(np.bitwise_or.reduce(bel, initial=0)) == int(st["found"][e])
            assert not (bel & ~np.uint32(hm)).any()
            words = obs[0, offs[e]:offs[e + 1]].reshape(s["n"], -1)[:, -1]
            np.testing.assert_array_equal(words, bel)
            if done[0, e]:
                assert not bel.any()
            else:
                assert ((prev[lo:hi] & ~bel) == 0).all()
                grew += int((bel != prev[lo:hi]).any())
                if not s["flags"] & wl.OCCLUDE:
                    for i in range(s["S"]):
                        m = seen_by(s, st["pos_x"][lo:hi], st["pos_y"][lo:hi], i)
                        assert (int(bel[i]) & m) == m
        prev = st["belief"].copy()
    assert grew > 0


def test_trajectory_invariants():
    check_trajectory_invariants()


def test_state_round_trip():
    specs = radio_specs(20, 9)
    a = o.OracleBatch(specs)
    a.reset(3)
    a.step(37)
    b = o.OracleBatch(specs)
    b.set_state(a.get_state())
    for x, y in zip(a.step(40), b.step(40)):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a.belief, b.belief)


def test_negative_codes_and_no_radio_envs_unchanged():
    """Without radio an action byte outside 0..4 is still stay; with radio
    a negative byte other than -1 is stay without a message."""
    sp = wl.spec(6, 6, 4, 1, 3, 0, S=2, flags=wl.COLLIDE, L=50)
    a = o.OracleBatch([sp])
    b = o.OracleBatch([sp])
    a.reset(2)
    b.reset(2)
    for v in (5, 7, 100, -2, -128):
        x = a.step(1, actions=np.full((1, 4), v, np.int8))
        y = b.step(1, actions=np.zeros((1, 4), np.int8))
        for u, w in zip(x, y):
            np.testing.assert_array_equal(u, w)
