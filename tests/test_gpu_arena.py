"""Arena ranges (hase_reset_range / hase_step_resident / hase_release_range)
on the GPU: every range's outputs equal, bit for bit, those of the batch that
hase_create + hase_reset make of the same envs (and the oracle's), whatever
else is admitted, stepped or released around it, through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as o  # noqa: E402
from paper_2604_27162_amd import hase, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

SPECS = {
    "plain": wl.spec(16, 16, 2, 2, 3, 10),
    "multi": wl.spec(32, 32, 10, 4, 4, 15),
    "big": wl.spec(64, 64, 5, 3, 4, 20),
    "explore_los": wl.spec(24, 40, 3, 3, 4, 12, flags=wl.DEFAULT_FLAGS | wl.EXPLORE | wl.OCCLUDE),
    "terrain": wl.with_terrain(wl.spec(20, 20, 6, 2, 4, 10)),
    "radio": wl.spec(16, 24, 7, 4, 4, 10, flags=wl.DEFAULT_FLAGS | wl.RADIO),
    "short_episodes": wl.spec(12, 12, 4, 2, 4, 15, L=9),
    "mid8": wl.spec(16, 16, 8, 3, 4, 20, L=30),
}


def alone(spec, count, seed, steps, env_id_base, maps=False):
    """The same envs as a batch of their own."""
    b = hase.HaseBatch([spec] * count, env_id_base=env_id_base, device=DEV)
    obs0 = b.reset(seed)
    out = b.step(steps, maps=maps)
    torch.cuda.synchronize()
    b.close()
    return obs0, out


def check_range(name, out, count, seed, steps, base):
    spec = SPECS[name]
    maps = "map" in out
    obs0, ref = alone(spec, count, seed, steps, base, maps=maps)
    assert torch.equal(out["obs0"], obs0), f"{name} obs0"
    for k, want in zip(("obs", "rew", "done", "map"), ref):
        assert torch.equal(out[k][:steps], want), f"{name} {k}"


def test_ranges_match_batches_and_oracle():
    ar = hase.HaseArena(600, max_height=64, max_width=64, max_agents=10, max_ranges=16,
                        device=DEV)
    plan = [("plain", 0, 150, 11, 40, 0), ("multi", 150, 37, 12, 100, 5),
            ("big", 200, 21, 13, 77, 0), ("explore_los", 230, 45, 14, 64, 1000),
            ("terrain", 290, 33, 15, 50, 7), ("radio", 330, 29, 16, 45, 3),
            ("short_episodes", 400, 70, 17, 90, 0), ("mid8", 480, 53, 18, 100, 9)]
    outs = {}
    for name, first, count, seed, steps, base in plan:
        print(f"case: admit {name} at {first} x {count}", flush=True)
        out = ar.alloc_outputs(SPECS[name], count, steps, maps=True)
        ar.reset_range(first, count, SPECS[name], seed, steps, out, env_id_base=base)
        outs[name] = out
    for _ in range(7):  # 7 x 16 steps: every budget runs out, the rest are no-ops
        ar.step(16)
    torch.cuda.synchronize()
    for name, first, count, seed, steps, base in plan:
        assert ar.range_error(first) == -1
        check_range(name, outs[name], count, seed, steps, base)
    # ranges of 16-lane tiles and of 8-lane tiles (5 and 8 agents) against
    # the oracle as well
    for name, first, count, seed, steps, base in (plan[1], plan[2], plan[-1]):
        ob = o.OracleBatch([SPECS[name]] * count, env_id_base=base)
        assert np.array_equal(hase.as_u32(outs[name]["obs0"]), ob.reset(seed)), name
        oo, orr, od = ob.step(steps)
        assert np.array_equal(hase.as_u32(outs[name]["obs"]), oo), name
        assert np.array_equal(outs[name]["rew"].cpu().numpy().view(np.uint32), orr.view(np.uint32)), name
        assert np.array_equal(outs[name]["done"].cpu().numpy(), od), name
    ar.close()


def test_admission_while_others_step_and_slot_reuse():
    """Requests join mid-flight, leave, and their slots are taken by others."""
    ar = hase.HaseArena(300, max_height=32, max_width=32, max_agents=10, max_ranges=4,
                        device=DEV)
    a = ("plain", 0, 100, 21, 60, 0)
    b = ("multi", 100, 50, 22, 70, 0)
    c = ("short_episodes", 0, 90, 23, 33, 9)  # into a's slots after a leaves
    oa = ar.alloc_outputs(SPECS["plain"], 100, 60)
    ar.reset_range(0, 100, SPECS["plain"], 21, 60, oa)
    ar.step(25)
    ob_ = ar.alloc_outputs(SPECS["multi"], 50, 70)
    ar.reset_range(100, 50, SPECS["multi"], 22, 70, ob_)
    ar.step(20)
    ar.step(20)  # a reaches its budget (65 > 60)
    ar.release_range(0)
    oc = ar.alloc_outputs(SPECS["short_episodes"], 90, 33)
    ar.reset_range(0, 90, SPECS["short_episodes"], 23, 33, oc, env_id_base=9)
    for _ in range(4):
        ar.step(12)
    torch.cuda.synchronize()
    check_range(*a[:1], oa, a[2], a[3], a[4], a[5])
    check_range(*b[:1], ob_, b[2], b[3], b[4], b[5])
    check_range(*c[:1], oc, c[2], c[3], c[4], c[5])
    ar.close()


def test_range_argument_errors():
    ar = hase.HaseArena(64, max_height=16, max_width=16, max_agents=4, max_ranges=2, device=DEV)
    sp = SPECS["plain"]
    out = ar.alloc_outputs(sp, 10, 5)
    ar.reset_range(10, 10, sp, 1, 5, out)
    cases = [
        (5, 10, sp, 5),                      # overlaps the range at 10
        (19, 3, sp, 5),                      # starts inside it
        (60, 10, sp, 5),                     # past the arena
        (30, 4, SPECS["multi"], 5),          # beyond the caps
        (30, 4, sp, 0),                      # zero budget
    ]
    for first, count, spec, steps in cases:
        with pytest.raises(hase.HaseError) as ei:
            ar.reset_range(first, count, spec, 1, steps, ar.alloc_outputs(spec, count, max(steps, 1)))
        assert ei.value.code == hase.EINVAL, (first, count)
    ar.reset_range(30, 4, sp, 2, 5, ar.alloc_outputs(sp, 4, 5))
    with pytest.raises(hase.HaseError):  # max_ranges = 2
        ar.reset_range(40, 4, sp, 3, 5, ar.alloc_outputs(sp, 4, 5))
    with pytest.raises(hase.HaseError):
        ar.release_range(11)
    ar.release_range(30)
    ar.reset_range(40, 4, sp, 3, 5, ar.alloc_outputs(sp, 4, 5))
    # batch operations refuse an arena
    assert hase.load().hase_observe(ar._h, None) == hase.EINVAL
    ar.close()


def test_range_without_room_is_reported_and_steps_safely():
    """Envs drawn with too few free cells: the range reports the same first
    env as the oracle's reset, and stepping it until release is harmless to
    the other ranges."""
    bad = wl.spec(5, 5, 20, 1, 3, 22)
    specs = [bad] * 40
    with pytest.raises(ValueError) as eo:
        o.OracleBatch(specs).reset(9)
    first_bad = int(str(eo.value).split()[1])
    ar = hase.HaseArena(200, max_height=16, max_width=16, max_agents=20, max_ranges=4, device=DEV)
    good = SPECS["plain"]
    og = ar.alloc_outputs(good, 60, 30)
    ar.reset_range(100, 60, good, 31, 30, og)
    ob_ = ar.alloc_outputs(bad, 40, 30)
    ar.reset_range(0, 40, bad, 9, 30, ob_)
    assert ar.range_error(0) == first_bad
    assert ar.range_error(100) == -1
    # the same reports in the ranges' pinned error words, written in stream order
    assert int(ob_["err"][0]) == first_bad and int(og["err"][0]) == -1
    for _ in range(3):
        ar.step(10)
    ar.release_range(0)
    torch.cuda.synchronize()
    check_range("plain", og, 60, 31, 30, 0)
    ar.close()
