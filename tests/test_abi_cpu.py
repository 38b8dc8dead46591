"""The C-ABI library on the CPU: it loads, exports every function include/hase.h
declares, and its host-only calls (layout, validation, error strings) behave.
No call here launches GPU work."""
import ctypes
import os
import re

import pytest

from paper_2604_27162_amd import hase, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hase.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hase.LIB_PATH):
        from paper_2604_27162_amd import build
        build.build(quiet=True)
    return hase.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hase_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(hase.EXPORTS)


def test_layout_matches_definition(lib):
    specs = wl.uneven_specs(500, 4)
    lay = hase.query_layout(specs)
    words = sum(s["n"] * s["C"] * (((2 * s["r"] + 1) ** 2 + 31) // 32) for s in specs)
    assert lay.obs_words_per_step == words
    assert lay.agents_total == sum(s["n"] for s in specs)
    assert lay.n_envs == 500
    assert lay.cells_total == sum(s["H"] * s["W"] for s in specs)
    assert lay.state_bytes % 256 == 0 and lay.state_bytes > lay.cells_total


def test_uniform_layout(lib):
    lay = hase.query_layout(wl.workload_specs("single16k"))
    assert lay.obs_words_per_step == 16384 * 2 * 3 * 2
    assert lay.agents_total == 32768


@pytest.mark.parametrize("bad", [dict(H=1), dict(W=65), dict(n=0), dict(n=21), dict(S=5, n=4),
                                 dict(r=0), dict(r=5), dict(C=2), dict(C=5), dict(wall_pct=100),
                                 dict(flags=128), dict(L=0),
                                 dict(flags=32, water_pct=60, mud_pct=40),
                                 dict(flags=32, stuck_pct=101), dict(flags=32, speed=(101,) * 9),
                                 dict(flags=32, classes=3), dict(flags=32, classes=1 << 8)])
def test_invalid_spec_rejected(lib, bad):
    s = wl.spec(8, 8, 4, 2, 3, 10)
    s.update(bad)
    with pytest.raises(hase.HaseError) as ei:
        hase.query_layout([s, wl.spec(8, 8, 4, 2, 3, 10)])
    assert ei.value.code == hase.EINVAL


def test_invalid_batch_desc(lib):
    lay = hase.Layout()
    arr = (hase.EnvSpec * 2)(hase.spec_struct(wl.spec(8, 8, 2, 2, 3, 10)),
                             hase.spec_struct(wl.spec(8, 8, 2, 2, 3, 10)))
    for desc in (hase.BatchDesc(0, arr, 1, 0), hase.BatchDesc(5, arr, 2, 0),
                 hase.BatchDesc(3, None, 1, 0)):
        assert lib.hase_query_layout(ctypes.byref(desc), ctypes.byref(lay)) == hase.EINVAL
        assert lib.hase_last_error()


def test_create_rejects_bad_memory_without_touching_the_gpu(lib):
    arr = (hase.EnvSpec * 1)(hase.spec_struct(wl.spec(8, 8, 2, 2, 3, 10)))
    desc = hase.BatchDesc(4, arr, 1, 0)
    h = ctypes.c_void_p()
    assert lib.hase_create(ctypes.byref(desc), None, 1 << 20, None, ctypes.byref(h)) == hase.EINVAL
    assert lib.hase_create(ctypes.byref(desc), 0x1001, 1 << 20, None, ctypes.byref(h)) == hase.EINVAL
    assert lib.hase_create(ctypes.byref(desc), 0x100000, 16, None, ctypes.byref(h)) == hase.ENOMEM
    assert not h.value


def test_null_handles(lib):
    assert lib.hase_step(None, 1, None, None, None, None, 0) == hase.EINVAL
    assert lib.hase_reset(None, 1, None) == hase.EINVAL
    assert lib.hase_observe(None, None) == hase.EINVAL
    assert lib.hase_destroy(None) == hase.OK


def test_error_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert lib.hase_strerror(code)


def test_arena_query_validates(lib):
    assert hase.query_arena(1000, 64, 64, 10, 64) % 256 == 0
    small = hase.query_arena(1000, 16, 16, 2, 64)
    assert small < hase.query_arena(1000, 64, 64, 10, 64)
    for bad in (dict(n_slots=0), dict(max_height=1), dict(max_width=65), dict(max_agents=0),
                dict(max_agents=21), dict(max_ranges=0)):
        kw = dict(n_slots=10, max_height=16, max_width=16, max_agents=4, max_ranges=4)
        kw.update(bad)
        with pytest.raises(hase.HaseError) as ei:
            hase.query_arena(**kw)
        assert ei.value.code == hase.EINVAL


def test_arena_calls_reject_null_handles(lib):
    assert lib.hase_step_resident(None, 1) == hase.EINVAL
    assert lib.hase_release_range(None, 0) == hase.EINVAL
    assert lib.hase_reset_range(None, 0, 1, None, 1, 0, 1, None) == hase.EINVAL
