"""CPU checks of the autotuner's host logic: cache keys, search space, and
the JSON cache round trip (the GPU search itself runs in
tests/test_gpu_tuning.py)."""

import json

from paper_2003_02585_amd import autotune as A


def test_shape_key_names_what_decides_performance():
    k = A.shape_key((2048, 2048), (16, 16), 16, True, 2, 3)
    assert k == "d2 ne160x160 P16x16 ops3 c64 r2"
    k3 = A.shape_key((96, 96, 96), (3, 3, 3), 6, False, 1, 1)
    assert k3 == "d3 ne44x44x44 P3x3x3 ops1 c128 r1"


def test_search_space_holds_only_compiled_values():
    c64 = A.candidates(2, True)
    c128 = A.candidates(2, False)
    assert len(c64) == 2 * 2 * 3 * 2 and len(c128) == 2 * 4 * 2 - 2
    assert {c["sweep_nw"] for c in c64} == {4, 8}
    assert {c["sweep_kb"] for c in c64} == {6, 8, 10}
    assert {c["sweep_kb"] for c in c128} == {3, 4, 5, 6}
    assert {c["solve_ng"] for c in c128} == {1}
    assert [c["gemm_skinny"] for c in A.candidates(3, True)] == [1, 2]


def test_cache_round_trip(tmp_path):
    p = tmp_path / "t.json"
    assert A.load(str(p)) == {}
    e = {"d2 ne160x160 P8x8 ops1 c64 r1": {"params": {"solve_ng": 1, "sweep_rw": 2,
                                                      "sweep_kb": 10, "gemm_skinny": 0},
                                           "ms": 4.0, "default_ms": 4.1, "columns": 16}}
    A.save(e, str(p))
    assert A.load(str(p)) == e
    assert json.load(open(p))["version"] == 1


def test_committed_cache_is_valid():
    for key, e in A.load().items():
        assert set(e["params"]) == {"solve_ng", "sweep_rw", "sweep_kb", "gemm_skinny",
                                    "sweep_nw", "sweep_sched"}
        assert e["ms"] <= e["default_ms"] + 1e-9, key
        dim = int(key.split()[0][1:])
        mixed = " c64 " in key
        allowed = A.candidates(dim, mixed) + [dict(solve_ng=0, sweep_rw=0, sweep_kb=0,
                                                   gemm_skinny=0, sweep_nw=0, sweep_sched=0)]
        assert e["params"] in allowed, key
