"""Host logic of the autotuner: the coordinate search and the database."""
import json
import math

import pytest

from paper_2603_14040_amd import autotune as at


def test_search_reaches_separable_minimum():
    # cost separable in the knobs: coordinate descent must find the minimum
    best = {"a": 3, "b": (1, 0), "c": 20}
    knobs = [at.Knob("a", [1, 2, 3, 4]), at.Knob("b", [(0, 0), (0, 1), (1, 0), (1, 1)]), at.Knob("c", [10, 20, 30])]

    def cost(p):
        return (10.0 + abs(p["a"] - best["a"]) + 3 * (tuple(p["b"]) != best["b"]) + abs(p["c"] - best["c"]) / 10)

    r = at.coordinate_search(cost, knobs, {"a": 1, "b": (0, 0), "c": 10})
    assert r.params == best and r.cost == 10.0
    # every distinct parameter set measured once
    keys = [json.dumps(p, sort_keys=True) for p, _ in r.trials]
    assert len(keys) == len(set(keys))


def test_search_discards_unusable_and_keeps_start_when_nothing_gains():
    knobs = [at.Knob("x", [0, 1, 2])]
    r = at.coordinate_search(lambda p: math.inf if p["x"] == 2 else 5.0 - 0.01 * p["x"], knobs, {"x": 0},
                             rel_gain=0.02)
    assert r.params == {"x": 0}                # 0.2 % faster is below the 2 % threshold
    r = at.coordinate_search(lambda p: math.inf if p["x"] != 1 else 1.0, knobs, {"x": 0})
    assert r.params == {"x": 1} and r.cost == 1.0


def test_search_second_round_uses_interaction():
    # b only pays once a has moved: a second pass must pick it up
    knobs = [at.Knob("b", [0, 1]), at.Knob("a", [0, 1])]
    table = {(0, 0): 10.0, (0, 1): 8.0, (1, 0): 10.5, (1, 1): 5.0}
    r = at.coordinate_search(lambda p: table[(p["b"], p["a"])], knobs, {"a": 0, "b": 0}, rounds=3)
    assert r.params == {"a": 1, "b": 1}


def test_masks_and_solver_kwargs():
    assert at.plan_to_masks([(1, 0), (0, 1), (1, 1)], [0, 1, 3]) == (0b1001, 0b1010)
    p = {"L0": (0, 0), "L1": (1, 1), "nu_pre": 3, "nu_post": 2, "nu_growth": 1.5, "uzawa_steps": 1, "restart": 30,
         "coarse_level": 4}
    kw = at.solver_kwargs(p, [0, 1])
    assert kw == dict(nu_pre=3, nu_post=2, nu_growth=1.5, uzawa_steps=1, restart=30, msweep=0b10, tile_shape=0b10,
                      coarse_level=4, omega=1.0, alpha=1.0, accel="fgmres", beta=1.0, smoother=1, ras_tile=32,
                      ras_inner=4)
    kw = at.solver_kwargs(dict(p, accel="anderson", beta=0.7), [0, 1])
    assert kw["accel"] == "anderson" and kw["beta"] == 0.7
    ks = at.knobs_for([0, 1, 2], [5])
    names = [k.name for k in ks]
    assert names[:7] == ["alpha", "uzawa_steps", "nu_pre", "nu_post", "omega", "nu_growth", "krylov"]
    # accelerator and restart move together: every (accelerator, restart) pair is one candidate
    kry = list(ks[6].candidates)
    assert ("fgmres", 20) in kry and ("gcr", 8) in kry and len(kry) == 2 * len(set(r for _, r in kry))
    assert "coarse_level" in names and names[-3:] == ["L0", "L1", "L2"]
    assert {a for a, _ in at.knobs_for([0], accels=("fgmres",))[6].candidates} == {"fgmres"}
    # a joint krylov entry overrides accel and restart
    kw = at.solver_kwargs(dict(p, krylov=("gcr", 8)), [0, 1])
    assert kw["accel"] == "gcr" and kw["restart"] == 8
    # the second starting point names a joint entry
    assert at.ALT_START["krylov"] == ("gcr", 8)


def test_database_round_trip(tmp_path):
    path = tmp_path / "db.json"
    db = at.TuningDB(str(path))
    k = at.TuningDB.key(1024, 1024, 1, "AMD Instinct MI355X", "tephra 0.1.0", "grf")
    db.put(k, {"params": {"nu_pre": 2}, "ms": 12.5})
    again = at.TuningDB(str(path))
    assert again.get(k) == {"params": {"nu_pre": 2}, "ms": 12.5}
    assert again.get(k + "x") is None
    path.write_text("[1, 2]")
    with pytest.raises(ValueError):
        at.TuningDB(str(path))
