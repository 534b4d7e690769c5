"""Host logic of the autotuner: table format, warm start and the greedy
search, driven by a synthetic cost instead of GPU timings."""
import os

import pytest

import paper_2506_12718_amd as pafc
from paper_2506_12718_amd import tune


class FakeLib:
    """set_tuning records the active line; describe is the real (host-only)
    planner with its defaults."""

    def __init__(self):
        self.active = None

    def set_tuning(self, text):
        self.active = text

    def describe(self, dims, dt):
        pafc.set_tuning(None)
        return pafc.describe(dims, dt)

    def cfg(self):
        if not self.active:
            return {"split": 0, "W": 0, "Wo": 0, "g3": 0, "g5": 0}
        f = self.active.split()
        return dict(zip(("split", "W", "Wo", "g3", "g5"), map(int, f[2:])))


def test_line_and_table_roundtrip(tmp_path):
    cfg = {"split": 625, "W": 4, "Wo": 16, "g3": 0, "g5": 1}
    text = tune.line("c128", 78125, cfg)
    assert text == "c128 78125 625 4 16 0 1"
    p = tmp_path / "t.txt"
    p.write_text("# header\n" + text + "   # comment\nc64 729 0 0 0 2 0\n")
    t = tune.read_table(str(p))
    assert t[("c128", 78125)] == dict(cfg, g3i=0)
    assert t[("c64", 729)]["g3"] == 2
    # the inner pieces' radix-3 grouping is an optional eighth field
    cfg3 = {"split": 0, "W": 0, "Wo": 0, "g3": 2, "g5": 0, "g3i": 1}
    assert tune.line("c128", 2187, cfg3) == "c128 2187 0 0 0 2 0 1"
    p.write_text(tune.line("c128", 2187, cfg3) + "\n")
    assert tune.read_table(str(p))[("c128", 2187)] == cfg3
    pafc.set_tuning(tune.line("c128", 2187, cfg3))
    pafc.set_tuning(None)
    assert tune.read_table(str(tmp_path / "missing.txt")) == {}
    # the planner accepts every line the tuner writes
    pafc.set_tuning(text)
    pafc.set_tuning(None)


def test_candidates_follow_the_factorisation():
    lib = FakeLib()
    base = {"split": 0, "W": 0, "Wo": 0, "g3": 0, "g5": 0}
    assert tune.candidates(lib, "c128", 2187, "g3", base) == [1, 2, 3]
    assert tune.candidates(lib, "c128", 2187, "g3i", base) == [1, 2, 3]
    assert tune.candidates(lib, "c128", 3125, "g3i", base) == []
    assert tune.candidates(lib, "c128", 2187, "g5", base) == []
    assert tune.candidates(lib, "c128", 3125, "g5", base) == [1, 2]
    splits = tune.candidates(lib, "c128", 78125, "split", base)
    assert 0 in splits and all(s == 0 or 78125 % s == 0 for s in splits)


def _cost(cfg):
    # optimum: g5 = 1, split = 625, W = 4; everything else neutral
    c = 1.0
    c -= 0.3 if cfg["g5"] == 1 else 0.0
    c -= 0.2 if cfg["split"] == 625 else 0.0
    c -= 0.1 if cfg["split"] == 625 and cfg["W"] == 4 else 0.0
    return c


def test_greedy_search_reaches_the_optimum():
    lib = FakeLib()
    cfg, best, log = tune.tune_one(lib, None, "c128", 78125, lambda: _cost(lib.cfg()))
    assert cfg["g5"] == 1 and cfg["split"] == 625 and cfg["W"] == 4
    assert best == pytest.approx(0.4)
    assert log[0][0] == "default" and log[0][1] == pytest.approx(1.0)
    assert lib.active is None  # the tuner leaves no override behind


def test_warm_start_keeps_a_better_previous_entry():
    lib = FakeLib()
    # a cost the greedy order cannot find from the defaults: Wo = 8 only
    # pays together with g5 = 0, and g5 = 1 alone looks better first
    def cost():
        c = lib.cfg()
        if c["Wo"] == 8 and c["g5"] in (0, 2):
            return 0.5
        return 0.9 if c["g5"] == 1 else 1.0
    prev = {"split": 0, "W": 0, "Wo": 8, "g3": 0, "g5": 0}
    cold, t_cold, _ = tune.tune_one(lib, None, "c64", 1953125, cost)
    warm, t_warm, _ = tune.tune_one(lib, None, "c64", 1953125, cost, prev)
    assert t_warm == pytest.approx(0.5) and warm["Wo"] == 8
    assert t_warm <= t_cold
