"""The input recipes (no GPU): sector splits of the configs as their
docstrings and the design's readings state them, seeded draws reproducible
and independent per tensor, batched draws within their ranges."""
import numpy as np

from synth import (CONFIGS, batched_draws, binomial_sectors, config, draw, virtual_sectors_for_D,
                   TENSOR_INDEX)


def test_binomial_sectors_examples():
    assert binomial_sectors(64, 5) == {-4: 4, -2: 16, 0: 24, 2: 16, 4: 4}
    assert binomial_sectors(200, 7) == {-6: 3, -4: 19, -2: 47, 0: 62, 2: 47, 4: 19, 6: 3}
    assert binomial_sectors(40, 5) == {-4: 3, -2: 10, 0: 15, 2: 10, 4: 2}
    for total in (16, 33, 64, 99, 100, 160, 200):
        for n in (3, 5, 7):
            s = binomial_sectors(total, n)
            assert sum(s.values()) == total
            assert all(q % 2 == 0 for q in s)


def test_virtual_sectors_for_D():
    for D in range(4, 9):
        s = virtual_sectors_for_D(D)
        assert sum(s.values()) == D and set(s) == {-2, 0, 2} and s[-2] == s[2]


def test_config_legs():
    assert config(2)["chi"] == binomial_sectors(64, 5) and config(2)["virt"] == {-2: 1, 0: 4, 2: 1}
    assert sum(config(4)["chi"].values()) == 200 and sum(config(4)["virt"].values()) == 8
    assert config(1)["seed"] == 1809 and config(2)["seed"] == 1810
    assert config(6)["group"] == "Z2" and config(6)["chi"] == {0: 32, 1: 32}
    c = config(2)
    c["chi"] = {}
    assert config(2)["chi"] == binomial_sectors(64, 5)    # config() hands out copies
    assert set(CONFIGS) == {1, 2, 3, 4, 5, 6}


def test_draws_are_seeded_and_independent():
    a = draw((1810, TENSOR_INDEX["C1"]), 1000)
    assert np.array_equal(a, draw((1810, TENSOR_INDEX["C1"]), 1000))
    b = draw((1810, TENSOR_INDEX["C2"]), 1000)
    c = draw((1811, TENSOR_INDEX["C1"]), 1000)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.1 and abs(np.corrcoef(a, c)[0, 1]) < 0.1
    assert abs(a.mean()) < 0.15 and abs(a.std() - 1.0) < 0.1
    # a longer draw extends a shorter one (block layouts of different sizes share a prefix)
    assert np.array_equal(draw((7, 1), 10), draw((7, 1), 20)[:10])


def test_batched_draws_ranges():
    d = batched_draws(seed=1813, batch=64)
    assert len(d) == 64 and d == batched_draws(seed=1813, batch=64)
    for x in d:
        assert 4 <= x["D"] <= 8 and 32 <= x["chi_total"] <= 160
        assert sum(x["chi"].values()) == x["chi_total"]
        assert len(x["chi"]) <= (5 if x["chi_total"] < 100 else 7)
