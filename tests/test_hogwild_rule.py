"""The rule that holds a Hogwild layout (one draw of a random process) to the
distribution of the oracle's layouts over seeds, and its stored reference.

The reference (tests/golden/grid32_hogwild_spread.json) must be what the
oracle computes; the rule must accept layouts of the same process and
reject ones from a changed method.  Both sides here are oracle runs on the
CPU: fresh seeds (in both update orders) stand for the Hogwild runs, and
the planted mistakes (a tenth of the iterations; a four times larger step)
are planted in the oracle's parameters.  Grid workload: 32x32, k=3, M=5,
b=3, T=300, one level, eta0 = 1/4 (Sec. 4.2's b for lattices), in R^2 and
R^3."""
import json

import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import GRID_SPREAD, check_spread, layout_stats, oracle_spread

KW = dict(k=3, M=5, b=3, T=300, max_levels=1, eta0=0.25)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", ["sync", "seq"])
def test_stored_spread_is_the_oracles(oracle_lib, dim, mode):
    with open(GRID_SPREAD) as f:
        d = json.load(f)
    assert d["seeds"] == 64
    g = gen.grid(32, 32)
    for seed in (0, 37, 63):
        y, sim, _ = oracle_lib.layout(g, seed=seed, return_all=True, dim=dim, mode=mode, **KW)
        obj, npv = layout_stats(g, KW, sim, y)
        assert np.isclose(obj, d["spread"][str(dim)][mode]["objective"][seed], rtol=1e-12, atol=0)
        assert np.isclose(npv, d["spread"][str(dim)][mode]["np"][seed], rtol=1e-12, atol=0)


def _draws(oracle_lib, dim, runs=8, **change):
    g = gen.grid(32, 32)
    sim = oracle_lib.similarity(g, KW["k"])
    run = dict(KW, **change)
    return [layout_stats(g, KW, sim, oracle_lib.layout(g, seed=100 + s, dim=dim,
                                                       mode=("sync", "seq")[s % 2], **run))
            for s in range(runs)]


@pytest.mark.parametrize("dim", [2, 3])
def test_rule_accepts_fresh_draws_of_the_same_process(oracle_lib, dim):
    check_spread(oracle_spread(KW, dim), _draws(oracle_lib, dim))


@pytest.mark.parametrize("change", [dict(T=30), dict(eta0=1.0)])
def test_rule_rejects_a_changed_method(oracle_lib, change):
    with pytest.raises(AssertionError):
        check_spread(oracle_spread(KW, 2), _draws(oracle_lib, 2, **change))
