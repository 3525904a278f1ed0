"""Shared helpers of the GPU tests: a context on cuda:0 and comparisons."""
import json
import os
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise_rel(y, ref) -> float:
    """max_i ||y_i - ref_i||_inf / max_i ||ref_i||_inf."""
    y = np.asarray(y, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(y - ref).max() / max(np.abs(ref).max(), 1e-30))


_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        import torch
        from paper_2008_07799_amd import drgraph
        assert torch.cuda.is_available(), "GPU tests need a GPU"
        torch.cuda.set_device(0)
        _ctx = drgraph.Context(0)
    return _ctx


def dev_graph(csr):
    from paper_2008_07799_amd import drgraph
    return drgraph.to_device(csr)


def zeros_y(n, dtype=None):
    import torch
    return torch.zeros((n, 2), dtype=dtype or torch.float32, device="cuda")


def to_y(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()



def layout_stats(g, kw, sim, y):
    """Final sampled objective and NP of layout y (the tests' evaluation)."""
    from oracle import evaluate
    y = np.asarray(y, np.float64)
    return (evaluate.objective_eval(sim, y, M=kw["M"], b=kw["b"], gamma=0.1),
            evaluate.neighbourhood_preservation(g, y))



GRID_SPREAD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "grid32_hogwild_spread.json")


def oracle_spread(kw, dim=2):
    """Objective and NP of the oracle's layouts of the grid workload over
    seeds 0..63, in Jacobi (sync) and in Gauss-Seidel order, as rows of an
    array; stored by tests/golden/make_grid_hogwild_spread.py (which calls
    only the oracle) for the parameters kw must repeat."""
    with open(GRID_SPREAD) as f:
        d = json.load(f)
    for key in ("k", "M", "b", "T", "max_levels", "eta0"):
        assert kw[key] == d["params"][key], (key, kw[key], d["params"][key])
    ref = [(o, p) for m in ("sync", "seq")
           for o, p in zip(d["spread"][str(dim)][m]["objective"], d["spread"][str(dim)][m]["np"])]
    return np.array(ref)

def check_spread(ref, got, width=4.0):
    """Every row of got (objective, NP) within the mean of ref +- width
    standard deviations, and the mean of got within width two-sample
    standard errors of the mean of ref."""
    got = np.asarray(got, np.float64)
    for q, name in ((0, "objective"), (1, "NP")):
        mo, so = ref[:, q].mean(), ref[:, q].std(ddof=1)
        mg, sg = got[:, q].mean(), got[:, q].std(ddof=1)
        se = np.sqrt(so * so / len(ref) + sg * sg / len(got))
        say(f"  {name}: oracle mean {mo:.4f} sd {so:.4f}; hogwild mean {mg:.4f} sd {sg:.4f} "
            f"min {got[:, q].min():.4f} max {got[:, q].max():.4f}")
        assert np.all(np.abs(got[:, q] - mo) <= width * so), (name, got[:, q], mo, so)
        assert abs(mg - mo) <= width * se, (name, mg, mo, se)


def hogwild_vs_oracle_spread(oracle_lib, g, kw, gpu_layout, dim=2, runs=8, width=4.0):
    """Holds Hogwild layouts of the grid workload to the distribution of the
    oracle's layouts.

    A Hogwild run (Sec. 3.2.2's updates applied in place while other nodes
    read them) follows an update order the hardware picks, so its result is
    one draw of a random process and no single oracle run is its reference.
    On the grid workload (32x32, k=3, b=3) the final objective varies by
    about 8% (one standard deviation) from seed to seed, in 2-D and 3-D, NP
    by about 0.03, and the range of a few runs misses a fresh draw often.
    The reference is the oracle's 64 seeds in Jacobi and 64 in Gauss-Seidel
    order (oracle_spread), the two ends between which Hogwild updates fall;
    gpu_layout(seed) returns the GPU layout of the same parameters, for
    seeds 0..runs-1, evaluated on the oracle's similarity.  Checked by
    check_spread for the sampled objective and NP."""
    ref = oracle_spread(kw, dim)
    sim = oracle_lib.similarity(g, kw["k"])
    got = [layout_stats(g, kw, sim, gpu_layout(seed)) for seed in range(runs)]
    check_spread(ref, got, width)
