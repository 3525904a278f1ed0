"""Writes grid32_hogwild_spread.json: the final sampled objective and NP of
the oracle's layouts of the grid workload (32x32 grid, k=3, M=5, b=3, T=300,
one level, eta0 = 1/4) for seeds 0..63, in Jacobi (sync) and Gauss-Seidel
(seq) order, in R^2 and R^3.  Calls only the oracle and its evaluators.

    python tests/golden/make_grid_hogwild_spread.py
"""
import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

KW = dict(k=3, M=5, b=3, T=300, max_levels=1, eta0=0.25)
SEEDS = 64
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid32_hogwild_spread.json")


def one(task):
    from oracle import drgo, evaluate
    from paper_2008_07799_amd import gen
    dim, mode, seed = task
    g = gen.grid(32, 32)
    y, sim, _ = drgo.layout(g, seed=seed, return_all=True, dim=dim, mode=mode, **KW)
    return (evaluate.objective_eval(sim, y, M=KW["M"], b=KW["b"], gamma=0.1),
            evaluate.neighbourhood_preservation(g, y))


def main():
    tasks = [(dim, mode, seed) for dim in (2, 3) for mode in ("sync", "seq")
             for seed in range(SEEDS)]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(one, tasks)
    out = {"params": dict(KW, graph="grid 32x32", gamma_eval=0.1, M_eval=50),
           "seeds": SEEDS, "spread": {}}
    for (dim, mode, seed), (obj, npv) in zip(tasks, res):
        d = out["spread"].setdefault(str(dim), {}).setdefault(mode, {"objective": [], "np": []})
        d["objective"].append(obj)
        d["np"].append(npv)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
