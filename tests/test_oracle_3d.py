"""Pins of the oracle's three-dimensional layouts (Sec. 3.1: positions in
R^2 or R^3; the forces of Eq. gradient act along the offset in any
dimension).  Marked "not gpu"."""
import math

import numpy as np
import pytest

from paper_2008_07799_amd import gen


def _setup(oracle_lib, n=30, p=0.15, k=2, sub=0, scale=1.5):
    g = gen.random_graph(n, p, seed=31, sub=sub)
    sim = oracle_lib.similarity(g, k)
    y = np.random.default_rng(100 + sub).uniform(-scale, scale, size=(n, 3))
    return g, sim, y


def _rotation(seed):
    """A random proper rotation of R^3 (QR of a Gaussian matrix)."""
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_init_3d_extends_the_2d_layout(oracle_lib):
    """Coordinate c of node v is word c of its Philox block: the first two
    columns are the 2-D layout, the third lies on the same 2^-23 grid."""
    y3 = oracle_lib.init(5000, 7, 2, dim=3)
    y2 = oracle_lib.init(5000, 7, 2)
    assert np.array_equal(y3[:, :2], y2)
    z = y3[:, 2]
    assert z.min() >= -1.0 and z.max() < 1.0
    assert np.array_equal(np.round((z + 1.0) * 2 ** 23), (z + 1.0) * 2 ** 23)
    assert abs(z.mean()) < 0.05 and not np.array_equal(z, y3[:, 0])


@pytest.mark.parametrize("b", [1, 1.5, 2, 2.5, 3])
def test_sampled_gradient_3d_matches_central_differences(oracle_lib, b):
    g, sim, y = _setup(oracle_lib, sub=int(2 * b))
    grad = oracle_lib.objective_grad(sim, y, M=5, b=b, gamma=0.1, seed=3, it=7)
    assert grad.shape == (g.n, 3)
    h = 1e-6
    rng = np.random.default_rng(int(2 * b))
    for i in rng.choice(g.n, 10, replace=False):
        for c in (0, 1, 2):
            yp, ym = y.copy(), y.copy()
            yp[i, c] += h
            ym[i, c] -= h
            fd = (oracle_lib.objective(sim, yp, 5, b, 0.1, 3, 7)
                  - oracle_lib.objective(sim, ym, 5, b, 0.1, 3, 7)) / (2 * h)
            assert fd == pytest.approx(grad[i, c], rel=1e-5, abs=1e-7)


def test_exact_gradient_3d_matches_central_differences(oracle_lib):
    g, sim, y = _setup(oracle_lib, n=20, sub=11)
    grad = oracle_lib.objective_exact_grad(sim, y, M=5, b=2, gamma=0.1)
    h = 1e-6
    for i in range(0, g.n, 3):
        for c in (0, 1, 2):
            yp, ym = y.copy(), y.copy()
            yp[i, c] += h
            ym[i, c] -= h
            fd = (oracle_lib.objective_exact(sim, yp, 5, 2, 0.1)
                  - oracle_lib.objective_exact(sim, ym, 5, 2, 0.1)) / (2 * h)
            assert fd == pytest.approx(grad[i, c], rel=1e-5, abs=1e-7)


def test_planar_3d_layout_reduces_to_2d(oracle_lib):
    """With every z = 0 the 3-D step, iteration, objective and gradient are
    the 2-D ones with a zero third component (bit for bit: the same
    operations, and z adds exact zeros)."""
    g, sim, y3 = _setup(oracle_lib, n=60, p=0.08, sub=4)
    y3[:, 2] = 0.0
    y2 = y3[:, :2].copy()
    for clip in (math.inf, 0.3):
        s3 = oracle_lib.step_direction(sim, y3, None, 5, 2, 0.1, clip, 1, 2)
        s2 = oracle_lib.step_direction(sim, y2, None, 5, 2, 0.1, clip, 1, 2)
        assert np.array_equal(s3[:, :2], s2) and not s3[:, 2].any()
    assert oracle_lib.objective(sim, y3, 5, 3, 0.1, 4, 1) == oracle_lib.objective(sim, y2, 5, 3,
                                                                                 0.1, 4, 1)
    g3 = oracle_lib.objective_grad(sim, y3, 5, 3, 0.1, 4, 1)
    g2 = oracle_lib.objective_grad(sim, y2, 5, 3, 0.1, 4, 1)
    assert np.array_equal(g3[:, :2], g2) and not g3[:, 2].any()
    h = oracle_lib.hierarchy(g, seed=1, rho=0.9, min_nodes=5, max_levels=2)
    cm = h.cmaps[-1]
    a3 = np.zeros((h.sizes[-1], 3))
    a3[:, :2] = np.random.default_rng(5).uniform(-2, 2, size=(h.sizes[-1], 2))
    a2 = a3[:, :2].copy()
    for seq in (False, True):
        b3, b2 = a3.copy(), a2.copy()
        oracle_lib.iter_sync(sim, b3, cm, 5, 1, 0.1, 0.6, 4.0, 2, 3, seq=seq)
        oracle_lib.iter_sync(sim, b2, cm, 5, 1, 0.1, 0.6, 4.0, 2, 3, seq=seq)
        assert np.array_equal(b3[:, :2], b2) and not b3[:, 2].any()


def test_3d_rotation_and_translation_invariance(oracle_lib):
    """L^ depends on distances only: rotating the layout leaves it and
    rotates the gradient; the total force and the total torque (a 3-vector)
    vanish; a shift changes nothing."""
    g, sim, y = _setup(oracle_lib, n=120, p=0.04, sub=6)
    Rm = _rotation(3)
    L0 = oracle_lib.objective(sim, y, 5, 2, 0.1, 9, 1)
    L1 = oracle_lib.objective(sim, y @ Rm.T, 5, 2, 0.1, 9, 1)
    assert L1 == pytest.approx(L0, rel=1e-12)
    G0 = oracle_lib.objective_grad(sim, y, 5, 2, 0.1, 9, 1)
    G1 = oracle_lib.objective_grad(sim, y @ Rm.T, 5, 2, 0.1, 9, 1)
    scale = np.abs(G0).sum()
    assert np.abs(G1 - G0 @ Rm.T).max() < 1e-10 * scale
    assert np.abs(G0.sum(axis=0)).max() < 1e-12 * scale
    torque = np.cross(y, G0).sum(axis=0)
    assert np.abs(torque).max() < 1e-11 * scale * np.abs(y).max()
    G2 = oracle_lib.objective_grad(sim, y + np.array([0.5, -2.0, 3.0]), 5, 2, 0.1, 9, 1)
    assert np.abs(G2 - G0).max() < 1e-10 * scale


def test_3d_monte_carlo_step_and_exact_gradient(oracle_lib):
    """As in 2-D: the mean of the one-sided step over negative draws is its
    exact expectation, which is half the gradient of the expected objective."""
    g, sim, y = _setup(oracle_lib, n=25, p=0.2, k=1, sub=8)
    S = 2000
    acc = np.zeros_like(y)
    acc2 = np.zeros_like(y)
    for s in range(S):
        gd = oracle_lib.step_direction(sim, y, None, 5, 2, 0.1, math.inf, s, 0)
        acc += gd
        acc2 += gd * gd
    mean = acc / S
    se = np.sqrt(np.maximum(acc2 / S - mean ** 2, 0) / S)
    expd = oracle_lib.step_expected(sim, y, 5, 2, 0.1)
    assert (np.abs(mean - expd) / np.maximum(se, 1e-15)).max() < 5.0
    assert np.allclose(oracle_lib.objective_exact_grad(sim, y, 5, 2, 0.1), 2 * expd,
                       rtol=1e-6, atol=1e-9)


def test_3d_layout_runs_and_spreads(oracle_lib):
    """A whole 3-D multilevel layout stays finite and uses the third axis."""
    g = gen.grid(12, 12)
    y = oracle_lib.layout(g, k=2, M=5, b=2, T=60, min_nodes=20, seed=1, dim=3, eta0=0.5)
    assert y.shape == (144, 3) and np.isfinite(y).all()
    assert y[:, 2].std() > 0.1 * y[:, :2].std()
