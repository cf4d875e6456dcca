"""Pins of the oracle's squeeze limiter and pressure step (Sec. 3.4, 3.8, Cor. of Sec. 4).

Hand-worked cases come from tests/golden/limiter_worked.json.  Properties:
alpha in [0, 1]; the weighted element mean is conserved; a mean inside the
box puts every limited node inside the box (Corollary, existence of alpha);
alpha is the largest feasible factor (the squeeze limiter of Sec. 2.4 applied
per component and coupled by the minimum); after the pressure step the
nodal pressure is at least the floor when the mean's pressure is above it.
"""

import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 1.4


def press(w, d):
    m2 = sum(w[1 + j] ** 2 for j in range(d))
    return (GAMMA - 1) * (w[d + 1] - 0.5 * m2 / w[0])


def run_limit(sol, bmin, bmax, c=None, d=1):
    sol = np.asarray(sol, dtype=np.float64)
    n_s = sol.shape[1]
    c = np.ones(n_s) if c is None else np.asarray(c, dtype=np.float64)
    b = np.array(list(bmin) + list(bmax), dtype=np.float64)[:, None]
    lim, al, st = oracle.limit(d, GAMMA, sol, b, c, n_s)
    return lim, al[:, 0], st[0]


def test_worked_cases():
    fx = json.load(open(os.path.join(GOLDEN, "limiter_worked.json")))
    for case in fx["cases"]:
        lim, al, st = run_limit(case["solution"], case["bounds_min"], case["bounds_max"])
        assert al[0] == pytest.approx(case["alpha"], abs=1e-15), case["name"]
        if "alpha_p" in case:
            assert al[1] == pytest.approx(case["alpha_p"], abs=1e-15), case["name"]
            np.testing.assert_allclose(lim, np.array(case["limited"]), rtol=1e-14, atol=1e-15)
        else:
            ap = eval(case["alpha_p_expr"], {"__builtins__": {}})
            assert al[1] == pytest.approx(ap, rel=1e-14), case["name"]
            assert st & oracle.ST_PSTEP
            # pressure is concave along the blend, so every node ends at or above the floor
            P = [press(lim[:, j], 1) for j in range(lim.shape[1])]
            assert min(P) >= 1e-12 - 1e-15


def _random_element(rng, d, n_s):
    rho = rng.uniform(0.5, 2.0, n_s)
    U = rng.uniform(-1, 1, (d, n_s))
    p = rng.uniform(0.3, 3.0, n_s)
    w = np.vstack([rho, rho * U, p / (GAMMA - 1) + 0.5 * rho * (U ** 2).sum(0)])
    return w


@pytest.mark.parametrize("d", [1, 2])
def test_limiter_properties(d):
    rng = np.random.default_rng(3 + d)
    n_s = 9
    nv = d + 2
    for trial in range(200):
        w = _random_element(rng, d, n_s)
        c = rng.uniform(0.2, 1.0, n_s)
        mean = (w * c).sum(1) / c.sum()
        span = w.max(1) - w.min(1)
        # bounds around the mean, sometimes tighter than the nodal range
        f_lo = rng.uniform(0.0, 1.2, nv)
        f_hi = rng.uniform(0.0, 1.2, nv)
        bmin = mean - f_lo * (mean - w.min(1)) - 1e-3 * span * (trial % 3 == 0)
        bmax = mean + f_hi * (w.max(1) - mean)
        lim, al, st = run_limit(w, bmin, bmax, c, d)
        a = al[0]
        assert 0.0 <= a <= 1.0
        # conservation of the weighted element mean
        lmean = (lim * c).sum(1) / c.sum()
        np.testing.assert_allclose(lmean, mean, rtol=1e-13, atol=1e-13 * np.abs(w).max())
        if st & oracle.ST_PSTEP:
            continue
        # feasibility: every limited node inside the box (Corollary of Sec. 4)
        tol = 1e-12 * (np.abs(w).max(1) + 1)
        assert np.all(lim.min(1) >= bmin - tol) and np.all(lim.max(1) <= bmax + tol)
        # maximality: a slightly larger factor breaks some bound, unless alpha = 1
        if a < 1.0:
            a2 = a * (1 + 1e-6) + 1e-9
            trial_w = mean[:, None] + a2 * (w - mean[:, None])
            viol = (trial_w.min(1) < bmin - tol) | (trial_w.max(1) > bmax + tol)
            assert viol.any()
        else:
            np.testing.assert_allclose(lim, w, rtol=1e-14, atol=1e-14 * np.abs(w).max())


def test_each_component_is_the_scalar_squeeze_limiter():
    """With one component binding, alpha equals the Sec. 2.4 scalar factor of
    that component and the other components only follow."""
    sol = [[1.0, 2.0, 4.0, 1.0], [0.1, 0.2, -0.1, -0.2], [5.0, 6.0, 7.0, 6.0]]
    c = [1.0, 2.0, 1.0, 2.0]
    w = np.array(sol)
    cc = np.array(c)
    mean = (w * cc).sum(1) / cc.sum()
    bmin = [1.2, -1.0, 0.0]
    bmax = [3.0, 1.0, 100.0]
    lim, al, st = run_limit(sol, bmin, bmax, c)
    # density: max node 4 vs bound 3, min node 1 vs bound 1.2
    expect = min(1.0, abs((3.0 - mean[0]) / (4.0 - mean[0])), abs((1.2 - mean[0]) / (1.0 - mean[0])))
    assert al[0] == pytest.approx(expect, rel=1e-15)
    assert lim[0].max() == pytest.approx(3.0, rel=1e-14) or lim[0].min() == pytest.approx(1.2, rel=1e-14)


def test_epsilon_rule_flattens_element():
    sol = [[1.0, 1.0, 1.0], [0.1, 0.3, 0.2], [3.0, 3.5, 2.5]]
    lim, al, st = run_limit(sol, [0.5, -1.0, 0.0], [2.0, 1.0, 10.0])
    assert al[0] == 0.0 and (st & oracle.ST_EPS_RULE)
    w = np.array(sol)
    np.testing.assert_allclose(lim, np.repeat(w.mean(1, keepdims=True), 3, 1), rtol=1e-15)


@pytest.mark.parametrize("d", [1, 2])
def test_pressure_step_restores_floor(d):
    rng = np.random.default_rng(21 + d)
    n_s = 6
    for trial in range(200):
        w = _random_element(rng, d, n_s)
        c = rng.uniform(0.2, 1.0, n_s)
        # push energy down at one node so that its pressure goes negative
        j = trial % n_s
        w[d + 1, j] -= rng.uniform(0.5, 3.0) * w[d + 1, j]
        big = 1e6
        lim, al, st = run_limit(w, [-big] * (d + 2), [big] * (d + 2), c, d)
        mean = (w * c).sum(1) / c.sum()
        Pbar = press(mean, d)
        P = np.array([press(lim[:, i], d) for i in range(n_s)])
        if Pbar > 1e-12:
            assert P.min() >= 1e-12 - 1e-13 * abs(w[d + 1]).max()
        if st & oracle.ST_PSTEP:
            assert 0 <= al[1] < 1


def test_mean_below_pressure_floor_flattens():
    # mean with zero pressure: alpha_P = 0 and the flag is raised
    sol = [[1.0, 1.2], [1.0, -1.0], [0.5, -0.5]]
    lim, al, st = run_limit(sol, [-10, -10, -10], [10, 10, 10])
    assert al[0] == 1.0
    assert al[1] == 0.0 and (st & oracle.ST_PMEAN_FLOOR) and (st & oracle.ST_PSTEP)
    np.testing.assert_allclose(lim, [[1.1, 1.1], [0.0, 0.0], [0.0, 0.0]], atol=1e-15)


def test_nonfinite_bounds_pass_through():
    sol = [[1.0, 2.0], [0.1, 0.2], [3.0, 4.0]]
    lim, al, st = run_limit(sol, [np.nan] * 3, [np.nan] * 3)
    assert st & oracle.ST_BAD_BOUNDS
    np.testing.assert_array_equal(lim, np.array(sol))
