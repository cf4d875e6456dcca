"""Pins of the oracle in three dimensions (d = 3): the 3D velocity grids the
paper's conclusion names as the costly extension.  Single-state moments,
axis-permutation symmetry, ordering/positivity (Thm. 4.5), the limiter's
properties and the Riemann-averaged states in 3D."""

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import GRID_STENCIL

GAMMA = 1.4


def prim_to_cons(rho, U, p, gamma=GAMMA):
    U = np.asarray(U, dtype=np.float64)
    return np.concatenate([[rho], rho * U, [p / (gamma - 1) + 0.5 * rho * (U ** 2).sum()]])


def bounds_of(states, n=(40, 40, 40), k=8.0, r=0.0, n_s=None, rowptr=None, cols=None):
    n_s = states.shape[1] if n_s is None else n_s
    rp = np.array([0, 1], dtype=np.int32) if rowptr is None else rowptr
    cl = np.array([0], dtype=np.int32) if cols is None else cols
    return oracle.bounds(3, GAMMA, states, rp, cl, n_s, GRID_STENCIL, n, k=k, r_fac=r)


@pytest.mark.parametrize("U,rho,p", [((0.3, -1.2, 0.7), 1.3, 0.9), ((2.0, 0.0, -0.5), 0.2, 4.0)])
def test_single_state_reproduces_its_moments(U, rho, p):
    w = prim_to_cons(rho, U, p)[:, None]
    b, st = bounds_of(w)
    assert st[0] == 0
    np.testing.assert_allclose(b[:5, 0], w[:, 0], rtol=1e-12, atol=1e-12 * abs(w).max())
    np.testing.assert_allclose(b[5:, 0], w[:, 0], rtol=1e-12, atol=1e-12 * abs(w).max())


def test_single_state_relaxed_closed_form():
    w = prim_to_cons(0.7, (0.5, 1.0, -0.25), 1.1)[:, None]
    r = 1e-3
    b, _ = bounds_of(w, r=r)
    np.testing.assert_allclose(b[0, 0], (1 - r) * w[0, 0], rtol=1e-12)
    np.testing.assert_allclose(b[5, 0], (1 + r) * w[0, 0], rtol=1e-12)
    np.testing.assert_allclose(b[4, 0], (1 - r) * w[4, 0], rtol=1e-12)
    np.testing.assert_allclose(b[9, 0], (1 + r) * w[4, 0], rtol=1e-12)


def test_axis_permutation_permutes_momentum_bounds():
    rng = np.random.default_rng(3)
    S = 6
    W = np.stack([prim_to_cons(np.exp(rng.uniform(-1, 1)), rng.uniform(-2, 2, 3),
                               np.exp(rng.uniform(-1, 1))) for _ in range(S)], 1)
    b, _ = bounds_of(W, n=(20, 24, 28), k=4.0, r=1e-3)
    P = W[[0, 2, 3, 1, 4]]                                  # (u, v, w) -> (v, w, u)
    bp, _ = bounds_of(P, n=(24, 28, 20), k=4.0, r=1e-3)
    for off in (0, 5):
        np.testing.assert_allclose(bp[off + 0], b[off + 0], rtol=1e-12)
        np.testing.assert_allclose(bp[off + 4], b[off + 4], rtol=1e-12)
        np.testing.assert_allclose(bp[off + 1], b[off + 2], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(bp[off + 2], b[off + 3], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(bp[off + 3], b[off + 1], rtol=1e-12, atol=1e-13)


def test_hex_stencil_ordering_and_positivity():
    wl = synth.make_hex_workload(N=2, seed=4, grid_nodes=20)
    b, st = oracle.workload_bounds(wl)
    assert not st.any() or not (st & (oracle.ST_INADMISSIBLE | oracle.ST_BAD_STENCIL)).any()
    S = wl.states.reshape(5, wl.n_elem, wl.n_s)
    for e in range(wl.n_elem):
        sten = wl.cols[wl.rowptr[e]:wl.rowptr[e + 1]]
        rho = S[0, sten].ravel()
        E = S[4, sten].ravel()
        # k = 4 truncation (~6e-5 per dimension) and relaxation r = 1e-3
        assert b[0, e] <= rho.min() * (1 + 1e-3) and b[5, e] >= rho.max() * (1 - 1e-3)
        assert b[4, e] <= E.min() * (1 + 1e-3) and b[9, e] >= E.max() * (1 - 1e-3)
        assert b[0, e] > 0 and b[4, e] > 0
        for j in range(3):
            m = S[1 + j, sten].ravel()
            scale = np.abs(S[1:4, sten]).max() + np.sqrt(rho.max() * E.max())
            assert b[1 + j, e] <= m.min() + 1e-3 * scale and b[6 + j, e] >= m.max() - 1e-3 * scale


def test_limiter_3d_properties():
    wl = synth.make_hex_workload(N=2, seed=5, grid_nodes=16)
    wl.target = wl.states + 4.0 * (wl.target - wl.states)
    b, _ = oracle.workload_bounds(wl)
    lim, al, st = oracle.workload_limit(wl, b)
    c = wl.node_weights / wl.node_weights.sum()
    L = lim.reshape(5, wl.n_elem, wl.n_s)
    T = wl.target.reshape(5, wl.n_elem, wl.n_s)
    np.testing.assert_allclose((L * c).sum(2), (T * c).sum(2), rtol=1e-13, atol=1e-13)
    assert np.all((al[0] >= 0) & (al[0] <= 1))
    ok = (st & (oracle.ST_MEAN_OUTSIDE | oracle.ST_EPS_RULE)) == 0
    tol = 1e-12 * np.abs(b).max(0)
    assert np.all(L.min(2)[:, ok] >= b[:5, ok] - tol[ok])
    assert np.all(L.max(2)[:, ok] <= b[5:, ok] + tol[ok])


def test_riemann_3d_fixed_point_and_symmetry():
    rng = np.random.default_rng(6)
    W = np.stack([prim_to_cons(np.exp(rng.uniform(-1, 1)), rng.uniform(-2, 2, 3),
                               np.exp(rng.uniform(-1, 1))) for _ in range(20)], 1)
    n = rng.standard_normal((3, 10))
    n /= np.linalg.norm(n, axis=0)
    a, _ = oracle.riemann(3, GAMMA, W, np.arange(10), np.arange(10, 20), n)
    b, _ = oracle.riemann(3, GAMMA, W, np.arange(10, 20), np.arange(10), -n)
    np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-14)
    f, _ = oracle.riemann(3, GAMMA, np.hstack([W, W]), np.arange(20), np.arange(20, 40),
                          np.tile(n, 2))
    np.testing.assert_allclose(f, W, rtol=1e-14, atol=1e-14)
