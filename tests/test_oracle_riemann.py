"""Pins of the oracle's Riemann-averaged states (Thm. 4.3 of Sec. 4) and, through
them, of its bounds: the discrete Riemann-averaged distribution of two stencil
states is a convex combination of their Maxwellians at every velocity node
when lambda >= max |u.n| over the grid, so its quadrature moments must lie
inside the element's strict (r = 0) bounds."""

import numpy as np
import pytest

import oracle
import synth


def rand_states(rng, n, d=2, gamma=1.4):
    rho = np.exp(rng.uniform(-2, 2, n))
    p = np.exp(rng.uniform(-2, 3, n))
    U = rng.uniform(-3, 3, (d, n))
    E = p / (gamma - 1) + 0.5 * rho * (U ** 2).sum(0)
    return np.vstack([rho, rho * U, E])


def test_identical_states_are_fixed_points():
    rng = np.random.default_rng(1)
    w = rand_states(rng, 20)
    st = np.hstack([w, w])
    ni, nj = np.arange(20), np.arange(20) + 20
    n = rng.standard_normal((2, 20))
    n /= np.linalg.norm(n, axis=0)
    for lam in (None, np.full(20, 7.0)):
        bar, s = oracle.riemann(2, 1.4, st, ni, nj, n, lam)
        np.testing.assert_allclose(bar, w, rtol=1e-14, atol=1e-14)
        assert not s.any()


def test_swap_and_flip_normal_is_symmetric():
    rng = np.random.default_rng(2)
    st = rand_states(rng, 40)
    ni, nj = np.arange(20), np.arange(20, 40)
    n = rng.standard_normal((2, 20))
    n /= np.linalg.norm(n, axis=0)
    a, _ = oracle.riemann(2, 1.4, st, ni, nj, n)
    b, _ = oracle.riemann(2, 1.4, st, nj, ni, -n)
    np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-14)


def test_one_dimensional_density_by_hand():
    # rho_bar = (rho_i + rho_j)/2 - (rho_j u_j - rho_i u_i)/(2 lambda); lambda from
    # |u| + sqrt(gamma p / rho) of each state
    st = np.array([[1.0, 0.125], [0.3, -0.05], [2.5 + 0.5 * 0.09, 0.25 + 0.5 * 0.02]])
    gamma = 1.4
    u = st[1] / st[0]
    p = (gamma - 1) * (st[2] - 0.5 * st[1] * u)
    lam = max(abs(u) + np.sqrt(gamma * p / st[0]))
    bar, _ = oracle.riemann(1, gamma, st, [0], [1], np.array([[1.0]]))
    assert bar[0, 0] == pytest.approx(0.5 * (1.0 + 0.125) - (st[1, 1] - st[1, 0]) / (2 * lam),
                                      rel=1e-15)


def maxwellians(states, gamma, d, ux, uy):
    rho = states[0]
    U = states[1:3] / rho
    th = (gamma - 1) * (states[3] - 0.5 * rho * (U ** 2).sum(0)) / rho
    c2 = (ux[None, :, None] - U[0][:, None, None]) ** 2 + (uy[None, None, :] - U[1][:, None, None]) ** 2
    g = rho[:, None, None] / (2 * np.pi * th[:, None, None]) * np.exp(-c2 / (2 * th[:, None, None]))
    return g, th


def test_discrete_riemann_averaged_moments_lie_in_the_bounds():
    """Thm. 4.3 on the discrete grid, for every face pair of a small FR mesh."""
    wl = synth.make_quad_fr_workload(N=4, seed=9, grid_nodes=24)
    g = wl.grid
    gamma, d = wl.gamma, 2
    delta = oracle.delta(2, gamma)
    b, _ = oracle.bounds(2, gamma, wl.states, wl.rowptr, wl.cols, 1, g.mode, g.n[:2], g.lo, g.hi,
                         g.k, 0.0, n_src=wl.n_state_nodes)
    P = wl.meta["face_pairs"]
    checked = 0
    for q in range(0, P["ni"].size, 3):
        e = P["elem"][q]
        sten = wl.cols[wl.rowptr[e]:wl.rowptr[e + 1]]
        S = wl.states[:, sten]
        rho = S[0]
        U = S[1:3] / rho
        th = (gamma - 1) * (S[3] - 0.5 * rho * (U ** 2).sum(0)) / rho
        lo = (U - g.k * np.sqrt(th)).min(1)
        hi = (U + g.k * np.sqrt(th)).max(1)
        ux = np.linspace(lo[0], hi[0], g.n[0])
        uy = np.linspace(lo[1], hi[1], g.n[1])
        M = np.outer(np.r_[0.5, np.ones(g.n[0] - 2), 0.5] * (ux[1] - ux[0]),
                     np.r_[0.5, np.ones(g.n[1] - 2), 0.5] * (uy[1] - uy[0]))
        pair = wl.states[:, [P["ni"][q], P["nj"][q]]]
        gg, thp = maxwellians(pair, gamma, d, ux, uy)
        n = P["normals"][:, q]
        un = ux[:, None] * n[0] + uy[None, :] * n[1]
        lam = np.abs(un).max()
        wa = 0.5 + 0.5 * un / lam                 # convex weights of g_i and g_j
        gb = wa * gg[0] + (1 - wa) * gg[1]
        gI = wa * gg[0] * 0.5 * thp[0] * delta + (1 - wa) * gg[1] * 0.5 * thp[1] * delta
        h = 0.5 * (ux[:, None] ** 2 + uy[None, :] ** 2)
        mom = [(M * gb).sum(), (M * ux[:, None] * gb).sum(), (M * uy[None, :] * gb).sum(),
               (M * (h * gb + gI)).sum()]
        for v in range(4):
            tol = 1e-12 * max(abs(b[v, e]), abs(b[4 + v, e]), 1.0)
            assert b[v, e] - tol <= mom[v] <= b[4 + v, e] + tol, (q, v, b[v, e], mom[v], b[4 + v, e])
        checked += 1
    assert checked >= 60


def test_riemann_states_with_grid_speed_lie_in_relaxed_bounds():
    """The exact-flux formula with lambda = the velocity box's extent along n
    differs from the discrete moments only by quadrature/truncation error,
    which the relaxation r = 1e-3 covers."""
    wl = synth.make_quad_fr_workload(N=6, seed=10, grid_nodes=48)
    g = wl.grid
    b, _ = oracle.bounds(2, wl.gamma, wl.states, wl.rowptr, wl.cols, 1, g.mode, g.n[:2], g.lo,
                         g.hi, g.k, 1e-3, n_src=wl.n_state_nodes)
    P = wl.meta["face_pairs"]
    # lambda: max |u.n| over the element's velocity box corners
    rho = wl.states[0]
    U = wl.states[1:3] / rho
    th = (wl.gamma - 1) * (wl.states[3] - 0.5 * rho * (U ** 2).sum(0)) / rho
    lam = np.empty(P["ni"].size)
    for q in range(lam.size):
        e = P["elem"][q]
        sten = wl.cols[wl.rowptr[e]:wl.rowptr[e + 1]]
        lo = (U[:, sten] - g.k * np.sqrt(th[sten])).min(1)
        hi = (U[:, sten] + g.k * np.sqrt(th[sten])).max(1)
        n = P["normals"][:, q]
        lam[q] = max(abs(lo @ n), abs(hi @ n), abs(lo[0] * n[0] + hi[1] * n[1]),
                     abs(hi[0] * n[0] + lo[1] * n[1]))
    bar, st = oracle.riemann(2, wl.gamma, wl.states, P["ni"], P["nj"], P["normals"], lam,
                             b, P["elem"])
    assert not st.any(), f"{int((st > 0).sum())} of {st.size} outside"
    # with the macroscopic wavespeed estimate (the remark after the theorem)
    _, st2 = oracle.riemann(2, wl.gamma, wl.states, P["ni"], P["nj"], P["normals"], None,
                            b, P["elem"])
    print(f"[riemann] wavespeed estimate: {int((st2 > 0).sum())} of {st2.size} outside the bounds")
