"""Pins of the oracle's variants: independent limiting (Sec. 3.4), zero-weight
nodes and node-level stencils (the solution + flux point stencils of Sec. 5),
and the per-state energy integrand (reading (A) of the internal-energy model
of Sec. 3.6).  Each pin is a property the mathematics fixes, not a retyped
formula.
"""

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import GRID_GLOBAL, GRID_STENCIL, GridSpec


def quad(seed=3, N=4, n=24, mode=GRID_STENCIL):
    wl = synth.make_quad_workload(N=N, seed=seed, grid_nodes=n, grid_mode=mode, name="v_quad")
    if mode == GRID_GLOBAL:
        assert wl.grid.hi[0] > wl.grid.lo[0]
    return wl


def scalar_squeeze(w, c, bmin, bmax, eps=1e-13):
    """Zhang-Shu squeeze of one scalar component (Sec. 2.4)."""
    wbar = (c * w).sum() / c.sum()
    dp, dm = w.max() - wbar, w.min() - wbar
    if abs(dp) < eps or abs(dm) < eps:
        a = 0.0
    else:
        a = min(1.0, abs((bmax - wbar) / dp), abs((bmin - wbar) / dm))
    return wbar + a * (w - wbar), a


# ------------------------------------------------------------ independent alpha

def test_independent_alpha_is_the_scalar_limiter_per_component():
    """Each component is the scalar squeeze limiter (Sec. 2.4) with its own
    alpha_i; the pressure step then scales every component by alpha_P."""
    wl = quad(seed=11, N=6)
    wl.target = wl.states + 3.0 * (wl.target - wl.states)
    b, _ = oracle.workload_bounds(wl)
    lim, al, st = oracle.workload_limit(wl, b, independent=True)
    c = wl.node_weights
    n_limited = 0
    for e in range(wl.n_elem):
        sl = slice(e * wl.n_s, (e + 1) * wl.n_s)
        amin = 1.0
        for v in range(4):
            w = wl.target[v, sl]
            ref, a = scalar_squeeze(w, c, b[v, e], b[4 + v, e])
            amin = min(amin, a)
            wbar = (c * w).sum() / c.sum()
            ref = wbar + al[1, e] * (ref - wbar)          # pressure step on top
            np.testing.assert_allclose(lim[v, sl], ref, rtol=1e-13, atol=1e-13 * abs(ref).max())
        assert al[0, e] == pytest.approx(amin, rel=1e-11, abs=1e-15)   # mean: compensated vs plain sum
        n_limited += amin < 1.0
    assert n_limited > wl.n_elem // 2


def test_independent_equals_coupled_when_one_component_binds():
    wl = quad(seed=12, N=6)
    b, _ = oracle.workload_bounds(wl)
    lim_c, al_c, st_c = oracle.workload_limit(wl, b)
    lim_i, al_i, st_i = oracle.workload_limit(wl, b, independent=True)
    # elements left alone by both forms agree exactly; alpha_min is the same
    np.testing.assert_array_equal(al_c[0], al_i[0])
    same = al_c[0] == 1.0
    nodes = (np.nonzero(same)[0][:, None] * wl.n_s + np.arange(wl.n_s)).ravel()
    np.testing.assert_array_equal(lim_c[:, nodes], lim_i[:, nodes])


def test_independent_limits_each_component_into_its_bounds_and_keeps_the_mean():
    wl = quad(seed=13, N=6)
    wl.target = wl.states + 2.0 * (wl.target - wl.states)
    b, _ = oracle.workload_bounds(wl)
    lim, al, st = oracle.workload_limit(wl, b, independent=True)
    c = wl.node_weights / wl.node_weights.sum()
    L = lim.reshape(4, wl.n_elem, wl.n_s)
    T = wl.target.reshape(4, wl.n_elem, wl.n_s)
    np.testing.assert_allclose((L * c).sum(2), (T * c).sum(2), rtol=1e-13, atol=1e-13)
    ok = (st & (oracle.ST_MEAN_OUTSIDE | oracle.ST_EPS_RULE)) == 0
    tol = 1e-12 * np.abs(b).max(0)
    assert np.all(L.min(2)[:, ok] >= b[:4, ok] - tol[ok])
    assert np.all(L.max(2)[:, ok] <= b[4:, ok] + tol[ok])
    # before any pressure step, independent limiting keeps every node at least
    # as far from the mean as coupled limiting (alpha_i >= alpha_min)
    lc, _, stc = oracle.workload_limit(wl, b)
    Lc = lc.reshape(4, wl.n_elem, wl.n_s)
    mean = (T * c).sum(2, keepdims=True)
    no_p = ((st | stc) & oracle.ST_PSTEP) == 0
    assert no_p.sum() >= 4
    d_ind = np.abs(L - mean)[:, no_p]
    d_cpl = np.abs(Lc - mean)[:, no_p]
    assert np.all(d_ind >= d_cpl - 1e-12 * np.abs(mean[:, no_p]))


# ------------------------------------------------------------ zero-weight nodes

def test_zero_weight_copies_of_nodes_change_nothing():
    wl = quad(seed=14, N=5)
    wl.target = wl.states + 8.0 * (wl.target - wl.states)
    b, _ = oracle.workload_bounds(wl)
    lim, al, st = oracle.workload_limit(wl, b)
    # V gets 4 extra nodes per element: copies of nodes 0..3, with weight 0
    T = wl.target.reshape(4, wl.n_elem, wl.n_s)
    T2 = np.concatenate([T, T[:, :, :4]], axis=2).reshape(4, -1)
    c2 = np.concatenate([wl.node_weights, np.zeros(4)])
    lim2, al2, st2 = oracle.limit(2, wl.gamma, T2, b, c2, wl.n_s + 4)
    np.testing.assert_array_equal(al2, al)
    np.testing.assert_array_equal(st2, st)
    L2 = lim2.reshape(4, wl.n_elem, wl.n_s + 4)
    np.testing.assert_array_equal(L2[:, :, :wl.n_s].reshape(4, -1), lim)
    np.testing.assert_array_equal(L2[:, :, wl.n_s:], L2[:, :, :4])


def test_weights_must_have_a_positive_sum():
    wl = quad(seed=15, N=2)
    b, _ = oracle.workload_bounds(wl)
    with pytest.raises(ValueError):
        oracle.limit(2, wl.gamma, wl.target, b, np.zeros(wl.n_s), wl.n_s)
    with pytest.raises(ValueError):
        oracle.limit(2, wl.gamma, wl.target, b, -wl.node_weights, wl.n_s)


# ------------------------------------------------------------ node-level stencils

@pytest.mark.parametrize("mode", [GRID_STENCIL, GRID_GLOBAL])
def test_node_stencil_listing_the_element_nodes_is_identical(mode):
    wl = quad(seed=16, N=4, mode=mode)
    b, st = oracle.workload_bounds(wl)
    # the same stencil, written out node by node
    cols_n = (wl.cols[:, None].astype(np.int64) * wl.n_s + np.arange(wl.n_s)).ravel()
    rowptr_n = wl.rowptr.astype(np.int64) * wl.n_s
    g = wl.grid
    bn, stn = oracle.bounds(2, wl.gamma, wl.states, rowptr_n, cols_n, 1, g.mode, g.n[:2],
                            g.lo, g.hi, g.k, wl.r_fac, n_src=wl.n_elem * wl.n_s)
    np.testing.assert_array_equal(bn, b)
    np.testing.assert_array_equal(stn, st)


def test_node_stencil_subset_gives_inner_bounds():
    """Fewer stencil nodes can only tighten the bounds (min over a subset)."""
    wl = quad(seed=17, N=4, mode=GRID_GLOBAL)
    g = wl.grid
    cols_n = (wl.cols[:, None].astype(np.int64) * wl.n_s + np.arange(wl.n_s)).ravel()
    rowptr_n = wl.rowptr.astype(np.int64) * wl.n_s
    full, _ = oracle.bounds(2, wl.gamma, wl.states, rowptr_n, cols_n, 1, g.mode, g.n[:2], g.lo,
                            g.hi, g.k, wl.r_fac, n_src=wl.n_elem * wl.n_s)
    keep = np.ones(cols_n.size, bool)
    keep[1::3] = False                       # drop every third node (rows stay non-empty)
    counts = np.add.reduceat(keep.astype(np.int64), rowptr_n[:-1])
    rp = np.concatenate([[0], np.cumsum(counts)])
    sub, _ = oracle.bounds(2, wl.gamma, wl.states, rp, cols_n[keep], 1, g.mode, g.n[:2], g.lo,
                           g.hi, g.k, wl.r_fac, n_src=wl.n_elem * wl.n_s)
    tol = 1e-13 * np.abs(full)
    assert np.all(sub[:4] >= full[:4] - tol[:4])
    assert np.all(sub[4:] <= full[4:] + tol[4:])


def test_node_stencil_rejects_out_of_range_nodes():
    wl = quad(seed=18, N=2)
    g = wl.grid
    rowptr = np.array([0, 2], dtype=np.int64)
    cols = np.array([0, wl.n_elem * wl.n_s], dtype=np.int64)   # one past the last node
    b, st = oracle.bounds(2, wl.gamma, wl.states, rowptr, cols, 1, g.mode, g.n[:2], g.lo,
                          g.hi, g.k, wl.r_fac, n_src=wl.n_elem * wl.n_s)
    assert st[0] & oracle.ST_BAD_STENCIL and np.isnan(b).all()


# ------------------------------------------------------------ energy reading (A)

def test_energy_per_state_equals_reduced_for_one_state():
    wl = quad(seed=19, N=3)
    wl.rowptr = np.arange(wl.n_elem + 1, dtype=np.int32)
    wl.cols = np.arange(wl.n_elem, dtype=np.int32)
    # single-node stencils: one state per element
    g = wl.grid
    cols_n = (np.arange(wl.n_elem) * wl.n_s).astype(np.int64)
    rp = np.arange(wl.n_elem + 1, dtype=np.int64)
    a, _ = oracle.bounds(2, wl.gamma, wl.states, rp, cols_n, 1, g.mode, g.n[:2], g.lo, g.hi,
                         g.k, wl.r_fac, n_src=wl.n_elem * wl.n_s, energy_mode=1)
    bb, _ = oracle.bounds(2, wl.gamma, wl.states, rp, cols_n, 1, g.mode, g.n[:2], g.lo, g.hi,
                          g.k, wl.r_fac, n_src=wl.n_elem * wl.n_s, energy_mode=0)
    np.testing.assert_array_equal(a[[0, 1, 2, 4, 5, 6]], bb[[0, 1, 2, 4, 5, 6]])
    np.testing.assert_allclose(a[[3, 7]], bb[[3, 7]], rtol=1e-14)


@pytest.mark.parametrize("mode", [GRID_STENCIL, GRID_GLOBAL])
def test_energy_per_state_is_inside_reduced(mode):
    """min_i g_i (h + c_i) >= min_i g_i h + min_i g_i c_i node by node, and the
    reverse for max: reading (A) lies inside reading (B); rho and m untouched."""
    wl = quad(seed=20, N=5, mode=mode)
    a, sa = oracle.workload_bounds(wl, energy_mode=1)
    b, sb = oracle.workload_bounds(wl, energy_mode=0)
    np.testing.assert_array_equal(a[[0, 1, 2, 4, 5, 6]], b[[0, 1, 2, 4, 5, 6]])
    np.testing.assert_array_equal(sa, sb)
    assert np.all(a[3] >= b[3] * (1 - 1e-14))
    assert np.all(a[7] <= b[7] * (1 + 1e-14))
    # and strictly tighter where different states win g and g_I
    assert (a[3] > b[3] * (1 + 1e-9)).any() and (a[7] < b[7] * (1 - 1e-9)).any()


def test_energy_per_state_contains_every_stencil_energy():
    """Thm. 4.5 analogue: each stencil state's energy lies in its bounds (up to
    the quadrature error of a fine grid, k = 8 box)."""
    wl = quad(seed=21, N=3, n=64)
    wl.grid = GridSpec(GRID_STENCIL, (64, 64), k=8.0)
    a, _ = oracle.workload_bounds(wl, energy_mode=1, r_fac=0.0)
    E = wl.states[3].reshape(wl.n_elem, wl.n_s)
    for e in range(wl.n_elem):
        sten = wl.cols[wl.rowptr[e]:wl.rowptr[e + 1]]
        Es = E[sten].ravel()
        assert a[3, e] <= Es.min() * (1 + 1e-6)
        assert a[7, e] >= Es.max() * (1 - 1e-6)
