"""Pins of the oracle's analytic subgradient against finite differences of the
oracle's own forward pass (bounds + limiter), J = sum G * limited.

Central differences with h = 1e-6 max(1, |x|); a DoF whose forward and
backward one-sided differences disagree sits within h of a kink of the
min/max envelopes or of the limiter's active set, and is only counted.
"""

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import GRID_GLOBAL, GRID_STENCIL, GridSpec


def J_of(wl, states, solution, G):
    g = wl.grid
    b, _ = oracle.bounds(wl.dim, wl.gamma, states, wl.rowptr, wl.cols, wl.n_s, g.mode,
                         g.n[: wl.dim], g.lo, g.hi, g.k, wl.r_fac)
    lim, _, _ = oracle.limit(wl.dim, wl.gamma, solution, b, wl.node_weights, wl.n_s)
    return float((G * lim).sum())


def fd_check(wl, which, n_dofs=40, seed=0, tol=2e-5):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal(wl.target.shape)
    gsol, gst, _ = oracle.workload_backward(wl, G)
    an = gst if which == "states" else gsol
    base = {"states": wl.states, "solution": wl.target}
    nv, nn = wl.states.shape
    dofs = [(int(rng.integers(nv)), int(rng.integers(nn))) for _ in range(n_dofs)]
    errs, kinks = [], 0
    scale = np.abs(an).max()
    J0 = abs(J_of(wl, wl.states, wl.target, G))
    assert scale > 1e-6 * J0, "degenerate case: the gradient vanishes"
    for v, i in dofs:
        x = base[which]
        h = 1e-6 * max(1.0, abs(x[v, i]))
        vals = {}
        for sgn in (-1, 0, 1):
            y = x.copy()
            y[v, i] += sgn * h
            st = y if which == "states" else wl.states
            so = y if which == "solution" else wl.target
            vals[sgn] = J_of(wl, st, so, G)
        fwd = (vals[1] - vals[0]) / h
        bwd = (vals[0] - vals[-1]) / h
        cen = (vals[1] - vals[-1]) / (2 * h)
        if abs(fwd - bwd) > 1e-3 * (abs(cen) + 1e-3 * scale):
            kinks += 1
            continue
        noise = 1e3 * np.finfo(float).eps * J0 / h      # rounding floor of the difference
        errs.append(abs(cen - an[v, i]) / max(abs(an[v, i]), 1e-3 * scale, noise))
    print(f"[fd] {wl.name} {which}: {len(errs)} smooth DoFs, max rel err "
          f"{max(errs) if errs else 0:.2e}, {kinks} near kinks", flush=True)
    assert len(errs) >= 0.7 * n_dofs
    assert max(errs) < tol, max(errs)


@pytest.mark.parametrize("which", ["states", "solution"])
def test_line_global_grid(which):
    wl = synth.make_line_workload(n_elem=6, seed=31, grid_nodes=64, name="fd_line")
    fd_check(wl, which)


@pytest.mark.parametrize("which", ["states", "solution"])
def test_line_stencil_grid(which):
    wl = synth.make_line_workload(n_elem=6, seed=32, name="fd_line_st")
    wl.grid = GridSpec(GRID_STENCIL, (101, 1), k=5.0)
    fd_check(wl, which)


@pytest.mark.parametrize("which", ["states", "solution"])
def test_quad_stencil_grid(which):
    wl = synth.make_quad_workload(N=3, seed=33, grid_nodes=20, name="fd_quad")
    fd_check(wl, which, n_dofs=30)


def test_quad_global_grid_states():
    wl = synth.make_quad_workload(N=3, seed=34, field_kind="sine", grid_nodes=24,
                                  grid_mode=GRID_GLOBAL, name="fd_quad_gl")
    wl.target = wl.states + 30.0 * (wl.target - wl.states)   # make the bounds bind
    fd_check(wl, "states", n_dofs=30)


def test_tri_stencil_grid_states():
    wl = synth.make_tri_workload(N=2, seed=35, grid_nodes=16, outer=(0.5, 0.3), name="fd_tri")
    wl.target = wl.states + 20.0 * (wl.target - wl.states)
    fd_check(wl, "states", n_dofs=30)


def test_pressure_step_gradient():
    """Elements where the pressure step fires carry the alpha_P terms."""
    wl = synth.make_line_workload(n_elem=6, seed=36, grid_nodes=64, r_fac=0.97, name="fd_pstep")
    wl.target = wl.target.copy()
    # wide (heavily relaxed) bounds keep alpha near 1; energy pushed below the
    # kinetic energy at a few nodes makes their pressure negative
    for i in (5, 13, 18):
        wl.target[2, i] = 0.3 * 0.5 * wl.target[1, i] ** 2 / wl.target[0, i]
    b, _ = oracle.workload_bounds(wl)
    _, _, st = oracle.workload_limit(wl, b)
    assert (st & oracle.ST_PSTEP).any()
    fd_check(wl, "solution", n_dofs=40, seed=3)



def _dedup_rows(rowptr, cols):
    rp, cl = [0], []
    for e in range(rowptr.size - 1):
        seen = []
        for c in cols[rowptr[e]:rowptr[e + 1]]:
            if c not in seen:
                seen.append(int(c))
        cl.extend(seen)
        rp.append(len(cl))
    return np.array(rp, dtype=np.int32), np.array(cl, dtype=np.int32)


@pytest.mark.parametrize("N,seed", [(1, 41), (2, 40)])
def test_duplicate_stencil_entries(N, seed):
    """Periodic meshes one or two elements wide list the same neighbour more
    than once in a stencil row (left = right, down = up).  The bounds depend
    on the set of stencil states only (eq. fminmax takes min/max over the
    states), so the gradient with the repeated entries must equal the one
    with each row reduced to distinct entries; finite differences of the
    forward pin it too."""
    wl = synth.make_quad_workload(N=N, seed=seed, grid_nodes=20, name=f"fd_dup{N}")
    row = wl.cols[wl.rowptr[0]:wl.rowptr[1]]
    assert len(np.unique(row)) < len(row)
    wl.target = wl.states + 20.0 * (wl.target - wl.states)
    G = np.random.default_rng(seed).standard_normal(wl.target.shape)
    gsol, gst, gb = oracle.workload_backward(wl, G)
    rp, cl = _dedup_rows(wl.rowptr, wl.cols)
    g = wl.grid
    gsol1, gst1, gb1 = oracle.backward(wl.dim, wl.gamma, wl.states, rp, cl, wl.n_s, g.mode,
                                       g.n[:2], g.lo, g.hi, g.k, wl.r_fac, wl.target,
                                       wl.node_weights, G)
    for a, b in ((gsol, gsol1), (gst, gst1), (gb, gb1)):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.abs(b).max())
    fd_check(wl, "states", n_dofs=30, seed=N)


@pytest.mark.parametrize("case", ["quad", "line"])
def test_gradient_is_scale_invariant(case):
    """J = sum G limited is homogeneous of degree one in (states, solution)
    (moments linear in the Maxwellians, Sec. 3.3; eq. limiter and
    eq. doublelimit commute with scaling away from the absolute floors), so
    its gradient must not change when both are scaled.  A factor of the
    wrong degree in the chain rule (e.g. a missing 1/rho in d ln g / d rho)
    breaks this."""
    if case == "quad":
        wl = synth.make_quad_workload(N=3, seed=38, grid_nodes=20, name="sc_quad")
        wl.target = wl.states + 10.0 * (wl.target - wl.states)
    else:
        wl = synth.make_line_workload(n_elem=6, seed=39, grid_nodes=64, name="sc_line")
    G = np.random.default_rng(5).standard_normal(wl.target.shape)
    ref = oracle.workload_backward(wl, G)
    scale = max(np.abs(ref[1]).max(), np.abs(ref[0]).max())
    assert scale > 0
    for f in (3.0, 0.25):
        got = oracle.backward(wl.dim, wl.gamma, f * wl.states, wl.rowptr, wl.cols, wl.n_s,
                              wl.grid.mode, wl.grid.n[: wl.dim], wl.grid.lo, wl.grid.hi,
                              wl.grid.k, wl.r_fac, f * wl.target, wl.node_weights, G)
        for a, b in zip(got, ref):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-10 * np.abs(b).max())
