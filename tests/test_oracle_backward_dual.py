"""Pins of the oracle's analytic subgradient against forward-mode derivatives
(dual numbers, tests/_dual.py) of a separate NumPy restatement of the
forward pass, one unit direction per DoF of (states, solution) on small
inputs.  Unlike finite differences this is exact up to rounding, so each
entry is held to 1e-12 relative to max(|ref|, 1e-3 of the largest entry).
Covered: 1D global and per-stencil boxes (the box ends move with their
states), 2D quads and P2 triangles on per-stencil boxes, and the pressure
step."""

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import GRID_STENCIL, GridSpec

import _dual

TOL = 1e-12


def dual_gradient(wl, G):
    g = wl.grid
    J = _dual.objective(wl.dim, wl.gamma, wl.states, wl.target, wl.rowptr, wl.cols, wl.n_s,
                        g.mode, g.n[: wl.dim], g.lo, g.hi, g.k, wl.r_fac, wl.node_weights, G)
    nv, nn = wl.states.shape
    return J.v, J.d[: nv * nn].reshape(nv, nn), J.d[nv * nn:].reshape(nv, nn)


def compare(wl, seed=0):
    G = np.random.default_rng(seed).standard_normal(wl.target.shape)
    gsol, gst, _ = oracle.workload_backward(wl, G)
    Jv, dst, dsol = dual_gradient(wl, G)
    # the restated forward reproduces the oracle's objective
    b, _ = oracle.workload_bounds(wl)
    lim, _, _ = oracle.workload_limit(wl, b)
    Jo = float((G * lim).sum())
    assert abs(float(Jv) - Jo) <= 1e-12 * max(1.0, abs(Jo))
    worst = {}
    for name, a, ref in (("states", gst, dst), ("solution", gsol, dsol)):
        scale = np.abs(ref).max()
        assert scale > 0
        err = np.abs(a - ref) / np.maximum(np.abs(ref), 1e-3 * scale)
        worst[name] = float(err.max())
        assert worst[name] <= TOL, f"{wl.name} d/d{name}: {worst[name]:.2e}"
    print(f"[dual] {wl.name}: d/dstates {worst['states']:.1e}, d/dsolution "
          f"{worst['solution']:.1e}", flush=True)


def test_line_global_box():
    compare(synth.make_line_workload(n_elem=3, seed=41, name="d_line"))


def test_line_stencil_box():
    wl = synth.make_line_workload(n_elem=3, seed=42, name="d_line_st")
    wl.grid = GridSpec(GRID_STENCIL, (96, 1), k=6.0)
    wl.target = wl.states + 20.0 * (wl.target - wl.states)
    compare(wl, seed=1)


def test_quad_stencil_box():
    wl = synth.make_quad_workload(N=3, p=1, seed=43, grid_nodes=12, name="d_quad")
    wl.target = wl.states + 10.0 * (wl.target - wl.states)
    compare(wl, seed=2)


def test_tri_stencil_box():
    wl = synth.make_tri_workload(N=2, seed=45, grid_nodes=10, outer=(0.5, 0.3), name="d_tri")
    wl.target = wl.states + 20.0 * (wl.target - wl.states)
    compare(wl, seed=3)


def test_pressure_step():
    wl = synth.make_line_workload(n_elem=4, seed=36, grid_nodes=48, r_fac=0.97, name="d_pstep")
    wl.target = wl.target.copy()
    for i in (5, 9, 13):
        wl.target[2, i] = 0.3 * 0.5 * wl.target[1, i] ** 2 / wl.target[0, i]
    b, _ = oracle.workload_bounds(wl)
    _, _, st = oracle.workload_limit(wl, b)
    assert (st & oracle.ST_PSTEP).any()
    compare(wl, seed=4)
