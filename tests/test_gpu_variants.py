"""GPU vs oracle for the variants of the method:

- independent per-component limiting (Sec. 3.4), KBL_FLAG_INDEPENDENT_ALPHA;
- node-level stencils (solution + flux points, Sec. 5) through
  kbl_compute_bounds_nodes, and the limiter on V with zero-weight flux points;
- energy bounds from the per-state integrand (reading (A) of Sec. 3.6),
  KBL_FLAG_ENERGY_PERSTATE.

Tolerances as for the default method: 1e-12 relative (momentum against the
stencil's momentum scale) for bounds, 1e-11 for limited values.
"""

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import GRID_GLOBAL, GRID_STENCIL, GridSpec
from tests._parity import (bounds_error, element_value_scale, limited_error,
                           node_stencil_momentum_scale, stencil_momentum_scale)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def kbl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2407_20966_amd as kbl
    return kbl


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def vgrid_of(kbl, wl):
    g = wl.grid
    return kbl.make_vgrid(g.mode, g.n[: wl.dim], g.lo, g.hi, g.k)


# ---------------------------------------------------------------- independent alpha

@pytest.mark.parametrize("amp", [1.0, 3.0])
def test_independent_alpha_matches_oracle(kbl, amp):
    wl = synth.make_quad_workload(N=16, seed=70, grid_nodes=32, name="ind")
    wl.target = wl.states + amp * (wl.target - wl.states)
    rb, _ = oracle.workload_bounds(wl)
    rl, ral, rls = oracle.workload_limit(wl, rb, independent=True)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac, independent_alpha=True)
    lim, al, ls = kbl.limit(dev(wl.target), dev(rb), wl.node_weights, wl.n_s, prm)
    torch.cuda.synchronize()
    lim = lim.cpu().numpy()
    err, _ = limited_error(lim, rl, element_value_scale(wl, wl.target), wl.n_s)
    print(f"[variants] independent alpha x{amp}: limited err {err:.2e}, p-steps "
          f"{((rls & oracle.ST_PSTEP) > 0).sum()}/{wl.n_elem}", flush=True)
    assert err <= TOL
    assert np.array_equal(ls.cpu().numpy().view(np.uint32), rls)
    np.testing.assert_allclose(al.cpu().numpy(), ral, rtol=1e-11, atol=1e-14)
    # and it differs from the coupled form where more than one component binds
    lc, _, _ = kbl.limit(dev(wl.target), dev(rb), wl.node_weights, wl.n_s,
                         kbl.make_params(wl.gamma, r_fac=wl.r_fac))
    torch.cuda.synchronize()
    assert not np.array_equal(lc.cpu().numpy(), lim)


# ---------------------------------------------------------------- node-level stencils

def fr_inputs(kbl, wl):
    return dev(wl.states), dev(wl.rowptr), dev(wl.cols), vgrid_of(kbl, wl)


def check_fr(kbl, wl, elems=None):
    st, rp, cl, vg = fr_inputs(kbl, wl)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    b, s = kbl.compute_bounds_nodes(st, rp, cl, vg, prm)
    torch.cuda.synchronize()
    g = wl.grid
    rb, rs = oracle.bounds(2, wl.gamma, wl.states, wl.rowptr, wl.cols, 1, g.mode, g.n[:2], g.lo,
                           g.hi, g.k, wl.r_fac, elems=elems, n_src=wl.n_state_nodes)
    sel = np.arange(wl.n_elem) if elems is None else elems
    mscale = node_stencil_momentum_scale(wl.states, wl.rowptr, wl.cols, 2, sel)
    err, _ = bounds_error(b.cpu().numpy()[:, sel], rb, 2, mscale)
    assert np.array_equal(s.cpu().numpy().view(np.uint32)[sel], rs)
    # limiter on V: 16 solution points (Gauss-Legendre weights) + 16 flux points (weight 0)
    lim, al, ls = kbl.limit(dev(wl.target), b, wl.v_weights, wl.n_v, prm)
    torch.cuda.synchronize()
    rl, ral, rls = oracle.limit(2, wl.gamma, wl.target, rb, wl.v_weights, wl.n_v, elems=elems)
    nodes = (sel[:, None] * wl.n_v + np.arange(wl.n_v)[None, :]).ravel()
    T = wl.target.reshape(4, wl.n_elem, wl.n_v)[:, sel]
    scale = np.abs(T).max(2)
    scale[1:3] = np.maximum(scale[1:3], mscale[None, :])
    lerr, _ = limited_error(lim.cpu().numpy()[:, nodes], rl, scale, wl.n_v)
    print(f"[variants] {wl.name}: node-stencil bounds err {err:.2e}, limited err {lerr:.2e}, "
          f"limited {(ral[0] < 1).sum()}/{len(sel)}", flush=True)
    assert err <= TOL
    assert lerr <= TOL
    return b


def test_fr_node_stencil_full(kbl):
    check_fr(kbl, synth.make_quad_fr_workload(N=12, seed=71, name="fr12"))


@pytest.mark.parametrize("n", [20, 48, 64])
def test_fr_node_stencil_grid_sizes(kbl, n):
    check_fr(kbl, synth.make_quad_fr_workload(N=6, seed=72 + n, grid_nodes=n, name=f"fr_n{n}"))


def test_fr_node_stencil_full_size_sampled(kbl):
    wl = synth.make_workload("quad256_fr")
    check_fr(kbl, wl, elems=synth.sample_elements(wl, 192))


def test_node_stencil_listing_element_nodes_is_bit_identical(kbl):
    wl = synth.make_quad_workload(N=12, seed=73, grid_nodes=48, name="nodes_eq")
    st = dev(wl.states)
    vg = vgrid_of(kbl, wl)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    b1, s1 = kbl.compute_bounds(st, dev(wl.rowptr), dev(wl.cols), wl.n_s, vg, prm)
    cols_n = (wl.cols[:, None].astype(np.int64) * wl.n_s + np.arange(wl.n_s)).ravel()
    b2, s2 = kbl.compute_bounds_nodes(st, dev((wl.rowptr * wl.n_s).astype(np.int32)),
                                      dev(cols_n.astype(np.int32)), vg, prm)
    torch.cuda.synchronize()
    assert torch.equal(b1, b2) and torch.equal(s1, s2)


def test_node_stencil_bad_node_ids(kbl):
    wl = synth.make_quad_fr_workload(N=4, seed=74, name="fr_bad")
    cols = wl.cols.copy()
    cols[48 * 3 + 5] = wl.n_state_nodes          # one past the last node
    st, rp, _, vg = fr_inputs(kbl, wl)
    b, s = kbl.compute_bounds_nodes(st, rp, dev(cols), vg, kbl.make_params(wl.gamma))
    torch.cuda.synchronize()
    s = s.cpu().numpy().view(np.uint32)
    assert s[3] & kbl.ST_BAD_STENCIL and np.isnan(b.cpu().numpy()[:, 3]).all()
    assert not (s[[0, 1, 2]] & kbl.ST_BAD_STENCIL).any()


# ---------------------------------------------------------------- energy reading (A)

def check_energy(kbl, wl, elems=None):
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac, energy_perstate=True)
    b, s = kbl.compute_bounds(dev(wl.states), dev(wl.rowptr), dev(wl.cols), wl.n_s,
                              vgrid_of(kbl, wl), prm)
    torch.cuda.synchronize()
    rb, rs = oracle.workload_bounds(wl, elems=elems, energy_mode=1)
    sel = np.arange(wl.n_elem) if elems is None else elems
    err, _ = bounds_error(b.cpu().numpy()[:, sel], rb, wl.dim, stencil_momentum_scale(wl, sel))
    print(f"[variants] energy per state {wl.name} grid {wl.grid.n[:wl.dim]}: bounds err {err:.2e}",
          flush=True)
    assert err <= TOL
    assert np.array_equal(s.cpu().numpy().view(np.uint32)[sel], rs)


@pytest.mark.parametrize("n", [(13, 7), (16, 16), (30, 30), (48, 48), (64, 64), (50, 61)])
def test_energy_perstate_quads(kbl, n):
    wl = synth.make_quad_workload(N=8, seed=80 + n[0], grid_nodes=n[0], name=f"eA_{n}")
    wl.grid = GridSpec(GRID_STENCIL, n, k=4.0)
    check_energy(kbl, wl)


def test_energy_perstate_global_box_and_triangles(kbl):
    check_energy(kbl, synth.make_quad_workload(N=8, seed=90, field_kind="sine", grid_nodes=64,
                                               grid_mode=GRID_GLOBAL, name="eA_global"))
    check_energy(kbl, synth.make_tri_workload(N=8, seed=91, grid_nodes=48, name="eA_tri"))


@pytest.mark.parametrize("n", [64, 700, 4096])
def test_energy_perstate_line(kbl, n):
    wl = synth.make_line_workload(n_elem=16, seed=92 + n, name=f"eA_line{n}")
    wl.grid = GridSpec(GRID_STENCIL, (n, 1), k=8.0)
    check_energy(kbl, wl)


def test_energy_perstate_full_size_sampled(kbl):
    wl = synth.make_workload("quad256")
    check_energy(kbl, wl, elems=synth.sample_elements(wl, 128))


def test_energy_perstate_monatomic(kbl):
    # delta = 0: the per-state integrand is g |u|^2 / 2, as in the default reading
    wl = synth.make_quad_workload(N=6, seed=93, grid_nodes=32, gamma=2.0, name="eA_mono")
    check_energy(kbl, wl)


@pytest.mark.parametrize("case", ["quad", "line"])
def test_energy_perstate_extreme_temperature_ratio(kbl, case):
    """Every fifth element at rest with theta = 1e-12 among states at theta
    ~ 1: the value-space factors exp(A), exp(B) of the cold states underflow
    to 0 over most of the box (clamped table exp), as in the oracle."""
    if case == "quad":
        wl = synth.make_quad_workload(N=8, seed=94, grid_nodes=32, name="eA_cold")
    else:
        wl = synth.make_line_workload(n_elem=64, seed=95, name="eA_cold_line")
    d = wl.dim
    st = wl.states.copy()
    cold = np.arange(wl.n_elem)[::5]
    nodes = (cold[:, None] * wl.n_s + np.arange(wl.n_s)[None, :]).ravel()
    st[1:1 + d, nodes] = 0.0
    st[d + 1, nodes] = 1e-12 * st[0, nodes] / (wl.gamma - 1.0)
    wl.states = st
    check_energy(kbl, wl)
