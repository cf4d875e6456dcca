"""GPU (HIP, FP64) vs the FP64 oracle, element by element, through the C-ABI.

Tolerance: 1e-12 relative (density and energy against |ref|; momentum against
the element momentum scale of tests/_parity.py).  Cases span every kernel
instantiation (1D and 2D tile shapes), ragged velocity grids, global and
per-stencil boxes, uneven stencils, the five named workloads (full or on a
seeded element sample) and the degenerate inputs the method has.
"""

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import GRID_GLOBAL, GRID_STENCIL, GridSpec, quad_block_stencils
from tests._parity import (bounds_error, element_value_scale, limited_error,
                           stencil_momentum_scale)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def kbl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2407_20966_amd as kbl
    return kbl


def run_gpu(kbl, wl, r_fac=None, bounds_override=None):
    dev = torch.device("cuda:0")
    st = torch.from_numpy(wl.states).to(dev)
    rp = torch.from_numpy(wl.rowptr).to(dev)
    cl = torch.from_numpy(wl.cols).to(dev)
    tg = torch.from_numpy(wl.target).to(dev)
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[: wl.dim], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac if r_fac is None else r_fac)
    b, s = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
    bl = b if bounds_override is None else torch.from_numpy(bounds_override).to(dev)
    lim, al, ls = kbl.limit(tg, bl, wl.node_weights, wl.n_s, prm)
    torch.cuda.synchronize()
    u32 = lambda t: t.cpu().numpy().view(np.uint32)
    return (b.cpu().numpy(), u32(s), lim.cpu().numpy(), al.cpu().numpy(), u32(ls))


def check_workload(kbl, wl, elems=None, r_fac=None, tol=TOL):
    print(f"[parity] {wl.name} n_elem={wl.n_elem} grid={wl.grid.n[:wl.dim]} "
          f"mode={wl.grid.mode} sample={None if elems is None else len(elems)}", flush=True)
    b, s, lim, al, ls = run_gpu(kbl, wl, r_fac)
    rb, rs = oracle.workload_bounds(wl, elems=elems, r_fac=r_fac)
    sel = np.arange(wl.n_elem) if elems is None else elems
    mscale = stencil_momentum_scale(wl, sel)
    err, _ = bounds_error(b[:, sel], rb, wl.dim, mscale)
    assert err <= tol, f"bounds error {err:.3e}"
    assert np.array_equal(s[sel], rs), "bounds status differs"
    # limiter end to end: GPU bounds -> GPU limit vs oracle bounds -> oracle limit
    rl, ral, rls = oracle.workload_limit(wl, rb, elems=elems)
    nodes = (sel[:, None] * wl.n_s + np.arange(wl.n_s)[None, :]).ravel()
    scale = element_value_scale(wl, wl.target, sel)
    lerr, _ = limited_error(lim[:, nodes], rl, scale, wl.n_s)
    assert lerr <= tol, f"limited error {lerr:.3e}"
    # status may differ only where the oracle sits on a decision threshold
    diff = ls[sel] != rls
    if diff.any():
        near = np.abs(ral[0] - 1.0) < 1e-9
        assert np.all(near[diff]), f"limiter status differs at {np.nonzero(diff)[0][:10]}"
    # alpha agrees through its effect on the nodes (alpha * max|w - mean|)
    span = (wl.target.reshape(wl.dim + 2, wl.n_elem, wl.n_s).max(2)
            - wl.target.reshape(wl.dim + 2, wl.n_elem, wl.n_s).min(2))[:, sel]
    rel_span = (span / np.where(scale > 0, scale, 1)).max(0)
    assert np.all(np.abs(al[0, sel] - ral[0]) * rel_span <= tol)
    print(f"[parity] {wl.name}: bounds err {err:.2e}, limited err {lerr:.2e}, "
          f"limited elements {(ral[0] < 1).sum()}/{len(sel)}, p-steps {((rls & 0x10) > 0).sum()}",
          flush=True)
    return err, lerr, ls[sel], rls


# ---------------------------------------------------------------- 1D

def test_line64_full(kbl):
    check_workload(kbl, synth.make_workload("line64"))


def test_line64_strict_bounds(kbl):
    check_workload(kbl, synth.make_workload("line64"), r_fac=0.0)


@pytest.mark.parametrize("n", [33, 256, 700, 2048, 4096])
def test_line_grid_sizes(kbl, n):
    # paper's 1D setting: k = 8 per-stencil box, up to 2048 nodes; plus ragged sizes
    wl = synth.make_line_workload(n_elem=24, seed=5 + n, name=f"line_n{n}")
    wl.grid = GridSpec(GRID_STENCIL, (n, 1), k=8.0)
    check_workload(kbl, wl)


# ---------------------------------------------------------------- 2D quads

@pytest.mark.parametrize("n", [(13, 7), (16, 16), (20, 30), (37, 45), (48, 48), (64, 64), (50, 61)])
def test_quad_tile_shapes_stencil_box(kbl, n):
    wl = synth.make_quad_workload(N=10, seed=100 + n[0], grid_nodes=n[0], name=f"quad_{n}")
    wl.grid = GridSpec(GRID_STENCIL, n, k=4.0)
    check_workload(kbl, wl)


def test_quad_global_box(kbl):
    wl = synth.make_quad_workload(N=12, seed=77, field_kind="sine", grid_nodes=64,
                                  grid_mode=GRID_GLOBAL, name="quad_sine_global")
    check_workload(kbl, wl)


def test_quad256_sampled(kbl):
    wl = synth.make_workload("quad256")
    check_workload(kbl, wl, elems=synth.sample_elements(wl, 384))


def test_quad1024_sine_sampled(kbl):
    wl = synth.make_workload("quad1024_sine")
    check_workload(kbl, wl, elems=synth.sample_elements(wl, 128))


def test_quad512_sampled(kbl):
    wl = synth.make_workload("quad512")
    check_workload(kbl, wl, elems=synth.sample_elements(wl, 128))


# ---------------------------------------------------------------- triangles

def test_tri_small_full(kbl):
    wl = synth.make_tri_workload(N=16, seed=9, name="tri16")
    check_workload(kbl, wl)


def test_tri2m_sampled(kbl):
    wl = synth.make_workload("tri2m")
    check_workload(kbl, wl, elems=synth.sample_elements(wl, 256))


# ---------------------------------------------------------------- edge cases

def test_empty_input(kbl):
    dev = torch.device("cuda:0")
    st = torch.zeros((4, 0), dtype=torch.float64, device=dev)
    rp = torch.zeros(1, dtype=torch.int32, device=dev)
    cl = torch.zeros(0, dtype=torch.int32, device=dev)
    vg = kbl.make_vgrid(GRID_STENCIL, (16, 16), k=4.0)
    prm = kbl.make_params(1.4)
    b, s = kbl.compute_bounds(st, rp, cl, 16, vg, prm)
    lim, al, ls = kbl.limit(st, b, np.ones(16), 16, prm)
    torch.cuda.synchronize()
    assert b.shape == (8, 0) and lim.shape == (4, 0)


def test_inadmissible_and_bad_rows(kbl):
    wl = synth.make_quad_workload(N=8, seed=3, grid_nodes=24, name="quad_bad")
    wl.states = wl.states.copy()
    # negative pressure at one node of element 10; NaN in element 20
    wl.states[3, 10 * 16 + 5] = 0.1 * wl.states[3, 10 * 16 + 5] - 50.0
    wl.states[1, 20 * 16 + 2] = np.nan
    wl.cols = wl.cols.copy()
    wl.cols[5 * 7 + 2] = wl.n_elem + 3          # out-of-range element id in row 7
    # a bad row that also lists the inadmissible element 10: reported as a bad row alone
    r = next(e for e in range(wl.n_elem) if e != 10 and 10 in wl.cols[5 * e:5 * e + 5])
    j = next(j for j in range(5) if wl.cols[5 * r + j] != 10)
    wl.cols[5 * r + j] = -1
    wl.rowptr = wl.rowptr.copy()
    b, s, lim, al, ls = run_gpu(kbl, wl)
    rb, rs = oracle.workload_bounds(wl)
    assert np.array_equal(s, rs)
    assert s[7] & kbl.ST_BAD_STENCIL
    assert s[r] == kbl.ST_BAD_STENCIL
    assert (s[10] & kbl.ST_INADMISSIBLE) and (s[20] & kbl.ST_INADMISSIBLE)
    assert np.array_equal(np.isnan(b), np.isnan(rb))
    good = ~np.isnan(rb).any(0)
    err, _ = bounds_error(b[:, good], rb[:, good], 2, stencil_momentum_scale(wl)[good])
    assert err <= TOL
    # the limiter passes elements with NaN bounds through unchanged
    bad_el = np.nonzero(~good)[0]
    assert np.all(ls[bad_el] == kbl.ST_BAD_BOUNDS)
    nodes = (bad_el[:, None] * 16 + np.arange(16)).ravel()
    np.testing.assert_array_equal(lim[:, nodes], wl.target[:, nodes])


def test_monatomic_gamma(kbl):
    # gamma = 1 + 2/d: no internal degrees of freedom (delta = 0)
    wl = synth.make_quad_workload(N=8, seed=4, grid_nodes=32, gamma=2.0, name="quad_mono")
    check_workload(kbl, wl)
    wl1 = synth.make_line_workload(n_elem=16, seed=4, gamma=3.0, name="line_mono")
    check_workload(kbl, wl1)


@pytest.mark.parametrize("case", ["quad", "line"])
def test_extreme_temperature_ratio(kbl, case):
    """Every fifth element at rest with theta = 1e-12 among states at theta
    of order 1: far out in the cold states' tails the log-Maxwellian reaches
    about -1e13 (per-stencil box, quad) or -7e13 (global box, line), beyond
    the 32-bit range of the exp's argument reduction, which clamps first; the
    envelopes underflow to 0 and rho_min is floored, as in the oracle."""
    if case == "quad":
        wl = synth.make_quad_workload(N=8, seed=71, grid_nodes=32, name="quad_cold")
    else:
        wl = synth.make_line_workload(n_elem=64, seed=72, name="line_cold")
    d = wl.dim
    st = wl.states.copy()
    cold = np.arange(wl.n_elem)[::5]
    nodes = (cold[:, None] * wl.n_s + np.arange(wl.n_s)[None, :]).ravel()
    st[1:1 + d, nodes] = 0.0
    st[d + 1, nodes] = 1e-12 * st[0, nodes] / (wl.gamma - 1.0)
    wl.states = st
    check_workload(kbl, wl)


def test_stencils_beyond_one_lds_chunk(kbl):
    """25-element stencils of 16 nodes (400 states): the FP64 kernel stages
    the coefficients in LDS in chunks of 256 states; bounds at 1e-12.  The
    wide bounds make the pressure step (eq. pmin, eq. doublelimit) act on
    most elements at low pressure, where the limited nodes are ill
    conditioned: rescaling the inputs by 3 moves the oracle's own result by
    about 1.5e-12.  The limiter is checked on the oracle's bounds against
    1e-12 or four times the larger of that rounding spread of both sides
    (the bar of the backward tests)."""
    wl = synth.make_quad_workload(N=6, seed=13, grid_nodes=24, name="quad_big")
    wl.rowptr, wl.cols = quad_block_stencils(6, 2)
    assert (np.diff(wl.rowptr) * wl.n_s).min() > 256
    b, s, _, _, _ = run_gpu(kbl, wl)
    rb, rs = oracle.workload_bounds(wl)
    err, _ = bounds_error(b, rb, wl.dim, stencil_momentum_scale(wl))
    assert err <= TOL, f"bounds error {err:.3e}"
    assert np.array_equal(s, rs)
    scale = element_value_scale(wl, wl.target)

    def both(f):
        t0 = wl.target
        wl.target = t0 * f
        try:
            g = run_gpu(kbl, wl, bounds_override=rb * f)
            r = oracle.workload_limit(wl, rb * f)
        finally:
            wl.target = t0
        return g[2] / f, g[4], r[0] / f, r[2]

    lim, ls, rl, rls = both(1.0)
    assert np.array_equal(ls, rls)
    spread = np.zeros_like(rl)
    for f in (3.0, 0.7, 1.3):
        g, _, r, _ = both(f)
        spread = np.maximum(spread, np.maximum(np.abs(g - lim), np.abs(r - rl)))
    _, e = limited_error(lim, rl, scale, wl.n_s)
    _, sp = limited_error(spread + rl, rl, scale, wl.n_s)
    assert np.all(e <= np.maximum(TOL, 4.0 * sp)), f"limited error {e.max():.3e}"
    print(f"[parity] quad_big: bounds err {err:.2e}, limited err {e.max():.2e} "
          f"(spread {sp.max():.2e}), p-steps {((rls & 0x10) > 0).sum()}/{wl.n_elem}", flush=True)


def test_single_element_stencils(kbl):
    wl = synth.make_quad_workload(N=6, seed=12, grid_nodes=40, name="quad_self")
    wl.rowptr = np.arange(wl.n_elem + 1, dtype=np.int32)
    wl.cols = np.arange(wl.n_elem, dtype=np.int32)
    check_workload(kbl, wl)


def test_determinism(kbl):
    wl = synth.make_quad_workload(N=16, seed=21, grid_nodes=48, name="quad_det")
    a = run_gpu(kbl, wl)
    b = run_gpu(kbl, wl)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


def test_limit_in_place(kbl):
    wl = synth.make_quad_workload(N=8, seed=31, grid_nodes=24, name="quad_inplace")
    dev = torch.device("cuda:0")
    st = torch.from_numpy(wl.states).to(dev)
    rp = torch.from_numpy(wl.rowptr).to(dev)
    cl = torch.from_numpy(wl.cols).to(dev)
    vg = kbl.make_vgrid(GRID_STENCIL, (24, 24), k=4.0)
    prm = kbl.make_params(wl.gamma)
    b, _ = kbl.compute_bounds(st, rp, cl, 16, vg, prm)
    sol = torch.from_numpy(wl.target).to(dev)
    ref, _, _ = kbl.limit(sol, b, wl.node_weights, 16, prm)
    kbl.limit(sol, b, wl.node_weights, 16, prm, out=sol)
    torch.cuda.synchronize()
    assert torch.equal(sol, ref)


def _pressure_cases(wl, rng):
    """Targets that make the pressure step of Sec. 3.8 fire.  In some elements
    the energy of a few nodes is pushed below their kinetic energy (P < 0 at
    those nodes, P(mean) > 0: alpha_P of eq. doublelimit blends them back to
    P = p_floor); in others every node moves with one velocity and carries
    no internal energy, so P(mean) = 0 <= p_floor and alpha_P = 0 flattens the
    element to its mean."""
    d, n_s = wl.dim, wl.n_s
    tg = wl.target.copy()
    E = d + 1
    el = rng.permutation(wl.n_elem)
    low, flat = el[: wl.n_elem // 6], el[wl.n_elem // 6: wl.n_elem // 6 + max(2, wl.n_elem // 20)]
    for e in low:
        for j in rng.choice(n_s, 2, replace=False):
            i = e * n_s + j
            ke = 0.5 * sum(tg[1 + k, i] ** 2 for k in range(d)) / tg[0, i]
            tg[E, i] = 0.3 * ke
    for e in flat:
        i = e * n_s + np.arange(n_s)
        U = tg[1:1 + d, i].sum(1) / tg[0, i].sum()
        tg[1:1 + d, i] = tg[0, i][None, :] * U[:, None]
        tg[E, i] = 0.5 * tg[0, i] * float((U ** 2).sum())
    wl.target = tg
    return wl


@pytest.mark.parametrize("case", ["line", "quad", "tri"])
def test_pressure_step_and_flattening_fire(kbl, case):
    """Both branches of the pressure step (Sec. 3.8 eq. pmin, eq. doublelimit)
    are taken, with the oracle's status bit for bit and the limited nodes at
    the FP64 tolerance."""
    rng = np.random.default_rng(900)
    if case == "line":
        wl = synth.make_line_workload(n_elem=48, seed=901, r_fac=0.9, name="line_pstep")
    elif case == "quad":
        wl = synth.make_quad_workload(N=8, seed=902, grid_nodes=24, r_fac=0.9, name="quad_pstep")
    else:
        wl = synth.make_tri_workload(N=6, seed=903, grid_nodes=24, outer=(0.5, 0.3), r_fac=0.9,
                                     name="tri_pstep")
    wl = _pressure_cases(wl, rng)
    _, _, ls, rls = check_workload(kbl, wl)
    assert np.array_equal(ls, rls)
    assert ((rls & kbl.ST_PSTEP) != 0).sum() >= 3
    assert ((rls & kbl.ST_PMEAN_FLOOR) != 0).sum() >= 2
    # a P-step element with alpha_P > 0 exists next to the flattened ones
    assert (((rls & kbl.ST_PSTEP) != 0) & ((rls & kbl.ST_PMEAN_FLOOR) == 0)).any()


def test_limiter_alone_on_oracle_bounds(kbl):
    """Same bounds on both sides isolate the limiter kernel."""
    wl = synth.make_quad_workload(N=32, seed=41, grid_nodes=32, name="quad_lim")
    rb, _ = oracle.workload_bounds(wl)
    _, _, lim, al, ls = run_gpu(kbl, wl, bounds_override=rb)
    rl, ral, rls = oracle.workload_limit(wl, rb)
    scale = element_value_scale(wl, wl.target)
    lerr, _ = limited_error(lim, rl, scale, wl.n_s)
    assert lerr <= TOL
    assert np.array_equal(ls, rls)


# every FP64 2D tile configuration (forced through the tuning knob), each on a
# ragged grid that leaves some of its threads' nodes outside the grid
from paper_2407_20966_amd._lib import FP64_TILES  # noqa: E402

FP64_TILE_EXTENTS = {t: (bx * tx, by * ty) for t, (bx, by, tx, ty, _) in FP64_TILES.items()}


@pytest.mark.parametrize("tile", sorted(FP64_TILE_EXTENTS))
def test_every_fp64_tile(kbl, monkeypatch, tile):
    mx, my = FP64_TILE_EXTENTS[tile]
    n = (mx - 3, my - 2)
    wl = synth.make_quad_workload(N=6, seed=300 + tile, grid_nodes=n[0], name=f"quad_tile{tile}")
    wl.grid = GridSpec(GRID_STENCIL, n, k=4.0)
    monkeypatch.setenv("KBL_BOUNDS_TILE", str(tile))
    check_workload(kbl, wl)
