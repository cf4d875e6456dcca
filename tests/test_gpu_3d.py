"""GPU (HIP, FP64) vs the FP64 oracle for d = 3 velocity grids, through the
C-ABI: bounds, limiter and Riemann-averaged states on hexahedral stencils.

Tolerance as for d <= 2: 1e-12 relative (density and energy against |ref|,
momentum against the element momentum scale), limited nodes 1e-11 of the
element value scale.  Cases: every 3D tile configuration with ragged x, y
and z (slab) extents, global and per-stencil boxes, delta = 0 (gamma = 5/3),
strict bounds, stencils of more than 256 states (several state chunks per
slab), inadmissible states and bad rows, node-level stencils, and the
full-size 32^3-element workload on a seeded element sample in the launch
configuration the benchmark uses.
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


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def run_gpu(kbl, wl, r_fac=None, independent=False, autotune=False):
    st, rp, cl, tg = dev(wl.states), dev(wl.rowptr), dev(wl.cols), dev(wl.target)
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[:3], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac if r_fac is None else r_fac,
                          independent_alpha=independent)
    if autotune:
        kbl.autotune_bounds(st, rp, cl, wl.n_s, vg, prm)
    b, s = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
    lim, al, ls = kbl.limit(tg, b, wl.node_weights, wl.n_s, prm)
    torch.cuda.synchronize()
    return b.cpu().numpy(), u32(s), lim.cpu().numpy(), al.cpu().numpy(), u32(ls)


def check(kbl, wl, elems=None, r_fac=None, independent=False, autotune=False, tol=TOL):
    print(f"[3d] {wl.name} n_elem={wl.n_elem} grid={tuple(wl.grid.n[:3])} mode={wl.grid.mode} "
          f"gamma={wl.gamma} sample={None if elems is None else len(elems)}", flush=True)
    b, s, lim, al, ls = run_gpu(kbl, wl, r_fac, independent, autotune)
    rb, rs = oracle.workload_bounds(wl, elems=elems, r_fac=r_fac)
    sel = np.arange(wl.n_elem) if elems is None else elems
    err, _ = bounds_error(b[:, sel], rb, 3, stencil_momentum_scale(wl, sel))
    assert err <= tol, f"bounds error {err:.3e}"
    assert np.array_equal(s[sel], rs), "bounds status differs"
    ok = ~np.isnan(rb).any(0)
    if ok.any():
        rl, ral, rls = oracle.workload_limit(wl, rb, elems=elems, independent=independent)
        nodes = (sel[:, None] * wl.n_s + np.arange(wl.n_s)[None, :]).ravel()
        scale = element_value_scale(wl, wl.target, sel)
        lerr, _ = limited_error(lim[:, nodes], rl, scale, wl.n_s)
        assert lerr <= tol, f"limited error {lerr:.3e}"
        diff = ls[sel] != rls
        if diff.any():
            near = np.abs(ral[0] - 1.0) < 1e-9
            assert np.all(near[diff]), f"limiter status differs at {np.nonzero(diff)[0][:10]}"
    else:
        lerr = 0.0
    print(f"[3d] {wl.name}: bounds err {err:.2e}, limited err {lerr:.2e}", flush=True)
    return b, s


def hex_wl(N, n, seed, mode=GRID_STENCIL, gamma=1.4, name="hex"):
    wl = synth.make_hex_workload(N=N, seed=seed, grid_nodes=n[0], gamma=gamma, name=name)
    if mode == GRID_STENCIL:
        wl.grid = GridSpec(GRID_STENCIL, tuple(n), k=4.0)
    else:
        # one box for all elements: the extremes of U -+ 4 sqrt(theta)
        d = 3
        rho = wl.states[0]
        U = wl.states[1:1 + d] / rho
        P = (gamma - 1) * (wl.states[d + 1] - 0.5 * (wl.states[1:1 + d] ** 2).sum(0) / rho)
        sd = np.sqrt(P / rho)
        lo = tuple(float((U[j] - 4 * sd).min()) for j in range(d))
        hi = tuple(float((U[j] + 4 * sd).max()) for j in range(d))
        wl.grid = GridSpec(GRID_GLOBAL, tuple(n), lo=lo, hi=hi)
    return wl


def test_hex_small_full(kbl):
    check(kbl, hex_wl(3, (12, 12, 12), seed=11))


TILE_EXTENTS = None


def _extents(kbl):
    from paper_2407_20966_amd import _lib as L
    return {t: (bx * tx, by * ty, bz * tz) for t, (bx, by, bz, tx, ty, tz) in L.FP64_TILES_3D.items()}


@pytest.mark.parametrize("tile", range(9))
def test_every_3d_tile(kbl, monkeypatch, tile):
    mx, my, slab = _extents(kbl)[tile]
    n = (mx - 3, my - 2, slab + 3)     # ragged x, y and a ragged last slab
    wl = hex_wl(2, n, seed=40 + tile, name=f"hex_tile{tile}")
    monkeypatch.setenv("KBL_BOUNDS_TILE", str(tile))
    check(kbl, wl)


def test_hex_global_box(kbl):
    check(kbl, hex_wl(3, (16, 14, 9), seed=12, mode=GRID_GLOBAL, name="hex_global"))


@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.2])
def test_hex_gamma(kbl, gamma):
    # gamma = 5/3: delta = 0 in 3D, no internal degrees of freedom (Sec. 3.6)
    check(kbl, hex_wl(2, (20, 20, 20), seed=13, gamma=gamma, name=f"hex_g{gamma:.3f}"))


def test_hex_extreme_temperature_ratio(kbl):
    """Every fifth element at rest with theta = 1e-12: the log-Maxwellian
    reaches about -1e13 in the cold states' tails (clamped exp, underflow
    to 0, rho_min floored), as in the oracle."""
    wl = hex_wl(2, (12, 12, 12), seed=16, name="hex_cold")
    st = wl.states.copy()
    cold = np.arange(wl.n_elem)[::5]
    nodes = (cold[:, None] * wl.n_s + np.arange(wl.n_s)[None, :]).ravel()
    st[1:4, nodes] = 0.0
    st[4, nodes] = 1e-12 * st[0, nodes] / (wl.gamma - 1.0)
    wl.states = st
    check(kbl, wl)


def test_hex_strict_bounds_and_independent_alpha(kbl):
    wl = hex_wl(3, (12, 12, 12), seed=14, name="hex_r0")
    check(kbl, wl, r_fac=0.0)
    check(kbl, wl, independent=True)


def test_hex_stencil_over_256_states(kbl):
    # 11 elements x 27 nodes = 297 states: two state chunks per slab, the
    # first restaged on every slab after the first
    wl = hex_wl(3, (12, 12, 13), seed=15, name="hex_big_stencil")
    rng = np.random.default_rng(15)
    rows = [np.concatenate([[e], rng.choice(np.delete(np.arange(wl.n_elem), e), 10, replace=False)])
            for e in range(wl.n_elem)]
    wl.rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    wl.cols = np.concatenate(rows).astype(np.int32)
    check(kbl, wl)


def test_hex_bad_inputs(kbl):
    wl = hex_wl(3, (12, 12, 12), seed=16, name="hex_bad")
    wl.states = wl.states.copy()
    wl.states[0, 5 * wl.n_s + 3] = -1.0                    # negative density in element 5
    wl.states[4, 9 * wl.n_s] = np.inf                      # non-finite energy in element 9
    wl.cols = wl.cols.copy()
    wl.cols[wl.rowptr[2] + 1] = wl.n_elem + 7              # element id out of range in row 2
    b, s = check(kbl, wl)
    assert (s[5] & 0x1) and (s[9] & 0x1) and (s[2] & 0x100)
    assert np.isnan(b[:, [2, 5, 9]]).all()


def test_hex32_full_size_sample(kbl):
    # the benchmark workload at full size (32^3 elements, 24^3 velocity nodes),
    # autotuned launch like the benchmark, compared on a seeded sample
    wl = synth.make_workload("hex32")
    elems = np.sort(np.random.default_rng(17).choice(wl.n_elem, 12, replace=False))
    elems = np.unique(np.concatenate([[0, wl.n_elem - 1], elems]))
    check(kbl, wl, elems=elems, autotune=True)


def test_hex_node_stencils(kbl):
    # node-level stencils: each row lists 60 random nodes (one state each)
    wl = hex_wl(3, (14, 14, 14), seed=18, name="hex_nodes")
    rng = np.random.default_rng(18)
    n_nodes = wl.states.shape[1]
    n_rows = 40
    rows = [rng.choice(n_nodes, 60, replace=False) for _ in range(n_rows)]
    rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    cols = np.concatenate(rows).astype(np.int32)
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[:3], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    b, s = kbl.compute_bounds_nodes(dev(wl.states), dev(rowptr), dev(cols), vg, prm)
    torch.cuda.synchronize()
    rb, rs = oracle.bounds(3, wl.gamma, wl.states, rowptr, cols, 1, g.mode, g.n[:3], g.lo, g.hi,
                           g.k, wl.r_fac, n_src=n_nodes)
    ms = node_stencil_momentum_scale(wl.states, rowptr, cols, 3, np.arange(n_rows))
    err, _ = bounds_error(b.cpu().numpy(), rb, 3, ms)
    print(f"[3d] node stencils: bounds err {err:.2e}", flush=True)
    assert err <= TOL
    assert np.array_equal(u32(s), rs)


def hex_face_pairs(wl, N):
    """Node pairs across the x, y and z faces of a periodic N^3 hex mesh
    (p = 2, nodes (jz*3 + jy)*3 + jx), normals pointing from i to j."""
    n1 = 3
    ni, nj, nrm, el = [], [], [], []
    for e in range(wl.n_elem):
        ez, rem = divmod(e, N * N)
        ey, ex = divmod(rem, N)
        nb = [((ez * N + ey) * N + (ex + 1) % N, 0), ((ez * N + (ey + 1) % N) * N + ex, 1),
              ((((ez + 1) % N) * N + ey) * N + ex, 2)]
        for f, axis in nb:
            for a in range(n1):
                for b in range(n1):
                    if axis == 0:
                        li, lj = (a * n1 + b) * n1 + 2, (a * n1 + b) * n1 + 0
                    elif axis == 1:
                        li, lj = (a * n1 + 2) * n1 + b, (a * n1 + 0) * n1 + b
                    else:
                        li, lj = (2 * n1 + a) * n1 + b, (0 * n1 + a) * n1 + b
                    ni.append(e * wl.n_s + li)
                    nj.append(f * wl.n_s + lj)
                    nv = [0.0, 0.0, 0.0]
                    nv[axis] = 1.0
                    nrm.append(nv)
                    el.append(e)
    return (np.array(ni, np.int32), np.array(nj, np.int32),
            np.ascontiguousarray(np.array(nrm).T), np.array(el, np.int32))


def test_hex_riemann_states(kbl):
    N = 3
    wl = hex_wl(N, (12, 12, 12), seed=19, name="hex_rs")
    b, _ = oracle.workload_bounds(wl)
    ni, nj, nrm, el = hex_face_pairs(wl, N)
    # a rotated frame as well: unit normals in general position
    rng = np.random.default_rng(19)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    for normals in (nrm, np.ascontiguousarray(q @ nrm)):
        prm = kbl.make_params(wl.gamma)
        bar, st = kbl.riemann_states(dev(wl.states), dev(ni), dev(nj), dev(normals), prm,
                                     bounds=dev(b), elem=dev(el))
        torch.cuda.synchronize()
        bar, st = bar.cpu().numpy(), u32(st)
        rbar, rst = oracle.riemann(3, wl.gamma, wl.states, ni, nj, normals, None, b, el)
        wi, wj = wl.states[:, ni], wl.states[:, nj]
        scale = np.maximum(np.abs(wi), np.abs(wj))
        mom = np.sqrt(np.abs(wi[0] * wi[-1])) + np.sqrt(np.abs(wj[0] * wj[-1]))
        scale[1:4] = np.maximum(scale[1:4], mom)
        err = (np.abs(bar - rbar) / scale).max()
        print(f"[3d] riemann: err {err:.2e}, {(rst > 0).sum()}/{rst.size} outside", flush=True)
        assert err <= 1e-13
        diff = st != rst
        if diff.any():
            e = el[diff]
            near = np.zeros(diff.sum(), bool)
            for v in range(5):
                for row in (v, 5 + v):
                    near |= np.abs(rbar[v, diff] - b[row, e]) <= 1e-12 * scale[v, diff]
            assert near.all()
