"""Mixed-precision bounds (FP32 envelopes; BF16/FP16 MFMA or FP32 VALU
contraction) against the FP64 oracle and the FP64 GPU path.

Tolerance: 1e-5 relative (density/energy against |ref|, momentum against
the element momentum scale), and every bound must keep rho_min > 0 and
E_min > 0.  Per-variable errors are printed for the record.
"""

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import GRID_GLOBAL, GRID_STENCIL, GridSpec, quad_block_stencils
from tests._parity import bounds_error, element_value_scale, limited_error, stencil_momentum_scale

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
PRECS = {"fp32": 3, "fp16": 2, "bf16": 1}


@pytest.fixture(scope="module")
def kbl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2407_20966_amd as kbl
    return kbl


def gpu_bounds(kbl, wl, precision):
    dev = torch.device("cuda:0")
    st = torch.from_numpy(wl.states).to(dev)
    rp = torch.from_numpy(wl.rowptr).to(dev)
    cl = torch.from_numpy(wl.cols).to(dev)
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[: wl.dim], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac, precision=precision)
    b, s = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
    torch.cuda.synchronize()
    return b.cpu().numpy(), s.cpu().numpy().view(np.uint32)


def per_variable(err, dim):
    nv = dim + 2
    names = ["rho"] + [f"m{j}" for j in range(dim)] + ["E"]
    out = {}
    for v in range(nv):
        out[names[v]] = float(max(err[v].max(), err[nv + v].max())) if err.size else 0.0
    return out


def check(kbl, wl, prec, elems=None):
    b, s = gpu_bounds(kbl, wl, PRECS[prec])
    sel = np.arange(wl.n_elem) if elems is None else elems
    rb, rs = oracle.workload_bounds(wl, elems=elems)
    mscale = stencil_momentum_scale(wl, sel)
    err, emat = bounds_error(b[:, sel], rb, wl.dim, mscale)
    pv = per_variable(emat, wl.dim)
    print(f"[mixed] {wl.name} {prec}: max err {err:.2e} per variable "
          + ", ".join(f"{k} {v:.1e}" for k, v in pv.items()), flush=True)
    assert err <= TOL, f"{prec} bounds error {err:.3e}"
    assert np.array_equal(s[sel] & ~np.uint32(0x2), rs & ~np.uint32(0x2))
    good = ~np.isnan(b).any(0)
    assert np.all(b[0, good] > 0)
    # the energy lower bound is positive wherever the oracle's is (it is 0
    # where the lower envelope underflows over the whole box)
    epos = good.copy()
    epos[sel] &= rb[wl.dim + 1] > 0
    if elems is not None:
        epos[np.setdiff1d(np.arange(wl.n_elem), sel)] = False
    assert np.all(b[wl.dim + 1, epos] > 0)
    return b


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("n", [(16, 16), (13, 29), (32, 32), (48, 48), (40, 64), (64, 64)])
def test_mixed_small_stencil_box(kbl, prec, n):
    wl = synth.make_quad_workload(N=8, seed=200 + n[0] + n[1], grid_nodes=n[0], name=f"mq_{n}")
    wl.grid = GridSpec(GRID_STENCIL, n, k=4.0)
    check(kbl, wl, prec)


# every mixed tile configuration (forced through the tuning knob) in every
# form, each on a ragged grid that leaves some of its lanes' nodes outside
from paper_2407_20966_amd._lib import MIXED_TILES  # noqa: E402

MIXED_TILE_EXTENTS = {t: (16 * txw * nw, 16 * ks) for t, (txw, ks, nw) in MIXED_TILES.items()}


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("tile", sorted(MIXED_TILE_EXTENTS))
def test_every_mixed_tile(kbl, monkeypatch, tile, prec):
    mx, my = MIXED_TILE_EXTENTS[tile]
    n = (mx - 3, my - 2)
    wl = synth.make_quad_workload(N=6, seed=400 + tile, grid_nodes=n[0], name=f"mq_tile{tile}")
    wl.grid = GridSpec(GRID_STENCIL, n, k=4.0)
    monkeypatch.setenv("KBL_MIXED_TILE", str(tile))
    check(kbl, wl, prec)


@pytest.mark.parametrize("prec", list(PRECS))
def test_mixed_global_box(kbl, prec):
    wl = synth.make_quad_workload(N=12, seed=78, field_kind="sine", grid_nodes=64,
                                  grid_mode=GRID_GLOBAL, name="mq_sine_global")
    check(kbl, wl, prec)


@pytest.mark.parametrize("prec", list(PRECS))
def test_mixed_quad1024_sine_sampled(kbl, prec):
    wl = synth.make_workload("quad1024_sine")
    check(kbl, wl, prec, elems=synth.sample_elements(wl, 96))


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_mixed_quad256_sampled(kbl, prec):
    wl = synth.make_workload("quad256")
    check(kbl, wl, prec, elems=synth.sample_elements(wl, 192))


@pytest.mark.parametrize("prec", list(PRECS))
def test_mixed_extreme_temperature_ratio(kbl, prec):
    """Every fifth element at rest with theta = 1e-12 among states at theta
    ~ 1: the cold states set the log-peak reference ~27 above the others, so
    the envelopes at the nodes sit ~1e-12 below it.  The kernel must
    rescale before the FP16/BF16 splits of the y stage (which resolve ~2^-38
    of their largest value) or those bounds come out 0."""
    wl = synth.make_quad_workload(N=8, seed=96, grid_nodes=32, name="mq_cold")
    st = wl.states.copy()
    cold = np.arange(wl.n_elem)[::5]
    nodes = (cold[:, None] * wl.n_s + np.arange(wl.n_s)[None, :]).ravel()
    st[1:3, nodes] = 0.0
    st[3, nodes] = 1e-12 * st[0, nodes] / (wl.gamma - 1.0)
    wl.states = st
    check(kbl, wl, prec)


def test_mixed_tri2m_sampled(kbl):
    wl = synth.make_workload("tri2m")
    check(kbl, wl, "fp16", elems=synth.sample_elements(wl, 160))


@pytest.mark.parametrize("name", ["quad256", "quad1024_sine"])
def test_mixed_full_vs_fp64_gpu(kbl, name):
    """All elements: mixed vs the FP64 GPU path (itself 1e-12 of the oracle)."""
    wl = synth.make_workload(name)
    b64, _ = gpu_bounds(kbl, wl, 0)
    mscale = stencil_momentum_scale(wl)
    for prec in PRECS:
        b, _ = gpu_bounds(kbl, wl, PRECS[prec])
        err, emat = bounds_error(b, b64, 2, mscale)
        pv = per_variable(emat, 2)
        print(f"[mixed-full] {name} {prec}: max err {err:.2e} per variable "
              + ", ".join(f"{k} {v:.1e}" for k, v in pv.items()), flush=True)
        assert err <= TOL
        assert np.all(b[0] > 0) and np.all(b[3] > 0)


def test_mixed_limiter_end_to_end(kbl):
    """Bounds from the mixed path feed the FP64 limiter: the limited nodes must
    lie in those bounds (mean inside) and keep the element mean.  The difference
    to the FP64 chain is reported only: alpha = |(b - mean)/(max w - mean)| is
    ill-conditioned where a bound sits next to the mean."""
    wl = synth.make_quad_workload(N=32, seed=55, grid_nodes=48, name="mq_lim")
    dev = torch.device("cuda:0")
    tg = torch.from_numpy(wl.target).to(dev)
    prm = kbl.make_params(wl.gamma)
    out = {}
    for prec in (0, 3, 2, 1):
        b, _ = gpu_bounds(kbl, wl, prec)
        lim, al, st = kbl.limit(tg, torch.from_numpy(b).to(dev), wl.node_weights, wl.n_s, prm)
        torch.cuda.synchronize()
        out[prec] = (b, lim.cpu().numpy(), st.cpu().numpy().view(np.uint32))
    nv, n_s = 4, wl.n_s
    c = wl.node_weights / wl.node_weights.sum()
    for prec in (3, 2, 1):
        b, lim, st = out[prec]
        L = lim.reshape(nv, wl.n_elem, n_s)
        T = wl.target.reshape(nv, wl.n_elem, n_s)
        np.testing.assert_allclose((L * c).sum(2), (T * c).sum(2), rtol=1e-12, atol=1e-12)
        ok = (st & 0x50) == 0          # no pressure step, mean inside the bounds
        scale = np.abs(T).max(2)
        tol = 1e-12 * (scale + 1)
        assert np.all((L.min(2) >= b[:nv] - tol)[:, ok]) and np.all((L.max(2) <= b[nv:] + tol)[:, ok])
        lerr, _ = limited_error(lim, out[0][1], element_value_scale(wl, wl.target), n_s)
        print(f"[mixed] limited nodes, precision {prec} bounds vs FP64 bounds: {lerr:.2e} "
              f"(elements checked for feasibility: {ok.sum()}/{wl.n_elem})", flush=True)


_WL_CACHE = {}


def _workload(name):
    if name not in _WL_CACHE:
        _WL_CACHE.clear()            # keep one large workload alive at a time
        _WL_CACHE[name] = synth.make_workload(name)
    return _WL_CACHE[name]


# limiter decisions that switch discontinuously (Sec. 3.4 epsilon rule,
# Sec. 3.8 pressure step and alpha_P = 0): an element whose bounds sit within
# the mixed tolerance of such a threshold may take the other branch
BRANCH_BITS = np.uint32(0x4 | 0x10 | 0x20)


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("name,n_sample", [("quad256", 160), ("quad1024_sine", 96),
                                           ("tri2m", 128)])
def test_mixed_limited_vs_oracle(kbl, name, n_sample, prec):
    """End to end: mixed bounds -> FP64 limiter on the GPU against oracle
    bounds -> oracle limiter (eq. alpha, eq. limiter, eq. pmin, eq. doublelimit),
    node by node on a seeded element sample, at the mixed tolerance 1e-5
    relative to the element's value scale."""
    wl = _workload(name)
    sel = synth.sample_elements(wl, n_sample)
    b, _ = gpu_bounds(kbl, wl, PRECS[prec])
    dev = torch.device("cuda:0")
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    lim, al, ls = kbl.limit(torch.from_numpy(wl.target).to(dev), torch.from_numpy(b).to(dev),
                            wl.node_weights, wl.n_s, prm)
    torch.cuda.synchronize()
    lim, ls = lim.cpu().numpy(), ls.cpu().numpy().view(np.uint32)[sel]
    rb, _ = oracle.workload_bounds(wl, elems=sel)
    rl, ral, rls = oracle.workload_limit(wl, rb, elems=sel)
    nodes = (sel[:, None] * wl.n_s + np.arange(wl.n_s)[None, :]).ravel()
    scale = element_value_scale(wl, wl.target, sel)
    _, err = limited_error(lim[:, nodes], rl, scale, wl.n_s)
    ties = ((ls ^ rls) & BRANCH_BITS) != 0
    worst = float(err[:, ~ties].max()) if (~ties).any() else 0.0
    print(f"[mixed-limited] {name} {prec}: max err {worst:.2e} over {len(sel)} elements "
          f"({int((ral[0] < 1).sum())} limited, {int(((rls & 0x10) != 0).sum())} p-steps), "
          f"{int(ties.sum())} branch ties", flush=True)
    assert ties.sum() <= max(1, len(sel) // 100)
    assert worst <= TOL


def test_mixed_determinism(kbl):
    wl = synth.make_quad_workload(N=16, seed=23, grid_nodes=64, name="mq_det")
    for prec in PRECS.values():
        a, _ = gpu_bounds(kbl, wl, prec)
        b, _ = gpu_bounds(kbl, wl, prec)
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_mixed_stencils_beyond_256_states_are_flagged(kbl):
    """The mixed kernel keeps at most 256 stencil states in LDS: larger
    stencils get KBL_ST_TOO_LARGE and NaN bounds (the FP64 path computes
    them), smaller ones in the same launch are unaffected."""
    wl = synth.make_quad_workload(N=6, seed=14, grid_nodes=24, name="mq_big")
    rp_big, cl_big = quad_block_stencils(6, 2)
    # every other element keeps its 5-element face stencil (80 states)
    rows = []
    for e in range(wl.n_elem):
        src = (wl.rowptr, wl.cols) if e % 2 else (rp_big, cl_big)
        rows.append(src[1][src[0][e]:src[0][e + 1]])
    wl.rowptr = np.concatenate([[0], np.cumsum([len(x) for x in rows])]).astype(np.int32)
    wl.cols = np.concatenate(rows).astype(np.int32)
    big = np.arange(wl.n_elem) % 2 == 0
    for prec in (kbl.PREC_MIXED_FP32, kbl.PREC_MIXED_FP16, kbl.PREC_MIXED_BF16):
        b, s = gpu_bounds(kbl, wl, prec)
        assert np.all(s[big] & kbl.ST_TOO_LARGE) and np.isnan(b[:, big]).all()
        assert not (s[~big] & kbl.ST_TOO_LARGE).any() and np.isfinite(b[:, ~big]).all()
        rb, _ = oracle.workload_bounds(wl, elems=np.nonzero(~big)[0])
        sel = np.nonzero(~big)[0]
        err, _ = bounds_error(b[:, sel], rb, 2, stencil_momentum_scale(wl, sel))
        assert err <= 1e-5, err
