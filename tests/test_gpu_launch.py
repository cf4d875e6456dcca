"""Launch configurations of the bounds kernels: persistent grids and autotuning.

Every launch shape (one workgroup per element, several elements per
workgroup, persistent grids walking the elements in a grid stride) must give
bit-identical results to the default launch with the same tile; the
autotuned choice must stay within the FP64
parity tolerance of the oracle (and, for the mixed forms, within the mixed
tolerance), on uneven triangle stencils and on quads.
"""

import numpy as np
import pytest

import oracle
import synth
from tests._parity import bounds_error, stencil_momentum_scale

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kbl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2407_20966_amd as kbl
    yield kbl
    kbl._lib.lib().kbl_autotune_clear()


def dev_inputs(kbl, wl, precision=0):
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[: wl.dim], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac, precision=precision)
    return t(wl.states), t(wl.rowptr), t(wl.cols), vg, prm


def bounds(kbl, wl, precision=0):
    st, rp, cl, vg, prm = dev_inputs(kbl, wl, precision)
    b, s = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
    torch.cuda.synchronize()
    return b.cpu().numpy(), s.cpu().numpy()


@pytest.mark.parametrize("blocks", [1, 7, 300, 0, -3, -64, -100000])
@pytest.mark.parametrize("case", ["tri", "quad", "line"])
def test_persistent_grid_is_bit_identical(kbl, monkeypatch, case, blocks):
    if case == "tri":
        wl = synth.make_tri_workload(N=12, seed=61, grid_nodes=32, name="p_tri")
    elif case == "quad":
        wl = synth.make_quad_workload(N=20, seed=62, grid_nodes=40, name="p_quad")
    else:
        wl = synth.make_line_workload(n_elem=500, seed=63, name="p_line")
    print(f"[launch] {wl.name} persistent blocks={blocks}", flush=True)
    monkeypatch.delenv("KBL_PERSISTENT_BLOCKS", raising=False)
    ref = bounds(kbl, wl)
    monkeypatch.setenv("KBL_PERSISTENT_BLOCKS", str(blocks))
    got = bounds(kbl, wl)
    for x, y in zip(ref, got):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    if case == "quad":
        for prec in (kbl.PREC_MIXED_FP16, kbl.PREC_MIXED_FP32):
            monkeypatch.delenv("KBL_PERSISTENT_BLOCKS")
            ref = bounds(kbl, wl, prec)
            monkeypatch.setenv("KBL_PERSISTENT_BLOCKS", str(blocks))
            got = bounds(kbl, wl, prec)
            for x, y in zip(ref, got):
                assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (3, 1e-5), (2, 1e-5)])
def test_autotuned_choice_keeps_parity(kbl, precision, tol):
    wl = synth.make_tri_workload(N=24, seed=64, grid_nodes=48, name="t_tri")
    st, rp, cl, vg, prm = dev_inputs(kbl, wl, precision)
    idx = kbl.autotune_bounds(st, rp, cl, wl.n_s, vg, prm, sample_elems=1000)
    assert idx >= 0
    b, s = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
    torch.cuda.synchronize()
    rb, rs = oracle.workload_bounds(wl)
    err, _ = bounds_error(b.cpu().numpy(), rb, 2, stencil_momentum_scale(wl))
    print(f"[launch] autotune precision={precision}: candidate {idx}, bounds err {err:.2e}",
          flush=True)
    assert err <= tol
    mask = np.uint32(0xFFFFFFFF if precision == 0 else ~np.uint32(kbl.ST_RHO_FLOOR))
    assert np.array_equal(s.cpu().numpy().view(np.uint32) & mask, rs & mask)
    kbl._lib.lib().kbl_autotune_clear()
