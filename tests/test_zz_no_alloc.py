"""kbl_bounds_limit_backward_noalloc (the backward on the library's static
device array, for callers that cannot allocate) against
kbl_bounds_limit_backward with a caller workspace, through the C-ABI: two
calls in a row, the second on a smaller input, each bit for bit equal to the
workspace call (same kernels, deterministic), and the size limit."""

import ctypes as C

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kbl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2407_20966_amd as kbl
    return kbl


def _inputs(kbl, wl, seed):
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[: wl.dim], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    G = np.random.default_rng(seed).standard_normal(wl.target.shape)
    return t(wl.states), t(wl.rowptr), t(wl.cols), t(wl.target), t(G), vg, prm


def noalloc_backward(kbl, wl, st, rp, cl, tg, G, vg, prm):
    from paper_2407_20966_amd import _lib as L
    p = lambda x: C.c_void_p(x.data_ptr())
    n_elem = rp.numel() - 1
    gst = torch.empty_like(st)
    gsol = torch.empty_like(st)
    gb = torch.empty((2 * (wl.dim + 2), n_elem), dtype=torch.float64, device=st.device)
    status = torch.empty(n_elem, dtype=torch.int32, device=st.device)
    w = np.ascontiguousarray(wl.node_weights, dtype=np.float64)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.lib().kbl_bounds_limit_backward_noalloc(
        C.byref(prm), wl.dim, n_elem, wl.n_s, cl.numel(), p(st), p(rp), p(cl), C.byref(vg),
        None, None, p(tg), w.ctypes.data_as(C.c_void_p), p(G), p(gst), p(gsol), p(gb),
        p(status), stream)
    assert rc == L.KBL_OK, rc
    return gst, gsol, gb, status


@pytest.mark.parametrize("fwd", [False, True])
def test_matches_the_workspace_call_twice(kbl, fwd):
    """A larger input, then a smaller one on the same array (it keeps the
    first call's contents); each result equals the workspace call's."""
    for N, n, seed in ((24, 48, 11), (6, 32, 12)):
        wl = synth.make_quad_workload(N=N, seed=seed, grid_nodes=n, name=f"na{N}")
        wl.target = wl.states + 10.0 * (wl.target - wl.states)
        print(f"[noalloc] quad N={N} grid {n}", flush=True)
        st, rp, cl, tg, G, vg, prm = _inputs(kbl, wl, seed)
        ref = kbl.bounds_limit_backward(st, rp, cl, wl.n_s, vg, prm, tg, wl.node_weights, G)
        got = noalloc_backward(kbl, wl, st, rp, cl, tg, G, vg, prm)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        if fwd:
            # and the forward entry points still agree afterwards
            b2, _ = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
            torch.cuda.synchronize()
            assert torch.isfinite(b2).all()


def test_rejects_sizes_beyond_the_array(kbl):
    from paper_2407_20966_amd import _lib as L
    wl = synth.make_quad_workload(N=4, seed=13, grid_nodes=16, name="na_big")
    st, rp, cl, tg, G, vg, prm = _inputs(kbl, wl, 13)
    fake = C.c_void_p(st.data_ptr())
    n_elem, nnz = 1 << 20, 5 << 20          # 2.7 GB of gradient slots
    assert L.lib().kbl_backward_workspace_bytes(2, n_elem, 16, nnz) > L.NOALLOC_WORKSPACE_BYTES
    rc = L.lib().kbl_bounds_limit_backward_noalloc(
        C.byref(prm), 2, n_elem, 16, nnz, fake, fake, fake, C.byref(vg), None, None, fake,
        np.ones(16).ctypes.data_as(C.c_void_p), fake, fake, fake, fake, fake, None)
    assert rc == L.KBL_ERR_WORKSPACE
