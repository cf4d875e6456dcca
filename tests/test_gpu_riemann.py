"""GPU Riemann-averaged states (Thm. 4.3) vs the oracle: the averaged states
to 1e-13 relative (momentum against the pair's momentum scale), and the
bounds check bit-exact except for states within 1e-12 of a bound."""

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kbl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2407_20966_amd as kbl
    return kbl


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def compare(kbl, dim, gamma, states, ni, nj, normals, lam=None, bounds=None, elem=None):
    prm = kbl.make_params(gamma)
    bar, st = kbl.riemann_states(dev(states), dev(ni), dev(nj), dev(normals), prm,
                                 lam=None if lam is None else dev(lam),
                                 bounds=None if bounds is None else dev(bounds),
                                 elem=None if elem is None else dev(elem))
    torch.cuda.synchronize()
    bar = bar.cpu().numpy()
    st = st.cpu().numpy().view(np.uint32)
    rbar, rst = oracle.riemann(dim, gamma, states, ni, nj, normals, lam, bounds, elem)
    assert np.array_equal(np.isnan(bar), np.isnan(rbar))
    ok = ~np.isnan(rbar).any(0)
    wi = states[:, np.clip(ni, 0, states.shape[1] - 1)]
    wj = states[:, np.clip(nj, 0, states.shape[1] - 1)]
    scale = np.maximum(np.abs(wi), np.abs(wj))
    mom = np.sqrt(np.abs(wi[0] * wi[-1])) + np.sqrt(np.abs(wj[0] * wj[-1]))
    scale[1:1 + dim] = np.maximum(scale[1:1 + dim], mom)
    err = (np.abs(bar - rbar) / scale)[:, ok].max() if ok.any() else 0.0
    diff = st != rst
    if diff.any() and bounds is not None:
        # only where the state sits on a bound
        e = elem[diff]
        near = np.zeros(diff.sum(), bool)
        for v in range(dim + 2):
            for row in (v, dim + 2 + v):
                near |= np.abs(rbar[v, diff] - bounds[row, e]) <= 1e-12 * scale[v, diff]
        assert near.all(), f"status differs away from the bounds at {np.nonzero(diff)[0][:8]}"
    return err, rst


def fr_pairs(wl):
    P = wl.meta["face_pairs"]
    return P["ni"], P["nj"], P["normals"], P["elem"]


def test_fr_face_pairs_with_bounds(kbl):
    wl = synth.make_quad_fr_workload(N=8, seed=100, grid_nodes=32, name="rs_fr")
    g = wl.grid
    b, _ = oracle.bounds(2, wl.gamma, wl.states, wl.rowptr, wl.cols, 1, g.mode, g.n[:2], g.lo,
                         g.hi, g.k, wl.r_fac, n_src=wl.n_state_nodes)
    ni, nj, nrm, el = fr_pairs(wl)
    err, st = compare(kbl, 2, wl.gamma, wl.states, ni, nj, nrm, bounds=b, elem=el)
    print(f"[riemann] fr8 (wavespeed estimate): err {err:.2e}, {int((st > 0).sum())}/{st.size} "
          f"outside", flush=True)
    assert err <= 1e-13
    lam = np.full(ni.size, 25.0)
    err2, _ = compare(kbl, 2, wl.gamma, wl.states, ni, nj, nrm, lam=lam, bounds=b, elem=el)
    assert err2 <= 1e-13


def test_fr_full_size_all_pairs(kbl):
    wl = synth.make_workload("quad256_fr")
    ni, nj, nrm, el = fr_pairs(wl)
    err, st = compare(kbl, 2, wl.gamma, wl.states, ni, nj, nrm)
    print(f"[riemann] quad256_fr: {ni.size} pairs, err {err:.2e}", flush=True)
    assert err <= 1e-13


def test_line_pairs_and_bad_inputs(kbl):
    wl = synth.make_line_workload(n_elem=16, seed=101, name="rs_line")
    n = wl.n_nodes
    ni = np.arange(n - 1, dtype=np.int32)
    nj = ni + 1
    nrm = np.ones((1, n - 1))
    states = wl.states.copy()
    states[0, 7] = -1.0                        # inadmissible node
    ni[3] = n + 5                              # out of range id
    err, st = compare(kbl, 1, wl.gamma, states, ni, nj, nrm)
    assert err <= 1e-13
    assert st[3] & kbl.RS_BAD_INPUT and st[6] & kbl.RS_BAD_INPUT and st[7] & kbl.RS_BAD_INPUT
    assert not (st[[0, 1, 2, 4, 5, 8]] & kbl.RS_BAD_INPUT).any()


def test_empty(kbl):
    z = torch.zeros((4, 3), dtype=torch.float64, device="cuda:0")
    e = torch.zeros(0, dtype=torch.int32, device="cuda:0")
    bar, st = kbl.riemann_states(z, e, e, torch.zeros((2, 0), dtype=torch.float64, device="cuda:0"),
                                 kbl.make_params(1.4))
    torch.cuda.synchronize()
    assert bar.shape == (4, 0)
