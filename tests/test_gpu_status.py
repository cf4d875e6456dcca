"""kbl_status_summary: per-bit counts of status words, reduced on the device,
against NumPy counts of the same words (exact integers), and against the
oracle's per-element status of Sec. 3.4 / 3.8 conditions on a small mesh."""

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


def np_counts(words):
    w = np.asarray(words, dtype=np.uint32)
    return np.array([int(((w >> b) & 1).sum()) for b in range(32)], dtype=np.int64)


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000, 1 << 20, (1 << 20) + 3])
def test_random_words(kbl, n):
    rng = np.random.default_rng(n)
    w = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    st = torch.from_numpy(w.view(np.int32)).to("cuda:0")
    out = kbl.status_summary(st)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np_counts(w))


def test_repeated_calls_overwrite(kbl):
    w = np.full(5000, 0x11, dtype=np.uint32)
    st = torch.from_numpy(w.view(np.int32)).to("cuda:0")
    out = torch.full((32,), 7, dtype=torch.int64, device="cuda:0")
    kbl.status_summary(st, out=out)
    kbl.status_summary(st[:100], out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np_counts(w[:100]))


def test_against_oracle_status(kbl):
    """Bounds and limiter status of a small mesh where the pressure step and
    alpha_P = 0 both occur: GPU counts equal the oracle's counts."""
    from tests.test_gpu_parity import _pressure_cases
    wl = synth.make_quad_workload(N=8, seed=902, grid_nodes=24, r_fac=0.9, name="st_quad")
    wl = _pressure_cases(wl, np.random.default_rng(900))
    dev = torch.device("cuda:0")
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[:2], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    b, bs = kbl.compute_bounds(torch.from_numpy(wl.states).to(dev),
                               torch.from_numpy(wl.rowptr).to(dev),
                               torch.from_numpy(wl.cols).to(dev), wl.n_s, vg, prm)
    _, _, ls = kbl.limit(torch.from_numpy(wl.target).to(dev), b, wl.node_weights, wl.n_s, prm)
    cb = kbl.status_summary(bs)
    cl = kbl.status_summary(ls)
    torch.cuda.synchronize()
    rb, rbs = oracle.workload_bounds(wl)
    _, _, rls = oracle.workload_limit(wl, rb)
    assert np.array_equal(cb.cpu().numpy(), np_counts(rbs))
    assert np.array_equal(cl.cpu().numpy(), np_counts(rls))
    assert cl[4].item() >= 3 and cl[5].item() >= 2        # KBL_ST_PSTEP, KBL_ST_PMEAN_FLOOR


def test_tri2m_limiter_status(kbl):
    """The 2M-triangle workload: device counts of the full bounds and limiter
    status equal NumPy's counts of the same arrays."""
    wl = synth.make_workload("tri2m")
    dev = torch.device("cuda:0")
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[:2], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    b, bs = kbl.compute_bounds(torch.from_numpy(wl.states).to(dev),
                               torch.from_numpy(wl.rowptr).to(dev),
                               torch.from_numpy(wl.cols).to(dev), wl.n_s, vg, prm)
    _, _, ls = kbl.limit(torch.from_numpy(wl.target).to(dev), b, wl.node_weights, wl.n_s, prm)
    cb = kbl.status_summary(bs)
    cl = kbl.status_summary(ls)
    torch.cuda.synchronize()
    got_b, got_l = cb.cpu().numpy(), cl.cpu().numpy()
    assert np.array_equal(got_b, np_counts(bs.cpu().numpy().view(np.uint32)))
    assert np.array_equal(got_l, np_counts(ls.cpu().numpy().view(np.uint32)))
    print(f"[status] tri2m: limited {got_l[3]}, eps rule {got_l[2]}, p-steps {got_l[4]}, "
          f"rho floor {got_b[1]}", flush=True)
