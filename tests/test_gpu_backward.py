"""Hand-written backward (bounds + limiter) on the GPU.

- against the oracle's analytic subgradient on small inputs, per DoF: each
  entry relative to max(|ref|, 1e-3 of the largest |ref| of its element), at
  1e-12 or, where FP64 rounding alone moves the entry further, at 4 times
  the sum of how far rounding moves it on each side (measured through the
  scaling invariance of the gradient, see rounding_spread); in 1D/2D, global
  and per-stencil velocity boxes, triangles, stencils that list a neighbour
  twice;
- against central finite differences of the GPU forward on the 512x512 quad
  workload (200 seeded DoFs, h = 1e-7 max(1, |x|), J = sum w rho_limited with
  w ~ N(0, 1); J is summed over the elements a DoF can affect only, so the
  difference does not drown in the rounding of the full sum), tolerance 1e-6;
- autograd wiring, determinism, and the symmetric-stencil check.
"""

import numpy as np
import pytest

import oracle
import synth
from synth.workloads import GRID_GLOBAL, GRID_STENCIL, GridSpec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kbl():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2407_20966_amd as kbl
    return kbl


def dev_inputs(kbl, wl):
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g = wl.grid
    vg = kbl.make_vgrid(g.mode, g.n[: wl.dim], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    return t(wl.states), t(wl.target), t(wl.rowptr), t(wl.cols), vg, prm


def gpu_backward(kbl, wl, G):
    st, tg, rp, cl, vg, prm = dev_inputs(kbl, wl)
    gst, gsol, gb, s = kbl.bounds_limit_backward(st, rp, cl, wl.n_s, vg, prm, tg,
                                                 wl.node_weights,
                                                 torch.from_numpy(G).to(st.device))
    torch.cuda.synchronize()
    return gst.cpu().numpy(), gsol.cpu().numpy(), gb.cpu().numpy(), s.cpu().numpy().view(np.uint32)


def dof_scale(ref, n_per_elem):
    """Per entry: max(|ref|, 1e-3 max |ref| of the entry's element); arrays
    [rows, n_elem * n_per_elem], element-major."""
    rows = ref.shape[0]
    r = np.abs(ref).reshape(rows, -1, n_per_elem)
    elem_max = r.max(axis=(0, 2))[None, :, None]
    scale = np.maximum(r, 1e-3 * elem_max)
    return np.where(scale > 0, scale, 1.0).reshape(ref.shape)


SCALINGS = (3.0, 0.7, 1.3)


def rounding_spread(backward, wl, ref):
    """Per entry, how far FP64 rounding alone moves a gradient.  J = sum G
    limited is homogeneous of degree one in (states, solution): the bounds
    scale with the states (the moments of eq. rhobounds ... mpbounds are
    linear in the Maxwellians, whose shape does not change), and so do the
    limited nodes (eq. limiter, eq. doublelimit) away from the absolute
    floors.  Its gradient is therefore unchanged when both are scaled by
    s > 0; what changes is the rounding of every intermediate.  The largest
    change over a few s (not powers of two) measures it.  `backward(wl)`
    returns (dJ/dstates, dJ/dsolution, dJ/dbounds)."""
    st0, tg0 = wl.states, wl.target
    spread = [np.zeros_like(x) for x in ref]
    try:
        for f in SCALINGS:
            wl.states, wl.target = st0 * f, tg0 * f
            for i, x in enumerate(backward(wl)):
                spread[i] = np.maximum(spread[i], np.abs(x - ref[i]))
    finally:
        wl.states, wl.target = st0, tg0
    return spread


def compare_with_oracle(kbl, wl, seed=0, tol=1e-12):
    G = np.random.default_rng(seed).standard_normal(wl.target.shape)
    gst, gsol, gb, st = gpu_backward(kbl, wl, G)
    rsol, rst, rgb = oracle.workload_backward(wl, G)

    def on_gpu(w):
        r = gpu_backward(kbl, w, G)
        return r[0], r[1], r[2]

    def on_oracle(w):
        r = oracle.workload_backward(w, G)
        return r[1], r[0], r[2]

    sp_g = rounding_spread(on_gpu, wl, (gst, gsol, gb))
    sp_o = rounding_spread(on_oracle, wl, (rst, rsol, rgb))
    out = {}
    for (name, a, b, k), sg, so in zip((("states", gst, rst, wl.n_s),
                                        ("solution", gsol, rsol, wl.n_s),
                                        ("bounds", gb, rgb, 1)), sp_g, sp_o):
        scale = dof_scale(b, k)
        err = np.abs(a - b) / scale
        bar = np.maximum(tol, 4.0 * (sg + so) / scale)
        worst = float((err / bar).max()) if err.size else 0.0
        out[name] = (float(err.max()) if err.size else 0.0, int((bar > tol).sum()), err.size)
        assert worst <= 1.0, (f"{wl.name} d/d{name}: error {out[name][0]:.3e}, "
                              f"{worst:.2f} of its bar")
    print(f"[bwd] {wl.name}: " + ", ".join(
        f"d/d{k} {v[0]:.1e} ({v[1]}/{v[2]} DoFs past 1e-12 by rounding)" for k, v in out.items()),
        flush=True)
    assert not (st & kbl.ST_ASYMMETRIC).any()
    return out


def test_line_global(kbl):
    compare_with_oracle(kbl, synth.make_line_workload(n_elem=12, seed=41, name="b_line"))


def test_line_stencil_box(kbl):
    wl = synth.make_line_workload(n_elem=12, seed=42, name="b_line_st")
    wl.grid = GridSpec(GRID_STENCIL, (300, 1), k=6.0)
    compare_with_oracle(kbl, wl)


@pytest.mark.parametrize("n", [16, 24, 37, 48, 64])
def test_quad_stencil_box(kbl, n):
    wl = synth.make_quad_workload(N=4, seed=43 + n, grid_nodes=n, name=f"b_quad{n}")
    wl.target = wl.states + 10.0 * (wl.target - wl.states)
    compare_with_oracle(kbl, wl)


def test_quad_few_limited(kbl):
    """The unamplified target: most elements bind no bound, their bounds'
    adjoint is zero and the kernel skips them; the gradient must still match
    the oracle's dense evaluation everywhere."""
    wl = synth.make_quad_workload(N=8, seed=48, grid_nodes=24, name="b_quad_sparse")
    st, tg, rp, cl, vg, prm = dev_inputs(kbl, wl)
    b, _ = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
    _, alpha, _ = kbl.limit(tg, b, wl.node_weights, wl.n_s, prm)
    n_lim = int((alpha[0] < 1).sum().item())
    print(f"[bwd] b_quad_sparse: {n_lim}/{wl.n_elem} elements limited", flush=True)
    assert 0 < n_lim < wl.n_elem // 2
    compare_with_oracle(kbl, wl)


def test_quad_global_box(kbl):
    wl = synth.make_quad_workload(N=4, seed=44, field_kind="sine", grid_nodes=32,
                                  grid_mode=GRID_GLOBAL, name="b_quad_gl")
    wl.target = wl.states + 30.0 * (wl.target - wl.states)
    compare_with_oracle(kbl, wl)


def test_tri_stencil_box(kbl):
    wl = synth.make_tri_workload(N=3, seed=45, grid_nodes=24, outer=(0.5, 0.3), name="b_tri")
    wl.target = wl.states + 20.0 * (wl.target - wl.states)
    compare_with_oracle(kbl, wl)


def test_pressure_step_and_shock(kbl):
    wl = synth.make_tri_workload(N=3, seed=46, grid_nodes=24, name="b_tri_shock")
    compare_with_oracle(kbl, wl)
    wl2 = synth.make_line_workload(n_elem=8, seed=47, r_fac=0.97, name="b_pstep")
    wl2.target = wl2.target.copy()
    for i in (5, 13, 18):
        wl2.target[2, i] = 0.3 * 0.5 * wl2.target[1, i] ** 2 / wl2.target[0, i]
    compare_with_oracle(kbl, wl2)


@pytest.mark.parametrize("N", [1, 2])
def test_duplicate_stencil_entries(kbl, N):
    """Periodic meshes one or two elements wide: each stencil row lists a
    neighbour twice (left = right, down = up) and the gather must count it
    once."""
    wl = synth.make_quad_workload(N=N, seed=60 + N, grid_nodes=24, name=f"b_dup{N}")
    row = wl.cols[wl.rowptr[0]:wl.rowptr[1]]
    assert len(np.unique(row)) < len(row)
    wl.target = wl.states + 20.0 * (wl.target - wl.states)
    compare_with_oracle(kbl, wl)


def test_stencils_beyond_256_states_are_flagged(kbl):
    """The backward keeps at most 256 stencil states in LDS: elements with
    larger stencils get KBL_ST_TOO_LARGE and their states no gradient through
    their bounds, while the limiter's part of the gradient (d/dsolution,
    d/dbounds) is still complete."""
    from synth.workloads import quad_block_stencils
    wl = synth.make_quad_workload(N=6, seed=15, grid_nodes=24, name="b_big")
    wl.rowptr, wl.cols = quad_block_stencils(6, 2)
    wl.target = wl.states + 10.0 * (wl.target - wl.states)
    G = np.random.default_rng(6).standard_normal(wl.target.shape)
    gst, gsol, gb, st = gpu_backward(kbl, wl, G)
    assert np.all(st & kbl.ST_TOO_LARGE)
    assert np.isfinite(gst).all()
    rsol, _, rgb = oracle.workload_backward(wl, G)

    def on_gpu(w):
        r = gpu_backward(kbl, w, G)
        return r[1], r[2]

    def on_oracle(w):
        r = oracle.workload_backward(w, G)
        return r[0], r[2]

    sp_g = rounding_spread(on_gpu, wl, (gsol, gb))
    sp_o = rounding_spread(on_oracle, wl, (rsol, rgb))
    assert np.abs(gb).max() > 0
    for a, b, k, sg, so in ((gsol, rsol, wl.n_s, sp_g[0], sp_o[0]),
                            (gb, rgb, 1, sp_g[1], sp_o[1])):
        scale = dof_scale(b, k)
        bar = np.maximum(1e-12, 4.0 * (sg + so) / scale)
        assert (np.abs(a - b) / scale / bar).max() <= 1.0


def test_quad512_finite_differences(kbl):
    """Config of the differentiation form: full 512^2 mesh, 200 DoFs."""
    wl = synth.make_workload("quad512")
    rng = np.random.default_rng(240720966 + 4)
    w = rng.standard_normal(wl.n_nodes)
    G = np.zeros_like(wl.states)
    G[0] = w
    gst, gsol, _, _ = gpu_backward(kbl, wl, G)
    grad = gst + gsol                  # the solution is W + Delta: both paths
    st, tg, rp, cl, vg, prm = dev_inputs(kbl, wl)
    wt = torch.from_numpy(w).to(st.device)

    def J_local(elems):
        b, _ = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
        lim, _, _ = kbl.limit(tg, b, wl.node_weights, wl.n_s, prm)
        idx = torch.from_numpy((elems[:, None] * wl.n_s + np.arange(wl.n_s)).ravel()).to(st.device)
        return float((lim[0, idx] * wt[idx]).sum().item())

    n_dofs = 200
    errs, kinks = [], 0
    gscale = np.abs(grad).max()
    for _ in range(n_dofs):
        v = int(rng.integers(4))
        n = int(rng.integers(wl.n_nodes))
        E = n // wl.n_s
        aff = np.unique(wl.cols[wl.rowptr[E]:wl.rowptr[E + 1]]).astype(np.int64)
        x0 = float(wl.states[v, n])
        h = 1e-7 * max(1.0, abs(x0))
        vals = {}
        for sgn in (-1, 0, 1):
            st[v, n] = x0 + sgn * h
            tg[v, n] = float(wl.target[v, n]) + sgn * h
            vals[sgn] = J_local(aff)
        st[v, n] = x0
        tg[v, n] = float(wl.target[v, n])
        fwd = (vals[1] - vals[0]) / h
        bwd = (vals[0] - vals[-1]) / h
        cen = (vals[1] - vals[-1]) / (2 * h)
        if abs(fwd - bwd) > 1e-3 * (abs(cen) + 1e-6 * gscale):
            kinks += 1
            continue
        noise = 1e3 * np.finfo(float).eps * max(abs(vals[0]), 1.0) / h
        errs.append(abs(cen - grad[v, n]) / max(abs(grad[v, n]), 1e-6 * gscale, noise))
    print(f"[fd-gpu] quad512: {len(errs)} smooth DoFs, max rel err {max(errs):.2e}, "
          f"median {np.median(errs):.1e}, {kinks} within h of a kink", flush=True)
    assert len(errs) >= 0.8 * n_dofs
    assert max(errs) <= 1e-6


def test_autograd_function(kbl):
    wl = synth.make_quad_workload(N=6, seed=48, grid_nodes=32, name="b_autograd")
    st, tg, rp, cl, vg, prm = dev_inputs(kbl, wl)
    delta = (tg - st).detach()
    x = st.clone().requires_grad_(True)
    w = torch.from_numpy(np.random.default_rng(3).standard_normal(wl.n_nodes)).to(st.device)
    lim = kbl.bounds_and_limit(x, x + delta, rp, cl, wl.n_s, vg, prm, wl.node_weights)
    J = (lim[0] * w).sum()
    J.backward()
    G = torch.zeros_like(st)
    G[0] = w
    gst, gsol, _, _ = kbl.bounds_limit_backward(st, rp, cl, wl.n_s, vg, prm, tg, wl.node_weights, G)
    torch.cuda.synchronize()
    assert torch.equal(x.grad, gst + gsol)


def test_backward_determinism(kbl):
    wl = synth.make_quad_workload(N=8, seed=49, grid_nodes=48, name="b_det")
    G = np.random.default_rng(1).standard_normal(wl.target.shape)
    a = gpu_backward(kbl, wl, G)
    b = gpu_backward(kbl, wl, G)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


def test_asymmetric_stencil_flagged(kbl):
    wl = synth.make_quad_workload(N=6, seed=50, grid_nodes=16, name="b_asym")
    wl.cols = wl.cols.copy()
    wl.cols[5 * 7 + 4] = 20           # element 7 lists element 20, which does not list 7
    G = np.random.default_rng(2).standard_normal(wl.target.shape)
    _, _, _, st = gpu_backward(kbl, wl, G)
    assert st[7] & kbl.ST_ASYMMETRIC


@pytest.mark.parametrize("precision", [0, 3, 2])
def test_forward_bounds_handover_is_bit_identical(kbl, precision):
    """Passing the forward's bounds/status gives exactly the recomputed result."""
    wl = synth.make_quad_workload(N=8, seed=51, grid_nodes=48, name="b_handover")
    st, tg, rp, cl, vg, _ = dev_inputs(kbl, wl)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac, precision=precision)
    G = torch.from_numpy(np.random.default_rng(4).standard_normal(wl.target.shape)).to(st.device)
    a = kbl.bounds_limit_backward(st, rp, cl, wl.n_s, vg, prm, tg, wl.node_weights, G)
    b0, s0 = kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm)
    b = kbl.bounds_limit_backward(st, rp, cl, wl.n_s, vg, prm, tg, wl.node_weights, G,
                                  fwd_bounds=b0, fwd_status=s0)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("precision,name", [(3, "fp32"), (2, "fp16"), (1, "bf16")])
def test_mixed_backward_error_vs_fp64(kbl, precision, name):
    """Gradient of the mixed-precision forward (FP32 envelope winners, limiter
    on the mixed bounds) against the FP64 gradient: reported, and bounded
    loosely (the limiter's ratio terms amplify the 1e-7 bound differences)."""
    wl = synth.make_quad_workload(N=32, seed=52, grid_nodes=48, name="b_mixed")
    st, tg, rp, cl, vg, prm = dev_inputs(kbl, wl)
    prm_m = kbl.make_params(wl.gamma, r_fac=wl.r_fac, precision=precision)
    G = torch.zeros_like(st)
    G[0] = torch.from_numpy(np.random.default_rng(5).standard_normal(wl.n_nodes)).to(st.device)
    ref = kbl.bounds_limit_backward(st, rp, cl, wl.n_s, vg, prm, tg, wl.node_weights, G)
    mix = kbl.bounds_limit_backward(st, rp, cl, wl.n_s, vg, prm_m, tg, wl.node_weights, G)
    again = kbl.bounds_limit_backward(st, rp, cl, wl.n_s, vg, prm_m, tg, wl.node_weights, G)
    torch.cuda.synchronize()
    g_ref = (ref[0] + ref[1]).cpu().numpy()
    g_mix = (mix[0] + mix[1]).cpu().numpy()
    scale = np.abs(g_ref).max()
    err = np.abs(g_mix - g_ref)
    share = (err <= 1e-6 * scale).mean()
    print(f"[bwd-mixed] {name}: max err {err.max() / scale:.2e}, p99 "
          f"{np.quantile(err, 0.99) / scale:.2e} of the max gradient; "
          f"{100 * share:.1f}% of DoFs within 1e-6", flush=True)
    assert err.max() <= 5e-2 * scale
    assert share >= 0.9
    for x, y in zip(mix, again):
        assert torch.equal(x, y)
