"""Host-side checks of the C-ABI (no GPU needed, no kernel is launched).

- libkbl.so loads and exports every entry point include/kbl.h declares;
- the ctypes mirrors of kbl_params / kbl_vgrid match the C layout (gcc);
- argument errors are returned synchronously, before any HIP call.
"""

import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2407_20966_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = C.c_void_p(0x10000)   # never dereferenced: every call below fails validation first


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libkbl.so not built (run __graft_entry__.build())")
    return L.lib()


def test_header_declares_expected_entry_points():
    syms = L.header_symbols()
    for s in ("kbl_compute_bounds", "kbl_limit", "kbl_status_string", "kbl_version",
              "kbl_default_params", "kbl_bounds_limit_backward", "kbl_backward_workspace_bytes",
              "kbl_autotune_bounds", "kbl_autotune_clear", "kbl_compute_bounds_nodes",
              "kbl_riemann_states", "kbl_status_summary"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in L.header_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True)
    if out.returncode == 0:
        exported = {ln.split()[-1] for ln in out.stdout.splitlines() if ln.strip()}
        assert set(L.header_symbols()) <= exported


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "kbl.h"\n'
        "int main(void){\n"
        ' printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(kbl_params), offsetof(kbl_params, precision),'
        " offsetof(kbl_params, eps_alpha), sizeof(kbl_vgrid), offsetof(kbl_vgrid, lo),"
        " offsetof(kbl_vgrid, k));\n return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals == [C.sizeof(L.Params), L.Params.precision.offset, L.Params.eps_alpha.offset,
                    C.sizeof(L.VGrid), L.VGrid.lo.offset, L.VGrid.k.offset]


def test_defaults_and_strings(lib):
    p = L.Params()
    lib.kbl_default_params(C.byref(p), 1.4)
    assert (p.gamma, p.r_fac, p.rho_floor, p.p_floor, p.eps_alpha) == (1.4, 1e-3, 1e-12, 1e-12, 1e-13)
    assert p.precision == L.PREC_FP64 and p.flags == 0
    for code in range(7):
        assert lib.kbl_status_string(code)
    assert lib.kbl_version() >= 100


def _params(lib, gamma=1.4, **kw):
    p = L.Params()
    lib.kbl_default_params(C.byref(p), gamma)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _grid(mode=L.GRID_STENCIL, n=(48, 48), lo=(-1, -1), hi=(1, 1), k=4.0):
    g = L.VGrid()
    g.mode = mode
    g.n[0], g.n[1] = n
    g.lo[0], g.lo[1] = lo
    g.hi[0], g.hi[1] = hi
    g.k = k
    return g


def _bounds(lib, p, g, dim=2, n_elem=4, n_s=16, nnz=20, ptrs=True):
    P = FAKE if ptrs else None
    return lib.kbl_compute_bounds(C.byref(p), dim, n_elem, n_s, nnz, P, P, P, C.byref(g), P, None, None)


@pytest.mark.parametrize("case,expect", [
    (dict(dim=4), L.KBL_ERR_ARG),
    (dict(dim=0), L.KBL_ERR_ARG),
    (dict(n_elem=-1), L.KBL_ERR_ARG),
    (dict(n_s=0), L.KBL_ERR_ARG),
    (dict(nnz=-3), L.KBL_ERR_ARG),
    (dict(ptrs=False), L.KBL_ERR_ARG),
])
def test_bounds_rejects_bad_sizes(lib, case, expect):
    assert _bounds(lib, _params(lib), _grid(), **case) == expect


@pytest.mark.parametrize("pkw,expect", [
    (dict(gamma=1.0), L.KBL_ERR_GAMMA),
    (dict(gamma=0.5), L.KBL_ERR_GAMMA),
    (dict(gamma=2.5), L.KBL_ERR_GAMMA),          # delta = 2/1.5 - 2 < 0 in 2D
    (dict(r_fac=1.0), L.KBL_ERR_ARG),
    (dict(r_fac=-1e-3), L.KBL_ERR_ARG),
    (dict(rho_floor=-1.0), L.KBL_ERR_ARG),
    (dict(eps_alpha=float("nan")), L.KBL_ERR_ARG),
    (dict(flags=0x100), L.KBL_ERR_ARG),
    (dict(flags=L.FLAG_ENERGY_PERSTATE, precision=L.PREC_MIXED_FP32), L.KBL_ERR_UNSUPPORTED),
    (dict(precision=7), L.KBL_ERR_UNSUPPORTED),
])
def test_bounds_rejects_bad_params(lib, pkw, expect):
    gamma = pkw.pop("gamma", 1.4)
    assert _bounds(lib, _params(lib, gamma, **pkw), _grid()) == expect


@pytest.mark.parametrize("gkw,expect", [
    (dict(n=(1, 48)), L.KBL_ERR_GRID),
    (dict(n=(48, 1)), L.KBL_ERR_GRID),
    (dict(n=(65, 48)), L.KBL_ERR_GRID),
    (dict(k=0.0), L.KBL_ERR_GRID),
    (dict(k=float("inf")), L.KBL_ERR_GRID),
    (dict(mode=L.GRID_GLOBAL, lo=(1, 0), hi=(1, 1)), L.KBL_ERR_GRID),
    (dict(mode=L.GRID_GLOBAL, lo=(0, 0), hi=(1, float("nan"))), L.KBL_ERR_GRID),
    (dict(mode=5), L.KBL_ERR_GRID),
])
def test_bounds_rejects_bad_grid(lib, gkw, expect):
    assert _bounds(lib, _params(lib), _grid(**gkw)) == expect


def test_mixed_precision_is_2d_only(lib):
    for prec in (L.PREC_MIXED_BF16, L.PREC_MIXED_FP16, L.PREC_MIXED_FP32):
        assert _bounds(lib, _params(lib, precision=prec), _grid(n=(64, 2)), dim=1) == L.KBL_ERR_UNSUPPORTED


def test_bounds_1d_grid_limit(lib):
    g = _grid(n=(4097, 2))
    assert _bounds(lib, _params(lib), g, dim=1) == L.KBL_ERR_GRID


def _limit(lib, p, w, dim=2, n_elem=4, n_s=None):
    n_s = len(w) if n_s is None else n_s
    wa = np.ascontiguousarray(w, dtype=np.float64)
    return lib.kbl_limit(C.byref(p), dim, n_elem, n_s, FAKE, FAKE,
                         wa.ctypes.data_as(C.c_void_p), FAKE, None, None, None)


def test_limit_rejects_bad_weights(lib):
    p = _params(lib)
    assert _limit(lib, p, [1.0, -1.0, 1.0]) == L.KBL_ERR_ARG
    assert _limit(lib, p, [1.0, float("nan")]) == L.KBL_ERR_ARG
    assert _limit(lib, p, [1.0] * 65) == L.KBL_ERR_ARG      # n_s > 64
    assert lib.kbl_limit(C.byref(p), 2, 4, 4, FAKE, FAKE, None, FAKE, None, None, None) == L.KBL_ERR_ARG


def test_limit_rejects_bad_params(lib):
    assert _limit(lib, _params(lib, 1.0), [1.0, 1.0]) == L.KBL_ERR_GAMMA
    assert _limit(lib, _params(lib), [1.0, 1.0], dim=4) == L.KBL_ERR_ARG
    assert _limit(lib, _params(lib), [1.0, 1.0], n_elem=-2) == L.KBL_ERR_ARG


def _backward(lib, p, g, dim=2, n_elem=4, n_s=16, nnz=20, ws_bytes=None, weights=None,
              fwd_b=None, fwd_s=None):
    w = np.ones(n_s) if weights is None else np.asarray(weights, dtype=np.float64)
    need = lib.kbl_backward_workspace_bytes(dim, n_elem, n_s, nnz)
    wsb = need if ws_bytes is None else ws_bytes
    return lib.kbl_bounds_limit_backward(C.byref(p), dim, n_elem, n_s, nnz, FAKE, FAKE, FAKE,
                                         C.byref(g), fwd_b, fwd_s, FAKE,
                                         w.ctypes.data_as(C.c_void_p), FAKE, FAKE, FAKE, None,
                                         None, FAKE, wsb, None)


def test_backward_workspace_size(lib):
    # recomputed bounds + status + dJ/dbounds + one slot per (stencil entry, node, variable)
    n = lib.kbl_backward_workspace_bytes(2, 1000, 16, 5000)
    assert n >= 4 * 5000 * 16 * 8 + 2 * 8 * 1000 * 8 + 4 * 1000
    assert lib.kbl_backward_workspace_bytes(3, 10, 4, 10) == 0


def test_backward_rejects_bad_arguments(lib):
    g = _grid()
    assert _backward(lib, _params(lib), g, ws_bytes=16) == L.KBL_ERR_WORKSPACE
    assert _backward(lib, _params(lib, precision=7), g) == L.KBL_ERR_UNSUPPORTED
    assert _backward(lib, _params(lib, precision=L.PREC_MIXED_FP16), _grid(n=(64, 2)),
                     dim=1, n_s=4) == L.KBL_ERR_UNSUPPORTED
    assert _backward(lib, _params(lib), g, fwd_b=FAKE, fwd_s=None) == L.KBL_ERR_ARG
    assert _backward(lib, _params(lib, gamma=1.0), g) == L.KBL_ERR_GAMMA
    assert _backward(lib, _params(lib), _grid(n=(65, 48))) == L.KBL_ERR_GRID
    assert _backward(lib, _params(lib), _grid(n=(2049, 2)), dim=1, n_s=4) == L.KBL_ERR_GRID
    assert _backward(lib, _params(lib), g, weights=[0.0] * 16) == L.KBL_ERR_ARG   # zero sum


def _autotune(lib, p, g, dim=2, n_elem=4, n_s=16, nnz=20):
    return lib.kbl_autotune_bounds(C.byref(p), dim, n_elem, n_s, nnz, FAKE, FAKE, FAKE,
                                   C.byref(g), FAKE, None, 0, None)


def test_autotune_rejects_bad_arguments(lib):
    g = _grid()
    assert _autotune(lib, _params(lib, gamma=1.0), g) == -1
    assert _autotune(lib, _params(lib), _grid(n=(65, 48))) == -1
    assert _autotune(lib, _params(lib, precision=7), g) == -1
    assert _autotune(lib, _params(lib, precision=L.PREC_MIXED_FP16), _grid(n=(64, 2)), dim=1) == -1
    assert _autotune(lib, _params(lib), g, n_elem=0) == -1
    lib.kbl_autotune_clear()


def _bounds_nodes(lib, p, g, n_elem=4, n_nodes=64, nnz=20, ptrs=True):
    P = FAKE if ptrs else None
    return lib.kbl_compute_bounds_nodes(C.byref(p), 2, n_elem, n_nodes, nnz, P, P, P, C.byref(g),
                                        P, None, None)


def test_node_stencil_rejects_bad_arguments(lib):
    g = _grid()
    assert _bounds_nodes(lib, _params(lib), g, n_nodes=-1) == L.KBL_ERR_ARG
    assert _bounds_nodes(lib, _params(lib), g, ptrs=False) == L.KBL_ERR_ARG
    assert _bounds_nodes(lib, _params(lib, 1.0), g) == L.KBL_ERR_GAMMA
    assert _bounds_nodes(lib, _params(lib), _grid(n=(65, 48))) == L.KBL_ERR_GRID


def test_limit_weights_may_be_zero_but_not_all():
    p = _params(lib=L.lib())
    lib = L.lib()
    assert _limit(lib, p, [0.0, 0.0, 0.0]) == L.KBL_ERR_ARG
    # zero weights on some nodes are accepted: the call then fails only on the
    # (fake) device pointers, which it never reaches without a GPU, so check
    # the argument validation through an empty element count instead
    w = np.array([1.0, 0.0, 2.0])
    assert lib.kbl_limit(C.byref(p), 2, 0, 3, None, None, w.ctypes.data_as(C.c_void_p),
                         None, None, None, None) == L.KBL_OK


def test_backward_default_method_only(lib):
    g = _grid()
    for flags in (L.FLAG_INDEPENDENT_ALPHA, L.FLAG_ENERGY_PERSTATE):
        assert _backward(lib, _params(lib, flags=flags), g) == L.KBL_ERR_UNSUPPORTED


def _riemann(lib, p, dim=2, n_pairs=4, n_nodes=8, bounds=None, elem=None, n_elem=0, ptrs=True):
    P = FAKE if ptrs else None
    return lib.kbl_riemann_states(C.byref(p), dim, n_pairs, n_nodes, P, P, P, P, None, bounds,
                                  elem, n_elem, P, None, None)


def test_riemann_rejects_bad_arguments(lib):
    p = _params(lib)
    assert _riemann(lib, p, dim=4) == L.KBL_ERR_ARG
    assert _riemann(lib, p, n_pairs=-1) == L.KBL_ERR_ARG
    assert _riemann(lib, p, ptrs=False) == L.KBL_ERR_ARG
    assert _riemann(lib, p, bounds=FAKE, elem=None, n_elem=4) == L.KBL_ERR_ARG
    assert _riemann(lib, p, bounds=FAKE, elem=FAKE, n_elem=0) == L.KBL_ERR_ARG
    assert _riemann(lib, _params(lib, 1.0)) == L.KBL_ERR_GAMMA
    assert _riemann(lib, p, n_pairs=0, ptrs=False) == L.KBL_OK      # nothing to do, no launch


def _grid3(mode=L.GRID_STENCIL, n=(24, 24, 24), k=4.0):
    g = L.VGrid()
    g.mode = mode
    for j in range(3):
        g.n[j] = n[j]
        g.lo[j], g.hi[j] = -1.0, 1.0
    g.k = k
    return g


def test_three_dimensional_rejections(lib):
    # every case returns before any launch (the pointers are fake)
    p = _params(lib)
    assert _bounds(lib, p, _grid3(n=(24, 24, 1)), dim=3, n_s=27) == L.KBL_ERR_GRID
    assert _bounds(lib, p, _grid3(n=(24, 65, 24)), dim=3, n_s=27) == L.KBL_ERR_GRID
    assert _bounds(lib, p, _grid3(n=(24, 24, 65)), dim=3, n_s=27) == L.KBL_ERR_GRID
    # delta = 2/(gamma-1) - 3 < 0 for gamma > 5/3
    assert _bounds(lib, _params(lib, 1.7), _grid3(), dim=3, n_s=27) == L.KBL_ERR_GAMMA
    for prec in (L.PREC_MIXED_BF16, L.PREC_MIXED_FP16, L.PREC_MIXED_FP32):
        assert _bounds(lib, _params(lib, precision=prec), _grid3(), dim=3, n_s=27) == L.KBL_ERR_UNSUPPORTED
        assert _autotune(lib, _params(lib, precision=prec), _grid3(), dim=3, n_s=27) == -1
    pe = _params(lib, flags=L.FLAG_ENERGY_PERSTATE)
    assert _bounds(lib, pe, _grid3(), dim=3, n_s=27) == L.KBL_ERR_UNSUPPORTED
    assert _autotune(lib, pe, _grid3(), dim=3, n_s=27) == -1
    assert _backward(lib, p, _grid3(), dim=3, n_s=27) == L.KBL_ERR_UNSUPPORTED
    assert lib.kbl_backward_workspace_bytes(3, 10, 27, 10) == 0
    assert _bounds(lib, p, _grid3(), dim=3, n_s=27, ptrs=False) == L.KBL_ERR_ARG
    assert _riemann(lib, p, dim=3, ptrs=False) == L.KBL_ERR_ARG
    assert _limit(lib, p, [1.0] * 27, dim=3, n_elem=-1) == L.KBL_ERR_ARG


def _tile_table(src, macro):
    import re
    text = open(os.path.join(ROOT, "paper_2407_20966_amd", "csrc", src)).read()
    rows = re.findall(rf"^\s*{macro}\(([^)]*)\),", text, flags=re.M)
    return {i: tuple(int(x) for x in r.split(",")) for i, r in enumerate(rows)}


def test_python_tile_tables_match_the_kernels():
    # the tile indices accepted by KBL_BOUNDS_TILE / KBL_MIXED_TILE and
    # returned by kbl_autotune_bounds are positions in these tables
    assert _tile_table("bounds_fp64.hip", "KBL_TILE") == L.FP64_TILES
    assert _tile_table("bounds_fp64_3d.hip", "KBL_TILE3") == L.FP64_TILES_3D
    assert _tile_table("bounds_mixed.hip", "KBL_MTILE") == L.MIXED_TILES


# ---------------------------------------------------------------- 1D FR solver

def _fr_cfg(**kw):
    c = L.Fr1dCfg()
    c.p, c.bc, c.n_elem, c.x0, c.x1, c.limit, c.reserved = 3, L.FR_PERIODIC, 16, 0.0, 1.0, 1, 0
    for k, v in kw.items():
        if k in ("left", "right"):
            for i in range(3):
                getattr(c, k)[i] = v[i]
        else:
            setattr(c, k, v)
    return c


def test_fr1d_struct_layout_matches_c(tmp_path):
    src = tmp_path / "fr.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "kbl_fr1d.h"\n'
        "int main(void){\n"
        ' printf("%zu %zu %zu %zu %zu\\n", sizeof(kbl_fr1d), offsetof(kbl_fr1d, n_elem),'
        " offsetof(kbl_fr1d, left), offsetof(kbl_fr1d, right), offsetof(kbl_fr1d, limit));\n"
        " return 0;}\n")
    exe = tmp_path / "fr"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals == [C.sizeof(L.Fr1dCfg), L.Fr1dCfg.n_elem.offset, L.Fr1dCfg.left.offset,
                    L.Fr1dCfg.right.offset, L.Fr1dCfg.limit.offset]


@pytest.mark.parametrize("kw", [dict(p=0), dict(p=8), dict(n_elem=1), dict(x1=0.0), dict(bc=5),
                                dict(limit=2), dict(reserved=1)])
def test_fr1d_rejects_bad_config(lib, kw):
    c = _fr_cfg(**kw)
    assert lib.kbl_fr1d_columns(C.byref(c)) == 0
    assert lib.kbl_fr1d_workspace_bytes(C.byref(c)) == 0
    assert lib.kbl_fr1d_rhs(C.byref(c), 1.4, FAKE, FAKE, None) == L.KBL_ERR_ARG
    assert lib.kbl_fr1d_max_speed(C.byref(c), 1.4, FAKE, FAKE, None) == L.KBL_ERR_ARG


def test_fr1d_sizes():
    lib = L.lib()
    c = _fr_cfg()
    assert lib.kbl_fr1d_columns(C.byref(c)) == 16 * 6
    d = _fr_cfg(bc=L.FR_DIRICHLET, left=(1, 0, 2.5), right=(0.125, 0, 0.25))
    assert lib.kbl_fr1d_columns(C.byref(d)) == 18 * 6
    assert lib.kbl_fr1d_workspace_bytes(C.byref(d)) >= 8 * 3 * 18 * 6 + 8 * 3 * 16 * 4 + 8 * 6 * 18


def test_fr1d_step_and_limit_argument_errors(lib):
    # every case returns before any launch (the pointers are fake)
    p = _params(lib)
    g = L.VGrid()
    g.mode, g.n[0], g.k = L.GRID_STENCIL, 256, 8.0
    c = _fr_cfg()
    ws = lib.kbl_fr1d_workspace_bytes(C.byref(c))

    def step(cfg=c, prm=p, grid=g, dt=1e-3, U=FAKE, wsb=ws):
        return lib.kbl_fr1d_step(C.byref(cfg), C.byref(prm), C.byref(grid), dt, U, FAKE, wsb,
                                 None, None)

    def lim(cfg=c, prm=p, grid=g, U=FAKE, wsb=ws):
        return lib.kbl_fr1d_limit(C.byref(cfg), C.byref(prm), C.byref(grid), U, FAKE, wsb, None, None)

    for fn in (step, lim):
        assert fn(wsb=ws - 1) == L.KBL_ERR_WORKSPACE
        assert fn(U=None) == L.KBL_ERR_ARG
        assert fn(prm=_params(lib, precision=L.PREC_MIXED_FP32)) == L.KBL_ERR_UNSUPPORTED
        assert fn(prm=_params(lib, flags=L.FLAG_ENERGY_PERSTATE)) == L.KBL_ERR_UNSUPPORTED
        assert fn(prm=_params(lib, gamma=1.0)) == L.KBL_ERR_GAMMA
        bad = L.VGrid()
        bad.mode, bad.n[0], bad.k = L.GRID_STENCIL, 5000, 8.0
        assert fn(grid=bad) == L.KBL_ERR_GRID
        dirich = _fr_cfg(bc=L.FR_DIRICHLET, left=(1.0, 0.0, -1.0), right=(0.125, 0.0, 0.25))
        assert fn(cfg=dirich, wsb=lib.kbl_fr1d_workspace_bytes(C.byref(dirich))) == L.KBL_ERR_ARG
    assert step(dt=0.0) == L.KBL_ERR_ARG
    assert step(dt=float("nan")) == L.KBL_ERR_ARG


def test_status_summary_rejects_bad_arguments(lib):
    assert lib.kbl_status_summary(FAKE, -1, FAKE, None) == L.KBL_ERR_ARG
    assert lib.kbl_status_summary(FAKE, 10, None, None) == L.KBL_ERR_ARG
    assert lib.kbl_status_summary(None, 10, FAKE, None) == L.KBL_ERR_ARG
