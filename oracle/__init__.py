"""FP64 CPU oracle for kinetic maximum-principle bounds and the squeeze limiter.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the bench import this package.  It wraps ``liboracle.so``
(built from ``kbl_oracle.c`` with gcc, FP64, no fast-math) through ctypes and
shares no code with the HIP library.

Functions take NumPy arrays and the plain workload fields; see
``kbl_oracle.c`` for the passages of the paper each step follows.

Parity status: bounds and limiter are pinned by the closed-form, printed-value,
invariant and brute-force checks in ``tests/test_oracle_*.py``.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kbl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ST_INADMISSIBLE = 0x1
ST_RHO_FLOOR = 0x2
ST_EPS_RULE = 0x4
ST_LIMITED = 0x8
ST_PSTEP = 0x10
ST_PMEAN_FLOOR = 0x20
ST_MEAN_OUTSIDE = 0x40
ST_BAD_BOUNDS = 0x80
ST_BAD_STENCIL = 0x100

RHO_FLOOR = 1e-12     # Sec. 3.8
P_FLOOR = 1e-12       # Sec. 3.8
EPS_ALPHA = 1e-13     # Sec. 3.4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2 -fopenmp, strict IEEE)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-D_DEFAULT_SOURCE", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.oracle_bounds.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                                      C.c_int, P, P, P, C.c_double,
                                      C.c_int64, C.c_int64, C.c_int, C.c_int64, P, P, P, P,
                                      C.c_int64, C.c_int, P, P]
        lib.oracle_bounds.restype = C.c_int
        lib.oracle_limit.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                                     C.c_int64, C.c_int, P, P, P, C.c_int, P, C.c_int64, P, P, P]
        lib.oracle_limit.restype = C.c_int
        lib.oracle_backward.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_int, P, P, P, C.c_double, C.c_int64,
                                        C.c_int, P, P, P, P, P, P, P, P, P]
        lib.oracle_backward.restype = C.c_int
        lib.oracle_riemann.argtypes = [C.c_int, C.c_double, C.c_int64, C.c_int64, P, P, P, P, P,
                                       P, P, C.c_int64, P, P]
        lib.oracle_riemann.restype = C.c_int
        lib.oracle_delta.argtypes = [C.c_int, C.c_double]
        lib.oracle_delta.restype = C.c_double
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def bounds(dim: int, gamma: float, states: np.ndarray, rowptr: np.ndarray,
           cols: np.ndarray, n_s: int, grid_mode: int, n, lo=(0.0, 0.0),
           hi=(0.0, 0.0), k: float = 4.0, r_fac: float = 1e-3,
           rho_floor: float = RHO_FLOOR,
           elems: Optional[np.ndarray] = None, energy_mode: int = 0,
           n_src: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Kinetic bounds [2(d+2), n_sel] and status [n_sel] (Sec. 3.3-3.8).

    cols list source units of n_s nodes each: elements (n_src = n_elem, the
    default) or, with n_s = 1, single nodes of a node-level stencil.
    energy_mode 0: separate g_T / g_I envelopes; 1: per-state energy integrand.
    """
    lib = _load()
    states = np.ascontiguousarray(states, dtype=np.float64)
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    n_elem = rowptr.size - 1
    if n_src is None:
        n_src = n_elem
    assert states.shape == (dim + 2, n_src * n_s)
    if elems is not None:
        elems = np.ascontiguousarray(elems, dtype=np.int64)
        n_sel = elems.size
    else:
        n_sel = n_elem
    n_arr = np.array(list(n) + [2] * (3 - len(n)), dtype=np.int32)[:3]
    lo_arr = np.array(list(lo) + [0.0] * (3 - len(lo)), dtype=np.float64)[:3]
    hi_arr = np.array(list(hi) + [0.0] * (3 - len(hi)), dtype=np.float64)[:3]
    out = np.empty((2 * (dim + 2), n_sel), dtype=np.float64)
    st = np.empty(n_sel, dtype=np.uint32)
    rc = lib.oracle_bounds(dim, gamma, r_fac, rho_floor, grid_mode, _p(n_arr), _p(lo_arr),
                           _p(hi_arr), k, n_elem, n_src, n_s, cols.size, _p(states), _p(rowptr),
                           _p(cols), _p(elems), n_sel, energy_mode, _p(out), _p(st))
    if rc != 0:
        raise ValueError("oracle_bounds rejected its arguments")
    return out, st


def limit(dim: int, gamma: float, solution: np.ndarray, bounds_sel: np.ndarray,
          node_weights: np.ndarray, n_s: int, p_floor: float = P_FLOOR,
          eps: float = EPS_ALPHA, elems: Optional[np.ndarray] = None,
          independent: bool = False):
    """Squeeze limiter + pressure step (Sec. 3.4, 3.8); coupled alpha_min, or
    per-component alpha_i with ``independent``.  Weights may be zero (nodes
    outside the mean, e.g. flux points) but must have a positive sum.

    Returns (limited [d+2, n_sel*n_s], alpha [2, n_sel], status [n_sel]).
    ``bounds_sel`` holds one column per selected element.
    """
    lib = _load()
    solution = np.ascontiguousarray(solution, dtype=np.float64)
    bounds_sel = np.ascontiguousarray(bounds_sel, dtype=np.float64)
    c = np.ascontiguousarray(node_weights, dtype=np.float64)
    n_elem = solution.shape[1] // n_s
    if elems is not None:
        elems = np.ascontiguousarray(elems, dtype=np.int64)
        n_sel = elems.size
    else:
        n_sel = n_elem
    assert bounds_sel.shape == (2 * (dim + 2), n_sel)
    lim = np.empty((dim + 2, n_sel * n_s), dtype=np.float64)
    al = np.empty((2, n_sel), dtype=np.float64)
    st = np.empty(n_sel, dtype=np.uint32)
    rc = lib.oracle_limit(dim, gamma, p_floor, eps, n_elem, n_s, _p(solution), _p(bounds_sel),
                          _p(c), int(bool(independent)), _p(elems), n_sel, _p(lim), _p(al),
                          _p(st))
    if rc != 0:
        raise ValueError("oracle_limit rejected its arguments")
    return lim, al, st


def backward(dim, gamma, states, rowptr, cols, n_s, grid_mode, n, lo, hi, k, r_fac,
             solution, node_weights, grad_limited, rho_floor=RHO_FLOOR, p_floor=P_FLOOR,
             eps=EPS_ALPHA):
    """Analytic subgradient: (dJ/dsolution, dJ/dstates, dJ/dbounds) for
    G = dJ/dlimited (all elements, serial)."""
    lib = _load()
    states = np.ascontiguousarray(states, dtype=np.float64)
    solution = np.ascontiguousarray(solution, dtype=np.float64)
    G = np.ascontiguousarray(grad_limited, dtype=np.float64)
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    c = np.ascontiguousarray(node_weights, dtype=np.float64)
    n_elem = rowptr.size - 1
    n_arr = np.array(list(n) + [2] * (3 - len(n)), dtype=np.int32)[:3]
    lo_arr = np.array(list(lo) + [0.0] * (3 - len(lo)), dtype=np.float64)[:3]
    hi_arr = np.array(list(hi) + [0.0] * (3 - len(hi)), dtype=np.float64)[:3]
    gsol = np.empty_like(solution)
    gst = np.empty_like(states)
    gb = np.empty((2 * (dim + 2), n_elem), dtype=np.float64)
    rc = lib.oracle_backward(dim, gamma, r_fac, rho_floor, p_floor, eps, grid_mode, _p(n_arr),
                             _p(lo_arr), _p(hi_arr), k, n_elem, n_s, _p(states), _p(rowptr),
                             _p(cols), _p(solution), _p(c), _p(G), _p(gsol), _p(gst), _p(gb))
    if rc != 0:
        raise ValueError("oracle_backward rejected its arguments")
    return gsol, gst, gb


def workload_backward(wl, grad_limited, solution=None):
    g = wl.grid
    return backward(wl.dim, wl.gamma, wl.states, wl.rowptr, wl.cols, wl.n_s, g.mode,
                    g.n[: wl.dim], g.lo, g.hi, g.k, wl.r_fac,
                    wl.target if solution is None else solution, wl.node_weights, grad_limited)


def riemann(dim: int, gamma: float, states: np.ndarray, ni: np.ndarray, nj: np.ndarray,
            normals: np.ndarray, lam: Optional[np.ndarray] = None,
            bounds: Optional[np.ndarray] = None, elem: Optional[np.ndarray] = None):
    """Riemann-averaged states of Thm. 4.3 (Sec. 4) for node pairs (i, j) with
    unit normals [d, n_pairs]; lam per pair or None for the wavespeed estimate.
    Returns (bar [d+2, n_pairs], status [n_pairs]): bit v = below w_min,v,
    bit 8+v = above w_max,v of the pair's element (when bounds are given),
    bit 16 = bad node id or inadmissible input state."""
    lib = _load()
    states = np.ascontiguousarray(states, dtype=np.float64)
    ni = np.ascontiguousarray(ni, dtype=np.int32)
    nj = np.ascontiguousarray(nj, dtype=np.int32)
    normals = np.ascontiguousarray(normals, dtype=np.float64)
    n_pairs = ni.size
    assert nj.size == n_pairs and normals.shape == (dim, n_pairs)
    lam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    if bounds is not None:
        bounds = np.ascontiguousarray(bounds, dtype=np.float64)
        elem = np.ascontiguousarray(elem, dtype=np.int32)
    n_elem = 0 if bounds is None else bounds.shape[1]
    bar = np.empty((dim + 2, n_pairs), dtype=np.float64)
    st = np.empty(n_pairs, dtype=np.uint32)
    rc = lib.oracle_riemann(dim, gamma, n_pairs, states.shape[1], _p(states), _p(ni), _p(nj),
                            _p(normals), _p(lam), _p(bounds), _p(elem), n_elem, _p(bar), _p(st))
    if rc != 0:
        raise ValueError("oracle_riemann rejected its arguments")
    return bar, st


def delta(dim: int, gamma: float) -> float:
    return _load().oracle_delta(dim, gamma)


def workload_bounds(wl, elems=None, r_fac=None, energy_mode=0):
    """Convenience: bounds of a synth.Workload (or a selection of its elements)."""
    g = wl.grid
    return bounds(wl.dim, wl.gamma, wl.states, wl.rowptr, wl.cols, wl.n_s, g.mode,
                  g.n[: wl.dim], g.lo, g.hi, g.k, wl.r_fac if r_fac is None else r_fac,
                  elems=elems, energy_mode=energy_mode)


def workload_limit(wl, bounds_sel, elems=None, independent=False):
    return limit(wl.dim, wl.gamma, wl.target, bounds_sel, wl.node_weights, wl.n_s, elems=elems,
                 independent=independent)
