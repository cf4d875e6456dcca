"""Error metrics for GPU-vs-oracle parity (no bounds/limiter arithmetic here).

Relative error is taken against |reference| for density and energy (both
positive), and against an element momentum scale for momentum, whose bounds
can be near zero: s_m = max over the element's stencil nodes of
|m|_1 + sqrt(rho E)  (|m| <= sqrt(2 rho E) for admissible states).
"""

from __future__ import annotations

import numpy as np


def stencil_momentum_scale(wl, elems=None):
    """Per element: max over stencil nodes of |m|_1 + sqrt(rho*E)."""
    d = wl.dim
    st = wl.states
    node_scale = np.abs(st[1:1 + d]).sum(0) + np.sqrt(np.abs(st[0] * st[d + 1]))
    el = node_scale.reshape(wl.n_elem, wl.n_s).max(1)
    starts = wl.rowptr[:-1].astype(np.int64)
    sizes = np.diff(wl.rowptr.astype(np.int64))
    cols = np.clip(wl.cols, 0, wl.n_elem - 1)      # rows with bad ids are excluded by callers
    full = np.maximum.reduceat(el[cols], starts)
    full[sizes == 0] = 0.0
    return full if elems is None else full[elems]


def node_stencil_momentum_scale(states, rowptr, cols, dim, elems):
    """Node-level stencils: max over the listed nodes of |m|_1 + sqrt(rho*E)."""
    node_scale = np.abs(states[1:1 + dim]).sum(0) + np.sqrt(np.abs(states[0] * states[dim + 1]))
    return np.array([node_scale[cols[rowptr[e]:rowptr[e + 1]]].max() for e in elems])


def element_value_scale(wl, arr, elems=None):
    """Per (variable, element): max |arr| over the element's nodes, momentum rows
    floored by sqrt(rho E) of the element."""
    d = wl.dim
    a = np.abs(arr).reshape(d + 2, wl.n_elem, wl.n_s).max(2)
    rhoE = np.sqrt(np.abs(arr[0] * arr[d + 1])).reshape(wl.n_elem, wl.n_s).max(1)
    a[1:1 + d] = np.maximum(a[1:1 + d], rhoE)
    return a if elems is None else a[:, elems]


def bounds_error(got, ref, dim, mscale):
    """Max normalised error over all bound rows; NaN must match NaN."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nv = dim + 2
    nan_g, nan_r = np.isnan(got), np.isnan(ref)
    assert np.array_equal(nan_g, nan_r), "NaN pattern differs"
    err = np.zeros_like(ref)
    ok = ~nan_r
    for row in range(2 * nv):
        v = row % nv
        denom = np.abs(ref[row]) if v in (0, nv - 1) else np.maximum(np.abs(ref[row]), mscale)
        denom = np.where(denom > 0, denom, 1.0)
        err[row] = np.where(ok[row], np.abs(got[row] - ref[row]) / denom, 0.0)
    return float(err.max()) if err.size else 0.0, err


def limited_error(got, ref, scale_ve, n_s):
    """Max error of limited nodes normalised by the element value scale."""
    nv = got.shape[0]
    n_el = got.shape[1] // n_s
    g = got.reshape(nv, n_el, n_s)
    r = ref.reshape(nv, n_el, n_s)
    denom = np.where(scale_ve > 0, scale_ve, 1.0)[:, :, None]
    err = np.abs(g - r) / denom
    return float(err.max()) if err.size else 0.0, err
