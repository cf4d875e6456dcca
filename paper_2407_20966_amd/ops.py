"""PyTorch-facing calls of libkbl: tensors in, tensors out, nothing computed here.

Every function checks tensor placement/dtype/layout, allocates outputs with
torch, and forwards raw device pointers plus torch's current HIP stream to
the C-ABI in include/kbl.h.  All arithmetic runs in the HIP kernels.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import torch

from . import _lib as L


def make_params(gamma: float, r_fac: float = 1e-3, rho_floor: float = 1e-12,
                p_floor: float = 1e-12, eps_alpha: float = 1e-13,
                precision: int = L.PREC_FP64, independent_alpha: bool = False,
                energy_perstate: bool = False) -> L.Params:
    p = L.Params()
    L.lib().kbl_default_params(C.byref(p), float(gamma))
    p.r_fac = float(r_fac)
    p.rho_floor = float(rho_floor)
    p.p_floor = float(p_floor)
    p.eps_alpha = float(eps_alpha)
    p.precision = int(precision)
    p.flags = ((L.FLAG_INDEPENDENT_ALPHA if independent_alpha else 0)
               | (L.FLAG_ENERGY_PERSTATE if energy_perstate else 0))
    return p


def make_vgrid(mode: int, n: Sequence[int], lo: Sequence[float] = (0.0, 0.0, 0.0),
               hi: Sequence[float] = (0.0, 0.0, 0.0), k: float = 4.0) -> L.VGrid:
    """Velocity grid (Sec. 3.7): nodes per direction `n` (one entry per
    dimension), the GLOBAL box [lo, hi], or the STENCIL extent `k`."""
    g = L.VGrid()
    g.mode = int(mode)
    nn = list(n) + [2] * (3 - len(n))
    lo = list(lo) + [0.0] * (3 - len(lo))
    hi = list(hi) + [0.0] * (3 - len(hi))
    for j in range(3):
        g.n[j] = int(nn[j])
        g.lo[j] = float(lo[j])
        g.hi[j] = float(hi[j])
    g.k = float(k)
    return g


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device: torch.device, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return C.c_void_p(s.cuda_stream)


def _check(t: torch.Tensor, name: str, dtype: torch.dtype, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a HIP device (got {t.device})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _out(t: Optional[torch.Tensor], name: str, dtype: torch.dtype, device, shape):
    """A caller-supplied output tensor, checked like an input and for its exact
    shape (the kernels write every entry of it), or a new one."""
    if t is None:
        return torch.empty(shape, dtype=dtype, device=device)
    _check(t, name, dtype, device)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def compute_bounds(states: torch.Tensor, rowptr: torch.Tensor, cols: torch.Tensor, n_s: int,
                   vgrid: L.VGrid, params: L.Params, out: Optional[torch.Tensor] = None,
                   status: Optional[torch.Tensor] = None,
                   stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Kinetic bounds [2(d+2), n_elem] (FP64) and per-element status (int32 view of uint32)."""
    _check(states, "states", torch.float64)
    dev = states.device
    _check(rowptr, "rowptr", torch.int32, dev)
    _check(cols, "cols", torch.int32, dev)
    dim = states.shape[0] - 2
    n_elem = rowptr.numel() - 1
    if states.dim() != 2 or states.shape[1] != n_elem * n_s:
        raise ValueError(f"states must be [d+2, n_elem*n_s] = [*, {n_elem * n_s}], got {tuple(states.shape)}")
    out = _out(out, "out", torch.float64, dev, (2 * (dim + 2), n_elem))
    status = _out(status, "status", torch.int32, dev, (n_elem,))
    rc = L.lib().kbl_compute_bounds(C.byref(params), dim, n_elem, int(n_s), cols.numel(),
                                    _ptr(states), _ptr(rowptr), _ptr(cols), C.byref(vgrid),
                                    _ptr(out), _ptr(status), _stream(dev, stream))
    if rc != L.KBL_OK:
        raise L.KblError(rc, "kbl_compute_bounds")
    return out, status


def compute_bounds_nodes(states: torch.Tensor, rowptr: torch.Tensor, cols: torch.Tensor,
                         vgrid: L.VGrid, params: L.Params, out: Optional[torch.Tensor] = None,
                         status: Optional[torch.Tensor] = None,
                         stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Bounds for node-level stencils: row e of the CSR lists node ids (columns of
    `states`), e.g. an element's solution and flux points plus its neighbours'
    flux points on the shared faces."""
    _check(states, "states", torch.float64)
    dev = states.device
    _check(rowptr, "rowptr", torch.int32, dev)
    _check(cols, "cols", torch.int32, dev)
    dim = states.shape[0] - 2
    n_elem = rowptr.numel() - 1
    if states.dim() != 2:
        raise ValueError("states must be [d+2, n_nodes]")
    out = _out(out, "out", torch.float64, dev, (2 * (dim + 2), n_elem))
    status = _out(status, "status", torch.int32, dev, (n_elem,))
    rc = L.lib().kbl_compute_bounds_nodes(C.byref(params), dim, n_elem, states.shape[1],
                                          cols.numel(), _ptr(states), _ptr(rowptr), _ptr(cols),
                                          C.byref(vgrid), _ptr(out), _ptr(status),
                                          _stream(dev, stream))
    if rc != L.KBL_OK:
        raise L.KblError(rc, "kbl_compute_bounds_nodes")
    return out, status


def riemann_states(states: torch.Tensor, node_i: torch.Tensor, node_j: torch.Tensor,
                   normals: torch.Tensor, params: L.Params, lam: Optional[torch.Tensor] = None,
                   bounds: Optional[torch.Tensor] = None, elem: Optional[torch.Tensor] = None,
                   stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Riemann-averaged states (Thm. 4.3) of node pairs and their KBL_RS_* status
    against the bounds of each pair's element (see kbl_riemann_states)."""
    _check(states, "states", torch.float64)
    dev = states.device
    _check(node_i, "node_i", torch.int32, dev)
    _check(node_j, "node_j", torch.int32, dev)
    _check(normals, "normals", torch.float64, dev)
    dim = states.shape[0] - 2
    n_pairs = node_i.numel()
    if node_j.numel() != n_pairs or tuple(normals.shape) != (dim, n_pairs):
        raise ValueError("node_j/normals do not match node_i")
    if lam is not None:
        _check(lam, "lam", torch.float64, dev)
        if lam.numel() != n_pairs:
            raise ValueError("lam must have one entry per pair")
    n_elem = 0
    if (bounds is None) != (elem is None):
        raise ValueError("bounds and elem go together")
    if bounds is not None:
        _check(bounds, "bounds", torch.float64, dev)
        _check(elem, "elem", torch.int32, dev)
        if bounds.dim() != 2 or bounds.shape[0] != 2 * (dim + 2):
            raise ValueError(f"bounds must be [2(d+2), n_elem] = [{2 * (dim + 2)}, *]")
        if elem.numel() != n_pairs:
            raise ValueError("elem must have one entry per pair")
        n_elem = bounds.shape[1]
    bar = torch.empty((dim + 2, n_pairs), dtype=torch.float64, device=dev)
    status = torch.empty(n_pairs, dtype=torch.int32, device=dev)
    rc = L.lib().kbl_riemann_states(C.byref(params), dim, n_pairs, states.shape[1], _ptr(states),
                                    _ptr(node_i), _ptr(node_j), _ptr(normals), _ptr(lam),
                                    _ptr(bounds), _ptr(elem), n_elem, _ptr(bar), _ptr(status),
                                    _stream(dev, stream))
    if rc != L.KBL_OK:
        raise L.KblError(rc, "kbl_riemann_states")
    return bar, status


def autotune_bounds(states: torch.Tensor, rowptr: torch.Tensor, cols: torch.Tensor, n_s: int,
                    vgrid: L.VGrid, params: L.Params, sample_elems: int = 32768,
                    stream=None) -> int:
    """Times the launch configurations of compute_bounds on these inputs and keeps
    the fastest for this problem shape (see kbl_autotune_bounds).  Synchronises."""
    _check(states, "states", torch.float64)
    dev = states.device
    _check(rowptr, "rowptr", torch.int32, dev)
    _check(cols, "cols", torch.int32, dev)
    dim = states.shape[0] - 2
    n_elem = rowptr.numel() - 1
    if states.dim() != 2 or states.shape[1] != n_elem * n_s:
        raise ValueError(f"states must be [d+2, n_elem*n_s] = [*, {n_elem * n_s}]")
    out = torch.empty((2 * (dim + 2), n_elem), dtype=torch.float64, device=dev)
    status = torch.empty(n_elem, dtype=torch.int32, device=dev)
    idx = L.lib().kbl_autotune_bounds(C.byref(params), dim, n_elem, int(n_s), cols.numel(),
                                      _ptr(states), _ptr(rowptr), _ptr(cols), C.byref(vgrid),
                                      _ptr(out), _ptr(status), int(sample_elems),
                                      _stream(dev, stream))
    if idx < 0:
        raise L.KblError(L.KBL_ERR_ARG, "kbl_autotune_bounds")
    return int(idx)


def limit(solution: torch.Tensor, bounds: torch.Tensor, node_weights, n_s: int,
          params: L.Params, out: Optional[torch.Tensor] = None,
          alpha: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None,
          stream=None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """Squeeze limiter + pressure step: (limited, alpha [2, n_elem], status)."""
    _check(solution, "solution", torch.float64)
    dev = solution.device
    _check(bounds, "bounds", torch.float64, dev)
    dim = solution.shape[0] - 2
    if solution.dim() != 2 or bounds.dim() != 2:
        raise ValueError("solution and bounds must be 2D")
    n_elem = bounds.shape[1]
    if solution.shape[1] != n_elem * n_s or bounds.shape[0] != 2 * (dim + 2):
        raise ValueError("solution/bounds shapes do not match n_s and the dimension")
    w = torch.as_tensor(node_weights, dtype=torch.float64).cpu().contiguous()
    if w.numel() != n_s:
        raise ValueError("node_weights must have n_s entries")
    out = _out(out, "out", torch.float64, dev, tuple(solution.shape))
    alpha = _out(alpha, "alpha", torch.float64, dev, (2, n_elem))
    status = _out(status, "status", torch.int32, dev, (n_elem,))
    rc = L.lib().kbl_limit(C.byref(params), dim, n_elem, int(n_s), _ptr(solution), _ptr(bounds),
                           C.c_void_p(w.data_ptr()), _ptr(out), _ptr(alpha), _ptr(status),
                           _stream(dev, stream))
    if rc != L.KBL_OK:
        raise L.KblError(rc, "kbl_limit")
    return out, alpha, status


def bounds_limit_backward(states: torch.Tensor, rowptr: torch.Tensor, cols: torch.Tensor,
                          n_s: int, vgrid: L.VGrid, params: L.Params, solution: torch.Tensor,
                          node_weights, grad_limited: torch.Tensor,
                          fwd_bounds: Optional[torch.Tensor] = None,
                          fwd_status: Optional[torch.Tensor] = None, stream=None):
    """Gradients of J(limit(solution, bounds(states))) for G = dJ/dlimited.

    Returns (dJ/dstates, dJ/dsolution, dJ/dbounds, status).  params.precision
    selects the forward that is differentiated (FP64 or a mixed form).  The
    forward's bounds and status may be passed in; otherwise they are
    recomputed.  The workspace is a torch allocation sized by
    kbl_backward_workspace_bytes.
    """
    _check(states, "states", torch.float64)
    dev = states.device
    for t, nm in ((solution, "solution"), (grad_limited, "grad_limited")):
        _check(t, nm, torch.float64, dev)
        if t.shape != states.shape:
            raise ValueError(f"{nm} must have the shape of states")
    _check(rowptr, "rowptr", torch.int32, dev)
    _check(cols, "cols", torch.int32, dev)
    dim = states.shape[0] - 2
    n_elem = rowptr.numel() - 1
    if states.dim() != 2 or states.shape[1] != n_elem * n_s:
        raise ValueError(f"states must be [d+2, n_elem*n_s] = [*, {n_elem * n_s}]")
    if (fwd_bounds is None) != (fwd_status is None):
        raise ValueError("fwd_bounds and fwd_status go together")
    if fwd_bounds is not None:
        _check(fwd_bounds, "fwd_bounds", torch.float64, dev)
        _check(fwd_status, "fwd_status", torch.int32, dev)
        if tuple(fwd_bounds.shape) != (2 * (dim + 2), n_elem) or fwd_status.numel() != n_elem:
            raise ValueError("fwd_bounds/fwd_status do not match the element count")
    w = torch.as_tensor(node_weights, dtype=torch.float64).cpu().contiguous()
    nbytes = L.lib().kbl_backward_workspace_bytes(dim, n_elem, int(n_s), cols.numel())
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=dev)
    gst = torch.empty_like(states)
    gsol = torch.empty_like(states)
    gb = torch.empty((2 * (dim + 2), n_elem), dtype=torch.float64, device=dev)
    status = torch.empty(n_elem, dtype=torch.int32, device=dev)
    rc = L.lib().kbl_bounds_limit_backward(
        C.byref(params), dim, n_elem, int(n_s), cols.numel(), _ptr(states), _ptr(rowptr),
        _ptr(cols), C.byref(vgrid), _ptr(fwd_bounds), _ptr(fwd_status), _ptr(solution),
        C.c_void_p(w.data_ptr()), _ptr(grad_limited), _ptr(gst), _ptr(gsol), _ptr(gb),
        _ptr(status), _ptr(ws), ws.numel(), _stream(dev, stream))
    if rc != L.KBL_OK:
        raise L.KblError(rc, "kbl_bounds_limit_backward")
    return gst, gsol, gb, status


def status_summary(status: torch.Tensor, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """Per-bit counts [32] (int64) of a status tensor (see kbl_status_summary);
    enqueued on the stream, no host synchronisation."""
    _check(status, "status", torch.int32)
    dev = status.device
    out = _out(out, "out", torch.int64, dev, (32,))
    rc = L.lib().kbl_status_summary(_ptr(status), status.numel(), _ptr(out),
                                    _stream(dev, stream))
    if rc != L.KBL_OK:
        raise L.KblError(rc, "kbl_status_summary")
    return out


class KineticBoundsLimit(torch.autograd.Function):
    """limited = limit(solution, bounds(states)) with the hand-written backward.

    Gradients flow to `states` (through the kinetic bounds) and to `solution`
    (through the limiter).  Besides the inputs only the bounds and their
    status (2(d+2) + 1 numbers per element) are kept; the min/max
    distributions are recomputed in the backward.
    """

    @staticmethod
    def forward(ctx, states, solution, rowptr, cols, n_s, vgrid, params, node_weights):
        bounds, bstatus = compute_bounds(states, rowptr, cols, n_s, vgrid, params)
        limited, _, _ = limit(solution, bounds, node_weights, n_s, params)
        ctx.save_for_backward(states, solution, rowptr, cols, bounds, bstatus)
        ctx.n_s, ctx.vgrid, ctx.params, ctx.node_weights = n_s, vgrid, params, node_weights
        return limited

    @staticmethod
    def backward(ctx, grad_limited):
        states, solution, rowptr, cols, bounds, bstatus = ctx.saved_tensors
        gst, gsol, _, _ = bounds_limit_backward(states, rowptr, cols, ctx.n_s, ctx.vgrid,
                                                ctx.params, solution, ctx.node_weights,
                                                grad_limited.contiguous(), fwd_bounds=bounds,
                                                fwd_status=bstatus)
        return gst, gsol, None, None, None, None, None, None


def bounds_and_limit(states, solution, rowptr, cols, n_s, vgrid, params, node_weights):
    """Differentiable bounds + limit (see KineticBoundsLimit)."""
    return KineticBoundsLimit.apply(states, solution, rowptr, cols, n_s, vgrid, params,
                                    node_weights)
