"""1D flux reconstruction Euler solver with the kinetic bounds and squeeze
limiter after every SSP-RK3 stage (include/kbl_fr1d.h).  Argument
marshalling and the time loop only: every step runs in libkbl.so."""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import _lib as L
from .ops import make_params, make_vgrid


class FR1D:
    """Solver state on one HIP device.

    The state tensor ``U`` is [3, columns] in the layout of kbl_fr1d.h
    (p + 3 nodes per element: p + 1 Gauss-Legendre solution points, then the
    left and right end values; two ghost elements with Dirichlet
    boundaries)."""

    def __init__(self, p: int, n_elem: int, x0: float, x1: float, gamma: float = 1.4,
                 bc: str = "periodic", left: Optional[Sequence[float]] = None,
                 right: Optional[Sequence[float]] = None, limit: bool = True,
                 r_fac: float = 1e-3, n_u: int = 2048, k: float = 8.0,
                 device: str = "cuda:0", stream=None):
        cfg = L.Fr1dCfg()
        cfg.p = int(p)
        cfg.bc = L.FR_PERIODIC if bc == "periodic" else L.FR_DIRICHLET
        cfg.n_elem = int(n_elem)
        cfg.x0, cfg.x1 = float(x0), float(x1)
        for v in range(3):
            cfg.left[v] = 0.0 if left is None else float(left[v])
            cfg.right[v] = 0.0 if right is None else float(right[v])
        cfg.limit = 1 if limit else 0
        self.cfg = cfg
        self.p, self.n_elem, self.gamma = int(p), int(n_elem), float(gamma)
        self.n_v = self.p + 3
        lib = L.lib()
        cols = lib.kbl_fr1d_columns(C.byref(cfg))
        if cols <= 0:
            raise L.KblError(L.KBL_ERR_ARG, "kbl_fr1d_columns")
        self.cols = int(cols)
        self.device = torch.device(device)
        self.U = torch.zeros((3, self.cols), dtype=torch.float64, device=self.device)
        self.R = torch.empty((3, self.n_elem * (self.p + 1)), dtype=torch.float64,
                             device=self.device)
        self.ws = torch.empty(lib.kbl_fr1d_workspace_bytes(C.byref(cfg)), dtype=torch.uint8,
                              device=self.device)
        self.status = torch.zeros(self.cols // self.n_v, dtype=torch.int32, device=self.device)
        self._speed = torch.empty(1, dtype=torch.float64, device=self.device)
        self.params = make_params(gamma, r_fac=r_fac)
        self.vgrid = make_vgrid(L.GRID_STENCIL, (n_u,), k=k)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _check(self, rc, where):
        if rc != L.KBL_OK:
            raise L.KblError(rc, where)

    # solution points of the real elements [3, n_elem, p + 1]
    def solution_view(self) -> torch.Tensor:
        n = self.n_elem * self.n_v
        return self.U[:, :n].view(3, self.n_elem, self.n_v)[:, :, :self.p + 1]

    def set_solution(self, Us) -> None:
        """Writes the solution points (array-like [3, n_elem, p + 1]) and
        limits them (end values and ghosts are written too)."""
        t = torch.as_tensor(Us, dtype=torch.float64).to(self.device)
        if tuple(t.shape) != (3, self.n_elem, self.p + 1):
            raise ValueError(f"expected [3, {self.n_elem}, {self.p + 1}], got {tuple(t.shape)}")
        self.solution_view().copy_(t)
        self.limit()

    def solution(self) -> torch.Tensor:
        return self.solution_view().clone()

    def rhs(self) -> torch.Tensor:
        self._check(L.lib().kbl_fr1d_rhs(C.byref(self.cfg), self.gamma,
                                         C.c_void_p(self.U.data_ptr()),
                                         C.c_void_p(self.R.data_ptr()), self._s()),
                    "kbl_fr1d_rhs")
        return self.R.view(3, self.n_elem, self.p + 1)

    def limit(self) -> None:
        self._check(L.lib().kbl_fr1d_limit(C.byref(self.cfg), C.byref(self.params),
                                           C.byref(self.vgrid), C.c_void_p(self.U.data_ptr()),
                                           C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                           C.c_void_p(self.status.data_ptr()), self._s()),
                    "kbl_fr1d_limit")

    def step(self, dt: float) -> None:
        self._check(L.lib().kbl_fr1d_step(C.byref(self.cfg), C.byref(self.params),
                                          C.byref(self.vgrid), float(dt),
                                          C.c_void_p(self.U.data_ptr()),
                                          C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                          C.c_void_p(self.status.data_ptr()), self._s()),
                    "kbl_fr1d_step")

    def max_speed(self) -> float:
        self._check(L.lib().kbl_fr1d_max_speed(C.byref(self.cfg), self.gamma,
                                               C.c_void_p(self.U.data_ptr()),
                                               C.c_void_p(self._speed.data_ptr()), self._s()),
                    "kbl_fr1d_max_speed")
        return float(self._speed.item())

    def _device_step(self, tdt: torch.Tensor, cfl: float, t_end: float, stream) -> None:
        lib = L.lib()
        sp = C.c_void_p(stream.cuda_stream)
        self._check(lib.kbl_fr1d_cfl_dt(C.byref(self.cfg), self.gamma,
                                        C.c_void_p(self.U.data_ptr()), float(cfl), float(t_end),
                                        C.c_void_p(tdt.data_ptr()), sp), "kbl_fr1d_cfl_dt")
        self._check(lib.kbl_fr1d_step_dev(C.byref(self.cfg), C.byref(self.params),
                                          C.byref(self.vgrid), C.c_void_p(tdt.data_ptr()),
                                          C.c_void_p(self.U.data_ptr()),
                                          C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                          C.c_void_p(self.status.data_ptr()), sp),
                    "kbl_fr1d_step_dev")

    def run_device(self, t_end: float, cfl: float, batch: int = 0,
                   max_steps: int = 10_000_000) -> int:
        """As run(), with the time step computed on the device (no host sync
        per step).  batch > 0: batches of that many steps are captured once
        in a HIP graph and replayed while the end time is more than two
        batches away; the remaining steps run one by one.  Returns the
        number of steps."""
        tdt = torch.zeros(2, dtype=torch.float64, device=self.device)
        graph = None
        if batch > 0:
            graph = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream(self.device)
            side.wait_stream(self.stream)
            with torch.cuda.graph(graph, stream=side):
                for _ in range(batch):
                    self._device_step(tdt, cfl, t_end, side)
            self.stream.wait_stream(side)
        n = 0
        while n < max_steps:
            t, dt = (float(v) for v in tdt.tolist())
            if not (t == t and dt == dt):
                raise FloatingPointError(f"non-admissible state after {n} steps")
            if t >= t_end:
                break
            if graph is not None and n > 0 and t + 2.0 * batch * dt < t_end:
                graph.replay()
                n += batch
            else:
                self._device_step(tdt, cfl, t_end, self.stream)
                n += 1
        return n

    def run(self, t_end: float, cfl: float, max_steps: int = 10_000_000) -> int:
        """Steps to t_end with dt = cfl * h / ((2p + 1) max|u| + c).
        Returns the number of steps; raises if the state stops being admissible."""
        h = (self.cfg.x1 - self.cfg.x0) / self.n_elem
        t, n = 0.0, 0
        while t < t_end * (1.0 - 1e-14) and n < max_steps:
            s = self.max_speed()
            if not (s == s) or s <= 0.0:
                raise FloatingPointError(f"non-admissible state after {n} steps (t = {t})")
            dt = min(cfl * h / ((2 * self.p + 1) * s), t_end - t)
            self.step(dt)
            t += dt
            n += 1
        return n
