"""Initial conditions of the 1D test problems of Sec. 6 at the Gauss-Legendre
solution points of a uniform mesh (input generation only: no part of the
scheme, the bounds or the limiter lives here).

* Sod shock tube on [0, 1], Dirichlet, diaphragm at 0.5, t = 0.2:
  (rho, u, P) = (1, 0, 1) left, (0.125, 0, 0.1) right; gamma = 1.4.
* Convecting density pulse on [-0.5, 0.5], periodic, t = 1:
  rho = 1 + exp(-sigma x^2), u = 1, P = 1, sigma = 500; gamma = 1.4.
* Leblanc shock tube on [0, 9], Dirichlet, diaphragm at 3, t = 6:
  (rho, u, P) = (1, 0, (gamma-1) 1e-1) left, (1e-3, 0, (gamma-1) 1e-10)
  right; gamma = 5/3 (the problem's usual ratio; the paper does not state it).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


@dataclass
class Problem1D:
    name: str
    p: int
    n_elem: int
    x0: float
    x1: float
    gamma: float
    bc: str                      # "periodic" or "dirichlet"
    t_end: float
    U0: np.ndarray               # [3, n_elem, p + 1] conserved states at the solution points
    x: np.ndarray                # [n_elem, p + 1] solution point coordinates
    left: Optional[np.ndarray] = None
    right: Optional[np.ndarray] = None
    riemann: Optional[Tuple] = None   # ((rho, u, P)_L, (rho, u, P)_R, x_diaphragm)
    meta: dict = field(default_factory=dict)


def solution_points(p: int, n_elem: int, x0: float, x1: float) -> np.ndarray:
    xi, _ = np.polynomial.legendre.leggauss(p + 1)
    h = (x1 - x0) / n_elem
    return (x0 + h * np.arange(n_elem))[:, None] + 0.5 * h * (xi[None, :] + 1.0)


def _cons(rho, u, P, gamma):
    rho = np.asarray(rho, dtype=np.float64)
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), rho.shape)
    P = np.broadcast_to(np.asarray(P, dtype=np.float64), rho.shape)
    return np.stack([rho, rho * u, P / (gamma - 1.0) + 0.5 * rho * u * u])


def _shock_tube(name, p, n_elem, x0, x1, xd, WL, WR, gamma, t_end):
    x = solution_points(p, n_elem, x0, x1)
    left = x <= xd
    rho = np.where(left, WL[0], WR[0])
    u = np.where(left, WL[1], WR[1])
    P = np.where(left, WL[2], WR[2])
    return Problem1D(name, p, n_elem, x0, x1, gamma, "dirichlet", t_end, _cons(rho, u, P, gamma),
                     x, left=_cons(np.array(WL[0]), WL[1], WL[2], gamma),
                     right=_cons(np.array(WR[0]), WR[1], WR[2], gamma),
                     riemann=(WL, WR, xd))


def sod(p: int, n_elem: int) -> Problem1D:
    return _shock_tube("sod", p, n_elem, 0.0, 1.0, 0.5, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, 0.2)


def leblanc(p: int, n_elem: int) -> Problem1D:
    g = 5.0 / 3.0
    return _shock_tube("leblanc", p, n_elem, 0.0, 9.0, 3.0, (1.0, 0.0, (g - 1.0) * 1e-1),
                       (1e-3, 0.0, (g - 1.0) * 1e-10), g, 6.0)


def pulse(p: int, n_elem: int, sigma: float = 500.0, t: float = 0.0) -> Problem1D:
    """The pulse at time t (exact: the initial profile translated by t)."""
    x = solution_points(p, n_elem, -0.5, 0.5)
    xs = (x - t + 0.5) % 1.0 - 0.5
    U = _cons(1.0 + np.exp(-sigma * xs * xs), 1.0, 1.0, 1.4)
    return Problem1D("pulse", p, n_elem, -0.5, 0.5, 1.4, "periodic", 1.0, U, x,
                     meta={"sigma": sigma})
