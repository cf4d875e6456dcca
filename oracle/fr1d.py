"""Plain FP64 reference of a one-dimensional flux reconstruction (FR) Euler
solver with the kinetic bounds and squeeze limiter after every Runge-Kutta
stage: the numerical setup of Sec. 5 in 1D.

TEST INFRASTRUCTURE ONLY.  Used by the test suite (and nothing in the
library); it shares no code with the HIP solver.  Written from the
definitions, slow and direct:

* Solution points: the p + 1 Gauss-Legendre nodes of each element; flux
  points: the two element ends (an open node set, Sec. 5).
* FR (Huynh's flux reconstruction with the DG correction functions, i.e. the
  left/right Radau polynomials g_L = (-1)^p/2 (P_p - P_{p+1}),
  g_R(x) = g_L(-x)): the discontinuous flux is the Lagrange interpolant of
  the point fluxes; at each element end it is corrected to the common
  interface flux,
      du_j/dt = -(2/h) [ sum_k D_jk F_k + (F*_L - f_L) g_L'(x_j)
                                        + (F*_R - f_R) g_R'(x_j) ].
* Common interface flux: HLLC (Toro, Spruce and Speares 1994) with the
  wave-speed estimates S_L = min(u_L - c_L, u_R - c_R),
  S_R = max(u_L + c_L, u_R + c_R).
* Time: three-stage third-order SSP Runge-Kutta (Shu-Osher form), with the
  limiter applied after every stage (Sec. 5).
* Limiter: every stage follows the overview of Sec. 3.9: the bounds are
  taken from the stage's input state over the node stencil S = the
  element's solution points and both end values plus the neighbours' end
  values on the shared faces; the updated state is then limited (squeeze
  limiter and pressure step) over V = the element's solution points and end
  values, with zero mean weight on the end values (Sec. 5; the bounds and
  limiter of Sec. 3 from the ``oracle`` package).  Initial data: elements
  with a non-admissible node value are limited once into the bounds of the
  solution points of the element and its two face neighbours.
* Boundaries: periodic, or Dirichlet through constant ghost states on both
  sides (the common flux at a boundary face is the HLLC flux against the
  ghost state, and the ghost's end value joins the boundary element's
  stencil).
"""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
from numpy.polynomial import legendre as _leg
from numpy.polynomial import polynomial as _pw

from . import bounds as _bounds
from . import limit as _limit

GRID_STENCIL = 1


def gl_nodes(p: int):
    """Gauss-Legendre nodes and weights on [-1, 1] (p + 1 points)."""
    return _leg.leggauss(p + 1)


def lagrange_operators(xi: np.ndarray):
    """Values of the Lagrange basis of the nodes xi at -1 and +1, and the
    differentiation matrix D[j, k] = l_k'(xi_j)."""
    n = xi.size
    basis = []
    for k in range(n):
        others = np.delete(xi, k)
        basis.append(_pw.polyfromroots(others) / np.prod(xi[k] - others))
    at_m1 = np.array([_pw.polyval(-1.0, c) for c in basis])
    at_p1 = np.array([_pw.polyval(1.0, c) for c in basis])
    D = np.array([[_pw.polyval(xi[j], _pw.polyder(basis[k])) for k in range(n)]
                  for j in range(n)])
    return at_m1, at_p1, D


def correction_functions(p: int):
    """Legendre-series coefficients of Huynh's DG correction functions
    g_L = (-1)^p/2 (P_p - P_{p+1}) and g_R(x) = g_L(-x) = (P_p + P_{p+1})/2."""
    cp = np.zeros(p + 2)
    cp[p] = 1.0
    cq = np.zeros(p + 2)
    cq[p + 1] = 1.0
    gL = (-1.0) ** p * 0.5 * (cp - cq)
    gR = 0.5 * (cp + cq)
    return gL, gR


def pressure(U: np.ndarray, gamma: float) -> np.ndarray:
    rho, m, E = U[0], U[1], U[2]
    return (gamma - 1.0) * (E - 0.5 * m * m / rho)


def euler_flux(U: np.ndarray, gamma: float) -> np.ndarray:
    """Euler flux (Sec. 2.1) of conserved states [3, ...]."""
    rho, m, E = U[0], U[1], U[2]
    u = m / rho
    P = pressure(U, gamma)
    return np.stack([m, m * u + P, (E + P) * u])


def hllc_flux(UL: np.ndarray, UR: np.ndarray, gamma: float) -> np.ndarray:
    """HLLC flux (Toro, Spruce and Speares 1994) for left/right states [3, n]."""
    rl, ml, El = UL
    rr, mr, Er = UR
    ul, ur = ml / rl, mr / rr
    pl, pr = pressure(UL, gamma), pressure(UR, gamma)
    cl, cr = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
    SL = np.minimum(ul - cl, ur - cr)
    SR = np.maximum(ul + cl, ur + cr)
    Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur))
    FL, FR = euler_flux(UL, gamma), euler_flux(UR, gamma)

    def star(r, u, p, E, S):
        f = r * (S - u) / (S - Ss)
        return np.stack([f, f * Ss, f * (E / r + (Ss - u) * (Ss + p / (r * (S - u))))])

    FsL = FL + SL * (star(rl, ul, pl, El, SL) - UL)
    FsR = FR + SR * (star(rr, ur, pr, Er, SR) - UR)
    return np.where(0.0 <= SL, FL, np.where(0.0 <= Ss, FsL, np.where(0.0 <= SR, FsR, FR)))


class FR1D:
    """Plain FR solver on n_elem uniform elements of [x0, x1].

    Solution arrays are [3, n_elem, p + 1] conserved states at the solution
    points.  bc is "periodic" or "dirichlet" (with left/right conserved
    states)."""

    def __init__(self, p: int, n_elem: int, x0: float, x1: float, gamma: float,
                 bc: str = "periodic", left: Optional[Sequence[float]] = None,
                 right: Optional[Sequence[float]] = None):
        self.p, self.n_elem, self.gamma, self.bc = p, n_elem, gamma, bc
        self.x0, self.x1 = x0, x1
        self.h = (x1 - x0) / n_elem
        self.xi, self.w = gl_nodes(p)
        self.at_m1, self.at_p1, self.D = lagrange_operators(self.xi)
        gL, gR = correction_functions(p)
        self.dgL = _leg.legval(self.xi, _leg.legder(gL))
        self.dgR = _leg.legval(self.xi, _leg.legder(gR))
        self.left = None if left is None else np.asarray(left, dtype=np.float64)
        self.right = None if right is None else np.asarray(right, dtype=np.float64)
        if bc == "dirichlet":
            assert self.left is not None and self.right is not None
        elif bc != "periodic":
            raise ValueError(bc)

    def node_x(self) -> np.ndarray:
        """Physical coordinates of the solution points [n_elem, p + 1]."""
        xl = self.x0 + self.h * np.arange(self.n_elem)
        return xl[:, None] + 0.5 * self.h * (self.xi[None, :] + 1.0)

    def faces(self, U):
        """Left and right end values [3, n_elem] of the solution polynomials."""
        return U @ self.at_m1, U @ self.at_p1

    def rhs(self, U: np.ndarray) -> np.ndarray:
        g = self.gamma
        F = euler_flux(U, g)
        uL, uR = self.faces(U)
        fL, fR = F @ self.at_m1, F @ self.at_p1
        # common flux at the right end of every element
        nxt = np.roll(uL, -1, axis=1)
        if self.bc == "dirichlet":
            nxt[:, -1] = self.right
        Fs_right = hllc_flux(uR, nxt, g)
        if self.bc == "periodic":
            Fs_left = np.roll(Fs_right, 1, axis=1)
        else:
            Fs_left = np.empty_like(Fs_right)
            Fs_left[:, 1:] = Fs_right[:, :-1]
            Fs_left[:, 0] = hllc_flux(self.left[:, None], uL[:, :1], g)[:, 0]
        dF = np.einsum("jk,vek->vej", self.D, F)
        corr = ((Fs_left - fL)[:, :, None] * self.dgL[None, None, :]
                + (Fs_right - fR)[:, :, None] * self.dgR[None, None, :])
        return -(2.0 / self.h) * (dF + corr)

    # ------------------------------------------------------------- limiter
    def stencil_layout(self, initial: bool = False):
        """V-layout node numbering and the node-stencil CSR.

        Every element (and, with Dirichlet boundaries, one constant ghost
        element on each side, numbered n_elem and n_elem + 1) owns p + 3
        consecutive nodes: its p + 1 solution points, then its left and right
        end values.  Row e lists the element's own nodes and the neighbours'
        end values on the two shared faces (Sec. 5).  With initial=True row e
        lists the solution points of the element and of its two face
        neighbours instead (used once, on initial data).  Ghost rows list
        their own nodes."""
        n_s = self.p + 1
        n_v = n_s + 2
        n_tot = self.n_elem + (2 if self.bc == "dirichlet" else 0)
        rows = []
        for e in range(self.n_elem):
            if self.bc == "periodic":
                lnb, rnb = (e - 1) % self.n_elem, (e + 1) % self.n_elem
            else:
                lnb = e - 1 if e > 0 else self.n_elem
                rnb = e + 1 if e < self.n_elem - 1 else self.n_elem + 1
            if initial:
                rows.append([q * n_v + j for q in (e, lnb, rnb) for j in range(n_s)])
            else:
                rows.append(list(e * n_v + np.arange(n_v)) + [lnb * n_v + n_s + 1, rnb * n_v + n_s])
        for e in range(self.n_elem, n_tot):
            rows.append(list(e * n_v + np.arange(n_v)))
        rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
        cols = np.concatenate(rows).astype(np.int32)
        return n_v, n_tot, rowptr, cols

    def v_states(self, U: np.ndarray) -> np.ndarray:
        """States in the V layout [3, n_tot * (p + 3)]."""
        n_v, n_tot, _, _ = self.stencil_layout()
        uL, uR = self.faces(U)
        V = np.concatenate([U, uL[:, :, None], uR[:, :, None]], axis=2)
        if self.bc == "dirichlet":
            ghosts = np.stack([np.repeat(self.left[:, None], n_v, 1),
                               np.repeat(self.right[:, None], n_v, 1)], axis=1)
            V = np.concatenate([V, ghosts], axis=1)
        return np.ascontiguousarray(V.reshape(3, n_tot * n_v))

    def bounds(self, U: np.ndarray, n_u: int = 2048, k: float = 8.0, r_fac: float = 1e-3,
               initial: bool = False):
        """Kinetic bounds [6, n_tot] and status of every node stencil of U
        (steps 1-3 of the overview in Sec. 3.9)."""
        _, _, rowptr, cols = self.stencil_layout(initial)
        V = self.v_states(U)
        return _bounds(1, self.gamma, V, rowptr, cols, 1, GRID_STENCIL, (n_u,), k=k,
                       r_fac=r_fac, n_src=V.shape[1])

    def limit_into(self, U: np.ndarray, b: np.ndarray, return_info: bool = False):
        """Squeeze limiter and pressure step of U over V into the bounds b
        (steps 5-7 of Sec. 3.9); end values carry zero mean weight."""
        n_v, n_tot, _, _ = self.stencil_layout()
        V = self.v_states(U)
        cw = np.concatenate([self.w, [0.0, 0.0]])
        lim, alpha, lst = _limit(1, self.gamma, V, b, cw, n_v)
        out = lim.reshape(3, n_tot, n_v)[:, :self.n_elem, :self.p + 1].copy()
        return (out, alpha, lst) if return_info else out

    def limit_initial(self, U: np.ndarray, n_u: int = 2048, k: float = 8.0,
                      r_fac: float = 1e-3) -> np.ndarray:
        """Initial data: an element whose polynomial has a non-admissible node
        value (rho <= 0 or P <= 0 at a solution point or end value, as the
        end values of discontinuous data can) is limited into the bounds of
        the solution points of the element and its two face neighbours; every
        other element is left as it is (NaN bounds pass it through)."""
        b, _ = self.bounds(U, n_u, k, r_fac, initial=True)
        n_v, n_tot, _, _ = self.stencil_layout()
        V = self.v_states(U).reshape(3, n_tot, n_v)
        good = ((V[0] > 0) & (pressure(V, self.gamma) > 0)).all(1)
        b = b.copy()
        b[:, good] = np.nan
        return self.limit_into(U, b)

    # ------------------------------------------------------------- time
    def step(self, U: np.ndarray, dt: float, limiter: bool = True, n_u: int = 2048,
             k: float = 8.0, r_fac: float = 1e-3) -> np.ndarray:
        """One SSP-RK3 step.  Every stage follows Sec. 3.9: bounds from the
        stage's input state, the update, then the limiting of the updated
        state into those bounds."""
        def stage(Uin, combine):
            b = self.bounds(Uin, n_u, k, r_fac)[0] if limiter else None
            Unew = combine(Uin + dt * self.rhs(Uin))
            return self.limit_into(Unew, b) if limiter else Unew

        U1 = stage(U, lambda y: y)
        U2 = stage(U1, lambda y: 0.75 * U + 0.25 * y)
        return stage(U2, lambda y: (1.0 / 3.0) * U + (2.0 / 3.0) * y)

    def max_speed(self, U: np.ndarray) -> float:
        u = U[1] / U[0]
        c = np.sqrt(self.gamma * pressure(U, self.gamma) / U[0])
        return float(np.max(np.abs(u) + c))

    def mean(self, U: np.ndarray) -> np.ndarray:
        """Element means [3, n_elem] (Gauss-Legendre weights)."""
        return 0.5 * U @ self.w


def conserved(rho, u, P, gamma):
    rho = np.asarray(rho, dtype=np.float64)
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), rho.shape)
    P = np.broadcast_to(np.asarray(P, dtype=np.float64), rho.shape)
    return np.stack([rho, rho * u, P / (gamma - 1.0) + 0.5 * rho * u * u])
