"""Seeded synthetic meshes, stencils and shock-laden Euler fields.

Every array here is an *input*: nodal conserved states ``[rho, m_1..m_d, E]``
(SoA, ``[d+2][n_elem*n_s]``, element-major nodes), an element-level stencil
in CSR form (self included, self first), positive element quadrature
weights, a velocity-grid description and a target solution to be limited.

Shapes and value ranges follow the discretisations the paper runs (Sec. 5:
Gauss-Legendre solution nodes on lines/quads, triangles with a positive
interior nodal rule, uniform trapezoid velocity grids with k=4) and the
shock tubes of Sec. 6 (Sod-type jumps, Leblanc-type ratios).  No dataset is
read: all fields are generated from seeds (PCG64).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, Optional, Tuple

import numpy as np

BASE_SEED = 240720966

GRID_GLOBAL = 0
GRID_STENCIL = 1


@dataclass
class GridSpec:
    """Velocity-grid description.

    mode GLOBAL uses the same box ``[lo, hi]`` for every element; mode STENCIL
    lets the consumer derive the box per element from its stencil with extent
    factor ``k``.  ``n`` counts nodes per direction, endpoints included.
    """

    mode: int
    n: Tuple[int, ...]
    lo: Tuple[float, ...] = (0.0, 0.0)
    hi: Tuple[float, ...] = (0.0, 0.0)
    k: float = 4.0


@dataclass
class Workload:
    name: str
    dim: int
    gamma: float
    n_elem: int
    n_s: int
    states: np.ndarray          # [dim+2, n_elem*n_s] float64 (stencil states)
    target: np.ndarray          # [dim+2, n_elem*n_s] float64 (solution to limit)
    rowptr: np.ndarray          # int32 [n_elem+1]
    cols: np.ndarray            # int32 [nnz]
    node_weights: np.ndarray    # float64 [n_s] > 0
    grid: GridSpec
    r_fac: float = 1e-3
    seed: int = BASE_SEED
    meta: Dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return self.n_elem * self.n_s

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def stencil_sizes(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def n_vel(self) -> int:
        return int(np.prod(self.grid.n[: self.dim]))

    def pairs(self) -> int:
        """(stencil state, velocity node) pairs one bounds pass evaluates."""
        return int(self.stencil_sizes().sum()) * self.n_s * self.n_vel()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _to_conserved(gamma: float, rho, vel, p) -> np.ndarray:
    """Primitive (rho, U, p) -> conserved rows [rho, rho*U..., E]."""
    vel = [np.asarray(v, dtype=np.float64) for v in vel]
    ke = 0.5 * rho * sum(v * v for v in vel)
    rows = [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke]
    return np.stack([np.ascontiguousarray(r, dtype=np.float64).ravel() for r in rows])


def _fourier(rng: np.random.Generator, x, y, n_modes: int = 8) -> np.ndarray:
    """Smooth periodic perturbation with unit max amplitude bound."""
    out = np.zeros_like(x)
    amps = rng.uniform(0.5, 1.0, n_modes)
    kx = rng.integers(-4, 5, n_modes)
    ky = rng.integers(-4, 5, n_modes)
    ph = rng.uniform(0.0, 2 * np.pi, n_modes)
    for a, i, j, f in zip(amps, kx, ky, ph):
        out = out + a * np.sin(2 * np.pi * (i * x + j * y) + f)
    return out / amps.sum()


def _limit_target(rng, states, rowptr, cols, n_s, weights, jump_ratio=1.5,
                  amp_jump=0.05, amp_smooth=2e-3):
    """W' = W + Delta with Delta of zero weighted element mean.

    Delta_{v,j} = A_e * R_{e,v} * s_{v,j}; R is the stencil range of variable
    v, A_e is larger where the stencil density ratio exceeds ``jump_ratio``,
    s is a seeded +-1 pattern projected to zero weighted mean.
    """
    nv, n_nodes = states.shape
    n_elem = n_nodes // n_s
    per_el = states.reshape(nv, n_elem, n_s)
    el_max = per_el.max(axis=2)
    el_min = per_el.min(axis=2)
    starts = rowptr[:-1].astype(np.int64)
    smax = np.maximum.reduceat(el_max[:, cols], starts, axis=1)
    smin = np.minimum.reduceat(el_min[:, cols], starts, axis=1)
    rng_v = smax - smin                                   # [nv, n_elem]
    ratio = smax[0] / smin[0]
    amp = np.where(ratio > jump_ratio, amp_jump, amp_smooth)  # [n_elem]
    s = rng.choice(np.array([-1.0, 1.0]), size=(nv, n_elem, n_s))
    w = weights / weights.sum()
    s = s - (s * w).sum(axis=2, keepdims=True)
    delta = amp[None, :, None] * rng_v[:, :, None] * s
    target = (per_el + delta).reshape(nv, n_nodes)
    return np.ascontiguousarray(target), ratio > jump_ratio


# ----------------------------------------------------------------------------
# 1D periodic line, Gauss-Legendre nodes, self + 2 face neighbours.
# ----------------------------------------------------------------------------

def make_line_workload(n_elem: int = 64, p: int = 3, seed: int = BASE_SEED,
                       grid_nodes: int = 64, extent: float = 12.0,
                       gamma: float = 1.4, r_fac: float = 1e-3,
                       jump: bool = True, name: str = "line") -> Workload:
    rng = _rng(seed)
    xi, wq = np.polynomial.legendre.leggauss(p + 1)
    n_s = p + 1
    h = 1.0 / n_elem
    x = (np.arange(n_elem)[:, None] + 0.5 * (xi[None, :] + 1.0)) * h
    phi1, phi2 = rng.uniform(0.0, 2 * np.pi, 2)
    xs = (n_elem // 2 + rng.uniform(0.2, 0.8)) * h if jump else 2.0
    left = x < xs
    rho = (1.25 + 0.75 * np.sin(2 * np.pi * x + phi1)) * np.where(left, 1.0, 0.125)
    pr = np.where(left, 1.0, 0.1)
    u = np.sin(2 * np.pi * x + phi2)
    states = _to_conserved(gamma, rho, [u], pr)
    e = np.arange(n_elem)
    cols = np.stack([e, (e - 1) % n_elem, (e + 1) % n_elem], axis=1).ravel()
    rowptr = np.arange(0, 3 * n_elem + 1, 3)
    theta_max = float((pr / rho).max())
    half = extent * np.sqrt(theta_max)
    grid = GridSpec(GRID_GLOBAL, (grid_nodes, 1), (-half, 0.0), (half, 0.0), 0.0)
    cols = cols.astype(np.int32)
    rowptr = rowptr.astype(np.int32)
    target, jumpy = _limit_target(rng, states, rowptr, cols, n_s, wq)
    return Workload(name, 1, gamma, n_elem, n_s, states, target, rowptr, cols,
                    wq.astype(np.float64), grid, r_fac, seed,
                    {"theta_max": theta_max, "jump_elems": np.nonzero(jumpy)[0]})


# ----------------------------------------------------------------------------
# 2D periodic quads, tensor Gauss-Legendre nodes, self + 4 face neighbours.
# ----------------------------------------------------------------------------

def _quad_geometry(N: int, p: int):
    xi, wq = np.polynomial.legendre.leggauss(p + 1)
    n1 = p + 1
    ex = np.arange(N)
    # element e = ey*N + ex ; node j = jy*n1 + jx
    X = (ex[None, :, None, None] + 0.5 * (xi[None, None, None, :] + 1.0)) / N
    Y = (ex[:, None, None, None] + 0.5 * (xi[None, None, :, None] + 1.0)) / N
    X = np.broadcast_to(X, (N, N, n1, n1)).reshape(N * N, n1 * n1)
    Y = np.broadcast_to(Y, (N, N, n1, n1)).reshape(N * N, n1 * n1)
    w2 = (wq[:, None] * wq[None, :]).ravel()
    ey, exx = np.divmod(np.arange(N * N), N)
    cols = np.stack([
        ey * N + exx,
        ey * N + (exx - 1) % N,
        ey * N + (exx + 1) % N,
        ((ey - 1) % N) * N + exx,
        ((ey + 1) % N) * N + exx,
    ], axis=1).ravel().astype(np.int32)
    rowptr = np.arange(0, 5 * N * N + 1, 5).astype(np.int32)
    return X, Y, w2, cols, rowptr


def quad_block_stencils(N: int, r: int):
    """CSR rows of a periodic N x N quad mesh listing every element within r
    cells in each direction, self first: (2r + 1)^2 elements per row."""
    rows = []
    for e in range(N * N):
        ey, ex = divmod(e, N)
        row = [e]
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                if dx or dy:
                    row.append(((ey + dy) % N) * N + (ex + dx) % N)
        rows.append(row)
    rowptr = np.concatenate([[0], np.cumsum([len(x) for x in rows])]).astype(np.int32)
    return rowptr, np.concatenate(rows).astype(np.int32)


def make_quad_workload(N: int = 256, p: int = 3, seed: int = BASE_SEED + 1,
                       field_kind: str = "riemann4", grid_nodes: int = 48,
                       grid_mode: int = GRID_STENCIL, k: float = 4.0,
                       extent: float = 12.0, gamma: float = 1.4,
                       r_fac: float = 1e-3, name: str = "quad") -> Workload:
    rng = _rng(seed)
    X, Y, w2, cols, rowptr = _quad_geometry(N, p)
    n_s = (p + 1) ** 2
    off = rng.uniform(0.2, 0.8, 2)
    xs = (N // 2 + off[0]) / N
    ys = (N // 2 + off[1]) / N
    if field_kind == "riemann4":
        quad = (X >= xs).astype(np.int64) + 2 * (Y >= ys).astype(np.int64)
        rho_q = np.exp(rng.uniform(np.log(0.1), np.log(10.0), 4))
        p_q = np.exp(rng.uniform(np.log(0.1), np.log(100.0), 4))
        r_q = rng.uniform(0.0, 3.0, 4)
        a_q = rng.uniform(0.0, 2 * np.pi, 4)
        rho = rho_q[quad] * (1.0 + 0.01 * _fourier(rng, X, Y))
        pr = p_q[quad] * (1.0 + 0.01 * _fourier(rng, X, Y))
        ux = (r_q * np.cos(a_q))[quad] + 0.03 * _fourier(rng, X, Y)
        uy = (r_q * np.sin(a_q))[quad] + 0.03 * _fourier(rng, X, Y)
    elif field_kind == "sine":
        ph = rng.uniform(0.0, 2 * np.pi, 3)
        left = X < xs
        rho = (1.25 + 0.75 * np.sin(2 * np.pi * (X + Y) + ph[0])) * np.where(left, 1.0, 0.125)
        pr = np.where(left, 1.0, 0.1)
        ux = np.sin(2 * np.pi * X + ph[1])
        uy = np.sin(2 * np.pi * Y + ph[2])
    else:
        raise ValueError(field_kind)
    states = _to_conserved(gamma, rho, [ux, uy], pr)
    theta_max = float((pr / rho).max())
    if grid_mode == GRID_GLOBAL:
        half = extent * np.sqrt(theta_max)
        grid = GridSpec(GRID_GLOBAL, (grid_nodes, grid_nodes), (-half, -half), (half, half), 0.0)
    else:
        grid = GridSpec(GRID_STENCIL, (grid_nodes, grid_nodes), (0.0, 0.0), (0.0, 0.0), k)
    target, jumpy = _limit_target(rng, states, rowptr, cols, n_s, w2)
    return Workload(name, 2, gamma, N * N, n_s, states, target, rowptr, cols,
                    w2.astype(np.float64), grid, r_fac, seed,
                    {"theta_max": theta_max, "jump_elems": np.nonzero(jumpy)[0], "N": N})


# ----------------------------------------------------------------------------
# 2D jittered triangles (periodic square), vertex-neighbour stencils.
# ----------------------------------------------------------------------------

# Six-point interior rule on the reference triangle, degree 4, positive
# weights (two symmetric orbits; Dunavant 1985).  Used as a P2 nodal set and
# as the element quadrature weights c of the element mean.
_TRI_ORBITS = ((0.445948490915965, 0.223381589678011),
               (0.091576213509771, 0.109951743655322))


def _tri_nodes():
    bary, wts = [], []
    for a, w in _TRI_ORBITS:
        b = 1.0 - 2.0 * a
        for lam in ((a, a, b), (a, b, a), (b, a, a)):
            bary.append(lam)
            wts.append(w)
    return np.array(bary), np.array(wts)


def _vertex_stencil(tris: np.ndarray, n_vert: int):
    n_tri = tris.shape[0]
    inc_v = tris.ravel()
    inc_t = np.repeat(np.arange(n_tri), 3)
    order = np.argsort(inc_v, kind="stable")
    inc_v, inc_t = inc_v[order], inc_t[order]
    vptr = np.zeros(n_vert + 1, dtype=np.int64)
    np.add.at(vptr, inc_v + 1, 1)
    vptr = np.cumsum(vptr)
    deg = np.diff(vptr)
    maxdeg = int(deg.max())
    table = np.full((n_vert, maxdeg), -1, dtype=np.int64)
    slot = np.arange(inc_v.size) - vptr[inc_v]
    table[inc_v, slot] = inc_t
    cand = table[tris].reshape(n_tri, 3 * maxdeg)
    big = np.int64(n_tri + 1)
    cand = np.where(cand < 0, big, cand)
    self_id = np.arange(n_tri)[:, None]
    cand = np.where(cand == self_id, big, cand)        # self is placed first
    cand.sort(axis=1)
    keep = np.ones_like(cand, dtype=bool)
    keep[:, 1:] = cand[:, 1:] != cand[:, :-1]
    keep &= cand != big
    sizes = keep.sum(axis=1) + 1
    rowptr = np.zeros(n_tri + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(sizes)
    cols = np.empty(int(rowptr[-1]), dtype=np.int64)
    cols[rowptr[:-1]] = np.arange(n_tri)
    rest = np.broadcast_to((rowptr[:-1] + 1)[:, None], cand.shape) + np.cumsum(keep, axis=1) - 1
    cols[rest[keep]] = cand[keep]
    return rowptr.astype(np.int32), cols.astype(np.int32)


def make_tri_workload(N: int = 1000, seed: int = BASE_SEED + 3, grid_nodes: int = 64,
                      k: float = 4.0, gamma: float = 1.4, r_fac: float = 1e-3,
                      jitter: float = 0.2, outer=(1e-3, 1e-5), name: str = "tri") -> Workload:
    """Periodic N x N lattice of jittered vertices, every cell split along a
    seeded diagonal: 2 N^2 triangles, all of them with full vertex-neighbour
    stencils (11 to 16 elements)."""
    rng = _rng(seed)
    h = 1.0 / N
    jx = rng.uniform(-jitter, jitter, N * N) * h
    jy = rng.uniform(-jitter, jitter, N * N) * h
    cy, cx = np.divmod(np.arange(N * N), N)

    def corner(a, b):
        # vertex id (wrapped) and its position unwrapped next to cell (cx, cy)
        vid = ((cy + b) % N) * N + (cx + a) % N
        return vid, (cx + a) * h + jx[vid], (cy + b) * h + jy[vid]

    c00, c10, c01, c11 = corner(0, 0), corner(1, 0), corner(0, 1), corner(1, 1)
    diag = rng.integers(0, 2, N * N).astype(bool)

    def pick(p, q):
        return np.where(diag[:, None], p, q)

    tri_of = lambda i: (np.stack([c00[i], c10[i], c11[i]], 1), np.stack([c00[i], c10[i], c01[i]], 1),
                        np.stack([c00[i], c11[i], c01[i]], 1), np.stack([c10[i], c11[i], c01[i]], 1))
    parts = [tri_of(i) for i in range(3)]          # ids, x, y: [N^2, 3] per triangle kind
    t1 = [pick(P[0], P[1]) for P in parts]
    t2 = [pick(P[2], P[3]) for P in parts]
    tris, tx, ty = (np.stack([t1[i], t2[i]], axis=1).reshape(2 * N * N, 3) for i in range(3))
    n_tri = tris.shape[0]
    bary, wts = _tri_nodes()
    X = bary @ tx.T                # [6, n_tri]
    Y = bary @ ty.T
    X = np.ascontiguousarray(X.T)  # [n_tri, 6]
    Y = np.ascontiguousarray(Y.T)
    r = np.hypot(X - 0.5, Y - 0.5)
    inside = r < 0.3
    rho = np.where(inside, 1.0, outer[0]) * (1.0 + 0.01 * _fourier(rng, X, Y))
    pr = np.where(inside, 1.0, outer[1]) * (1.0 + 0.01 * _fourier(rng, X, Y))
    speed = 0.5 * np.where(inside, r / 0.3, 0.3 / np.maximum(r, 1e-12))
    rs = np.maximum(r, 1e-12)
    ux = speed * (X - 0.5) / rs + 0.005 * _fourier(rng, X, Y)
    uy = speed * (Y - 0.5) / rs + 0.005 * _fourier(rng, X, Y)
    states = _to_conserved(gamma, rho, [ux, uy], pr)
    rowptr, cols = _vertex_stencil(tris, N * N)
    grid = GridSpec(GRID_STENCIL, (grid_nodes, grid_nodes), (0.0, 0.0), (0.0, 0.0), k)
    target, jumpy = _limit_target(rng, states, rowptr, cols, 6, wts)
    return Workload(name, 2, gamma, n_tri, 6, states, target, rowptr, cols,
                    wts.astype(np.float64), grid, r_fac, seed,
                    {"theta_max": float((pr / rho).max()), "jump_elems": np.nonzero(jumpy)[0],
                     "N": N})


# ----------------------------------------------------------------------------
# 3D periodic hexahedra, tensor Gauss-Legendre nodes, self + 6 face neighbours.
# ----------------------------------------------------------------------------

def _fourier3(rng: np.random.Generator, x, y, z, n_modes: int = 8) -> np.ndarray:
    """Smooth periodic 3D perturbation with unit max amplitude bound."""
    out = np.zeros_like(x)
    amps = rng.uniform(0.5, 1.0, n_modes)
    k = rng.integers(-3, 4, (n_modes, 3))
    ph = rng.uniform(0.0, 2 * np.pi, n_modes)
    for a, (i, j, l), f in zip(amps, k, ph):
        out += a * np.sin(2 * np.pi * (i * x + j * y + l * z) + f)
    return out / amps.sum()


def make_hex_workload(N: int = 32, p: int = 2, seed: int = BASE_SEED + 6,
                      grid_nodes: int = 24, k: float = 4.0, gamma: float = 1.4,
                      r_fac: float = 1e-3, name: str = "hex") -> Workload:
    """3D Euler on periodic N^3 hexahedra, p = 2 (27 Gauss-Legendre nodes per
    element), face stencils of 7 elements (189 states), an eight-octant
    Riemann field (rho ~ logU[0.1, 10], p ~ logU[0.1, 100], |U| <= 3) with a
    1% smooth perturbation, per-stencil velocity box (k = 4) of grid_nodes^3."""
    rng = _rng(seed)
    n1 = p + 1
    n_s = n1 ** 3
    xi, wq = np.polynomial.legendre.leggauss(n1)
    n_elem = N ** 3
    ez, rem = np.divmod(np.arange(n_elem), N * N)
    ey, ex = np.divmod(rem, N)
    t = 0.5 * (xi + 1.0)
    # node j = (jz*n1 + jy)*n1 + jx
    jz, jr = np.divmod(np.arange(n_s), n1 * n1)
    jy, jx = np.divmod(jr, n1)
    X = (ex[:, None] + t[jx][None, :]) / N
    Y = (ey[:, None] + t[jy][None, :]) / N
    Z = (ez[:, None] + t[jz][None, :]) / N
    off = rng.uniform(0.2, 0.8, 3)
    cut = (N // 2 + off) / N
    octant = ((X >= cut[0]).astype(np.int64) + 2 * (Y >= cut[1]).astype(np.int64)
              + 4 * (Z >= cut[2]).astype(np.int64))
    rho_o = np.exp(rng.uniform(np.log(0.1), np.log(10.0), 8))
    p_o = np.exp(rng.uniform(np.log(0.1), np.log(100.0), 8))
    r_o = rng.uniform(0.0, 3.0, 8)
    d = rng.standard_normal((8, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rho = rho_o[octant] * (1.0 + 0.01 * _fourier3(rng, X, Y, Z))
    pr = p_o[octant] * (1.0 + 0.01 * _fourier3(rng, X, Y, Z))
    vel = [(r_o[:, None] * d)[:, c][octant] + 0.03 * _fourier3(rng, X, Y, Z) for c in range(3)]
    states = _to_conserved(gamma, rho, vel, pr)
    own = np.arange(n_elem)
    nb = lambda dx, dy, dz: ((ez + dz) % N) * N * N + ((ey + dy) % N) * N + (ex + dx) % N
    cols = np.stack([own, nb(-1, 0, 0), nb(1, 0, 0), nb(0, -1, 0), nb(0, 1, 0), nb(0, 0, -1),
                     nb(0, 0, 1)], 1).ravel().astype(np.int32)
    rowptr = np.arange(0, 7 * n_elem + 1, 7).astype(np.int32)
    w3 = (wq[jz] * wq[jy] * wq[jx]).astype(np.float64)
    grid = GridSpec(GRID_STENCIL, (grid_nodes,) * 3, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), k)
    target, jumpy = _limit_target(rng, states, rowptr, cols, n_s, w3)
    return Workload(name, 3, gamma, n_elem, n_s, states, target, rowptr, cols, w3, grid, r_fac,
                    seed, {"jump_elems": np.nonzero(jumpy)[0], "N": N})


# ----------------------------------------------------------------------------
# 2D quads with the node-level stencil of an FR scheme: solution points plus
# flux points on the faces (the stencil the paper runs, Sec. 5).
# ----------------------------------------------------------------------------

@dataclass
class NodeWorkload:
    """Inputs of the node-level path.

    states  [dim+2, n_state_nodes]: every node a stencil may list; the first
            n_elem*n_sol are solution points (element-major), then n_elem*n_flux
            flux points (element-major, face-major: faces x-, x+, y-, y+).
    rowptr, cols: per element, the node ids of its stencil.
    target  [dim+2, n_elem*n_v]: the values to limit on V (per element: the
            n_sol solution points, then its n_flux own flux points).
    v_weights [n_v]: mean weights on V (Gauss-Legendre on solution points,
            zero on flux points).
    """

    name: str
    dim: int
    gamma: float
    n_elem: int
    n_sol: int
    n_flux: int
    states: np.ndarray
    rowptr: np.ndarray
    cols: np.ndarray
    target: np.ndarray
    v_weights: np.ndarray
    grid: GridSpec
    r_fac: float = 1e-3
    seed: int = BASE_SEED
    meta: Dict = field(default_factory=dict)

    @property
    def n_v(self) -> int:
        return self.n_sol + self.n_flux

    @property
    def n_state_nodes(self) -> int:
        return self.states.shape[1]

    def n_vel(self) -> int:
        return int(np.prod(self.grid.n[: self.dim]))

    def pairs(self) -> int:
        return int(self.rowptr[-1]) * self.n_vel()


def _lagrange_at(xi: np.ndarray, x: float) -> np.ndarray:
    """Values at x of the Lagrange basis on the nodes xi."""
    out = np.ones(xi.size)
    for i in range(xi.size):
        for k in range(xi.size):
            if k != i:
                out[i] *= (x - xi[k]) / (xi[i] - xi[k])
    return out


def _admissible(gamma: float, w: np.ndarray) -> np.ndarray:
    """rho > 0 and p > 0 per column of conserved states (input screening only)."""
    rho = w[0]
    ke = 0.5 * (w[1] ** 2 + w[2] ** 2) / np.where(rho > 0, rho, 1.0)
    return (rho > 0) & ((gamma - 1.0) * (w[3] - ke) > 0) & np.isfinite(w).all(0)


def make_quad_fr_workload(N: int = 64, p: int = 3, seed: int = BASE_SEED + 5,
                          grid_nodes: int = 48, k: float = 4.0, gamma: float = 1.4,
                          r_fac: float = 1e-3, name: str = "quad_fr") -> NodeWorkload:
    """Periodic quads, p = 3: per element the 16 Gauss-Legendre solution points,
    its 16 flux points (4 per face, at the Gauss-Legendre abscissae along the
    face) and the 16 flux points of its 4 face neighbours on the shared faces:
    48 stencil states; V = the 16 solution + 16 own flux points.

    Flux-point states are the element polynomial (Lagrange interpolant of the
    solution points) evaluated on the face; an element whose face values come
    out inadmissible (rho <= 0 or p <= 0, at jumps) takes the sampled field
    values at its face points instead.  The field is the four-quadrant Riemann
    field of make_quad_workload; the limiter target is W + Delta (zero mean on
    the solution points) extended to the flux points by the same interpolant.
    """
    rng = _rng(seed)
    n1 = p + 1
    n_s = n1 * n1
    xi, wq = np.polynomial.legendre.leggauss(n1)
    ex = np.arange(N)
    n_elem = N * N
    ey_e, ex_e = np.divmod(np.arange(n_elem), N)
    # solution points (node j = jy*n1 + jx)
    Xs = ((ex_e[:, None] + 0.5 * (xi[None, :] + 1.0)) / N)[:, None, :].repeat(n1, 1).reshape(n_elem, n_s)
    Ys = ((ey_e[:, None] + 0.5 * (xi[None, :] + 1.0)) / N)[:, :, None].repeat(n1, 2).reshape(n_elem, n_s)
    # flux points: faces x- (x = left edge), x+, y-, y+; n1 points each
    t = 0.5 * (xi + 1.0)
    Xf = np.stack([np.repeat(ex_e[:, None] / N, n1, 1), np.repeat((ex_e[:, None] + 1) / N, n1, 1),
                   (ex_e[:, None] + t[None]) / N, (ex_e[:, None] + t[None]) / N], 1)
    Yf = np.stack([(ey_e[:, None] + t[None]) / N, (ey_e[:, None] + t[None]) / N,
                   np.repeat(ey_e[:, None] / N, n1, 1), np.repeat((ey_e[:, None] + 1) / N, n1, 1)], 1)
    Xf = Xf.reshape(n_elem, 4 * n1)
    Yf = Yf.reshape(n_elem, 4 * n1)

    # four-quadrant Riemann field, sampled anywhere
    off = rng.uniform(0.2, 0.8, 2)
    xs, ys = (N // 2 + off[0]) / N, (N // 2 + off[1]) / N
    rho_q = np.exp(rng.uniform(np.log(0.1), np.log(10.0), 4))
    p_q = np.exp(rng.uniform(np.log(0.1), np.log(100.0), 4))
    r_q = rng.uniform(0.0, 3.0, 4)
    a_q = rng.uniform(0.0, 2 * np.pi, 4)
    modes = [(rng.uniform(0.5, 1.0, 8), rng.integers(-4, 5, 8), rng.integers(-4, 5, 8),
              rng.uniform(0.0, 2 * np.pi, 8)) for _ in range(4)]

    def smooth(m, X, Y):
        amps, kx, ky, ph = m
        out = np.zeros_like(X)
        for a, i, j, f in zip(amps, kx, ky, ph):
            out += a * np.sin(2 * np.pi * (i * X + j * Y) + f)
        return out / amps.sum()

    def field(X, Y):
        q = (X >= xs).astype(np.int64) + 2 * (Y >= ys).astype(np.int64)
        rho = rho_q[q] * (1.0 + 0.01 * smooth(modes[0], X, Y))
        pr = p_q[q] * (1.0 + 0.01 * smooth(modes[1], X, Y))
        ux = (r_q * np.cos(a_q))[q] + 0.03 * smooth(modes[2], X, Y)
        uy = (r_q * np.sin(a_q))[q] + 0.03 * smooth(modes[3], X, Y)
        return _to_conserved(gamma, rho, [ux, uy], pr)

    W = field(Xs.ravel(), Ys.ravel()).reshape(4, n_elem, n1, n1)    # [v, e, jy, jx]
    Lm, Lp = _lagrange_at(xi, -1.0), _lagrange_at(xi, 1.0)

    def faces(Wn):                                           # [v, e, jy, jx] -> [v, e, 4*n1]
        return np.concatenate([np.einsum("veyx,x->vey", Wn, Lm), np.einsum("veyx,x->vey", Wn, Lp),
                               np.einsum("veyx,y->vex", Wn, Lm), np.einsum("veyx,y->vex", Wn, Lp)],
                              axis=2)

    F = faces(W)
    ok = _admissible(gamma, F.reshape(4, -1)).reshape(n_elem, 4 * n1).all(1)
    if (~ok).any():
        F[:, ~ok] = field(Xf[~ok].ravel(), Yf[~ok].ravel()).reshape(4, int((~ok).sum()), 4 * n1)
    sol = W.reshape(4, n_elem * n_s)
    states = np.concatenate([sol, F.reshape(4, n_elem * 4 * n1)], axis=1)

    # stencil: own solution points, own flux points, neighbours' flux points on the shared faces
    base = n_elem * n_s
    fl = lambda e, f: base + e[:, None] * (4 * n1) + f * n1 + np.arange(n1)[None, :]
    left = ey_e * N + (ex_e - 1) % N
    right = ey_e * N + (ex_e + 1) % N
    down = ((ey_e - 1) % N) * N + ex_e
    up = ((ey_e + 1) % N) * N + ex_e
    own = np.arange(n_elem)
    cols = np.concatenate([own[:, None] * n_s + np.arange(n_s)[None, :],
                           fl(own, 0), fl(own, 1), fl(own, 2), fl(own, 3),
                           fl(left, 1), fl(right, 0), fl(down, 3), fl(up, 2)], axis=1)
    per = cols.shape[1]
    cols = cols.ravel().astype(np.int32)
    rowptr = np.arange(0, per * n_elem + 1, per).astype(np.int32)

    # limiter target on V
    w2 = (wq[:, None] * wq[None, :]).ravel()
    el_cols = np.stack([own, left, right, down, up], 1).ravel().astype(np.int32)
    el_rowptr = np.arange(0, 5 * n_elem + 1, 5).astype(np.int32)
    tsol, jumpy = _limit_target(rng, sol, el_rowptr, el_cols, n_s, w2)
    T = tsol.reshape(4, n_elem, n1, n1)
    target = np.concatenate([T.reshape(4, n_elem, n_s), faces(T)], axis=2).reshape(4, -1)
    v_weights = np.concatenate([w2, np.zeros(4 * n1)])
    grid = GridSpec(GRID_STENCIL, (grid_nodes, grid_nodes), (0.0, 0.0), (0.0, 0.0), k)
    # face pairs: each own flux point with the neighbour's flux point at the same
    # place, outward unit normal, and the element whose bounds apply
    nbr_face = [(left, 1), (right, 0), (down, 3), (up, 2)]
    normal = [(-1.0, 0.0), (1.0, 0.0), (0.0, -1.0), (0.0, 1.0)]
    pi = np.stack([fl(own, f) for f in range(4)], 1).reshape(n_elem, -1)
    pj = np.stack([fl(nb, g) for nb, g in nbr_face], 1).reshape(n_elem, -1)
    pn = np.repeat(np.array(normal)[None, :, None, :], n_elem, 0)
    pn = np.repeat(pn, n1, 2).reshape(n_elem, 4 * n1, 2)
    pairs = {"ni": pi.ravel().astype(np.int32), "nj": pj.ravel().astype(np.int32),
             "normals": np.ascontiguousarray(pn.reshape(-1, 2).T),
             "elem": np.repeat(own, 4 * n1).astype(np.int32)}
    return NodeWorkload(name, 2, gamma, n_elem, n_s, 4 * n1, np.ascontiguousarray(states),
                        rowptr, cols, np.ascontiguousarray(target), v_weights, grid, r_fac, seed,
                        {"jump_elems": np.nonzero(jumpy)[0], "face_fallback": int((~ok).sum()),
                         "N": N, "face_pairs": pairs})


def make_workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)


def sample_elements(wl: Workload, n: int, seed: int = 7) -> np.ndarray:
    """Seeded element sample: half uniform, half from jump-spanning stencils."""
    rng = _rng(wl.seed + seed)
    n = min(n, wl.n_elem)
    jumps = np.asarray(wl.meta.get("jump_elems", np.zeros(0, dtype=np.int64)))
    n_j = min(len(jumps), n // 2)
    pick_j = rng.choice(jumps, n_j, replace=False) if n_j else np.zeros(0, dtype=np.int64)
    rest = rng.choice(wl.n_elem, n - n_j, replace=False)
    out = np.unique(np.concatenate([pick_j, rest]).astype(np.int64))
    return out


# Named workloads: the five configurations the method is exercised on.
WORKLOADS: Dict[str, Callable[..., Workload]] = {
    # 1D, 64 elements, p=3, 12-state stencils, 64-node global grid on +-12 sqrt(theta_max)
    "line64": lambda **kw: make_line_workload(**{"n_elem": 64, "seed": BASE_SEED + 0,
                                                 "name": "line64", **kw}),
    # 2D 256^2 quads, p=3, 80-state stencils, 48x48 per-stencil grid (k=4), FP64
    "quad256": lambda **kw: make_quad_workload(**{"N": 256, "seed": BASE_SEED + 1,
                                                  "grid_nodes": 48, "name": "quad256", **kw}),
    # 2D 1024^2 quads, p=3, sine + Sod jump field, 64x64 global grid on +-12 sqrt(theta_max)
    "quad1024_sine": lambda **kw: make_quad_workload(**{"N": 1024, "seed": BASE_SEED + 2,
                                                        "field_kind": "sine", "grid_nodes": 64,
                                                        "grid_mode": GRID_GLOBAL,
                                                        "name": "quad1024_sine", **kw}),
    # 2M P2 triangles, vertex-neighbour stencils (uneven), 64x64 per-stencil grid
    "tri2m": lambda **kw: make_tri_workload(**{"N": 1000, "seed": BASE_SEED + 3,
                                               "name": "tri2m", **kw}),
    # 512^2 quads, p=3, 48x48 per-stencil grid, used for the backward
    "quad512": lambda **kw: make_quad_workload(**{"N": 512, "seed": BASE_SEED + 4,
                                                  "grid_nodes": 48, "name": "quad512", **kw}),
    # 32^3 hexahedra, p=2, 189-state face stencils, 24^3 per-stencil velocity grid
    "hex32": lambda **kw: make_hex_workload(**{"N": 32, "seed": BASE_SEED + 6, "grid_nodes": 24,
                                               "name": "hex32", **kw}),
    # 256^2 quads, p=3, node-level stencils of solution + flux points (48 states)
    "quad256_fr": lambda **kw: make_quad_fr_workload(**{"N": 256, "seed": BASE_SEED + 5,
                                                        "grid_nodes": 48, "name": "quad256_fr",
                                                        **kw}),
}
