"""Forward-mode derivatives of the bounds + limiter, for pinning the oracle's
analytic subgradient (test infrastructure; shares no code with oracle/).

A value carries its derivatives along K directions: `Dual(v, d)` with
d.shape == v.shape + (K,).  The forward pass below restates the method in
plain NumPy on dual numbers, in the paper's order:

- the Maxwellian of every stencil state at every velocity node, direct form
  g = rho (2 pi theta)^(-d/2) exp(-|u - U|^2 / (2 theta)) and g_I =
  (theta delta / 2) g (Sec. 2.2, Sec. 3.6);
- the min/max envelopes, relaxed by (1 -+ r) (eq. fminmax, eq. relaxed);
- the trapezoid rule on the global box or on the per-stencil box U -+ k
  sqrt(theta) (eq. truncdomain, Sec. 3.7), whose nodes and weights move with
  the extreme states;
- the moment bounds with the momentum split by the sign of u (eq. rhobounds,
  mmbounds, mpbounds, Ebounds) and the density floor (Sec. 3.8);
- the squeeze limiter with the epsilon rule and the coupled minimum (eq.
  alpha, eq. limiter) and the pressure step (eq. pmin, eq. doublelimit).

A min or max passes on the derivative of the element it picks.  Ties (which
seeded inputs do not produce) follow the conventions of the backward: the
first state for a maximum envelope and the last for a minimum one, the
first state for a box end, the first component and side for alpha.
"""

import numpy as np


class Dual:
    __slots__ = ("v", "d")

    def __init__(self, v, d):
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)

    @staticmethod
    def const(v, k):
        v = np.asarray(v, dtype=np.float64)
        return Dual(v, np.zeros(v.shape + (k,)))

    @property
    def k(self):
        return self.d.shape[-1]

    def __getitem__(self, idx):
        if not isinstance(idx, tuple):
            idx = (idx,)
        return Dual(self.v[idx], self.d[idx + (slice(None),)])

    def _lift(self, o):
        return o if isinstance(o, Dual) else Dual.const(np.broadcast_to(o, np.shape(o)), self.k)

    def __add__(self, o):
        o = self._lift(o)
        return Dual(self.v + o.v, self.d + o.d)

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __sub__(self, o):
        return self + (-self._lift(o))

    def __rsub__(self, o):
        return self._lift(o) - self

    def __mul__(self, o):
        o = self._lift(o)
        return Dual(self.v * o.v, self.d * o.v[..., None] + o.d * self.v[..., None])

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = self._lift(o)
        q = self.v / o.v
        return Dual(q, (self.d - o.d * q[..., None]) / o.v[..., None])

    def __rtruediv__(self, o):
        return self._lift(o) / self

    def sum(self, axis):
        ax = axis if axis >= 0 else self.v.ndim + axis
        return Dual(self.v.sum(axis=ax), self.d.sum(axis=ax))


def exp(x):
    e = np.exp(x.v)
    return Dual(e, x.d * e[..., None])


def log(x):
    return Dual(np.log(x.v), x.d / x.v[..., None])


def sqrt(x):
    s = np.sqrt(x.v)
    return Dual(s, x.d / (2.0 * s[..., None]))


def fabs(x):
    sg = np.where(x.v < 0.0, -1.0, 1.0)
    return Dual(np.abs(x.v), x.d * sg[..., None])


def pick(x, idx, axis=0):
    """Entries of x at index idx along axis (idx has x's shape without it)."""
    i = np.expand_dims(idx, axis)
    return Dual(np.take_along_axis(x.v, i, axis).squeeze(axis),
                np.take_along_axis(x.d, i[..., None], axis).squeeze(axis))


def argmax_first(v, axis=0):
    return np.argmax(v, axis=axis)


def argmin_last(v, axis=0):
    n = v.shape[axis]
    return n - 1 - np.argmin(np.flip(v, axis=axis), axis=axis)


def where(c, a, b):
    return Dual(np.where(c, a.v, b.v), np.where(c[..., None], a.d, b.d))


def element_bounds(dim, gamma, W, idx, grid_mode, n, lo, hi, k, r_fac, rho_floor):
    """Bounds [2(d+2)] (min rows, then max rows) of one element whose stencil
    lists the node states W[:, idx] (W a Dual [d+2, n_nodes])."""
    K = W.k
    delta = (2.0 - dim * (gamma - 1.0)) / (gamma - 1.0)
    st = W[:, idx]
    rho = st[0]
    U = [st[1 + j] / rho for j in range(dim)]
    mm = st[1] * st[1]
    for j in range(1, dim):
        mm = mm + st[1 + j] * st[1 + j]
    theta = (gamma - 1.0) * (st[dim + 1] - 0.5 * mm / rho) / rho
    # velocity nodes and trapezoid weights per direction
    axes, wts = [], []
    for j in range(dim):
        if grid_mode == 1:
            sd = sqrt(theta)
            lo_s = U[j] - k * sd
            hi_s = U[j] + k * sd
            a = pick(lo_s, np.asarray(np.argmin(lo_s.v)))
            b = pick(hi_s, argmax_first(hi_s.v))
        else:
            a, b = Dual.const(lo[j], K), Dual.const(hi[j], K)
        h = (b - a) / float(n[j] - 1)
        t = np.arange(n[j], dtype=np.float64)
        u = Dual(a.v + t * h.v, a.d[None, :] + t[:, None] * h.d[None, :])
        end = np.where((t == 0) | (t == n[j] - 1), 0.5, 1.0)
        w = Dual(end * h.v, end[:, None] * h.d[None, :])
        axes.append(u)
        wts.append(w)

    def grid(x, j):
        """Per-direction array x [n_j] broadcast over the node grid."""
        shape = [1] * dim
        shape[j] = n[j]
        return Dual(x.v.reshape(shape), x.d.reshape(shape + [K]))

    def per_state(x):
        return Dual(x.v.reshape((-1,) + (1,) * dim), x.d.reshape((-1,) + (1,) * dim + (K,)))

    q = None
    for j in range(dim):
        du = grid(axes[j], j) - per_state(U[j])
        q = du * du if q is None else q + du * du
    th = per_state(theta)
    g = per_state(rho) * power_neg_half_d(2.0 * np.pi * th, dim) * exp(-(q / (2.0 * th)))
    gI = (0.5 * delta) * th * g
    fTmin = (1.0 - r_fac) * pick(g, argmin_last(g.v))
    fTmax = (1.0 + r_fac) * pick(g, argmax_first(g.v))
    fImin = (1.0 - r_fac) * pick(gI, argmin_last(gI.v))
    fImax = (1.0 + r_fac) * pick(gI, argmax_first(gI.v))
    M = grid(wts[0], 0)
    for j in range(1, dim):
        M = M * grid(wts[j], j)
    u2 = None
    for j in range(dim):
        uj = grid(axes[j], j)
        u2 = uj * uj if u2 is None else u2 + uj * uj

    def total(x):
        for _ in range(dim):
            x = x.sum(0)
        return x

    rho_min = total(M * fTmin)
    rho_max = total(M * fTmax)
    if rho_min.v < rho_floor:
        rho_min = Dual.const(rho_floor, K)
    E_min = total(M * (0.5 * u2 * fTmin + fImin))
    E_max = total(M * (0.5 * u2 * fTmax + fImax))
    m_min, m_max = [], []
    for j in range(dim):
        uj = grid(axes[j], j)
        neg = np.broadcast_to(uj.v < 0.0, fTmin.v.shape)
        lo_env = where(neg, fTmax, fTmin)
        hi_env = where(neg, fTmin, fTmax)
        m_min.append(total(M * uj * lo_env))
        m_max.append(total(M * uj * hi_env))
    return [rho_min] + m_min + [E_min], [rho_max] + m_max + [E_max]


def power_neg_half_d(x, dim):
    """x^(-d/2)."""
    return exp(log(x) * (-0.5 * dim))


def pressure(gamma, w, dim):
    mm = w[1] * w[1]
    for j in range(2, dim + 1):
        mm = mm + w[j] * w[j]
    return (gamma - 1.0) * (w[dim + 1] - 0.5 * mm / w[0])


def element_limit(dim, gamma, w, c, bmin, bmax, eps, p_floor):
    """Limited nodes of one element: w a Dual [d+2, n_s], bounds lists of
    Duals per variable."""
    nv = dim + 2
    K = w.k
    csum = float(np.sum(c))
    wbar = [(w[v] * c).sum(0) / csum for v in range(nv)]
    alpha = Dual.const(1.0, K)
    for v in range(nv):
        jmax = argmax_first(w[v].v)
        jmin = int(np.argmin(w[v].v))
        dp = pick(w[v], np.asarray(jmax)) - wbar[v]
        dm = pick(w[v], np.asarray(jmin)) - wbar[v]
        if abs(dm.v) < eps or abs(dp.v) < eps:
            av = Dual.const(0.0, K)
        else:
            av = Dual.const(1.0, K)
            ru = fabs((bmax[v] - wbar[v]) / dp)
            rl = fabs((bmin[v] - wbar[v]) / dm)
            if ru.v < av.v:
                av = ru
            if rl.v < av.v:
                av = rl
        if av.v < alpha.v:
            alpha = av
    wt = [wbar[v] + alpha * (w[v] - wbar[v]) for v in range(nv)]
    P = pressure(gamma, wt, dim)
    Pv = np.where(np.isnan(P.v), -np.inf, P.v)
    jp = int(np.argmin(Pv))
    if Pv[jp] < p_floor:
        pbar = pressure(gamma, wbar, dim)
        if pbar.v > p_floor:
            aP = fabs((p_floor - pbar) / (pick(P, np.asarray(jp)) - pbar))
        else:
            aP = Dual.const(0.0, K)
        wt = [wbar[v] + aP * (wt[v] - wbar[v]) for v in range(nv)]
    return wt


def objective(dim, gamma, states, solution, rowptr, cols, n_s, grid_mode, n, lo, hi, k,
              r_fac, weights, G, rho_floor=1e-12, p_floor=1e-12, eps=1e-13):
    """J = sum G * limited as a Dual, seeded with one unit direction per DoF of
    (states, solution): J.d[i] is dJ/d(DoF i), states first, row-major."""
    nv, nn = states.shape
    K = 2 * nv * nn
    eye = np.eye(K)
    W = Dual(states, eye[: nv * nn].reshape(nv, nn, K))
    S = Dual(solution, eye[nv * nn:].reshape(nv, nn, K))
    J = Dual.const(0.0, K)
    n_elem = len(rowptr) - 1
    for e in range(n_elem):
        elems = cols[rowptr[e]:rowptr[e + 1]]
        idx = (elems[:, None] * n_s + np.arange(n_s)[None, :]).ravel()
        bmin, bmax = element_bounds(dim, gamma, W, idx, grid_mode, n, lo, hi, k, r_fac,
                                    rho_floor)
        own = np.arange(e * n_s, (e + 1) * n_s)
        lim = element_limit(dim, gamma, S[:, own], weights, bmin, bmax, eps, p_floor)
        for v in range(nv):
            J = J + (lim[v] * G[v, own]).sum(0)
    return J
