"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each check is independent of the oracle's own arithmetic: closed-form
Maxwellian moments (Sec. 2.2, 3.6), the paper's printed truncation figures
(Sec. 3.7, golden fixture), exact erf integrals of two-state envelopes
(Sec. 3.3 notes analytic integration is possible in 1D), the theorems of
Sec. 4 as invariants, and brute-force adaptive quadrature.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GL = 0
ST = 1


def conserved(gamma, rho, U, p):
    U = list(U)
    return [rho] + [rho * u for u in U] + [p / (gamma - 1.0) + 0.5 * rho * sum(u * u for u in U)]


def one_element(gamma, prims):
    """Single element whose nodes are the given primitive states; stencil = itself."""
    cols = np.array([0], dtype=np.int32)
    rowptr = np.array([0, 1], dtype=np.int32)
    st = np.array([conserved(gamma, *q) for q in prims], dtype=np.float64).T.copy()
    return st, rowptr, cols, len(prims)


def run_bounds(d, gamma, prims, mode, n, lo=(0, 0), hi=(0, 0), k=4.0, r=0.0, floor=0.0):
    st, rp, cl, ns = one_element(gamma, prims)
    b, s = oracle.bounds(d, gamma, st, rp, cl, ns, mode, n, lo, hi, k, r, rho_floor=floor)
    return b[:, 0], s[0]


def half_moments(rho, U, th):
    """Textbook half-line first moments of a 1D Maxwellian: (int_{u<0} u g, int_{u>=0} u g)."""
    s = math.sqrt(th)
    z = U / s
    phi = math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    neg = rho * (U * special.ndtr(-z) - s * phi)
    pos = rho * (U * special.ndtr(z) + s * phi)
    return neg, pos


# ---------------------------------------------------------------- Sec. 3.6

def test_internal_degrees_of_freedom():
    # delta = 2/(gamma-1) - d: 4 in 1D and 3 in 2D for gamma = 1.4, 0 for a monatomic gas
    assert oracle.delta(1, 1.4) == pytest.approx(4.0, rel=1e-15)
    assert oracle.delta(2, 1.4) == pytest.approx(3.0, rel=1e-15)
    assert abs(oracle.delta(1, 3.0)) < 1e-15
    assert abs(oracle.delta(2, 2.0)) < 1e-15


# ------------------------------------------- Thm 4.1 + closed-form moments

@pytest.mark.parametrize("d", [1, 2])
def test_constant_state_reproduces_moments(d):
    gamma = 1.4
    U = (0.7, -1.3)[:d]
    q = (1.7, U, 2.3)
    prims = [q] * 4
    n = (801, 161)[d - 1]
    b, s = run_bounds(d, gamma, prims, ST, (n, n), k=10.0, r=0.0)
    w = conserved(gamma, *q)
    nv = d + 2
    assert s == 0
    for v in range(nv):
        assert b[v] == pytest.approx(w[v], rel=1e-12, abs=1e-12)
        assert b[nv + v] == pytest.approx(w[v], rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("d", [1, 2])
def test_relaxed_single_state_closed_form(d):
    """rho, E scale by (1 -+ r); momentum split follows the half-line moments.

    The split puts a derivative kink at u_j = 0, so the grid is symmetric with
    0 on a node and one Richardson step removes the h^2 term of the kink."""
    gamma, r = 1.4, 1e-3
    U = (0.9, -0.4)[:d]
    rho, p = 0.8, 1.1
    th = p / rho
    L = 12.0 * math.sqrt(th) + 1.0
    ns = (801, 1601)
    res = [run_bounds(d, gamma, [(rho, U, p)], GL, (n, n), (-L, -L), (L, L), r=r)[0] for n in ns]
    b = res[1]
    rich = (4 * res[1] - res[0]) / 3
    w = conserved(gamma, rho, U, p)
    nv = d + 2
    for v in (0, d + 1):
        assert b[v] == pytest.approx((1 - r) * w[v], rel=1e-12)
        assert b[nv + v] == pytest.approx((1 + r) * w[v], rel=1e-12)
    for j in range(d):
        neg, pos = half_moments(rho, U[j], th)
        assert rich[1 + j] == pytest.approx((1 + r) * neg + (1 - r) * pos, rel=1e-11, abs=1e-13)
        assert rich[nv + 1 + j] == pytest.approx((1 - r) * neg + (1 + r) * pos, rel=1e-11, abs=1e-13)
        # the kink-free combination needs no extrapolation
        assert b[1 + j] + b[nv + 1 + j] == pytest.approx(2 * rho * U[j], rel=1e-12)


def test_monatomic_energy_has_no_internal_part():
    gamma = 3.0          # d = 1 monatomic: delta = 0
    q = (1.2, (0.3,), 0.9)
    b, _ = run_bounds(1, gamma, [q], ST, (801,), k=10.0, r=0.0)
    assert b[2] == pytest.approx(conserved(gamma, *q)[2], rel=1e-12)


# --------------------------------------------- printed figures of Sec. 3.7

def test_truncation_error_matches_printed_values():
    fx = json.load(open(os.path.join(GOLDEN, "truncation_sec3_7.json")))
    rho, U, p = 1.0, 0.37, 0.8
    deficits = {}
    for k in (3.0, 3.5, 4.0, 8.0):
        b, _ = run_bounds(1, 1.4, [(rho, (U,), p)], ST, (20001,), k=k, r=0.0)
        deficits[k] = 1.0 - b[0] / rho
        assert deficits[k] == pytest.approx(special.erfc(k / math.sqrt(2)), rel=1e-5, abs=2e-16)
    # k = 4: "approximately 6e-5"
    assert float(f"{deficits[4.0]:.0e}") == fx["printed_relative_error"]["4"]
    # k = 8: "approximately 1e-15"
    assert 0 < deficits[8.0] < 5 * fx["printed_relative_error"]["8"]
    # relaxation 1e-3 needs k >= 3.5: 3.5 is enough, 3.0 is not
    assert deficits[fx["printed_k_for_rfac_1e-3"]] <= 1e-3 < deficits[3.0]


# --------------------------------------------- exact two-state integrals

def gauss_interval_moments(A, U, th, a, b):
    """int_a^b u^p A exp(-(u-U)^2/(2 th)) du for p = 0, 1, 2 (erf closed form)."""
    s = math.sqrt(th)
    za = -np.inf if a == -np.inf else (a - U) / s
    zb = np.inf if b == np.inf else (b - U) / s
    J0 = math.sqrt(2 * math.pi) * (special.ndtr(zb) - special.ndtr(za))
    ea = 0.0 if np.isinf(za) else math.exp(-0.5 * za * za)
    eb = 0.0 if np.isinf(zb) else math.exp(-0.5 * zb * zb)
    J1 = ea - eb
    J2 = (0.0 if np.isinf(za) else za * ea) - (0.0 if np.isinf(zb) else zb * eb) + J0
    m0 = A * s * J0
    m1 = A * s * (U * J0 + s * J1)
    m2 = A * s * (U * U * J0 + 2 * U * s * J1 + s * s * J2)
    return m0, m1, m2


def crossings(A1, U1, t1, A2, U2, t2):
    c2 = 1.0 / t2 - 1.0 / t1
    c1 = 2 * U1 / t1 - 2 * U2 / t2
    c0 = U2 * U2 / t2 - U1 * U1 / t1 + 2 * math.log(A1 / A2)
    if abs(c2) < 1e-300:
        return [] if c1 == 0 else [-c0 / c1]
    disc = c1 * c1 - 4 * c2 * c0
    if disc <= 0:
        return []
    r = math.sqrt(disc)
    return sorted([(-c1 - r) / (2 * c2), (-c1 + r) / (2 * c2)])


def env_moments(gs, which):
    """Exact moments (orders 0-2) of the pointwise min/max of scaled 1D Gaussians
    (A, U, theta), split into u < 0 and u >= 0 parts."""
    bps = set([0.0])
    for i in range(len(gs)):
        for j in range(i + 1, len(gs)):
            bps.update(crossings(*gs[i], *gs[j]))
    edges = [-np.inf] + sorted(bps) + [np.inf]
    out = {"neg": np.zeros(3), "pos": np.zeros(3)}
    for a, b in zip(edges[:-1], edges[1:]):
        mid = (a + b) / 2 if np.isfinite(a) and np.isfinite(b) else (b - 1.0 if np.isfinite(b) else a + 1.0)
        vals = [A * math.exp(-(mid - U) ** 2 / (2 * th)) for A, U, th in gs]
        i = int(np.argmax(vals)) if which == "max" else int(np.argmin(vals))
        m = np.array(gauss_interval_moments(*gs[i], a, b))
        out["neg" if b <= 0 else "pos"] += m
    return out


def exact_two_state_bounds(gamma, s1, s2):
    """Exact untruncated (r=0) bounds of a two-state 1D stencil, reduced-energy reading."""
    dl = 2.0 / (gamma - 1.0) - 1.0
    G = []
    for rho, U, p in (s1, s2):
        th = p / rho
        A = rho / math.sqrt(2 * math.pi * th)
        G.append((A, U, th))
    GI = [(A * 0.5 * th * dl, U, th) for (A, U, th) in G]

    Tmin, Tmax = env_moments(G, "min"), env_moments(G, "max")
    Imin, Imax = env_moments(GI, "min"), env_moments(GI, "max")
    tot = lambda e, p: e["neg"][p] + e["pos"][p]
    rho_min, rho_max = tot(Tmin, 0), tot(Tmax, 0)
    m_min = Tmax["neg"][1] + Tmin["pos"][1]
    m_max = Tmin["neg"][1] + Tmax["pos"][1]
    E_min = 0.5 * tot(Tmin, 2) + tot(Imin, 0)
    E_max = 0.5 * tot(Tmax, 2) + tot(Imax, 0)
    return np.array([rho_min, m_min, E_min, rho_max, m_max, E_max])


def test_two_state_equal_temperature_exact_richardson():
    """Kinks placed on grid nodes: trapezoid error is c h^2 + O(h^4), so a
    Richardson step must meet the exact erf integrals closely."""
    gamma = 1.4
    s1 = (1.0, -0.5, 1.0)      # rho, U, p  (theta = 1)
    s2 = (1.0, 0.75, 1.0)      # crossing at u = 0.125; the momentum split is at 0
    ex = exact_two_state_bounds(gamma, s1, s2)
    L = 16.0
    res = []
    for n in (2049, 4097):
        b, _ = run_bounds(1, gamma, [(s1[0], (s1[1],), s1[2]), (s2[0], (s2[1],), s2[2])],
                          GL, (n,), lo=(-L,), hi=(L,), r=0.0)
        res.append(b)
    rich = (4 * res[1] - res[0]) / 3
    scale = np.abs(ex) + 1.0
    assert np.all(np.abs(res[1] - ex) / scale < 1e-5)
    assert np.all(np.abs(rich - ex) / scale < 1e-10), (rich - ex) / scale


def test_two_state_general_converges_second_order():
    gamma = 1.4
    s1 = (2.0, -0.6, 1.5)
    s2 = (0.3, 1.1, 0.05)
    ex = exact_two_state_bounds(gamma, s1, s2)
    errs = []
    for n in (1001, 4001, 16001):
        b, _ = run_bounds(1, gamma, [(s1[0], (s1[1],), s1[2]), (s2[0], (s2[1],), s2[2])],
                          ST, (n,), k=12.0, r=0.0)
        errs.append(np.max(np.abs(b - ex) / (np.abs(ex) + 1.0)))
    assert errs[2] < 1e-7
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4   # h -> h/4 gives ~16x


# ------------------------------------------------- 2D adaptive brute force

def test_two_state_2d_against_semi_analytic_quadrature():
    """Along x the envelope of two 2D Maxwellians is an envelope of scaled 1D
    Gaussians (exact erf moments); the y integral is adaptive quadrature."""
    gamma = 1.4
    dl = 2.0 / (gamma - 1.0) - 2.0
    sts = [(1.0, (0.4, -0.2), 0.7), (0.5, (-0.3, 0.5), 0.2)]
    par = []
    for rho, U, p in sts:
        th = p / rho
        par.append((rho / (2 * math.pi * th), U, th))

    def xline(y, scale_I):
        gs = []
        for A, U, th in par:
            amp = A * math.exp(-(y - U[1]) ** 2 / (2 * th)) * (0.5 * th * dl if scale_I else 1.0)
            gs.append((amp, U[0], th))
        return gs

    def q(f):
        return integrate.quad(f, -12, 12, limit=400, epsabs=1e-14, epsrel=1e-13)[0]

    def tot(e, p):
        return e["neg"][p] + e["pos"][p]

    rho_min = q(lambda y: tot(env_moments(xline(y, False), "min"), 0))
    rho_max = q(lambda y: tot(env_moments(xline(y, False), "max"), 0))
    mx_min = q(lambda y: (lambda lo, hi: hi["neg"][1] + lo["pos"][1])(
        env_moments(xline(y, False), "min"), env_moments(xline(y, False), "max")))
    e_max = q(lambda y: (lambda T, I: 0.5 * tot(T, 2) + 0.5 * y * y * tot(T, 0) + tot(I, 0))(
        env_moments(xline(y, False), "max"), env_moments(xline(y, True), "max")))
    ref = {0: rho_min, 4: rho_max, 1: mx_min, 7: e_max}
    box = 7.0
    bs = [run_bounds(2, gamma, sts, GL, (n, n), lo=(-box, -box), hi=(box, box), r=0.0)[0]
          for n in (201, 801)]
    rich = (16 * bs[1] - bs[0]) / 15
    err = lambda b: max(abs(b[i] - v) / (abs(v) + 1e-2) for i, v in ref.items())
    errs = [err(b) for b in bs]
    # second-order convergence (h -> h/4 gives ~16x) towards the reference
    assert 12 < errs[0] / errs[1] < 20, errs
    assert err(rich) < 2e-6, err(rich)


# -------------------------------------------------- Sec. 4 invariants

def _random_stencil(rng, d, n_states, jump=True):
    out = []
    for i in range(n_states):
        side = (i % 2) if jump else 0
        rho = math.exp(rng.uniform(math.log(0.1), math.log(10))) * (1e-2 if side else 1.0)
        p = math.exp(rng.uniform(math.log(0.1), math.log(100))) * (1e-3 if side else 1.0)
        U = tuple(rng.uniform(-3, 3, d))
        out.append((rho, U, p))
    return out


@pytest.mark.parametrize("d", [1, 2])
def test_ordering_positivity_and_mean_in_bounds(d):
    """Thm 4.2 (rho_min, E_min > 0), Thm 4.5 first half (the weighted mean of the
    stencil states lies in the bounds), and min/max ordering of each component."""
    gamma, r = 1.4, 1e-3
    rng = np.random.default_rng(11 + d)
    n = (2001, 201)[d - 1]
    nv = d + 2
    for trial in range(6):
        prims = _random_stencil(rng, d, 6, jump=trial % 2 == 0)
        b, s = run_bounds(d, gamma, prims, ST, (n, n), k=5.0, r=r)
        W = np.array([conserved(gamma, *q) for q in prims])      # [S, nv]
        c = rng.uniform(0.1, 1.0, len(prims))
        mean = (c[:, None] * W).sum(0) / c.sum()
        assert b[0] > 0 and b[d + 1] > 0
        for v in range(nv):
            scale = max(np.abs(W[:, v]).max(), 1.0) if 1 <= v <= d else 0.0
            assert b[v] <= W[:, v].min() + 1e-9 * scale
            assert b[nv + v] >= W[:, v].max() - 1e-9 * scale
            assert b[v] <= mean[v] <= b[nv + v]


def test_monotone_in_stencil():
    """A larger stencil can only widen the bounds (fixed global grid)."""
    gamma = 1.4
    rng = np.random.default_rng(5)
    prims = _random_stencil(rng, 2, 5)
    lo, hi = (-9.0, -9.0), (9.0, 9.0)
    small, _ = run_bounds(2, gamma, prims[:3], GL, (64, 64), lo, hi, r=1e-3)
    big, _ = run_bounds(2, gamma, prims, GL, (64, 64), lo, hi, r=1e-3)
    tol = 1e-13 * (np.abs(big) + 1)
    assert np.all(big[:4] <= small[:4] + tol[:4])
    assert np.all(big[4:] >= small[4:] - tol[4:])


@pytest.mark.parametrize("mode", [GL, ST])
def test_homogeneity(mode):
    gamma = 1.4
    rng = np.random.default_rng(8)
    prims = _random_stencil(rng, 2, 4)
    lo, hi = (-10.0, -10.0), (10.0, 10.0)
    b1, _ = run_bounds(2, gamma, prims, mode, (48, 48), lo, hi, k=4.0, r=1e-3)
    c = 37.5
    prims_c = [(c * rho, U, c * p) for rho, U, p in prims]
    b2, _ = run_bounds(2, gamma, prims_c, mode, (48, 48), lo, hi, k=4.0, r=1e-3)
    assert np.allclose(b2, c * b1, rtol=1e-13, atol=1e-13 * c * np.abs(b1).max())


def test_reflection_symmetry():
    gamma = 1.4
    rng = np.random.default_rng(9)
    prims = _random_stencil(rng, 1, 6)
    refl = [(rho, (-U[0],), p) for rho, U, p in prims]
    b, _ = run_bounds(1, gamma, prims, GL, (301,), (-12.0,), (12.0,), r=1e-3)
    br, _ = run_bounds(1, gamma, refl, GL, (301,), (-12.0,), (12.0,), r=1e-3)
    s = np.abs(b).max()
    assert abs(br[0] - b[0]) < 1e-14 * s and abs(br[3] - b[3]) < 1e-14 * s
    assert abs(br[2] - b[2]) < 1e-14 * s and abs(br[5] - b[5]) < 1e-14 * s
    assert abs(br[1] + b[4]) < 1e-14 * s and abs(br[4] + b[1]) < 1e-14 * s


def test_relaxation_is_affine_in_r():
    gamma = 1.4
    rng = np.random.default_rng(10)
    prims = _random_stencil(rng, 2, 5)
    bs = [run_bounds(2, gamma, prims, ST, (40, 40), k=4.0, r=r)[0] for r in (0.0, 1e-3, 4e-3)]
    # rho and E bounds scale exactly by (1 -+ r)
    for v in (0, 3):
        assert bs[1][v] == pytest.approx(0.999 * bs[0][v], rel=1e-13)
        assert bs[1][4 + v] == pytest.approx(1.001 * bs[0][4 + v], rel=1e-13)
    # momentum bounds are affine in r
    s = np.abs(bs[0]).max()
    assert np.all(np.abs((bs[2] - bs[0]) - 4 * (bs[1] - bs[0])) < 1e-12 * s)


def test_inadmissible_state_flags_element():
    gamma = 1.4
    prims = [(1.0, (0.1,), 1.0), (1.0, (0.1,), -0.5)]
    b, s = run_bounds(1, gamma, prims, ST, (64,), k=4.0)
    assert s & oracle.ST_INADMISSIBLE
    assert np.all(np.isnan(b))


def test_density_floor_applies():
    gamma = 1.4
    # two cold, far-apart streams: the min envelope has almost no mass
    prims = [(1.0, (-5.0,), 1e-4), (1.0, (5.0,), 1e-4)]
    b, s = run_bounds(1, gamma, prims, ST, (400,), k=4.0, r=0.0, floor=1e-12)
    assert b[0] == 1e-12 and (s & oracle.ST_RHO_FLOOR)
