"""Pins of the oracle's hybrid ion-sphere / Debye potential (section II.A, Eq. 4-7).

Reading: inside r' the ion-sphere form Q/r + c1 - c2 r^2, outside the Debye form
c3 exp(-r/lambda)/r, r' from Eq. 7, c1..c3 from matching value, slope and curvature
at r' (the oracle solves the three linear conditions numerically).  The pins come
from elsewhere: a closed form of c3 and c2 worked by hand from the same conditions
(evaluated in 40-digit arithmetic), the ion-sphere potential of Eq. 5 (which the
inner branch must equal up to a constant, with R from Eq. 4), the limits of Eq. 7,
the Debye potential as the high-density limit, and the force as minus the energy
gradient (CPU only)."""
import math

import mpmath
import numpy as np
import pytest

import oracle
from paper_2401_03180_amd import synth

GRID = [(Q, lam, ne) for Q in (1, 2, 5, 8, 16) for lam in (0.05, 0.15, 0.5, 1.0, 3.0)
        for ne in (1e-3, 0.1, 5.0, 74.0, 300.0)]


def _closed_form(Q, lam, ne, rp=None):
    """Hand-worked solution in 40-digit arithmetic.  Eliminating c2 between the slope
    and curvature conditions gives c3 = 3Q / (r'^3 u0 (t^2 + t/r' + 1/r'^2)) with
    u0 = e^{-r'/lambda}/r' and t = 1/lambda + 1/r'; the slope condition then gives
    c2 = (c3 u0 t - Q/r'^2) / (2 r') and the value condition c1.  rp: evaluate at this
    r' instead of Eq. 7's."""
    mpmath.mp.dps = 40
    Q, lam, ne = mpmath.mpf(Q), mpmath.mpf(lam), mpmath.mpf(ne)
    R = mpmath.cbrt(3 * Q / (4 * mpmath.pi * ne))
    if rp is None:
        rp = lam * (mpmath.cbrt((R / lam) ** 3 + 1) - 1)
    rp = mpmath.mpf(rp)
    u0 = mpmath.exp(-rp / lam) / rp
    t = 1 / lam + 1 / rp
    c3 = 3 * Q / (rp ** 3 * u0 * (t * t + t / rp + 1 / rp ** 2))
    c2 = (c3 * u0 * t - Q / rp ** 2) / (2 * rp)
    c1 = c3 * u0 - Q / rp + c2 * rp ** 2
    return float(R), float(rp), float(c1), float(c2), float(c3)


@pytest.mark.parametrize("Q,lam,ne", GRID)
def test_coefficients_match_hand_solution(Q, lam, ne):
    """The numerical solve against the hand solution at the same r'; r' against Eq. 7
    in 40 digits (Eq. 7 loses about eps/a^3 to cancellation, a = R/lambda)."""
    h = oracle.hybrid_coeffs(Q, lam, ne)
    R, rp, _, _, _ = _closed_form(Q, lam, ne)
    a3 = (R / lam) ** 3
    assert h[0] == pytest.approx(rp, rel=1e-15 * (4 + 4 / a3))
    assert 0.0 < h[0] < R
    _, _, c1, c2, c3 = _closed_form(Q, lam, ne, rp=h[0])
    scale = Q / h[0] ** 3                     # size of the curvature condition's terms
    assert h[3] == pytest.approx(c3, rel=1e-10)
    assert abs(h[2] - c2) <= 1e-12 * scale
    assert abs(h[1] - c1) <= 1e-12 * Q / h[0]


@pytest.mark.parametrize("Q,lam,ne", [g for g in GRID
                                      if (3 * g[0] / (4 * math.pi * g[2])) ** (1 / 3) >= 0.3 * g[1]])
def test_curvature_is_the_uniform_electron_sphere(Q, lam, ne):
    """With r' from Eq. 7 the matched inner curvature is that of Eq. 5's uniform
    electron sphere: c2 = -Q/(2R^3) = -2 pi n_e / 3, the same for every charge
    (checked where Eq. 7 keeps its digits, R >= 0.3 lambda)."""
    h = oracle.hybrid_coeffs(Q, lam, ne)
    assert h[2] == pytest.approx(-2.0 * math.pi * ne / 3.0, rel=1e-9)


@pytest.mark.parametrize("Q,lam,ne", [(1, 0.15, 74.0), (8, 0.15, 74.0), (3, 0.5, 5.0),
                                      (1, 1.0, 1.43e-3), (16, 0.05, 300.0)])
def test_inner_branch_is_ion_sphere_plus_constant(Q, lam, ne):
    """For r < r' the potential differs from Eq. 5 (R from Eq. 4) by one constant."""
    h = oracle.hybrid_coeffs(Q, lam, ne)
    R = (3.0 * Q / (4.0 * math.pi * ne)) ** (1.0 / 3.0)
    rs = h[0] * np.array([0.05, 0.2, 0.5, 0.8, 0.99])
    d = [oracle.hybrid_phi(Q, h, 1.0 / lam, r)[0] - (Q / r - Q / (2 * R) * (3 - r * r / R ** 2))
         for r in rs]
    assert np.ptp(d) <= 1e-9 * max(abs(v) for v in d) + 1e-9 * Q / h[0]


@pytest.mark.parametrize("Q,lam,ne", [(1, 0.15, 74.0), (8, 0.15, 74.0), (3, 0.5, 5.0),
                                      (2, 1.0, 0.1), (16, 0.05, 300.0)])
def test_value_slope_curvature_continuous_at_r_prime(Q, lam, ne):
    h = oracle.hybrid_coeffs(Q, lam, ne)
    kap, rp = 1.0 / lam, h[0]
    eps = 1e-6 * rp

    def branch(side):
        """phi, phi' and phi'' of one branch at r', by central differences inside it."""
        c = rp - 3 * eps if side < 0 else rp + 3 * eps
        f = [oracle.hybrid_phi(Q, h, kap, c + k * eps)[0] for k in (-1, 0, 1)]
        p = oracle.hybrid_phi(Q, h, kap, c)
        d1 = -p[1] / c
        d2 = (f[0] - 2 * f[1] + f[2]) / eps ** 2
        # move the values to r' with their Taylor terms
        return f[1] - side * 3 * eps * d1, d1, d2

    vi, si, ci = branch(-1)
    vo, so, co = branch(+1)
    scale = Q / rp
    assert abs(vi - vo) <= 1e-7 * scale
    assert abs(si - so) <= 1e-4 * scale / rp
    assert abs(ci - co) <= 1e-3 * scale / rp ** 2


def test_transition_radius_limits():
    """Eq. 7: r' -> R - lambda as lambda/R -> 0 and r' -> R^3/(3 lambda^2) as lambda/R -> inf."""
    Q, ne = 4.0, 2.0
    R = (3.0 * Q / (4.0 * math.pi * ne)) ** (1.0 / 3.0)
    lam = 1e-3 * R
    assert oracle.hybrid_coeffs(Q, lam, ne)[0] == pytest.approx(R - lam, rel=1e-6)
    lam = 1e3 * R
    h = oracle.hybrid_coeffs(Q, lam, ne)
    assert h[0] == pytest.approx(R ** 3 / (3 * lam ** 2), rel=1e-3)
    assert h[3] == pytest.approx(Q, rel=1e-3)          # bare charge seen outside
    assert np.array_equal(oracle.hybrid_coeffs(Q, math.inf, ne), [0.0, 0.0, 0.0, Q])
    assert np.array_equal(oracle.hybrid_coeffs(0, 0.3, ne), [0.0, 0.0, 0.0, 0.0])


def _charged_water(seed):
    s = synth.water_small(n_steps=2)
    rng = np.random.default_rng(seed)
    s.q = np.minimum(rng.integers(0, 4, s.n_atoms), s.qmax[s.elem]).astype(np.int8)
    return s


def test_high_density_limit_is_debye():
    """n_e -> infinity shrinks the ion sphere to nothing: the hybrid forces and energy
    become the Debye ones (Eq. 2 + Eq. 8)."""
    s = _charged_water(1)
    lam = 0.3
    kap = np.array([1.0 / lam])
    tab = oracle.hybrid_table([lam], [1e12], 9)
    h = oracle.forces(s, kappa=kap, hybrid=tab)
    d = oracle.forces(s, kappa=kap)
    for k in ("fx", "fy", "fz"):
        assert np.allclose(h[k], d[k], rtol=0, atol=1e-8 * d["a_atom"].max())
    assert h["epot"][0] == pytest.approx(d["epot"][0], rel=1e-8)
    assert h["npairs"] == d["npairs"]


def test_hybrid_newton_third_law_and_rows():
    s = _charged_water(2)
    lam = 0.15
    tab = oracle.hybrid_table([lam], [40.0], 9)
    h = oracle.forces(s, kappa=np.array([1 / lam]), hybrid=tab)
    scale = h["a_atom"].max()
    for k in ("fx", "fy", "fz"):
        assert abs(h[k].sum()) <= 1e-9 * scale * s.n_atoms ** 0.5
    rows = np.arange(0, s.n_atoms, 7)
    r = oracle.forces_rows(s, rows, kappa=np.array([1 / lam]), hybrid=tab)
    for k in ("fx", "fy", "fz"):
        assert np.allclose(r[k], h[k][rows], rtol=0, atol=1e-10 * scale)
    assert np.allclose(r["e_atom"], h["e_atom"][rows], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("q1,q2,r", [(3, 5, 0.05), (3, 5, 0.12), (3, 5, 0.6), (1, 8, 0.1),
                                     (6, 0, 0.3)])
def test_hybrid_pair_force_is_minus_gradient_and_symmetric(q1, q2, r):
    """Two ions with different r' (inside both, between, outside both): F = -dE/dr by
    central differences; exchanging the ions leaves the energy unchanged."""
    from test_oracle_pins import two_atoms
    lam, ne = 0.15, 40.0
    tab = oracle.hybrid_table([lam], [ne], 9)
    u = np.array([0.48, -0.6, 0.64])

    def energy(rr, a, b):
        s = two_atoms(rr * u, a, b, c6=1e-3, c12=1e-6, lam=lam)
        return oracle.forces(s, kappa=np.array([1 / lam]), hybrid=tab)

    res = energy(r, q1, q2)
    h = 1e-6 * r
    dE = (energy(r + h, q1, q2)["epot"][0] - energy(r - h, q1, q2)["epot"][0]) / (2 * h)
    F2 = np.array([res["fx"][1], res["fy"][1], res["fz"][1]])
    assert F2 @ u == pytest.approx(-dE, rel=1e-6, abs=1e-9)
    assert energy(r, q2, q1)["epot"][0] == pytest.approx(res["epot"][0], rel=1e-14)
