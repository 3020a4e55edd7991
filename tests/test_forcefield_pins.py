"""Pins of the oracle's force-field terms of section II.B (readings): Morse bonds and
harmonic angles scaled by the mean charge of their atoms (Eq. 9, Eq. 10), LJ omitted
for bonded 1-2 and 1-3 pairs, and LJ radii scaled with the charge (Eq. 11).  Pinned by
the Morse closed form, forces as minus numerical energy gradients, vanishing net force
and torque, a molecule at its equilibrium geometry, the periodic image invariance, and
the shifted LJ minimum (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from paper_2401_03180_amd import synth
from test_oracle_pins import two_atoms


def _atoms(p, q, periodic=False, L=4.0, types=None):
    p = np.asarray(p, dtype=np.float64)
    n = p.shape[0]
    s = two_atoms([0.3, 0.0, 0.0], 0, 0, periodic=periodic, L=L)
    typ = np.zeros(n, np.uint8) if types is None else np.asarray(types, np.uint8)
    return synth.System(**{**s.__dict__, "x": p[:, 0].copy(), "y": p[:, 1].copy(),
                           "z": p[:, 2].copy(), "vx": np.zeros(n), "vy": np.zeros(n),
                           "vz": np.zeros(n), "elem": typ.copy(), "type": typ,
                           "atom_id": np.arange(n, dtype=np.uint32), "inv_mass": np.ones(n),
                           "q": np.asarray(q, np.int8),
                           "sys_offsets": np.array([0, n], dtype=np.int64)})


def _energy(s, ff, p):
    return oracle.bonded(s, ff, x=p[:, 0], y=p[:, 1], z=p[:, 2])["epot"][0]


def _num_grad(s, ff, p, h=1e-7):
    g = np.zeros_like(p)
    for a in range(p.shape[0]):
        for k in range(3):
            pp, pm = p.copy(), p.copy()
            pp[a, k] += h
            pm[a, k] -= h
            g[a, k] = (_energy(s, ff, pp) - _energy(s, ff, pm)) / (2 * h)
    return g


BOND = (430.0, 18.0, 0.109)


@pytest.mark.parametrize("q,c", [((0, 0), 1.0), ((1, 0), 0.5), ((1, 1), 0.0), ((3, 0), 0.0)])
def test_morse_closed_form_and_charge_scale(q, c):
    """V = c D_e (1 - e^{-beta (r - b_e)})^2 with c = max(0, 1 - (q1 + q2)/2)."""
    De, beta, be = BOND
    for r in (0.08, 0.109, 0.15, 0.4, 3.0):
        s = _atoms([[0, 0, 0], [r, 0, 0]], q)
        ff = oracle.ForceField(2, bonds=[[0, 1]], bond_par=[BOND])
        out = oracle.bonded(s, ff)
        V = c * De * (1 - math.exp(-beta * (r - be))) ** 2
        assert out["epot"][0] == pytest.approx(V, rel=1e-12, abs=1e-12)
        assert out["fx"][0] == pytest.approx(-out["fx"][1], rel=1e-14, abs=1e-14)
    s = _atoms([[0, 0, 0], [be, 0, 0]], q)
    assert np.all(oracle.bonded(s, oracle.ForceField(2, bonds=[[0, 1]], bond_par=[BOND]))["fx"]
                  == 0.0)


def test_bonded_forces_are_minus_gradient():
    rng = np.random.default_rng(4)
    p = np.array([[0.0, 0.0, 0.0], [0.11, 0.01, -0.02], [-0.03, 0.1, 0.04],
                  [0.02, -0.05, 0.1]]) + rng.normal(0, 0.01, (4, 3))
    s = _atoms(p, [1, 0, 2, 0])
    ff = oracle.ForceField(4, bonds=[[0, 1], [0, 2], [0, 3]], bond_par=[BOND] * 3,
                           angles=[[1, 0, 2], [1, 0, 3], [2, 0, 3]],
                           angle_par=[(330.0, 1.9106)] * 3)
    out = oracle.bonded(s, ff)
    F = np.stack([out["fx"], out["fy"], out["fz"]], 1)
    G = _num_grad(s, ff, p)
    assert np.allclose(F, -G, rtol=1e-6, atol=1e-5)
    assert np.allclose(F.sum(0), 0.0, atol=1e-9)                    # no net force
    assert np.allclose(np.cross(p, F).sum(0), 0.0, atol=1e-9)       # no net torque


def test_molecule_at_equilibrium_has_no_bonded_force():
    tmpl = synth.methane_template() + np.array([1.0, 1.0, 1.0])
    s = _atoms(tmpl, [0] * 5)
    d = synth.molecular_force_field(s, "methane")
    ff = oracle.ForceField(5, bonds=d["bonds"], bond_par=d["bond_par"], angles=d["angles"],
                           angle_par=d["angle_par"])
    out = oracle.bonded(s, ff)
    assert abs(out["epot"][0]) < 1e-20
    for k in ("fx", "fy", "fz"):
        assert np.max(np.abs(out[k])) < 1e-9


def test_periodic_image_invariance():
    """A molecule straddling the periodic boundary feels the same bonded forces as the
    same molecule in one piece."""
    p = synth.methane_template() * 1.07 + np.array([0.02, 1.0, 3.99])
    ff_d = synth.molecular_force_field(_atoms(p, [0] * 5), "methane")
    ff = oracle.ForceField(5, bonds=ff_d["bonds"], bond_par=ff_d["bond_par"],
                           angles=ff_d["angles"], angle_par=ff_d["angle_par"])
    whole = oracle.bonded(_atoms(p, [1, 0, 0, 1, 0], periodic=True, L=4.0), ff)
    wrapped = p % 4.0
    split = oracle.bonded(_atoms(wrapped, [1, 0, 0, 1, 0], periodic=True, L=4.0), ff)
    for k in ("fx", "fy", "fz"):
        assert np.allclose(whole[k], split[k], rtol=1e-9, atol=1e-9)
    assert split["epot"][0] == pytest.approx(whole["epot"][0], rel=1e-9)


def test_exclusion_removes_only_lj():
    """An excluded pair interacts through the screened Coulomb term only: the same
    as the pair with its LJ parameters set to zero."""
    for q1, q2 in ((0, 0), (2, 1)):
        a = two_atoms([0.2, 0.05, 0.0], q1, q2, c6=2e-3, c12=3e-6, lam=0.4)
        b = two_atoms([0.2, 0.05, 0.0], q1, q2, c6=0.0, c12=0.0, lam=0.4)
        ff = oracle.ForceField(2, excl=[[1, 0]])
        fa = oracle.forces(a, ff=ff)
        fb = oracle.forces(b)
        for k in ("fx", "fy", "fz", "e_atom"):
            assert np.array_equal(fa[k], fb[k])
        assert oracle.forces(a)["fx"][0] != fa["fx"][0]            # the LJ term matters


def _lj_part(r, q, z, sig, eps):
    """x-force on atom 1 of a two-atom pair at separation r (no screening) from the
    Lennard-Jones term alone: the full pair with the Eq. 11 charge scaling of the
    radii minus the Coulomb-only pair; and the same for the energy."""
    c6, c12 = synth.lj_tables_lorentz_berthelot(sig, eps)
    full = two_atoms([r, 0, 0], q[0], q[1], lam=math.inf)
    full.type = np.array([0, 1], np.uint8)
    full.c6, full.c12 = c6, c12
    coul = two_atoms([r, 0, 0], q[0], q[1], lam=math.inf)
    ff = oracle.ForceField(2, inv_z=1.0 / np.asarray(z, np.float64), sigma=np.asarray(sig))
    a, b = oracle.forces(full, ff=ff), oracle.forces(coul)
    return a["fx"][1] - b["fx"][1], a["epot"][0] - b["epot"][0]


@pytest.mark.parametrize("q1,q2,z1,z2", [(0, 0, 6, 6), (2, 0, 6, 6), (3, 4, 8, 6), (1, 1, 1, 6)])
def test_charge_scaled_lj_minimum(q1, q2, z1, z2):
    """Equal neutral radii: with no screening the LJ part of the force vanishes at
    2^(1/6) sigma s with s = (1 - q1/Z1 + 1 - q2/Z2)/2 (Eq. 11: each radius shrinks
    by its own c, the pair radius is their mean)."""
    sigma, eps = 0.3, 0.5
    s_fac = 0.5 * ((1 - q1 / z1) + (1 - q2 / z2))
    if s_fac == 0.0:
        pytest.skip("no LJ left")
    rstar = 2 ** (1 / 6) * sigma * s_fac
    args = ((q1, q2), (z1, z2), (sigma, sigma), (eps, eps))
    scale = 24 * eps / rstar
    assert abs(_lj_part(rstar, *args)[0]) < 1e-9 * scale
    assert _lj_part(rstar * 0.97, *args)[0] > 0.0                  # repulsive inside
    assert _lj_part(rstar * 1.03, *args)[0] < 0.0                  # attractive outside


@pytest.mark.parametrize("q1,q2", [(0, 0), (0, 1), (3, 0), (5, 1), (2, 1)])
def test_charge_scaled_lj_unequal_radii(q1, q2):
    """Unequal neutral radii (water O 0.3166 nm, Z 8 against H 0.10 nm, Z 1): Eq. 11
    shrinks each radius to c sigma with c = 1 - q/Z, and the pair radius is the mean
    of the scaled radii, so the LJ force vanishes at r* = 2^(1/6) (c1 s1 + c2 s2)/2
    and the LJ energy there is -sqrt(e1 e2) (epsilon is not scaled).  For O-H+ this
    is the case where scaling the pair radius by the mean of c would differ."""
    sig, eps, z = (0.3166, 0.10), (0.65, 0.02), (8, 1)
    c = (1 - q1 / z[0], 1 - q2 / z[1])
    rad = 0.5 * (c[0] * sig[0] + c[1] * sig[1])
    rstar = 2 ** (1 / 6) * rad
    args = ((q1, q2), z, sig, eps)
    e12 = math.sqrt(eps[0] * eps[1])
    f, e = _lj_part(rstar, *args)
    assert abs(f) < 1e-9 * 24 * e12 / rstar
    assert e == pytest.approx(-e12, rel=1e-9)
    assert _lj_part(rstar * 0.97, *args)[0] > 0.0
    assert _lj_part(rstar * 1.03, *args)[0] < 0.0
    # the other reading (pair radius times the mean of c) puts the minimum elsewhere
    # whenever the charges differ in their c
    other = 2 ** (1 / 6) * 0.5 * (sig[0] + sig[1]) * 0.5 * (c[0] + c[1])
    if abs(c[0] - c[1]) > 1e-12:
        assert abs(_lj_part(other, *args)[0]) > 1e-3 * 24 * e12 / rstar


def test_charge_scaled_lj_needs_radii():
    with pytest.raises(ValueError):
        oracle.ForceField(2, inv_z=[1.0, 1.0])


def test_force_field_newton_and_rows():
    s = synth.methane_clusters(n_clusters=2, lo=300, hi=600, n_steps=2)
    rng = np.random.default_rng(8)
    s.q = np.minimum(rng.integers(0, 4, s.n_atoms), s.qmax[s.elem]).astype(np.int8)
    d = synth.molecular_force_field(s, "methane")
    s.c6, s.c12 = d["c6"], d["c12"]
    ff = oracle.ForceField(s.n_atoms, inv_z=1.0 / d["z"], sigma=d["sigma"], excl=d["excl"],
                           bonds=d["bonds"],
                           bond_par=d["bond_par"], angles=d["angles"], angle_par=d["angle_par"])
    nb = oracle.forces(s, ff=ff)
    bo = oracle.bonded(s, ff)
    for k in ("fx", "fy", "fz"):
        for b in range(s.n_systems):
            a0, a1 = s.sys_offsets[b], s.sys_offsets[b + 1]
            tot = nb[k][a0:a1] + bo[k][a0:a1]
            assert abs(tot.sum()) < 1e-8 * np.abs(tot).max()
    rows = np.arange(0, s.n_atoms, 5)
    r = oracle.forces_rows(s, rows, ff=ff)
    for k in ("fx", "fy", "fz"):
        assert np.allclose(r[k], nb[k][rows], rtol=1e-12, atol=1e-9)
