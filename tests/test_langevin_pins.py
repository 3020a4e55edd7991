"""Pins of the oracle's Langevin coupling (section II.B, Eq. 13-14): the random
numbers are standard normals, the deterministic part is the exact solution of the
friction term, and the stationary state and velocity autocorrelation are those of the
Ornstein-Uhlenbeck process the coupling defines (CPU only)."""
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2401_03180_amd import synth


def _state(sys):
    pos = [sys.x.copy(), sys.y.copy(), sys.z.copy()]
    vel = [sys.vx.copy(), sys.vy.copy(), sys.vz.copy()]
    zero = np.zeros(sys.n_atoms)
    return pos, vel, (zero, zero, zero)


def test_normals_are_independent_standard_normals():
    z = np.array([oracle.langevin_normals(a, s, b, 2401031800 + b)
                  for a in range(400) for s in range(1, 41) for b in range(2)])
    n = z.shape[0]
    assert np.all(np.abs(z.mean(axis=0)) < 5.0 / np.sqrt(n))
    assert np.all(np.abs(z.var(axis=0) - 1.0) < 5.0 * np.sqrt(2.0 / n))
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5.0 / np.sqrt(n))
    for k in range(3):
        assert stats.kstest(z[:, k], "norm").pvalue > 1e-4
    # a different step, system or seed gives different numbers
    a = oracle.langevin_normals(7, 5, 0, 11)
    for other in ((7, 6, 0, 11), (7, 5, 1, 11), (7, 5, 0, 12), (8, 5, 0, 11)):
        assert not np.allclose(a, oracle.langevin_normals(*other))


def test_zero_temperature_is_the_exact_friction_solution():
    """kT = 0 and F = 0: v_N = c1^N v_0 and x_N = x_0 + (dt/2)(1 + c1) v_0 (1 - c1^N)/(1 - c1)."""
    s = synth.water_small(n_steps=60)
    pos, vel, F = _state(s)
    gamma = np.array([[3.0, 20.0]])                    # ps^-1 per element (O, H)
    c1 = oracle.langevin_c1(gamma, s.dt)
    kt = np.zeros((1, s.n_steps + 1))
    x0, v0 = pos[0].copy(), vel[0].copy()
    N = 60
    for step in range(1, N + 1):
        oracle.vv_langevin(s, step, c1, kt, F, pos, vel)
    c = c1[0, s.elem]
    assert np.allclose(vel[0], c ** N * v0, rtol=1e-12, atol=0)
    xN = x0 + 0.5 * s.dt * (1.0 + c) * v0 * (1.0 - c ** N) / (1.0 - c)
    assert np.allclose(pos[0], xN, rtol=0, atol=1e-13)


def test_no_friction_reduces_to_velocity_verlet():
    s = synth.water_small(n_steps=4)
    rng = np.random.default_rng(3)
    f = tuple(rng.normal(0, 50.0, s.n_atoms) for _ in range(3))
    p1, v1, _ = _state(s)
    p2, v2, _ = _state(s)
    oracle.vv_langevin(s, 1, np.ones((1, 2)), np.full((1, 5), 2.5), f, p1, v1)
    oracle.vv(0, s.dt, s.inv_mass, f, p2, v2)
    for k in range(3):
        assert np.array_equal(v1[k], v2[k])
        assert np.allclose(p1[k], p2[k], rtol=0, atol=1e-15)


@pytest.fixture(scope="module")
def stationary_run():
    """Zero forces, constant k_B T_e, c1 = 0.8 for both elements: 400 steps from rest."""
    s = synth.water_small(n_steps=400)
    pos, vel, F = _state(s)
    for v in vel:
        v[:] = 0.0
    kT = 2.5                                            # kJ/mol
    c1 = np.full((1, 2), 0.8)
    kt = np.full((1, s.n_steps + 1), kT)
    hist = []
    for step in range(1, 401):
        oracle.vv_langevin(s, step, c1, kt, F, pos, vel)
        hist.append(np.stack([v.copy() for v in vel]))
    return s, kT, 0.8, np.array(hist)                  # [step, 3, N]


def test_stationary_velocity_variance_is_kT_over_m(stationary_run):
    """<m v^2> = kT per component: the exact OU update keeps the equilibrium variance."""
    s, kT, c1, h = stationary_run
    w = h[100:] ** 2 / s.inv_mass[None, None, :] / kT   # m v^2 / kT, unit mean
    mean = w.mean()
    # correlation time of v^2 ~ 1/(1 - c1^2) steps: effective samples
    n_eff = w[:, :, :].size * (1.0 - c1 ** 2) / (1.0 + c1 ** 2)
    assert abs(mean - 1.0) < 5.0 * np.sqrt(2.0 / n_eff)


def test_velocity_autocorrelation_is_c1_power(stationary_run):
    """<v(t) v(t + n dt)> / <v^2> = c1^n for the OU process."""
    s, kT, c1, h = stationary_run
    v = h[100:] / np.sqrt(s.inv_mass)[None, None, :]    # sqrt(m) v: variance kT
    base = (v * v).mean()
    for n in (1, 2, 5):
        acf = (v[:-n] * v[n:]).mean() / base
        assert abs(acf - c1 ** n) < 0.02
