"""The seeded generators hit the stated atom counts, densities and element mixes."""
import numpy as np
import pytest

from paper_2401_03180_amd import synth


def test_water_small():
    s = synth.water_small()
    assert s.n_atoms == 1536 and s.periodic
    assert s.mass_density_g_cm3() == pytest.approx(1.0, abs=0.01)
    assert np.all(np.bincount(s.elem) == [512, 1024])
    assert s.rc < 0.5 * s.box.min()
    # rigid geometry: O-H 0.1 nm
    P = s.positions()
    assert np.allclose(np.linalg.norm(P[1::3] - P[0::3], axis=1), 0.1, atol=1e-12)
    # zero net momentum
    m = 1 / s.inv_mass
    assert abs((m * s.vx).sum()) < 1e-9


def test_water_pulse_schedule():
    s = synth.water_pulse()
    assert s.n_atoms == 98304
    assert s.mass_density_g_cm3() == pytest.approx(1.0, abs=0.01)
    assert s.lambda_d[0, 0] == 1.0 and s.lambda_d[0, 1000] == pytest.approx(0.15)
    assert s.g[0].argmax() == 500 and s.g[0].max() == pytest.approx(1.0)
    assert s.base.max() == 5e-3


def test_water_pulse_other_time_step():
    # the same schedule in time at half the step: ramp end, pulse peak and the
    # ionization probability per unit time unchanged; the default is the 0.1 fs box
    s, h = synth.water_pulse(n_steps=1000), synth.water_pulse(n_steps=2000, dt_fs=0.05)
    assert h.dt == pytest.approx(s.dt / 2)
    assert np.array_equal(h.lambda_d[0, ::2], s.lambda_d[0])
    assert h.g[0].argmax() == 1000
    np.testing.assert_allclose(h.g[0, ::2], s.g[0], rtol=1e-12, atol=1e-300)
    assert h.base.max() / h.dt == pytest.approx(s.base.max() / s.dt, rel=1e-12)
    assert np.array_equal(h.x, s.x) and np.array_equal(h.vx, s.vx)
    d = synth.water_pulse(n_steps=1000, dt_fs=0.1)
    assert all(np.array_equal(getattr(d, n), getattr(s, n))
               for n in ("lambda_d", "g", "base", "x", "vx"))


def test_protein_mix():
    s = synth.protein_crystal()
    assert s.n_atoms == 524288
    assert np.all(np.bincount(s.elem) == synth.PROTEIN_COUNTS)
    assert s.mass_density_g_cm3() == pytest.approx(1.29, abs=0.01)
    assert list(s.qmax) == [1, 6, 7, 8, 16]


def test_methane_clusters():
    s = synth.methane_clusters()
    n = np.diff(s.sys_offsets)
    assert s.n_systems == 256 and not s.periodic
    assert n.min() >= 1000 and n.max() <= 20000 and np.all(n % 5 == 0)
    assert 1.3e6 < s.n_atoms < 2.0e6
    assert len(set(s.seeds.tolist())) == 256
    # per-system atom ids restart at zero
    assert s.atom_id[s.sys_offsets[1]] == 0
    # Lennard-Jones between C atoms only (no bonded terms or exclusions on this path)
    assert s.c6[0, 0] > 0 and s.c12[0, 0] > 0
    assert not s.c6[1].any() and not s.c12[1].any() and not s.c6[:, 1].any()


def test_water_large_counts():
    s = synth.water_large(n_per_dim=16, L=34.8 / 7)
    assert s.n_atoms % 3 == 1
    full = synth.water_large()
    assert full.n_atoms == 4194304


def test_subsystem_is_the_system_alone():
    s = synth.methane_clusters(n_clusters=4, lo=100, hi=400, n_steps=3)
    b = 2
    sb = s.subsystem(b)
    a0, a1 = s.sys_offsets[b], s.sys_offsets[b + 1]
    assert sb.n_systems == 1 and sb.n_atoms == a1 - a0
    assert np.array_equal(sb.x, s.x[a0:a1]) and np.array_equal(sb.atom_id, s.atom_id[a0:a1])
    assert np.array_equal(sb.g[0], s.g[b]) and sb.seeds[0] == s.seeds[b]
