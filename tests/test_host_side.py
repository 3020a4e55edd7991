"""Host-side pieces that need no GPU: the benchmark's one-GPU contract, the library's
host helpers for g(r) and S(q) against the oracle, and the synthetic inputs of the
optional terms (electron density consistent with the Debye-length schedule through
Eq. 3, coupling tables, molecular topologies)."""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2401_03180_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_time_step_option():
    # the pulse box at another step keeps its schedule in time (twice the steps at half
    # the step); the option is refused for the other workloads
    sys.path.insert(0, ROOT)
    import bench
    assert bench.schedule_len("water_98304") == 1000
    assert bench.schedule_len("water_98304", 0.05) == 2000
    s = bench.make_system("water_98304", 0, 0.05)
    assert s.n_steps == 2000 and s.dt == pytest.approx(5e-5)
    with pytest.raises(SystemExit):
        bench.make_system("water_1536", 0, 0.05)


def test_host_rdf_helpers_match_oracle():
    from paper_2401_03180_amd import md
    rng = np.random.default_rng(11)
    counts = rng.integers(0, 50000, 250).astype(np.uint64)
    for same in (True, False):
        g = md.md_rdf_normalize(counts, 1.0, 32768, 65536, same, 9.93 ** 3)
        assert np.allclose(g, oracle.rdf_normalize(counts, 1.0, 32768, 65536, same, 9.93 ** 3),
                           rtol=1e-13, atol=0)
    q = np.linspace(0.5, 100.0, 64)
    S = md.md_structure_factor(g, 1.0, 33.4, q)
    assert np.allclose(S, oracle.structure_factor(g, 1.0, 33.4, q), rtol=1e-12, atol=1e-12)
    for bad in (np.array([0.0]), np.array([-1.0])):
        with pytest.raises(md.MDError):
            md.md_structure_factor(g, 1.0, 33.4, bad)
    with pytest.raises(md.MDError):
        md.md_rdf_normalize(counts, 1.0, 10, 10, True, 0.0)


def test_electron_density_reproduces_the_debye_schedule():
    """Eq. 3 with the synthetic T_e and n_e gives back the workload's lambda_D."""
    s = synth.water_pulse(n_steps=1000)
    te = synth.electron_temperature_ev(s)
    ne = synth.hybrid_inputs(s)
    for k in (0, 250, 500, 750, 1000):
        lam = oracle.debye_length_nm(te[0, k], ne[0, k] * 1e27)
        assert lam == pytest.approx(s.lambda_d[0, k], rel=1e-9)
    assert np.all(np.diff(te[0]) >= 0.0)
    assert te[0, 0] == pytest.approx(0.0259 + (30.0 - 0.0259) * s.g[0, 0] / s.g[0].sum())
    assert te[0, -1] == pytest.approx(30.0)


def test_langevin_inputs_shapes_and_units():
    s = synth.methane_clusters(n_clusters=3, lo=300, hi=600, n_steps=20)
    gamma, kt = synth.langevin_inputs(s)
    assert gamma.shape == (3, 2) and kt.shape == (3, 21)
    assert np.all(gamma[:, 0] == 2.0) and np.all(gamma[:, 1] == 5.0)
    te = synth.electron_temperature_ev(s)
    assert np.allclose(kt, te * synth.EV_KJ_PER_MOL)
    # 300 K is k_B T = 2.494 kJ/mol
    assert 0.0259 * synth.EV_KJ_PER_MOL == pytest.approx(synth.K_B * 300.0, rel=2e-3)


@pytest.mark.parametrize("kind,per,nh", [("water", 3, 2), ("methane", 5, 4)])
def test_molecular_topology(kind, per, nh):
    s = synth.water_small(2) if kind == "water" else synth.methane_clusters(
        n_clusters=2, lo=300, hi=400, n_steps=2)
    d = synth.molecular_force_field(s, kind)
    nmol = s.n_atoms // per
    assert d["bonds"].shape == (nmol * nh, 2)
    assert d["angles"].shape == (nmol * nh * (nh - 1) // 2, 3)
    # bonds join the heavy atom (element 0) to a hydrogen of the same molecule, and the
    # bond length in the synthetic geometry is the Morse equilibrium distance
    b = d["bonds"]
    assert np.all(s.elem[b[:, 0]] == 0) and np.all(s.elem[b[:, 1]] == 1)
    assert np.all(b[:, 0] // per == b[:, 1] // per)
    r = np.sqrt((s.x[b[:, 0]] - s.x[b[:, 1]]) ** 2 + (s.y[b[:, 0]] - s.y[b[:, 1]]) ** 2 +
                (s.z[b[:, 0]] - s.z[b[:, 1]]) ** 2)
    r = np.minimum(r, np.inf)
    if s.periodic:
        L = s.box[0, 0]
        dv = np.stack([s.x[b[:, 0]] - s.x[b[:, 1]], s.y[b[:, 0]] - s.y[b[:, 1]],
                       s.z[b[:, 0]] - s.z[b[:, 1]]], 1)
        dv -= L * np.round(dv / L)
        r = np.sqrt((dv ** 2).sum(1))
    assert np.allclose(r, d["bond_par"][0, 2], atol=0.02)
    a = d["angles"]
    assert np.all(s.elem[a[:, 1]] == 0) and np.all(s.elem[a[:, [0, 2]]] == 1)
    assert d["excl"].shape[0] == b.shape[0] + a.shape[0]
    assert np.all(d["c6"] > 0) and np.all(d["c6"] == d["c6"].T)


def test_tuned_cache_covers_every_benchmark_leg():
    """The launch-configuration cache holds an entry for each workload the benchmark
    times (the 4.19 M-atom box in both precisions, the pulse box, the protein crystal,
    the batched methane clusters), each within the library's accepted ranges."""
    import json
    from paper_2401_03180_amd import autotune
    data = json.load(open(autotune.CACHE))
    need = ["gfx950|water_4194304|prec0", "gfx950|water_4194304|prec1",
            "gfx950|water_98304|prec1", "gfx950|protein_524288|prec1",
            "gfx950|methane_256|prec1"]
    for key in need:
        assert key in data, key
    for key, e in data.items():
        assert e["cluster_group"] in (1, 2, 4, 8), key
        assert 0.0 < e["skin"] < 0.5, key
        assert 0 <= e["fast_capacity"] <= 65536, key
        assert e["ms_per_step"] > 0.0, key
        # the chosen configuration is the fastest trial of its search
        best = min(t["ms_per_step"] for t in e.get("trials", [e]))
        assert e["ms_per_step"] <= best + 1e-9, key
