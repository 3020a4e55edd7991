"""GPU parity on the workloads as the benchmark runs them: the 98,304-atom pulse box
through the pulse (graph replays, automatic rebuilds, fast atoms) with the partners
of sampled atoms compared one by one, and energy conservation of a closed system
(no ionization, truncation negligible) against the oracle's."""
import math

import numpy as np
import pytest

import oracle
from paper_2401_03180_amd import synth
from gpu_util import force_error, oracle_kappa, require_gpu, say

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5}          # MD_FP64, MD_FP32_KAHAN
PRECS = [0, 1]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _partners(pairs, rows):
    """Per sampled row the ascending partners from an (i, j) pair array."""
    both = np.concatenate([pairs, pairs[:, ::-1]])
    both = both[np.isin(both[:, 0], rows)]
    both = both[np.lexsort((both[:, 1], both[:, 0]))]
    starts = np.searchsorted(both[:, 0], rows, side="left")
    ends = np.searchsorted(both[:, 0], rows, side="right")
    return [both[a:b, 1] for a, b in zip(starts, ends)]


@pytest.mark.parametrize("prec", PRECS)
def test_water_pulse_through_the_pulse(prec):
    """The 98,304-atom box replayed as graphs from step 0 to step 550 (pulse peak at
    step 500): charges bit-exact, then for 1,000 sampled atoms the partner set equal to
    the oracle's one by one and the forces within the tolerance, at the positions and
    charges the GPU reached."""
    import torch
    from paper_2401_03180_amd import md
    steps = 550
    s = synth.water_pulse(n_steps=1000)
    say("water_98304 graph 0..550 prec", prec)
    eng = md.Engine(s, prec)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        eng.set_step(0, st)
        eng.build(md.MD_BUILD_FORCE, st)
        eng.forces(energy=True, stream=st)
        g = eng.graph(md.MD_BUILD_AUTO, st, energy=True, ekin=True)
        for _ in range(steps):
            md.md_graph_launch(g, st)
        st.synchronize()
    assert eng.sync_check(raise_on_flags=False) == 0
    assert eng.get_step() == steps
    stats = eng.stats()
    assert stats["n_builds"] > 1                     # rebuilds happened on the way
    q = eng.host("q")
    qref = s.q.copy()
    for k in range(1, steps + 1):
        oracle.ionize(s, qref, k)
    assert np.array_equal(q, qref)
    assert (q > 0).mean() > 0.01                     # the pulse has charged the box
    x, y, z = eng.host("x"), eng.host("y"), eng.host("z")
    F = (eng.host("fx"), eng.host("fy"), eng.host("fz"))
    rng = np.random.default_rng(77 + prec)
    rows = np.sort(rng.choice(s.n_atoms, 1000, replace=False))
    ref = oracle.forces_rows(s, rows, q=q, x=x, y=y, z=z, kappa=oracle_kappa(s, steps))
    assert force_error(tuple(f[rows] for f in F), ref) <= TOL[prec]
    gp = _partners(eng.debug_pairs(prec=prec), rows)
    op = oracle.pairs_rows(s, rows, x=x, y=y, z=z)
    for r in range(rows.size):
        assert np.array_equal(gp[r], op[r]), rows[r]
    eng.close()


def _nve_box(seed=13):
    """343 atoms (mass 12) on a jittered 7^3 lattice of spacing 0.4 nm in a 2.8 nm
    periodic cube, fixed charges in {0, 1, 2}, LJ sigma 0.3 nm / eps 0.5 kJ/mol,
    lambda_D 0.05 nm (kappa rc = 20: truncation negligible), no ionization, 300 K."""
    rng = np.random.default_rng(seed)
    n, L = 343, 2.8
    P = synth.lattice_sites(7, L / 7) + rng.uniform(-0.03, 0.03, size=(n, 3))
    c6, c12 = synth.lj_tables_lorentz_berthelot([0.3], [0.5])
    v = rng.standard_normal((n, 3)) * math.sqrt(synth.K_B * 300.0 / 12.0)
    v -= v.mean(0)
    S = 1000
    return synth.System(
        name="nve", x=P[:, 0].copy(), y=P[:, 1].copy(), z=P[:, 2].copy(), vx=v[:, 0].copy(),
        vy=v[:, 1].copy(), vz=v[:, 2].copy(), elem=np.zeros(n, np.uint8),
        type=np.zeros(n, np.uint8), atom_id=np.arange(n, dtype=np.uint32),
        inv_mass=np.full(n, 1 / 12.0), q=rng.integers(0, 3, n).astype(np.int8),
        sys_offsets=np.array([0, n], np.int64), periodic=True, box=np.array([[L, L, L]]),
        rc=1.0, skin=0.1, dt=1e-3, n_steps=S, lambda_d=np.full((1, S + 1), 0.05),
        g=np.ones((1, S + 1)), base=np.zeros((1, 3)), qmax=np.array([2], np.int8), c6=c6,
        c12=c12, seeds=np.array([5], np.uint64))


def test_nve_drift_matches_oracle():
    """1,000 velocity-Verlet steps of 1 fs of a closed system: the total energy
    E = E_pot + E_kin of the FP64 path follows the oracle's step by step (its maximum
    deviation from E(0), the drift, agrees to 1e-6 of the energy scale); the FP32
    path's drift is reported and bounded by a few times the oracle's."""
    from paper_2401_03180_amd import md
    s = _nve_box()
    steps = s.n_steps
    ref = oracle.run(s, steps, record_every=1, ionize_on=False)
    e_ref = np.array(ref["epot"])[:, 0] + np.array(ref["ekin"])[:, 0]
    scale = np.abs(np.array(ref["epot"])[:, 0]).max() + np.array(ref["ekin"])[:, 0].max()
    drift_ref = np.max(np.abs(e_ref - e_ref[0]))
    assert drift_ref < 1e-3 * scale                  # the oracle itself conserves energy
    drifts = {}
    for prec in PRECS:
        say("nve drift prec", prec)
        eng = md.Engine(s, prec)
        eng.set_step(0)
        eng.build()
        eng.forces(energy=True)
        e = [eng.host("epot")[0] + oracle.ekin(s, eng.host("vx"), eng.host("vy"),
                                               eng.host("vz"))[0]]
        for _ in range(steps):
            eng.step(md.MD_BUILD_AUTO, energy=True, ekin=True)
            e.append(eng.host("epot")[0] + eng.host("ekin")[0])
        eng.sync_check()
        assert np.all(eng.host("q") == s.q)             # no ionization
        eng.close()
        e = np.array(e)
        drifts[prec] = np.max(np.abs(e - e[0]))
        if prec == 0:
            assert np.max(np.abs(e - e_ref)) <= 1e-6 * scale
            assert abs(drifts[0] - drift_ref) <= 1e-6 * scale
        else:
            assert drifts[1] <= 3.0 * drift_ref + 1e-5 * scale
    say("nve drift oracle %.3e fp64 %.3e fp32 %.3e (energy scale %.3e)"
        % (drift_ref, drifts[0], drifts[1], scale))
