"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same
seeded inputs.  Pair sets and integer charges must be bit-exact, the integrator
bit-exact given identical forces, and per-atom forces within
e_F = max_i |dF_i| / A_i <= 1e-10 (FP64 path) / 1e-5 (FP32 path)."""
import math

import numpy as np
import pytest

import oracle
from paper_2401_03180_amd import synth
from gpu_util import force_error, oracle_kappa, random_charges, require_gpu, say, sorted_pairs

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5}          # MD_FP64, MD_FP32_KAHAN
PRECS = [0, 1]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def make_engine(sys, prec, **kw):
    from paper_2401_03180_amd.md import Engine
    return Engine(sys, prec, **kw)


def set_q(eng, q):
    import torch
    eng.q.copy_(torch.as_tensor(q, dtype=torch.int8))


def gpu_forces(eng, prec):
    eng.forces(prec=prec, energy=True)
    eng.sync_check()
    return (eng.host("fx"), eng.host("fy"), eng.host("fz")), eng.host("epot")


# ------------------------------------------------------------------ small bulk water

@pytest.mark.parametrize("prec", PRECS)
def test_water_small_pairs_forces_energy(prec):
    s = synth.water_small()
    s.q = random_charges(s, 1)
    say("water_small pairs/forces prec", prec)
    eng = make_engine(s, prec)
    set_q(eng, s.q)
    eng.build()
    F, epot = gpu_forces(eng, prec)
    ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, 0))
    assert force_error(F, ref) <= TOL[prec]
    esc = np.abs(ref["e_atom"]).sum() * 2
    assert abs(epot[0] - ref["epot"][0]) <= TOL[prec] * esc
    gp = sorted_pairs(eng.debug_pairs(prec=prec))
    op = oracle.pairs(s)
    assert gp.shape == op.shape and np.array_equal(gp, op)
    # per-atom energies e_i = 1/2 sum_j phi_ij of the debug export
    e_atom, n = eng.atom_energies(prec)
    assert n == op.shape[0]
    de = np.abs(e_atom - ref["e_atom"])
    assert np.all(de <= TOL[prec] * (np.abs(ref["e_atom"]) + ref["a_atom"]))
    assert abs(e_atom.sum() - epot[0]) <= 1e-12 * esc
    st = eng.stats()
    assert st["flags"] == 0 and st["n_builds"] == 1
    eng.close()


@pytest.mark.parametrize("prec", PRECS)
def test_forces_with_other_screening_and_unscreened_lj(prec):
    s = synth.water_small()
    s.q = random_charges(s, 2, hi=9)
    s.lambda_d[:] = np.inf              # kappa = 0: plain Coulomb
    s.screen_lj = False
    say("unscreened prec", prec)
    eng = make_engine(s, prec)
    set_q(eng, s.q)
    eng.build()
    F, _ = gpu_forces(eng, prec)
    ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, 0))
    assert force_error(F, ref) <= TOL[prec]
    eng.close()


def _adversarial_system():
    """Pairs of atoms placed so that their FP64 r^2 straddles rc^2 by a few ulp, along
    axes, diagonals and across the periodic seam; pairs are 3 nm apart from each other."""
    rc, L = 1.0, 12.0
    rng = np.random.default_rng(5)
    P = []
    centers = synth.lattice_sites(4, 3.0)
    dirs = [np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0.6, 0.8, 0]),
            np.array([0.48, 0.6, 0.64])]
    k = 0
    for c in centers:
        d = dirs[k % len(dirs)]
        scale = rc * (1.0 + (k % 9 - 4) * 2.0 ** -52)
        a = c.copy()
        if k % 7 == 3:
            a[0] = 0.2 * rng.random()       # straddle the x seam: partner at negative x
            b = a - d * scale
        else:
            b = a + d * scale
        P += [a, b]
        k += 1
    P = np.array(P)
    n = P.shape[0]
    z = np.zeros(n)
    return synth.System(
        name="adv", x=P[:, 0].copy(), y=P[:, 1].copy(), z=P[:, 2].copy(), vx=z.copy(),
        vy=z.copy(), vz=z.copy(), elem=np.zeros(n, np.uint8), type=np.zeros(n, np.uint8),
        atom_id=np.arange(n, dtype=np.uint32), inv_mass=np.ones(n),
        q=np.ones(n, np.int8), sys_offsets=np.array([0, n], np.int64), periodic=True,
        box=np.array([[L, L, L]]), rc=rc, skin=0.1, dt=1e-4, n_steps=1,
        lambda_d=np.full((1, 2), 0.3), g=np.ones((1, 2)), base=np.zeros((1, 2)),
        qmax=np.array([1], np.int8), c6=np.zeros((1, 1)), c12=np.zeros((1, 1)),
        seeds=np.array([3], np.uint64))


@pytest.mark.parametrize("prec", PRECS)
def test_adversarial_cutoff_pairs(prec):
    s = _adversarial_system()
    op = oracle.pairs(s)
    assert 0 < op.shape[0] < s.n_atoms // 2      # some at-cutoff pairs are in, some out
    say("adversarial prec", prec)
    eng = make_engine(s, prec)
    eng.build()
    gp = sorted_pairs(eng.debug_pairs(prec=prec))
    assert np.array_equal(gp, op)
    eng.close()


# ------------------------------------------------------------------ ionization, integrator

def test_ionization_bit_exact_every_step():
    s = synth.water_small(n_steps=200)
    say("ionize water_small 200 steps")
    eng = make_engine(s, 1)
    q = s.q.copy()
    for step in range(1, 201):
        eng.set_step(step)
        eng.ionize()
        oracle.ionize(s, q, step)
        if step % 20 == 0 or step < 5:
            assert np.array_equal(eng.host("q"), q), step
    assert np.array_equal(eng.host("q"), q)
    assert q.sum() > 0
    eng.sync_check()
    eng.close()


def test_ionization_pulse_window_bit_exact():
    s = synth.water_pulse()
    s.base[:] = np.where(s.base > 0, 0.2, 0.0)      # large probabilities: many jumps
    say("ionize water_pulse window")
    eng = make_engine(s, 1)
    q = s.q.copy()
    for step in range(480, 521):
        eng.set_step(step)
        eng.ionize()
        oracle.ionize(s, q, step)
    assert np.array_equal(eng.host("q"), q)
    assert (q > 0).mean() > 0.5
    eng.close()


def test_integrator_bit_exact_given_forces():
    import torch
    s = synth.water_small()
    say("integrator bit-exact")
    eng = make_engine(s, 0)
    rng = np.random.default_rng(9)
    F = [rng.standard_normal(s.n_atoms) * 500.0 for _ in range(3)]
    for t, f in zip((eng.fx, eng.fy, eng.fz), F):
        t.copy_(torch.as_tensor(f))
    pos = [s.x.copy(), s.y.copy(), s.z.copy()]
    vel = [s.vx.copy(), s.vy.copy(), s.vz.copy()]
    eng.set_step(0)
    for rep in range(3):
        eng.vv(0)
        oracle.vv(0, s.dt, s.inv_mass, F, pos, vel)
        eng.vv(1, ekin=True)
        oracle.vv(1, s.dt, s.inv_mass, F, pos, vel)
    for name, ref in zip(("x", "y", "z", "vx", "vy", "vz"), (*pos, *vel)):
        assert np.array_equal(eng.host(name), ref), name
    assert eng.get_step() == 3
    ek = oracle.ekin(s, *vel)
    assert eng.host("ekin")[0] == pytest.approx(ek[0], rel=1e-13)
    eng.close()


# ------------------------------------------------------------------ full steps

def _run_engine(eng, n, build_mode):
    eng.set_step(0)
    eng.build()
    eng.forces(energy=True)
    qs, ep = [], []
    for _ in range(n):
        eng.step(build_mode=build_mode)
        qs.append(eng.host("q"))
        ep.append(eng.host("epot")[0])
    eng.sync_check()
    return qs, ep


@pytest.mark.parametrize("prec", PRECS)
def test_trajectory_against_oracle(prec):
    """20 full steps (ionize + forces + VV) of the small water box: charges bit-exact
    every step; positions within a bound set by the force tolerance."""
    s = synth.water_small(n_steps=20)
    s.base[:] = np.where(s.base > 0, 0.05, 0.0)
    say("trajectory prec", prec)
    eng = make_engine(s, prec)
    qs, ep = _run_engine(eng, 20, 0)
    ref = oracle.run(s, 20)
    for k in range(20):
        assert np.array_equal(qs[k], ref["q"][k + 1]), k
    tol = 1e-9 if prec == 0 else 2e-6
    for name in ("x", "y", "z"):
        assert np.max(np.abs(eng.host(name) - ref[name])) < tol, name
    eps = np.abs(np.array(ep) - np.array(ref["epot"][1:])[:, 0]).max()
    assert eps <= (1e-9 if prec == 0 else 1e-4) * np.abs(ref["epot"][-1][0]) + 1e-6
    eng.close()


# ------------------------------------------------------------------ full-size bench workload

@pytest.mark.parametrize("prec", PRECS)
def test_water_pulse_sampled_rows(prec):
    """98,304-atom pulse box in the benchmark's configuration: forces, and the number of
    partners of every sampled atom, against the oracle's full-j rows."""
    s = synth.water_pulse()
    s.q = random_charges(s, 3, hi=4)
    say("water_pulse sampled rows prec", prec)
    eng = make_engine(s, prec)
    set_q(eng, s.q)
    eng.set_step(700)
    eng.build()
    F, _ = gpu_forces(eng, prec)
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(s.n_atoms, 2000, replace=False))
    ref = oracle.forces_rows(s, rows, q=s.q, kappa=oracle_kappa(s, 700))
    Fg = tuple(f[rows] for f in F)
    assert force_error(Fg, ref) <= TOL[prec]
    pairs = eng.debug_pairs(prec=prec)
    cnt = np.bincount(pairs.reshape(-1), minlength=s.n_atoms)
    assert np.array_equal(cnt[rows], ref["row_hits"])
    eng.close()


# ------------------------------------------------------------------ batched vacuum clusters

@pytest.mark.parametrize("prec", PRECS)
def test_vacuum_batched_clusters(prec):
    s = synth.methane_clusters(n_clusters=5, lo=300, hi=4000, n_steps=10)
    s.q = random_charges(s, 4)
    k = 3
    say("methane batched prec", prec)
    eng = make_engine(s, prec, density_hint=100.0)
    set_q(eng, s.q)
    eng.set_step(k)
    eng.build()
    F, epot = gpu_forces(eng, prec)
    ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, k))
    assert force_error(F, ref) <= TOL[prec]
    for b in range(s.n_systems):
        a0, a1 = s.sys_offsets[b], s.sys_offsets[b + 1]
        assert abs(epot[b] - ref["epot"][b]) <= TOL[prec] * 2 * np.abs(ref["e_atom"][a0:a1]).sum()
    gp = sorted_pairs(eng.debug_pairs(prec=prec))
    assert np.array_equal(gp, oracle.pairs(s))
    eng.close()
    # every system alone gives the same pair set and forces within tolerance
    for b in (0, 3):
        a0, a1 = int(s.sys_offsets[b]), int(s.sys_offsets[b + 1])
        sb = s.subsystem(b)
        say("methane single system", b, "prec", prec)
        e1 = make_engine(sb, prec, density_hint=100.0)
        set_q(e1, sb.q)
        e1.set_step(k)
        e1.build()
        F1, _ = gpu_forces(e1, prec)
        for c in range(3):
            assert np.allclose(F1[c], F[c][a0:a1], rtol=0, atol=TOL[prec] * ref["a_atom"][a0:a1].max())
        p1 = sorted_pairs(e1.debug_pairs(prec=prec)) + a0
        sel = (gp[:, 0] >= a0) & (gp[:, 0] < a1)
        assert np.array_equal(p1, gp[sel])
        e1.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("G", [1, 2, 4, 8])
def test_every_cluster_group_and_skin(prec, G):
    """Every launch configuration the autotuner can choose (i-clusters per work-group,
    skin) gives the oracle's pair set and forces, periodic and batched vacuum.  The
    library halves a group whose candidate table would not fit one work-group's LDS
    (groups of 8 on the small water box): the size in use is at most the one asked."""
    cases = [(synth.water_small(n_steps=10), 5, {}),
             (synth.methane_clusters(n_clusters=4, lo=300, hi=3000, n_steps=10), 3,
              {"density_hint": 100.0})]
    for ci, (s, k, kw) in enumerate(cases):
        s.q = random_charges(s, 7 + ci)
        ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, k))
        op = oracle.pairs(s)
        for skin in (0.06, 0.12):
            say("cluster group", G, "skin", skin, "case", s.name, "prec", prec)
            eng = make_engine(s, prec, cluster_group=G, skin=skin, **kw)
            set_q(eng, s.q)
            eng.set_step(k)
            eng.build()
            F, epot = gpu_forces(eng, prec)
            assert force_error(F, ref) <= TOL[prec]
            for b in range(s.n_systems):
                a0, a1 = s.sys_offsets[b], s.sys_offsets[b + 1]
                esc = 2 * np.abs(ref["e_atom"][a0:a1]).sum()
                assert abs(epot[b] - ref["epot"][b]) <= TOL[prec] * esc
            assert np.array_equal(sorted_pairs(eng.debug_pairs(prec=prec)), op)
            st = eng.stats()
            assert st["cluster_group"] in (1, 2, 4, 8) and st["cluster_group"] <= G
            assert st["flags"] == 0
            eng.close()


# ------------------------------------------------------------------ graphs

def test_graph_replay_matches_eager():
    """Captured steps replayed several times, with eager work and synchronizations in
    between, reproduce the eager steps bit for bit (deterministic kernels)."""
    import torch
    s = synth.water_small(n_steps=12)
    s.base[:] = np.where(s.base > 0, 0.05, 0.0)
    say("graph vs eager")
    ea = make_engine(s, 1)
    eb = make_engine(s, 1)
    for e in (ea, eb):
        e.set_step(0)
        e.build()
        e.forces(energy=False)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        g_reb = eb.graph(1, stream)          # forced rebuild every step
        g_auto = eb.graph(0, stream)         # device-decided rebuild
    # capture does not execute anything; both engines start from the same state
    for step in range(12):
        reb = step % 4 == 3
        ea.step(build_mode=1 if reb else 0, energy=False, ekin=False)
        torch.cuda.synchronize()
        from paper_2401_03180_amd.md import md_graph_launch
        md_graph_launch(g_reb if reb else g_auto, stream)
        stream.synchronize()
        _ = eb.host("x")                       # eager work between replays
        for name in ("x", "vx", "q", "fx"):
            assert np.array_equal(ea.host(name), eb.host(name)), (step, name)
    assert ea.get_step() == eb.get_step() == 12
    ea.sync_check()
    eb.sync_check()
    ea.close()
    eb.close()


# ------------------------------------------------------------------ edge cases / errors

def _tiny_system(n, periodic=True, L=5.0, seed=0, nsys=1):
    """n atoms on randomly chosen sites of a jittered 0.4 nm lattice (no close contacts)."""
    rng = np.random.default_rng(seed)
    m = max(2, int(L / 0.4))
    sites = synth.lattice_sites(m, L / m)
    P = sites[rng.permutation(sites.shape[0])[:n]] + rng.uniform(-0.05, 0.05, size=(n, 3))
    z = np.zeros(n)
    offs = np.linspace(0, n, nsys + 1).astype(np.int64)
    atom_id = np.concatenate([np.arange(offs[b + 1] - offs[b]) for b in range(nsys)]).astype(np.uint32)
    return synth.System(
        name="tiny", x=P[:, 0].copy(), y=P[:, 1].copy(), z=P[:, 2].copy(), vx=z.copy(),
        vy=z.copy(), vz=z.copy(), elem=np.zeros(n, np.uint8), type=np.zeros(n, np.uint8),
        atom_id=atom_id, inv_mass=np.ones(n), q=rng.integers(0, 3, n).astype(np.int8),
        sys_offsets=offs, periodic=periodic,
        box=np.tile([[L, L, L]], (nsys, 1)) if periodic else None, rc=1.0, skin=0.1,
        dt=1e-4, n_steps=4, lambda_d=np.full((nsys, 5), 0.3), g=np.ones((nsys, 5)),
        base=np.full((1, 3), 0.5), qmax=np.array([2], np.int8), c6=np.full((1, 1), 1e-3),
        c12=np.full((1, 1), 1e-6), seeds=np.arange(1, nsys + 1, dtype=np.uint64))


@pytest.mark.parametrize("n,periodic,nsys", [(1, True, 1), (13, True, 1), (37, False, 1),
                                             (50, False, 3), (203, True, 2)])
def test_ragged_and_degenerate_sizes(n, periodic, nsys):
    s = _tiny_system(n, periodic, nsys=nsys)
    for prec in PRECS:
        say("ragged n", n, "periodic", periodic, "nsys", nsys, "prec", prec)
        eng = make_engine(s, prec)
        set_q(eng, s.q)
        eng.build()
        F, _ = gpu_forces(eng, prec)
        ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, 0))
        assert force_error(F, ref) <= TOL[prec]
        assert np.array_equal(sorted_pairs(eng.debug_pairs(prec=prec)), oracle.pairs(s))
        eng.close()


def test_empty_system_in_batch():
    s = _tiny_system(40, periodic=False, nsys=2)
    s.sys_offsets = np.array([0, 0, 40], np.int64)
    s.atom_id = np.arange(40, dtype=np.uint32)
    say("empty system in batch")
    eng = make_engine(s, 1)
    set_q(eng, s.q)
    eng.build()
    F, epot = gpu_forces(eng, 1)
    ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, 0))
    assert force_error(F, ref) <= 1e-5
    assert epot[0] == 0.0
    eng.close()


def _pile_system(n_pile, spacing, seed):
    """A tiny periodic system with `n_pile` atoms packed on a jittered cubic lattice of
    the given spacing around one point (far more atoms per grid bin than the grid is
    sized for); the background atoms near that point are dropped."""
    s = _tiny_system(64, True, L=5.0, seed=seed)
    c = np.array([1.2345, 3.1416, 2.7183])
    keep = np.linalg.norm(np.stack([s.x, s.y, s.z], 1) - c, axis=1) > 0.8
    m = int(math.ceil(n_pile ** (1.0 / 3.0)))
    rng = np.random.default_rng(seed + 1)
    P = (synth.lattice_sites(m, spacing)[:n_pile] - 0.5 * m * spacing + c +
         rng.uniform(-0.1 * spacing, 0.1 * spacing, size=(n_pile, 3)))
    B = np.stack([s.x, s.y, s.z], 1)[keep]
    X = np.concatenate([B, P])
    n = X.shape[0]
    q = np.concatenate([s.q[keep], rng.integers(0, 3, n_pile).astype(np.int8)])
    z = np.zeros(n)
    return synth.System(
        name="pile", x=X[:, 0].copy(), y=X[:, 1].copy(), z=X[:, 2].copy(), vx=z.copy(),
        vy=z.copy(), vz=z.copy(), elem=np.zeros(n, np.uint8), type=np.zeros(n, np.uint8),
        atom_id=np.arange(n, dtype=np.uint32), inv_mass=np.ones(n), q=q,
        sys_offsets=np.array([0, n], np.int64), periodic=True, box=s.box, rc=1.0, skin=0.1,
        dt=1e-4, n_steps=4, lambda_d=np.full((1, 5), 0.3), g=np.ones((1, 5)),
        base=np.full((1, 3), 0.5), qmax=np.array([2], np.int8), c6=np.full((1, 1), 1e-3),
        c12=np.full((1, 1), 1e-6), seeds=np.array([1], np.uint64))


def test_dense_bins_are_sorted_and_exact():
    """Grid bins holding over a hundred atoms (their slot order comes from the heap sort
    above 32 atoms per bin, from the work-group's rank sort above 128): the pair set is
    the oracle's in both precisions and the FP64 forces match it; two builds give
    bit-identical forces.  The grid is sized from the mean density (about a hundredth
    of the pile's), the per-atom list capacity is given for the pile."""
    from paper_2401_03180_amd import md
    s = _pile_system(216, 0.05, 3)
    ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, 0))
    op = oracle.pairs(s)
    for prec in PRECS:
        say("dense bins: 216 atoms at 0.05 nm spacing, prec", prec)
        eng = make_engine(s, prec, max_neighbors=512)
        set_q(eng, s.q)
        eng.build()
        assert np.array_equal(sorted_pairs(eng.debug_pairs(prec=prec)), op)
        F, _ = gpu_forces(eng, prec)
        if prec == 0:
            assert force_error(F, ref) <= TOL[0]
        eng.build(md.MD_BUILD_FORCE)
        F2, _ = gpu_forces(eng, prec)
        assert all(np.array_equal(a, b) for a, b in zip(F, F2))
        assert eng.sync_check(raise_on_flags=False) == 0
        eng.close()
    # 600 atoms 0.003 nm apart: one bin of 600, sorted by the whole work-group (FP64:
    # the LJ cores at that distance overflow FP32)
    s = _pile_system(600, 0.003, 5)
    ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, 0))
    say("dense bins: 600 atoms in one bin")
    eng = make_engine(s, 0, density_hint=2000.0)
    set_q(eng, s.q)
    eng.build()
    assert np.array_equal(sorted_pairs(eng.debug_pairs(prec=0)), oracle.pairs(s))
    F, _ = gpu_forces(eng, 0)
    assert force_error(F, ref) <= TOL[0]
    eng.build(md.MD_BUILD_FORCE)
    F2, _ = gpu_forces(eng, 0)
    assert all(np.array_equal(a, b) for a, b in zip(F, F2))
    assert eng.sync_check(raise_on_flags=False) == 0
    eng.close()


def test_box_too_small_is_geometry_error():
    from paper_2401_03180_amd.md import MDError, MD_ERR_GEOMETRY
    s = _tiny_system(20, True, L=2.1)
    with pytest.raises(MDError) as e:
        make_engine(s, 1)
    assert e.value.status == MD_ERR_GEOMETRY


def test_device_flags_are_reported():
    import torch
    from paper_2401_03180_amd import md
    s = _tiny_system(64, True)
    # no fast-atom capacity: one atom beyond skin/2 already makes a rebuild due
    eng = make_engine(s, 1, fast_capacity=-1)
    eng.build()
    # step counter beyond the bound tables
    say("flag: step")
    eng.set_step(s.n_steps + 3)
    eng.ionize()
    assert eng.sync_check(raise_on_flags=False) & md.MD_FLAG_STEP
    md.md_clear_flags(eng.ctx)
    assert eng.sync_check() == 0
    # displacement beyond skin/2 without a rebuild
    say("flag: skin")
    eng.set_step(0)
    eng.x.add_(0.2)
    eng.vv(0)                      # zero velocity, zero force: tracks the displacement
    eng.forces()
    assert eng.sync_check(raise_on_flags=False) & md.MD_FLAG_SKIN
    md.md_clear_flags(eng.ctx)
    eng.build()
    eng.forces()
    assert eng.sync_check() == 0
    # non-finite position
    say("flag: nonfinite")
    x = eng.x.clone()
    eng.x[5] = float("nan")
    eng.build()
    assert eng.sync_check(raise_on_flags=False) & md.MD_FLAG_NONFINITE
    eng.x.copy_(x)
    md.md_clear_flags(eng.ctx)
    # type outside the table
    say("flag: bad type")
    eng.type[3] = 7
    eng.build()
    assert eng.sync_check(raise_on_flags=False) & md.MD_FLAG_BAD_INPUT
    eng.close()
    # neighbour list too small: the per-atom lists are written by the first force
    # call after a rebuild, which reports the overflow
    for prec in (0, 1):
        say("flag: list overflow, precision %d" % prec)
        s2 = synth.water_small()
        e2 = make_engine(s2, prec, max_neighbors=16)
        e2.build()
        e2.forces()
        assert e2.sync_check(raise_on_flags=False) & md.MD_FLAG_LIST_OVERFLOW
        e2.close()


# ------------------------------------------------------------------ fast atoms

def _fast_case(periodic, n_fast, seed):
    """A system, per-atom displacements (most below skin/2 = 0.05 nm, `n_fast` of them
    beyond it, among them both atoms of some bonded pairs) and charges."""
    rng = np.random.default_rng(seed)
    if periodic:
        s = synth.water_small(n_steps=5)
    else:
        s = synth.methane_clusters(n_clusters=3, lo=300, hi=2000, n_steps=5)
    s.q = random_charges(s, seed)
    n = s.n_atoms
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    disp = u * rng.uniform(0.0, 0.045, n)[:, None]
    half = n_fast // 2
    lead = rng.choice(n - 1, half, replace=False)
    fast = np.unique(np.concatenate([lead, lead + 1]))[:n_fast]
    disp[fast] = u[fast] * rng.uniform(0.06, 0.3, fast.size)[:, None]
    return s, disp, fast


def _displace(eng, s, disp):
    """Move every atom by `disp` through phase 0 of velocity Verlet with zero force,
    which also flags the atoms beyond skin/2 of the build positions."""
    import torch
    for c, name in enumerate(("vx", "vy", "vz")):
        getattr(eng, name).copy_(torch.as_tensor(disp[:, c] / s.dt))
    for name in ("fx", "fy", "fz"):
        getattr(eng, name).zero_()
    eng.vv(0, ekin=False)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("n_fast,cap", [(24, 64), (24, 8192), (400, 1024), (400, 8192)])
def test_fast_atoms_exact_without_rebuild(prec, periodic, n_fast, cap):
    """Atoms beyond skin/2 of their build positions (no rebuild): the fast-atom
    kernels supply their pairs; pair set, forces and energies match the oracle at the
    new positions.  A capacity of 8,192 passes 16 work-groups per CU of the one-launch
    form, so the pass runs as two launches; 400 fast atoms within reach of one column
    of the small water box pass one LDS chunk of 256, so they are staged chunk by chunk."""
    from paper_2401_03180_amd import md
    s, disp, fast = _fast_case(periodic, n_fast, 21 + periodic)
    assert fast.size > 256 if n_fast > 256 else fast.size == n_fast
    say("fast atoms", "periodic" if periodic else "vacuum", "prec", prec, "n_fast", n_fast,
        "capacity", cap)
    eng = make_engine(s, prec, fast_capacity=cap, density_hint=0.0 if periodic else 100.0)
    set_q(eng, s.q)
    eng.set_step(0)
    eng.build()
    _displace(eng, s, disp)
    eng.build(md.MD_BUILD_AUTO)
    st = eng.stats()
    assert st["n_builds"] == 1 and st["n_fast"] == fast.size and st["n_fast_raw"] == fast.size
    F, epot = gpu_forces(eng, prec)
    x, y, z = eng.host("x"), eng.host("y"), eng.host("z")
    ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, 1), x=x, y=y, z=z)
    assert force_error(F, ref) <= TOL[prec]
    for b in range(s.n_systems):
        a0, a1 = s.sys_offsets[b], s.sys_offsets[b + 1]
        esc = 2 * np.abs(ref["e_atom"][a0:a1]).sum()
        assert abs(epot[b] - ref["epot"][b]) <= TOL[prec] * esc
    gp = sorted_pairs(eng.debug_pairs(prec=prec))
    assert np.array_equal(gp, oracle.pairs(s, x=x, y=y, z=z))
    assert eng.stats()["flags"] == 0
    eng.close()


def test_fast_capacity_overflow_rebuilds():
    """More fast atoms than the capacity: the device requests a rebuild, MD_BUILD_AUTO
    performs it, and the forces are exact again; MD_BUILD_CHECK instead latches
    MD_FLAG_SKIN."""
    from paper_2401_03180_amd import md
    s, disp, fast = _fast_case(True, 24, 5)
    for mode in (md.MD_BUILD_AUTO, md.MD_BUILD_CHECK):
        say("fast capacity overflow, build mode", mode)
        eng = make_engine(s, 1, fast_capacity=4)
        set_q(eng, s.q)
        eng.set_step(0)
        eng.build()
        _displace(eng, s, disp)
        st = eng.stats()
        assert st["n_fast_raw"] == fast.size and st["n_fast"] == 4
        eng.build(mode)
        eng.forces()
        flags = eng.sync_check(raise_on_flags=False)
        if mode == md.MD_BUILD_AUTO:
            assert flags == 0 and eng.stats()["n_builds"] == 2
            F = (eng.host("fx"), eng.host("fy"), eng.host("fz"))
            ref = oracle.forces(s, q=s.q, kappa=oracle_kappa(s, 1), x=eng.host("x"),
                                y=eng.host("y"), z=eng.host("z"))
            assert force_error(F, ref) <= TOL[1]
        else:
            assert flags & md.MD_FLAG_SKIN and eng.stats()["n_builds"] == 1
        eng.close()


# ------------------------------------------------------------------ full-size workloads

def _graph_steps_then_sample(s, prec, steps, n_rows, seed, **kw):
    """Run `steps` graph replays of the full step (automatic rebuilds, fast atoms),
    then compare the forces of `n_rows` sampled atoms with the oracle's all-pairs rows
    at the positions and charges the GPU reached."""
    import torch
    from paper_2401_03180_amd import md
    eng = make_engine(s, prec, **kw)
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
    F = (eng.host("fx"), eng.host("fy"), eng.host("fz"))
    x, y, z, q = eng.host("x"), eng.host("y"), eng.host("z"), eng.host("q")
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(s.n_atoms, n_rows, replace=False))
    ref = oracle.forces_rows(s, rows, q=q, x=x, y=y, z=z, kappa=oracle_kappa(s, steps))
    assert force_error(tuple(f[rows] for f in F), ref) <= TOL[prec]
    # kinetic energy per system of the last replay (summed inside the fused phase 1)
    ek = oracle.ekin(s, eng.host("vx"), eng.host("vy"), eng.host("vz"))
    assert np.allclose(eng.host("ekin"), ek, rtol=1e-12, atol=0.0)
    stats = eng.stats()
    eng.close()
    return stats


@pytest.mark.parametrize("prec", PRECS)
def test_protein_crystal_full_size_sampled(prec):
    """524,288-atom protein-crystal-like box (rc 1.2 nm, charges up to Z): sampled
    forces after graph-replayed steps."""
    s = synth.protein_crystal(n_steps=6)
    s.base[:] = np.where(s.base > 0, 0.05, 0.0)      # charges on many atoms within 6 steps
    say("protein_524288 sampled rows prec", prec)
    st = _graph_steps_then_sample(s, prec, 6, 300, 31)
    assert st["n_atoms"] == 524288


@pytest.mark.parametrize("prec", PRECS)
def test_methane_batched_full_size_sampled(prec):
    """256 vacuum methane clusters (1.73 M atoms) in one batched context: sampled forces
    after graph-replayed steps with per-cluster pulses."""
    s = synth.methane_clusters(n_steps=2000)
    s.base[:] = np.where(s.base > 0, 1.0, 0.0)
    say("methane_256 sampled rows prec", prec)
    st = _graph_steps_then_sample(s, prec, 700, 400, 41, density_hint=100.0)
    assert st["n_atoms"] == s.n_atoms


@pytest.mark.parametrize("prec", PRECS)
def test_water_large_full_size_sampled(prec):
    """4,194,304-atom water box: sampled forces after graph-replayed steps, in both
    precisions (the FP32-against-FP64 comparison of the benchmark runs on this machine)."""
    s = synth.water_large(n_steps=4)
    s.base[:] = np.where(s.base > 0, 0.05, 0.0)
    say("water_4194304 sampled rows prec", prec)
    st = _graph_steps_then_sample(s, prec, 4, 200, 51 + prec)
    assert st["n_atoms"] == 4194304


@pytest.mark.gpu
def test_graph_step_kinetic_energy_every_replay():
    """The fused step sums the kinetic energy inside phase 1 (per-block partials as atomic
    words, emptied after use): every replay's value equals the oracle's sum over the
    velocities it produced, on a single system and on a batch of systems."""
    import torch
    from paper_2401_03180_amd import md
    for s in (synth.water_small(), synth.methane_clusters(n_clusters=6, n_steps=40)):
        say("fused kinetic energy", s.n_systems, "systems")
        eng = make_engine(s, 1)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            eng.set_step(0, st)
            eng.build(md.MD_BUILD_FORCE, st)
            eng.forces(energy=True, stream=st)
            g = eng.graph(md.MD_BUILD_AUTO, st, energy=True, ekin=True)
            for rep in range(12):
                md.md_graph_launch(g, st)
                st.synchronize()
                ek = oracle.ekin(s, eng.host("vx"), eng.host("vy"), eng.host("vz"))
                assert np.allclose(eng.host("ekin"), ek, rtol=1e-12, atol=0.0), rep
        assert eng.sync_check(raise_on_flags=False) == 0
        eng.close()


def test_many_systems_energy_sums():
    """150 systems, more than the 64 work-groups that share a batch's per-system sums:
    after each graph replay every system's kinetic energy is the oracle's sum over the
    velocities reached; at the end the potential energies of the last replay equal an
    eager force call's at the same state bit for bit, and the oracle's within the force
    tolerance."""
    import torch
    from paper_2401_03180_amd import md
    s = synth.methane_clusters(n_clusters=150, lo=100, hi=400, n_steps=40)
    s.base[:] = np.where(s.base > 0, 0.05, 0.0)       # charged ions from the first steps
    s.g[:] = 1.0
    assert s.n_systems == 150
    say("energy sums of 150 systems")
    eng = make_engine(s, 1, density_hint=100.0)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        eng.set_step(0, st)
        eng.build(md.MD_BUILD_FORCE, st)
        eng.forces(energy=True, stream=st)
        g = eng.graph(md.MD_BUILD_AUTO, st, energy=True, ekin=True)
        for rep in range(8):
            md.md_graph_launch(g, st)
            st.synchronize()
            ek = oracle.ekin(s, eng.host("vx"), eng.host("vy"), eng.host("vz"))
            assert np.allclose(eng.host("ekin"), ek, rtol=1e-12, atol=0.0), rep
        ep_graph = eng.host("epot").copy()
        eng.forces(energy=True, stream=st)
        st.synchronize()
        assert np.array_equal(eng.host("epot"), ep_graph)
    q = eng.host("q")
    assert (q > 0).any()
    ref = oracle.forces(s, q=q, kappa=oracle_kappa(s, eng.get_step()), x=eng.host("x"),
                        y=eng.host("y"), z=eng.host("z"))
    for b in range(s.n_systems):
        a0, a1 = s.sys_offsets[b], s.sys_offsets[b + 1]
        esc = 2 * np.abs(ref["e_atom"][a0:a1]).sum()
        assert abs(ep_graph[b] - ref["epot"][b]) <= TOL[1] * esc, b
    assert eng.sync_check(raise_on_flags=False) == 0
    eng.close()


@pytest.mark.parametrize("prec", PRECS)
def test_water_large_groups_of_eight_no_overflow(prec):
    """4,194,304-atom water box with 8 i-clusters per group, skin 0.09 nm: a group of 8
    often spans two columns, and its candidate table must not fill its capacity over
    130 graph-replayed steps (it did, latching MD_FLAG_LIST_OVERFLOW, with the headroom
    of groups of 4); sampled forces against the oracle at the end.  In FP64 the table
    of a group of 8 exceeds one work-group's LDS, so this is also the FP64 kernel's
    path that reads the candidates from global memory."""
    s = synth.water_large(n_steps=130)
    say("water_4194304 G=8 skin 0.09 130 steps prec", prec)
    st = _graph_steps_then_sample(s, prec, 130, 100, 61 + prec, cluster_group=8, skin=0.09,
                                  fast_capacity=1024)
    assert st["cluster_group"] == 8
    assert st["max_group_entries"] < st["group_entry_capacity"]
