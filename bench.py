"""Benchmark: atom-steps/s of the full screened-force + ionization step on one MI355X.

One step = device-side rebuild check / neighbour rebuild when due, stochastic
ionization, screened FP32 pair forces with compensated sums and the FP64 energy,
and the FP64 velocity-Verlet half steps with the kinetic-energy reduction.  Every
step is one replay of a captured HIP graph; inputs are resident in HBM before the
timed region.  Default workload: the 4,194,304-atom bulk-water box (1,398,101 H2O
plus one O in a 34.8 nm periodic cube, lambda_D 0.2 nm, rc 1.0 nm, per-step
ionization probability 1e-3), synthetic and seeded.  The schedule starts at step 0
(neutral atoms, one build); the timed steps follow the warm-up steps with no extra
build, so rebuilds fall where the workload puts them.

Beside the timed FP32 line it reports, on the same GPU: the plain FP64 force path
(FP32-vs-FP64 speedup); the force and per-atom energy error of both paths against
the FP64 oracle on the 65,536-atom sub-box of the 4.19 M-atom box; the whole
schedule (initial build included) in ms per step with its rebuild count; the
98,304-atom pulse box over its 1,000-step schedule; the 256 batched methane
clusters against the plain FP64 form with one system per launch, and over their
whole 2,000-step schedule; and the oracle timed on the host cores.

Prints ONE JSON line (rank 0, N = 1).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector (256 CU x 2.4 GHz x 256 FLOP/clk)
PEAK_FP32_NONPACKED_TFLOPS = 78.6
FLOP_PER_PAIR = 44                # forces 42 + energy 2, per pair inside the cutoff
FLOP_PER_PAIR_HYBRID = 57         # hybrid screening (Debye branch on both ions): 55 + 2
FLOP_QLJ_EXTRA = 10               # charge-scaled LJ radius: c_j 2, s 2, s^6 3, c6/c12 3
METRIC = "atom-steps/s for screened-force+ionize step; % FP32 VALU peak; FP32-vs-FP64 speedup"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


SCHEDULE = {"water_1536": 200, "water_98304": 1000, "protein_524288": 500,
            "methane_256": 2000, "water_4194304": 100}


def schedule_len(name, dt_fs=None):
    """Steps of the named workload's schedule (the pulse box at another time step: the
    same schedule in time)."""
    if dt_fs is None:
        return SCHEDULE[name]
    return int(round(SCHEDULE[name] * 0.1 / dt_fs))


def make_system(name, n_steps, dt_fs=None):
    """The named workload with its own schedule length, or n_steps if longer; dt_fs:
    the pulse box (water_98304) at another time step."""
    from paper_2401_03180_amd import synth
    if name not in SCHEDULE:
        raise SystemExit("unknown config " + name)
    if dt_fs is not None and name != "water_98304":
        raise SystemExit("--dt-fs applies to water_98304 only")
    S = max(int(n_steps), schedule_len(name, dt_fs))
    if name == "water_98304":
        return synth.water_pulse(n_steps=S, dt_fs=0.1 if dt_fs is None else dt_fs)
    if name == "water_1536":
        return synth.water_small(n_steps=S)
    if name == "protein_524288":
        return synth.protein_crystal(n_steps=S)
    if name == "water_4194304":
        return synth.water_large(n_steps=S)
    return synth.methane_clusters(n_steps=S)


STATE = ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "q")


def run_gpu(sys_, prec, steps, warmup, cluster_group, skin, pair_samples=5, use_graph=True,
            fast_capacity=0, langevin=None, hybrid=None, ff=None, schedule_steps=0,
            subbox=None, preroll_max=0):
    """The workload's schedule from step 0 (initial build and forces), up to its
    first automatic list rebuild when preroll_max > 0 (at most that many steps: the
    start from a lattice needs none for tens of steps, so a short window right after
    step 0 would hold none of the rebuilds of the rest of the schedule), `warmup`
    steps, then `steps` timed steps: replays of the captured step graph (or, with
    use_graph False, eager md_step calls), inputs resident, no build forced in
    between.  Then the same run is repeated from the initial state with the timed
    steps launched eagerly and the force-kernel timer on: the trajectory is
    deterministic, so the repetition launches exactly the kernels of the timed
    region (checked: identical final state and rebuild count) and gives the
    duration of every force-kernel launch.  A third run samples the pair counts
    between its steps (checked: identical final state).  schedule_steps > 0: the whole schedule (initial build,
    forces and that many graph steps) is timed once more from the initial state.
    subbox: the oracle rows of the error report (see subbox_errors), evaluated at
    the final state after a build at its positions.  langevin: (gamma, kt) tables
    of the electron-ion coupling, bound for the whole run, or None; hybrid: the
    free-electron density table of hybrid screening, or None; ff: md_bind_forcefield
    keyword arrays, or None."""
    import torch
    from paper_2401_03180_amd import md
    eng = md.Engine(sys_, prec, cluster_group=cluster_group, skin=skin,
                    fast_capacity=fast_capacity)
    if langevin is not None:
        eng.bind_langevin(*langevin)
    if hybrid is not None:
        eng.bind_hybrid(hybrid)
    if ff is not None:
        eng.bind_forcefield(**ff)
    out = {}
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        init = {n: getattr(eng, n).clone() for n in STATE}

        def restart():
            for n in STATE:
                getattr(eng, n).copy_(init[n])
            eng.set_step(0, stream)
            eng.build(md.MD_BUILD_FORCE, stream)
            eng.forces(energy=True, stream=stream)

        restart()
        if use_graph:
            graph = eng.graph(md.MD_BUILD_AUTO, stream, energy=True, ekin=True)
            one_step = lambda: md.md_graph_launch(graph, stream)
        else:
            one_step = lambda: eng.step(md.MD_BUILD_AUTO, energy=True, ekin=True, stream=stream)
        n_pre = 0
        if preroll_max > 0:
            b0 = eng.stats(stream)["n_builds"]
            while n_pre < preroll_max:
                one_step()
                n_pre += 1
                stream.synchronize()
                if eng.stats(stream)["n_builds"] > b0:
                    break
        for _ in range(warmup):
            one_step()
        stream.synchronize()
        st0 = eng.stats(stream)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            one_step()
        ev1.record(stream)
        stream.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        flags = eng.sync_check(stream, raise_on_flags=False)
        st1 = eng.stats(stream)
        final = {n: getattr(eng, n).clone() for n in STATE}
        step_end = eng.get_step(stream)

        # the same run again, the timed steps eager with the force-kernel timer
        restart()
        for _ in range(n_pre + warmup):
            one_step()
        stream.synchronize()
        st2 = eng.stats(stream)
        eng.timer_start(steps)
        for i in range(1, steps + 1):
            eng.step(md.MD_BUILD_AUTO, energy=True, ekin=True, stream=stream)
        durations = eng.timer_read()
        stream.synchronize()
        st3 = eng.stats(stream)
        same = all(torch.equal(getattr(eng, n), final[n]) for n in STATE)
        eng.timer_start(0)

        # and once more, the pair counts sampled between the steps (a count-only
        # export takes longer than a step: kept out of both timed runs)
        restart()
        for _ in range(n_pre + warmup):
            one_step()
        sample_at = set(int(v) for v in np.linspace(1, steps, pair_samples))
        pairs = []
        for i in range(1, steps + 1):
            one_step()
            if i in sample_at:
                stream.synchronize()
                pairs.append(eng.count_pairs(prec=prec, stream=stream))
        stream.synchronize()
        same = same and all(torch.equal(getattr(eng, n), final[n]) for n in STATE)

        if schedule_steps > 0:
            # the whole schedule, initial build and forces included (rebuilds: the
            # automatic ones during its steps)
            torch.cuda.synchronize()
            b0 = eng.stats(stream)["n_builds"] + 1
            for n in STATE:
                getattr(eng, n).copy_(init[n])
            stream.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            eng.set_step(0, stream)
            eng.build(md.MD_BUILD_FORCE, stream)
            eng.forces(energy=True, stream=stream)
            for _ in range(schedule_steps):
                one_step()
            e1.record(stream)
            stream.synchronize()
            st4 = eng.stats(stream)
            out.update(schedule_steps=schedule_steps,
                       schedule_ms_per_step=e0.elapsed_time(e1) / schedule_steps,
                       schedule_rebuilds=int(st4["n_builds"] - b0),
                       schedule_flags=eng.sync_check(stream, raise_on_flags=False))
        if subbox is not None:
            out["subbox"] = subbox_errors(eng, subbox, stream)
    eng.close()
    builds = st1["n_builds"] - st0["n_builds"]
    builds_replay = st3["n_builds"] - st2["n_builds"]
    d = np.asarray(durations, dtype=np.float64)
    out.update({"ms": ms, "wall_s": wall, "flags": flags, "pairs": float(np.mean(pairs)),
                "pairs_min": int(min(pairs)), "pairs_max": int(max(pairs)),
                "kernel_ms": float(d.mean()), "kernel_ms_median": float(np.median(d)),
                "kernel_ms_p90": float(np.percentile(d, 90)), "kernel_launches": int(d.size),
                "builds": builds, "builds_replay": builds_replay, "preroll_steps": n_pre,
                "replay_identical": bool(same and builds == builds_replay), "stats": st1,
                "step": step_end, "charged_fraction": float((final["q"] > 0).float().mean())})
    return out


def subbox_rows(sys_, n_rows=65536, threads=16):
    """The error-report sub-box: the n_rows atoms nearest, in the max norm under the
    minimum image, to the centre of the [0, L/4)^3 corner sub-cube (ties by index),
    the candidate partners (every atom within that radius plus rc of the centre: a
    superset of the rows' partners, so restricting the oracle's all-j loop to them
    leaves its sums unchanged) and the oracle threads."""
    L = sys_.box[0]
    c = L / 8.0
    P = sys_.positions()
    d = P - c
    d -= L * np.rint(d / L)
    dist = np.abs(d).max(axis=1)
    order = np.lexsort((np.arange(dist.size), dist))
    rows = np.sort(order[:n_rows])
    reach = dist[order[n_rows - 1]] + sys_.rc + 1e-6
    cand = np.flatnonzero(dist <= reach)
    return {"rows": rows, "cand": cand, "threads": threads}


def subbox_errors(eng, sb, stream):
    """Force and per-atom energy error of the FP32 and FP64 paths against the oracle
    on the sub-box rows, at the engine's current positions and charges after a build
    there (identical input snapshot for both paths)."""
    import oracle
    from paper_2401_03180_amd import md
    s = eng.sys
    eng.build(md.MD_BUILD_FORCE, stream)
    x, y, z, q = eng.host("x"), eng.host("y"), eng.host("z"), eng.host("q")
    step = eng.get_step(stream)
    got = {}
    for prec in (md.MD_FP32_KAHAN, md.MD_FP64):
        eng.forces(prec=prec, energy=True, stream=stream)
        F = (eng.host("fx"), eng.host("fy"), eng.host("fz"))
        e, _ = eng.atom_energies(prec=prec, stream=stream)
        got[prec] = (F, e)
    rows, cand = sb["rows"], sb["cand"]
    sub = s.copy()
    for n, v in (("x", x), ("y", y), ("z", z), ("q", q)):
        setattr(sub, n, v[cand].copy())
    for n in ("vx", "vy", "vz", "elem", "type", "inv_mass"):
        setattr(sub, n, getattr(s, n)[cand].copy())
    sub.atom_id = np.arange(cand.size, dtype=np.uint32)
    sub.sys_offsets = np.array([0, cand.size], np.int64)
    local = np.searchsorted(cand, rows)
    t = time.perf_counter()
    kap = oracle.kappa_from_lambda(s.lambda_d[:, step])
    ref = oracle.forces_rows(sub, local, kappa=kap, n_threads=sb["threads"])
    t_orc = time.perf_counter() - t
    A = ref["a_atom"]
    out = {"rows": int(rows.size), "candidates": int(cand.size), "step": int(step),
           "charged_fraction": float((q[rows] > 0).mean()), "oracle_s": t_orc,
           "pairs_per_row": float(np.mean(ref["row_hits"]))}
    for prec, name in ((md.MD_FP32_KAHAN, "fp32"), (md.MD_FP64, "fp64")):
        F, e = got[prec]
        dF = np.sqrt(sum((f[rows] - ref[k]) ** 2 for f, k in zip(F, ("fx", "fy", "fz"))))
        live = A > 0
        eF = float(np.max(dF[live] / A[live])) if live.any() else 0.0
        Fm = np.sqrt(ref["fx"] ** 2 + ref["fy"] ** 2 + ref["fz"] ** 2)
        big = Fm >= 0.1 * np.sqrt(np.mean(Fm ** 2))
        de = e[rows] - ref["e_atom"]
        out[name] = {"e_F": eF,
                     "rel_force_max_strong": float(np.max(dF[big] / Fm[big])),
                     "rel_force_p99_strong": float(np.percentile(dF[big] / Fm[big], 99)),
                     "rel_force_global": float(np.sqrt(np.sum(dF ** 2) / np.sum(Fm ** 2))),
                     "energy_rel": float(abs(de.sum()) / np.abs(ref["e_atom"]).sum()),
                     "atom_energy_max_rel": float(np.max(np.abs(de) /
                                                         (np.abs(ref["e_atom"]) + A + 1e-300)))}
    return out


def run_gpu_per_system(sys_, prec, steps, warmup, langevin=None, hybrid=None, ff_kind=None):
    """The plain form for batched workloads: every system in a context of its own,
    its step replayed as its own graph, systems one after another on one stream."""
    import torch
    from paper_2401_03180_amd import md
    engines, graphs = [], []
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for b in range(sys_.n_systems):
            sb = sys_.subsystem(b)
            e = md.Engine(sb, prec)
            if langevin is not None:
                e.bind_langevin(langevin[0][b:b + 1], langevin[1][b:b + 1])
            if hybrid is not None:
                e.bind_hybrid(hybrid[b:b + 1])
            if ff_kind is not None:
                e.bind_forcefield(**ff_binding(sb, ff_kind))
            e.set_step(0, stream)
            e.build(md.MD_BUILD_FORCE, stream)
            e.forces(energy=True, stream=stream)
            engines.append(e)
            graphs.append(e.graph(md.MD_BUILD_AUTO, stream, energy=True, ekin=True))
        for _ in range(warmup):
            for g in graphs:
                md.md_graph_launch(g, stream)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            for g in graphs:
                md.md_graph_launch(g, stream)
        ev1.record(stream)
        stream.synchronize()
        ms = ev0.elapsed_time(ev1)
        flags = 0
        for e in engines:
            flags |= e.sync_check(stream, raise_on_flags=False)
    for e in engines:
        e.close()
    return {"ms": ms, "flags": flags}


def ff_binding(sys_, kind):
    """Synthetic molecular force field of the workload: full LJ tables into sys_ and
    the md_bind_forcefield keyword arrays."""
    from paper_2401_03180_amd import synth
    d = synth.molecular_force_field(sys_, kind)
    sys_.c6, sys_.c12 = d["c6"], d["c12"]
    return {"z_type": d["z"], "sigma_type": d["sigma"], "excl": d["excl"], "bonds": d["bonds"],
            "bond_par": d["bond_par"], "angles": d["angles"], "angle_par": d["angle_par"]}


def run_rdf(sys_, r_max=1.0, n_bins=250, calls=20, warmup=3, steps=50):
    """Pair-distance histogram of the workload after `steps` graph-replayed steps
    (moved atoms included), timed with HIP events over `calls` calls on one stream;
    returns ms per call and the pairs counted per call."""
    import torch
    from paper_2401_03180_amd import md
    eng = md.Engine(sys_, md.MD_FP32_KAHAN)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eng.set_step(0, stream)
        eng.build(md.MD_BUILD_FORCE, stream)
        eng.forces(energy=True, stream=stream)
        g = eng.graph(md.MD_BUILD_AUTO, stream, energy=True, ekin=True)
        for _ in range(steps):
            md.md_graph_launch(g, stream)
        E = sys_.n_elements
        h = torch.zeros((sys_.n_systems, E, E, n_bins), dtype=torch.int64, device="cuda")
        for _ in range(warmup):
            eng.rdf(r_max, n_bins, hist=h, stream=stream)
        h.zero_()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(calls):
            eng.rdf(r_max, n_bins, hist=h, stream=stream)
        ev1.record(stream)
        stream.synchronize()
        flags = eng.sync_check(stream, raise_on_flags=False)
    eng.close()
    ms = ev0.elapsed_time(ev1) / calls
    pairs = int(h.sum().item()) // calls
    return {"rdf_ms_per_call": ms, "rdf_pairs_per_call": pairs,
            "rdf_pairs_per_s": pairs / (ms * 1e-3), "rdf_r_max": r_max, "rdf_bins": n_bins,
            "rdf_flags": flags}


def cpu_baseline(sys_, target_s=12.0, threads=None, langevin=None, hybrid=None, ff=None):
    """The oracle, as it stands: whole steps (all-pairs FP64 force rows of every atom,
    ionization and both velocity-Verlet half steps, phase 0 with the electron-ion
    coupling when langevin = (gamma, kt) is given, hybrid screening when the density
    table hybrid is given, the force-field terms of the oracle ForceField ff)
    repeated until about target_s
    seconds of work; when one step alone would exceed that, the force rows of a random
    subset of atoms are timed and scaled to all atoms."""
    import oracle
    if langevin is not None:
        c1 = oracle.langevin_c1(langevin[0], sys_.dt)

    def htab(s):
        if hybrid is None:
            return None
        return oracle.hybrid_table(sys_.lambda_d[:, s], hybrid[:, s], sys_.base.shape[1])

    def phase0(s, F, pos, vel):
        if langevin is None:
            oracle.vv(0, sys_.dt, sys_.inv_mass, F, pos, vel)
        else:
            oracle.vv_langevin(sys_, s, c1, langevin[1], F, pos, vel)

    n_host, n_aff = host_cores()
    # one GPU's share of the machine's host cores is 16, whatever the host has in all
    threads = threads or min(n_aff, 16)
    cores_note = ("%d threads: the %d-core share of one GPU (host: %d logical CPUs, %d in "
                  "this process's affinity mask)" % (threads, 16, n_host, n_aff)
                  if threads < n_aff else "%d threads on all %d logical CPUs of the affinity "
                  "mask (host: %d)" % (threads, n_aff, n_host))
    n = sys_.n_atoms
    rng = np.random.default_rng(0)
    kap = oracle.kappa_from_lambda(sys_.lambda_d[:, 1])
    probe = np.sort(rng.choice(n, min(n, 256), replace=False))
    t = time.perf_counter()
    oracle.forces_rows(sys_, probe, kappa=kap, n_threads=threads, hybrid=htab(1), ff=ff)
    per_row = (time.perf_counter() - t) / probe.size
    q = sys_.q.copy()
    pos = [sys_.x.copy(), sys_.y.copy(), sys_.z.copy()]
    vel = [sys_.vx.copy(), sys_.vy.copy(), sys_.vz.copy()]
    F = (np.zeros(n), np.zeros(n), np.zeros(n))
    if per_row * n <= target_s:
        rows = np.arange(n)
        t = time.perf_counter()
        steps = 0
        while time.perf_counter() - t < target_s and steps < sys_.n_steps:
            steps += 1
            s = steps
            phase0(s, F, pos, vel)
            oracle.ionize(sys_, q, s)
            out = oracle.forces_rows(sys_, rows, q=q, x=pos[0], y=pos[1], z=pos[2],
                                     kappa=oracle.kappa_from_lambda(sys_.lambda_d[:, s]),
                                     n_threads=threads, hybrid=htab(s), ff=ff)
            F = (out["fx"], out["fy"], out["fz"])
            if ff is not None:
                bo = oracle.bonded(sys_, ff, q=q, x=pos[0], y=pos[1], z=pos[2])
                F = tuple(f + bo[c] for f, c in zip(F, ("fx", "fy", "fz")))
            oracle.vv(1, sys_.dt, sys_.inv_mass, F, pos, vel)
        t_all = time.perf_counter() - t
        return {"value": n * steps / t_all, "unit": "atom-steps/s", "cores": threads,
                "cores_note": cores_note, "kind": "oracle",
                "sample": "O(N^2) FP64 oracle, %d whole steps of all %d atoms (all-pairs force "
                          "rows, ionize, velocity Verlet) in %.1f s" % (steps, n, t_all)}
    rows_n = int(min(n, max(256, target_s / max(per_row, 1e-9))))
    rows = np.sort(rng.choice(n, rows_n, replace=False))
    t = time.perf_counter()
    oracle.forces_rows(sys_, rows, kappa=kap, n_threads=threads, hybrid=htab(1), ff=ff)
    t_rows = time.perf_counter() - t
    t = time.perf_counter()
    phase0(1, F, pos, vel)
    oracle.ionize(sys_, q, 1)
    if ff is not None:
        oracle.bonded(sys_, ff, q=q, x=pos[0], y=pos[1], z=pos[2])
    oracle.vv(1, sys_.dt, sys_.inv_mass, F, pos, vel)
    t_elem = time.perf_counter() - t
    t_step = t_rows * n / rows_n + t_elem
    return {"value": n / t_step, "unit": "atom-steps/s", "cores": threads,
            "cores_note": cores_note, "kind": "oracle",
            "sample": "O(N^2) FP64 oracle: all-pairs force rows of %d of %d atoms (%.1f s) plus "
                      "ionize and velocity Verlet over all atoms, scaled to one whole step "
                      "(%.1f s)" % (rows_n, n, t_rows, t_step)}


def kernel_source_sha1():
    d = os.path.join(ROOT, "paper_2401_03180_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read() for f in ("md_force.hip", "md_internal.h"))
    return hashlib.sha1(src).hexdigest()


def profile_values(config):
    """The key: value lines of the committed rocprofv3 counter summary of the FP32 force
    kernel on the workload, if it was taken on the current force-kernel source; else
    an empty dict."""
    path = os.path.join(ROOT, "profiles", "force32_%s_counters.txt" % config)
    if not os.path.exists(path):
        return {}
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "|", "#")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha1") != kernel_source_sha1():
        return {}
    return kv


def traffic_from_profile(config):
    """HBM bytes per force launch from the committed counter summary, or None."""
    kv = profile_values(config)
    return float(kv["hbm_bytes_per_launch"]) if "hbm_bytes_per_launch" in kv else None


def run_schedule(sys_, prec, knobs, steps=None):
    """The workload's whole schedule (initial build and forces, then every step as a
    graph replay), timed with HIP events: ms per step, automatic rebuilds, flags."""
    import torch
    from paper_2401_03180_amd import md
    steps = sys_.n_steps if steps is None else steps
    eng = md.Engine(sys_, prec, cluster_group=knobs["cluster_group"], skin=knobs["skin"],
                    fast_capacity=knobs["fast_capacity"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        init = {n: getattr(eng, n).clone() for n in STATE}
        eng.set_step(0, stream)
        eng.build(md.MD_BUILD_FORCE, stream)       # a capture needs a built context
        g = eng.graph(md.MD_BUILD_AUTO, stream, energy=True, ekin=True)
        for n in STATE:
            getattr(eng, n).copy_(init[n])
        torch.cuda.synchronize()
        b0 = eng.stats(stream)["n_builds"] + 1     # + the forced build below
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        eng.set_step(0, stream)
        eng.build(md.MD_BUILD_FORCE, stream)
        eng.forces(energy=True, stream=stream)
        for _ in range(steps):
            md.md_graph_launch(g, stream)
        e1.record(stream)
        stream.synchronize()
        st = eng.stats(stream)
        flags = eng.sync_check(stream, raise_on_flags=False)
        charged = float((eng.host("q") > 0).mean())
    eng.close()
    ms = e0.elapsed_time(e1) / steps
    return {"steps": steps, "ms_per_step": ms, "value": sys_.n_atoms / (ms * 1e-3),
            "rebuilds": int(st["n_builds"] - b0), "flags": flags, "charged_fraction": charged}


def host_cores():
    n = os.cpu_count() or 1
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = n
    return n, aff


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="water_4194304")
    ap.add_argument("--cluster-group", type=int, default=0)
    ap.add_argument("--skin", type=float, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the other workloads (98,304-atom schedule, batched clusters)")
    ap.add_argument("--no-subbox", action="store_true",
                    help="skip the oracle error report on the 65,536-atom sub-box")
    ap.add_argument("--no-schedule", action="store_true",
                    help="skip the timing of the whole schedule (initial build included)")
    ap.add_argument("--fast-capacity", type=int, default=None)
    ap.add_argument("--tune", action="store_true",
                    help="search cluster group, skin and fast-atom capacity first and cache "
                         "the best (paper_2401_03180_amd/tuned.json)")
    ap.add_argument("--no-tuned", action="store_true", help="ignore the cached configuration")
    ap.add_argument("--eager", action="store_true",
                    help="launch the step kernels one by one instead of replaying a graph")
    ap.add_argument("--langevin", action="store_true",
                    help="bind the electron-ion coupling (synthetic gamma per element and "
                         "electron-temperature schedule) for every run")
    ap.add_argument("--hybrid", action="store_true",
                    help="bind hybrid ion-sphere / Debye screening (synthetic electron "
                         "density consistent with the Debye-length schedule)")
    ap.add_argument("--forcefield", action="store_true",
                    help="bind the synthetic molecular force field (Morse bonds, angles, "
                         "LJ exclusions, charge-scaled LJ radii, LJ on every element pair)")
    ap.add_argument("--dt-fs", type=float, default=None,
                    help="water_98304 only: another time step in fs with the same pulse and "
                         "screening schedule in time (the force-field run needs 0.05 fs)")
    ap.add_argument("--rdf", action="store_true",
                    help="also time the pair-distance histogram (1 nm, 250 bins) after the "
                         "timed steps' workload")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: run it with --gpus 1 (multi-GPU sharding is "
              "a design note, not built)", file=sys.stderr)
        raise SystemExit(2)

    import torch
    from paper_2401_03180_amd import md
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    md.lib()

    if a.calib_copy:
        # streaming kernel of known traffic (reads 1 GiB, writes 1 GiB): the scale
        # of the HBM byte counters
        src = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    PREROLL = 64          # most steps run before the timed window (to the first rebuild)
    S = a.warmup + a.steps + PREROLL
    from paper_2401_03180_amd import autotune

    def knobs(config, prec, steps=a.steps, warmup=a.warmup, cli=True):
        """Launch configuration: command line, else the cached tuning, else defaults."""
        if a.tune and cli:
            autotune.tune(config, lambda: make_system(config, S, a.dt_fs), prec, steps, warmup,
                          log=log)
        t = None if a.no_tuned else autotune.load(config, prec)
        k = {"cluster_group": 0, "skin": None, "fast_capacity": 0, "tuned": t is not None}
        if t is not None:
            k.update(cluster_group=t["cluster_group"], skin=t["skin"],
                     fast_capacity=t["fast_capacity"])
        if cli and a.cluster_group:
            k["cluster_group"] = a.cluster_group
        if cli and a.skin is not None:
            k["skin"] = a.skin
        if cli and a.fast_capacity is not None:
            k["fast_capacity"] = a.fast_capacity
        return k

    t_gen = time.perf_counter()
    base_sys = make_system(a.config, S, a.dt_fs)
    log("generated", a.config, "in %.1f s" % (time.perf_counter() - t_gen))
    sys32 = base_sys.copy()
    ff_kind = ("methane" if a.config.startswith("methane") else "water") if a.forcefield else None
    ff_runaway = bool(ff_kind) and a.config == "water_98304" and sys32.dt > 0.75e-4
    if ff_runaway:
        log("warning: with the molecular force field the pulse box's dynamics run away after "
            "the pulse at dt 0.1 fs (fast ions reach the small charge-scaled LJ cores within "
            "one step); --dt-fs 0.05 keeps them finite.  The FP64 leg is skipped at this step: "
            "one such run of it stalled past the divergence, cause not established")
    ffb = ff_binding(sys32, ff_kind) if ff_kind else None
    lg = None
    if a.langevin:
        from paper_2401_03180_amd import synth
        lg = synth.langevin_inputs(sys32)
    hy = None
    if a.hybrid:
        from paper_2401_03180_amd import synth
        hy = synth.hybrid_inputs(sys32)
    plain = ffb is None and lg is None and hy is None
    sb = None
    if a.config == "water_4194304" and plain and not a.no_subbox:
        sb = subbox_rows(sys32)
    k32 = knobs(a.config, md.MD_FP32_KAHAN)
    log("config", a.config, "atoms", sys32.n_atoms, "steps", a.steps, "warmup", a.warmup, k32)
    sched = min(sys32.n_steps, schedule_len(a.config, a.dt_fs)) if not a.no_schedule else 0
    r32 = run_gpu(sys32, md.MD_FP32_KAHAN, a.steps, a.warmup, k32["cluster_group"], k32["skin"],
                  use_graph=not a.eager, fast_capacity=k32["fast_capacity"], langevin=lg,
                  hybrid=hy, ff=ffb, schedule_steps=sched, subbox=sb, preroll_max=PREROLL)
    log("fp32", {k: v for k, v in r32.items() if k != "stats"})
    n = sys32.n_atoms
    value = n * a.steps / (r32["ms"] * 1e-3)
    st = r32["stats"]
    extra = {"flags": r32["flags"], "rebuilds_timed": r32["builds"],
             "preroll_steps": r32["preroll_steps"],
             "replay_identical": r32["replay_identical"],
             "charged_fraction_end": r32["charged_fraction"],
             "pairs_in_cutoff_mean": r32["pairs"], "pairs_min": r32["pairs_min"],
             "pairs_max": r32["pairs_max"], "force_launches_timed": r32["kernel_launches"],
             "force_kernel_ms_median": r32["kernel_ms_median"],
             "force_kernel_ms_p90": r32["kernel_ms_p90"],
             "list_codes": st["n_list_codes"],
             "codes_per_pair": st["n_list_codes"] / max(r32["pairs"], 1.0),
             # in-cutoff pair visits (each pair from both atoms) per list code slot
             "pair_efficiency": 2.0 * r32["pairs"] / max(st["n_list_codes"], 1),
             "groups": st["n_groups"], "cluster_group": st["cluster_group"],
             "max_group_entries": st["max_group_entries"],
             "group_entry_capacity": st["group_entry_capacity"],
             "max_list_len": st["max_list_len"], "list_capacity": st["list_capacity"]}
    if "schedule_ms_per_step" in r32:
        extra.update(schedule_steps=r32["schedule_steps"],
                     schedule_ms_per_step=r32["schedule_ms_per_step"],
                     schedule_value=n / (r32["schedule_ms_per_step"] * 1e-3),
                     schedule_rebuilds=r32["schedule_rebuilds"],
                     schedule_flags=r32["schedule_flags"])
    if "subbox" in r32:
        extra["subbox_errors"] = r32["subbox"]
        log("subbox", r32["subbox"])
    if not a.no_fp64 and not ff_runaway:
        if sys32.n_systems > 1:
            # batched workloads: the plain FP64 form runs one system per context and launch
            sys64 = base_sys.copy()
            ffb64 = ff_binding(sys64, ff_kind) if ff_kind else None
            r64 = run_gpu_per_system(sys64, md.MD_FP64, a.steps, a.warmup, langevin=lg, hybrid=hy,
                                     ff_kind=ff_kind)
            v64 = n * a.steps / (r64["ms"] * 1e-3)
            extra.update({"fp64_per_system_value": v64,
                          "fp64_per_system_ms_per_step": r64["ms"] / a.steps,
                          "batched_fp32_vs_per_system_fp64_speedup": value / v64,
                          "fp64_flags": r64["flags"]})
            log("fp64 per system", r64)
        else:
            sys64 = base_sys.copy()
            ffb64 = ff_binding(sys64, ff_kind) if ff_kind else None
            k64 = knobs(a.config, md.MD_FP64)
            r64 = run_gpu(sys64, md.MD_FP64, a.steps, a.warmup, k64["cluster_group"], k64["skin"],
                          use_graph=not a.eager, fast_capacity=k64["fast_capacity"], langevin=lg,
                          hybrid=hy, ff=ffb64, preroll_max=PREROLL)
            log("fp64", {k: v for k, v in r64.items() if k != "stats"})
            v64 = n * a.steps / (r64["ms"] * 1e-3)
            extra.update({"fp64_value": v64, "fp64_ms_per_step": r64["ms"] / a.steps,
                          "fp32_vs_fp64_speedup": value / v64,
                          "fp64_force_kernel_ms": r64["kernel_ms"],
                          "fp64_force_tflops": FLOP_PER_PAIR * r64["pairs"] /
                          (r64["kernel_ms"] * 1e-3) / 1e12,
                          "fp64_flags": r64["flags"], "fp64_rebuilds_timed": r64["builds"],
                          "fp64_preroll_steps": r64["preroll_steps"],
                          "fp64_replay_identical": r64["replay_identical"], "fp64_launch": k64})
        del sys64
    if not a.no_legs and plain:
        legs = {}
        if a.config != "water_98304":
            # the 98,304-atom pulse box over its whole 1,000-step schedule
            s2 = make_system("water_98304", 0)
            r = run_schedule(s2, md.MD_FP32_KAHAN, knobs("water_98304", md.MD_FP32_KAHAN,
                                                          cli=False))
            log("leg water_98304", r)
            legs["water_98304"] = r
            del s2
        if a.config != "methane_256":
            # 256 batched clusters against the plain FP64 form, one system per launch
            s4 = make_system("methane_256", 0)
            k4 = knobs("methane_256", md.MD_FP32_KAHAN, cli=False)
            r4 = run_gpu(s4.copy(), md.MD_FP32_KAHAN, a.steps, a.warmup, k4["cluster_group"],
                         k4["skin"], pair_samples=2, fast_capacity=k4["fast_capacity"])
            r4p = run_gpu_per_system(s4.copy(), md.MD_FP64, a.steps, a.warmup)
            # and the batch over its whole 2,000-step schedule (the clusters explode:
            # rebuilds every few steps late in it)
            r4s = run_schedule(s4.copy(), md.MD_FP32_KAHAN, k4)
            v4 = s4.n_atoms * a.steps / (r4["ms"] * 1e-3)
            v4p = s4.n_atoms * a.steps / (r4p["ms"] * 1e-3)
            legs["methane_256"] = {"atoms": s4.n_atoms, "systems": s4.n_systems, "launch": k4,
                                   "batched_fp32_ms_per_step": r4["ms"] / a.steps,
                                   "batched_fp32_value": v4,
                                   "batched_force_kernel_ms": r4["kernel_ms"],
                                   "per_system_fp64_ms_per_step": r4p["ms"] / a.steps,
                                   "per_system_fp64_value": v4p,
                                   "batched_fp32_vs_per_system_fp64_speedup": v4 / v4p,
                                   "batched_fp32_schedule_ms_per_step": r4s["ms_per_step"],
                                   "batched_fp32_schedule_rebuilds": r4s["rebuilds"],
                                   "flags": r4["flags"] | r4p["flags"] | r4s["flags"]}
            log("leg methane_256", legs["methane_256"])
            del s4
        extra["legs"] = legs

    if a.rdf:
        rr = run_rdf(make_system(a.config, S, a.dt_fs))
        log("rdf", rr)
        extra.update(rr)

    kernel_ms = r32["kernel_ms"]
    fpp = (FLOP_PER_PAIR_HYBRID if hy is not None else FLOP_PER_PAIR) + \
        (FLOP_QLJ_EXTRA if ffb is not None else 0)
    achieved = fpp * r32["pairs"] / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                # the counter summary covers the Debye kernel on the plain workload
                "traffic": traffic_from_profile(a.config) if plain else None,
                "kernel": "k_force32" + ("<HYBRID>" if hy is not None else "") +
                          ("<QLJ>" if ffb is not None else ""),
                "kernel_ms": kernel_ms,
                "flop_per_pair": fpp,
                "algorithmic_flop_per_launch": fpp * r32["pairs"],
                "frac_of_nonpacked_fp32": achieved / PEAK_FP32_NONPACKED_TFLOPS}

    kv = profile_values(a.config) if plain else {}
    if "valu_issue_per_cu_cycle" in kv:
        # from the committed counter summary (launches with current lists)
        extra.update(valu_issue_per_cu_cycle=float(kv["valu_issue_per_cu_cycle"]),
                     valu_lane_instructions_per_code=float(kv["valu_lane_instructions_per_code"]))
    out = {"metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": r32["ms"] / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": a.config, "atoms": n, "precision": "fp32 forces + kahan, "
                      "fp64 positions/integration/energies", "rc_nm": sys32.rc,
                      "skin_nm": k32["skin"] if k32["skin"] is not None else sys32.skin,
                      "cluster_group": st["cluster_group"],
                      "fast_capacity": k32["fast_capacity"], "tuned": k32["tuned"],
                      "systems": sys32.n_systems, "langevin": lg is not None,
                      "hybrid_screening": hy is not None,
                      "forcefield": ff_kind, "dt_fs": sys32.dt * 1e3,
                      "launch": "eager" if a.eager else "graph", "parallelism": "single-gpu"},
           "roofline": roofline, "extra": extra}
    if not a.no_cpu:
        off = None
        if ffb is not None:
            import oracle
            off = oracle.ForceField(sys32.n_atoms, inv_z=1.0 / ffb["z_type"],
                                    sigma=ffb["sigma_type"], excl=ffb["excl"],
                                    bonds=ffb["bonds"], bond_par=ffb["bond_par"],
                                    angles=ffb["angles"], angle_par=ffb["angle_par"])
        out["cpu_baseline"] = cpu_baseline(sys32, langevin=lg, hybrid=hy, ff=off)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
