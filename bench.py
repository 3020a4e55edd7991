"""Benchmark: atom-steps/s of the full screened-force + ionization step on one MI355X.

One step = device-side rebuild check / neighbour rebuild when due, stochastic
ionization, screened FP32 pair forces with compensated sums and the FP64 energy,
and the FP64 velocity-Verlet half steps with the kinetic-energy reduction.  Every
step is one replay of a captured HIP graph; inputs are resident in HBM before the
timed region.  Workload: the 98,304-atom bulk-water pulse box (32,768 H2O in a
9.93 nm periodic cube, lambda_D ramp 1.0 -> 0.15 nm, Gaussian pulse), synthetic
and seeded.

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
METRIC = "atom-steps/s for screened-force+ionize step; % FP32 VALU peak; FP32-vs-FP64 speedup"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_system(name, n_steps):
    from paper_2401_03180_amd import synth
    if name == "water_98304":
        return synth.water_pulse(n_steps=n_steps)
    if name == "water_1536":
        return synth.water_small(n_steps=n_steps)
    if name == "protein_524288":
        return synth.protein_crystal(n_steps=n_steps)
    if name == "water_4194304":
        return synth.water_large(n_steps=n_steps)
    if name == "methane_256":
        return synth.methane_clusters(n_steps=n_steps)
    raise SystemExit("unknown config " + name)


STATE = ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "q")


def run_gpu(sys_, prec, steps, warmup, cluster_group, skin, pair_samples=5):
    """Timed region: `steps` replays of the captured step graph, inputs resident.
    Then the same steps are replayed eagerly from a snapshot of the state at the
    start of the timed region, with the force-kernel timer on: the trajectory is
    deterministic, so the eager replay launches exactly the kernels of the timed
    region (checked: identical final state and rebuild count) and gives the
    duration of every force-kernel launch.  Pair counts are sampled between steps
    of the replay (where no list rebuild is pending)."""
    import torch
    from paper_2401_03180_amd import md
    eng = md.Engine(sys_, prec, cluster_group=cluster_group, skin=skin)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eng.set_step(0, stream)
        eng.build(md.MD_BUILD_FORCE, stream)
        eng.forces(energy=True, stream=stream)
        graph = eng.graph(md.MD_BUILD_AUTO, stream, energy=True, ekin=True)
        for _ in range(warmup):
            md.md_graph_launch(graph, stream)
        # the timed trajectory starts from a fresh build of the current positions
        eng.build(md.MD_BUILD_FORCE, stream)
        stream.synchronize()
        snap = {n: getattr(eng, n).clone() for n in STATE}
        k0 = eng.get_step(stream)
        st0 = eng.stats(stream)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            md.md_graph_launch(graph, stream)
        ev1.record(stream)
        stream.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        flags = eng.sync_check(stream, raise_on_flags=False)
        st1 = eng.stats(stream)
        final = {n: getattr(eng, n).clone() for n in STATE}
        step_end = eng.get_step(stream)

        # eager replay of the same steps with the force-kernel timer
        for n in STATE:
            getattr(eng, n).copy_(snap[n])
        eng.set_step(k0, stream)
        eng.build(md.MD_BUILD_FORCE, stream)
        stream.synchronize()
        st2 = eng.stats(stream)
        eng.timer_start(steps)
        sample_at = set(int(v) for v in np.linspace(1, steps, pair_samples))
        pairs = []
        for i in range(1, steps + 1):
            eng.step(md.MD_BUILD_AUTO, energy=True, ekin=True, stream=stream)
            if i in sample_at:
                stream.synchronize()
                pairs.append(eng.debug_pairs(prec=prec, stream=stream).shape[0])
        durations = eng.timer_read()
        stream.synchronize()
        st3 = eng.stats(stream)
        same = all(torch.equal(getattr(eng, n), final[n]) for n in STATE)
        eng.timer_start(0)
    eng.close()
    builds = st1["n_builds"] - st0["n_builds"]
    builds_replay = st3["n_builds"] - st2["n_builds"]
    d = np.asarray(durations, dtype=np.float64)
    return {"ms": ms, "wall_s": wall, "flags": flags, "pairs": float(np.mean(pairs)),
            "pairs_min": int(min(pairs)), "pairs_max": int(max(pairs)),
            "kernel_ms": float(d.mean()), "kernel_ms_median": float(np.median(d)),
            "kernel_ms_p90": float(np.percentile(d, 90)), "kernel_launches": int(d.size),
            "builds": builds, "builds_replay": builds_replay,
            "replay_identical": bool(same and builds == builds_replay), "stats": st1,
            "step": step_end}


def cpu_baseline(sys_, target_s=12.0, threads=None):
    """The oracle, as it stands, on a bounded sample of one step: full-j force rows for a
    random subset of atoms plus ionization and velocity Verlet over all atoms; the
    per-step time is extrapolated from the rows to all atoms."""
    import oracle
    threads = threads or min(os.cpu_count() or 1, 16)
    n = sys_.n_atoms
    rng = np.random.default_rng(0)
    kap = oracle.kappa_from_lambda(sys_.lambda_d[:, 1])
    probe = np.sort(rng.choice(n, 256, replace=False))
    t = time.perf_counter()
    oracle.forces_rows(sys_, probe, kappa=kap, n_threads=threads)
    per_row = (time.perf_counter() - t) / probe.size
    rows_n = int(min(n, max(256, target_s / max(per_row, 1e-9))))
    rows = np.sort(rng.choice(n, rows_n, replace=False))
    t = time.perf_counter()
    oracle.forces_rows(sys_, rows, kappa=kap, n_threads=threads)
    t_rows = time.perf_counter() - t
    q = sys_.q.copy()
    pos = [sys_.x.copy(), sys_.y.copy(), sys_.z.copy()]
    vel = [sys_.vx.copy(), sys_.vy.copy(), sys_.vz.copy()]
    F = (np.zeros(n), np.zeros(n), np.zeros(n))
    t = time.perf_counter()
    oracle.vv(0, sys_.dt, sys_.inv_mass, F, pos, vel)
    oracle.ionize(sys_, q, 1)
    oracle.vv(1, sys_.dt, sys_.inv_mass, F, pos, vel)
    t_elem = time.perf_counter() - t
    t_step = t_rows * n / rows_n + t_elem
    return {"value": n / t_step, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
            "sample": "O(N^2) FP64 oracle: full-j force rows of %d of %d atoms (%.1f s) plus "
                      "ionize and velocity Verlet over all atoms, extrapolated to one full "
                      "step (%.1f s)" % (rows_n, n, t_rows, t_step)}


def traffic_from_profile(kernel_src_hash):
    """HBM bytes per force launch from committed rocprofv3 counter runs, if they were
    taken on the current force-kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "force32_water_98304_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha1") != kernel_src_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="water_98304")
    ap.add_argument("--cluster-group", type=int, default=0)
    ap.add_argument("--skin", type=float, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
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

    S = a.warmup + a.steps
    sys32 = make_system(a.config, S)
    log("config", a.config, "atoms", sys32.n_atoms, "steps", a.steps, "warmup", a.warmup)
    r32 = run_gpu(sys32, md.MD_FP32_KAHAN, a.steps, a.warmup, a.cluster_group, a.skin)
    log("fp32", {k: v for k, v in r32.items() if k != "stats"})
    n = sys32.n_atoms
    value = n * a.steps / (r32["ms"] * 1e-3)
    extra = {"flags": r32["flags"], "rebuilds_timed": r32["builds"],
             "replay_identical": r32["replay_identical"],
             "pairs_in_cutoff_mean": r32["pairs"], "pairs_min": r32["pairs_min"],
             "pairs_max": r32["pairs_max"], "force_launches_timed": r32["kernel_launches"],
             "force_kernel_ms_median": r32["kernel_ms_median"],
             "force_kernel_ms_p90": r32["kernel_ms_p90"],
             "list_codes": r32["stats"]["n_list_codes"],
             "groups": r32["stats"]["n_groups"], "cluster_group": r32["stats"]["cluster_group"],
             "max_group_entries": r32["stats"]["max_group_entries"],
             "group_entry_capacity": r32["stats"]["group_entry_capacity"],
             "max_list_len": r32["stats"]["max_list_len"],
             "list_capacity": r32["stats"]["list_capacity"]}
    if not a.no_fp64:
        sys64 = make_system(a.config, S)
        r64 = run_gpu(sys64, md.MD_FP64, a.steps, a.warmup, a.cluster_group, a.skin)
        log("fp64", {k: v for k, v in r64.items() if k != "stats"})
        v64 = n * a.steps / (r64["ms"] * 1e-3)
        extra.update({"fp64_value": v64, "fp64_ms_per_step": r64["ms"] / a.steps,
                      "fp32_vs_fp64_speedup": value / v64,
                      "fp64_force_kernel_ms": r64["kernel_ms"], "fp64_flags": r64["flags"],
                      "fp64_replay_identical": r64["replay_identical"]})

    kernel_ms = r32["kernel_ms"]
    achieved = FLOP_PER_PAIR * r32["pairs"] / (kernel_ms * 1e-3) / 1e12
    src = open(os.path.join(ROOT, "paper_2401_03180_amd", "csrc", "md_force.hip"), "rb").read()
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": traffic_from_profile(hashlib.sha1(src).hexdigest()),
                "kernel": "k_force32", "kernel_ms": kernel_ms,
                "flop_per_pair": FLOP_PER_PAIR,
                "frac_of_nonpacked_fp32": achieved / PEAK_FP32_NONPACKED_TFLOPS}

    out = {"metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": r32["ms"] / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": a.config, "atoms": n, "precision": "fp32 forces + kahan, "
                      "fp64 positions/integration/energies", "rc_nm": sys32.rc,
                      "skin_nm": a.skin if a.skin is not None else sys32.skin,
                      "parallelism": "single-gpu"},
           "roofline": roofline, "extra": extra}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sys32)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
