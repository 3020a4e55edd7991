"""Launch-configuration search for the screened-force + ionization step.

The step's cost depends on three knobs that trade work against each other:

* ``cluster_group`` (i-clusters per force work-group, 1/2/4/8): more clusters share
  one staged candidate table (less staging per cluster) but the table grows and
  fewer work-groups fit the LDS;
* ``skin`` (Verlet buffer, nm): a thicker buffer means longer per-atom lists but
  fewer atoms beyond skin/2, hence fewer rebuilds;
* ``fast_capacity``: atoms beyond skin/2 handled by the fast-atom kernels before a
  rebuild is requested.

Each candidate runs the workload itself (a window of its own schedule, as graph
replays, inputs resident) and is timed with HIP events; coordinate descent visits
skin, then cluster_group, then fast_capacity.  The best configuration is cached per
(device architecture, workload, precision) in ``tuned.json`` beside this module.
"""
from __future__ import annotations

import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")

SKINS = (0.06, 0.075, 0.09, 0.1, 0.12)
GROUPS = (2, 4, 8)
FAST_SCALE = (0.25, 0.5, 1.0, 2.0)      # multiples of the automatic capacity


def device_arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def cache_key(workload: str, prec: int) -> str:
    return "%s|%s|prec%d" % (device_arch(), workload, prec)


def load(workload: str, prec: int):
    """Cached configuration for this device and workload, or None."""
    if not os.path.exists(CACHE):
        return None
    return json.load(open(CACHE)).get(cache_key(workload, prec))


def auto_fast_capacity(n_atoms: int) -> int:
    """The library's automatic capacity (md_config.fast_capacity = 0)."""
    return int(min(1024, max(64, n_atoms // 96)))


def time_config(make_system, prec, steps, warmup, cluster_group, skin, fast_capacity):
    """ms per step of `steps` graph replays after `warmup` replays."""
    import torch
    from . import md
    sys_ = make_system()
    eng = md.Engine(sys_, prec, cluster_group=cluster_group, skin=skin,
                    fast_capacity=fast_capacity)
    st = torch.cuda.Stream()
    try:
        with torch.cuda.stream(st):
            eng.set_step(0, st)
            eng.build(md.MD_BUILD_FORCE, st)
            eng.forces(energy=True, stream=st)
            g = eng.graph(md.MD_BUILD_AUTO, st, energy=True, ekin=True)
            for _ in range(warmup):
                md.md_graph_launch(g, st)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                md.md_graph_launch(g, st)
            e1.record(st)
            st.synchronize()
            flags = eng.sync_check(st, raise_on_flags=False)
            builds = eng.stats(st)["n_builds"]
        ms = e0.elapsed_time(e1) / steps
    finally:
        eng.close()
    if flags:
        return float("inf"), builds
    return ms, builds


def tune(workload, make_system, prec, steps, warmup, log=print, save=True):
    """Coordinate descent over skin, cluster_group and fast_capacity; returns the best
    configuration (and stores it in the cache)."""
    n = make_system().n_atoms
    best = {"cluster_group": 4, "skin": 0.1, "fast_capacity": auto_fast_capacity(n)}
    trials = []

    def run(cfg):
        t0 = time.perf_counter()
        ms, builds = time_config(make_system, prec, steps, warmup, cfg["cluster_group"],
                                 cfg["skin"], cfg["fast_capacity"])
        trials.append(dict(cfg, ms_per_step=ms, builds=builds))
        log("tune %s: %.4f ms/step, %d builds (%.1f s)" % (cfg, ms, builds,
                                                          time.perf_counter() - t0))
        return ms

    best_ms = run(best)
    for key, values in (("skin", SKINS), ("cluster_group", GROUPS),
                        ("fast_capacity", tuple(max(16, int(f * auto_fast_capacity(n)))
                                                for f in FAST_SCALE))):
        for v in values:
            if v == best[key]:
                continue
            cand = dict(best, **{key: v})
            ms = run(cand)
            if ms < best_ms:
                best, best_ms = cand, ms
    result = dict(best, ms_per_step=best_ms, steps=steps, warmup=warmup, trials=trials)
    if save:
        data = json.load(open(CACHE)) if os.path.exists(CACHE) else {}
        data[cache_key(workload, prec)] = result
        with open(CACHE, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return result
