"""ctypes binding of libmd_hip.so (include/md.h), with the same entry-point names.

The functions here only marshal arguments: torch CUDA tensors are passed as raw
device pointers, streams as hipStream_t handles.  Every step of the computation
runs in the library's HIP kernels.  Importing this module raises if the built
library is missing (run ``python -m paper_2401_03180_amd.build`` or
``__graft_entry__.build()``); there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmd_hip.so")

MD_OK, MD_ERR_ARG, MD_ERR_HIP, MD_ERR_CAPACITY = 0, -1, -2, -3
MD_ERR_GEOMETRY, MD_ERR_DEVICE, MD_ERR_STATE = -4, -5, -6
MD_FP64, MD_FP32_KAHAN = 0, 1
MD_BUILD_AUTO, MD_BUILD_FORCE, MD_BUILD_CHECK = 0, 1, 2
MD_FLAG_CELL_OVERFLOW, MD_FLAG_LIST_OVERFLOW, MD_FLAG_SKIN = 0x1, 0x2, 0x4
MD_FLAG_NONFINITE, MD_FLAG_STEP, MD_FLAG_BAD_INPUT = 0x8, 0x10, 0x20
MD_FLAG_BARRIER = 0x40
MD_MAX_TYPES, MD_MAX_ELEMENTS, MD_MAX_CHARGE_STATES = 8, 8, 128
MD_RDF_SCRATCH_BYTES = 32 << 20

EXPORTED = (
    "md_create", "md_destroy", "md_last_error", "md_bind_tables", "md_set_step", "md_get_step",
    "md_build_cells", "md_ionize_step", "md_screened_forces",
    "md_integrate_vv", "md_sync_check", "md_clear_flags", "md_debug_pairs", "md_get_stats",
    "md_force_timer_start", "md_force_timer_read", "md_step", "md_graph_create", "md_graph_launch", "md_graph_destroy", "md_debye_length_nm",
    "md_rates_from_fractions", "md_bind_langevin", "md_integrate_langevin", "md_bind_hybrid",
    "md_rdf_histogram", "md_rdf_normalize", "md_structure_factor", "md_bind_forcefield",
    "md_rdf_histogram_noalloc",
)


class md_config(ctypes.Structure):
    _fields_ = [("n_systems", ctypes.c_int32), ("n_types", ctypes.c_int32),
                ("n_elements", ctypes.c_int32), ("n_charge_states", ctypes.c_int32),
                ("periodic", ctypes.c_int32), ("screen_lj", ctypes.c_int32),
                ("rc", ctypes.c_double), ("skin", ctypes.c_double),
                ("capacity_atoms", ctypes.c_int64), ("cluster_group", ctypes.c_int32),
                ("max_neighbors", ctypes.c_int32), ("density_hint", ctypes.c_double),
                ("fast_capacity", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class md_stats(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int64), ("n_clusters", ctypes.c_int64),
                ("n_groups", ctypes.c_int64), ("n_entries", ctypes.c_int64),
                ("n_list_codes", ctypes.c_int64), ("max_list_len", ctypes.c_int64),
                ("list_capacity", ctypes.c_int64), ("max_group_entries", ctypes.c_int64),
                ("group_entry_capacity", ctypes.c_int64), ("n_builds", ctypes.c_int64),
                ("n_fast", ctypes.c_int64), ("n_fast_raw", ctypes.c_int64),
                ("cluster_group", ctypes.c_int32), ("flags", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class md_step_args(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("dt", ctypes.c_double),
                *[(n, ctypes.c_void_p) for n in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy",
                                                  "fz", "inv_mass", "elem", "type", "atom_id",
                                                  "q", "epot", "ekin")]]


class MDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("md status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    """Load libmd_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmd_hip.so is not built (%s); run paper_2401_03180_amd.build"
                              % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "md_create": [P, P, P], "md_destroy": [P], "md_last_error": [P],
            "md_bind_tables": [P, P, P, P, P, P, P, P, P, i64],
            "md_set_step": [P, i64, P], "md_get_step": [P, P, P],
            "md_build_cells": [P, P, P, P, P, i32, P],
            "md_ionize_step": [P, P, P, P, P],
            "md_screened_forces": [P, ctypes.c_int, P, P, P, P, P, P, P, P, P, P],
            "md_integrate_vv": [P, i32, f64, P, P, P, P, P, P, P, P, P, P, P, P],
            "md_sync_check": [P, P, P], "md_clear_flags": [P, P],
            "md_debug_pairs": [P, ctypes.c_int, P, P, P, P, P, P, i64, P, P],
            "md_get_stats": [P, P, P], "md_step": [P, P, i32, P],
            "md_force_timer_start": [P, i32], "md_force_timer_read": [P, P, i32, P],
            "md_graph_create": [P, P, i32, P, P], "md_graph_launch": [P, P],
            "md_graph_destroy": [P], "md_debye_length_nm": [f64, f64],
            "md_rates_from_fractions": [i64, i32, P, P],
            "md_bind_langevin": [P, P, P, f64],
            "md_bind_hybrid": [P, P],
            "md_rdf_histogram": [P, P, P, P, P, f64, i32, P, P],
            "md_rdf_histogram_noalloc": [P, P, P, P, P, f64, i32, P, P],
            "md_bind_forcefield": [P, P, P, P, i64, P, P, i64, P, P, i64],
            "md_rdf_normalize": [i32, f64, P, i64, i64, i32, f64, P],
            "md_structure_factor": [i32, f64, P, f64, i32, P, P],
            "md_integrate_langevin": [P, f64, P, P, P, P, P, P, P, P, P, P, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.md_last_error.restype = ctypes.c_char_p
        L.md_debye_length_nm.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(t):
    """Device (or host numpy) pointer of a tensor/array, or None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags.c_contiguous
        return t.ctypes.data
    assert t.is_contiguous(), "arrays must be contiguous"
    return t.data_ptr()


def _check(ctx, status):
    if status != MD_OK:
        raise MDError(status, lib().md_last_error(ctx).decode())


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# ---------------------------------------------------------------- thin wrappers (same names)

def md_create(cfg: md_config, sys_offsets: np.ndarray):
    offs = np.ascontiguousarray(sys_offsets, dtype=np.int64)
    h = ctypes.c_void_p()
    st = lib().md_create(ctypes.byref(cfg), offs.ctypes.data, ctypes.byref(h))
    _check(None, st)
    return h


def md_destroy(ctx):
    _check(None, lib().md_destroy(ctx))


def md_bind_tables(ctx, box, c6, c12, qmax, lambda_d, base, g, seeds, n_steps):
    arrs = [None if box is None else np.ascontiguousarray(box, np.float64),
            np.ascontiguousarray(c6, np.float64), np.ascontiguousarray(c12, np.float64),
            np.ascontiguousarray(qmax, np.int8), np.ascontiguousarray(lambda_d, np.float64),
            np.ascontiguousarray(base, np.float64), np.ascontiguousarray(g, np.float64),
            np.ascontiguousarray(seeds, np.uint64)]
    _check(ctx, lib().md_bind_tables(ctx, *[_ptr(a) for a in arrs], int(n_steps)))


def md_set_step(ctx, step, stream=None):
    _check(ctx, lib().md_set_step(ctx, int(step), _stream(stream)))


def md_get_step(ctx, stream=None) -> int:
    v = ctypes.c_int64()
    _check(ctx, lib().md_get_step(ctx, ctypes.byref(v), _stream(stream)))
    return v.value


def md_build_cells(ctx, x, y, z, type_, mode=MD_BUILD_FORCE, stream=None):
    _check(ctx, lib().md_build_cells(ctx, _ptr(x), _ptr(y), _ptr(z), _ptr(type_), int(mode),
                                     _stream(stream)))


def md_ionize_step(ctx, elem, atom_id, q, stream=None):
    _check(ctx, lib().md_ionize_step(ctx, _ptr(elem), _ptr(atom_id), _ptr(q), _stream(stream)))


def md_screened_forces(ctx, prec, x, y, z, q, type_, fx, fy, fz, epot=None, stream=None):
    _check(ctx, lib().md_screened_forces(ctx, int(prec), _ptr(x), _ptr(y), _ptr(z), _ptr(q),
                                         _ptr(type_), _ptr(fx), _ptr(fy), _ptr(fz), _ptr(epot),
                                         _stream(stream)))


def md_integrate_vv(ctx, phase, dt, inv_mass, fx, fy, fz, x, y, z, vx, vy, vz, ekin=None,
                    stream=None):
    _check(ctx, lib().md_integrate_vv(ctx, int(phase), float(dt), _ptr(inv_mass), _ptr(fx),
                                      _ptr(fy), _ptr(fz), _ptr(x), _ptr(y), _ptr(z), _ptr(vx),
                                      _ptr(vy), _ptr(vz), _ptr(ekin), _stream(stream)))


def md_bind_langevin(ctx, gamma, kt, dt):
    """gamma: host [B, E] ps^-1 (None unbinds); kt: host [B, S+1] kJ/mol."""
    if gamma is None:
        _check(ctx, lib().md_bind_langevin(ctx, None, None, float(dt)))
        return
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    k = np.ascontiguousarray(kt, dtype=np.float64)
    _check(ctx, lib().md_bind_langevin(ctx, g.ctypes.data, k.ctypes.data, float(dt)))


def md_bind_hybrid(ctx, ne):
    """ne: host [B, S+1] free-electron density in nm^-3 (None unbinds)."""
    if ne is None:
        _check(ctx, lib().md_bind_hybrid(ctx, None))
        return
    n = np.ascontiguousarray(ne, dtype=np.float64)
    _check(ctx, lib().md_bind_hybrid(ctx, n.ctypes.data))


def md_bind_forcefield(ctx, z_type=None, excl=None, bonds=None, bond_par=None, angles=None,
                       angle_par=None, sigma_type=None):
    """Host arrays (see include/md.h); None disables a part (z_type and sigma_type go
    together)."""
    def arr(a, dt, cols):
        if a is None:
            return None, 0
        v = np.ascontiguousarray(np.asarray(a, dtype=dt).reshape(-1, cols))
        return v, v.shape[0]
    z = None if z_type is None else np.ascontiguousarray(z_type, dtype=np.int8)
    sg = None if sigma_type is None else np.ascontiguousarray(sigma_type, dtype=np.float64)
    ex, nex = arr(excl, np.int32, 2)
    bo, nbo = arr(bonds, np.int32, 2)
    bp, _ = arr(bond_par, np.float64, 3)
    an, nan_ = arr(angles, np.int32, 3)
    ap, _ = arr(angle_par, np.float64, 2)
    ptr = lambda v: None if v is None else v.ctypes.data
    _check(ctx, lib().md_bind_forcefield(ctx, ptr(z), ptr(sg), ptr(ex), nex, ptr(bo), ptr(bp),
                                         nbo, ptr(an), ptr(ap), nan_))


def md_rdf_histogram(ctx, x, y, z, elem, r_max, n_bins, hist, stream=None):
    """hist: device int64/uint64 tensor [B, E, E, n_bins] (added to)."""
    _check(ctx, lib().md_rdf_histogram(ctx, _ptr(x), _ptr(y), _ptr(z), _ptr(elem), float(r_max),
                                       int(n_bins), _ptr(hist), _stream(stream)))


def md_rdf_histogram_noalloc(ctx, x, y, z, elem, r_max, n_bins, hist, stream=None):
    """md_rdf_histogram with the library's fixed per-device workspace (allocates
    nothing)."""
    _check(ctx, lib().md_rdf_histogram_noalloc(ctx, _ptr(x), _ptr(y), _ptr(z), _ptr(elem),
                                               float(r_max), int(n_bins), _ptr(hist),
                                               _stream(stream)))


def md_rdf_normalize(counts, r_max, n_a, n_b, same, volume) -> np.ndarray:
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    g = np.zeros(c.size)
    _check(None, lib().md_rdf_normalize(c.size, float(r_max), c.ctypes.data, int(n_a), int(n_b),
                                        int(bool(same)), float(volume), g.ctypes.data))
    return g


def md_structure_factor(g, r_max, rho0, q) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    S = np.zeros(q.size)
    _check(None, lib().md_structure_factor(g.size, float(r_max), g.ctypes.data, float(rho0),
                                           q.size, q.ctypes.data, S.ctypes.data))
    return S


def md_integrate_langevin(ctx, dt, inv_mass, elem, atom_id, fx, fy, fz, x, y, z, vx, vy, vz,
                          stream=None):
    _check(ctx, lib().md_integrate_langevin(ctx, float(dt), _ptr(inv_mass), _ptr(elem),
                                            _ptr(atom_id), _ptr(fx), _ptr(fy), _ptr(fz), _ptr(x),
                                            _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz),
                                            _stream(stream)))


def md_sync_check(ctx, stream=None, raise_on_flags=True) -> int:
    f = ctypes.c_uint32()
    st = lib().md_sync_check(ctx, _stream(stream), ctypes.byref(f))
    if st != MD_ERR_DEVICE or raise_on_flags:
        _check(ctx, st)
    return f.value


def md_clear_flags(ctx, stream=None):
    _check(ctx, lib().md_clear_flags(ctx, _stream(stream)))


def md_debug_pairs(ctx, prec, x, y, z, q, max_pairs, stream=None, e_atom=None) -> np.ndarray:
    """Pairs (i, j) of the evaluation; e_atom (host FP64 [N] numpy array, or None)
    receives the per-atom energies."""
    buf = np.empty((max(int(max_pairs), 1), 2), dtype=np.int32)
    n = ctypes.c_int64()
    _check(ctx, lib().md_debug_pairs(ctx, int(prec), _ptr(x), _ptr(y), _ptr(z), _ptr(q),
                                     ctypes.byref(n), buf.ctypes.data, int(max_pairs),
                                     None if e_atom is None else e_atom.ctypes.data,
                                     _stream(stream)))
    if n.value > max_pairs:
        raise MDError(MD_ERR_CAPACITY, "pair buffer too small: %d > %d" % (n.value, max_pairs))
    return buf[:n.value]


def md_count_pairs(ctx, prec, x, y, z, q, stream=None, e_atom=None) -> int:
    """Number of interacting pairs of the evaluation (nothing exported)."""
    n = ctypes.c_int64()
    _check(ctx, lib().md_debug_pairs(ctx, int(prec), _ptr(x), _ptr(y), _ptr(z), _ptr(q),
                                     ctypes.byref(n), None, 0,
                                     None if e_atom is None else e_atom.ctypes.data,
                                     _stream(stream)))
    return int(n.value)


def md_force_timer_start(ctx, capacity):
    _check(ctx, lib().md_force_timer_start(ctx, int(capacity)))


def md_force_timer_read(ctx) -> np.ndarray:
    """Kernel durations (ms) of the force launches timed since md_force_timer_start."""
    n = ctypes.c_int32()
    _check(ctx, lib().md_force_timer_read(ctx, None, 0, ctypes.byref(n)))
    out = np.zeros(max(n.value, 1), dtype=np.float32)
    _check(ctx, lib().md_force_timer_read(ctx, out.ctypes.data, n.value, ctypes.byref(n)))
    return out[:n.value]


def md_get_stats(ctx, stream=None) -> dict:
    s = md_stats()
    _check(ctx, lib().md_get_stats(ctx, ctypes.byref(s), _stream(stream)))
    return s.as_dict()


def md_step(ctx, args: md_step_args, build_mode=MD_BUILD_AUTO, stream=None):
    _check(ctx, lib().md_step(ctx, ctypes.byref(args), int(build_mode), _stream(stream)))


def md_graph_create(ctx, args: md_step_args, build_mode, stream):
    h = ctypes.c_void_p()
    _check(ctx, lib().md_graph_create(ctx, ctypes.byref(args), int(build_mode),
                                      _stream(stream), ctypes.byref(h)))
    return h


def md_graph_launch(graph, stream=None):
    st = lib().md_graph_launch(graph, _stream(stream))
    if st != MD_OK:
        raise MDError(st, "graph launch failed")


def md_graph_destroy(graph):
    lib().md_graph_destroy(graph)


def md_debye_length_nm(te_ev, ne_m3) -> float:
    return float(lib().md_debye_length_nm(float(te_ev), float(ne_m3)))


def md_rates_from_fractions(P) -> np.ndarray:
    P = np.ascontiguousarray(P, dtype=np.float64)
    out = np.zeros_like(P)
    _check(None, lib().md_rates_from_fractions(P.shape[0] - 1, P.shape[1] - 1, P.ctypes.data,
                                               out.ctypes.data))
    return out


# ---------------------------------------------------------------- system-level helper

class Engine:
    """Device-resident state of a synthetic System plus a library context.

    Holds torch CUDA tensors for every per-atom array and calls the C ABI in the
    method's order.  ``precision`` is MD_FP32_KAHAN or MD_FP64.
    """

    def __init__(self, sys, precision=MD_FP32_KAHAN, cluster_group=0, skin=None,
                 density_hint=0.0, max_neighbors=0, fast_capacity=0, device="cuda"):
        import torch
        self.torch = torch
        self.sys = sys
        self.prec = precision
        dev = torch.device(device)
        self.dev = dev
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        self.x, self.y, self.z = (t(a, torch.float64) for a in (sys.x, sys.y, sys.z))
        self.vx, self.vy, self.vz = (t(a, torch.float64) for a in (sys.vx, sys.vy, sys.vz))
        self.fx, self.fy, self.fz = (torch.zeros(sys.n_atoms, dtype=torch.float64, device=dev)
                                     for _ in range(3))
        self.inv_mass = t(sys.inv_mass, torch.float64)
        self.elem = t(sys.elem, torch.uint8)
        self.type = t(sys.type, torch.uint8)
        self.atom_id = t(sys.atom_id.astype(np.int32), torch.int32)
        self.q = t(sys.q, torch.int8)
        self.epot = torch.zeros(sys.n_systems, dtype=torch.float64, device=dev)
        self.ekin = torch.zeros(sys.n_systems, dtype=torch.float64, device=dev)
        cfg = md_config()
        cfg.n_systems = sys.n_systems
        cfg.n_types = sys.n_types
        cfg.n_elements = sys.n_elements
        cfg.n_charge_states = sys.base.shape[1]
        cfg.periodic = int(sys.periodic)
        cfg.screen_lj = int(sys.screen_lj)
        cfg.rc = sys.rc
        cfg.skin = sys.skin if skin is None else skin
        cfg.capacity_atoms = sys.n_atoms
        cfg.cluster_group = cluster_group
        cfg.max_neighbors = max_neighbors
        cfg.density_hint = density_hint
        cfg.fast_capacity = fast_capacity
        self.cfg = cfg
        self.ctx = md_create(cfg, sys.sys_offsets)
        md_bind_tables(self.ctx, sys.box, sys.c6, sys.c12, sys.qmax, sys.lambda_d, sys.base,
                       sys.g, sys.seeds, sys.n_steps)
        self.graphs = {}

    def close(self):
        for g in self.graphs.values():
            md_graph_destroy(g)
        self.graphs = {}
        if self.ctx is not None:
            md_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # individual calls
    def build(self, mode=MD_BUILD_FORCE, stream=None):
        md_build_cells(self.ctx, self.x, self.y, self.z, self.type, mode, stream)

    def ionize(self, stream=None):
        md_ionize_step(self.ctx, self.elem, self.atom_id, self.q, stream)

    def forces(self, prec=None, energy=True, stream=None):
        md_screened_forces(self.ctx, self.prec if prec is None else prec, self.x, self.y, self.z,
                           self.q, self.type, self.fx, self.fy, self.fz,
                           self.epot if energy else None, stream)

    def vv(self, phase, ekin=True, stream=None):
        md_integrate_vv(self.ctx, phase, self.sys.dt, self.inv_mass, self.fx, self.fy, self.fz,
                        self.x, self.y, self.z, self.vx, self.vy, self.vz,
                        self.ekin if ekin else None, stream)

    def bind_langevin(self, gamma, kt):
        """Bind (or, with gamma None, unbind) the electron-ion coupling; graphs captured
        before run the previous integrator and are dropped."""
        for g in self.graphs.values():
            md_graph_destroy(g)
        self.graphs = {}
        md_bind_langevin(self.ctx, gamma, kt, self.sys.dt)

    def bind_hybrid(self, ne):
        """Bind (or, with None, unbind) hybrid ion-sphere / Debye screening; graphs
        captured before use the previous force kernel and are dropped."""
        for g in self.graphs.values():
            md_graph_destroy(g)
        self.graphs = {}
        md_bind_hybrid(self.ctx, ne)

    def bind_forcefield(self, **kw):
        """md_bind_forcefield with keyword arrays (z_type, sigma_type, excl, bonds,
        bond_par, angles, angle_par); graphs captured before are dropped."""
        for g in self.graphs.values():
            md_graph_destroy(g)
        self.graphs = {}
        md_bind_forcefield(self.ctx, **kw)

    def rdf(self, r_max, n_bins, hist=None, stream=None):
        """Pair-distance histogram [B, E, E, n_bins] (int64 tensor; added to `hist`
        when given)."""
        torch = self.torch
        if hist is None:
            E = self.sys.n_elements
            hist = torch.zeros((self.sys.n_systems, E, E, n_bins), dtype=torch.int64,
                               device=self.dev)
        md_rdf_histogram(self.ctx, self.x, self.y, self.z, self.elem, r_max, n_bins, hist,
                         stream)
        return hist

    def langevin(self, stream=None):
        md_integrate_langevin(self.ctx, self.sys.dt, self.inv_mass, self.elem, self.atom_id,
                              self.fx, self.fy, self.fz, self.x, self.y, self.z, self.vx,
                              self.vy, self.vz, stream)

    def step_args(self, energy=True, ekin=True):
        a = md_step_args()
        a.prec = self.prec
        a.dt = self.sys.dt
        for n in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "inv_mass", "elem", "type",
                  "atom_id", "q"):
            setattr(a, n, _ptr(getattr(self, n)))
        a.epot = _ptr(self.epot) if energy else None
        a.ekin = _ptr(self.ekin) if ekin else None
        self._args = a
        return a

    def step(self, build_mode=MD_BUILD_AUTO, energy=True, ekin=True, stream=None):
        md_step(self.ctx, self.step_args(energy, ekin), build_mode, stream)

    def timer_start(self, capacity):
        md_force_timer_start(self.ctx, capacity)

    def timer_read(self):
        return md_force_timer_read(self.ctx)

    def set_step(self, k, stream=None):
        md_set_step(self.ctx, k, stream)

    def get_step(self, stream=None):
        return md_get_step(self.ctx, stream)

    def sync_check(self, stream=None, raise_on_flags=True):
        return md_sync_check(self.ctx, stream, raise_on_flags)

    def stats(self, stream=None):
        return md_get_stats(self.ctx, stream)

    def debug_pairs(self, prec=None, max_pairs=None, stream=None):
        if max_pairs is None:
            max_pairs = int(self.sys.n_atoms * 400 * (self.sys.rc + 0.2) ** 3) + 1024
        return md_debug_pairs(self.ctx, self.prec if prec is None else prec, self.x, self.y,
                              self.z, self.q, max_pairs, stream)

    def count_pairs(self, prec=None, stream=None):
        return md_count_pairs(self.ctx, self.prec if prec is None else prec, self.x, self.y,
                              self.z, self.q, stream)

    def atom_energies(self, prec=None, stream=None):
        """Per-atom energies e_i = 1/2 sum_j phi_ij of one evaluation at the current
        state (needs a build at the current positions) and the pair count."""
        e = np.zeros(self.sys.n_atoms, dtype=np.float64)
        n = md_count_pairs(self.ctx, self.prec if prec is None else prec, self.x, self.y,
                           self.z, self.q, stream, e_atom=e)
        return e, n

    def graph(self, build_mode, stream, energy=False, ekin=False):
        """Executable graph of one full step (captured once per argument set)."""
        key = (int(build_mode), energy, ekin)
        if key not in self.graphs:
            self.graphs[key] = md_graph_create(self.ctx, self.step_args(energy, ekin),
                                               build_mode, stream)
        return self.graphs[key]

    def host(self, name):
        return getattr(self, name).cpu().numpy()
