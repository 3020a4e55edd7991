"""CPU FP64 oracle for the screened-force + ionization step (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links, loads or
calls it, and the two share no code.

The arithmetic lives in ``md_oracle.c`` (plain C, FP64, contraction disabled);
this module compiles it with gcc and exposes thin ctypes wrappers over numpy
arrays, plus a reference trajectory driver that composes the steps in the
paper's order (ionize, screened forces, integrate).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "md_oracle.c")
_LIB = os.path.join(_HERE, "libmd_oracle.so")
_lock = threading.Lock()
_lib = None

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (FP contraction disabled)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
            L.orc_kappa_from_lambda.argtypes = [i64, P, P]
            L.orc_debye_length_nm.argtypes = [f64, f64]
            L.orc_debye_length_nm.restype = f64
            L.orc_rates_from_fractions.argtypes = [i64, i32, P, P]
            L.orc_forces.argtypes = [i64, P, i32, P, f64, P, P, P, P, P, i32, P, P, P, i32,
                                     P, P, P, P, P, P, P, i32, P, P, P, P]
            L.orc_forces.restype = i64
            L.orc_forces_rows.argtypes = [i64, P, P, P, i32, P, f64, P, P, P, P, P, i32, P, P,
                                          P, i32, P, P, P, P, P, P, i32, P, i32, P, P, P, P]
            L.orc_forces_rows.restype = i64
            L.orc_pairs.argtypes = [i64, P, i32, P, f64, P, P, P, P, P, i64]
            L.orc_pairs.restype = i64
            L.orc_pairs_rows.argtypes = [i64, P, P, P, i32, P, f64, P, P, P, P, P, i64, i32]
            L.orc_pairs_rows.restype = i64
            L.orc_pair_r2.argtypes = [i32, P, P, P, P, i64, i64]
            L.orc_pair_r2.restype = f64
            L.orc_philox4x32_10.argtypes = [P, P, P]
            L.orc_ionize.argtypes = [i64, P, P, P, P, P, i32, P, P, P, i64]
            L.orc_ionize.restype = i64
            L.orc_vv.argtypes = [i64, i32, f64, P, P, P, P, P, P, P, P, P, P]
            L.orc_langevin_normals.argtypes = [ctypes.c_uint32, i64, i64, ctypes.c_uint64, P]
            L.orc_vv_langevin.argtypes = [i64, P, P, i32, P, P, P, i64, i64, P, f64, P, P, P, P,
                                          P, P, P, P, P, P]
            L.orc_ekin.argtypes = [i64, P, P, P, P, P, P]
            L.orc_hybrid_coeffs.argtypes = [f64, f64, f64, P]
            L.orc_bonded.argtypes = [i64, P, i32, P, P, P, P, P, i64, P, P, i64, P, P, P, P, P,
                                     P]
            L.orc_rdf_histogram.argtypes = [i64, P, i32, P, P, P, P, P, i32, f64, i32, P]
            L.orc_rdf_normalize.argtypes = [i32, f64, P, i64, i64, i32, f64, P]
            L.orc_structure_factor.argtypes = [i32, f64, P, f64, i32, P, P]
            L.orc_hybrid_phi.argtypes = [f64, P, f64, f64, P, P]
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ------------------------------------------------------------------ schedules

def kappa_from_lambda(lambda_d) -> np.ndarray:
    lam = _c(lambda_d, np.float64)
    out = np.empty_like(lam)
    lib().orc_kappa_from_lambda(lam.size, _p(lam), _p(out))
    return out


def debye_length_nm(te_ev: float, ne_m3: float) -> float:
    return float(lib().orc_debye_length_nm(te_ev, ne_m3))


def rates_from_fractions(P) -> np.ndarray:
    P = _c(P, np.float64)
    S = P.shape[0] - 1
    Z = P.shape[1] - 1
    out = np.zeros_like(P)
    lib().orc_rates_from_fractions(S, Z, _p(P), _p(out))
    return out


# ------------------------------------------------------------------ hybrid screening

def hybrid_coeffs(Q, lambda_d, ne) -> np.ndarray:
    """(r', c1, c2, c3) of the hybrid potential of a charge-Q ion (Eq. 4-7 reading)."""
    out = np.empty(4)
    lib().orc_hybrid_coeffs(float(Q), float(lambda_d), float(ne), _p(out))
    return out


def hybrid_phi(Q, h, kappa, r):
    """(phi, -r dphi/dr) of the hybrid potential with coefficients h at distance r."""
    h = _c(h, np.float64)
    phi, w = ctypes.c_double(), ctypes.c_double()
    lib().orc_hybrid_phi(float(Q), _p(h), float(kappa), float(r), ctypes.byref(phi),
                         ctypes.byref(w))
    return phi.value, w.value


def hybrid_table(lambda_d, ne, n_q) -> np.ndarray:
    """[B, n_q, 4] coefficients for charges 0 .. n_q - 1 of every system, from the
    per-system Debye length and electron density of one force evaluation."""
    lam = np.atleast_1d(np.asarray(lambda_d, dtype=np.float64))
    n_e = np.atleast_1d(np.asarray(ne, dtype=np.float64))
    out = np.zeros((lam.size, n_q, 4))
    for b in range(lam.size):
        for Q in range(1, n_q):
            out[b, Q] = hybrid_coeffs(Q, lam[b], n_e[b])
    return out


# ------------------------------------------------------------------ force-field terms

class ForceField:
    """Optional terms of section II.B (readings): ``inv_z`` [T] = 1/Z per type with
    ``sigma`` [T] the neutral LJ radius per type: the radius of an atom shrinks to
    c sigma with c = 1 - q/Z (Eq. 11) and a pair's radius is the mean of the two
    scaled radii, so the pair's LJ radius is scaled by (c_i sigma_i + c_j sigma_j) /
    (sigma_i + sigma_j); ``excl`` lists the pairs (global atom indices) whose LJ
    term is omitted; ``bonds`` [n, 2] with ``bond_par`` [n, 3] = (D_e, beta, b_e) and
    ``angles`` [n, 3] (middle atom second) with ``angle_par`` [n, 2] = (k, theta0)
    are the Morse and harmonic-angle terms (Eq. 9, Eq. 10)."""

    def __init__(self, n_atoms, inv_z=None, excl=None, bonds=None, bond_par=None,
                 angles=None, angle_par=None, sigma=None):
        if (inv_z is None) != (sigma is None):
            raise ValueError("inv_z and sigma go together (Eq. 11 scales the radii)")
        self.inv_z = None if inv_z is None else _c(inv_z, np.float64)
        self.sigma = None if sigma is None else _c(sigma, np.float64)
        self.excl_off = self.excl = None
        if excl is not None:
            e = np.asarray(excl, dtype=np.int64).reshape(-1, 2)
            both = np.concatenate([e, e[:, ::-1]])
            both = both[np.lexsort((both[:, 1], both[:, 0]))]
            both = np.unique(both, axis=0)
            self.excl_off = _c(np.searchsorted(both[:, 0], np.arange(n_atoms + 1)), np.int64)
            self.excl = _c(both[:, 1], np.int64)
        z2 = np.zeros((0, 2), np.int32)
        self.bonds = _c(z2 if bonds is None else bonds, np.int32)
        self.bond_par = _c(np.zeros((0, 3)) if bond_par is None else bond_par, np.float64)
        self.angles = _c(np.zeros((0, 3), np.int32) if angles is None else angles, np.int32)
        self.angle_par = _c(np.zeros((0, 2)) if angle_par is None else angle_par, np.float64)

    def args(self):
        return _p(self.inv_z), _p(self.sigma), _p(self.excl_off), _p(self.excl)


def _ff_args(ff):
    return (None, None, None, None) if ff is None else ff.args()


def bonded(sys, ff, q=None, x=None, y=None, z=None):
    """Forces and per-system energies of the bonded terms alone."""
    x = _c(sys.x if x is None else x, np.float64)
    y = _c(sys.y if y is None else y, np.float64)
    z = _c(sys.z if z is None else z, np.float64)
    q = _c(sys.q if q is None else q, np.int8)
    n = x.shape[0]
    out = {k: np.zeros(n) for k in ("fx", "fy", "fz")}
    epot = np.zeros(sys.n_systems)
    box = None if sys.box is None else _c(sys.box, np.float64)
    lib().orc_bonded(sys.n_systems, _p(_c(sys.sys_offsets, np.int64)), int(sys.periodic), _p(box),
                     _p(x), _p(y), _p(z), _p(q), ff.bonds.shape[0], _p(ff.bonds),
                     _p(ff.bond_par), ff.angles.shape[0], _p(ff.angles), _p(ff.angle_par),
                     _p(out["fx"]), _p(out["fy"]), _p(out["fz"]), _p(epot))
    out["epot"] = epot
    return out


# ------------------------------------------------------------------ forces

def forces(sys, q=None, kappa=None, x=None, y=None, z=None, per_atom=True, hybrid=None,
           ff=None):
    """Brute-force FP64 forces for all systems of ``sys`` at positions (x, y, z)
    (default: the system's own), charges q and per-system kappa; ``hybrid`` (a
    ``hybrid_table``) switches the Coulomb term to the hybrid potential; ``ff`` (a
    ForceField) adds its LJ scaling and exclusions to the pair loop (its bonded terms
    are separate: ``bonded``).
    Returns dict(fx, fy, fz, e_atom, a_atom, epot, npairs)."""
    x = _c(sys.x if x is None else x, np.float64)
    y = _c(sys.y if y is None else y, np.float64)
    z = _c(sys.z if z is None else z, np.float64)
    q = _c(sys.q if q is None else q, np.int8)
    B = sys.n_systems
    if kappa is None:
        kappa = kappa_from_lambda(sys.lambda_d[:, 0])
    kappa = _c(np.broadcast_to(kappa, (B,)), np.float64)
    n = x.shape[0]
    out = {k: np.empty(n) for k in ("fx", "fy", "fz", "e_atom", "a_atom")}
    epot = np.empty(B)
    box = None if sys.box is None else _c(sys.box, np.float64)
    hyb, n_q = _hyb(hybrid, B, q)
    npairs = lib().orc_forces(B, _p(_c(sys.sys_offsets, np.int64)), int(sys.periodic), _p(box),
                              sys.rc, _p(x), _p(y), _p(z), _p(q),
                              _p(_c(sys.type, np.uint8)), sys.n_types,
                              _p(_c(sys.c6, np.float64)), _p(_c(sys.c12, np.float64)),
                              _p(kappa), int(sys.screen_lj), _p(out["fx"]), _p(out["fy"]),
                              _p(out["fz"]), _p(out["e_atom"]), _p(out["a_atom"]), _p(epot),
                              _p(hyb), n_q, *_ff_args(ff))
    out["epot"] = epot
    out["npairs"] = int(npairs)
    return out


def _hyb(hybrid, B, q):
    if hybrid is None:
        return None, 0
    h = _c(hybrid, np.float64)
    assert h.ndim == 3 and h.shape[0] == B and h.shape[2] == 4
    assert q.size == 0 or (q.min() >= 0 and q.max() < h.shape[1])
    return h, int(h.shape[1])


def forces_rows(sys, rows, q=None, kappa=None, x=None, y=None, z=None, n_threads=0,
                hybrid=None, ff=None):
    """F_i, e_i, A_i of the listed atoms against every atom of their system
    (OpenMP over rows)."""
    x = _c(sys.x if x is None else x, np.float64)
    y = _c(sys.y if y is None else y, np.float64)
    z = _c(sys.z if z is None else z, np.float64)
    q = _c(sys.q if q is None else q, np.int8)
    rows = _c(rows, np.int64)
    offs = _c(sys.sys_offsets, np.int64)
    sys_of_row = np.searchsorted(offs, rows, side="right").astype(np.int64) - 1
    B = sys.n_systems
    if kappa is None:
        kappa = kappa_from_lambda(sys.lambda_d[:, 0])
    kappa = _c(np.broadcast_to(kappa, (B,)), np.float64)
    m = rows.shape[0]
    out = {k: np.empty(m) for k in ("fx", "fy", "fz", "e_atom", "a_atom")}
    out["row_hits"] = np.empty(m, dtype=np.int64)
    box = None if sys.box is None else _c(sys.box, np.float64)
    hyb, n_q = _hyb(hybrid, B, q)
    hits = lib().orc_forces_rows(m, _p(rows), _p(sys_of_row), _p(offs), int(sys.periodic),
                                 _p(box), sys.rc, _p(x), _p(y), _p(z), _p(q),
                                 _p(_c(sys.type, np.uint8)), sys.n_types,
                                 _p(_c(sys.c6, np.float64)), _p(_c(sys.c12, np.float64)),
                                 _p(kappa), int(sys.screen_lj), _p(out["fx"]), _p(out["fy"]),
                                 _p(out["fz"]), _p(out["e_atom"]), _p(out["a_atom"]),
                                 _p(out["row_hits"]), int(n_threads), _p(hyb), n_q,
                                 *_ff_args(ff))
    out["hits"] = int(hits)
    return out


def pairs(sys, x=None, y=None, z=None, max_pairs=None) -> np.ndarray:
    """The pair set S as an int64 array of shape (|S|, 2), i < j, i-major."""
    x = _c(sys.x if x is None else x, np.float64)
    y = _c(sys.y if y is None else y, np.float64)
    z = _c(sys.z if z is None else z, np.float64)
    box = None if sys.box is None else _c(sys.box, np.float64)
    offs = _c(sys.sys_offsets, np.int64)
    cap = max_pairs if max_pairs is not None else 1 << 16
    while True:
        oi = np.empty(cap, dtype=np.int64)
        oj = np.empty(cap, dtype=np.int64)
        cnt = lib().orc_pairs(sys.n_systems, _p(offs), int(sys.periodic), _p(box), sys.rc,
                              _p(x), _p(y), _p(z), _p(oi), _p(oj), cap)
        if cnt <= cap:
            return np.stack([oi[:cnt], oj[:cnt]], axis=1)
        cap = int(cnt)


def pairs_rows(sys, rows, x=None, y=None, z=None, n_threads=0):
    """Partners of the listed atoms: a list with, per row, the ascending int64 array
    of every j != i of its system inside the cutoff (brute force over the system)."""
    x = _c(sys.x if x is None else x, np.float64)
    y = _c(sys.y if y is None else y, np.float64)
    z = _c(sys.z if z is None else z, np.float64)
    rows = _c(rows, np.int64)
    offs = _c(sys.sys_offsets, np.int64)
    sys_of_row = _c(np.searchsorted(offs, rows, side="right") - 1, np.int64)
    box = None if sys.box is None else _c(sys.box, np.float64)
    off = np.zeros(rows.size + 1, dtype=np.int64)
    cap = max(1, 512 * rows.size)
    while True:
        out = np.empty(cap, dtype=np.int64)
        tot = lib().orc_pairs_rows(rows.size, _p(rows), _p(sys_of_row), _p(offs),
                                   int(sys.periodic), _p(box), sys.rc, _p(x), _p(y), _p(z),
                                   _p(off), _p(out), cap, n_threads)
        if tot <= cap:
            return [out[off[r]:off[r + 1]].copy() for r in range(rows.size)]
        cap = int(tot)


def pair_r2(periodic, box, x, y, z, i, j) -> float:
    box = None if box is None else _c(box, np.float64)
    return float(lib().orc_pair_r2(int(periodic), _p(box), _p(_c(x, np.float64)),
                                   _p(_c(y, np.float64)), _p(_c(z, np.float64)), i, j))


# ------------------------------------------------------------------ RDF / S(q)

def rdf_histogram(sys, r_max, n_bins, x=None, y=None, z=None) -> np.ndarray:
    """uint64 [B, E, E, n_bins] pair-distance counts (upper triangle e_a <= e_b)."""
    x = _c(sys.x if x is None else x, np.float64)
    y = _c(sys.y if y is None else y, np.float64)
    z = _c(sys.z if z is None else z, np.float64)
    E = sys.n_elements
    hist = np.zeros((sys.n_systems, E, E, n_bins), dtype=np.uint64)
    box = None if sys.box is None else _c(sys.box, np.float64)
    lib().orc_rdf_histogram(sys.n_systems, _p(_c(sys.sys_offsets, np.int64)), int(sys.periodic),
                            _p(box), _p(x), _p(y), _p(z), _p(_c(sys.elem, np.uint8)), E,
                            float(r_max), int(n_bins), _p(hist))
    return hist


def rdf_normalize(counts, r_max, n_a, n_b, same, volume) -> np.ndarray:
    c = _c(counts, np.uint64)
    g = np.empty(c.size)
    lib().orc_rdf_normalize(c.size, float(r_max), _p(c), int(n_a), int(n_b), int(bool(same)),
                            float(volume), _p(g))
    return g


def structure_factor(g, r_max, rho0, q) -> np.ndarray:
    g = _c(g, np.float64)
    q = _c(np.atleast_1d(q), np.float64)
    S = np.empty(q.size)
    lib().orc_structure_factor(g.size, float(r_max), _p(g), float(rho0), q.size, _p(q), _p(S))
    return S


# ------------------------------------------------------------------ random numbers / charges

def philox4x32_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def ionize(sys, q, step: int, g_step=None) -> int:
    """Apply ionization step ``step`` (>= 1) to ``q`` in place; returns the jump count."""
    assert q.dtype == np.int8 and q.flags.c_contiguous
    if g_step is None:
        g_step = sys.g[:, step]
    g_step = _c(g_step, np.float64)
    return int(lib().orc_ionize(sys.n_systems, _p(_c(sys.sys_offsets, np.int64)),
                                _p(_c(sys.elem, np.uint8)), _p(_c(sys.atom_id, np.uint32)),
                                _p(q), _p(_c(sys.qmax, np.int8)), sys.base.shape[1],
                                _p(_c(sys.base, np.float64)), _p(g_step),
                                _p(_c(sys.seeds, np.uint64)), int(step)))


# ------------------------------------------------------------------ integrator

def vv(phase, dt, inv_mass, f, pos, vel):
    """In-place velocity-Verlet phase on (pos, vel) tuples of float64 arrays."""
    fx, fy, fz = (_c(a, np.float64) for a in f)
    for a in (*pos, *vel):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_vv(pos[0].shape[0], int(phase), float(dt), _p(_c(inv_mass, np.float64)),
                 _p(fx), _p(fy), _p(fz), _p(pos[0]), _p(pos[1]), _p(pos[2]), _p(vel[0]),
                 _p(vel[1]), _p(vel[2]))


def langevin_normals(atom_id, step, system, seed) -> np.ndarray:
    out = np.empty(3)
    lib().orc_langevin_normals(int(atom_id), int(step), int(system), int(seed), _p(out))
    return out


def langevin_c1(gamma, dt) -> np.ndarray:
    """c1 = exp(-gamma dt) per (system, element), with the C library's exp."""
    g = np.asarray(gamma, dtype=np.float64)
    return np.array([math.exp(-v * dt) for v in g.reshape(-1)]).reshape(g.shape)


def vv_langevin(sys, step, c1, kt, f, pos, vel):
    """Phase 0 with the Langevin coupling (in place); c1 [B, E], kt [B, S+1] in kJ/mol."""
    fx, fy, fz = (_c(a, np.float64) for a in f)
    for a in (*pos, *vel):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    c1 = _c(c1, np.float64)
    kt = _c(kt, np.float64)
    lib().orc_vv_langevin(sys.n_systems, _p(_c(sys.sys_offsets, np.int64)),
                          _p(_c(sys.elem, np.uint8)), int(c1.shape[1]),
                          _p(_c(sys.atom_id, np.uint32)), _p(c1), _p(kt), int(kt.shape[1]),
                          int(step), _p(_c(sys.seeds, np.uint64)), float(sys.dt),
                          _p(_c(sys.inv_mass, np.float64)), _p(fx), _p(fy), _p(fz), _p(pos[0]),
                          _p(pos[1]), _p(pos[2]), _p(vel[0]), _p(vel[1]), _p(vel[2]))


def ekin(sys, vx, vy, vz) -> np.ndarray:
    out = np.empty(sys.n_systems)
    lib().orc_ekin(sys.n_systems, _p(_c(sys.sys_offsets, np.int64)),
                   _p(_c(sys.inv_mass, np.float64)), _p(_c(vx, np.float64)),
                   _p(_c(vy, np.float64)), _p(_c(vz, np.float64)), _p(out))
    return out


def run(sys, n_steps, record_every=1, ionize_on=True):
    """Reference trajectory: F0 = F(x0, q0, kappa[0]); then for s = 1..n_steps:
    v += h F; x += dt v; ionize(s); F = F(x, q, kappa[s]); v += h F.
    Returns dict with final state and per-recorded-step charges, E_pot, E_kin."""
    x, y, z = sys.x.copy(), sys.y.copy(), sys.z.copy()
    vx, vy, vz = sys.vx.copy(), sys.vy.copy(), sys.vz.copy()
    q = sys.q.copy()
    kap = kappa_from_lambda(sys.lambda_d)
    F = forces(sys, q=q, kappa=kap[:, 0], x=x, y=y, z=z)
    rec = {"q": [q.copy()], "epot": [F["epot"].copy()], "ekin": [ekin(sys, vx, vy, vz)]}
    for s in range(1, n_steps + 1):
        vv(0, sys.dt, sys.inv_mass, (F["fx"], F["fy"], F["fz"]), (x, y, z), (vx, vy, vz))
        if ionize_on:
            ionize(sys, q, s)
        F = forces(sys, q=q, kappa=kap[:, s], x=x, y=y, z=z)
        vv(1, sys.dt, sys.inv_mass, (F["fx"], F["fy"], F["fz"]), (x, y, z), (vx, vy, vz))
        if s % record_every == 0:
            rec["q"].append(q.copy())
            rec["epot"].append(F["epot"].copy())
            rec["ekin"].append(ekin(sys, vx, vy, vz))
    return {"x": x, "y": y, "z": z, "vx": vx, "vy": vy, "vz": vz, "q": q, "F": F, **rec}
