"""Seeded synthetic inputs for the screened-force + ionization step.

This module only *generates inputs*: atom positions, velocities, elements,
masses, Lennard-Jones parameter tables, per-step Debye-length and pulse
envelope schedules, per-(element, charge) ionization-probability scales and
per-system seeds.  It contains none of the method's arithmetic (no pair
predicate, no force, no ionization rule, no integrator), so both the GPU path
and the CPU oracle can consume exactly the same arrays.

The paper's own samples (PDB water and lysozyme structures, a 45,000-atom
methane cluster prepared with GROMACS, CR outputs from Cretin) are not
available; the systems below stand in for their *shape*: element mix, number
density, box size, cutoff, screening length and pulse (paper section II.D,
sample descriptions; section IV.A, methane cluster).

Units are GROMACS units throughout: nm, ps, amu, kJ/mol, elementary charge.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# CODATA-2018 derived constants in GROMACS units.
K_E = 138.935457644382          # 1/(4 pi eps0), kJ mol^-1 nm e^-2
K_B = 0.00831446261815324       # Boltzmann constant, kJ mol^-1 K^-1
AVOGADRO = 6.02214076e23

MASS = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999, "S": 32.06}
Z_NUCLEAR = {"H": 1, "C": 6, "N": 7, "O": 8, "S": 16}

BASE_SEED = 2401031800

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 finalizer (Steele, Lea, Flood 2014); used to derive seeds."""
    x = (x + 0x9E3779B97F4A7C15) & MASK64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


@dataclasses.dataclass
class System:
    """One batch of B independent systems, concatenated in caller order.

    Per-atom arrays are structure-of-arrays in the caller's atom order.
    ``atom_id`` is the atom's local index inside its system; it keys the
    counter-based random stream of the ionization update.
    """
    name: str
    x: np.ndarray            # float64 [N]
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    elem: np.ndarray         # uint8 [N]  ionizable element index
    type: np.ndarray         # uint8 [N]  Lennard-Jones type index
    atom_id: np.ndarray      # uint32 [N] local index within its system
    inv_mass: np.ndarray     # float64 [N]
    q: np.ndarray            # int8 [N] integer charges (start neutral)
    sys_offsets: np.ndarray  # int64 [B+1]
    periodic: bool
    box: Optional[np.ndarray]  # float64 [B,3] (periodic) else None
    rc: float
    skin: float
    dt: float
    n_steps: int
    lambda_d: np.ndarray     # float64 [B, S+1] Debye length per force evaluation (inf = unscreened)
    g: np.ndarray            # float64 [B, S+1] pulse envelope per ionization step (index 0 unused)
    base: np.ndarray         # float64 [E, Q] per-(element, charge) per-step probability scale
    qmax: np.ndarray         # int8 [E] highest reachable charge per element
    c6: np.ndarray           # float64 [T, T]
    c12: np.ndarray          # float64 [T, T]
    seeds: np.ndarray        # uint64 [B]
    screen_lj: bool = True
    elements: tuple = ()
    description: str = ""

    @property
    def n_atoms(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_systems(self) -> int:
        return int(self.sys_offsets.shape[0] - 1)

    @property
    def n_types(self) -> int:
        return int(self.c6.shape[0])

    @property
    def n_elements(self) -> int:
        return int(self.qmax.shape[0])

    def positions(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def copy(self) -> "System":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = v.copy() if isinstance(v, np.ndarray) else v
        return System(**kw)

    def subsystem(self, b: int) -> "System":
        """System b alone (its atoms, schedules and seed), as a batch of one."""
        a0, a1 = int(self.sys_offsets[b]), int(self.sys_offsets[b + 1])
        out = self.copy()
        for name in ("x", "y", "z", "vx", "vy", "vz", "elem", "type", "atom_id", "inv_mass",
                     "q"):
            setattr(out, name, getattr(self, name)[a0:a1].copy())
        out.sys_offsets = np.array([0, a1 - a0], np.int64)
        out.lambda_d = self.lambda_d[b:b + 1].copy()
        out.g = self.g[b:b + 1].copy()
        out.seeds = self.seeds[b:b + 1].copy()
        if self.box is not None:
            out.box = self.box[b:b + 1].copy()
        return out

    def mass_density_g_cm3(self) -> float:
        """Mass density of system 0 (periodic only)."""
        assert self.box is not None
        n0, n1 = int(self.sys_offsets[0]), int(self.sys_offsets[1])
        m = np.sum(1.0 / self.inv_mass[n0:n1])  # amu
        vol_cm3 = float(np.prod(self.box[0])) * 1e-21
        return m / AVOGADRO / vol_cm3


# --------------------------------------------------------------------------
# Geometry helpers
# --------------------------------------------------------------------------

def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed rotation matrices from unit quaternions (Shoemake)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    qw = a * np.sin(2 * np.pi * u2)
    qx = a * np.cos(2 * np.pi * u2)
    qy = b * np.sin(2 * np.pi * u3)
    qz = b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    R[:, 0, 1] = 2 * (qx * qy - qz * qw)
    R[:, 0, 2] = 2 * (qx * qz + qy * qw)
    R[:, 1, 0] = 2 * (qx * qy + qz * qw)
    R[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    R[:, 1, 2] = 2 * (qy * qz - qx * qw)
    R[:, 2, 0] = 2 * (qx * qz - qy * qw)
    R[:, 2, 1] = 2 * (qy * qz + qx * qw)
    R[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    return R


def water_template() -> np.ndarray:
    """Rigid H2O: O at origin, O-H 0.1 nm, HOH angle 109.47 degrees. Rows O, H, H."""
    half = math.radians(109.47) / 2.0
    b = 0.1
    return np.array([[0.0, 0.0, 0.0],
                     [b * math.sin(half), 0.0, b * math.cos(half)],
                     [-b * math.sin(half), 0.0, b * math.cos(half)]])


def methane_template() -> np.ndarray:
    """Rigid CH4: C at origin, tetrahedral C-H 0.109 nm. Rows C, H, H, H, H."""
    s = 0.109 / math.sqrt(3.0)
    return np.array([[0, 0, 0], [s, s, s], [s, -s, -s], [-s, s, -s], [-s, -s, s]], dtype=np.float64)


def lattice_sites(n_per_dim: int, spacing: float, offset: float = 0.0) -> np.ndarray:
    g = (np.arange(n_per_dim) + 0.5) * spacing + offset
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def place_molecules(rng, centers: np.ndarray, template: np.ndarray) -> np.ndarray:
    R = random_rotations(rng, centers.shape[0])
    atoms = np.einsum("nij,aj->nai", R, template) + centers[:, None, :]
    return atoms.reshape(-1, 3)


def maxwell_velocities(rng, masses: np.ndarray, temperature: float,
                       sys_offsets: np.ndarray) -> np.ndarray:
    """Maxwell-Boltzmann velocities (nm/ps), COM momentum removed per system."""
    sigma = np.sqrt(K_B * temperature / masses)
    v = rng.standard_normal((masses.shape[0], 3)) * sigma[:, None]
    for b in range(sys_offsets.shape[0] - 1):
        a0, a1 = int(sys_offsets[b]), int(sys_offsets[b + 1])
        m = masses[a0:a1, None]
        v[a0:a1] -= (m * v[a0:a1]).sum(0) / m.sum()
    return v


def lj_tables_lorentz_berthelot(sigma, eps):
    """c6 = 4 eps sigma^6, c12 = 4 eps sigma^12 with Lorentz-Berthelot mixing.

    These are force-field *input* parameters (synthetic, not from any published
    force field); the pair potential that uses them lives elsewhere.
    """
    s = np.asarray(sigma, dtype=np.float64)
    e = np.asarray(eps, dtype=np.float64)
    sij = 0.5 * (s[:, None] + s[None, :])
    eij = np.sqrt(e[:, None] * e[None, :])
    return 4.0 * eij * sij ** 6, 4.0 * eij * sij ** 12


def gaussian_envelope(t: np.ndarray, t0: float, fwhm: float) -> np.ndarray:
    """Synthetic stand-in for the CR-driven ionization time profile: a unit-peak
    Gaussian pulse of the given FWHM (the paper models the X-ray pulse as
    Gaussian, section II.C)."""
    return np.exp(-4.0 * math.log(2.0) * (t - t0) ** 2 / (fwhm * fwhm))


def _finish(name, pos, vel, elem, typ, masses, sys_offsets, periodic, box, rc, skin, dt,
            n_steps, lambda_d, g, base, qmax, c6, c12, seed, elements, description,
            screen_lj=True) -> System:
    n = pos.shape[0]
    B = sys_offsets.shape[0] - 1
    atom_id = np.empty(n, dtype=np.uint32)
    for b in range(B):
        a0, a1 = int(sys_offsets[b]), int(sys_offsets[b + 1])
        atom_id[a0:a1] = np.arange(a1 - a0, dtype=np.uint32)
    seeds = np.array([splitmix64(seed + b) for b in range(B)], dtype=np.uint64)
    return System(
        name=name,
        x=np.ascontiguousarray(pos[:, 0]), y=np.ascontiguousarray(pos[:, 1]),
        z=np.ascontiguousarray(pos[:, 2]),
        vx=np.ascontiguousarray(vel[:, 0]), vy=np.ascontiguousarray(vel[:, 1]),
        vz=np.ascontiguousarray(vel[:, 2]),
        elem=elem.astype(np.uint8), type=typ.astype(np.uint8), atom_id=atom_id,
        inv_mass=1.0 / masses, q=np.zeros(n, dtype=np.int8),
        sys_offsets=sys_offsets.astype(np.int64), periodic=periodic,
        box=None if box is None else np.asarray(box, dtype=np.float64).reshape(B, 3),
        rc=float(rc), skin=float(skin), dt=float(dt), n_steps=int(n_steps),
        lambda_d=np.ascontiguousarray(lambda_d, dtype=np.float64),
        g=np.ascontiguousarray(g, dtype=np.float64),
        base=np.ascontiguousarray(base, dtype=np.float64),
        qmax=np.asarray(qmax, dtype=np.int8), c6=np.ascontiguousarray(c6),
        c12=np.ascontiguousarray(c12), seeds=seeds, screen_lj=screen_lj,
        elements=tuple(elements), description=description)


def _base_table(qmax, p):
    """Per-step probability scale base[e][q] = p_e for q < qmax[e], else 0."""
    Q = int(max(qmax)) + 1
    base = np.zeros((len(qmax), Q))
    for e, qm in enumerate(qmax):
        base[e, :qm] = p[e] if np.ndim(p) else p
    return base


# --------------------------------------------------------------------------
# Water (bulk, periodic): small parity case, 98k-atom pulse case, 4.2M-atom case
# --------------------------------------------------------------------------

WATER_SIGMA_OO = 0.3166
WATER_EPS_OO = 0.65


def _water_lj():
    c6 = np.zeros((2, 2))
    c12 = np.zeros((2, 2))
    c6[0, 0] = 4.0 * WATER_EPS_OO * WATER_SIGMA_OO ** 6
    c12[0, 0] = 4.0 * WATER_EPS_OO * WATER_SIGMA_OO ** 12
    return c6, c12


def water_box(n_per_dim: int, L: float, seed: int, jitter: float = 0.02,
              drop: int = 0, extra_lone_o: bool = False, temperature: float = 300.0):
    """Bulk water on a jittered cubic lattice, random rigid orientations.

    Atom order is molecule-major (O, H, H per molecule) in lattice order.
    ``drop`` random lattice sites are left empty; ``extra_lone_o`` places one
    oxygen atom at the first dropped site (used to make the 4.2M-atom box whole).
    """
    rng = np.random.default_rng(seed)
    spacing = L / n_per_dim
    sites = lattice_sites(n_per_dim, spacing)
    lone = None
    if drop:
        idx = rng.permutation(sites.shape[0])[:drop]
        keep = np.ones(sites.shape[0], dtype=bool)
        keep[idx] = False
        if extra_lone_o:
            lone = sites[idx[0]].copy()
        sites = sites[keep]
    sites = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    pos = place_molecules(rng, sites, water_template())
    nmol = sites.shape[0]
    elem = np.tile(np.array([0, 1, 1], dtype=np.uint8), nmol)
    if lone is not None:
        pos = np.concatenate([pos, lone[None, :]], axis=0)
        elem = np.concatenate([elem, np.array([0], dtype=np.uint8)])
    masses = np.where(elem == 0, MASS["O"], MASS["H"])
    offs = np.array([0, pos.shape[0]], dtype=np.int64)
    vel = maxwell_velocities(rng, masses, temperature, offs)
    return pos, vel, elem, masses, offs


def water_small(n_steps: int = 200) -> System:
    """512 rigid-geometry H2O (1,536 atoms), 2.48 nm periodic cube, lambda_D 0.3 nm,
    rc 1.0 nm, dt 0.1 fs, per-step ionization probability 1e-3 (O up to +8, H up to +1)."""
    seed = BASE_SEED + 0
    L = 2.48
    pos, vel, elem, masses, offs = water_box(8, L, seed)
    S = n_steps
    c6, c12 = _water_lj()
    qmax = [8, 1]
    return _finish("water_1536", pos, vel, elem, elem.copy(), masses, offs, True,
                   [[L, L, L]], 1.0, 0.1, 1e-4, S,
                   np.full((1, S + 1), 0.3), np.ones((1, S + 1)), _base_table(qmax, 1e-3),
                   qmax, c6, c12, seed, ("O", "H"),
                   "bulk water, 512 H2O, 2.48 nm periodic cube")


def water_pulse(n_steps: int = 1000, dt_fs: float = 0.1) -> System:
    """32,768 H2O (98,304 atoms), 9.93 nm periodic cube, lambda_D linear 1.0 -> 0.15 nm over
    the first 100 fs, Gaussian pulse FWHM 10 fs centred at 50 fs with peak ionization
    probability 5e-3 per 0.1 fs, rc 1.0 nm, dt 0.1 fs (1,000 steps to the end of the ramp).

    dt_fs: another time step with the same schedule in time (the ramp ends after
    round(100 / dt_fs) steps, the per-step probability scales with the step); the
    default reproduces the 0.1 fs tables exactly."""
    seed = BASE_SEED + 1
    L = 9.93
    pos, vel, elem, masses, offs = water_box(32, L, seed)
    S = n_steps
    dt = dt_fs * 1e-3
    k_ramp = float(round(100.0 / dt_fs))
    k = np.arange(S + 1, dtype=np.float64)
    lam = 1.0 - 0.85 * np.minimum(k, k_ramp) / k_ramp
    t_fs = k * dt * 1000.0
    g = gaussian_envelope(t_fs, 50.0, 10.0)
    c6, c12 = _water_lj()
    qmax = [8, 1]
    return _finish("water_98304", pos, vel, elem, elem.copy(), masses, offs, True,
                   [[L, L, L]], 1.0, 0.1, dt, S, lam[None, :], g[None, :],
                   _base_table(qmax, 5e-3 * (dt_fs / 0.1)), qmax, c6, c12, seed, ("O", "H"),
                   "bulk water, 32,768 H2O, 9.93 nm periodic cube, pulse-driven screening")


def water_large(n_steps: int = 100, n_per_dim: int = 112, L: float = 34.8) -> System:
    """1,398,101 H2O plus one lone O (4,194,304 atoms), 34.8 nm periodic cube,
    lambda_D 0.2 nm, rc 1.0 nm, dt 0.1 fs, per-step probability 1e-3."""
    seed = BASE_SEED + 4
    n_sites = n_per_dim ** 3
    target_mol = 1398101 if n_per_dim == 112 else int(n_sites * 0.995)
    drop = n_sites - target_mol
    pos, vel, elem, masses, offs = water_box(n_per_dim, L, seed, drop=drop, extra_lone_o=True)
    S = n_steps
    c6, c12 = _water_lj()
    qmax = [8, 1]
    return _finish("water_4194304", pos, vel, elem, elem.copy(), masses, offs, True,
                   [[L, L, L]], 1.0, 0.1, 1e-4, S, np.full((1, S + 1), 0.2),
                   np.ones((1, S + 1)), _base_table(qmax, 1e-3), qmax, c6, c12, seed,
                   ("O", "H"), "bulk water, 4.19M atoms, 34.8 nm periodic cube")


# --------------------------------------------------------------------------
# Protein-crystal-like solid
# --------------------------------------------------------------------------

PROTEIN_ELEMENTS = ("H", "C", "N", "O", "S")
PROTEIN_COUNTS = (262144, 162529, 41943, 52429, 5243)       # sums to 524,288
PROTEIN_SIGMA = (0.11, 0.34, 0.33, 0.30, 0.36)                 # synthetic
PROTEIN_EPS = (0.10, 0.40, 0.70, 0.80, 1.00)                   # synthetic


def protein_crystal(n_steps: int = 500, scale: int = 1) -> System:
    """524,288 atoms, element mix H/C/N/O/S, 81^3 jittered cubic lattice with random
    vacancies in a 17 nm periodic cube, per-element LJ (Lorentz-Berthelot), charges up
    to Z, lambda_D 0.25 nm, rc 1.2 nm, dt 0.05 fs.  ``scale`` > 1 shrinks the box
    linearly by that factor (same density) for small test cases."""
    seed = BASE_SEED + 2
    rng = np.random.default_rng(seed)
    n_dim = 81 // scale
    L = 17.0 * n_dim / 81.0
    counts = np.array(PROTEIN_COUNTS) if scale == 1 else np.maximum(
        (np.array(PROTEIN_COUNTS) * (n_dim ** 3 * 0.9864) / 524288).astype(int), 1)
    n = int(counts.sum())
    sites = lattice_sites(n_dim, L / n_dim)
    keep = rng.permutation(sites.shape[0])[:n]
    keep.sort()
    pos = sites[keep] + rng.uniform(-0.02, 0.02, size=(n, 3))
    elem = np.repeat(np.arange(5, dtype=np.uint8), counts)
    elem = elem[rng.permutation(n)]
    masses = np.array([MASS[e] for e in PROTEIN_ELEMENTS])[elem]
    offs = np.array([0, n], dtype=np.int64)
    vel = maxwell_velocities(rng, masses, 300.0, offs)
    c6, c12 = lj_tables_lorentz_berthelot(PROTEIN_SIGMA, PROTEIN_EPS)
    qmax = [Z_NUCLEAR[e] for e in PROTEIN_ELEMENTS]
    S = n_steps
    return _finish("protein_%d" % n, pos, vel, elem, elem.copy(), masses, offs, True,
                   [[L, L, L]], 1.2, 0.1, 5e-5, S, np.full((1, S + 1), 0.25),
                   np.ones((1, S + 1)), _base_table(qmax, 1e-3), qmax, c6, c12, seed,
                   PROTEIN_ELEMENTS, "protein-crystal-like solid, %.2f nm periodic cube" % L)


# --------------------------------------------------------------------------
# Batched vacuum methane clusters
# --------------------------------------------------------------------------

METHANE_SPACING = 0.399   # nm, 0.42 g/cm^3 of CH4


def methane_clusters(n_clusters: int = 256, n_steps: int = 2000, lo: int = 1000,
                     hi: int = 20000, seed_offset: int = 3) -> System:
    """Non-periodic spherical CH4 clusters, atom counts log-uniform in [lo, hi]
    (rounded down to whole molecules), each with its own seed, pulse peak
    probability (log-uniform in [1e-3, 1e-2]) and Debye-length ramp 0.8 -> 0.1 nm
    over 2,000 steps; Gaussian FWHM 15 fs centred at 30 fs; rc 1.0 nm, dt 0.05 fs;
    Lennard-Jones C-C only."""
    seed = BASE_SEED + seed_offset
    rng = np.random.default_rng(seed)
    n_b = 5 * np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n_clusters)) / 5).astype(int)
    n_b = np.maximum(n_b, 5)
    tmpl = methane_template()
    all_pos, all_elem = [], []
    for b in range(n_clusters):
        nm = n_b[b] // 5
        nd = int(math.ceil((nm * 6 / math.pi) ** (1 / 3))) + 3
        sites = lattice_sites(nd, METHANE_SPACING, -nd * METHANE_SPACING / 2)
        sites = sites + rng.uniform(-0.03, 0.03, size=sites.shape)
        r = np.linalg.norm(sites, axis=1)
        order = np.argsort(r, kind="stable")[:nm]
        centers = sites[np.sort(order)]
        all_pos.append(place_molecules(rng, centers, tmpl))
        all_elem.append(np.tile(np.array([0, 1, 1, 1, 1], dtype=np.uint8), nm))
    pos = np.concatenate(all_pos)
    elem = np.concatenate(all_elem)
    offs = np.concatenate([[0], np.cumsum(n_b)]).astype(np.int64)
    masses = np.where(elem == 0, MASS["C"], MASS["H"])
    vel = maxwell_velocities(rng, masses, 300.0, offs)
    S = n_steps
    dt = 5e-5
    k = np.arange(S + 1, dtype=np.float64)
    lam = 0.8 - 0.7 * np.minimum(k, 2000.0) / 2000.0
    t_fs = k * dt * 1000.0
    g = gaussian_envelope(t_fs, 30.0, 15.0)
    peak = np.exp(rng.uniform(math.log(1e-3), math.log(1e-2), n_clusters))
    # per-cluster fluence is folded into the envelope so that base[] stays per element
    g_b = peak[:, None] * g[None, :]
    lam_b = np.repeat(lam[None, :], n_clusters, axis=0)
    # Lennard-Jones between C atoms only: this path has no bonded terms and no
    # exclusions, so an H-C or H-H term would push the atoms of every molecule apart
    # in the first step (C-H 0.109 nm against sigma 0.295 nm); the water boxes keep
    # their LJ on O-O for the same reason
    c6, c12 = lj_tables_lorentz_berthelot((0.34, 0.25), (0.40, 0.10))
    c6[1, :] = c6[:, 1] = 0.0
    c12[1, :] = c12[:, 1] = 0.0
    qmax = [6, 1]
    return _finish("methane_%dx" % n_clusters, pos, vel, elem, elem.copy(), masses, offs,
                   False, None, 1.0, 0.1, dt, S, lam_b, g_b, _base_table(qmax, 1.0), qmax,
                   c6, c12, seed, ("C", "H"),
                   "%d vacuum CH4 clusters, %d atoms" % (n_clusters, pos.shape[0]))


def molecular_force_field(sys: System, kind: str):
    """Synthetic bonded topology and parameters for the molecules of a water or
    methane workload (atoms of one molecule are consecutive: O H H or C H H H H):
    Morse bonds to the heavy atom, harmonic H-X-H angles, LJ exclusions for the 1-2
    and 1-3 pairs they define, Lennard-Jones tables for every element pair
    (Lorentz-Berthelot), and Z and the neutral LJ radius sigma per type for the
    charge scaling of the LJ radii.  Returns a dict of numpy arrays (global atom
    indices)."""
    if kind == "water":
        per, nh, Z = 3, 2, (8, 1)
        sig, eps = (0.3166, 0.10), (0.65, 0.02)
        bond = (450.0, 22.0, 0.1)                         # D_e kJ/mol, beta 1/nm, b_e nm
        ang = (380.0, math.radians(109.47))               # k kJ/mol/rad^2, theta0
    elif kind == "methane":
        per, nh, Z = 5, 4, (6, 1)
        sig, eps = (0.34, 0.25), (0.40, 0.10)
        bond = (430.0, 18.0, 0.109)
        ang = (330.0, math.acos(-1.0 / 3.0))
    else:
        raise ValueError(kind)
    n = sys.n_atoms
    assert n % per == 0
    heavy = np.arange(0, n, per)
    bonds = np.stack([np.repeat(heavy, nh),
                      (heavy[:, None] + 1 + np.arange(nh)[None, :]).ravel()], 1)
    pairs = [(a, b) for a in range(nh) for b in range(a + 1, nh)]
    angles = np.array([(h + 1 + a, h, h + 1 + b) for h in heavy for a, b in pairs])
    c6, c12 = lj_tables_lorentz_berthelot(sig, eps)
    excl = np.concatenate([bonds, angles[:, [0, 2]]])
    return {"bonds": bonds.astype(np.int32),
            "bond_par": np.tile(np.array(bond), (bonds.shape[0], 1)),
            "angles": angles.astype(np.int32),
            "angle_par": np.tile(np.array(ang), (angles.shape[0], 1)),
            "excl": excl.astype(np.int64), "c6": c6, "c12": c12,
            "z": np.array(Z, dtype=np.int8), "sigma": np.array(sig, dtype=np.float64)}


EV_KJ_PER_MOL = 96.48533212      # 1 eV per particle in kJ/mol


def electron_temperature_ev(sys: System, te0_ev: float = 0.0259,
                            te_peak_ev: float = 30.0) -> np.ndarray:
    """Synthetic T_e [B, S+1] in eV (the paper takes it from the CR code): rising from
    te0 (300 K) to te_peak with the running integral of each system's pulse envelope."""
    cum = np.cumsum(sys.g, axis=1)
    frac = cum / np.maximum(cum[:, -1:], 1e-300)
    return te0_ev + (te_peak_ev - te0_ev) * frac


def langevin_inputs(sys: System, gamma_ps=None, te0_ev: float = 0.0259,
                    te_peak_ev: float = 30.0):
    """Synthetic electron-ion coupling inputs: gamma [B, E] in ps^-1, one constant
    value per element (default 2 ps^-1 for the first element, 5 ps^-1 for the rest:
    equilibration over hundreds of fs), and k_B T_e [B, S+1] in kJ/mol from
    electron_temperature_ev."""
    E = sys.n_elements
    if gamma_ps is None:
        gamma_ps = [2.0 if e == 0 else 5.0 for e in range(E)]
    gamma = np.tile(np.asarray(gamma_ps, dtype=np.float64)[None, :E], (sys.n_systems, 1))
    te = electron_temperature_ev(sys, te0_ev, te_peak_ev)
    return np.ascontiguousarray(gamma), np.ascontiguousarray(te * EV_KJ_PER_MOL)


EPS0_SI = 8.8541878128e-12        # F/m
E_CHARGE_SI = 1.602176634e-19     # C


def hybrid_inputs(sys: System, te0_ev: float = 0.0259, te_peak_ev: float = 30.0) -> np.ndarray:
    """Synthetic free-electron density n_e [B, S+1] in nm^-3, consistent with the
    system's Debye-length schedule through Eq. 3 at the temperature of
    electron_temperature_ev: n_e = eps0 k_B T_e / (e^2 lambda_D^2).  Unscreened steps
    (lambda_D = inf) get n_e = 1 nm^-3 (unused there)."""
    te = electron_temperature_ev(sys, te0_ev, te_peak_ev)
    lam_m = sys.lambda_d * 1e-9
    with np.errstate(divide="ignore", invalid="ignore"):
        ne_m3 = EPS0_SI * te / (E_CHARGE_SI * lam_m ** 2)
    ne = np.where(np.isfinite(sys.lambda_d), ne_m3 * 1e-27, 1.0)
    return np.ascontiguousarray(ne)


CONFIGS = {
    "water_1536": water_small,
    "water_98304": water_pulse,
    "protein_524288": protein_crystal,
    "methane_256": methane_clusters,
    "water_4194304": water_large,
}
