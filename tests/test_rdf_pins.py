"""Pins of the oracle's pair-distance histograms, g(r) and partial structure factors
(section II.C, Eq. 18): exact shell counts of perfect lattices, an independent k-d
tree count, the ideal gas, and the closed-form structure factor of a step-function
g (CPU only)."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_2401_03180_amd import synth


def lattice_system(a, n, elem_fn=None, jitter=0.0, seed=0, periodic=True):
    """n^3 simple-cubic sites of spacing a in a periodic cube of side n a."""
    g = np.arange(n) * a
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    idx = np.stack(np.meshgrid(*(np.arange(n),) * 3, indexing="ij"), -1).reshape(-1, 3)
    if jitter:
        p = p + np.random.default_rng(seed).uniform(-jitter, jitter, p.shape)
    N = p.shape[0]
    elem = (np.zeros(N, np.uint8) if elem_fn is None else elem_fn(idx).astype(np.uint8))
    E = int(elem.max()) + 1
    L = n * a
    return synth.System(
        name="lattice", x=p[:, 0].copy(), y=p[:, 1].copy(), z=p[:, 2].copy(),
        vx=np.zeros(N), vy=np.zeros(N), vz=np.zeros(N), elem=elem, type=elem.copy(),
        atom_id=np.arange(N, dtype=np.uint32), inv_mass=np.ones(N), q=np.zeros(N, np.int8),
        sys_offsets=np.array([0, N], dtype=np.int64), periodic=periodic,
        box=np.array([[L, L, L]]) if periodic else None, rc=1.0, skin=0.1, dt=1e-4,
        n_steps=1, lambda_d=np.full((1, 2), 0.3), g=np.ones((1, 2)),
        base=np.zeros((E, 2)), qmax=np.zeros(E, np.int8), c6=np.zeros((E, E)),
        c12=np.zeros((E, E)), seeds=np.array([1], np.uint64), screen_lj=True)


def test_simple_cubic_shell_counts():
    """Coordination shells of a simple-cubic lattice: 6, 12, 8, 6, 24, 24 neighbours at
    a, a sqrt2, a sqrt3, 2a, a sqrt5, a sqrt6 -> N z / 2 pairs in the shell's bin."""
    a, n = 0.3137, 7
    s = lattice_system(a, n)
    N = s.n_atoms
    r_max, nb = 0.8, 160
    h = oracle.rdf_histogram(s, r_max, nb)[0, 0, 0]
    dr = r_max / nb
    shells = {1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24}
    expect = np.zeros(nb, dtype=np.uint64)
    for m, zc in shells.items():
        expect[int(a * math.sqrt(m) / dr)] += N * zc // 2
    assert np.array_equal(h, expect)


def test_rock_salt_partial_counts():
    """Two elements alternating on the cubic sites: nearest neighbours are all unlike
    pairs, the second shell (a sqrt2) all like pairs, the third unlike again."""
    a, n = 0.2817, 6
    s = lattice_system(a, n, elem_fn=lambda i: i.sum(axis=1) % 2)
    N = s.n_atoms
    r_max, nb = 0.55, 110
    h = oracle.rdf_histogram(s, r_max, nb)[0]
    dr = r_max / nb
    k1, k2, k3 = (int(a * math.sqrt(m) / dr) for m in (1, 2, 3))
    assert h[0, 1, k1] == N * 6 // 2 and h[0, 0, k1] == 0 and h[1, 1, k1] == 0
    assert h[0, 0, k2] == (N // 2) * 12 // 2 and h[1, 1, k2] == (N // 2) * 12 // 2
    assert h[0, 1, k2] == 0
    assert h[0, 1, k3] == N * 8 // 2
    assert h[1, 0].sum() == 0                       # only the upper triangle is used


def test_histogram_matches_kdtree():
    """A jittered two-element lattice: the histogram equals binned k-d tree distances."""
    a, n = 0.25, 8
    s = lattice_system(a, n, elem_fn=lambda i: (i[:, 0] * 7 + i[:, 1] * 3 + i[:, 2]) % 3,
                       jitter=0.08, seed=5)
    r_max, nb = 0.9, 90
    h = oracle.rdf_histogram(s, r_max, nb)[0]
    L = n * a
    pts = np.stack([s.x % L, s.y % L, s.z % L], 1)
    t = cKDTree(pts, boxsize=L)
    pairs = t.query_pairs(r_max, output_type="ndarray")
    d = pts[pairs[:, 0]] - pts[pairs[:, 1]]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(1))
    ea = np.minimum(s.elem[pairs[:, 0]], s.elem[pairs[:, 1]])
    eb = np.maximum(s.elem[pairs[:, 0]], s.elem[pairs[:, 1]])
    for p in range(3):
        for q in range(p, 3):
            sel = (ea == p) & (eb == q) & (r < r_max)
            ref, _ = np.histogram(r[sel], bins=nb, range=(0.0, r_max))
            assert np.array_equal(h[p, q], ref.astype(np.uint64)), (p, q)


def test_ideal_gas_gives_unit_g():
    rng = np.random.default_rng(3)
    N, L = 6000, 4.0
    s = lattice_system(1.0, 2)
    p = rng.uniform(0, L, (N, 3))
    s2 = synth.System(**{**s.__dict__, "x": p[:, 0].copy(), "y": p[:, 1].copy(),
                         "z": p[:, 2].copy(), "elem": (np.arange(N) % 2).astype(np.uint8),
                         "sys_offsets": np.array([0, N], dtype=np.int64),
                         "box": np.array([[L, L, L]]), "base": np.zeros((2, 2)),
                         "qmax": np.zeros(2, np.int8), "c6": np.zeros((2, 2)),
                         "c12": np.zeros((2, 2))})
    r_max, nb = 1.5, 30
    h = oracle.rdf_histogram(s2, r_max, nb, x=p[:, 0], y=p[:, 1], z=p[:, 2])[0]
    na = nb_ = N // 2
    for (a, b, same) in ((0, 0, True), (0, 1, False), (1, 1, True)):
        g = oracle.rdf_normalize(h[a, b], r_max, na, nb_, same, L ** 3)
        expect = oracle.rdf_normalize(np.ones(nb, np.uint64), r_max, na, nb_, same, L ** 3)
        sig = np.sqrt(1.0 / np.maximum(h[a, b].astype(float), 1.0))
        ok = slice(6, None)                       # shells with enough pairs
        assert np.all(np.abs(g[ok] - 1.0) < 5 * sig[ok] + 1e-12), (a, b)
        assert expect[5] > 0


@pytest.mark.parametrize("sigma,rho", [(0.3, 30.0), (0.28, 33.4)])
def test_step_function_structure_factor_closed_form(sigma, rho):
    """g = 0 below sigma and 1 above: Eq. 18 integrates to
    S(q) = 1 - 4 pi rho (sin(q sigma) - q sigma cos(q sigma)) / q^3; the midpoint rule
    with sigma on a bin edge is within O(dr^2)."""
    r_max, nb = 1.2, 12000
    dr = r_max / nb
    centres = (np.arange(nb) + 0.5) * dr
    g = np.where(centres < sigma, 0.0, 1.0)
    q = np.linspace(2.0, 60.0, 30)
    S = oracle.structure_factor(g, r_max, rho, q)
    ref = 1.0 - 4 * np.pi * rho * (np.sin(q * sigma) - q * sigma * np.cos(q * sigma)) / q ** 3
    assert np.max(np.abs(S - ref)) < 1e-3
    # g = 1 everywhere: S = 1 exactly
    assert np.array_equal(oracle.structure_factor(np.ones(nb), r_max, rho, q), np.ones(q.size))
