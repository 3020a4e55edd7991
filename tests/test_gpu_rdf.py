"""GPU parity of the pair-distance histograms behind g_ab(r) and the partial
structure factors of section II.C (Eq. 18): counts bit-exact against the oracle's
brute-force histogram on the same positions, including atoms that moved beyond
skin/2 of the neighbour build; the host helpers for g and S(q) against the
oracle's."""
import numpy as np
import pytest

import oracle
from paper_2401_03180_amd import synth
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def make_engine(sys, prec=1, **kw):
    from paper_2401_03180_amd.md import Engine
    return Engine(sys, prec, **kw)


def gpu_hist(eng, r_max, n_bins):
    h = eng.rdf(r_max, n_bins)
    eng.sync_check()
    return h.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("r_max,n_bins", [(1.0, 200), (0.47, 1), (0.999, 2048)])
def test_water_histogram_exact(r_max, n_bins):
    s = synth.water_small(n_steps=2)
    say("rdf water", r_max, n_bins)
    eng = make_engine(s)
    eng.set_step(0)
    eng.build()
    h = gpu_hist(eng, r_max, n_bins)
    assert np.array_equal(h, oracle.rdf_histogram(s, r_max, n_bins))
    eng.close()


def test_moved_atoms_and_accumulation():
    """Atoms displaced beyond skin/2 of the build (handled by the brute-force pass):
    still exact; a second call adds the same counts."""
    from test_gpu_parity import _displace, _fast_case
    for periodic in (True, False):
        s, disp, fast = _fast_case(periodic, 40, 91 + periodic)
        say("rdf moved atoms periodic", periodic)
        eng = make_engine(s, density_hint=0.0 if periodic else 100.0)
        eng.set_step(0)
        eng.build()
        _displace(eng, s, disp)
        x, y, z = eng.host("x"), eng.host("y"), eng.host("z")
        ref = oracle.rdf_histogram(s, 0.95, 190, x=x, y=y, z=z)
        h = eng.rdf(0.95, 190)
        eng.rdf(0.95, 190, hist=h)
        eng.sync_check()
        assert np.array_equal(h.cpu().numpy().view(np.uint64), 2 * ref), periodic
        eng.close()


def test_batched_clusters_histogram():
    s = synth.methane_clusters(n_clusters=5, lo=300, hi=4000, n_steps=2)
    say("rdf methane batched")
    eng = make_engine(s, density_hint=100.0)
    eng.set_step(0)
    eng.build()
    h = gpu_hist(eng, 1.0, 100)
    assert np.array_equal(h, oracle.rdf_histogram(s, 1.0, 100))
    eng.close()


def test_lattice_shells_on_gpu():
    """Perfect simple-cubic lattice: the GPU histogram has the exact shell counts."""
    from test_rdf_pins import lattice_system
    a, n = 0.3137, 8
    s = lattice_system(a, n)
    say("rdf lattice")
    eng = make_engine(s)
    eng.set_step(0)
    eng.build()
    h = gpu_hist(eng, 0.8, 160)[0, 0, 0]
    assert np.array_equal(h, oracle.rdf_histogram(s, 0.8, 160)[0, 0, 0])
    N = s.n_atoms
    assert h[int(a / 0.005)] == N * 6 // 2 and h.sum() == N * (6 + 12 + 8 + 6 + 24 + 24) // 2
    eng.close()


def test_host_helpers_match_oracle():
    from paper_2401_03180_amd import md
    rng = np.random.default_rng(2)
    counts = rng.integers(0, 10000, 300).astype(np.uint64)
    for same in (True, False):
        g = md.md_rdf_normalize(counts, 1.0, 32768, 65536, same, 9.93 ** 3)
        ref = oracle.rdf_normalize(counts, 1.0, 32768, 65536, same, 9.93 ** 3)
        assert np.allclose(g, ref, rtol=1e-13, atol=0)
    q = np.linspace(1.0, 80.0, 50)
    Sg = md.md_structure_factor(g, 1.0, 33.4, q)
    assert np.allclose(Sg, oracle.structure_factor(g, 1.0, 33.4, q), rtol=1e-12, atol=1e-12)
    with pytest.raises(md.MDError):
        md.md_structure_factor(g, 1.0, 33.4, np.array([0.0]))


def test_rdf_argument_errors():
    from paper_2401_03180_amd import md
    s = synth.water_small(n_steps=2)
    say("rdf argument errors")
    eng = make_engine(s)
    with pytest.raises(md.MDError) as e:
        eng.rdf(1.0, 10)
    assert e.value.status == md.MD_ERR_STATE
    eng.build()
    for r_max, nb in ((0.0, 10), (1.01, 10), (0.5, 0), (0.5, 4096)):
        with pytest.raises(md.MDError) as e:
            eng.rdf(r_max, nb)
        assert e.value.status == md.MD_ERR_ARG
    eng.close()


def test_water_pulse_full_size_histogram():
    """98,304-atom water after six graph-replayed steps at the pulse peak (ionization,
    rebuilds, fast atoms): O-O, O-H and H-H counts to 1 nm equal the oracle's
    all-pairs histogram, and their total is the number of pairs in the cutoff."""
    import torch
    from paper_2401_03180_amd import md
    s = synth.water_pulse(n_steps=600)
    say("rdf water_98304")
    eng = make_engine(s)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        eng.set_step(494, st)
        eng.build(md.MD_BUILD_FORCE, st)
        eng.forces(energy=True, stream=st)
        g = eng.graph(md.MD_BUILD_AUTO, st, energy=True, ekin=True)
        for _ in range(6):
            md.md_graph_launch(g, st)
        h = eng.rdf(1.0, 250, stream=st)
        st.synchronize()
    assert eng.sync_check(raise_on_flags=False) == 0
    x, y, z = eng.host("x"), eng.host("y"), eng.host("z")
    ref = oracle.rdf_histogram(s, 1.0, 250, x=x, y=y, z=z)
    got = h.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref)
    assert got.sum() == eng.debug_pairs().shape[0]
    eng.close()
