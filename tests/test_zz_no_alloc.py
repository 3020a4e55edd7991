"""The no-allocation histogram entry point (md_rdf_histogram_noalloc) through the C ABI
against md_rdf_histogram, which allocates its workspace: bit-identical integer counts
on two calls in a row on two contexts, the second with fewer atoms, so the fixed
workspace holds the first call's contents when the second runs.  Also: the workspace
limit is reported as MD_ERR_CAPACITY."""
import numpy as np
import pytest

from paper_2401_03180_amd import synth
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _hist(eng, fn, r_max, n_bins):
    import torch
    E = eng.sys.n_elements
    h = torch.zeros((eng.sys.n_systems, E, E, n_bins), dtype=torch.int64, device="cuda")
    fn(eng.ctx, eng.x, eng.y, eng.z, eng.elem, r_max, n_bins, h)
    torch.cuda.synchronize()
    return h.cpu().numpy()


def test_noalloc_histogram_matches_allocating_one():
    import torch
    from paper_2401_03180_amd import md
    big = synth.water_pulse(n_steps=20)
    small = synth.water_small(n_steps=20)
    cases = [(big, 1.0, 250), (small, 0.8, 97)]
    for s, r_max, n_bins in cases:
        say("no-alloc histogram", s.name, s.n_atoms, "atoms")
        eng = md.Engine(s, md.MD_FP32_KAHAN)
        eng.set_step(0)
        eng.build()
        eng.forces()
        for _ in range(8):                       # some atoms move; a few beyond skin/2
            eng.step(md.MD_BUILD_AUTO)
        eng.sync_check()
        want = _hist(eng, md.md_rdf_histogram, r_max, n_bins)
        got = _hist(eng, md.md_rdf_histogram_noalloc, r_max, n_bins)
        assert want.sum() > 0
        assert np.array_equal(got, want)
        got2 = _hist(eng, md.md_rdf_histogram_noalloc, r_max, n_bins)
        assert np.array_equal(got2, want)
        eng.close()


def test_noalloc_histogram_rejects_too_large_a_context():
    """1.73 M atoms (256 methane clusters) need about 28 bytes each, more than the
    32 MiB array: MD_ERR_CAPACITY, and nothing is launched."""
    import torch
    from paper_2401_03180_amd import md
    s = synth.methane_clusters(n_steps=2)
    assert 25 * s.n_atoms > md.MD_RDF_SCRATCH_BYTES
    say("no-alloc histogram capacity", s.n_atoms, "atoms")
    eng = md.Engine(s, md.MD_FP32_KAHAN, density_hint=100.0)
    eng.set_step(0)
    eng.build()
    h = torch.zeros((s.n_systems, s.n_elements, s.n_elements, 10), dtype=torch.int64,
                    device="cuda")
    with pytest.raises(md.MDError) as e:
        md.md_rdf_histogram_noalloc(eng.ctx, eng.x, eng.y, eng.z, eng.elem, 1.0, 10, h)
    assert e.value.status == md.MD_ERR_CAPACITY
    eng.sync_check()
    assert int(h.abs().sum().item()) == 0
    eng.close()
