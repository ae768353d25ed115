"""GPU test of the allocation-free entry point fr_map_noalloc (C ABI).

Three calls in a row on shrinking inputs -- the 1M-voxel PET-like job
(staging rows do not fit the fixed scratch: direct map-major stores), the
100,544-voxel PET workload (staging rows and transpose) and a small job
with Ng = 128 at radius 2 (the generic kernel's region) -- each compared with
fr_map on the same inputs (bit-identical) and with the FP64 oracle (parity
rule); a job larger than the fixed scratch is refused with FR_E_CAPACITY
before any work is enqueued.
"""
import sys

import numpy as np
import pytest

from helpers import format_report, parity_report, to_dev
from oracle import oracle as O
from paper_2609_19190_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_19190_amd import binding
    binding.lib()
    return binding


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_matches_fr_map_on_successive_calls(B):
    import torch
    cases = [synth.pet_large(4), synth.pet_lesion(1),
             synth.random_case(501, shape=(11, 12, 13), dtype=np.float32, radius=2, levels=128,
                               mode=O.FBN, value=128)]
    rng = np.random.default_rng(17)
    for case in cases:
        say("fr_map_noalloc", case.name, "n_mask", case.n_mask, "r", case.radius, "Ng", case.value)
        vol, mask = to_dev(case)
        args = (vol, mask, case.spacing, case.mode, case.value, case.lower, case.radius,
                case.families, case.n_mask)
        ref = B.fr_map(*args)
        ng_ref = B.fr_map_check()
        out = torch.full_like(ref, 7.0)
        B.fr_map_noalloc(*args, out=out)
        assert B.fr_map_check() == ng_ref
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.cpu().numpy().view(np.uint32)), case.name
        samp = np.arange(case.n_mask) if case.n_mask <= 5000 else \
            np.sort(rng.choice(case.n_mask, size=300, replace=False))
        orc = O.spatial_map(case, sample=samp)
        ok, rows = parity_report(got[:, samp], orc, O.map_names(case.families))
        assert ok, format_report(rows, only_bad=True)
        del vol, mask, ref, out
        torch.cuda.empty_cache()


def test_noalloc_refuses_jobs_beyond_its_scratch(B):
    import torch
    shape = (256, 512, 512)  # 67 M voxels: the level volume alone exceeds 64 MiB
    vol = torch.zeros(shape, dtype=torch.int16, device="cuda:0")
    mask = torch.zeros(shape, dtype=torch.uint8, device="cuda:0")
    mask[0, 0, 0] = 1
    out = torch.full((18, 1), 7.0, dtype=torch.float32, device="cuda:0")
    with pytest.raises(B.FrError) as e:
        B.fr_map_noalloc(vol, mask, (1, 1, 1), O.FBN, 8, float("nan"), 1, 1, 1, out=out)
    assert e.value.code == B.FR_E_CAPACITY
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
