"""GPU tests of batched mapping (fr_batch_*).

A batch must give every job exactly the maps fr_map gives it alone (same
arithmetic, so bit-identical including the non-finite pattern), whatever the
mix of raw types, radii, bin counts and family sets; graph replays must
match the eager launch; device-side data errors must skip only the failing
job; and the 64-VOI CT workload must agree with the oracle on a sample.
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


def job_of(case, vol, mask, **over):
    j = dict(volume=vol, mask=mask, spacing=case.spacing, mode=case.mode, value=case.value,
             lower=case.lower, radius=case.radius, families=case.families, n_mask=case.n_mask)
    j.update(over)
    return j


def plain(B, case, vol, mask):
    return B.fr_map(vol, mask, case.spacing, case.mode, case.value, case.lower, case.radius,
                    case.families, case.n_mask)


def same_bits(a, b):
    a = np.ascontiguousarray(a, np.float32).view(np.uint32)
    b = np.ascontiguousarray(b, np.float32).view(np.uint32)
    return a.shape == b.shape and np.array_equal(a, b)


def mixed_cases():
    """Mixed batch: both raw types, radii 1-3, FBN and FBW, 32- and 64-level
    variants, family subsets, ragged sizes."""
    F = synth
    spec = [
        (301, (12, 14, 16), np.float32, 1, O.FBN, 8, F.FAM_ALL),
        (302, (10, 13, 17), np.int16, 2, O.FBW, 25.0, F.FAM_ALL),
        (303, (14, 12, 11), np.float32, 3, O.FBN, 48, F.FAM_ALL),
        (304, (9, 16, 15), np.int16, 1, O.FBN, 64, F.FAM_GLCM | F.FAM_NGTDM),
        (305, (16, 16, 16), np.float32, 2, O.FBN, 16, F.FAM_FIRSTORDER | F.FAM_GLSZM),
        (306, (11, 15, 13), np.float32, 2, O.FBN, 60, F.FAM_ALL),
        (307, (8, 9, 10), np.int16, 3, O.FBW, 30.0, F.FAM_GLRLM | F.FAM_GLDM),
        (308, (13, 11, 12), np.float32, 1, O.FBN, 32, F.FAM_ALL),
    ]
    cs = []
    for seed, shape, dt, r, mode, val, fam in spec:
        cs.append(synth.random_case(seed, shape=shape, dtype=dt, radius=r, families=fam,
                                    mode=mode, value=val))
    return cs


def test_mixed_batch_equals_plain_and_oracle(B):
    import torch
    cases = mixed_cases()
    dev = [to_dev(c) for c in cases]
    jobs = [job_of(c, v, m) for c, (v, m) in zip(cases, dev)]
    say("mixed batch:", [(c.name, c.radius, c.value, c.n_mask) for c in cases])
    bt = B.Batch(jobs)
    try:
        plan = bt.describe()
        say("plan", plan)
        assert sum(p["jobs"] for p in plan) == len(cases)
        bt.launch()
        rc, st, ng = bt.status()
        assert rc == B.FR_OK and st == [0] * len(cases), (rc, st)
        for c, (v, m), out in zip(cases, dev, bt.outs):
            ref = plain(B, c, v, m)
            torch.cuda.synchronize()
            assert same_bits(out.cpu().numpy(), ref.cpu().numpy()), c.name
            orc = O.spatial_map(c)
            ok, rows = parity_report(out.cpu().numpy(), orc, O.map_names(c.families))
            assert ok, c.name + "\n" + format_report(rows, only_bad=True)
            lv, ng1, _, _, _ = B.fr_discretise(v, m, c.mode, c.value, c.lower)
            assert ng[cases.index(c)] == ng1
    finally:
        bt.close()


def test_graph_replays_match_eager(B):
    import torch
    cases = mixed_cases()[:5]
    dev = [to_dev(c) for c in cases]
    jobs = [job_of(c, v, m) for c, (v, m) in zip(cases, dev)]
    bt = B.Batch(jobs)
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            bt.launch(stream=s)
        s.synchronize()
        eager = [o.cpu().numpy().copy() for o in bt.outs]
        for rep in range(3):
            for o in bt.outs:  # eager work between replays
                o.fill_(float("inf"))
            torch.cuda.synchronize()
            bt.launch(stream=s, use_graph=True)
            rc, st, _ = bt.status(stream=s)
            assert rc == B.FR_OK, st
            for q, o in enumerate(bt.outs):
                assert same_bits(o.cpu().numpy(), eager[q]), (rep, cases[q].name)
        # new volume values, same settings: the replay maps the new data
        v0, m0 = dev[0]
        v0.copy_(torch.flip(v0, dims=[2]))
        torch.cuda.synchronize()
        bt.launch(stream=s, use_graph=True)
        s.synchronize()
        ref = plain(B, cases[0], v0, m0)
        torch.cuda.synchronize()
        assert same_bits(bt.outs[0].cpu().numpy(), ref.cpu().numpy())
    finally:
        bt.close()


def test_autotune_keeps_results(B):
    import torch
    cases = mixed_cases()
    dev = [to_dev(c) for c in cases]
    jobs = [job_of(c, v, m) for c, (v, m) in zip(cases, dev)]
    bt = B.Batch(jobs)
    try:
        bt.launch()
        torch.cuda.synchronize()
        before = [o.cpu().numpy().copy() for o in bt.outs]
        bt.autotune()
        after_tune = [o.cpu().numpy().copy() for o in bt.outs]
        say("tuned plan", bt.describe())
        bt.launch()
        rc, st, _ = bt.status()
        assert rc == B.FR_OK
        for q, o in enumerate(bt.outs):
            assert same_bits(after_tune[q], before[q]), cases[q].name
            assert same_bits(o.cpu().numpy(), before[q]), cases[q].name
    finally:
        bt.close()


def test_device_errors_skip_only_failing_jobs(B):
    import torch
    good = synth.random_case(311, shape=(10, 12, 14), radius=2, value=16)
    wrong_count = synth.random_case(312, shape=(10, 12, 14), radius=1, value=8)
    # a fixed bin width giving about 200 levels: 5x5x5 cubes with more than
    # 64 present levels, mapped through the 64-level and generic passes
    many_levels = synth.random_case(313, shape=(12, 12, 12), radius=2, mode=O.FBW, value=0.06)
    too_many_bins = synth.random_case(314, shape=(8, 8, 8), radius=1, mode=O.FBW, value=1e-3)
    cs = [good, wrong_count, many_levels, too_many_bins]
    dev = [to_dev(c) for c in cs]
    outs = []
    for c in cs:
        outs.append(torch.full((O.map_count(c.families), c.n_mask + 1), 7.0, device="cuda:0"))
    jobs = [job_of(good, *dev[0], out=outs[0][:, :good.n_mask].contiguous()),
            job_of(wrong_count, *dev[1], n_mask=wrong_count.n_mask + 1, out=outs[1]),
            job_of(many_levels, *dev[2], out=outs[2][:, :many_levels.n_mask].contiguous()),
            job_of(too_many_bins, *dev[3], out=outs[3][:, :too_many_bins.n_mask].contiguous())]
    bt = B.Batch(jobs)
    try:
        bt.launch()
        rc, st, ng = bt.status()
        say("status", st, "ng", ng)
        assert rc == B.FR_E_RANGE
        assert st == [B.FR_OK, B.FR_E_ARG, B.FR_OK, B.FR_E_RANGE]
        assert 64 < ng[2] <= 255
        for q in (0, 2):
            ref = plain(B, cs[q], *dev[q])
            torch.cuda.synchronize()
            assert same_bits(bt.outs[q].cpu().numpy(), ref.cpu().numpy()), cs[q].name
        for q in (1, 3):
            assert bool((bt.outs[q] == 7.0).all()), cs[q].name
    finally:
        bt.close()


def test_host_errors(B):
    c = synth.random_case(321, shape=(8, 9, 10))
    v, m = to_dev(c)
    for over, code in [(dict(radius=6), B.FR_E_RANGE), (dict(families=0), B.FR_E_RANGE),
                       (dict(mode=O.FBN, value=256.0, radius=3), B.FR_E_RANGE),
                       (dict(n_mask=0), B.FR_E_ARG), (dict(value=-1.0), B.FR_E_ARG),
                       (dict(spacing=(1.0, 0.0, 1.0)), B.FR_E_ARG)]:
        with pytest.raises(B.FrError) as ei:
            B.Batch([job_of(c, v, m, **over)])
        assert ei.value.code == code, (over, ei.value)
    import torch
    small = torch.empty((3, 5), dtype=torch.float32, device="cuda:0")
    with pytest.raises(B.FrError) as ei:
        B.Batch([job_of(c, v, m, out=small)])
    assert ei.value.code == B.FR_E_CAPACITY


def test_batch_ct_64_vois(B):
    """The 64-VOI CT workload: every job bit-identical to its plain fr_map,
    and an oracle sample of 24 voxels per job."""
    import torch
    cases = synth.batch_ct()
    say("batch_ct voxels", sum(c.n_mask for c in cases))
    dev = [to_dev(c) for c in cases]
    bt = B.Batch([job_of(c, v, m) for c, (v, m) in zip(cases, dev)])
    try:
        say("plan", bt.describe())
        bt.launch()
        rc, st, _ = bt.status()
        assert rc == B.FR_OK, st
        rng = np.random.default_rng(64)
        for q, (c, (v, m)) in enumerate(zip(cases, dev)):
            ref = plain(B, c, v, m)
            torch.cuda.synchronize()
            got = bt.outs[q].cpu().numpy()
            assert same_bits(got, ref.cpu().numpy()), c.name
            samp = np.sort(rng.choice(c.n_mask, size=min(24, c.n_mask), replace=False))
            orc = O.spatial_map(c, sample=samp)
            ok, rows = parity_report(got[:, samp], orc, O.map_names(c.families))
            assert ok, c.name + "\n" + format_report(rows, only_bad=True)
        say("batch_ct ok")
    finally:
        bt.close()
