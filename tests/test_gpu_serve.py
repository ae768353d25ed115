"""GPU tests of the served request loop (fr_server_*).

Each served job must give exactly the maps fr_map gives it alone (same
kernels, bit-identical) whatever else is in flight; admission must respect
the arena budget; device-side job errors must fail only that job; outputs
must stay resident until released; a short Poisson stream of the served
workload must agree with the oracle on a sample.
"""
import sys
import time

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


def same_bits(a, b):
    a = np.ascontiguousarray(a, np.float32).view(np.uint32)
    b = np.ascontiguousarray(b, np.float32).view(np.uint32)
    return a.shape == b.shape and np.array_equal(a, b)


def alone(B, case, vol, mask):
    import torch
    out = B.fr_map(vol, mask, case.spacing, case.mode, case.value, case.lower, case.radius,
                   case.families, case.n_mask)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def mixed_cases():
    F = synth
    spec = [
        (401, (14, 16, 18), np.float32, 1, O.FBN, 16, F.FAM_ALL),
        (402, (12, 15, 17), np.int16, 2, O.FBW, 25.0, F.FAM_ALL),
        (403, (16, 14, 13), np.float32, 3, O.FBN, 48, F.FAM_ALL),
        (404, (10, 16, 15), np.int16, 1, O.FBN, 64, F.FAM_GLCM | F.FAM_NGTDM),
        (405, (18, 18, 18), np.float32, 2, O.FBN, 16, F.FAM_FIRSTORDER | F.FAM_GLSZM),
        (406, (13, 15, 13), np.float32, 2, O.FBN, 60, F.FAM_ALL),
        (407, (9, 11, 12), np.int16, 3, O.FBW, 30.0, F.FAM_GLRLM | F.FAM_GLDM),
        (408, (15, 13, 14), np.float32, 1, O.FBN, 32, F.FAM_ALL),
    ]
    return [synth.random_case(seed, shape=shape, dtype=dt, radius=r, families=fam, mode=mode,
                              value=val) for seed, shape, dt, r, mode, val, fam in spec]


def test_mixed_in_flight_equals_alone(B):
    import torch
    cases = mixed_cases() + synth.batch_ct(n_jobs=6)
    dev = [to_dev(c) for c in cases]
    ref = [alone(B, c, v, m) for c, (v, m) in zip(cases, dev)]
    srv = B.Server(1 << 30, slots=4)
    try:
        # half at once, the rest while the first ones are running
        tickets = [srv.submit_case(c, v, m) for c, (v, m) in zip(cases[:7], dev[:7])]
        time.sleep(0.002)
        tickets += [srv.submit_case(c, v, m) for c, (v, m) in zip(cases[7:], dev[7:])]
        for t in tickets:
            srv.wait(t, 60000.0)
        st = srv.stats()
        say("stats", st)
        assert st["completed"] == len(cases) and st["failed"] == 0
        assert st["max_inflight"] >= 2, "jobs never overlapped"
        for c, t, r in zip(cases, tickets, ref):
            res = srv.result(t)
            assert res.done == 1 and res.status == 0, (c.name, res.status)
            got = srv.maps(t)
            torch.cuda.synchronize()
            assert same_bits(got.cpu().numpy(), r), c.name
            assert res.t_submit <= res.t_admit <= res.t_done
        done = set()
        while len(done) < len(tickets):
            done.update(srv.poll())
        assert done == set(tickets)
        for t in tickets:
            srv.release(t)
        assert srv.stats()["arena_used_bytes"] == 0
    finally:
        srv.close()


def test_admission_by_footprint(B):
    import torch
    cases = synth.batch_ct(n_jobs=10)
    dev = [to_dev(c) for c in cases]
    jobs = [B.make_job(v, m, c.spacing, c.mode, c.value, c.lower, c.radius, c.families, c.n_mask)
            for c, (v, m) in zip(cases, dev)]
    fp = [B.fr_server_footprint(j) for j in jobs]
    budget = int(max(fp) * 1.2) + (1 << 20)
    say("footprints MB", [round(f / 1e6, 1) for f in fp], "budget MB", budget / 1e6)
    srv = B.Server(budget, slots=4)
    try:
        tickets = [srv.submit_case(c, v, m) for c, (v, m) in zip(cases, dev)]
        peak_seen = 0
        done = []
        while len(done) < len(tickets):  # release as they finish so later jobs fit
            for t in srv.poll():
                done.append(t)
                res = srv.result(t)
                assert res.status == 0
                q = tickets.index(t)
                got = srv.maps(t)
                torch.cuda.synchronize()
                assert same_bits(got.cpu().numpy(), alone(B, cases[q], *dev[q])), cases[q].name
                srv.release(t)
            peak_seen = max(peak_seen, srv.stats()["arena_used_bytes"])
            time.sleep(0.0005)
        st = srv.stats()
        say("stats", st)
        assert st["arena_peak_bytes"] <= budget
        assert st["completed"] == len(cases)
    finally:
        srv.close()
    # a job larger than the whole arena is refused at submission
    q = int(np.argmax(fp))
    tiny = B.Server(max(fp[q] // 2, 1 << 20), slots=1)
    try:
        with pytest.raises(B.FrError) as ei:
            tiny.submit_case(cases[q], *dev[q])
        assert ei.value.code == B.FR_E_CAPACITY
    finally:
        tiny.close()


def test_device_error_fails_only_that_job(B):
    import torch
    good = synth.random_case(411, shape=(12, 12, 12), radius=2, value=16)
    bad = synth.random_case(412, shape=(12, 12, 12), radius=1, value=8)
    gv, gm = to_dev(good)
    bv, bm = to_dev(bad)
    srv = B.Server(1 << 28, slots=2)
    try:
        t_bad = srv.submit(bv, bm, bad.spacing, bad.mode, bad.value, bad.lower, bad.radius,
                           bad.families, bad.n_mask - 1)
        t_good = srv.submit_case(good, gv, gm)
        srv.wait(t_bad, 60000.0)
        srv.wait(t_good, 60000.0)
        rb, rg = srv.result(t_bad), srv.result(t_good)
        assert rb.done == 1 and rb.status == B.FR_E_ARG and not rb.maps
        assert rg.status == 0
        with pytest.raises(B.FrError):
            srv.maps(t_bad)
        got = srv.maps(t_good)
        torch.cuda.synchronize()
        assert same_bits(got.cpu().numpy(), alone(B, good, gv, gm))
        assert srv.stats()["failed"] == 1
        with pytest.raises(B.FrError) as ei:
            srv.release(123456)
        assert ei.value.code == B.FR_E_ARG
        # host-side checks refuse the job before queueing
        with pytest.raises(B.FrError) as ei:
            srv.submit(gv, gm, good.spacing, good.mode, good.value, good.lower, 6, good.families,
                       good.n_mask)
        assert ei.value.code == B.FR_E_RANGE
    finally:
        srv.close()


def test_failure_paths_leave_other_jobs_identical(B):
    """Host-forced failure paths on a live server (one slot, submission
    order): an injected allocation failure, a running job and a queued job
    cancelled, a queued job whose deadline passes; every other job's maps are
    bit-identical to fr_map alone and the arena is empty after release."""
    import torch
    cases = synth.batch_ct(n_jobs=8)
    dev = [to_dev(c) for c in cases]
    ref = [alone(B, c, v, m) for c, (v, m) in zip(cases, dev)]
    big = int(np.argmax([c.n_mask for c in cases]))
    order = [big] + [i for i in range(len(cases)) if i != big]
    srv = B.Server(4 << 30, slots=1)
    try:
        srv.inject_alloc_failures(1)
        t_fail = srv.submit_case(cases[order[1]], *dev[order[1]])
        tickets = {}
        for k, q in enumerate(order):
            tickets[q] = srv.submit_case(cases[q], *dev[q], deadline_ms=0.3 if k == 3 else 0.0)
        srv.cancel(tickets[order[0]])  # running (or about to run)
        srv.cancel(tickets[order[2]])  # queued behind it
        for t in [t_fail] + list(tickets.values()):
            srv.wait(t, 60000.0)
        expect = {order[0]: B.FR_E_CANCELLED, order[2]: B.FR_E_CANCELLED, order[3]: B.FR_E_TIMEOUT}
        assert srv.result(t_fail).status == B.FR_E_NOMEM and not srv.result(t_fail).maps
        for q, t in tickets.items():
            res = srv.result(t)
            say(cases[q].name, "status", res.status)
            assert res.done == 1 and res.status == expect.get(q, B.FR_OK), (cases[q].name, res.status)
            if res.status == B.FR_OK:
                got = srv.maps(t)
                torch.cuda.synchronize()
                assert same_bits(got.cpu().numpy(), ref[q]), cases[q].name
            else:
                assert not res.maps
        with pytest.raises(B.FrError) as ei:  # a finished job cannot be cancelled
            srv.cancel(tickets[order[1]])
        assert ei.value.code == B.FR_E_ARG
        st = srv.stats()
        say("stats", st)
        assert st["failed"] == 4 and st["completed"] == len(cases) + 1
        for t in [t_fail] + list(tickets.values()):
            srv.release(t)
        assert srv.stats()["arena_used_bytes"] == 0
    finally:
        srv.close()


def test_bounded_bypass_on_a_live_server(B):
    """A head job that does not fit is passed by at most max_bypass later
    jobs; every job's maps equal fr_map alone."""
    import torch
    cases = synth.batch_ct(n_jobs=6)
    dev = [to_dev(c) for c in cases]
    jobs = [B.make_job(v, m, c.spacing, c.mode, c.value, c.lower, c.radius, c.families, c.n_mask)
            for c, (v, m) in zip(cases, dev)]
    fp = [B.fr_server_footprint(j) for j in jobs]
    big = int(np.argmax(fp))
    small = [i for i in range(len(cases)) if i != big]
    blocker = small[0]
    # the blocker and the big job cannot share the arena; each small one fits
    # beside the blocker
    budget = max(fp[big], fp[blocker] + max(fp[i] for i in small[1:])) + (1 << 16)
    assert budget < fp[blocker] + fp[big]
    srv = B.Server(budget, slots=8, max_bypass=2)
    try:
        t_block = srv.submit_case(cases[blocker], *dev[blocker])
        t_big = srv.submit_case(cases[big], *dev[big])
        t_small = [srv.submit_case(cases[i], *dev[i]) for i in small[1:]]

        def check_release(i, t):
            res = srv.result(t)
            assert res.status == 0
            got = srv.maps(t)
            torch.cuda.synchronize()
            assert same_bits(got.cpu().numpy(), alone(B, cases[i], *dev[i])), cases[i].name
            srv.release(t)  # a finished job holds its block until released

        # every finished job is checked and released at once: a finished
        # job holds its block until released, and the big one fits only
        # once the blocker's block (and those of the jobs that passed it)
        # are free
        pending = dict(zip([t_block, t_big] + t_small, [blocker, big] + small[1:]))
        t_admit = {}
        t_end = time.monotonic() + 20.0
        while pending and time.monotonic() < t_end:
            for t in list(pending):
                r = srv.result(t)
                if r.done:
                    t_admit[t] = r.t_admit
                    check_release(pending.pop(t), t)
            time.sleep(0.0005)
        assert not pending, "jobs not finished"
        passed = [t for t in t_small if t_admit[t] < t_admit[t_big]]
        say("passed the big job:", len(passed), "of", len(t_small))
        assert len(passed) <= 2
    finally:
        srv.close()


def test_outputs_stay_resident(B):
    import torch
    first = synth.random_case(421, shape=(14, 14, 14), radius=2, value=32)
    fv, fm = to_dev(first)
    others = synth.batch_ct(n_jobs=8)
    odev = [to_dev(c) for c in others]
    srv = B.Server(1 << 30, slots=4)
    try:
        t0 = srv.submit_case(first, fv, fm)
        srv.wait(t0, 60000.0)
        ts = [srv.submit_case(c, v, m) for c, (v, m) in zip(others, odev)]
        for t in ts:
            srv.wait(t, 60000.0)
            srv.release(t)
        got = srv.maps(t0)
        torch.cuda.synchronize()
        assert same_bits(got.cpu().numpy(), alone(B, first, fv, fm))
        srv.release(t0)
    finally:
        srv.close()


def test_short_poisson_stream_against_oracle(B):
    """40 jobs of the served workload arriving as a Poisson stream; every
    result equals fr_map alone and a sample of voxels equals the oracle."""
    import torch
    pool = synth.serve_pool(n=8)
    pdev = [to_dev(c) for c in pool]
    jobs = synth.serve_jobs(n_jobs=40, pool_size=len(pool))
    arr = synth.poisson_arrivals(3, len(jobs), rate=200.0)
    srv = B.Server(4 << 30, slots=4)
    rng = np.random.default_rng(77)
    try:
        t_start = time.monotonic()
        tickets = []
        for (pi, ng, r), ta in zip(jobs, arr):
            while time.monotonic() - t_start < ta:
                time.sleep(0.0002)
            c = pool[pi]
            tickets.append(srv.submit_case(c, *pdev[pi], radius=r, value=float(ng)))
        for t in tickets:
            srv.wait(t, 120000.0)
        st = srv.stats()
        say("stats", st)
        assert st["completed"] == len(jobs) and st["failed"] == 0
        assert 0 < st["p50_ms"] <= st["p99_ms"]
        checked = 0
        for (pi, ng, r), t in zip(jobs, tickets):
            c = pool[pi]
            v, m = pdev[pi]
            got = srv.maps(t)
            ref = B.fr_map(v, m, c.spacing, c.mode, float(ng), c.lower, r, c.families, c.n_mask)
            torch.cuda.synchronize()
            g = got.cpu().numpy()
            assert same_bits(g, ref.cpu().numpy()), (pi, ng, r)
            if checked < 6:
                samp = np.sort(rng.choice(c.n_mask, size=16, replace=False))
                orc = O.spatial_map(vol=c.volume, mask=c.mask, spacing=c.spacing, mode=c.mode,
                                    value=float(ng), lower=c.lower, radius=r,
                                    families=c.families, sample=samp)
                ok, rows = parity_report(g[:, samp], orc, O.map_names(c.families))
                assert ok, f"pool {pi} ng {ng} r {r}\n" + format_report(rows, only_bad=True)
                checked += 1
            srv.release(t)
    finally:
        srv.close()
