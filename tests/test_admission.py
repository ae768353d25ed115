"""Admission policy of the served loop, replayed on the host in virtual time
(fr_admission_replay: the server's own admission code with a virtual HBM
budget and no device).

Pins: submission order when every job fits; first-fit placement inside the
budget; a head job that does not fit is passed by at most max_bypass later
jobs; a queued job past its deadline leaves without running; a cancelled job
never runs (queued) or ends cancelled (running); injected allocation
failures fail exactly the next admissions and nothing else; a job larger
than the budget is refused.  A random-script test checks every replay
against an independent Python model of the same rules.
"""
import numpy as np
import pytest

from paper_2609_19190_amd import binding as B

U = 256  # the arena's allocation unit

S, X, C, F = B.FR_ADMIT_SUBMIT, B.FR_ADMIT_CANCEL, B.FR_ADMIT_COMPLETE, B.FR_ADMIT_FAIL_NEXT
ADM, EXP, CAN, FAIL, REJ = (B.FR_ADMITTED, B.FR_ADMIT_EXPIRED, B.FR_ADMIT_CANCELLED,
                            B.FR_ADMIT_ALLOC_FAILED, B.FR_ADMIT_REJECTED)


def sub(t, ticket, units, deadline_ms=0.0):
    return dict(t=t, kind=S, ticket=ticket, bytes=units * U, deadline_ms=deadline_ms)


def done(t, ticket):
    return dict(t=t, kind=C, ticket=ticket)


def outcomes(recs):
    return [(tk, oc) for _, tk, _, oc in recs]


def test_submission_order_and_first_fit():
    ev = [sub(0, 1, 4), sub(0, 2, 4), sub(0, 3, 4), done(1, 1), done(2, 2), done(3, 3)]
    r = B.fr_admission_replay(10 * U, 4, 0, ev)
    assert outcomes(r) == [(1, ADM), (2, ADM), (3, ADM)]
    off = {tk: o for _, tk, o, _ in r}
    assert off[1] == 0 and off[2] == 4 * U
    assert off[3] == 0  # job 3 waits for job 1's block, then takes it (first fit)
    assert [t for t, tk, _, _ in r if tk == 3] == [1]


def test_slots_bound_admission():
    ev = [sub(0, 1, 1), sub(0, 2, 1), sub(0, 3, 1), done(5, 2)]
    r = B.fr_admission_replay(10 * U, 2, 0, ev)
    assert outcomes(r) == [(1, ADM), (2, ADM), (3, ADM)]
    assert [t for t, tk, _, _ in r if tk == 3] == [5]


@pytest.mark.parametrize("max_bypass", [0, 1, 2, 5])
def test_bounded_bypass_of_a_head_that_does_not_fit(max_bypass):
    # R holds 10 of 16 units; H needs 8 (waits for R); S1..S3 need 1 each
    ev = [sub(0, 100, 10), sub(1, 1, 8), sub(2, 11, 1), sub(3, 12, 1), sub(4, 13, 1),
          done(10, 100)]
    r = B.fr_admission_replay(16 * U, 8, max_bypass, ev)
    order = [tk for _, tk, _, oc in r if oc == ADM]
    t_adm = {tk: t for t, tk, _, oc in r if oc == ADM}
    k = min(max_bypass, 3)
    # the first k small jobs pass H at their arrival; the others wait behind
    # it and follow it once R has finished
    assert order == [100] + [11, 12, 13][:k] + [1] + [11, 12, 13][k:]
    assert [t_adm[tk] for tk in [11, 12, 13][:k]] == [2, 3, 4][:k]
    assert t_adm[1] == 10 and all(t_adm[tk] == 10 for tk in [11, 12, 13][k:])


def test_head_admitted_after_the_jobs_that_passed_it_complete():
    ev = [sub(0, 100, 6), sub(1, 1, 8), sub(2, 11, 1), sub(3, 12, 1), sub(4, 13, 1),
          done(10, 100), done(11, 11), done(12, 12)]
    r = B.fr_admission_replay(10 * U, 8, 2, ev)
    assert outcomes(r) == [(100, ADM), (11, ADM), (12, ADM), (1, ADM), (13, ADM)]
    t = {tk: tt for tt, tk, _, _ in r}
    assert t[1] == 12 and t[13] == 12  # H needs 8 contiguous units: free only after 11 and 12


def test_deadline_expires_a_queued_job_only():
    ev = [sub(0, 1, 8), sub(0.001, 2, 8, deadline_ms=5.0), sub(0.002, 3, 1, deadline_ms=5.0),
          sub(0.010, 4, 1), done(0.020, 1)]
    # strict order: 2 waits behind 1 and 3 behind 2; both expire at the
    # first event after their deadline, then 4 runs
    r = B.fr_admission_replay(10 * U, 4, 0, ev)
    assert outcomes(r) == [(1, ADM), (2, EXP), (3, EXP), (4, ADM)]
    assert [t for t, tk, _, oc in r if oc == EXP] == [0.010, 0.010]
    # with one bypass allowed, 3 passes 2 at once and runs; only 2 expires
    r = B.fr_admission_replay(10 * U, 4, 1, ev)
    assert outcomes(r) == [(1, ADM), (3, ADM), (2, EXP), (4, ADM)]


def test_cancel_queued_and_running():
    ev = [sub(0, 1, 8), sub(0, 2, 8), sub(0, 3, 2), dict(t=1, kind=X, ticket=2),
          dict(t=2, kind=X, ticket=1), done(3, 1), done(4, 3)]
    r = B.fr_admission_replay(10 * U, 4, 0, ev)
    assert (2, CAN) in outcomes(r) and (2, ADM) not in outcomes(r)
    assert outcomes(r).count((1, ADM)) == 1
    # the running job ends cancelled when its work completes
    assert [(t, oc) for t, tk, _, oc in r if tk == 1] == [(0, ADM), (3, CAN)]
    assert (3, ADM) in outcomes(r)


def test_injected_allocation_failure_fails_only_the_next_admissions():
    base = [sub(0, 1, 2), sub(0, 2, 2), sub(0, 3, 2)]
    clean = B.fr_admission_replay(10 * U, 4, 0, base)
    inj = B.fr_admission_replay(10 * U, 4, 0, [dict(t=0, kind=F, value=1)] + base)
    assert outcomes(inj) == [(1, FAIL), (2, ADM), (3, ADM)]
    # the failed job keeps no block: the others are placed as if it never was
    assert [o for _, tk, o, oc in inj if oc == ADM] == [o for _, tk, o, _ in clean][:2]
    inj2 = B.fr_admission_replay(10 * U, 4, 0, [dict(t=0, kind=F, value=2)] + base)
    assert outcomes(inj2) == [(1, FAIL), (2, FAIL), (3, ADM)]


def test_job_larger_than_the_budget_is_refused():
    r = B.fr_admission_replay(10 * U, 4, 0, [sub(0, 1, 11), sub(0, 2, 10)])
    assert outcomes(r) == [(1, REJ), (2, ADM)]


def test_replay_argument_errors():
    with pytest.raises(B.FrError) as e:
        B.fr_admission_replay(10 * U, 4, 0, [sub(1, 1, 1), sub(0.5, 2, 1)])
    assert e.value.code == B.FR_E_ARG
    with pytest.raises(B.FrError):
        B.fr_admission_replay(10 * U, 4, 0, [sub(0, 1, 1), sub(0, 1, 1)])
    with pytest.raises(B.FrError):
        B.fr_admission_replay(10 * U, 4, 0, [sub(0, 1, 11), done(1, 1)])
    with pytest.raises(B.FrError):
        B.fr_admission_replay(10 * U, 0, 0, [sub(0, 1, 1)])


class Model:
    """The admission rules written out independently: queue in submission
    order, first-fit blocks over [0, budget), bounded bypass per head,
    deadlines at each step, injected failures on the next admissions."""

    def __init__(self, budget, slots, k):
        self.free = [(0, budget)]
        self.budget, self.slots, self.k = budget, slots, k
        self.q, self.run, self.head, self.passed, self.fail = [], {}, None, 0, 0
        self.cancelled = set()

    def alloc(self, n):
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                self.free[i:i + 1] = [(o + n, sz - n)] if sz > n else []
                return o
        return -1

    def release(self, o, n):
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for a, sz in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + sz)
            else:
                merged.append((a, sz))
        self.free = merged

    def step(self, t, out):
        keep = []
        for j in self.q:
            if j[2] > 0 and t >= j[2]:
                out.append((t, j[0], -1, EXP))
            else:
                keep.append(j)
        self.q = keep
        while len(self.run) < self.slots and self.q:
            if self.q[0][0] != self.head:
                self.head, self.passed = self.q[0][0], 0
            pick, o = 0, self.alloc(self.q[0][1])
            if o < 0 and self.passed < self.k:
                for i in range(1, len(self.q)):
                    o = self.alloc(self.q[i][1])
                    if o >= 0:
                        pick = i
                        break
            if o < 0:
                break
            tk, n, _ = self.q.pop(pick)
            if pick:
                self.passed += 1
            if self.fail:
                self.fail -= 1
                self.release(o, n)
                out.append((t, tk, -1, FAIL))
                continue
            # invariant: running blocks stay inside the budget and never overlap
            assert 0 <= o and o + n <= self.budget
            assert all(o + n <= o2 or o2 + n2 <= o for o2, n2 in self.run.values())
            self.run[tk] = (o, n)
            out.append((t, tk, o, ADM))

    def apply(self, e, out):
        t = e["t"]
        if e["kind"] == S:
            if e["bytes"] > self.budget:
                out.append((t, e["ticket"], -1, REJ))
            else:
                dl = t + e["deadline_ms"] * 1e-3 if e["deadline_ms"] > 0 else 0.0
                self.q.append((e["ticket"], e["bytes"], dl))
        elif e["kind"] == X:
            if any(j[0] == e["ticket"] for j in self.q):
                self.q = [j for j in self.q if j[0] != e["ticket"]]
                out.append((t, e["ticket"], -1, CAN))
            else:
                self.cancelled.add(e["ticket"])
        elif e["kind"] == C:
            o, n = self.run.pop(e["ticket"])
            self.release(o, n)
            if e["ticket"] in self.cancelled:
                out.append((t, e["ticket"], -1, CAN))
        elif e["kind"] == F:
            self.fail = e["value"]
        self.step(t, out)


def random_script(rng, n_jobs):
    """Submissions, completions of running jobs, cancellations and failure
    injections in time order, valid for the rules above (the model tracks
    which jobs run)."""
    budget = int(rng.integers(8, 40)) * U
    slots = int(rng.integers(1, 6))
    k = int(rng.integers(0, 4))
    m = Model(budget, slots, k)
    ev, out, t, nxt = [], [], 0.0, 1
    state = {}
    while nxt <= n_jobs or m.run:
        t += float(rng.exponential(0.002))
        u = rng.random()
        if nxt <= n_jobs and (u < 0.45 or not m.run):
            units = int(rng.integers(1, budget // U + 3))
            dl = float(rng.choice([0.0, 0.0, 1.0, 5.0, 20.0]))
            e = dict(t=t, kind=S, ticket=nxt, bytes=units * U, deadline_ms=dl)
            nxt += 1
        elif u < 0.55 and (m.q or m.run):
            cand = [j[0] for j in m.q] + [tk for tk in m.run if tk not in m.cancelled]
            if not cand:
                continue
            e = dict(t=t, kind=X, ticket=int(rng.choice(cand)))
        elif u < 0.6:
            e = dict(t=t, kind=F, value=int(rng.integers(0, 3)))
        elif m.run:
            e = dict(t=t, kind=C, ticket=int(rng.choice(list(m.run))))
        else:
            continue
        ev.append(e)
        m.apply(e, out)
    return budget, slots, k, ev, out


@pytest.mark.parametrize("seed", range(12))
def test_replay_matches_an_independent_model(seed):
    rng = np.random.default_rng(seed)
    budget, slots, k, ev, expect = random_script(rng, 60)
    got = B.fr_admission_replay(budget, slots, k, ev)
    assert len(got) == len(expect)
    for g, x in zip(got, expect):
        assert g[1:] == x[1:] and abs(g[0] - x[0]) < 1e-12, (g, x)
    assert any(x[3] == ADM for x in expect)
