"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Levels and integer matrices must be bit-exact; maps must satisfy the parity
rule of tests/helpers.py with an identical non-finite pattern.  Cases span
several workgroups and ragged tails, every supported radius, both raw types,
both discretisations, family subsets, image borders, isolated voxels, and
the full-size synthetic CT/PET workloads (sampled where the oracle would be
slow).
"""
import math
import os
import sys

import numpy as np
import pytest

from helpers import format_report, parity_report, to_dev
from oracle import oracle as O
from paper_2609_19190_amd import synth

pytestmark = pytest.mark.gpu
ALL = 63


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


def gpu_maps(B, case, families=None, radius=None):
    import torch
    fam = case.families if families is None else families
    r = case.radius if radius is None else radius
    vol, mask = to_dev(case)
    out = B.fr_map(vol, mask, case.spacing, case.mode, case.value, case.lower, r, fam, case.n_mask)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_maps(gpu, orc, fam, label):
    ok, rows = parity_report(gpu, orc, O.map_names(fam))
    assert ok, f"{label}\n" + format_report(rows, only_bad=True)
    return rows


def matrix_keys(families):
    """Matrices the kernel counts for a family mask (the level histogram is
    always counted; the others only for their own family)."""
    keys = ["hist"]
    if families & 8:
        keys.append("glszm")
    if families & 2:
        keys.append("glcm")
    if families & 4:
        keys.append("glrlm")
    if families & 16:
        keys.append("gldm")
    if families & 32:
        keys += ["ngtdm_n", "ngtdm_S"]
    return keys


def small_cases():
    cs = []
    for seed, r, dt, lv, mode, val, fam in [
        (101, 1, np.float32, None, O.FBN, 8, ALL),
        (102, 2, np.float32, None, O.FBN, 16, ALL),
        (103, 3, np.float32, None, O.FBN, 12, ALL),
        (104, 1, np.int16, None, O.FBW, 25.0, ALL),
        (105, 2, np.int16, None, O.FBW, 40.0, ALL),
        (106, 3, np.int16, None, O.FBW, 60.0, ALL),
        (107, 2, np.float32, 2, O.FBN, 2, ALL),      # two raw values: large zones, long runs
        (108, 3, np.float32, 3, O.FBN, 3, ALL),
        (109, 1, np.float32, None, O.FBN, 64, ALL),  # many levels at r = 1
        (110, 2, np.float32, None, O.FBN, 32, 1 | 8),
        (111, 3, np.int16, None, O.FBN, 20, 2 | 32),
        (112, 2, np.float32, None, O.FBN, 64, ALL),  # up to 64 local levels at r = 2
    ]:
        c = synth.random_case(seed, shape=(13, 17, 19), dtype=dt, radius=r, levels=lv, mode=mode,
                              value=val, families=fam)
        cs.append(c)
    # FBW with an explicit lower bound below the data
    c = synth.random_case(113, shape=(9, 11, 12), dtype=np.int16, radius=2, mode=O.FBW, value=50.0,
                          lower=-400.0)
    cs.append(c)
    # radius 1 with 65..255 gray levels (level values beyond 64; at most 27 per cube)
    cs.append(synth.random_case(114, shape=(13, 17, 19), dtype=np.float32, radius=1, mode=O.FBN,
                                value=255))
    cs.append(synth.random_case(115, shape=(13, 17, 19), dtype=np.int16, radius=1, mode=O.FBW,
                                value=25.0, lower=-1000.0, bone=True))  # Ng = 107
    # FBW lower bound above part of the VOI: those voxels are raised to level 1
    for seed, r in ((116, 2), (117, 1), (118, 3)):
        cs.append(synth.random_case(seed, shape=(13, 17, 19), dtype=np.int16, radius=r,
                                    mode=O.FBW, value=25.0, lower=0.0))
    # more than 64 levels at radius 2 and 3: neighbourhoods with 33..64 and
    # more than 64 present levels take the 64-level and the generic passes
    cs.append(synth.random_case(119, shape=(11, 12, 13), dtype=np.float32, radius=2, levels=128,
                                mode=O.FBN, value=128))
    cs.append(synth.random_case(120, shape=(10, 11, 12), dtype=np.float32, radius=3, levels=100,
                                mode=O.FBN, value=100))
    cs.append(synth.random_case(121, shape=(12, 13, 14), dtype=np.int16, radius=2, mode=O.FBW,
                                value=25.0, lower=-1000.0, bone=True))
    cs.append(synth.random_case(122, shape=(11, 12, 13), dtype=np.int16, radius=3, mode=O.FBW,
                                value=25.0, lower=-1000.0, bone=True))
    # radii 4 and 5: the generic kernel alone
    cs.append(synth.random_case(123, shape=(12, 13, 14), dtype=np.float32, radius=4, mode=O.FBN,
                                value=16))
    cs.append(synth.random_case(124, shape=(13, 14, 15), dtype=np.int16, radius=5, mode=O.FBW,
                                value=40.0))
    cs.append(synth.random_case(125, shape=(11, 12, 13), dtype=np.float32, radius=4, levels=3,
                                mode=O.FBN, value=3, families=1 | 8 | 16))
    return cs


@pytest.mark.parametrize("case", small_cases(), ids=lambda c: f"{c.name}_r{c.radius}_f{c.families}")
def test_small_case_levels_matrices_maps(B, case):
    import torch
    say("case", case.name, case.volume.shape, case.volume.dtype, "r", case.radius, "mode", case.mode,
        "value", case.value, "fam", case.families, "n_mask", case.n_mask)
    vol, mask = to_dev(case)
    lev, ng, xmin, xmax, n = B.fr_discretise(vol, mask, case.mode, case.value, case.lower)
    olev, ong, oxmin, oxmax = O.discretise(case.volume, case.mask, case.mode, case.value, case.lower)
    assert n == case.n_mask and ng == ong and xmin == oxmin and xmax == oxmax
    assert np.array_equal(lev.cpu().numpy(), olev)
    if np.isfinite(case.lower):
        say("voxels below the lower bound:", int((case.volume[case.mask > 0] < case.lower).sum()))
    # matrices of every mask voxel, bit-exact (every k-th one for large Ng:
    # the dense tables are Ng x Ng per voxel)
    samp = np.arange(case.n_mask, dtype=np.int64)
    if ng > 64 or case.radius >= 4:
        samp = samp[:: max(1, len(samp) // 200)]
    res = B.fr_map_matrices(vol, mask, case.spacing, case.mode, case.value, case.lower, case.radius,
                            case.families, case.n_mask, torch.from_numpy(samp), ng)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in res.items()}
    pts = np.argwhere(case.mask)
    keys = matrix_keys(case.families)
    for q in range(0, len(samp), max(1, len(samp) // 150)):
        s = samp[q]
        m = O.matrices(olev, case.volume, ng, tuple(int(v) for v in pts[s]), case.radius)
        for key in keys:
            assert np.array_equal(res[key][q], m[key]), f"{key} differs at compact index {s}"
    orc = O.spatial_map(case)
    check_maps(res["maps"], orc[:, samp], case.families, "sampled kernel")
    gpu = gpu_maps(B, case)
    check_maps(gpu, orc, case.families, "fr_map")
    assert np.array_equal(gpu[:, samp].view(np.uint32), res["maps"].view(np.uint32))


def test_ct_tiny_full(B):
    case = synth.tiny_ct(0)
    say("ct tiny", case.n_mask)
    gpu = gpu_maps(B, case)
    orc = O.spatial_map(case)
    rows = check_maps(gpu, orc, case.families, "ct tiny")
    say(format_report(rows))


def test_pet_full_families_full(B):
    case = synth.pet_lesion(1)
    say("pet 128x128x64 r2 ng32", case.n_mask)
    gpu = gpu_maps(B, case)
    orc = O.spatial_map(case)
    rows = check_maps(gpu, orc, case.families, "pet full")
    say(format_report(rows))
    gpu2 = gpu_maps(B, case)  # deterministic: bit-identical on a second run
    assert np.array_equal(gpu.view(np.uint32), gpu2.view(np.uint32))


def test_pet_full_matrices_sampled(B):
    import torch
    case = synth.pet_lesion(1)
    vol, mask = to_dev(case)
    olev, ng, _, _ = O.discretise(case.volume, case.mask, case.mode, case.value)
    lev = B.fr_discretise(vol, mask, case.mode, case.value)[0]
    assert np.array_equal(lev.cpu().numpy(), olev)
    rng = np.random.default_rng(5)
    samp = np.sort(rng.choice(case.n_mask, size=300, replace=False)).astype(np.int64)
    res = B.fr_map_matrices(vol, mask, case.spacing, case.mode, case.value, case.lower, case.radius,
                            case.families, case.n_mask, torch.from_numpy(samp), ng)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in res.items()}
    pts = np.argwhere(case.mask)
    for q, s in enumerate(samp):
        m = O.matrices(olev, case.volume, ng, tuple(int(v) for v in pts[s]), case.radius)
        for key in ("glcm", "glrlm", "glszm", "gldm", "ngtdm_n", "ngtdm_S", "hist"):
            assert np.array_equal(res[key][q], m[key]), f"{key} differs at compact index {s}"


def test_pet_large_sampled(B):
    import torch
    case = synth.pet_large(4)
    say("pet large 256x256x128 r3 ng64", case.n_mask)
    assert abs(case.n_mask - 1_000_000) <= 10_000
    vol, mask = to_dev(case)
    lev = B.fr_discretise(vol, mask, case.mode, case.value)[0]
    olev, ng, _, _ = O.discretise(case.volume, case.mask, case.mode, case.value)
    assert np.array_equal(lev.cpu().numpy(), olev)
    gpu = gpu_maps(B, case)
    rng = np.random.default_rng(9)
    samp = np.sort(rng.choice(case.n_mask, size=1500, replace=False)).astype(np.int64)
    orc = O.spatial_map(case, sample=samp)
    rows = check_maps(gpu[:, samp], orc, case.families, "pet large (sampled)")
    say(format_report(rows))
    res = B.fr_map_matrices(vol, mask, case.spacing, case.mode, case.value, case.lower, case.radius,
                            case.families, case.n_mask, torch.from_numpy(samp[:40]), ng)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in res.items()}
    pts = np.argwhere(case.mask)
    for q, s in enumerate(samp[:40]):
        m = O.matrices(olev, case.volume, ng, tuple(int(v) for v in pts[s]), case.radius)
        for key in ("glcm", "glrlm", "glszm", "gldm", "ngtdm_n", "ngtdm_S", "hist"):
            assert np.array_equal(res[key][q], m[key]), f"{key} differs at compact index {s}"


def _golden(fname):
    env = {"log2": math.log2, "sqrt": math.sqrt, "exp": math.exp, "__builtins__": {}}
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", fname)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split("=", 1)
                out[k.strip()] = float(eval(v, env))
    return out


def test_line5_closed_form_on_gpu(B):
    vol = np.zeros((5, 5, 9), np.float32)
    mask = np.zeros((5, 5, 9), np.uint8)
    vol[2, 2, 2:7] = [10, 12, 30, 31, 35]
    mask[2, 2, 2:7] = 1
    case = synth.Case("line5", vol, mask, (1.0, 1.5, 2.5), O.FBN, 2, float("nan"), 2, ALL)
    gpu = gpu_maps(B, case)
    gold = _golden("line5_handderived.txt")
    for k, name in enumerate(O.map_names(ALL)):
        want = gold[name]
        assert abs(gpu[k, 2] - want) <= max(1e-7, 1e-5 * abs(want)), (name, gpu[k, 2], want)


def test_checkerboard_closed_form_on_gpu(B):
    z, y, x = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    vol = ((x + y + z) % 2 + 1).astype(np.float32)
    case = synth.Case("checker", vol, np.ones((3, 3, 3), np.uint8), (1, 1, 1), O.FBN, 2,
                      float("nan"), 1, 2)
    gpu = gpu_maps(B, case)
    gold = _golden("checker3_handderived.txt")
    for k, name in enumerate(O.map_names(2)):
        want = gold[name]
        assert abs(gpu[k, 13] - want) <= max(1e-7, 1e-5 * abs(want)), (name, gpu[k, 13], want)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_constant_interior(B, r):
    n = 2 * r + 5
    vol = np.full((n, n, n), 100.0, np.float32)
    mask = np.ones((n, n, n), np.uint8)
    case = synth.Case("const", vol, mask, (1, 1, 1), O.FBW, 25.0, 0.0, r, ALL)
    gpu = gpu_maps(B, case)
    orc = O.spatial_map(case)
    check_maps(gpu, orc, ALL, f"constant r={r}")


def test_isolated_voxels_and_borders(B):
    vol = np.arange(4 * 5 * 6, dtype=np.float32).reshape(4, 5, 6) % 7
    mask = np.zeros((4, 5, 6), np.uint8)
    mask[0, 0, 0] = 1          # corner, isolated
    mask[3, 4, 5] = 1          # opposite corner, isolated
    mask[1:3, 1:4, 2:5] = 1    # a block
    mask[0, 2, 5] = 1          # border voxel touching nothing
    case = synth.Case("isolated", vol, mask, (1, 1, 1), O.FBN, 5, float("nan"), 1, ALL)
    for r in (1, 2, 3):
        gpu = gpu_maps(B, case, radius=r)
        orc = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBN, value=5, radius=r,
                            families=ALL)
        check_maps(gpu, orc, ALL, f"isolated r={r}")


def test_degenerate_shapes(B):
    for shape in [(1, 1, 1), (1, 1, 40), (1, 30, 1), (25, 1, 1), (2, 3, 2)]:
        rng = np.random.default_rng(sum(shape))
        vol = rng.integers(-50, 50, size=shape).astype(np.int16)
        mask = np.ones(shape, np.uint8)
        case = synth.Case("shape", vol, mask, (1, 1, 1), O.FBN, 6, float("nan"), 2, ALL)
        gpu = gpu_maps(B, case)
        orc = O.spatial_map(case)
        check_maps(gpu, orc, ALL, f"shape {shape}")


def test_errors(B):
    import torch
    case = synth.random_case(120, shape=(6, 7, 8))
    vol, mask = to_dev(case)
    with pytest.raises(B.FrError) as e:
        B.fr_map(vol, mask, case.spacing, O.FBN, 8, float("nan"), 6, ALL, case.n_mask)
    assert e.value.code == B.FR_E_RANGE
    with pytest.raises(B.FrError) as e:
        B.fr_map(vol, mask, case.spacing, O.FBN, 8, float("nan"), 1, 64, case.n_mask)
    assert e.value.code == B.FR_E_RANGE
    with pytest.raises(B.FrError) as e:
        B.fr_map(vol, mask, case.spacing, O.FBN, 256, float("nan"), 2, ALL, case.n_mask)
    assert e.value.code == B.FR_E_RANGE
    small = torch.empty(10, dtype=torch.float32, device="cuda:0")
    with pytest.raises(B.FrError) as e:
        B.fr_map(vol, mask, case.spacing, O.FBN, 8, float("nan"), 1, ALL, case.n_mask, out=small)
    assert e.value.code == B.FR_E_CAPACITY
    with pytest.raises(B.FrError) as e:
        B.fr_map(vol, mask, case.spacing, O.FBN, 8, float("nan"), 1, ALL, 0)
    assert e.value.code == B.FR_E_EMPTY_MASK
    with pytest.raises(B.FrError) as e:  # fixed bin width giving > 255 levels
        B.fr_discretise(vol, mask, O.FBW, 1e-3)
    assert e.value.code == B.FR_E_RANGE
    for bad in (dict(glcm_distance=0), dict(glcm_distance=11), dict(gldm_alpha=-1),
                dict(aggregation=2)):
        with pytest.raises(B.FrError) as e:
            B.fr_map(vol, mask, case.spacing, O.FBN, 8, float("nan"), 1, ALL, case.n_mask,
                     options=B.map_options(**bad))
        assert e.value.code in (B.FR_E_RANGE, B.FR_E_ARG), bad
    with pytest.raises(B.FrError) as e:
        B.fr_map(vol, mask, (1.0, 0.0, 1.0), O.FBN, 8, float("nan"), 1, ALL, case.n_mask)
    assert e.value.code == B.FR_E_ARG
    # a host pointer is refused before any work is enqueued
    with pytest.raises(B.FrError) as e:
        B.lib()
        B._check(B.lib().fr_map(case.volume.ctypes.data, 2, 8, 7, 6, mask.data_ptr(),
                                (B.ctypes.c_double * 3)(1, 1, 1), O.FBN, 8.0, float("nan"), 1, ALL,
                                case.n_mask, torch.empty(1, device="cuda:0").data_ptr(), 10 ** 9,
                                None))
    assert e.value.code == B.FR_E_ARG


def test_device_data_errors_leave_output_untouched(B):
    """fr_map enqueues without waiting: data errors (mask count, empty mask,
    more than 255 FBW levels) are found on the device, reported by
    fr_map_status, and stop every later kernel of the call."""
    import torch
    case = synth.random_case(126, shape=(9, 10, 11), radius=2, value=16)
    vol, mask = to_dev(case)
    n = case.n_mask
    cnt = O.map_count(ALL)
    for label, m, nm, mode, val, code in [
            ("count", mask, n + 1, O.FBN, 16, B.FR_E_ARG),
            ("empty", torch.zeros_like(mask), 5, O.FBN, 16, B.FR_E_EMPTY_MASK),
            ("fbw>255", mask, n, O.FBW, 1e-3, B.FR_E_RANGE)]:
        out = torch.full((cnt, nm), 7.0, dtype=torch.float32, device="cuda:0")
        B.fr_map(vol, m, case.spacing, mode, val, float("nan"), case.radius, ALL, nm, out=out)
        rc, _ = B.fr_map_status()
        assert rc == code, label
        assert bool((out == 7.0).all()), label
    out = B.fr_map(vol, mask, case.spacing, O.FBN, 16, float("nan"), case.radius, ALL, n)
    assert B.fr_map_check() == 16
    check_maps(out.cpu().numpy(), O.spatial_map(case), ALL, "after errors")


def test_fr_map_is_asynchronous(B):
    """fr_map returns before the device has finished: the host call takes a
    small part of the mapping time and an event recorded after it is still
    pending; fr_map_check then synchronises and reports success."""
    import time
    import torch
    case = synth.pet_large(4)
    vol, mask = to_dev(case)
    out = torch.empty((O.map_count(case.families), case.n_mask), dtype=torch.float32, device="cuda:0")
    args = (vol, mask, case.spacing, case.mode, case.value, case.lower, case.radius, case.families,
            case.n_mask)
    B.fr_map(*args, out=out)  # first call: scratch allocation
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    B.fr_map(*args, out=out, stream=stream)
    host_ms = (time.perf_counter() - t0) * 1e3
    ev = torch.cuda.Event()
    ev.record(stream)
    pending = not ev.query()
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t0) * 1e3
    say(f"fr_map host {host_ms:.3f} ms, enqueue to done {total_ms:.2f} ms, pending {pending}")
    assert pending and host_ms < 0.25 * total_ms
    assert B.fr_map_check(stream) == int(case.value)


def _present_levels(levels, radius):
    """Distinct levels per cube (full mask, so every level of V has a GLCM
    neighbour in V): the size n of each voxel's MCC problem."""
    nz, ny, nx = levels.shape
    out = np.empty(levels.size, dtype=np.int64)
    q = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                c = levels[max(0, z - radius):z + radius + 1, max(0, y - radius):y + radius + 1,
                           max(0, x - radius):x + radius + 1]
                out[q] = len(np.unique(c))
                q += 1
    return out


@pytest.mark.parametrize("radius,ng,shape", [(1, 32, (9, 10, 11)), (2, 32, (13, 14, 15)),
                                             (3, 32, (11, 12, 13)), (2, 48, (12, 13, 14)),
                                             (2, 128, (11, 12, 13)), (3, 100, (10, 11, 12))])
def test_mcc_level_count_classes(B, radius, ng, shape):
    """Neighbourhoods of i.i.d. uniform levels over a full mask: the MCC
    problem sizes span the one-column (n <= 16), two-column (17..32, with
    n = 32 exactly, whose last sub-diagonal entry is read from the matrix)
    and, for Ng > 32, the 64-level instance's one-problem-per-wave MCC and,
    for Ng > 64, the generic kernel's; every map against the oracle."""
    rng = np.random.default_rng(1000 + 10 * radius + ng)
    vol = rng.integers(0, ng, size=shape).astype(np.float32)
    vol.flat[0], vol.flat[1] = 0.0, float(ng - 1)  # raw k -> level k + 1
    mask = np.ones(shape, dtype=np.uint8)
    case = synth.Case(f"uniform_r{radius}_ng{ng}", vol, mask, (1.0, 1.0, 1.0), O.FBN, float(ng),
                      float("nan"), radius, ALL, {})
    olev = O.discretise(vol, mask, O.FBN, float(ng))[0]
    ns = _present_levels(olev.reshape(shape), radius)
    hist = np.bincount(ns, minlength=ng + 1)
    say("case", case.name, "n_mask", case.n_mask, "problem sizes",
        {k: int(v) for k, v in enumerate(hist) if v})
    assert (ns >= 17).any()
    if radius == 1:
        assert (ns <= 16).any()
    if radius >= 2 and ng == 32:
        assert (ns == 32).any()
    if 32 < ng <= 64:
        assert (ns > 32).any() and ((ns >= 17) & (ns <= 32)).any()
    if ng > 64:  # 33..64 levels (64-level pass) and more (the generic kernel's MCC)
        assert (ns > 64).any() and ((ns > 32) & (ns <= 64)).any()
    gpu = gpu_maps(B, case)
    orc = O.spatial_map(case)
    check_maps(gpu, orc, ALL, case.name)


def _b_spectrum(P):
    """Eigenvalues of B = D^-1/2 P D^-1/2 - v v^T over the present levels of
    a co-occurrence matrix (numpy's symmetric solver)."""
    P = np.asarray(P, dtype=np.float64)
    P = P / P.sum()
    px = P.sum(axis=1)
    keep = px > 0
    P, px = P[np.ix_(keep, keep)], px[keep]
    r = np.sqrt(px)
    return np.linalg.eigvalsh(P / np.outer(r, r) - np.outer(r, r))


@pytest.mark.parametrize("radius,ng,shape", [(1, 32, (10, 11, 12)), (2, 32, (12, 13, 14)),
                                             (3, 64, (11, 12, 13))])
def test_mcc_smallest_eigenvalue_dominates(B, radius, ng, shape):
    """Levels from the lower half of the range on even x and from the upper
    half on odd x: co-occurrences run mostly between the two halves, so the
    smallest eigenvalue of B is often the larger in size and the MCC
    searches fall back from the one-sided to the two-sided count (problem
    sizes: one and two columns per lane at radius 1 and 2, the 64-level
    solver at radius 3).  The spectra are checked with numpy on a sample,
    every map against the oracle."""
    rng = np.random.default_rng(2000 + 10 * radius + ng)
    x = np.arange(shape[2])[None, None, :]
    lo_half = rng.integers(0, ng // 2, size=shape)
    hi_half = rng.integers(ng // 2, ng, size=shape)
    vol = np.where(x % 2 == 0, lo_half, hi_half).astype(np.float32)
    vol.flat[0], vol.flat[1] = 0.0, float(ng - 1)  # raw k -> level k + 1
    mask = np.ones(shape, dtype=np.uint8)
    case = synth.Case(f"halves_r{radius}_ng{ng}", vol, mask, (1.0, 1.0, 1.0), O.FBN, float(ng),
                      float("nan"), radius, ALL, {})
    olev, ong, _, _ = O.discretise(vol, mask, O.FBN, float(ng))
    pts = np.argwhere(mask)
    dominated = 0
    for s in rng.choice(len(pts), size=24, replace=False):
        ev = _b_spectrum(O.matrices(olev, vol, ong, tuple(int(v) for v in pts[s]), radius)["glcm"])
        dominated += -ev[0] > ev[-1]
    say("case", case.name, "sampled neighbourhoods with |lambda_min| > lambda_max:", dominated, "of 24")
    assert dominated >= 3
    ns = _present_levels(olev.reshape(shape), radius)
    if radius == 3:
        assert (ns > 32).any()
    gpu = gpu_maps(B, case)
    orc = O.spatial_map(case)
    check_maps(gpu, orc, ALL, case.name)


@pytest.mark.parametrize("radius", [2, 3])
def test_uniform_high_levels(B, radius):
    """A CT-like int16 volume at 3000 HU with 10 % scattered values in
    [-1000, 5000] HU, FBW 25 HU from -1000 HU: uniform neighbourhoods at
    level 161 of Ng = 241, whose large-zone and dependence emphasis sums
    (c i^2 j^2 up to ~4e9) exceed 32 bits; every map against the oracle."""
    rng = np.random.default_rng(3000 + radius)
    shape = (12, 12, 12)
    vol = np.full(shape, 3000, dtype=np.int16)
    pick = rng.random(shape) < 0.10
    vol[pick] = rng.integers(-1000, 5001, size=int(pick.sum())).astype(np.int16)
    vol.flat[0], vol.flat[1] = -1000, 5000
    mask = np.ones(shape, dtype=np.uint8)
    case = synth.Case(f"uniform_high_r{radius}", vol, mask, (1.0, 1.0, 2.0), O.FBW, 25.0, -1000.0,
                      radius, ALL, {})
    olev, ong, _, _ = O.discretise(vol, mask, O.FBW, 25.0, -1000.0)
    assert ong == 241 and (olev == 161).mean() > 0.85
    gpu = gpu_maps(B, case)
    orc = O.spatial_map(case)
    check_maps(gpu, orc, ALL, case.name)


# --------------------------------------------------------------------------
# extraction variants (fr_map_ex): GLCM distance, GLDM alpha, averaged
# --------------------------------------------------------------------------
VARIANTS = [dict(glcm_distance=2), dict(gldm_alpha=2), dict(averaged=True),
            dict(glcm_distance=3, gldm_alpha=1, averaged=True)]


def _opts(B, v):
    return B.map_options(glcm_distance=v.get("glcm_distance", 1), gldm_alpha=v.get("gldm_alpha", 0),
                         aggregation=B.FR_AVERAGED if v.get("averaged") else B.FR_MERGED)


@pytest.mark.parametrize("seed,r,dt,mode,val", [(131, 1, np.float32, O.FBN, 8),
                                                (132, 2, np.int16, O.FBW, 25.0),
                                                (133, 3, np.float32, O.FBN, 20),
                                                (134, 4, np.int16, O.FBW, 30.0)])
@pytest.mark.parametrize("v", VARIANTS, ids=lambda v: "_".join(f"{k}{int(x)}" for k, x in v.items()))
def test_variants_levels_matrices_maps(B, seed, r, dt, mode, val, v):
    import torch
    case = synth.random_case(seed, shape=(11, 12, 13), dtype=dt, radius=r, mode=mode, value=val)
    say("case", case.name, "r", r, "variant", v, "n_mask", case.n_mask)
    vol, mask = to_dev(case)
    olev, ng, _, _ = O.discretise(case.volume, case.mask, case.mode, case.value, case.lower)
    opt = _opts(B, v)
    samp = np.arange(0, case.n_mask, max(1, case.n_mask // 120), dtype=np.int64)
    res = B.fr_map_matrices(vol, mask, case.spacing, case.mode, case.value, case.lower, r, ALL,
                            case.n_mask, torch.from_numpy(samp), ng, options=opt)
    torch.cuda.synchronize()
    res = {k: t.cpu().numpy() for k, t in res.items()}
    pts = np.argwhere(case.mask)
    for q in range(0, len(samp), 4):
        s = samp[q]
        m = O.matrices(olev, case.volume, ng, tuple(int(c) for c in pts[s]), r,
                       glcm_distance=v.get("glcm_distance", 1), gldm_alpha=v.get("gldm_alpha", 0))
        for key in ("glcm", "glrlm", "glszm", "gldm", "ngtdm_n", "ngtdm_S", "hist"):
            assert np.array_equal(res[key][q], m[key]), f"{key} differs at compact index {s}"
    orc = O.spatial_map(case, **v)
    check_maps(res["maps"], orc[:, samp], ALL, f"sampled {v}")
    out = B.fr_map(vol, mask, case.spacing, case.mode, case.value, case.lower, r, ALL, case.n_mask,
                   options=opt)
    B.fr_map_check()
    gpu = out.cpu().numpy()
    check_maps(gpu, orc, ALL, f"fr_map_ex {v}")
    assert np.array_equal(gpu[:, samp].view(np.uint32), res["maps"].view(np.uint32))


def test_variant_stripes_closed_form_on_gpu(B):
    z, y, x = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    vol = (x % 2 + 1).astype(np.float32)
    case = synth.Case("stripes", vol, np.ones((3, 3, 3), np.uint8), (1, 1, 1), O.FBN, 2,
                      float("nan"), 1, 2 | 4)
    gold = _golden("stripes3_handderived.txt")
    names = O.map_names(2 | 4)
    for averaged, prefix in ((False, "merged_"), (True, "avg_")):
        out = B.fr_map(*to_dev(case), case.spacing, case.mode, case.value, case.lower, 1, 2 | 4,
                       case.n_mask, options=B.map_options(
                           aggregation=B.FR_AVERAGED if averaged else B.FR_MERGED))
        B.fr_map_check()
        got = out.cpu().numpy()[:, 13]
        n = 0
        for k, name in enumerate(names):
            if prefix + name in gold:
                want = gold[prefix + name]
                assert abs(got[k] - want) <= max(1e-7, 1e-5 * abs(want)), (prefix + name, got[k], want)
                n += 1
        assert n >= 10
