"""fr_scalar (host FP64 whole-VOI features) against the oracle.

fr_scalar is a second, independent implementation (Householder + Sturm
bisection for MCC where the oracle uses Jacobi; sparse zone tables; its own
loops); both are FP64, so they must agree to rounding: |a - b| <= 1e-9
max(1, |b|) with an identical NaN pattern.  On the GPU, the map value at a
voxel whose cube covers the whole VOI must equal the scalar value (the
definitions coincide there), within the map parity tolerance.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_19190_amd import synth

ALL = 63


@pytest.fixture(scope="module")
def B():
    from paper_2609_19190_amd import binding
    binding.lib()
    return binding


def agree(a, b, names, tol=1e-9):
    bad = []
    for k, n in enumerate(names):
        x, y = a[k], b[k]
        if np.isnan(x) or np.isnan(y):
            if not (np.isnan(x) and np.isnan(y)):
                bad.append((n, x, y))
            continue
        if abs(x - y) > tol * max(1.0, abs(y)):
            bad.append((n, x, y))
    return bad


CASES = [
    (11, {}),
    (12, dict(dtype=np.int16, mode=O.FBW, value=25.0)),
    (13, dict(levels=3)),
    (14, dict(shape=(5, 6, 7), mask_fill=0.3)),
    (15, dict(value=64)),
    (16, dict(shape=(20, 22, 18), value=32)),
    (17, dict(dtype=np.int16, levels=2, mode=O.FBN, value=2)),
    (18, dict(dtype=np.int16, mode=O.FBW, value=10.0, lower=-200.0)),
]


@pytest.mark.parametrize("seed,kw", CASES)
def test_scalar_matches_oracle(B, seed, kw):
    c = synth.random_case(seed, **kw)
    got = B.fr_scalar(c.volume, c.mask, c.spacing, c.mode, c.value, c.lower, ALL)
    ref = O.scalar(c, families=ALL)
    bad = agree(got, ref, O.map_names(ALL))
    assert not bad, bad


def test_scalar_family_subsets(B):
    c = synth.random_case(21)
    full = B.fr_scalar(c.volume, c.mask, c.spacing, c.mode, c.value, c.lower, ALL)
    names = O.map_names(ALL)
    for fam in (1, 2, 4, 8, 16, 32, 1 | 32, 2 | 8 | 16):
        sub = B.fr_scalar(c.volume, c.mask, c.spacing, c.mode, c.value, c.lower, fam)
        want = [full[names.index(n)] for n in O.map_names(fam)]
        assert np.array_equal(np.asarray(want), sub, equal_nan=True), fam


def test_scalar_single_voxel_and_constant(B):
    vol = np.zeros((3, 3, 3), np.float32)
    mask = np.zeros((3, 3, 3), np.uint8)
    mask[1, 1, 1] = 1
    got = B.fr_scalar(vol, mask, (1, 1, 1), O.FBN, 8, float("nan"), ALL)
    ref = O.scalar(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBN, value=8, families=ALL)
    assert not agree(got, ref, O.map_names(ALL))
    vol = np.full((4, 5, 6), 7.0, np.float32)
    mask = np.ones((4, 5, 6), np.uint8)
    got = B.fr_scalar(vol, mask, (1, 1, 1), O.FBN, 8, float("nan"), ALL)
    ref = O.scalar(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBN, value=8, families=ALL)
    assert not agree(got, ref, O.map_names(ALL))


def test_scalar_errors(B):
    c = synth.random_case(31)
    with pytest.raises(B.FrError) as ei:
        B.fr_scalar(c.volume, np.zeros_like(c.mask), c.spacing, c.mode, c.value, c.lower, ALL)
    assert ei.value.code == B.FR_E_EMPTY_MASK
    with pytest.raises(B.FrError) as ei:
        B.fr_scalar(c.volume, c.mask, c.spacing, O.FBW, 1e-4, float("nan"), ALL)
    assert ei.value.code == B.FR_E_RANGE
    with pytest.raises(B.FrError) as ei:
        B.fr_scalar(c.volume, c.mask, (1.0, -1.0, 1.0), c.mode, c.value, c.lower, ALL)
    assert ei.value.code == B.FR_E_ARG
    with pytest.raises(B.FrError) as ei:
        B.fr_scalar(c.volume, c.mask, c.spacing, c.mode, c.value, c.lower, 64)
    assert ei.value.code == B.FR_E_RANGE


@pytest.mark.gpu
@pytest.mark.parametrize("r", [1, 2, 3])
def test_map_at_covering_voxel_equals_scalar(B, r):
    """A VOI inside a (2r+1)^3 box centred on a mask voxel: that voxel's map
    equals fr_scalar of the VOI."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from helpers import ABS_TOL, REL_TOL, to_dev
    rng = np.random.default_rng(40 + r)
    S = 2 * r + 1
    shape = (S + 2, S + 3, S + 4)
    vol = rng.gamma(2.0, 1.5, size=shape).astype(np.float32)
    mask = np.zeros(shape, np.uint8)
    mask[1:1 + S, 1:1 + S, 2:2 + S] = (rng.random((S, S, S)) < 0.8)
    cz, cy, cx = 1 + r, 1 + r, 2 + r
    mask[cz, cy, cx] = 1
    ng = min(16, S ** 3)
    c = synth.Case("cover", vol, mask, (1.0, 1.5, 2.0), O.FBN, float(ng), float("nan"), r, ALL)
    sc = B.fr_scalar(vol, mask, c.spacing, c.mode, c.value, c.lower, ALL)
    v, m = to_dev(c)
    maps = B.fr_map(v, m, c.spacing, c.mode, c.value, c.lower, r, ALL, c.n_mask)
    torch.cuda.synchronize()
    lin = np.flatnonzero(mask.ravel())
    k = int(np.searchsorted(lin, (cz * shape[1] + cy) * shape[2] + cx))
    got = maps.cpu().numpy()[:, k].astype(np.float64)
    for q, n in enumerate(O.map_names(ALL)):
        x, y = got[q], sc[q]
        if np.isnan(y):
            assert np.isnan(x), n
        else:
            assert abs(x - y) <= max(ABS_TOL, REL_TOL * abs(y)), (n, x, y)
