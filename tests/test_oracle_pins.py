"""Pins of the FP64 oracle to things other than itself.

Each test checks the oracle against what the definitions and mathematics
fix: hand-derived closed forms (tests/golden/*_handderived.txt), library
routines (numpy percentiles and moments, scipy connected-component labelling
and neighbourhood correlation, numpy's general eigensolver), brute-force
enumeration on tiny inputs written differently from the oracle, and
invariants (pair/run/zone totals, identities between features, the cube
symmetries, map == scalar when the kernel covers the VOI).
"""
import math
import os

import numpy as np
import pytest
from scipy import ndimage, stats

from oracle import oracle as O
from paper_2609_19190_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL = 63
NAMES = O.map_names(ALL)


def load_golden(fname):
    env = {"log2": math.log2, "sqrt": math.sqrt, "exp": math.exp, "__builtins__": {}}
    out = {}
    with open(os.path.join(GOLDEN, fname)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, expr = line.split("=", 1)
            out[name.strip()] = float(eval(expr, env))
    return out


def compact_index(mask, zyx):
    """Raster-order rank of voxel zyx among the mask voxels."""
    flat = np.flatnonzero(mask.ravel())
    lin = np.ravel_multi_index(zyx, mask.shape)
    return int(np.searchsorted(flat, lin))


# --------------------------------------------------------------------------
# neighbourhood extraction written independently of the oracle
# --------------------------------------------------------------------------
def cube(levels, vol, centre, r):
    """member/level/raw arrays of the (2r+1)^3 cube around centre; voxels
    outside the image or the mask are non-members."""
    S = 2 * r + 1
    pad = r
    L = np.pad(levels, pad)
    V = np.pad(vol.astype(np.float64), pad)
    z, y, x = (c + pad for c in centre)
    lev = L[z - r:z + r + 1, y - r:y + r + 1, x - r:x + r + 1].astype(np.int64)
    raw = V[z - r:z + r + 1, y - r:y + r + 1, x - r:x + r + 1]
    member = lev > 0
    assert lev.shape == (S, S, S)
    return member, lev, raw


OFFS26 = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
          if (dz, dy, dx) != (0, 0, 0)]


def brute_glcm(member, lev, ng):
    """All ordered member pairs at Chebyshev distance exactly 1."""
    pts = np.argwhere(member)
    g = lev[member]
    d = np.abs(pts[:, None, :] - pts[None, :, :]).max(axis=2)
    a, b = np.nonzero(d == 1)
    P = np.zeros((ng, ng), np.int64)
    np.add.at(P, (g[a] - 1, g[b] - 1), 1)
    return P


def brute_glrlm(member, lev, ng):
    """Walk every line of the box in each of 13 directions from the box
    boundary and split it into runs of equal level among members."""
    S0, S1, S2 = member.shape
    lmax = max(member.shape)
    R = np.zeros((ng, lmax), np.int64)
    dirs = [(0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 1), (0, -1, 1), (1, 0, 1), (-1, 0, 1),
            (1, 1, 0), (-1, 1, 0), (1, 1, 1), (-1, 1, 1), (1, -1, 1), (-1, -1, 1)]
    inb = lambda p: 0 <= p[0] < S0 and 0 <= p[1] < S1 and 0 <= p[2] < S2
    for d in dirs:
        for p in np.ndindex(S0, S1, S2):
            prev = (p[0] - d[0], p[1] - d[1], p[2] - d[2])
            if inb(prev):
                continue  # not a line start
            line = []
            q = p
            while inb(q):
                line.append(lev[q] if member[q] else 0)
                q = (q[0] + d[0], q[1] + d[1], q[2] + d[2])
            k = 0
            while k < len(line):
                if line[k] == 0:
                    k += 1
                    continue
                e = k
                while e + 1 < len(line) and line[e + 1] == line[k]:
                    e += 1
                R[line[k] - 1, e - k] += 1
                k = e + 1
    return R


def brute_glszm(member, lev, ng, zmax):
    Z = np.zeros((ng, zmax), np.int64)
    for g in range(1, ng + 1):
        lab, n = ndimage.label(member & (lev == g), structure=np.ones((3, 3, 3)))
        if n:
            sizes = np.bincount(lab.ravel())[1:]
            for s in sizes:
                Z[g - 1, s - 1] += 1
    return Z


def brute_gldm(member, lev, ng):
    D = np.zeros((ng, 27), np.int64)
    for g in range(1, ng + 1):
        ind = (member & (lev == g)).astype(np.int64)
        same = ndimage.correlate(ind, np.ones((3, 3, 3), np.int64), mode="constant") - ind
        for k in same[ind > 0]:
            D[g - 1, k] += 1
    return D


def brute_ngtdm(member, lev, ng):
    m = member.astype(np.int64)
    lv = lev * m
    ones = np.ones((3, 3, 3), np.int64)
    cnt = ndimage.correlate(m, ones, mode="constant") - m
    lsum = ndimage.correlate(lv, ones, mode="constant") - lv
    n = np.zeros(ng, np.int64)
    s = np.zeros(ng)
    sel = member & (cnt > 0)
    for g, c, t in zip(lev[sel], cnt[sel], lsum[sel]):
        n[g - 1] += 1
        s[g - 1] += abs(g - t / c)
    return n, s


# --------------------------------------------------------------------------
# discretisation
# --------------------------------------------------------------------------
def test_fbn_ramp_equal_bins():
    # a ramp of Ng*m distinct values puts exactly m values in every bin
    ng, m = 8, 5
    vals = np.arange(ng * m, dtype=np.float32).reshape(1, 1, -1)
    mask = np.ones_like(vals, dtype=np.uint8)
    lev, ngo, xmin, xmax = O.discretise(vals, mask, O.FBN, ng)
    assert ngo == ng and xmin == 0 and xmax == ng * m - 1
    assert np.array_equal(np.bincount(lev.ravel())[1:], np.full(ng, m))
    assert lev.ravel()[0] == 1 and lev.ravel()[-1] == ng  # X = Xmax -> Ng


def test_fbn_bin_edges_and_constant():
    # range 4, Ng 4: bin edges at 1,2,3 -> value on an edge opens the next bin
    vals = np.array([0, 0.999, 1, 1.5, 2, 3, 3.999, 4], np.float32).reshape(1, 1, -1)
    mask = np.ones_like(vals, dtype=np.uint8)
    lev, ng, _, _ = O.discretise(vals, mask, O.FBN, 4)
    assert lev.ravel().tolist() == [1, 1, 2, 2, 3, 4, 4, 4]
    const = np.full((2, 2, 2), 7.5, np.float32)
    lev, ng, _, _ = O.discretise(const, np.ones((2, 2, 2), np.uint8), O.FBN, 16)
    assert (lev == 1).all() and ng == 16


def test_fbw_edges_lower_bound_and_mask():
    # IBSI fixed bin width: g = floor((X - Xlo)/w) + 1, Ng = max level
    vals = np.array([-122, -98, -97, 0, 3, 205, 999], np.int16).reshape(1, 1, -1)
    mask = np.array([1, 1, 1, 1, 1, 1, 0], np.uint8).reshape(1, 1, -1)
    lev, ng, xmin, xmax = O.discretise(vals, mask, O.FBW, 25.0)
    # Xlo = VOI minimum -122: offsets 0, 24, 25, 122, 125, 327
    assert lev.ravel().tolist() == [1, 1, 2, 5, 6, 14, 0]
    assert ng == 14 and xmin == -122 and xmax == 205
    lev, ng, _, _ = O.discretise(vals, mask, O.FBW, 25.0, lower=-1000.0)
    # offsets from -1000: 878, 902, 903, 1000, 1003, 1205 -> floor(/25)+1
    assert lev.ravel().tolist() == [36, 37, 37, 41, 41, 49, 0] and ng == 49


def test_fbw_lower_bound_above_values_clamps_to_level_one():
    # a lower bound above part of the VOI: floor((X - Xlo)/w) + 1 < 1 is
    # raised to level 1 (the reading for values below the bound); Ng stays
    # the level of the VOI maximum
    vals = np.array([-122, -98, -97, 0, 3, 205, 999], np.int16).reshape(1, 1, -1)
    mask = np.array([1, 1, 1, 1, 1, 1, 0], np.uint8).reshape(1, 1, -1)
    lev, ng, xmin, xmax = O.discretise(vals, mask, O.FBW, 25.0, lower=0.0)
    # offsets -122, -98, -97, 0, 3, 205 -> floor(/25)+1 = -4, -3, -3, 1, 1, 9
    assert lev.ravel().tolist() == [1, 1, 1, 1, 1, 9, 0] and ng == 9
    lev, ng, _, _ = O.discretise(vals, mask, O.FBW, 25.0, lower=-100.0)
    # offsets -22, 2, 3, 100, 103, 305 -> 0 (raised to 1), 1, 1, 5, 5, 13
    assert lev.ravel().tolist() == [1, 1, 1, 5, 5, 13, 0] and ng == 13
    # a bound above the VOI maximum: every voxel at level 1, Ng = 1
    lev, ng, _, _ = O.discretise(vals, mask, O.FBW, 25.0, lower=300.0)
    assert lev.ravel().tolist() == [1, 1, 1, 1, 1, 1, 0] and ng == 1


def test_ct_tiny_ng():
    c = synth.tiny_ct(0)
    lev, ng, xmin, xmax = O.discretise(c.volume, c.mask, c.mode, c.value)
    assert ng == int((xmax - xmin) // 25) + 1 == 14
    assert c.n_mask == 2176


# --------------------------------------------------------------------------
# hand-derived closed forms
# --------------------------------------------------------------------------
def _line5_case():
    vol = np.zeros((5, 5, 9), np.float32)
    mask = np.zeros((5, 5, 9), np.uint8)
    vol[2, 2, 2:7] = [10, 12, 30, 31, 35]
    mask[2, 2, 2:7] = 1
    return vol, mask


def test_line5_all_families_closed_form():
    vol, mask = _line5_case()
    gold = load_golden("line5_handderived.txt")
    assert len(gold) == 93
    m = compact_index(mask, (2, 2, 4))
    out = O.spatial_map(vol=vol, mask=mask, spacing=(1.0, 1.5, 2.5), mode=O.FBN, value=2,
                        radius=2, families=ALL, sample=[m])[:, 0]
    for k, name in enumerate(NAMES):
        assert out[k] == pytest.approx(gold[name], rel=1e-12, abs=1e-12), name


def test_checkerboard_glcm_closed_form():
    z, y, x = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    vol = ((x + y + z) % 2 + 1).astype(np.float32)
    mask = np.ones((3, 3, 3), np.uint8)
    levels, ng, _, _ = O.discretise(vol, mask, O.FBN, 2)
    assert np.array_equal(levels, vol.astype(np.uint8))
    mats = O.matrices(levels, vol, ng, (1, 1, 1), 1)
    assert mats["glcm"].tolist() == [[72, 86], [86, 72]]
    gold = load_golden("checker3_handderived.txt")
    out = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBN, value=2, radius=1,
                        families=2, sample=[13])[:, 0]
    for k, name in enumerate(O.map_names(2)):
        assert out[k] == pytest.approx(gold[name], rel=1e-12, abs=1e-13), name
    # zones: the two parity classes are each face-diagonally connected
    assert sorted(np.argwhere(mats["glszm"]).tolist()) == [[0, 13], [1, 12]]
    # dependence: corners 4, face centres 9 (level 1); edges 6, centre 13 (level 2)
    D = mats["gldm"]
    assert D[0, 3] == 8 and D[0, 8] == 6 and D[1, 5] == 12 and D[1, 12] == 1 and D.sum() == 27


@pytest.mark.parametrize("r,pairs,runs,deps", [
    (1, 158, {1: 84, 2: 60, 3: 49}, {8: 8, 12: 12, 18: 6, 27: 1}),
    (2, 1036, {1: 156, 2: 132, 3: 108, 4: 84, 5: 109}, {8: 8, 12: 36, 18: 54, 27: 27}),
    (3, 3258, {1: 228, 2: 204, 3: 180, 4: 156, 5: 132, 6: 108, 7: 193},
     {8: 8, 12: 60, 18: 150, 27: 125}),
])
def test_constant_full_cube(r, pairs, runs, deps):
    # a constant interior neighbourhood at level c = 5 (FBW 25 from 0)
    n = 2 * r + 5
    vol = np.full((n, n, n), 100.0, np.float32)
    mask = np.ones((n, n, n), np.uint8)
    levels, ng, _, _ = O.discretise(vol, mask, O.FBW, 25.0, lower=0.0)
    assert ng == 5 and (levels == 5).all()
    c = n // 2
    mats = O.matrices(levels, vol, ng, (c, c, c), r)
    K = (2 * r + 1) ** 3
    assert mats["K"] == K
    # pairs of a full cube: 3 S^2 (S-1) + 6 S (S-1)^2 + 4 (S-1)^3
    S = 2 * r + 1
    assert 3 * S * S * (S - 1) + 6 * S * (S - 1) ** 2 + 4 * (S - 1) ** 3 == pairs
    assert mats["glcm"][4, 4] == 2 * pairs and mats["glcm"].sum() == 2 * pairs
    assert {j + 1: int(v) for j, v in enumerate(mats["glrlm"][4]) if v} == runs
    assert {k + 1: int(v) for k, v in enumerate(mats["gldm"][4]) if v} == deps
    assert mats["glszm"][4, K - 1] == 1 and mats["glszm"].sum() == 1
    out = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBW, value=25.0,
                        lower=0.0, radius=r, families=ALL,
                        sample=[compact_index(mask, (c, c, c))])[:, 0]
    f = dict(zip(NAMES, out))
    for nm in ("JointEnergy", "MaximumProbability", "Idm", "Id", "Idn", "Idmn", "Correlation", "MCC"):
        assert f["glcm_" + nm] == 1.0, nm
    for nm in ("JointEntropy", "SumEntropy", "DifferenceEntropy", "Contrast", "DifferenceAverage",
               "DifferenceVariance", "ClusterTendency", "ClusterShade", "ClusterProminence",
               "SumSquares", "InverseVariance", "Imc1", "Imc2"):
        assert f["glcm_" + nm] == 0.0, nm
    assert f["glcm_Autocorrelation"] == 25.0 and f["glcm_JointAverage"] == 5.0
    assert f["glcm_SumAverage"] == 10.0
    assert f["ngtdm_Coarseness"] == 1e6
    for nm in ("Contrast", "Busyness", "Complexity", "Strength"):
        assert f["ngtdm_" + nm] == 0.0, nm
    assert f["glszm_ZonePercentage"] == 1.0 / K and f["glszm_LargeAreaEmphasis"] == K * K
    assert f["firstorder_Variance"] == 0 and f["firstorder_Skewness"] == 0
    assert f["firstorder_Kurtosis"] == 0 and f["firstorder_Entropy"] == 0
    assert f["firstorder_Uniformity"] == 1.0
    assert f["glrlm_RunPercentage"] == pytest.approx(sum(runs.values()) / (13 * K), rel=1e-15)


# --------------------------------------------------------------------------
# brute force on tiny irregular inputs
# --------------------------------------------------------------------------
def _cases():
    out = []
    for seed, r, dtype, lv in [(11, 1, np.float32, None), (12, 2, np.float32, 3),
                               (13, 2, np.int16, None), (14, 3, np.float32, 2),
                               (15, 1, np.float32, 2), (16, 3, np.int16, None)]:
        c = synth.random_case(seed, shape=(9, 10, 11), dtype=dtype, radius=r, levels=lv,
                              mode=O.FBN, value=6)
        out.append(c)
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c.name}_r{c.radius}")
def test_matrices_match_brute_force(case):
    levels, ng, _, _ = O.discretise(case.volume, case.mask, case.mode, case.value)
    r = case.radius
    S = 2 * r + 1
    rng = np.random.default_rng(7)
    pts = np.argwhere(case.mask)
    pick = rng.choice(len(pts), size=min(12, len(pts)), replace=False)
    # always include voxels on the image border
    border = [i for i, p in enumerate(pts) if (p == 0).any() or (p == np.array(case.mask.shape) - 1).any()]
    pick = list(pick) + border[:3]
    for i in pick:
        centre = tuple(int(v) for v in pts[i])
        member, lev, raw = cube(levels, case.volume, centre, r)
        mats = O.matrices(levels, case.volume, ng, centre, r)
        K = int(member.sum())
        assert mats["K"] == K
        assert np.array_equal(mats["glcm"], brute_glcm(member, lev, ng))
        assert np.array_equal(mats["glrlm"], brute_glrlm(member, lev, ng))
        assert np.array_equal(mats["glszm"], brute_glszm(member, lev, ng, S ** 3))
        assert np.array_equal(mats["gldm"], brute_gldm(member, lev, ng))
        n, s = brute_ngtdm(member, lev, ng)
        assert np.array_equal(mats["ngtdm_n"], n)
        np.testing.assert_allclose(mats["ngtdm_s"], s, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(mats["ngtdm_S"] / 26771144400.0, s, rtol=1e-13, atol=1e-13)
        assert np.array_equal(mats["hist"], np.bincount(lev[member], minlength=ng + 1)[1:])
        np.testing.assert_array_equal(np.sort(mats["vals"]), np.sort(raw[member]))
        # totals
        assert (mats["glrlm"] * np.arange(1, S + 1)).sum() == 13 * K
        assert (mats["glszm"] * np.arange(1, S ** 3 + 1)).sum() == K
        assert mats["gldm"].sum() == K
        assert np.array_equal(mats["glcm"], mats["glcm"].T)


# --------------------------------------------------------------------------
# feature-level pins: library routines and identities
# --------------------------------------------------------------------------
def _random_maps(seed, r, families=ALL, ng=6, levels=None, shape=(9, 10, 11)):
    c = synth.random_case(seed, shape=shape, radius=r, levels=levels, mode=O.FBN, value=ng)
    out = O.spatial_map(vol=c.volume, mask=c.mask, spacing=c.spacing, mode=c.mode, value=c.value,
                        radius=r, families=families)
    return c, out


def test_firstorder_matches_numpy_scipy():
    rng = np.random.default_rng(3)
    for K in (1, 2, 3, 7, 27, 125, 343):
        vals = rng.gamma(2.0, 1.5, size=K)
        if K > 5:
            vals[:3] = vals[3]  # ties
        hist = np.bincount(rng.integers(0, 5, size=K), minlength=5)
        f = O.firstorder_features(vals, hist, voxel_volume=2.5)
        g = dict(zip(NAMES[:18], f))
        mu = vals.mean()
        assert g["firstorder_Mean"] == pytest.approx(mu, rel=1e-13)
        assert g["firstorder_Energy"] == pytest.approx(np.sum(vals ** 2), rel=1e-13)
        assert g["firstorder_TotalEnergy"] == pytest.approx(2.5 * np.sum(vals ** 2), rel=1e-13)
        assert g["firstorder_Variance"] == pytest.approx(np.var(vals), rel=1e-12, abs=1e-15)
        assert g["firstorder_RootMeanSquared"] == pytest.approx(np.sqrt(np.mean(vals ** 2)), rel=1e-13)
        assert g["firstorder_Minimum"] == vals.min() and g["firstorder_Maximum"] == vals.max()
        assert g["firstorder_Range"] == vals.max() - vals.min()
        for q, nm in ((10, "10Percentile"), (50, "Median"), (90, "90Percentile")):
            assert g["firstorder_" + nm] == pytest.approx(np.percentile(vals, q), rel=1e-13), nm
        iqr = np.percentile(vals, 75) - np.percentile(vals, 25)
        assert g["firstorder_InterquartileRange"] == pytest.approx(iqr, rel=1e-12, abs=1e-13)
        assert g["firstorder_MeanAbsoluteDeviation"] == pytest.approx(np.mean(np.abs(vals - mu)), rel=1e-12)
        p10, p90 = np.percentile(vals, [10, 90])
        sub = vals[(vals >= p10) & (vals <= p90)]
        if sub.size == 0:  # |V| = 2: no value lies inside [P10, P90]
            assert K == 2 and np.isnan(g["firstorder_RobustMeanAbsoluteDeviation"])
        else:
            assert g["firstorder_RobustMeanAbsoluteDeviation"] == pytest.approx(
                np.mean(np.abs(sub - sub.mean())), rel=1e-12, abs=1e-14)
        if K > 2:
            assert g["firstorder_Skewness"] == pytest.approx(stats.skew(vals, bias=True), rel=1e-10)
            assert g["firstorder_Kurtosis"] == pytest.approx(
                stats.kurtosis(vals, fisher=True, bias=True), rel=1e-10)
        ph = hist[hist > 0] / K
        assert g["firstorder_Entropy"] == pytest.approx(stats.entropy(ph, base=2), rel=1e-13, abs=1e-15)
        assert g["firstorder_Uniformity"] == pytest.approx(np.sum(ph ** 2), rel=1e-13)


def test_glcm_identities():
    """ClusterTendency + Contrast = 4 SumSquares, SumAverage = 2 JointAverage,
    DifferenceVariance = Contrast - DifferenceAverage^2,
    Autocorrelation - JointAverage^2 = Correlation * SumSquares,
    HXY1 = HXY2 = HX + HY, and the entropy/probability bounds."""
    c = synth.random_case(21, shape=(9, 10, 11), radius=2, mode=O.FBN, value=7)
    levels, ng, _, _ = O.discretise(c.volume, c.mask, c.mode, c.value)
    pts = np.argwhere(c.mask)
    for p in pts[::7]:
        mats = O.matrices(levels, c.volume, ng, tuple(int(v) for v in p), 2)
        if mats["glcm"].sum() == 0:
            continue
        f, ex = O.glcm_features(mats["glcm"])
        g = dict(zip(O.map_names(2), f))
        sc = max(1.0, abs(g["glcm_Contrast"]), abs(g["glcm_SumSquares"]))
        assert g["glcm_ClusterTendency"] + g["glcm_Contrast"] == pytest.approx(
            4 * g["glcm_SumSquares"], rel=1e-12, abs=1e-12 * sc)
        assert g["glcm_SumAverage"] == pytest.approx(2 * g["glcm_JointAverage"], rel=1e-13)
        assert g["glcm_DifferenceVariance"] == pytest.approx(
            g["glcm_Contrast"] - g["glcm_DifferenceAverage"] ** 2, rel=1e-10, abs=1e-12)
        if np.count_nonzero(mats["glcm"].sum(axis=1)) > 1:
            assert g["glcm_Autocorrelation"] - g["glcm_JointAverage"] ** 2 == pytest.approx(
                g["glcm_Correlation"] * g["glcm_SumSquares"], rel=1e-9, abs=1e-11)
        assert ex["HXY1"] == pytest.approx(ex["HX"] + ex["HY"], rel=1e-12, abs=1e-13)
        assert ex["HXY2"] == pytest.approx(ex["HX"] + ex["HY"], rel=1e-12, abs=1e-13)
        assert ex["HX"] == pytest.approx(ex["HY"], rel=1e-13, abs=1e-15)
        assert 0 < g["glcm_JointEnergy"] <= g["glcm_MaximumProbability"] <= 1
        assert g["glcm_Idm"] <= g["glcm_Id"] <= g["glcm_Idn"] + 1e-15
        assert -1e-12 <= g["glcm_MCC"] <= 1 + 1e-12
        assert -1 - 1e-12 <= g["glcm_Correlation"] <= 1 + 1e-12


def _mcc_numpy(P):
    p = P / P.sum()
    px = p.sum(axis=1)
    keep = px > 0
    p = p[np.ix_(keep, keep)]
    px = px[keep]
    if len(px) <= 1:
        return 1.0
    Q = (p[:, None, :] * p[None, :, :] / (px[:, None, None] * px[None, None, :])).sum(axis=2)
    ev = np.sort(np.linalg.eigvals(Q).real)
    return math.sqrt(max(ev[-2], 0.0))


def test_mcc_matches_general_eigensolver():
    for seed, r, nglev in [(31, 1, 5), (32, 2, 8), (33, 3, 12), (34, 2, 3)]:
        c = synth.random_case(seed, shape=(9, 10, 11), radius=r, mode=O.FBN, value=nglev)
        levels, ng, _, _ = O.discretise(c.volume, c.mask, c.mode, c.value)
        for p in np.argwhere(c.mask)[::11]:
            P = O.matrices(levels, c.volume, ng, tuple(int(v) for v in p), r)["glcm"]
            if P.sum() == 0:
                continue
            f, _ = O.glcm_features(P)
            assert f[15] == pytest.approx(_mcc_numpy(P), rel=1e-8, abs=1e-9)


def test_mcc_special_structures():
    # bipartite: two adjacent voxels of different levels -> A has eigenvalue -1
    P = np.array([[0, 1], [1, 0]], np.int64)
    assert O.glcm_features(P)[0][15] == pytest.approx(1.0, abs=1e-12)
    # block diagonal: levels {1,2} and {4,5} never co-occur -> eigenvalue 1 twice
    P = np.zeros((5, 5), np.int64)
    P[0, 0], P[0, 1], P[1, 0], P[1, 1] = 4, 3, 3, 2
    P[3, 3], P[3, 4], P[4, 3], P[4, 4] = 1, 5, 5, 6
    assert O.glcm_features(P)[0][15] == pytest.approx(1.0, abs=1e-12)
    # no pairs at all -> every GLCM map is NaN
    assert np.isnan(O.glcm_features(np.zeros((3, 3), np.int64))[0]).all()


def test_degenerate_isolated_voxel():
    vol = np.zeros((5, 5, 5), np.float32)
    mask = np.zeros((5, 5, 5), np.uint8)
    vol[2, 2, 2], mask[2, 2, 2] = 3.0, 1
    vol[0, 0, 0], mask[0, 0, 0] = 9.0, 1  # far away: not a neighbour
    out = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBN, value=4, radius=1,
                        families=ALL, sample=[1])[:, 0]
    f = dict(zip(NAMES, out))
    assert all(np.isnan(f[n]) for n in NAMES if n.startswith("glcm_"))
    assert all(np.isnan(f[n]) for n in NAMES if n.startswith("ngtdm_"))
    assert f["glrlm_RunPercentage"] == 1.0 and f["glszm_ZonePercentage"] == 1.0
    assert f["gldm_LargeDependenceEmphasis"] == 1.0
    assert f["firstorder_Mean"] == 3.0 and f["firstorder_Kurtosis"] == 0.0


def test_ngtdm_busyness_zero_denominator():
    # levels 1 and 2 with n = (2, 1): 1*2 == 2*1, so every |i p_i - j p_j| vanishes
    n = np.array([2, 1], np.int64)
    s = np.array([0.5, 1.0])
    f = O.ngtdm_features(n, s)
    assert f[2] == 0.0
    assert f[0] == pytest.approx(1.0 / (2 / 3 * 0.5 + 1 / 3 * 1.0), rel=1e-15)


# --------------------------------------------------------------------------
# whole-map invariants
# --------------------------------------------------------------------------
def test_map_equals_scalar_when_kernel_covers_voi():
    c = synth.random_case(41, shape=(4, 5, 6), radius=3, mode=O.FBN, value=5, mask_fill=0.6)
    maps = O.spatial_map(c, families=ALL)
    sc = O.scalar(c, families=ALL)
    # the cube of radius 5 covers the whole 4x5x6 image from every voxel
    maps5 = O.spatial_map(vol=c.volume, mask=c.mask, spacing=c.spacing, mode=c.mode, value=c.value,
                          radius=6, families=ALL)
    for k in range(len(NAMES)):
        np.testing.assert_allclose(maps5[k], np.full(maps5.shape[1], sc[k]), rtol=1e-12, atol=1e-12,
                                   err_msg=NAMES[k])
    assert maps.shape == maps5.shape


def _dense(maps, mask):
    out = np.full((maps.shape[0],) + mask.shape, np.nan)
    out[:, mask > 0] = maps
    return out


@pytest.mark.parametrize("r", [1, 2])
def test_cube_symmetries_move_maps(r):
    c = synth.random_case(51, shape=(7, 8, 9), radius=r, mode=O.FBN, value=6)
    base = _dense(O.spatial_map(c, families=ALL), c.mask)
    transforms = [
        lambda a: a[::-1], lambda a: a[:, ::-1], lambda a: a[:, :, ::-1],
        lambda a: np.transpose(a, (1, 0, 2)), lambda a: np.transpose(a, (2, 1, 0)),
        lambda a: np.transpose(a, (0, 2, 1))[::-1, :, ::-1],
    ]
    for T in transforms:
        vol = np.ascontiguousarray(T(c.volume))
        mask = np.ascontiguousarray(T(c.mask))
        got = _dense(O.spatial_map(vol=vol, mask=mask, spacing=c.spacing, mode=c.mode,
                                   value=c.value, radius=r, families=ALL), mask)
        want = np.stack([T(b) for b in base])
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-10)


def test_translation_invariance():
    c = synth.random_case(61, shape=(6, 7, 8), radius=2, mode=O.FBN, value=6)
    base = O.spatial_map(c, families=ALL)
    vol = np.zeros((10, 12, 9), np.float32)
    mask = np.zeros((10, 12, 9), np.uint8)
    vol[3:9, 2:9, 1:9] = c.volume
    mask[3:9, 2:9, 1:9] = c.mask
    got = O.spatial_map(vol=vol, mask=mask, spacing=c.spacing, mode=c.mode, value=c.value,
                        radius=2, families=ALL)
    np.testing.assert_allclose(got, base, rtol=1e-13, atol=1e-13)


def test_names_and_counts():
    assert O.map_count(ALL) == 93 and len(NAMES) == 93
    assert O.map_count(1 | 2) == 42
    counts = [O.map_count(1 << q) for q in range(6)]
    assert counts == [18, 24, 16, 16, 14, 5]  # Table 2 spatial benchmark column
    assert len(set(NAMES)) == 93


# --------------------------------------------------------------------------
# extraction variants: GLCM distance, GLDM alpha, averaged aggregation
# --------------------------------------------------------------------------
def _stripes3():
    z, y, x = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    vol = (x % 2 + 1).astype(np.float32)
    return vol, np.ones((3, 3, 3), np.uint8)


def test_stripes_merged_and_averaged_closed_form():
    """Hand-derived GLCM / GLRLM features of a striped cube whose directions
    differ (tests/golden/stripes3_handderived.txt): the merged maps from the
    summed counts, the averaged ones as the mean of the two per-direction
    matrix types."""
    vol, mask = _stripes3()
    gold = load_golden("stripes3_handderived.txt")
    fam = 2 | 4
    names = O.map_names(fam)
    centre = compact_index(mask, (1, 1, 1))
    merged = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBN, value=2, radius=1,
                           families=fam)[:, centre]
    avg = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBN, value=2, radius=1,
                        families=fam, averaged=True)[:, centre]
    checked = 0
    for k, name in enumerate(names):
        for prefix, got in (("avg_", avg[k]), ("merged_", merged[k])):
            if prefix + name in gold:
                want = gold[prefix + name]
                assert got == pytest.approx(want, rel=1e-12, abs=1e-12), (prefix + name, got, want)
                checked += 1
    assert checked == 24 + 6 + 12 + 4


def test_averaged_run_percentage_equals_merged():
    """By linearity the mean of the per-direction run percentages N_r,d / K is
    the merged N_r / 13K; the other features differ in general."""
    c = synth.random_case(61, shape=(7, 8, 9), radius=2, value=6)
    m = O.spatial_map(c, families=4)
    a = O.spatial_map(c, families=4, averaged=True)
    rp = O.map_names(4).index("glrlm_RunPercentage")
    np.testing.assert_allclose(a[rp], m[rp], rtol=1e-13)
    assert np.abs(a - m).max() > 1e-3


def test_averaged_equals_merged_on_constant_cube():
    vol = np.full((5, 5, 5), 3.0, np.float32)
    mask = np.ones_like(vol, np.uint8)
    for r in (1, 2):
        m = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBW, value=1.0, radius=r,
                          families=2)
        a = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBW, value=1.0, radius=r,
                          families=2, averaged=True)
        np.testing.assert_allclose(a, m, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("r,dist,pairs", [(1, 2, None), (2, 2, 603), (3, 2, 2285), (3, 3, 1516)])
def test_glcm_distance_pair_totals_on_full_cube(r, dist, pairs):
    """In a full (2r+1)^3 cube the pairs at offset d*m number prod_i (S - d|m_i|)
    for each of the 13 vectors m (3 axes, 6 face and 4 body diagonals);
    a distance of S or more leaves none."""
    S = 2 * r + 1
    if pairs is None:  # hand count for r = 1, d = 2: 3*9 + 6*3 + 4*1
        pairs = 3 * (S - 2) * S * S + 6 * (S - 2) ** 2 * S + 4 * (S - 2) ** 3
    n = 2 * r + 1 + 2 * r
    vol = np.full((n, n, n), 5.0, np.float32)
    mask = np.ones_like(vol, np.uint8)
    lev = O.discretise(vol, mask, O.FBN, 4)[0]
    m = O.matrices(lev, vol, 4, (n // 2, n // 2, n // 2), r, glcm_distance=dist)
    assert m["glcm"].sum() == 2 * pairs


def brute_glcm_dist(member, lev, ng, dist):
    """All ordered member pairs whose difference has every component in
    {-dist, 0, dist} and is not zero (the 26 vectors dist*m)."""
    pts = np.argwhere(member)
    g = lev[member]
    d = pts[:, None, :] - pts[None, :, :]
    ok = np.all((d == 0) | (np.abs(d) == dist), axis=2) & np.any(d != 0, axis=2)
    a, b = np.nonzero(ok)
    P = np.zeros((ng, ng), np.int64)
    np.add.at(P, (g[a] - 1, g[b] - 1), 1)
    return P


def brute_gldm_alpha(member, lev, ng, alpha):
    """k(v) - 1 = #26-neighbours u in V with |g_u - g_v| <= alpha, by loops."""
    D = np.zeros((ng, 27), np.int64)
    S0, S1, S2 = member.shape
    for p in zip(*np.nonzero(member)):
        k = 0
        for o in OFFS26:
            q = (p[0] + o[0], p[1] + o[1], p[2] + o[2])
            if 0 <= q[0] < S0 and 0 <= q[1] < S1 and 0 <= q[2] < S2 and member[q]:
                k += abs(int(lev[q]) - int(lev[p])) <= alpha
        D[lev[p] - 1, k] += 1
    return D


@pytest.mark.parametrize("seed,r,dist,alpha", [(71, 1, 2, 1), (72, 2, 2, 2), (73, 2, 3, 0),
                                               (74, 3, 2, 5), (75, 2, 4, 3)])
def test_variant_matrices_match_brute_force(seed, r, dist, alpha):
    c = synth.random_case(seed, shape=(8, 9, 10), radius=r, value=7)
    lev, ng, _, _ = O.discretise(c.volume, c.mask, c.mode, c.value)
    rng = np.random.default_rng(seed)
    pts = np.argwhere(c.mask)
    for s in rng.choice(len(pts), size=12, replace=False):
        ctr = tuple(int(v) for v in pts[s])
        m = O.matrices(lev, c.volume, ng, ctr, r, glcm_distance=dist, gldm_alpha=alpha)
        member, lv, _ = cube(lev, c.volume, ctr, r)
        assert np.array_equal(m["glcm"], brute_glcm_dist(member, lv, ng, dist))
        assert np.array_equal(m["gldm"], brute_gldm_alpha(member, lv, ng, alpha))
        assert m["gldm"].sum() == member.sum()


def test_gldm_alpha_covering_all_levels_on_checkerboard():
    """3x3x3 two-level checkerboard, alpha = 1 >= Ng - 1: every neighbour is
    dependent, so k(v) = 1 + the neighbours in the cube: corners (level 1)
    8, edge centres (level 2) 12, face centres (level 1) 18, the centre
    (level 2) 27."""
    z, y, x = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    vol = ((x + y + z) % 2 + 1).astype(np.float32)
    mask = np.ones((3, 3, 3), np.uint8)
    lev = O.discretise(vol, mask, O.FBN, 2)[0]
    D = O.matrices(lev, vol, 2, (1, 1, 1), 1, gldm_alpha=1)["gldm"]
    want = np.zeros((2, 27), np.int64)
    want[0, 7], want[1, 11], want[0, 17], want[1, 26] = 8, 12, 6, 1
    assert np.array_equal(D, want)
    f = O.spatial_map(vol=vol, mask=mask, spacing=(1, 1, 1), mode=O.FBN, value=2, radius=1,
                      families=16, gldm_alpha=1)[:, 13]
    names = O.map_names(16)
    lde = (8 * 64 + 12 * 144 + 6 * 324 + 729) / 27
    sde = (8 / 64 + 12 / 144 + 6 / 324 + 1 / 729) / 27
    assert f[names.index("gldm_LargeDependenceEmphasis")] == pytest.approx(lde, rel=1e-13)
    assert f[names.index("gldm_SmallDependenceEmphasis")] == pytest.approx(sde, rel=1e-13)
    assert f[names.index("gldm_GrayLevelNonUniformity")] == pytest.approx((14 ** 2 + 13 ** 2) / 27, rel=1e-13)
    assert f[names.index("gldm_DependenceNonUniformity")] == pytest.approx((64 + 144 + 36 + 1) / 27, rel=1e-13)


def test_variant_defaults_reproduce_the_plain_map():
    c = synth.random_case(76, shape=(7, 8, 9), radius=2, value=9)
    np.testing.assert_array_equal(O.spatial_map(c), O.spatial_map(c, glcm_distance=1, gldm_alpha=0,
                                                                  averaged=False))
