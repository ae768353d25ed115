"""Seeded synthetic inputs for radiomic spatial mapping.

This module only draws input volumes and masks.  It contains none of the
method's arithmetic (no discretisation, no texture counting, no features), so
both the GPU path and the CPU oracle can be fed from it without sharing any
of the computation that they are compared on.

The paper measures on a cropped breast DCE-MRI lesion (Computational
performance and Spatial concordance sections); that image is not available
here, so these volumes stand in for it with the value distributions of the
two modalities radiomic maps are usually computed on:

* CT-like int16 volumes in Hounsfield units, drawn from a three-component
  Gaussian mixture (means -50/40/120 HU, s.d. 20/15/30 HU), iid per voxel;
* PET-like float32 volumes in SUV, a gamma(shape 2, scale 1.5) background
  with a smoothed hot lesion added.

Every generator takes an integer seed and uses numpy's PCG64 stream, so a
given seed always yields the same volume.  Arrays are C-ordered [nz][ny][nx]
(x fastest); spacing tuples are (sx, sy, sz) in millimetres.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FBW = 1  # fixed bin width discretisation
FBN = 2  # fixed bin number discretisation


@dataclass
class Case:
    """One spatial-mapping job: inputs plus the settings the job uses."""

    name: str
    volume: np.ndarray          # int16 or float32, [nz][ny][nx]
    mask: np.ndarray            # uint8, [nz][ny][nx], nonzero = inside the VOI
    spacing: tuple              # (sx, sy, sz) mm
    mode: int                   # FBW or FBN
    value: float                # bin width (FBW) or bin count (FBN)
    lower: float                # FBW lower bound, NaN = VOI minimum
    radius: int                 # kernel radius in voxels (cube side 2r+1)
    families: int               # family bitmask (1 first-order ... 32 NGTDM)
    meta: dict = field(default_factory=dict)

    @property
    def n_mask(self) -> int:
        return int(np.count_nonzero(self.mask))


FAM_FIRSTORDER, FAM_GLCM, FAM_GLRLM, FAM_GLSZM, FAM_GLDM, FAM_NGTDM = 1, 2, 4, 8, 16, 32
FAM_ALL = 63


def ct_mixture(rng: np.random.Generator, shape, bone: bool = False) -> np.ndarray:
    """int16 CT-like values: equal-weight mixture N(-50,20), N(40,15), N(120,30),
    rounded half-to-even.  bone=True adds a fourth equal-weight component
    N(700, 250) (dense bone), so that a fixed bin width of 25 HU from a
    -1000 HU lower bound yields roughly 70-110 gray levels."""
    k = 4 if bone else 3
    comp = rng.integers(0, k, size=shape)
    means = np.array([-50.0, 40.0, 120.0, 700.0])[:k]
    sds = np.array([20.0, 15.0, 30.0, 250.0])[:k]
    x = rng.standard_normal(size=shape) * sds[comp] + means[comp]
    return np.rint(x).astype(np.int16)


def centred_grid(shape):
    """Index-space coordinates relative to the array centre ((n-1)/2 per axis)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) - (nz - 1) / 2.0,
                          np.arange(ny) - (ny - 1) / 2.0,
                          np.arange(nx) - (nx - 1) / 2.0, indexing="ij")
    return z, y, x


def ellipsoid_mask(shape, semi_xyz, centre_zyx=None) -> np.ndarray:
    nz, ny, nx = shape
    if centre_zyx is None:
        centre_zyx = ((nz - 1) / 2.0, (ny - 1) / 2.0, (nx - 1) / 2.0)
    z, y, x = np.meshgrid(np.arange(nz) - centre_zyx[0], np.arange(ny) - centre_zyx[1],
                          np.arange(nx) - centre_zyx[2], indexing="ij")
    a, b, c = semi_xyz
    return ((x / a) ** 2 + (y / b) ** 2 + (z / c) ** 2 <= 1.0).astype(np.uint8)


def tiny_ct(seed: int = 0) -> Case:
    """Small CT case: int16 32x32x16 (x,y,z), 1x1x2 mm, sphere of radius 8
    voxels at the array centre, fixed bin width 25 HU, radius 1,
    first-order + GLCM maps."""
    rng = np.random.default_rng(seed)
    shape = (16, 32, 32)
    vol = ct_mixture(rng, shape)
    z, y, x = centred_grid(shape)
    mask = (x * x + y * y + z * z <= 64.0).astype(np.uint8)
    return Case("ct_tiny_32x32x16_r1", vol, mask, (1.0, 1.0, 2.0), FBW, 25.0, float("nan"),
                1, FAM_FIRSTORDER | FAM_GLCM, {"modality": "CT"})


def _gamma_background(rng, shape):
    return rng.gamma(2.0, 1.5, size=shape)


def pet_lesion(seed: int = 1) -> Case:
    """PET-like case: float32 128x128x64 (x,y,z), 2x2x3 mm, gamma(2, 1.5)
    background plus 6 SUV x (ellipsoid indicator smoothed by a Gaussian of
    sigma 2 voxels); mask = the ellipsoid (semi-axes 40,30,20 voxels),
    fixed bin number 32, radius 2, all six families."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    shape = (64, 128, 128)
    bg = _gamma_background(rng, shape)
    mask = ellipsoid_mask(shape, (40.0, 30.0, 20.0))
    lesion = gaussian_filter(mask.astype(np.float64), sigma=2.0, mode="constant")
    vol = (bg + 6.0 * lesion).astype(np.float32)
    return Case("pet_128x128x64_r2_ng32", vol, mask, (2.0, 2.0, 3.0), FBN, 32.0, float("nan"),
                2, FAM_ALL, {"modality": "PET"})


def pet_large(seed: int = 4, target: int = 1_000_000) -> Case:
    """Large PET-like case: float32 256x256x128 (x,y,z), 2x2x3 mm, gamma
    background plus three Gaussian-blob lesions with seeded centres at least
    45 voxels from the borders and from each other; mask = union of three
    balls of a common radius chosen so the union holds target +- 1 % voxels;
    fixed bin number 64, radius 3, all six families."""
    rng = np.random.default_rng(seed)
    shape = (128, 256, 256)
    nz, ny, nx = shape
    centres = []
    while len(centres) < 3:
        c = (rng.uniform(45, nz - 1 - 45), rng.uniform(45, ny - 1 - 45), rng.uniform(45, nx - 1 - 45))
        if all(np.linalg.norm(np.subtract(c, d)) >= 45.0 for d in centres):
            centres.append(c)
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float32), np.arange(ny, dtype=np.float32),
                          np.arange(nx, dtype=np.float32), indexing="ij")
    d2 = [(z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2 for c in centres]
    dmin = np.minimum(np.minimum(d2[0], d2[1]), d2[2])
    lo, hi = 10.0, 80.0
    for _ in range(40):  # bisection on the common ball radius
        mid = 0.5 * (lo + hi)
        if np.count_nonzero(dmin <= mid * mid) < target:
            lo = mid
        else:
            hi = mid
    rad = hi
    mask = (dmin <= rad * rad).astype(np.uint8)
    vol = _gamma_background(rng, shape)
    for dd in d2:
        vol += 8.0 * np.exp(-dd / (2.0 * (0.6 * rad) ** 2))
    return Case("pet_256x256x128_r3_ng64", vol.astype(np.float32), mask, (2.0, 2.0, 3.0), FBN, 64.0,
                float("nan"), 3, FAM_ALL, {"modality": "PET", "ball_radius": rad, "centres": centres})


def random_case(seed: int, shape=(12, 14, 16), dtype=np.float32, radius=1, families=FAM_ALL,
                mode=FBN, value=8.0, lower=float("nan"), mask_fill=0.7, levels=None,
                bone: bool = False) -> Case:
    """Small irregular case for parity tests: random values, a random blobby
    mask (thresholded smooth noise) that has holes, isolated voxels and
    voxels on the volume border.  int16 volumes are CT-like (with a bone
    component if bone=True), float32 ones gamma(2, 1.5)."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    if dtype == np.int16:
        vol = ct_mixture(rng, shape, bone=bone)
    else:
        vol = (rng.gamma(2.0, 1.5, size=shape)).astype(np.float32)
    if levels is not None:  # few distinct raw values -> large zones and long runs
        vol = rng.integers(0, levels, size=shape).astype(dtype)
    noise = gaussian_filter(rng.standard_normal(shape), 1.2)
    thr = np.quantile(noise, 1.0 - mask_fill)
    mask = (noise >= thr).astype(np.uint8)
    return Case(f"random_{seed}", vol, mask, (1.0, 1.5, 2.5), mode, value, lower, radius, families, {})


def batch_ct(seed: int = 2, n_jobs: int = 64):
    """Batch of CT-like int16 VOIs (mixture as in tiny_ct, 1x1x2 mm), one
    PCG64 substream per VOI: ellipsoid mask with axes ratio 1 : 0.8 : 0.6
    holding s ~ log-U[1e3, 2e5] voxels, volume = mask bounding box plus an
    (r + 2)-voxel margin rounded up to a multiple of 8 per axis, fixed bin
    number Ng ~ U{16, 32, 64}, radius r ~ U{1, 2, 3}, all 93 maps."""
    seqs = np.random.SeedSequence(seed).spawn(n_jobs)
    jobs = []
    for q, ss in enumerate(seqs):
        rng = np.random.default_rng(ss)
        s = float(np.exp(rng.uniform(np.log(1e3), np.log(2e5))))
        ng = int(rng.choice([16, 32, 64]))
        r = int(rng.integers(1, 4))
        a = (s / (4.0 / 3.0 * np.pi * 0.8 * 0.6)) ** (1.0 / 3.0)
        semi = (a, 0.8 * a, 0.6 * a)  # x, y, z in voxels
        dims = []
        for ax in (semi[2], semi[1], semi[0]):  # z, y, x
            n = int(np.ceil(2 * ax + 1)) + 2 * (r + 2)
            dims.append(int(np.ceil(n / 8.0) * 8))
        shape = tuple(dims)
        vol = ct_mixture(rng, shape)
        mask = ellipsoid_mask(shape, semi)
        jobs.append(Case(f"batch{q}_r{r}_ng{ng}", vol, mask, (1.0, 1.0, 2.0), FBN, float(ng),
                         float("nan"), r, FAM_ALL, {"target_voxels": s}))
    return jobs


def _pet_voi(rng, s: float, r: int, ng: int, name: str) -> Case:
    """PET-like VOI of about s mask voxels: ellipsoid with axes ratio
    1 : 0.75 : 0.5 (the PET workload's 40 : 30 : 20), gamma(2, 1.5)
    background plus 6 SUV x the indicator smoothed by a Gaussian of sigma 2,
    volume = bounding box plus an (r + 2)-voxel margin rounded up to 8."""
    from scipy.ndimage import gaussian_filter

    a = (s / (4.0 / 3.0 * np.pi * 0.75 * 0.5)) ** (1.0 / 3.0)
    semi = (a, 0.75 * a, 0.5 * a)
    dims = [int(np.ceil((int(np.ceil(2 * ax + 1)) + 2 * (r + 2)) / 8.0) * 8)
            for ax in (semi[2], semi[1], semi[0])]
    shape = tuple(dims)
    bg = _gamma_background(rng, shape)
    mask = ellipsoid_mask(shape, semi)
    lesion = gaussian_filter(mask.astype(np.float64), sigma=2.0, mode="constant")
    vol = (bg + 6.0 * lesion).astype(np.float32)
    return Case(name, vol, mask, (2.0, 2.0, 3.0), FBN, float(ng), float("nan"), r, FAM_ALL,
                {"modality": "PET", "target_voxels": s})


def _ct_voi(rng, s: float, r: int, ng: int, name: str) -> Case:
    """CT-like VOI as in batch_ct (axes 1 : 0.8 : 0.6, 1x1x2 mm)."""
    a = (s / (4.0 / 3.0 * np.pi * 0.8 * 0.6)) ** (1.0 / 3.0)
    semi = (a, 0.8 * a, 0.6 * a)
    dims = [int(np.ceil((int(np.ceil(2 * ax + 1)) + 2 * (r + 2)) / 8.0) * 8)
            for ax in (semi[2], semi[1], semi[0])]
    shape = tuple(dims)
    vol = ct_mixture(rng, shape)
    mask = ellipsoid_mask(shape, semi)
    return Case(name, vol, mask, (1.0, 1.0, 2.0), FBN, float(ng), float("nan"), r, FAM_ALL,
                {"modality": "CT", "target_voxels": s})


def serve_pool(seed: int = 3, n: int = 32):
    """Input pool of the served stream: n VOIs, one PCG64 substream each,
    PET-like (probability 1/2, as the PET workload) or CT-like (as batch_ct),
    mask size s ~ log-U[5e3, 4e5] voxels.  The volume margin is sized for
    radius 3 so that any radius can be applied to every entry."""
    seqs = np.random.SeedSequence([seed, 0]).spawn(n)
    pool = []
    for q, ss in enumerate(seqs):
        rng = np.random.default_rng(ss)
        pet = bool(rng.random() < 0.5)
        s = float(np.exp(rng.uniform(np.log(5e3), np.log(4e5))))
        mk = _pet_voi if pet else _ct_voi
        pool.append(mk(rng, s, 3, 32, f"pool{q}_{'pet' if pet else 'ct'}"))
    return pool


def serve_jobs(seed: int = 3, n_jobs: int = 2000, pool_size: int = 32):
    """Job stream of the served workload: per job a pool entry (uniform),
    Ng ~ U{16, 32, 64} (fixed bin number) and radius r ~ U{1, 2, 3}, all 93
    maps; returns a list of (pool index, Ng, r)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 1]))
    idx = rng.integers(0, pool_size, size=n_jobs)
    ng = rng.choice([16, 32, 64], size=n_jobs)
    r = rng.integers(1, 4, size=n_jobs)
    return [(int(a), int(b), int(c)) for a, b, c in zip(idx, ng, r)]


def poisson_arrivals(seed: int, n_jobs: int, rate: float):
    """Arrival times (s, from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2]))
    return np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
