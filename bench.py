"""Benchmark: mask voxels mapped per second, plain spatial map, one MI355X.

Headline workload (default, the largest single-GPU configuration): the
PET-like float32 256x256x128 volume (2x2x3 mm), gamma background plus three
Gaussian-blob lesions, mask = union of three balls holding 1.00 M voxels,
fixed bin number Ng = 64, kernel radius 3 (7x7x7), all six families (93
maps, 0.372 GB of float32 output).  Inputs are synthetic and seeded and
resident in HBM before timing.

One step = one fr_map call: discretisation kernels, the fused map kernel
and the transpose into the map-major output, enqueued on one stream.  The
JSON line carries:
  roofline      the map kernel's algorithmic HBM bytes, LDS bytes and FP64
                flops per voxel (from the kernel's own bit-exact integer
                matrices of a seeded voxel sample) over its measured time,
                each against the peak re-measured on this GPU (stream copy,
                ds_read_b32, FP64 FMA); "bound" names the resource with the
                largest fraction
  cpu_baseline  the FP64 oracle on this host: median/min/max of 5 runs on
                all cores and on one core, over seeded voxel samples
  secondary     the PET 128x128x64 (r = 2, Ng = 32, 100,544 voxels) workload
  batched       (--batch) 64 CT-like VOIs: 64 plain fr_map calls vs one
                batched launch
  served        a Poisson stream of jobs through the continuous-batching server

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|pet|ct]
                  [--batch] [--serve-jobs N] [--no-cpu-baseline] [--no-ops]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 flops charged per logarithm in the entropy terms (a frexp, one
# reciprocal and a degree-15 odd series: about twenty FP64 operations).
FLOPS_PER_LOG2 = 20.0


def workload(name: str):
    from paper_2609_19190_amd import synth
    if name == "pet":
        return synth.pet_lesion(1)
    if name == "ct":
        return synth.tiny_ct(0)
    if name == "large":
        return synth.pet_large(4)
    raise SystemExit(f"unknown workload {name}")


def measure_peaks():
    """HBM copy, LDS read / atomic-add and FP64 FMA peaks of this GPU
    (libfrpeaks.so, built beside the library)."""
    path = os.path.join(ROOT, "paper_2609_19190_amd", "libfrpeaks.so")
    if not os.path.exists(path):
        raise SystemExit(f"{path} is missing: run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    L.frp_measure.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.frp_measure.restype = ctypes.c_int
    buf = (ctypes.c_double * 5)()
    if L.frp_measure(buf, 5, 1024) != 0:
        raise RuntimeError("frp_measure failed")
    return {"hbm_GBs": buf[0], "lds_GBs": buf[1], "lds_atomic_GBs": buf[2],
            "fp64_TFLOPs": buf[3], "cus": int(buf[4]), "source": "measured on this GPU"}


def algorithmic_counts(B, vol, mask, case, ng, n_sample=1024, seed=0):
    """Mean algorithmic work per voxel of the map kernel, from the kernel's
    own integer matrices of a seeded sample of voxels (they are bit-exact
    against the oracle in the parity tests).  With K = |V|, P = neighbour
    pairs in V (sum GLCM / 2), R = runs (sum GLRLM), L' = present GLCM
    levels, Ln = levels with an NGTDM voxel and nnz = the non-zero entries the
    feature sums read (GLCM upper triangle, GLRLM, GLSZM, GLDM, NGTDM):
      LDS bytes = 4 (4 P + R + K + nnz)      GLCM increments, GLDM and NGTDM
                  neighbour reads, zone-union edges, run increments,
                  histogram, feature reads (4-byte LDS operations)
      FP64 flops = 30 (nnz(GLCM upper) + Ln (Ln - 1) / 2)
                   + 20 x (one logarithm per non-zero entropy term)
                   + 4/3 L'^3 (Householder tridiagonalisation for the MCC)
    HBM bytes per voxel (not sampled): the maps written (4 B each) plus the
    level (1 B) and raw value (2 or 4 B) of every voxel of the mask's
    bounding box grown by r, and the 4-byte mask-voxel index, per mask voxel."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    ns = min(n_sample, case.n_mask)
    samp = np.sort(rng.choice(case.n_mask, size=ns, replace=False)).astype(np.int64)
    res = B.fr_map_matrices(vol, mask, case.spacing, case.mode, case.value, case.lower,
                            case.radius, case.families, case.n_mask, torch.from_numpy(samp), ng)
    torch.cuda.synchronize()
    P = res["glcm"].cpu().numpy().astype(np.int64)
    R = res["glrlm"].cpu().numpy()
    Z = res["glszm"].cpu().numpy()
    D = res["gldm"].cpu().numpy()
    n = res["ngtdm_n"].cpu().numpy()
    H = res["hist"].cpu().numpy()
    K = H.sum(axis=1).astype(np.float64)
    pairs = P.sum(axis=(1, 2)) / 2.0
    runs = R.sum(axis=(1, 2)).astype(np.float64)
    upper = np.triu(np.ones(P.shape[1:], bool))
    nnz_glcm = ((P > 0) & upper).sum(axis=(1, 2)).astype(np.float64)
    lp = (P.sum(axis=2) > 0).sum(axis=1).astype(np.float64)
    ln = (n > 0).sum(axis=1).astype(np.float64)
    nnz_r = (R > 0).sum(axis=(1, 2))
    nnz_z = (Z > 0).sum(axis=(1, 2))
    nnz_d = (D > 0).sum(axis=(1, 2))
    # entropy terms: joint (GLCM), marginal, |i-j| and i+j histograms, level
    # histogram, runs, zones, dependences
    g = np.arange(1, P.shape[1] + 1)
    nd = np.empty(ns)
    nsm = np.empty(ns)
    for q in range(ns):
        ii, jj = np.nonzero(P[q])
        nd[q] = np.unique(np.abs(g[ii] - g[jj])).size
        nsm[q] = np.unique(g[ii] + g[jj]).size
    logs = nnz_glcm + lp + nd + nsm + (H > 0).sum(axis=1) + nnz_r + nnz_z + nnz_d
    nnz = nnz_glcm + nnz_r + nnz_z + nnz_d + ln
    lds = 4.0 * (4 * pairs + runs + K + nnz)
    flops = 30.0 * (nnz_glcm + ln * (ln - 1) / 2) + FLOPS_PER_LOG2 * logs + (4.0 / 3.0) * lp ** 3
    # HBM: bounding box of the mask grown by r (clipped to the image)
    idx = np.argwhere(case.mask)
    lo = np.maximum(idx.min(axis=0) - case.radius, 0)
    hi = np.minimum(idx.max(axis=0) + case.radius + 1, case.mask.shape)
    nbox = float(np.prod(hi - lo))
    esize = case.volume.dtype.itemsize
    count = B.fr_map_count(case.families)
    hbm = 4.0 * count + 4.0 + (1.0 + esize) * nbox / case.n_mask
    return dict(hbm_bytes=hbm, lds_bytes=float(lds.mean()), fp64_flops=float(flops.mean()),
                K=float(K.mean()), pairs=float(pairs.mean()), runs=float(runs.mean()),
                L_mcc=float(lp.mean()), nnz=float(nnz.mean()), sample=int(ns))


def roofline(counts, M, kernel_ms, peaks, traffic, kernel_name):
    """Per-resource achieved rate of the map kernel (algorithmic work per
    launch / measured launch time) against the measured peak."""
    t = kernel_ms / 1e3
    res = {
        "hbm": {"achieved": counts["hbm_bytes"] * M / t / 1e9, "peak": peaks["hbm_GBs"], "unit": "GB/s",
                "per_voxel": counts["hbm_bytes"]},
        "lds": {"achieved": counts["lds_bytes"] * M / t / 1e9, "peak": peaks["lds_GBs"], "unit": "GB/s",
                "per_voxel": counts["lds_bytes"]},
        "fp64": {"achieved": counts["fp64_flops"] * M / t / 1e12, "peak": peaks["fp64_TFLOPs"],
                 "unit": "TFLOP/s", "per_voxel": counts["fp64_flops"]},
    }
    for v in res.values():
        v["frac"] = v["achieved"] / v["peak"]
    bound = max(res, key=lambda k: res[k]["frac"])
    b = res[bound]
    return {"bound": bound, "achieved": b["achieved"], "peak": b["peak"], "unit": b["unit"],
            "frac": b["frac"], "traffic": traffic, "kernel": kernel_name, "kernel_ms": kernel_ms,
            "kernel_source": kernel_source_hash(), "resources": res,
            "counts": {k: v for k, v in counts.items() if k not in ("hbm_bytes", "lds_bytes", "fp64_flops")},
            "peaks": peaks}


# whether the loaded library was built from this tree's sources (set by main)
LIBRARY_MATCHES = True


def kernel_source_hash() -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_2609_19190_amd", "csrc", "map_kernel.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(workload_name: str):
    """HBM bytes per map-kernel launch from the committed rocprofv3 PMC summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a copy of
    known size); None when that summary was taken on another kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_map_{workload_name}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash() or not LIBRARY_MATCHES:
        return None
    return float(kv["traffic_bytes_per_launch"])


def measured_valu(workload_name: str, n_mask: int, kernel_ms: float):
    """VALU issue of the map kernels from the committed rocprofv3 SQ summary
    (SQ_INSTS_VALU per voxel of k_map and per problem of k_mcc, one problem
    per voxel): issue cycles (4 per wave64 VALU instruction on a 16-lane
    SIMD) over the SIMD cycles of the measured map-kernel time at the 2.4 GHz
    engine clock on 1,024 SIMDs.  None when that summary was taken on another
    kernel source or the library is not this tree's."""
    path = os.path.join(ROOT, "profiles", f"k_map_{workload_name}_sq_counters.txt")
    if not os.path.exists(path) or not LIBRARY_MATCHES:
        return None
    per_voxel, section, src = {}, None, None
    for line in open(path):
        if line.startswith("kernel_source_sha256_16:"):
            src = line.split(":", 1)[1].strip()
        elif line.startswith("["):
            section = line[1:line.index("]")]
        elif line.startswith("SQ_INSTS_VALU:") and section:
            per_voxel[section] = float(line.split("per_voxel:")[1])
    if src != kernel_source_hash() or not per_voxel:
        return None
    valu = sum(per_voxel.values())
    issue_cycles = valu * n_mask * 4.0
    simd_cycles = 1024 * 2.4e9 * kernel_ms / 1e3
    return {"valu_insts_per_voxel": valu, "by_kernel": per_voxel, "issue_utilisation": issue_cycles / simd_cycles,
            "cycles_per_inst": 4, "clock_GHz": 2.4, "simds": 1024, "source": os.path.relpath(path, ROOT)}


def _cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def cpu_baseline(case, all_core_s=3.0, one_core_s=1.5, runs=5):
    """The FP64 oracle as it stands, on this host: `runs` timed runs on all
    cores (seeded sample sized for about all_core_s each) and on one core
    (about one_core_s each); median, min and max voxels/s of each."""
    import numpy as np
    from oracle import oracle as O
    ncpu = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", ncpu))
    threads = max(1, min(threads, ncpu))
    rng = np.random.default_rng(123)

    def rate(samp, nt):
        t0 = time.perf_counter()
        O.spatial_map(case, sample=samp, nthreads=nt)
        return samp.size / (time.perf_counter() - t0)

    def leg(nt, target_s):
        probe = np.sort(rng.choice(case.n_mask, size=min(200 * nt, case.n_mask), replace=False))
        r0 = rate(probe, nt)  # calibration (also warms the page cache)
        n = int(min(case.n_mask, max(100, r0 * target_s)))
        samp = np.sort(rng.choice(case.n_mask, size=n, replace=False))
        rs = sorted(rate(samp, nt) for _ in range(runs))
        return {"median": rs[len(rs) // 2], "min": rs[0], "max": rs[-1], "voxels_per_run": n,
                "threads": nt}

    all_c = leg(threads, all_core_s)
    one_c = leg(1, one_core_s)
    return {"value": all_c["median"], "unit": "mask voxels/s", "cores": threads, "kind": "oracle",
            "sample": f"median of {runs} runs over {all_c['voxels_per_run']} seeded random mask voxels "
                      f"of the same workload on {threads} threads (min {all_c['min']:.0f}, max "
                      f"{all_c['max']:.0f}); each run includes the oracle's discretisation of the "
                      f"whole volume",
            "all_cores": all_c, "one_core": one_c, "cpu_model": _cpu_model(), "nproc": ncpu}


def batch_leg_child(steps: int, warmup: int, timeout_s: float = 600.0):
    """The batched leg in a child process (this script with --batch-leg-only):
    its record, or what went wrong, without risking the rest of the run."""
    cmd = [sys.executable, os.path.abspath(__file__), "--batch-leg-only", "--steps", str(steps),
           "--warmup", str(warmup)]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout_s)
    except subprocess.TimeoutExpired:
        return {"error": f"batched leg exceeded {timeout_s:.0f} s"}
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"batched leg exited with status {r.returncode}",
                "stderr_tail": r.stderr.strip().splitlines()[-3:]}
    return json.loads(lines[-1])


def batch_leg(B, steps: int, warmup: int):
    """64 CT-like VOIs of uneven size and mixed (Ng, r): 64 plain fr_map calls
    per step against one batched launch per step (autotuned, replayed from a
    HIP graph), both from resident inputs; the batched maps must equal the
    plain ones bit for bit."""
    import torch
    from paper_2609_19190_amd import synth
    cases = synth.batch_ct()
    dev = torch.device("cuda:0")
    vols = [torch.from_numpy(c.volume).to(dev) for c in cases]
    masks = [torch.from_numpy(c.mask).to(dev) for c in cases]
    outs = [torch.empty((B.fr_map_count(c.families), c.n_mask), dtype=torch.float32, device=dev)
            for c in cases]
    total = sum(c.n_mask for c in cases)
    stream = torch.cuda.Stream()

    def plain_step():
        for c, v, m, o in zip(cases, vols, masks, outs):
            B.fr_map(v, m, c.spacing, c.mode, c.value, c.lower, c.radius, c.families, c.n_mask,
                     out=o, stream=stream)

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        stream.synchronize()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plain_step()
        plain_ms = timed(plain_step, steps)
        bt = B.Batch([dict(volume=v, mask=m, spacing=c.spacing, mode=c.mode, value=c.value,
                           lower=c.lower, radius=c.radius, families=c.families, n_mask=c.n_mask)
                      for c, v, m in zip(cases, vols, masks)])
        bt.autotune(stream=stream)
        graph_step = lambda: bt.launch(stream=stream, use_graph=True)
        for _ in range(warmup):
            graph_step()
        batched_ms = timed(graph_step, steps)
        eager_ms = timed(lambda: bt.launch(stream=stream), steps)
        rc, st, _ = bt.status(stream=stream)
    torch.cuda.synchronize()
    identical = rc == 0 and all(torch.equal(o.view(torch.int32), q.view(torch.int32))
                                for o, q in zip(outs, bt.outs))
    plan = bt.describe()
    bt.close()
    return {"workload": "batch_ct_64: 64 int16 CT-like VOIs, masks log-U[1e3,2e5] voxels, "
                        "Ng in {16,32,64}, r in {1,2,3}, 93 maps",
            "mask_voxels": total, "jobs": len(cases), "steps": steps, "warmup": warmup,
            "plain_value": total / (plain_ms / 1e3), "plain_ms_per_step": plain_ms,
            "batched_value": total / (batched_ms / 1e3), "batched_ms_per_step": batched_ms,
            "batched_eager_ms_per_step": eager_ms, "speedup": plain_ms / batched_ms,
            "graph": True, "identical_to_plain": bool(identical), "plan": plan,
            "unit": "mask voxels/s"}


def serve_leg(B, n_jobs: int, load: float = 0.8, slots: int = 4, budget_gib: float = 8.0,
              with_large: bool = True, max_bypass: int = 8):
    """Served stream: n_jobs map jobs drawn from a 32-VOI pool (PET- or
    CT-like, masks log-U[5e3, 4e5], Ng in {16,32,64}, r in {1,2,3}) arriving
    as a Poisson process at `load` x the plain path's measured job capacity,
    plus the 1M-voxel large job once in the middle of the stream; latency is
    counted from each job's scheduled arrival to its completion."""
    import numpy as np
    import torch
    from paper_2609_19190_amd import synth
    pool = synth.serve_pool(3, 32)
    dev = torch.device("cuda:0")
    pdev = [(torch.from_numpy(c.volume).to(dev), torch.from_numpy(c.mask).to(dev)) for c in pool]
    jobs = synth.serve_jobs(3, n_jobs, len(pool))
    specs = [(pool[pi], pdev[pi], ng, r) for pi, ng, r in jobs]
    if with_large:
        big = synth.pet_large(4)
        bdev = (torch.from_numpy(big.volume).to(dev), torch.from_numpy(big.mask).to(dev))
        specs.insert(n_jobs // 2, (big, bdev, int(big.value), big.radius))
    torch.cuda.synchronize()

    def plain(spec):
        c, (v, m), ng, r = spec
        return B.fr_map(v, m, c.spacing, c.mode, float(ng), c.lower, r, c.families, c.n_mask)

    # plain capacity: the first 48 jobs of the stream, one fr_map after another
    sample = specs[:48]
    for sp in sample[:4]:
        plain(sp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sp in sample:
        plain(sp)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    sample_vox = sum(sp[0].n_mask for sp in sample)
    rate = load * len(sample) / plain_s
    arrivals = synth.poisson_arrivals(3, len(specs), rate)

    srv = B.Server(int(budget_gib * (1 << 30)), slots, max_bypass)
    try:
        # saturated: the same 48 jobs submitted at once
        t0 = time.perf_counter()
        ts = [srv.submit_case(c, v, m, radius=r, value=float(ng)) for c, (v, m), ng, r in sample]
        for t in ts:
            srv.wait(t)
        sat_s = time.perf_counter() - t0
        for t in ts:
            srv.release(t)
        srv2_base = srv.stats()
        # open-loop Poisson stream
        lat, done_t = [], []
        tick_arrival = {}
        start = time.monotonic()
        i = 0
        n = len(specs)
        while len(lat) < n:
            now = time.monotonic() - start
            while i < n and arrivals[i] <= now:
                c, (v, m), ng, r = specs[i]
                t = srv.submit_case(c, v, m, radius=r, value=float(ng))
                tick_arrival[t] = start + arrivals[i]
                i += 1
            for t in srv.poll():
                res = srv.result(t)
                if res.status != 0:
                    raise RuntimeError(f"served job failed with status {res.status}")
                lat.append((res.t_done - tick_arrival[t]) * 1e3)
                done_t.append(res.t_done)
                srv.release(t)
            nxt = (arrivals[i] - (time.monotonic() - start)) if i < n else 0.001
            time.sleep(min(max(nxt, 0.0), 0.0005))
        st = srv.stats()
    finally:
        srv.close()
    vox = sum(sp[0].n_mask for sp in specs)
    span = max(done_t) - (start + arrivals[0])
    lat = np.sort(np.array(lat))
    rank = lambda q: float(lat[max(int(np.ceil(q * lat.size)) - 1, 0)])
    return {"workload": f"served: {len(specs)} jobs ({n_jobs} from a 32-VOI PET/CT pool, masks "
                        "log-U[5e3,4e5], Ng in {16,32,64}, r in {1,2,3}"
                        + (", plus the 1M-voxel 256x256x128 job" if with_large else "") + "), "
                        f"Poisson arrivals at {load} x plain capacity",
            "jobs": len(specs), "arrival_rate_jobs_per_s": rate, "load": load,
            "plain_capacity_jobs_per_s": len(sample) / plain_s,
            "value": vox / span, "unit": "mask voxels/s", "p50_ms": rank(0.50),
            "p99_ms": rank(0.99), "mean_ms": float(lat.mean()), "max_ms": float(lat[-1]),
            "slots": slots, "arena_gib": budget_gib, "max_bypass": max_bypass,
            "max_inflight": st["max_inflight"],
            "arena_peak_bytes": st["arena_peak_bytes"],
            "saturated": {"jobs": len(sample), "mask_voxels": sample_vox,
                          "plain_value": sample_vox / plain_s, "served_value": sample_vox / sat_s,
                          "speedup": plain_s / sat_s,
                          "max_inflight": srv2_base["max_inflight"]}}


def plain_leg(B, case, steps: int, warmup: int, with_counts: bool, peaks, traffic_name=None,
              repeats: bool = True):
    """steps timed fr_map calls on resident inputs; the map kernel's own time
    from the library's HIP events on the call stream; the roofline of it."""
    import torch
    dev = torch.device("cuda:0")
    vol = torch.from_numpy(case.volume).to(dev)
    mask = torch.from_numpy(case.mask).to(dev)
    M = case.n_mask
    count = B.fr_map_count(case.families)
    out = torch.empty((count, M), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        B.fr_map(vol, mask, case.spacing, case.mode, case.value, case.lower, case.radius,
                 case.families, M, out=out, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    B.fr_profile_enable(True)
    B.fr_profile_read()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = B.fr_profile_read()
    B.fr_profile_enable(False)
    ms_per_step = (t1 - t0) * 1e3 / steps
    kern_avg_ms = kern_ms / max(launches, 1)
    # spread: five more blocks of `steps` calls, each timed like the first
    reps = []
    for _ in range(5 if repeats else 0):
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - r0) * 1e3 / steps)
    reps.sort()
    _, ng, _, _, _ = B.fr_discretise(vol, mask, case.mode, case.value, case.lower)
    leg = {"value": M / (ms_per_step / 1e3), "ms_per_step": ms_per_step, "kernel_ms": kern_avg_ms,
           "repeats": ({"blocks": len(reps), "median_ms_per_step": reps[len(reps) // 2],
                        "min_ms_per_step": reps[0], "max_ms_per_step": reps[-1]} if reps else None),
           "config": {"workload": case.name, "mask_voxels": M,
                      "volume_xyz": list(case.volume.shape[::-1]), "raw_dtype": str(case.volume.dtype),
                      "radius": case.radius, "discretisation": "FBN" if case.mode == 2 else "FBW",
                      "ng": ng, "maps": count}}
    if with_counts:
        counts = algorithmic_counts(B, vol, mask, case, ng)
        leg["roofline"] = roofline(counts, M, kern_avg_ms, peaks,
                                   measured_traffic(traffic_name) if traffic_name else None,
                                   "k_map (fused map kernel)")
        # the limit the three-resource model does not count
        leg["roofline"]["valu_issue"] = measured_valu(traffic_name, M, kern_avg_ms) if traffic_name else None
    del vol, mask, out
    torch.cuda.empty_cache()
    return leg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "pet", "ct"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ops", action="store_true", help="skip the roofline's voxel sample")
    ap.add_argument("--no-secondary", action="store_true", help="skip the PET 128x128x64 leg")
    ap.add_argument("--no-repeats", action="store_true",
                    help="skip the five extra timed blocks that give the spread of a step")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-VOI plain-vs-batched leg (it runs in a child process, so "
                         "a failure there costs only its own record)")
    ap.add_argument("--batch", action="store_true", help=argparse.SUPPRESS)  # the default now
    ap.add_argument("--batch-leg-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--serve-jobs", type=int, default=2000,
                    help="jobs of the served Poisson stream (0: skip the served leg)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device (PMC calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the spatial-mapping path here is single-GPU "
              "(sharding across GPUs is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_19190_amd import binding as B
    from paper_2609_19190_amd import build as PB

    if args.batch_leg_only:  # the child process of the batched leg
        print(json.dumps(batch_leg(B, args.steps, args.warmup)), flush=True)
        return

    global LIBRARY_MATCHES
    library = {"source_hash": B.fr_source_hash(), "tree_hash": PB.source_hash()}
    library["matches"] = LIBRARY_MATCHES = library["source_hash"] == library["tree_hash"]
    if not LIBRARY_MATCHES:
        print(f"# WARNING: the library was built from other sources ({library['source_hash']}) than "
              f"this tree ({library['tree_hash']}): rebuild before measuring", file=sys.stderr, flush=True)

    peaks = measure_peaks() if not args.no_ops else None
    if peaks:
        peaks["spec"] = {"hbm_GBs": 8000.0, "lds_GBs": 256 * 128 * 2.4, "fp64_TFLOPs": 78.6}
    case = workload(args.workload)
    print(f"# headline {case.name}: {case.n_mask} voxels", file=sys.stderr, flush=True)
    head = plain_leg(B, case, args.steps, args.warmup, not args.no_ops, peaks, args.workload,
                     not args.no_repeats)
    if args.copy_mib:
        dev = torch.device("cuda:0")
        src = torch.ones(args.copy_mib * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    secondary = None
    if not args.no_secondary and args.workload != "pet":
        print("# secondary pet_128x128x64", file=sys.stderr, flush=True)
        secondary = plain_leg(B, workload("pet"), args.steps, args.warmup, not args.no_ops, peaks,
                              "pet", not args.no_repeats)
    batched = None
    if not args.no_batch:
        print("# batched leg (child process)", file=sys.stderr, flush=True)
        batched = batch_leg_child(min(args.steps, 10), max(args.warmup, 1))
    served = None
    if args.serve_jobs > 0:
        print("# served leg", file=sys.stderr, flush=True)
        served = serve_leg(B, args.serve_jobs)
    cpu = None
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(case)

    rec = {
        "metric": "mask voxels mapped/s (all map families), plain vs batched; p50/p99 job latency",
        "value": head["value"],
        "unit": "mask voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "output_dtype": "f32",
        "arithmetic": "integer texture matrices (int32/int64), FP64 features, float32 maps",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head.get("roofline"),
        "cpu_baseline": cpu,
        "secondary": secondary,
        "batched": batched,
        "served": served,
        "library": library,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
