"""Benchmark: mask voxels mapped per second, plain spatial map, one MI355X.

Workload (default): the PET-like float32 128x128x64 volume (2x2x3 mm),
gamma background plus a smoothed hot ellipsoid, ellipsoid mask of 100,544
voxels, fixed bin number Ng = 32, kernel radius 2 (5x5x5), all six families
(93 maps).  Inputs are synthetic and seeded, resident in HBM before timing.

One step = one fr_map call: discretisation kernels, the one host sync that
reads Ng and the mask count, the fused map kernel and the transpose into the
map-major output.  Prints one JSON line with the roofline and CPU-oracle
baseline objects, and a "batched" object: 64 CT-like VOIs of uneven size and
mixed (Ng, r), mapped by 64 plain fr_map calls per step and by one autotuned
batched launch per step replayed from a HIP graph; and a "served" object: a
Poisson stream of map jobs through the continuous-batching server, with
throughput and p50/p99 latency.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pet|ct|large]
                  [--no-batch] [--serve-jobs N] [--no-cpu-baseline] [--no-ops]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Per-lane-cycle peak of 32-bit integer / FP64 vector operations:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (the 78.6 TFLOP/s FP64 figure counts
# an FMA as two flops).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def workload(name: str):
    from paper_2609_19190_amd import synth
    if name == "pet":
        return synth.pet_lesion(1)
    if name == "ct":
        return synth.tiny_ct(0)
    if name == "large":
        return synth.pet_large(4)
    raise SystemExit(f"unknown workload {name}")


def algorithmic_ops(B, vol, mask, case, ng, n_sample=2048, seed=0):
    """Mean algorithmic lane-operations per voxel, from the kernel's own
    integer matrices of a seeded sample of voxels:
      39 K              26 neighbour tests + 13 run-continuation tests per voxel of V
      + P + E_eq + K    GLCM pair increments, zone unions, histogram
      + K ceil(log2 K)  order statistics
      + 18 K + 24 nnz(GLCM) + 16 nnz(GLRLM) + 16 zones + 14 nnz(GLDM) + 5 Ln^2
                        one term per matrix entry of each feature sum
      + 4/3 L'^3        Householder tridiagonalisation for MCC
    """
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
    eq = np.einsum("sii->s", P) / 2.0
    lp = (P.sum(axis=2) > 0).sum(axis=1).astype(np.float64)
    ln = (n > 0).sum(axis=1).astype(np.float64)
    ops = (39 * K + pairs + eq + K + K * np.ceil(np.log2(np.maximum(K, 1))) + 18 * K
           + 24 * (P > 0).sum(axis=(1, 2)) + 16 * (R > 0).sum(axis=(1, 2)) + 16 * Z.sum(axis=(1, 2))
           + 14 * (D > 0).sum(axis=(1, 2)) + 5 * ln ** 2 + (4.0 / 3.0) * lp ** 3)
    return float(ops.mean()), dict(K=float(K.mean()), pairs=float(pairs.mean()),
                                   L_mcc=float(lp.mean()), sample=int(ns))


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
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_baseline(case, target_s=30.0):
    """The FP64 oracle on a seeded sample of the same workload, all host cores."""
    import numpy as np
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    rng = np.random.default_rng(123)
    # calibrate on a small sample, then size the timed sample to ~target_s of wall time
    probe = np.sort(rng.choice(case.n_mask, size=min(2000, case.n_mask), replace=False))
    t0 = time.perf_counter()
    O.spatial_map(case, sample=probe, nthreads=threads)
    rate = probe.size / max(time.perf_counter() - t0, 1e-6)   # voxels per wall second
    # about target_s core-seconds of oracle work (at most the whole workload)
    n = int(min(case.n_mask, max(2000, rate * target_s / threads)))
    samp = np.sort(rng.choice(case.n_mask, size=n, replace=False))
    t0 = time.perf_counter()
    O.spatial_map(case, sample=samp, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "mask voxels/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} seeded random mask voxels of the same workload, family mask {case.families}, "
                      f"{dt:.1f} s wall on {threads} threads"}


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
              with_large: bool = True):
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

    srv = B.Server(int(budget_gib * (1 << 30)), slots)
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
            "slots": slots, "arena_gib": budget_gib, "max_inflight": st["max_inflight"],
            "arena_peak_bytes": st["arena_peak_bytes"],
            "saturated": {"jobs": len(sample), "mask_voxels": sample_vox,
                          "plain_value": sample_vox / plain_s, "served_value": sample_vox / sat_s,
                          "speedup": plain_s / sat_s,
                          "max_inflight": srv2_base["max_inflight"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pet", choices=["pet", "ct", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ops", action="store_true", help="skip the algorithmic-op sample")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-VOI plain-vs-batched leg")
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

    case = workload(args.workload)
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    B.fr_profile_enable(True)
    B.fr_profile_read()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = B.fr_profile_read()
    B.fr_profile_enable(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kern_avg_ms = kern_ms / max(launches, 1)
    value = M / (ms_per_step / 1e3)

    _, ng, _, _, _ = B.fr_discretise(vol, mask, case.mode, case.value, case.lower)
    if args.copy_mib:
        src = torch.ones(args.copy_mib * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    roof = {"bound": "alu", "achieved": None, "peak": ALU_PEAK_TOPS, "unit": "Top/s",
            "frac": None, "traffic": measured_traffic(args.workload),
            "kernel": "k_map (fused map kernel)", "kernel_ms": kern_avg_ms,
            "kernel_source": kernel_source_hash()}
    if not args.no_ops:
        per_vox, detail = algorithmic_ops(B, vol, mask, case, ng)
        achieved = per_vox * M / (kern_avg_ms / 1e3) / 1e12
        roof.update(achieved=achieved, frac=achieved / ALU_PEAK_TOPS, ops_per_voxel=per_vox,
                    ops_detail=detail)
    batched = None
    if not args.no_batch:
        batched = batch_leg(B, min(args.steps, 10), max(args.warmup, 1))
    served = None
    if args.serve_jobs > 0:
        served = serve_leg(B, args.serve_jobs)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case)

    rec = {
        "metric": "mask voxels mapped/s (all map families), plain vs batched; p50/p99 job latency",
        "value": value,
        "unit": "mask voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "mask_voxels": M, "volume_xyz": list(case.volume.shape[::-1]),
                   "raw_dtype": str(case.volume.dtype), "radius": case.radius,
                   "discretisation": "FBN" if case.mode == 2 else "FBW", "ng": ng, "maps": count},
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
