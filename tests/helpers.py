"""Shared helpers of the GPU parity tests: device inputs and the parity rule.

Parity rule (integer work bit-exact; float maps): a value passes when
|gpu - oracle| <= max(1e-7, 1e-5 |oracle|), and the non-finite pattern of
both sides must be identical.  The paper's concordance report (exact vs
non-exact-but-concordant, worst absolute/relative difference per map, CPU-CUDA
concordance section) is mirrored by `parity_report`.
"""
import numpy as np

ABS_TOL = 1e-7
REL_TOL = 1e-5


def to_dev(case):
    import torch
    vol = torch.from_numpy(np.ascontiguousarray(case.volume)).to("cuda:0")
    mask = torch.from_numpy(np.ascontiguousarray(case.mask)).to("cuda:0")
    return vol, mask


def parity_report(gpu, orc, names):
    """Per-map worst errors; returns (ok, rows)."""
    gpu = np.asarray(gpu, np.float64)
    orc = np.asarray(orc, np.float64)
    assert gpu.shape == orc.shape, (gpu.shape, orc.shape)
    rows = []
    ok = True
    for k, name in enumerate(names):
        g, o = gpu[k], orc[k]
        fin_g, fin_o = np.isfinite(g), np.isfinite(o)
        same_pattern = np.array_equal(fin_g, fin_o) and np.array_equal(np.isnan(g), np.isnan(o))
        f = fin_o & fin_g
        d = np.abs(g[f] - o[f])
        lim = np.maximum(ABS_TOL, REL_TOL * np.abs(o[f]))
        bad = int(np.count_nonzero(d > lim))
        dabs = float(d.max()) if d.size else 0.0
        drel = float((d / np.maximum(np.abs(o[f]), 1e-300)).max()) if d.size else 0.0
        exact = int(np.count_nonzero(d == 0))
        rows.append(dict(name=name, pattern=same_pattern, bad=bad, dabs=dabs, drel=drel,
                         exact=exact, n=int(f.sum())))
        ok &= same_pattern and bad == 0
    return ok, rows


def format_report(rows, only_bad=False):
    out = []
    for r in rows:
        if only_bad and r["pattern"] and r["bad"] == 0:
            continue
        out.append(f"{r['name']:<48} pattern={'ok' if r['pattern'] else 'DIFF'} bad={r['bad']:>6} "
                   f"dabs={r['dabs']:.3e} drel={r['drel']:.3e} exact={r['exact']}/{r['n']}")
    return "\n".join(out)
