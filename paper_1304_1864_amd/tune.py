"""Autotuner of the multisection shape (lanes per eigenvalue).

The eigenvalue intervals of every tree level are refined by multisection on
Sturm counts (Sec. 2, Alg. 1).  With L lanes per eigenvalue a pass counts at L
points and gains log2(L + 1) bits: a larger L means more counts in total but
fewer dependent passes, and which wins depends on how many eigenvalues a
launch holds (how full the device is) and how long their Sturm counts are.
This script times the two multisection stages (roots: MR3_STAGE_BISECT,
cluster members in their child nodes: MR3_STAGE_CBISECT) of synthetic solves
for every lane count the staged kernel has, keeps the fastest per launch key
(eigenvalue count and mean node rows, as mr3_stats reports them), and writes
the table the library compiles in (csrc/tuning_gfx950.inc); rebuild after.

    python -m paper_1304_1864_amd.tune [--out PATH] [--json PATH] [--quick]

Every input is synthetic and seeded (the generators of ``workloads``).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_OUT = os.path.join(HERE, "csrc", "tuning_gfx950.inc")


def bucket(v: int) -> tuple[int, int]:
    """Power-of-two range [2^k, 2^(k+1)) holding v >= 1."""
    k = int(math.floor(math.log2(max(v, 1))))
    return 1 << k, 1 << (k + 1)


def workloads(quick: bool):
    """(name, precision, kind, data) of the tuning solves: single problems of
    the paper's test-matrix kinds and batches of many small ones."""
    sys.path.insert(0, ROOT)
    import workloads as W

    out = []
    sizes64 = (2000, 20000) if quick else (1000, 4000, 10000, 20000)
    for n in sizes64:
        d, e, _ = W.prescribed_spectrum(n, 0)
        out.append((f"prescribed_n{n}_fp64", 64, "single", (d, e)))
    sizes32 = (4000,) if quick else (1000, 4000, 16000)
    for n in sizes32:
        out.append((f"uniform_n{n}_fp32", 32, "single", W.uniform(n, 0, np.float32)))
    out.append(("121noisy_n8192_fp32", 32, "single", W.toeplitz_121_noisy(8192, 0, 1e-6, np.float32)))
    counts = (4096,) if quick else (512, 4096)
    for c in counts:
        out.append((f"batch{c}_n32-1024_fp32", 32, "batch", W.batch_normal(c, 32, 1024, seed=0, dtype=np.float32)))
        out.append((f"batch{c}_n32-1024_fp64", 64, "batch", W.batch_normal(c, 32, 1024, seed=0, dtype=np.float64)))
    return out


def time_stages(mr3, h, fn, precision: int, lanes: int, reps: int):
    """Median device time of the two multisection stages at a forced lane
    count, and the launch keys the solve reported."""
    import torch

    h.set_params(precision=precision, profile=1, lanes_per_eig=lanes)
    fn()
    torch.cuda.synchronize()
    root, child = [], []
    st = None
    for _ in range(reps):
        fn()
        torch.cuda.synchronize()
        st = h.stats()
        root.append(st["stage_ms"][mr3.STAGES.index("bisect")])
        child.append(st["stage_ms"][mr3.STAGES.index("cbisect")])
    return (float(np.median(root)), float(np.median(child)), st)


def choose(times: dict[int, float], rel: float = 0.02) -> int:
    """Fastest lane count; within `rel` of it the smallest (least work)."""
    best = min(times.values())
    return min(L for L, t in times.items() if t <= best * (1.0 + rel))


def render(entries, notes) -> str:
    lines = [
        "// Multisection shapes measured on gfx950, written by paper_1304_1864_amd/tune.py",
        "// (python -m paper_1304_1864_amd.tune).  One MR3_TUNE(stage, precision,",
        "// count_lo, count_hi, rows_lo, rows_hi, lanes) per launch key; stage 0 = roots,",
        "// 1 = cluster members in their child nodes.  Keys not listed use the size rules.",
    ]
    for n in notes:
        lines.append("// " + n)
    for t in entries:
        lines.append("MR3_TUNE(%d, %d, %d, %d, %d, %d, %d)" % t)
    return "\n".join(lines) + "\n"


def parse(text: str):
    """Entries of a table file (the format render writes)."""
    out = []
    for line in text.splitlines():
        line = line.strip()
        if line.startswith("MR3_TUNE(") and line.endswith(")"):
            out.append(tuple(int(x) for x in line[len("MR3_TUNE("):-1].split(",")))
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--json", default=None, help="also write every measurement here")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args(argv)

    import torch

    sys.path.insert(0, ROOT)
    import paper_1304_1864_amd as mr3

    dev = torch.device("cuda:0")
    h = mr3.Handle(0)
    h.set_tuning([])  # size rules only while measuring
    meas, picks = [], {}
    for name, prec, kind, data in workloads(args.quick):
        dt = torch.float32 if prec == 32 else torch.float64
        if kind == "single":
            d, e = data
            dg = torch.from_numpy(np.ascontiguousarray(d)).to(dev, dt)
            eg = torch.from_numpy(np.ascontiguousarray(e)).to(dev, dt)
            fn = lambda dg=dg, eg=eg: mr3.solve(dg, eg, handle=h)
        else:
            ds = [torch.from_numpy(np.ascontiguousarray(p[0])).to(dev, dt) for p in data]
            es = [torch.from_numpy(np.ascontiguousarray(p[1])).to(dev, dt) for p in data]
            fn = lambda ds=ds, es=es: mr3.solve_batched(ds, es, handle=h)
        rt, ct, keys = {}, {}, None
        for L in mr3.LANE_CANDIDATES:
            r, c, st = time_stages(mr3, h, fn, prec, L, args.reps)
            rt[L], ct[L] = r, c
            keys = st
            meas.append({"workload": name, "precision": prec, "lanes": L, "root_ms": round(r, 4),
                         "child_ms": round(c, 4),
                         "root_key": [st["bisect_count"][0], st["bisect_rows"][0]],
                         "child_key": [st["bisect_count"][1], st["bisect_rows"][1]]})
        line = {"workload": name}
        for stage, times in ((mr3.MR3_TUNE_ROOT, rt), (mr3.MR3_TUNE_CHILD, ct)):
            count, rows = keys["bisect_count"][stage], keys["bisect_rows"][stage]
            if count <= 0:
                continue
            L = choose(times)
            key = (stage, prec) + bucket(count) + bucket(rows)
            # a key met twice keeps the choice of the workload with more time at stake
            if key not in picks or max(times.values()) > picks[key][1]:
                picks[key] = (L, max(times.values()), name, times[L], min(times.values()))
            line[("root" if stage == 0 else "child")] = {"count": count, "rows": rows, "lanes": L,
                                                          "ms": round(times[L], 3)}
        print(json.dumps(line), flush=True)
    h.close()
    entries = sorted(k + (v[0],) for k, v in picks.items())
    notes = ["device: " + torch.cuda.get_device_name(0)]
    for k, v in sorted(picks.items()):
        notes.append("%s stage %d: lanes %d, %.3f ms (slowest lane count %.3f ms)"
                     % (v[2], k[0], v[0], v[3], v[1]))
    with open(args.out, "w") as f:
        f.write(render(entries, notes))
    if args.json:
        with open(args.json, "w") as f:
            json.dump(meas, f, indent=1)
    print(f"wrote {len(entries)} entries to {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
