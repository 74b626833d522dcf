"""Measure the slice-count error model of dmp_autotune_slices on the GPU and
write csrc/tuned_table.h.

For every size n and slice count S the purification of a spectrum-controlled
Hamiltonian (half filled, gap 0.2 Ha) runs with S slices and with 11 slices;
the error is max |P_S - P_11| (the 11-slice run is FP64-level, so it serves as
the reference).  The model

    max |dP| ~ C n^a 2^(1 - 8 S)

is fitted by least squares to log2 of the errors above the FP64 noise floor,
and C is raised so that the model bounds every measured point.  INT8 and FP16
slices give bit-identical products, so one fit serves both kinds.

    python -m paper_2407_13299_amd.autotune --out csrc/tuned_table.h
"""
from __future__ import annotations

import argparse
import math
import os
import sys

import numpy as np

SIZES = (128, 256, 512, 1024, 1536, 2048, 3072)
SLICES = (4, 5, 6, 7, 8)
REF_SLICES = 11
NOISE = 1e-14          # below this the error is FP64 rounding, not the split


def measure(sizes=SIZES, slices=SLICES, seed=7, log=print):
    import torch
    from . import api
    from .workloads import spectrum_hamiltonian
    rows = []
    for n in sizes:
        h, _, _ = spectrum_hamiltonian(n, n // 2, seed=seed + n)
        hd = torch.from_numpy(h).cuda()
        p_ref, _, _ = api.purify(hd, n // 2, tol=1e-12, slices=REF_SLICES)
        for s in slices:
            p, _, info = api.purify(hd, n // 2, tol=1e-12, slices=s)
            torch.cuda.synchronize()
            err = float(torch.max(torch.abs(p - p_ref)).item())
            rows.append((n, s, err, info["stop"]))
            log(f"n={n:5d} S={s:2d} max|dP|={err:.3e} ({info['stop']})")
    return rows


def fit(rows):
    pts = [(n, s, e) for n, s, e, _ in rows if e > NOISE]
    if len(pts) < 3:
        raise RuntimeError("too few points above the noise floor to fit")
    # log2 e = log2 C + a log2 n + 1 - 8 S
    A = np.array([[1.0, math.log2(n)] for n, _, _ in pts])
    y = np.array([math.log2(e) - 1.0 + 8.0 * s for _, s, e in pts])
    (log2c, a), *_ = np.linalg.lstsq(A, y, rcond=None)
    # raise C so that the model bounds every measured point
    log2c = max(log2c, max(yy - a * math.log2(n) for (n, _, _), yy in zip(pts, y)))
    return 2.0 ** log2c, float(a)


def write_header(path, c, a, rows, target=1e-10):
    lines = [
        "// Slice-count error model used by dmp_autotune_slices:",
        "//   max|dP| ~ kTunedErrC[kind] * n^kTunedErrA[kind] * 2^-(8S - 1)",
        "// (index 0: INT8, 1: FP16; both kinds give bit-identical products),",
        "// and the default accuracy target of the batched entry point when it",
        "// picks S itself.  Written by paper_2407_13299_amd/autotune.py from",
        "// these measurements (spectrum-controlled H, half filled, gap 0.2 Ha,",
        f"// max |P_S - P_{REF_SLICES}|):",
    ]
    for n, s, e, stop in rows:
        lines.append(f"//   n = {n:5d}  S = {s:2d}  {e:.3e}  {stop}")
    lines += [
        "#pragma once",
        "namespace dmp {",
        f"constexpr double kTunedErrC[2] = {{{c:.6g}, {c:.6g}}};",
        f"constexpr double kTunedErrA[2] = {{{a:.6g}, {a:.6g}}};",
        f"constexpr double kTunedTarget = {target:g};",
        "}  // namespace dmp",
    ]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "csrc", "tuned_table.h"))
    ap.add_argument("--sizes", type=int, nargs="*", default=list(SIZES))
    args = ap.parse_args(argv)
    rows = measure(args.sizes, log=lambda m: print(m, flush=True))
    c, a = fit(rows)
    print(f"fit: C = {c:.4g}, a = {a:.4g}", flush=True)
    write_header(args.out, c, a, rows)
    print(f"wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
