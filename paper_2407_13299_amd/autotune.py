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

With --tiles it measures instead the tile choice of the purification
products per (kind, S, n): the tile height (64 or 128 rows) and whether the
last, partly filled round of tiles is split along the reduction.  For every
size a spectrum-controlled Hamiltonian runs a fixed number of iterations
under every choice (interleaved rounds, median of the rounds); a choice other
than the default (64-row tiles with a split tail, 128-row tiles beyond S = 7)
is taken only when it is faster by more than a margin, and the winners are
merged into size ranges written to csrc/tuned_tiles.h:

    python -m paper_2407_13299_amd.autotune --tiles --out csrc/tuned_tiles.h
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


# ---- tile choice -------------------------------------------------------------

TILE_SIZES = (256, 384, 512, 640, 768, 1024, 1280, 1536, 1792, 2048, 2560, 3072, 4096, 6144,
              8192)
TILE_CASES = (("int8", 6), ("int8", 7), ("int8", 8), ("fp16", 7))
TILE_ITERS = 10        # iterations per timed run (stopped by max_iter)
TILE_MARGIN = 0.015    # a non-default choice must be this much faster
KIND_IDS = {"int8": 1, "fp16": 2}
MAX_SLICES_64 = 8      # largest S with 64-row tiles (kMaxSlices64 in layout.hpp)
# slice range each measured (kind, S) stands for in the table (S = 9..12 have
# 128-row tiles only, the table's fallback)
S_RANGES = {("int8", 6): (1, 6), ("int8", 7): (7, 7), ("int8", 8): (8, 8),
            ("fp16", 7): (1, 8)}


def tile_choices(s):
    """(rb, split_tail) pairs that exist for S slices."""
    return [(2, 1), (2, 0), (4, 1), (4, 0)] if s <= MAX_SLICES_64 else [(4, 1), (4, 0)]


def default_choice(s):
    return (2, 1) if s <= MAX_SLICES_64 else (4, 1)


def measure_tiles(sizes=TILE_SIZES, cases=TILE_CASES, rounds=3, seed=11, log=print):
    """Median time of TILE_ITERS purification iterations per (kind, S, n,
    choice), the choices interleaved within each round."""
    import statistics
    import time

    import torch
    from . import _lib, api
    from .workloads import spectrum_hamiltonian
    lib = _lib.load()
    saved = {k: os.environ.get(k) for k in ("DMP_TILE_ROWS", "DMP_TAIL_SPLIT")}

    def use(rb, split):
        os.environ["DMP_TILE_ROWS"] = "64" if rb == 2 else "128"
        os.environ["DMP_TAIL_SPLIT"] = "1" if split else "0"

    rows = []
    try:
        for kind, s in cases:
            for n in sizes:
                h, _, _ = spectrum_hamiltonian(n, n // 2, seed=seed + n)
                hd = torch.from_numpy(h).cuda()
                P = torch.empty_like(hd)
                choices = tile_choices(s)
                wss = {}
                for c in choices:
                    use(*c)
                    wss[c] = torch.empty(lib.dmp_purify_workspace_bytes(n, s, KIND_IDS[kind]),
                                         dtype=torch.uint8, device="cuda")
                    api.purify(hd, n // 2, tol=1e-300, slices=s, kind=kind, max_iter=TILE_ITERS,
                               out=P, workspace=wss[c])          # warm-up and graph capture
                times = {c: [] for c in choices}
                for _ in range(rounds):
                    for c in choices:
                        use(*c)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        api.purify(hd, n // 2, tol=1e-300, slices=s, kind=kind,
                                   max_iter=TILE_ITERS, out=P, workspace=wss[c])
                        torch.cuda.synchronize()
                        times[c].append((time.perf_counter() - t0) * 1e3)
                med = {c: statistics.median(v) for c, v in times.items()}
                rows.append((kind, s, n, med))
                log(f"{kind} S={s} n={n}: " + ", ".join(
                    f"{32 * c[0]}/{'split' if c[1] else 'whole'} {t:.3f} ms" for c, t in med.items()))
                del wss
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return rows


def pick_tiles(rows, margin=TILE_MARGIN):
    """Winner per measured point: the default unless another choice is faster
    by more than ``margin``."""
    out = []
    for kind, s, n, med in rows:
        d = default_choice(s)
        best = min(med, key=med.get)
        win = best if med[best] < med[d] * (1.0 - margin) else d
        out.append((kind, s, n, win))
    return out


def tile_ranges(picks):
    """Merge the winners of each (kind, S) into size ranges [n_lo, n_hi]
    (boundaries half-way between measured sizes; the first range starts at 1,
    the last ends at 2^30)."""
    table = []
    for key in dict.fromkeys((k, s) for k, s, _, _ in picks):
        pts = sorted((n, c) for k, s, n, c in picks if (k, s) == key)
        lo = 1
        for i, (n, c) in enumerate(pts):
            last = i == len(pts) - 1
            hi = (1 << 30) if last else (n + pts[i + 1][0]) // 2
            if table and table[-1][0] == key and table[-1][3] == c:
                table[-1] = (key, table[-1][1], hi, c)
            else:
                table.append((key, lo, hi, c))
            lo = hi + 1
    return table


def write_tiles_header(path, rows, margin=TILE_MARGIN):
    picks = pick_tiles(rows, margin)
    table = tile_ranges(picks)
    lines = [
        "// Tile choice of the Ozaki purification products, used by dmp::tile_choice:",
        "// per kind and slice range, for n in [n_lo, n_hi], the tile height (rb = 2:",
        "// 64-row tiles, two workgroups per CU; rb = 4: 128-row tiles) and whether",
        "// the last, partly filled round of tiles is split along the reduction.",
        "// The first matching row wins; no match: 128-row tiles, split tail.",
        "// Written by paper_2407_13299_amd/autotune.py --tiles from these",
        f"// measurements (spectrum-controlled H, half filled, {TILE_ITERS} iterations, median",
        f"// of interleaved rounds, ms; a non-default choice must win by {margin:.1%}):",
    ]
    for (kind, s, n, med), (_, _, _, win) in zip(rows, picks):
        cells = "  ".join(f"{32 * c[0]}/{'split' if c[1] else 'whole'} {t:8.3f}"
                          for c, t in sorted(med.items()))
        lines.append(f"//   {kind} S={s:2d} n={n:5d}  {cells}  -> {32 * win[0]}/"
                     f"{'split' if win[1] else 'whole'}")
    lines += [
        "#pragma once",
        "namespace dmp {",
        "struct TileRule {",
        "    int kind;        // dmp_kind",
        "    int s_lo, s_hi;  // slice counts",
        "    int n_lo, n_hi;  // sizes",
        "    int rb;          // 2 or 4",
        "    int split_tail;  // 0 or 1",
        "};",
        "constexpr TileRule kTileTable[] = {",
    ]
    for (kind, s), lo, hi, (rb, split) in table:
        s_lo, s_hi = S_RANGES.get((kind, s), (s, s))
        hi_txt = "1 << 30" if hi == (1 << 30) else str(hi)
        lines.append(f"    {{{KIND_IDS[kind]}, {s_lo}, {s_hi}, {lo}, {hi_txt}, {rb}, {split}}},")
    lines += ["};", "}  // namespace dmp"]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "csrc", "tuned_table.h"))
    ap.add_argument("--sizes", type=int, nargs="*", default=None)
    ap.add_argument("--tiles", action="store_true",
                    help="measure the tile choice and write csrc/tuned_tiles.h")
    args = ap.parse_args(argv)
    if args.tiles:
        out = args.out
        if out.endswith("tuned_table.h"):
            out = os.path.join(os.path.dirname(out), "tuned_tiles.h")
        rows = measure_tiles(tuple(args.sizes or TILE_SIZES), log=lambda m: print(m, flush=True))
        table = write_tiles_header(out, rows)
        for row in table:
            print(row, flush=True)
        print(f"wrote {out}", flush=True)
        return 0
    rows = measure(tuple(args.sizes or SIZES), log=lambda m: print(m, flush=True))
    c, a = fit(rows)
    print(f"fit: C = {c:.4g}, a = {a:.4g}", flush=True)
    write_header(args.out, c, a, rows)
    print(f"wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
