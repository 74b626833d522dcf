"""The autotuner's fit and header writer (host logic; the measurement itself
needs the GPU and writes csrc/tuned_table.h)."""
import math
import re

from paper_2407_13299_amd import autotune


def test_fit_recovers_model_and_bounds_points(tmp_path):
    c0, a0 = 37.0, 1.3
    rows = []
    for n in (128, 512, 2048):
        for s in (4, 5, 6, 7):
            e = c0 * n ** a0 * 2.0 ** (1 - 8 * s) * (1.0 + 0.1 * ((n + s) % 3))
            rows.append((n, s, e, "converged"))
    rows.append((128, 8, 1e-16, "converged"))          # below the noise floor: ignored
    c, a = autotune.fit(rows)
    assert abs(a - a0) < 0.1
    for n, s, e, _ in rows[:-1]:
        assert c * n ** a * 2.0 ** (1 - 8 * s) >= e * (1 - 1e-12)
    out = tmp_path / "t.h"
    autotune.write_header(str(out), c, a, rows)
    text = out.read_text()
    vals = re.findall(r"kTunedErrC\[2\] = \{([^,]+), ([^}]+)\}", text)[0]
    assert math.isclose(float(vals[0]), c, rel_tol=1e-5) and vals[0] == vals[1].strip()
    assert "kTunedTarget = 1e-10" in text


def _tile_choice_exe(tmp_path):
    import os
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        import pytest
        pytest.skip("no g++")
    here = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(os.path.dirname(here), "paper_2407_13299_amd", "csrc")
    exe = str(tmp_path / "tile_choice")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", csrc,
                    "-I", os.path.join(os.path.dirname(here), "include"),
                    os.path.join(here, "host", "tile_choice.cpp"), os.path.join(csrc, "plan.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


def _tile_choice(exe, queries, forced=0):
    import subprocess
    text = "".join(f"{k} {s} {n} {forced}\n" for k, s, n in queries)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return [tuple(int(x) for x in line.split()) for line in out.splitlines()]


def test_tile_table_picks_the_measured_winners(tmp_path):
    """tuned_tiles.h as compiled into the library: for every size it was
    measured at, tile_choice returns the winner recorded beside the
    measurement; rows of one (kind, slice range) cover every size once;
    64-row tiles only up to S = 8."""
    import os
    hdr = os.path.join(os.path.dirname(autotune.__file__), "csrc", "tuned_tiles.h")
    text = open(hdr).read()
    rules = [tuple(int(v) if not v.strip().startswith("1 <<") else 1 << 30
                   for v in m.split(","))
             for m in re.findall(r"^\s*\{([^}]*)\},", text, re.M)]
    assert rules
    for k, s_lo, s_hi, n_lo, n_hi, rb, split in rules:
        assert rb in (2, 4) and split in (0, 1) and n_lo <= n_hi and s_lo <= s_hi
        assert rb == 4 or s_hi <= autotune.MAX_SLICES_64
    for key in {(r[0], r[1], r[2]) for r in rules}:
        spans = sorted((r[3], r[4]) for r in rules if (r[0], r[1], r[2]) == key)
        assert spans[0][0] == 1 and spans[-1][1] == 1 << 30
        assert all(a[1] + 1 == b[0] for a, b in zip(spans, spans[1:]))
    measured = re.findall(r"//\s+(int8|fp16) S=\s*(\d+) n=\s*(\d+) .*-> (\d+)/(split|whole)", text)
    exe = _tile_choice_exe(tmp_path)
    if measured:
        q = [(autotune.KIND_IDS[k], int(s), int(n)) for k, s, n, _, _ in measured]
        got = _tile_choice(exe, q)
        want = [(int(rows) // 32, 1 if sp == "split" else 0) for _, _, _, rows, sp in measured]
        assert got == want
    # 64-row tiles never beyond S = 8, whatever the table or the forced height says
    assert all(rb == 4 for rb, _ in _tile_choice(exe, [(1, 9, 512), (1, 12, 8192), (2, 9, 100)]))
    assert all(rb == 4 for rb, _ in _tile_choice(exe, [(1, 9, 512), (2, 12, 100)], forced=2))
    # the Markidis kind has no 64-row tiles
    assert all(rb == 4 for rb, _ in _tile_choice(exe, [(3, 2, 512)], forced=2))


def test_tile_ranges_merge_and_cover():
    picks = [("int8", 7, 256, (2, 1)), ("int8", 7, 512, (2, 1)), ("int8", 7, 1536, (4, 1)),
             ("int8", 7, 2048, (2, 0)), ("int8", 8, 512, (4, 1))]
    t = autotune.tile_ranges(picks)
    assert t == [(("int8", 7), 1, 1024, (2, 1)), (("int8", 7), 1025, 1792, (4, 1)),
                 (("int8", 7), 1793, 1 << 30, (2, 0)), (("int8", 8), 1, 1 << 30, (4, 1))]
    rows = [("int8", 7, 512, {(2, 1): 10.0, (2, 0): 9.95, (4, 1): 12.0, (4, 0): 12.0}),
            ("int8", 7, 1536, {(2, 1): 10.0, (2, 0): 10.0, (4, 1): 9.0, (4, 0): 9.5})]
    assert autotune.pick_tiles(rows) == [("int8", 7, 512, (2, 1)), ("int8", 7, 1536, (4, 1))]
