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
