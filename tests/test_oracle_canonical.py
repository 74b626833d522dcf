"""Pins for the canonical-purification oracle."""
import numpy as np
import pytest

from oracle import canonical, ozaki, projector
from paper_2407_13299_amd.workloads import (spectrum_hamiltonian,
                                            tight_binding_hamiltonian)


def test_converges_to_projector_spectrum():
    h, q, lam = spectrum_hamiltonian(256, 128, seed=0)
    r = canonical.purify(h, 128, tol=1e-12)
    p_ref, e_ref, _, _ = projector.eigh_projector(h, 128)
    assert r["stop"] == canonical.STOP_CONVERGED
    assert np.max(np.abs(r["P"] - p_ref)) < 1e-10
    assert abs(r["E"] - e_ref) < 1e-10
    # closed form from the construction
    assert abs(r["E"] - lam[lam < 0].sum()) < 1e-10


def test_converges_to_projector_tight_binding():
    h = tight_binding_hamiltonian(4, 4, 4, seed=1)
    r = canonical.purify(h, 64, tol=1e-10)
    p_ref, e_ref, _, _ = projector.eigh_projector(h, 64)
    assert r["stop"] == canonical.STOP_CONVERGED
    assert np.max(np.abs(r["P"] - p_ref)) < 1e-10
    assert abs(r["E"] - e_ref) < 1e-9


def test_trace_conserved_every_step():
    """tr f_c(P) = tr P exactly when c = t2 / t1 (the point of the canonical
    coefficient): check every iterate."""
    h = tight_binding_hamiltonian(3, 4, 3, seed=5)
    n = h.shape[0]
    nocc = n // 4
    p = canonical.initial_guess(h, nocc)
    assert abs(np.trace(p) - nocc) < 1e-11
    ev = np.linalg.eigvalsh(p)
    assert ev.min() >= -1e-12 and ev.max() <= 1 + 1e-12
    for _ in range(30):
        p2 = p @ p
        p3 = p2 @ p
        c, t1, t2 = canonical.coefficient(p, p2, p3)
        a, b, g = canonical.update_weights(c)
        p = a * p + b * p2 + g * p3
        assert abs(np.trace(p) - nocc) < 1e-9


def test_tie_branches_equal_mcweeny():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, 50)
    a1, b1, g1 = canonical.update_weights(0.5)
    a0, b0, g0 = 1.0, 3.0, -2.0   # McWeeny 3P^2 - 2P^3 written as weights
    assert (a1, b1, g1) == (0.0, 3.0, -2.0)
    # the c < 1/2 formula approaches the same polynomial
    c = 0.5 - 1e-12
    w = canonical.update_weights(c)
    assert np.allclose(w, (0.0, 3.0, -2.0), atol=1e-10)
    assert np.allclose(a1 * x + b1 * x ** 2 + g1 * x ** 3, 3 * x ** 2 - 2 * x ** 3)
    del a0, b0, g0


def test_fixed_points_and_monotone_map():
    """For every c in [0, 1] both maps fix 0 and 1 and keep [0, 1] in [0, 1]."""
    x = np.linspace(0, 1, 1001)
    for c in np.linspace(0, 1, 21):
        if c == 0.0:
            continue
        a, b, g = canonical.update_weights(c)
        f = a * x + b * x * x + g * x ** 3
        assert abs(f[0]) < 1e-15 and abs(f[-1] - 1) < 1e-13
        assert f.min() >= -1e-15 and f.max() <= 1 + 1e-13
        assert np.all(np.diff(f) >= -1e-15)


@pytest.mark.parametrize("maker", ["spectrum", "tb"])
def test_eigen_simulator_matches_matrix_iteration(maker):
    if maker == "spectrum":
        h, _, _ = spectrum_hamiltonian(128, 64, seed=2)
        nocc = 64
    else:
        h = tight_binding_hamiltonian(4, 4, 4, seed=1)
        nocc = 64
    r = canonical.purify(h, nocc, tol=1e-10)
    s = canonical.eigen_simulate(h, nocc, tol=1e-10)
    assert r["iters"] == s["iters"]
    cm = np.array([hh[0] for hh in r["history"]])
    cs = np.array([hh[0] for hh in s["history"]])
    # c_k agrees until the final noise-dominated steps
    k = max(1, len(cm) - 4)
    assert np.max(np.abs(cm[:k] - cs[:k])) < 1e-8
    em = np.array([hh[4] for hh in r["history"]])
    es = np.array([hh[4] for hh in s["history"]])
    assert np.max(np.abs(em - es)) < 1e-9


def test_energy_decreases_until_noise():
    h = tight_binding_hamiltonian(4, 4, 4, seed=1)
    s = canonical.eigen_simulate(h, 64, tol=1e-10)
    e = np.array([hh[4] for hh in s["history"]])
    de = np.diff(e)
    big = np.abs(de) > 1e-9
    assert np.all(de[big] < 0)


def test_special_occupations():
    h, _, _ = spectrum_hamiltonian(20, 10, seed=3)
    r0 = canonical.purify(h, 0)
    rn = canonical.purify(h, 20)
    assert np.array_equal(r0["P"], np.zeros((20, 20))) and r0["E"] == 0.0
    assert np.array_equal(rn["P"], np.eye(20)) and abs(rn["E"] - np.trace(h)) < 1e-14


def test_low_slice_purification_fails_to_converge_and_high_slices_match():
    """With very few slices the emulated products are too coarse: the run
    stagnates or hits the cap instead of converging (Sec. 3's halting rule).
    With enough slices the iteration count equals FP64's (pattern of Table 2's
    iteration rows, Sec. 4.5)."""
    h, _, _ = spectrum_hamiltonian(64, 32, seed=4)
    for s, want in ((2, canonical.STOP_STAGNATED), (3, canonical.STOP_STAGNATED)):
        r = canonical.purify(h, 32, tol=1e-8, max_iter=60,
                             matmul=lambda a, b: ozaki.ozaki_gemm(a, b, s))
        assert r["stop"] == want
    with np.errstate(all="ignore"):
        r1 = canonical.purify(h, 32, tol=1e-8, max_iter=60,
                              matmul=lambda a, b: ozaki.ozaki_gemm(a, b, 1))
    assert r1["stop"] == canonical.STOP_NONFINITE
    r64 = canonical.purify(h, 32, tol=1e-8)
    r7 = canonical.purify(h, 32, tol=1e-8,
                          matmul=lambda a, b: ozaki.ozaki_gemm(a, b, 7))
    assert r7["stop"] == canonical.STOP_CONVERGED
    assert r7["iters"] == r64["iters"]
    p_ref, e_ref, _, _ = projector.eigh_projector(h, 32)
    assert np.max(np.abs(r7["P"] - p_ref)) < 1e-10


def test_gershgorin_encloses_spectrum():
    h = tight_binding_hamiltonian(4, 3, 3, seed=9)
    lo, hi = canonical.gershgorin(h)
    ev = np.linalg.eigvalsh(h)
    assert lo <= ev[0] and ev[-1] <= hi


# A 4 x 4 symmetric H whose Gershgorin discs are worked out by hand (Sec. 2.3:
# lambda maps the spectrum into [0, 1]; the bounds come from the discs
# centre H_ii, radius sum_{j != i} |H_ij|):
#   row 0: centre  2, radius 1 + 0 + 0.5 = 1.5 -> [ 0.5, 3.5]
#   row 1: centre  0, radius 1 + 3 + 0   = 4   -> [-4,   4  ]
#   row 2: centre -4, radius 0 + 3 + 1   = 4   -> [-8,   0  ]
#   row 3: centre  1, radius 0.5 + 0 + 1 = 1.5 -> [-0.5, 2.5]
# so h_min = -8 (row 2) and h_max = 4 (row 1); tr H = -1, mu = -1/4.
HAND_H = np.array([[2.0, -1.0, 0.0, 0.5],
                   [-1.0, 0.0, 3.0, 0.0],
                   [0.0, 3.0, -4.0, 1.0],
                   [0.5, 0.0, 1.0, 1.0]])


def test_gershgorin_hand_computed_bounds():
    """Fails if the radius also counts |H_ii| (h_max would be 5.5), if the
    centre's sign is flipped (h_max 8) or if min and max are exchanged."""
    lo, hi = canonical.gershgorin(HAND_H)
    assert lo == -8.0 and hi == 4.0


def test_initial_scalars_hand_computed():
    """theta = nocc / n; lam = min(theta / (h_max - mu), (1 - theta) / (mu - h_min)).
    nocc = 1: 0.25 / 4.25 = 1/17 against 0.75 / 7.75 = 3/31, the first is smaller.
    nocc = 3: 0.75 / 4.25 = 3/17 against 0.25 / 7.75 = 1/31, the second is."""
    theta, mu, lam, lo, hi, which = canonical.initial_scalars(HAND_H, 1)
    assert (theta, mu, lo, hi, which) == (0.25, -0.25, -8.0, 4.0, 0)
    assert lam == pytest.approx(1.0 / 17.0, rel=1e-15)
    theta, mu, lam, lo, hi, which = canonical.initial_scalars(HAND_H, 3)
    assert (theta, mu, which) == (0.75, -0.25, 1)
    assert lam == pytest.approx(1.0 / 31.0, rel=1e-15)


def test_initial_guess_hand_computed():
    """P0 = lam (mu I - H) + theta I with lam = 1/17, mu = -1/4, theta = 1/4:
    P0_00 = (-1/4 - 2)/17 + 1/4 = 2/17, P0_01 = 1/17, P0_22 = (-1/4 + 4)/17 + 1/4
    = 8/17, P0_23 = -1/17; tr P0 = nocc."""
    p0 = canonical.initial_guess(HAND_H, 1)
    want = {(0, 0): 2.0 / 17, (0, 1): 1.0 / 17, (2, 2): 8.0 / 17, (2, 3): -1.0 / 17,
            (1, 3): 0.0}
    for (i, j), v in want.items():
        assert p0[i, j] == pytest.approx(v, rel=1e-14, abs=1e-16)
    assert np.trace(p0) == pytest.approx(1.0, rel=1e-14)
