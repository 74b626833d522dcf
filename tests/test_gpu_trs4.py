"""GPU parity of TRS4 purification and of the FP64 McWeeny refinement step."""
import os

import numpy as np
import pytest

from oracle import canonical, ozaki, projector, trs4
from paper_2407_13299_amd.workloads import (spectrum_hamiltonian,
                                            tight_binding_hamiltonian, workload)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dmp = pytest.importorskip("paper_2407_13299_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL_P = 1e-10
TOL_E = 1e-8


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def gpu_purify(h, nocc, **kw):
    p, e, info = dmp.purify(dev(h), nocc, **kw)
    torch.cuda.synchronize()
    return p.cpu().numpy(), e, info


@pytest.mark.parametrize("kind,s", [("native", 0), ("int8", 7), ("fp16", 7)])
def test_trs4_small_spectrum(kind, s):
    w = workload("small_spectrum")
    h, nocc = w["H"], w["nocc"]
    p, e, info = gpu_purify(h, nocc, tol=w["tol"], slices=max(s, 1), kind=kind, method="trs4")
    p_ref, e_ref, _, _ = projector.eigh_projector(h, nocc)
    assert info["stop"] == "converged" and info["method"] == "trs4"
    assert np.max(np.abs(p - p_ref)) < TOL_P
    assert abs(e - e_ref) < TOL_E
    assert np.array_equal(p, p.T)
    ref = trs4.purify(h, nocc, tol=w["tol"])
    assert abs(info["iters"] - ref["iters"]) <= 1
    # TRS4 initial-guess scalars: h_max and 1 / (h_max - h_min)
    h_min, h_max = canonical.gershgorin(h)
    assert abs(info["mu"] - h_max) < 1e-12 * abs(h_max)
    assert abs(info["lambda"] - 1.0 / (h_max - h_min)) < 1e-12 / (h_max - h_min)


@pytest.mark.parametrize("kind", ["int8", "native"])
def test_trs4_steps_match_oracle(kind):
    """After k = 1..9 steps the iterate equals the oracle's FP64 TRS4 (which
    forms F and G with plain products); the early steps visit all three
    branches on this matrix, including the ones without a second product."""
    h = tight_binding_hamiltonian(6, 6, 6, seed=11)
    n = h.shape[0]
    nocc = n // 4
    sim = trs4.eigen_simulate(h, nocc, tol=1e-30, max_iter=9)
    branches = [x[1] for x in sim["history"]]
    assert {0, 1, 2} <= set(branches) or {1, 2} <= set(branches)
    x = trs4.initial_guess(h)
    hd = dev(h)
    for k in range(1, 10):
        x, gamma, br, _, _ = trs4.step(x, nocc)
        assert br == branches[k - 1]
        assert min(abs(gamma), abs(gamma - 6.0)) > 1e-3    # branch not decided by rounding
        p, e, info = dmp.purify(hd, nocc, tol=1e-30, slices=8, kind=kind, max_iter=k,
                                method="trs4")
        torch.cuda.synchronize()
        assert info["iters"] == k and info["stop"] == "max_iter"
        assert info["products"] == sum(2 if b == trs4.BRANCH_RESET else 1 for b in branches[:k])
        d = np.max(np.abs(p.cpu().numpy() - x))
        assert d < 1e-12, (k, d)
        assert abs(e - float(np.sum(x * h))) < 1e-10
        if br == trs4.BRANCH_RESET:
            assert abs(info["trace"] - nocc) < 1e-9


def test_trs4_tight_binding_2048():
    w = workload("tb_2048")
    h, nocc = w["H"], w["nocc"]
    p, e, info = gpu_purify(h, nocc, tol=w["tol"], slices=7, kind="int8", method="trs4")
    p_ref, e_ref, _, _ = projector.eigh_projector(h, nocc)
    m = projector.measures(p, e, h, nocc, p_ref, e_ref)
    assert info["stop"] == "converged", info
    assert m["max_dP"] < TOL_P, m
    assert m["dE"] < TOL_E, m
    sim = trs4.eigen_simulate(h, nocc, tol=w["tol"])
    assert abs(info["iters"] - sim["iters"]) <= 1
    can = canonical.eigen_simulate(h, nocc, tol=w["tol"])
    assert info["iters"] * 3 < can["iters"]
    # INT8 and FP16 slices give the same products, hence the same iterates
    p16, e16, _ = gpu_purify(h, nocc, tol=w["tol"], slices=7, kind="fp16", method="trs4")
    assert np.array_equal(p, p16) and e == e16
    pn, en, infon = gpu_purify(h, nocc, tol=w["tol"], kind="native", method="trs4")
    assert abs(infon["iters"] - info["iters"]) <= 1   # the last gamma is rounding noise
    assert np.max(np.abs(pn - p)) < TOL_P


def test_trs4_batched_equals_single():
    sizes = [130, 257, 96]
    hs = [spectrum_hamiltonian(n, n // 3, seed=300 + i)[0] for i, n in enumerate(sizes)]
    noccs = [n // 3 for n in sizes]
    Ps, Es, infos = dmp.purify_batched([dev(h) for h in hs], noccs, tol=1e-10, slices=7,
                                       method="trs4")
    torch.cuda.synchronize()
    for h, nocc, P, E, inf in zip(hs, noccs, Ps, Es, infos):
        p1, e1, i1 = gpu_purify(h, nocc, tol=1e-10, slices=7, method="trs4")
        assert np.array_equal(P.cpu().numpy(), p1) and E == e1 and inf["iters"] == i1["iters"]
        assert inf["method"] == "trs4"


def test_trs4_special_occupations():
    h, _, _ = spectrum_hamiltonian(64, 32, seed=61)
    p0, e0, i0 = gpu_purify(h, 0, method="trs4")
    pn, en, i_n = gpu_purify(h, 64, method="trs4")
    assert np.all(p0 == 0) and e0 == 0.0 and i0["iters"] == 0
    assert np.array_equal(pn, np.eye(64)) and i_n["iters"] == 0


def test_trs4_full_size_tb_8192():
    ref = np.load(os.path.join(GOLDEN, "tb8192_reference.npz"))
    w = workload("tb_8192")
    h, nocc = w["H"], w["nocc"]
    hd = dev(h)
    del h
    p, e, info = dmp.purify(hd, nocc, tol=w["tol"], slices=7, kind="int8", method="trs4")
    torch.cuda.synchronize()
    assert info["stop"] == "converged", info
    assert info["iters"] < 25
    assert abs(e - float(ref["E"])) < TOL_E
    rows = p[torch.from_numpy(ref["rows"]).cuda()].cpu().numpy()
    assert np.max(np.abs(rows - ref["P_rows"])) < TOL_P
    samp = p[torch.from_numpy(ref["si"]).cuda(), torch.from_numpy(ref["sj"]).cuda()].cpu().numpy()
    assert np.max(np.abs(samp - ref["P_samples"])) < TOL_P
    assert torch.equal(p, p.T)


# ---- McWeeny refinement (Sec. 4.1) ----------------------------------------

def test_refinement_recovers_energy_at_low_slices():
    """At S = 5 the energy misses the 1e-8 bar; one FP64 McWeeny step brings
    it to the FP64 level (the effect reported in Sec. 4.1), while the
    unrefined energy is reported unchanged."""
    w = workload("tb_2048")
    h, nocc = w["H"], w["nocc"]
    p_ref, e_ref, _, _ = projector.eigh_projector(h, nocc)
    p0, e0, i0 = gpu_purify(h, nocc, tol=w["tol"], slices=5, kind="int8")
    p1, e1, i1 = gpu_purify(h, nocc, tol=w["tol"], slices=5, kind="int8", refine=True)
    assert i1["refined"] == 1 and i0["refined"] == 0
    assert i1["E_unrefined"] == e0 and i1["iters"] == i0["iters"]
    assert i0["products"] == 2 * i0["iters"] and i1["products"] == i0["products"] + 2
    assert abs(e0 - e_ref) > 1e-9
    assert abs(e1 - e_ref) < 1e-10
    assert abs(e1 - e_ref) < 1e-2 * abs(e0 - e_ref)
    assert np.array_equal(p1, p1.T)
    assert abs(i1["trace"] - nocc) < 1e-8


def test_refinement_matches_oracle_on_small_case():
    """Oracle: canonical purification with the oracle's own Ozaki products at
    S = 4, then its FP64 McWeeny step; both refined energies sit at the FP64
    level and agree, as do the refined projectors within the S = 4 noise."""
    h, _, lam = spectrum_hamiltonian(192, 80, seed=71)
    e_exact = float(np.sort(lam)[:80].sum())
    ref = canonical.purify(h, 80, tol=1e-8, matmul=lambda a, b: ozaki.ozaki_gemm(a, b, 4))
    p_or, e_or = trs4.mcweeny_refine(ref["P"], h)
    p, e, info = gpu_purify(h, 80, tol=1e-8, slices=4, kind="int8", refine=True)
    assert info["refined"] == 1
    assert abs(e_or - e_exact) < 1e-9 and abs(e - e_exact) < 1e-9
    assert abs(e - e_or) < 1e-9
    assert np.max(np.abs(p - p_or)) < 1e-5


def test_refinement_of_converged_fp64_run_is_idle():
    w = workload("small_spectrum")
    h, nocc = w["H"], w["nocc"]
    p0, e0, _ = gpu_purify(h, nocc, tol=w["tol"], kind="native")
    p1, e1, i1 = gpu_purify(h, nocc, tol=w["tol"], kind="native", refine=True)
    assert i1["refined"] == 1
    assert np.max(np.abs(p1 - p0)) < 1e-13 and abs(e1 - e0) < 1e-11
    # trs4 + refinement
    p2, e2, i2 = gpu_purify(h, nocc, tol=w["tol"], slices=7, method="trs4", refine=True)
    p_ref, e_ref, _, _ = projector.eigh_projector(h, nocc)
    assert i2["refined"] == 1 and np.max(np.abs(p2 - p_ref)) < TOL_P


def test_refinement_skipped_without_iterations():
    h, _, _ = spectrum_hamiltonian(64, 32, seed=61)
    p, e, info = gpu_purify(h, 0, refine=True)
    assert info["refined"] == 0 and np.all(p == 0)
