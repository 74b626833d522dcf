"""Hand-written adjoint of the purification (dL/dH for L = tr(P W))."""
import numpy as np
import pytest

from oracle import adjoint, canonical
from paper_2407_13299_amd.workloads import (spectrum_hamiltonian,
                                            symmetric_direction,
                                            symmetric_weight, workload)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dmp = pytest.importorskip("paper_2407_13299_amd")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def gpu_grad(h, nocc, w, tol=1e-10, slices=7, stride=0):
    tape = dmp.PurifyTape(dev(h), nocc, tol=tol, slices=slices, stride=stride)
    g = tape.backward(dev(w))
    torch.cuda.synchronize()
    return tape, g.cpu().numpy()


def test_tape_forward_equals_purify():
    h, _, _ = spectrum_hamiltonian(150, 60, seed=21)
    tape = dmp.PurifyTape(dev(h), 60, tol=1e-10, slices=7)
    p, e, info = dmp.purify(dev(h), 60, tol=1e-10, slices=7)
    torch.cuda.synchronize()
    assert torch.equal(tape.P, p) and tape.E == e and tape.info["iters"] == info["iters"]


@pytest.mark.parametrize("n,nocc,seed,k", [(96, 40, 22, 6), (130, 70, 23, 9), (150, 60, 24, 12)])
def test_adjoint_matches_oracle_adjoint(n, nocc, seed, k):
    """Before convergence (c well away from 1/2, so the branch is not decided
    by rounding) the GPU adjoint equals the oracle's reverse pass through the
    same number of steps."""
    h, _, _ = spectrum_hamiltonian(n, nocc, seed=seed)
    w = symmetric_weight(n, seed=seed + 100)
    tape = dmp.PurifyTape(dev(h), nocc, tol=1e-30, slices=8, max_iter=k, stride=3)
    g = tape.backward(dev(w)).cpu().numpy()
    ref = canonical.purify(h, nocc, tol=0.0, max_iter=k)
    branches = [hh[1] for hh in ref["history"]]
    c_gpu, t1_gpu, _ = tape.coefficients()
    c_ref = [hh[0] for hh in ref["history"]]
    assert all(abs(c - 0.5) > 1e-6 for c in c_ref)
    assert tape.branches() == branches          # same control flow as the FP64 oracle
    assert np.max(np.abs(np.array(c_gpu) - np.array(c_ref))) < 1e-12
    g_ref = adjoint.canonical_adjoint(h, nocc, w, branches)
    scale = np.max(np.abs(g_ref))
    assert np.max(np.abs(g - g_ref)) < 1e-11 * scale
    assert np.array_equal(g, g.T)


@pytest.mark.parametrize("n,nocc,seed", [(96, 40, 22), (130, 70, 23)])
def test_adjoint_converged_matches_perturbation(n, nocc, seed):
    h, _, _ = spectrum_hamiltonian(n, nocc, seed=seed)
    w = symmetric_weight(n, seed=seed + 100)
    tape, g = gpu_grad(h, nocc, w, tol=1e-10)
    assert tape.info["stop"] == "converged"
    gp = adjoint.perturbation_gradient(h, nocc, w)
    assert np.max(np.abs(g - gp)) < 1e-10 * np.max(np.abs(gp))


def test_adjoint_workload_2048_perturbation_formula():
    w = workload("adjoint_2048")
    h, nocc, W = w["H"], w["nocc"], w["W"]
    tape, g = gpu_grad(h, nocc, W, tol=w["tol"])
    assert tape.info["stop"] == "converged"
    gp = adjoint.perturbation_gradient(h, nocc, W)
    scale = np.max(np.abs(gp))
    assert np.max(np.abs(g - gp)) < 1e-6 * scale
    # invariances of the projector: shifts and scalings of H
    assert abs(np.trace(g)) < 1e-8 * scale * h.shape[0]
    assert abs(np.sum(g * h)) < 1e-8 * scale * h.shape[0]


def test_adjoint_finite_differences():
    n, nocc = 160, 64
    h, _, _ = spectrum_hamiltonian(n, nocc, seed=31)
    w = symmetric_weight(n, seed=32)
    _, g = gpu_grad(h, nocc, w, tol=1e-12)
    for seed in (33, 34):
        d = symmetric_direction(n, seed)
        hs = 1e-5
        lp = float(np.sum(dmp.purify(dev(h + hs * d), nocc, tol=1e-12, slices=7)[0].cpu().numpy() * w))
        lm = float(np.sum(dmp.purify(dev(h - hs * d), nocc, tol=1e-12, slices=7)[0].cpu().numpy() * w))
        fd = (lp - lm) / (2 * hs)
        an = float(np.sum(g * d))
        assert abs(fd - an) < 1e-6 * max(1.0, abs(fd)), (fd, an)


def test_checkpoint_stride_is_bitwise_invisible():
    h, _, _ = spectrum_hamiltonian(200, 90, seed=41)
    w = symmetric_weight(200, seed=42)
    t1, g1 = gpu_grad(h, 90, w, stride=1)
    k = t1.info["iters"]
    _, g2 = gpu_grad(h, 90, w, stride=int(np.ceil(np.sqrt(k))))
    _, g3 = gpu_grad(h, 90, w, stride=k + 5)
    assert np.array_equal(g1, g2) and np.array_equal(g1, g3)


def test_autograd_function():
    h, _, _ = spectrum_hamiltonian(120, 50, seed=51)
    w = symmetric_weight(120, seed=52)
    H = dev(h).requires_grad_(True)
    P = dmp.Purify.apply(H, 50, 1e-10, 7)
    loss = (P * dev(w)).sum()
    loss.backward()
    torch.cuda.synchronize()
    _, g = gpu_grad(h, 50, w, tol=1e-10)
    assert np.array_equal(H.grad.cpu().numpy(), g)


def test_special_occupation_gradient_is_zero():
    h, _, _ = spectrum_hamiltonian(64, 32, seed=61)
    w = symmetric_weight(64, seed=62)
    _, g = gpu_grad(h, 0, w)
    assert np.all(g == 0.0)
