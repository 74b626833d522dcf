"""GPU parity of the Markidis-scheme product (Sec. 4.5) and its use in
purification, set beside the Ozaki scheme (the comparison of Table 2, Sec. 4.5)."""
import numpy as np
import pytest

from oracle import canonical, markidis, projector, trs4
from paper_2407_13299_amd.workloads import spectrum_hamiltonian, workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dmp = pytest.importorskip("paper_2407_13299_amd")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def gemm(a, b, terms, **kw):
    c = dmp.ozaki_gemm(dev(a), dev(b), slices=terms, kind="markidis", **kw)
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("terms", [1, 2, 3, 4])
@pytest.mark.parametrize("m,n,k", [(200, 150, 333), (64, 64, 64), (257, 96, 1000)])
def test_gemm_within_fp32_accumulation_bound(terms, m, n, k):
    rng = np.random.default_rng(m + n + k + terms)
    a = rng.standard_normal((m, k)) * np.exp2(rng.integers(-20, 20, (m, 1)))
    b = rng.standard_normal((k, n)) * np.exp2(rng.integers(-20, 20, (1, n)))
    c = gemm(a, b, terms)
    ref = markidis.markidis_gemm(a, b, terms)
    bound = markidis.fp32_accumulation_bound(a, b, terms)
    assert np.all(np.abs(c - ref) <= bound)


def test_gemm_one_term_exact_on_small_integers():
    """Entries that are exact FP16 values after the power-of-two scaling and
    sums below 2^24: the FP32 accumulation is exact, so the GPU result is the
    exact product, bit for bit."""
    rng = np.random.default_rng(5)
    a = rng.integers(-8, 9, (96, 64)).astype(np.float64) * 2.0 ** 7
    b = rng.integers(-8, 9, (64, 80)).astype(np.float64) * 2.0 ** -3
    a[:, 0] = 8 * 2.0 ** 7      # fix every row maximum (scaling exponent)
    b[0, :] = 8 * 2.0 ** -3
    assert np.array_equal(gemm(a, b, 1), a @ b)
    assert np.array_equal(gemm(a, b, 4), a @ b)      # the low parts are zero


def test_gemm_transposes_and_nonfinite_rows():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((70, 90))
    b = rng.standard_normal((50, 90))
    c = dmp.ozaki_gemm(dev(a), dev(b), slices=3, kind="markidis", trans_b=True)
    torch.cuda.synchronize()
    ref = markidis.markidis_gemm(a, b.T, 3)
    assert np.all(np.abs(c.cpu().numpy() - ref) <= markidis.fp32_accumulation_bound(a, b.T, 3))
    a[3, 5] = np.nan
    c = gemm(a, b.T.copy(), 2)
    assert np.all(np.isnan(c[3])) and np.all(np.isfinite(np.delete(c, 3, axis=0)))


def test_gemm_error_against_terms():
    rng = np.random.default_rng(7)
    a = rng.uniform(0, 1, (256, 256))
    b = rng.uniform(0, 1, (256, 256))
    ref = a @ b
    err = [np.max(np.abs(gemm(a, b, t) - ref) / ref) for t in (1, 2, 3, 4)]
    assert err[0] > 1e-5 and err[2] < 1e-6 and err[3] < 1e-6
    oz = dmp.ozaki_gemm(dev(a), dev(b), slices=7)
    assert np.max(np.abs(oz.cpu().numpy() - ref) / ref) < 1e-13


def test_markidis_purification_accuracy_class():
    """The oracle's canonical purification with its own Markidis products and
    the GPU run land in the same accuracy class (the GPU adds FP32
    accumulation noise); neither reaches the FP64 level Ozaki S = 7 reaches."""
    h, _, lam = spectrum_hamiltonian(256, 128, seed=81)
    p_ref, e_ref, _, _ = projector.eigh_projector(h, 128)
    for terms in (1, 3):
        ref = canonical.purify(h, 128, tol=1e-8, matmul=lambda x, y: markidis.markidis_gemm(x, y, terms))
        d_or = np.max(np.abs(ref["P"] - p_ref))
        p, e, info = dmp.purify(dev(h), 128, tol=1e-8, slices=terms, kind="markidis")
        torch.cuda.synchronize()
        d_gpu = np.max(np.abs(p.cpu().numpy() - p_ref))
        assert d_gpu < 30 * max(d_or, 1e-9), (terms, d_gpu, d_or)
        assert d_gpu > 1e-11
    p, e, info = dmp.purify(dev(h), 128, tol=1e-10, slices=7)
    torch.cuda.synchronize()
    assert np.max(np.abs(p.cpu().numpy() - p_ref)) < 1e-10


def test_markidis_vs_ozaki_table():
    """Errors and iterations against the number of terms on the n = 2048
    tight-binding workload (the layout of Table 2: RMSD, commutator, energy,
    energy after one FP64 McWeeny step, iterations), with Ozaki S = 5 and 7
    and FP64 beside them."""
    w = workload("tb_2048")
    h, nocc = w["H"], w["nocc"]
    p_ref, e_ref, _, _ = projector.eigh_projector(h, nocc)
    hd = dev(h)
    rows = []
    for label, kw in [("markidis 1", dict(kind="markidis", slices=1)),
                      ("markidis 2", dict(kind="markidis", slices=2)),
                      ("markidis 3", dict(kind="markidis", slices=3)),
                      ("markidis 4", dict(kind="markidis", slices=4)),
                      ("ozaki 5", dict(kind="int8", slices=5)),
                      ("ozaki 7", dict(kind="int8", slices=7)),
                      ("fp64", dict(kind="native"))]:
        p, e, info = dmp.purify(hd, nocc, tol=w["tol"], **kw)
        _, e_mixed, info_r = dmp.purify(hd, nocc, tol=w["tol"], refine=True, **kw)
        torch.cuda.synchronize()
        assert info_r["E_unrefined"] == e
        m = projector.measures(p.cpu().numpy(), e, h, nocc, p_ref, e_ref)
        rows.append((label, m["rmsd"], m["commutator"], m["dE"], abs(e_mixed - e_ref),
                     info["iters"], info["stop"]))
    print("\n  method        RMSD      commutator  |dE|      |dE| refined  iters stop")
    for r in rows:
        print(f"  {r[0]:12s} {r[1]:.2e}  {r[2]:.2e}    {r[3]:.2e}  {r[4]:.2e}      {r[5]:4d}  {r[6]}")
    by = {r[0]: r for r in rows}
    assert by["markidis 3"][1] < by["markidis 1"][1]
    assert by["ozaki 7"][1] < 1e-3 * by["markidis 4"][1]
    assert by["ozaki 7"][3] < 1e-8 and by["fp64"][3] < 1e-8
    for t in ("markidis 3", "markidis 4"):
        assert by[t][4] < by[t][3]          # refinement improves the energy
