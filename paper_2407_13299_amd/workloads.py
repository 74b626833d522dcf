"""Seeded synthetic Hamiltonians (inputs only; none of the purification or
Ozaki arithmetic lives here).

The paper's test Hamiltonians (Sec. 4: DFT runs on Molnupiravir, selenite and
water clusters) are not available, so two synthetic families with the same
structure stand in for them: dense, real symmetric, orthogonal-basis
mean-field Hamiltonians of an insulator (a gap at the Fermi level), in Hartree.

* ``spectrum_hamiltonian``: H = Q diag(lambda) Q^T with a Haar-like orthogonal
  Q and a chosen spectrum (occupied levels in [-1, -0.1], virtual levels in
  [0.1, 1]), so the exact projector and energy are known in closed form.
* ``tight_binding_hamiltonian``: a periodic simple-cubic lattice with one s and
  three p orbitals per site (s at -0.5 Ha, p at +0.5 Ha), nearest-neighbour
  sigma-only Slater-Koster hoppings of magnitude 0.1 Ha and Gaussian on-site
  disorder.  At quarter filling (one electron pair per site) the clean model
  has a 0.2 Ha gap between the s-like and the p-like bands.

All generators use numpy's PCG64 ``default_rng`` and return float64 arrays
that are exactly symmetric.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "spectrum_hamiltonian",
    "tight_binding_hamiltonian",
    "symmetric_weight",
    "symmetric_direction",
    "batched_spectrum_sizes",
    "workload",
]


def spectrum_hamiltonian(n: int, nocc: int, seed: int,
                         occ=(-1.0, -0.1), virt=(0.1, 1.0)):
    """H = Q diag(lam) Q^T, Q from the QR factorisation of an N(0,1) matrix.

    The ``nocc`` occupied levels are U[occ], the rest U[virt]; both sets are
    drawn from the same generator after Q.  Returns (H, Q, lam) with ``lam``
    in the order of the columns of Q (not sorted).
    """
    if not (0 <= nocc <= n):
        raise ValueError("nocc must lie in [0, n]")
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    # fix the sign ambiguity of QR so Q does not depend on LAPACK conventions
    q = q * np.sign(np.diag(r))[None, :]
    lam = np.concatenate([rng.uniform(occ[0], occ[1], nocc),
                          rng.uniform(virt[0], virt[1], n - nocc)])
    h = (q * lam[None, :]) @ q.T
    h = 0.5 * (h + h.T)
    return h, q, lam


# orbital order on every site: s, p_x, p_y, p_z
_S, _PX = 0, 1


def tight_binding_hamiltonian(lx: int, ly: int, lz: int, seed: int | None,
                              e_s=-0.5, e_p=0.5, t=0.1, disorder=0.02):
    """Periodic sp^3-basis tight-binding Hamiltonian on an lx*ly*lz lattice.

    Site (x, y, z) has index (x*ly + y)*lz + z and its orbitals occupy rows
    4*site + (s, p_x, p_y, p_z).  Between a site r and its neighbour r + d
    along Cartesian axis d, the sigma-only Slater-Koster elements are
        <s(r)|H|s(r+d)>     = -t
        <s(r)|H|p_d(r+d)>   = +t,    <p_d(r)|H|s(r+d)> = -t
        <p_d(r)|H|p_d(r+d)> = +t
    and every pi element is zero.  On-site energies are e_s and e_p plus
    independent N(0, disorder^2) noise on each diagonal entry (no noise when
    ``seed`` is None or ``disorder`` is 0).  Needs every l >= 3 so that the
    two neighbours along an axis are distinct sites.
    """
    for l in (lx, ly, lz):
        if l < 3:
            raise ValueError("every lattice length must be >= 3")
    nsite = lx * ly * lz
    n = 4 * nsite
    h = np.zeros((n, n))
    x, y, z = np.meshgrid(np.arange(lx), np.arange(ly), np.arange(lz),
                          indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    site = (x * ly + y) * lz + z
    onsite = np.tile(np.array([e_s, e_p, e_p, e_p]), nsite)
    if seed is not None and disorder != 0.0:
        rng = np.random.default_rng(seed)
        onsite = onsite + rng.normal(0.0, disorder, n)
    h[np.arange(n), np.arange(n)] = onsite

    def put(i, j, v):
        h[i, j] += v
        h[j, i] += v

    for d, (dx, dy, dz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        nb = (((x + dx) % lx) * ly + (y + dy) % ly) * lz + (z + dz) % lz
        put(4 * site + _S, 4 * nb + _S, -t)
        put(4 * site + _S, 4 * nb + _PX + d, +t)
        put(4 * site + _PX + d, 4 * nb + _S, -t)
        put(4 * site + _PX + d, 4 * nb + _PX + d, +t)
    return h


def symmetric_weight(n: int, seed: int):
    """W with upper triangle (incl. diagonal) iid N(0,1)/sqrt(n), mirrored."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) / np.sqrt(n)
    u = np.triu(a)
    return u + np.triu(u, 1).T


def symmetric_direction(n: int, seed: int):
    """Random symmetric direction D (same recipe as ``symmetric_weight``)."""
    return symmetric_weight(n, seed)


def batched_spectrum_sizes(count: int, seed: int, lo=128, hi=1536):
    """Integer sizes n ~ U{lo..hi} (inclusive)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count)


def workload(name: str):
    """The named synthetic workloads.

    Returns a dict with H (or a list of them), nocc, tol and a description.
      small_spectrum   n=256 spectrum-controlled, nocc=128, tol 1e-12
      tb_2048          8^3 tight-binding lattice, n=2048, nocc=512
      tb_8192          16x16x8 tight-binding lattice, n=8192, nocc=2048
      batched_64       64 spectrum-controlled H, n ~ U{128..1536}, nocc=n//2
      adjoint_2048     tb_2048's H plus a symmetric weight W (L = tr(P W))
    """
    if name == "small_spectrum":
        h, _, _ = spectrum_hamiltonian(256, 128, seed=0)
        return dict(H=h, nocc=128, tol=1e-12,
                    desc="spectrum-controlled H, n=256, nocc=128")
    if name == "tb_2048":
        h = tight_binding_hamiltonian(8, 8, 8, seed=1)
        return dict(H=h, nocc=512, tol=1e-8,
                    desc="sp3 tight binding 8x8x8, n=2048, nocc=512")
    if name == "tb_8192":
        h = tight_binding_hamiltonian(16, 16, 8, seed=2)
        return dict(H=h, nocc=2048, tol=1e-8,
                    desc="sp3 tight binding 16x16x8, n=8192, nocc=2048")
    if name == "batched_64":
        sizes = batched_spectrum_sizes(64, seed=3)
        hs = [spectrum_hamiltonian(int(m), int(m) // 2, seed=1000 + b)[0]
              for b, m in enumerate(sizes)]
        return dict(H=hs, nocc=[int(m) // 2 for m in sizes], tol=1e-8,
                    desc="64 spectrum-controlled H, n~U{128..1536}, nocc=n//2")
    if name == "adjoint_2048":
        h = tight_binding_hamiltonian(8, 8, 8, seed=1)
        return dict(H=h, nocc=512, tol=1e-8, W=symmetric_weight(2048, seed=4),
                    desc="tb_2048 with L = tr(P W)")
    raise KeyError(name)
