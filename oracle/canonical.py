"""Canonical density-matrix purification in FP64 (test infrastructure).

The paper proposes Ozaki-scheme products inside density-matrix purification
(Sec. 1, citing Palser and Manolopoulos' canonical purification; Sec. 2.3 gives
McWeeny's grand-canonical form).  Canonical purification fixes the electron
count instead of the chemical potential:

  initial guess   P0 = lam (mu I - H) + theta I,  theta = nocc / n,
                  mu = tr(H) / n,
                  lam = min(theta / (h_max - mu), (1 - theta) / (mu - h_min)),
                  with [h_min, h_max] Gershgorin bounds of the spectrum of H,
                  so every eigenvalue of P0 lies in [0, 1] and tr P0 = nocc;
  coefficient     c = tr(P^2 - P^3) / tr(P - P^2), clamped to [0, 1];
  update          c >= 1/2:  P <- ((1 + c) P^2 - P^3) / c
                  c <  1/2:  P <- ((1 - 2c) P + (1 + c) P^2 - P^3) / (1 - c)
  energy          E = tr(P H);
  stopping        Sec. 3: converged when |E_k - E_{k-1}| < tol; stagnated
                  when the energy rose in each of the last two iterations
                  while changing by less than 1e-2 Ha; otherwise stop at
                  max_iter.  A non-finite energy (a run whose products are
                  far too coarse diverges) stops at once.

Readings where the paper is silent (listed in the design notes): the
Gershgorin bounds, c = 1/2 on the c >= 1/2 branch, c = 1/2 when tr(P - P^2)
is exactly zero, the clamp, the traces taken from the diagonals of the
differences P - P^2 and P^2 - P^3, and a default cap of 200 iterations.

Both updates are polynomials in P, so the iteration acts on every eigenvalue
of P separately; ``eigen_simulate`` runs the same map on the eigenvalues of
H and predicts the iteration count, c_k, the branches and E_k.
"""
from __future__ import annotations

import numpy as np

STOP_CONVERGED, STOP_STAGNATED, STOP_MAX_ITER, STOP_NONFINITE = 0, 1, 2, 3
STAGNATION_WINDOW = 1e-2


def gershgorin(h):
    """(h_min, h_max): every eigenvalue of symmetric h lies in this interval."""
    d = np.diag(h)
    r = np.sum(np.abs(h), axis=1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))


def initial_scalars(h, nocc):
    """(theta, mu, lam, h_min, h_max, which) of the canonical initial guess.

    ``which`` is 0 when lam = theta / (h_max - mu) is the smaller bound and 1
    when lam = (1 - theta) / (mu - h_min) is.
    """
    n = h.shape[0]
    theta = nocc / n
    mu = float(np.trace(h)) / n
    h_min, h_max = gershgorin(h)
    a = theta / (h_max - mu)
    b = (1.0 - theta) / (mu - h_min)
    which = 0 if a <= b else 1
    return theta, mu, min(a, b), h_min, h_max, which


def initial_guess(h, nocc):
    theta, mu, lam, _, _, _ = initial_scalars(h, nocc)
    n = h.shape[0]
    return lam * (mu * np.eye(n) - h) + theta * np.eye(n)


def coefficient(p, p2, p3):
    """(c, t1, t2) with t1 = tr(P - P^2), t2 = tr(P^2 - P^3), c clamped."""
    t1 = float(np.trace(p - p2))
    t2 = float(np.trace(p2 - p3))
    c = 0.5 if t1 == 0.0 else t2 / t1
    return min(max(c, 0.0), 1.0), t1, t2


def update_weights(c):
    """(alpha, beta, gamma) with P_new = alpha P + beta P^2 + gamma P^3."""
    if c >= 0.5:
        return 0.0, (1.0 + c) / c, -1.0 / c
    return (1.0 - 2.0 * c) / (1.0 - c), (1.0 + c) / (1.0 - c), -1.0 / (1.0 - c)


def purify(h, nocc, tol=1e-8, max_iter=200, matmul=np.matmul):
    """Run canonical purification with the given matrix product.

    Returns dict(P, E, iters, stop, history) where history holds, per
    iteration k, (c_k, branch_k, t1_k, t2_k, E_{k+1}).  ``matmul`` lets the
    tests run the same driver with an emulated product.
    """
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    if nocc == 0 or nocc == n:
        p = np.zeros((n, n)) if nocc == 0 else np.eye(n)
        return dict(P=p, E=float(np.trace(p @ h)), iters=0,
                    stop=STOP_CONVERGED, history=[])
    p = initial_guess(h, nocc)
    e_prev2 = None
    e_prev = float(np.sum(p * h))
    history = []
    stop = STOP_MAX_ITER
    for k in range(max_iter):
        p2 = matmul(p, p)
        p3 = matmul(p2, p)
        c, t1, t2 = coefficient(p, p2, p3)
        a, b, g = update_weights(c)
        p = a * p + b * p2 + g * p3
        e = float(np.sum(p * h))
        history.append((c, int(c >= 0.5), t1, t2, e))
        de = e - e_prev
        if not np.isfinite(e):
            stop = STOP_NONFINITE
            e_prev2, e_prev = e_prev, e
            break
        if abs(de) < tol:
            stop = STOP_CONVERGED
            e_prev2, e_prev = e_prev, e
            break
        if (e_prev2 is not None and de > 0 and e_prev - e_prev2 > 0
                and abs(de) < STAGNATION_WINDOW):
            stop = STOP_STAGNATED
            e_prev2, e_prev = e_prev, e
            break
        e_prev2, e_prev = e_prev, e
    return dict(P=p, E=e_prev, iters=len(history), stop=stop, history=history)


def eigen_simulate(h, nocc, tol=1e-8, max_iter=200):
    """The canonical iteration applied to the eigenvalues of P (FP64).

    x_0 = lam (mu - eps) + theta;  c, the update and E = sum x eps are the
    eigenvalue forms of the matrix expressions above.
    """
    eps = np.linalg.eigvalsh(h)
    n = h.shape[0]
    theta, mu, lam, _, _, _ = initial_scalars(h, nocc)
    x = lam * (mu - eps) + theta
    e_prev2, e_prev = None, float(np.sum(x * eps))
    history = []
    stop = STOP_MAX_ITER
    for _ in range(max_iter):
        t1 = float(np.sum(x - x * x))
        t2 = float(np.sum(x * x - x * x * x))
        c = 0.5 if t1 == 0.0 else t2 / t1
        c = min(max(c, 0.0), 1.0)
        a, b, g = update_weights(c)
        x = a * x + b * x * x + g * x * x * x
        e = float(np.sum(x * eps))
        history.append((c, int(c >= 0.5), t1, t2, e))
        de = e - e_prev
        if abs(de) < tol:
            stop = STOP_CONVERGED
            e_prev = e
            break
        if (e_prev2 is not None and de > 0 and e_prev - e_prev2 > 0
                and abs(de) < STAGNATION_WINDOW):
            stop = STOP_STAGNATED
            e_prev = e
            break
        e_prev2, e_prev = e_prev, e
    del n
    return dict(x=x, E=e_prev, iters=len(history), stop=stop, history=history)
