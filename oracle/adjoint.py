"""Derivatives of the density matrix with respect to H (test infrastructure).

Two independent routes to dL/dH for L = tr(P W), W symmetric:

* ``perturbation_gradient``: first-order perturbation theory of the exact
  projector.  With H = U diag(eps) U^T and W~ = U^T W U,
      dL/dH = U (M o W~) U^T,
      M_pq = 1 / (eps_occ - eps_virt) when exactly one of p, q is occupied
             (eps_occ the occupied one's level), 0 otherwise.
  Occupied-occupied and virtual-virtual rotations leave P unchanged, which is
  why only the occupied-virtual block survives.

* ``canonical_adjoint``: reverse-mode differentiation of the canonical
  purification sequence (initial guess, K updates) at a fixed branch
  pattern, including the dependence of every c_k on P_k and of the initial
  guess on tr H and on the Gershgorin bounds (a subgradient: the extremal
  row is held fixed).  For a symmetric adjoint Y of P_{k+1}
  and the update alpha P + beta P^2 + gamma P^3:
      Pbar = alpha Y + beta (Y P + P Y) + gamma (Y P^2 + P Y P + P^2 Y)
             + cbar * dc/dP,
      cbar  = <Y, alpha' P + beta' P^2 + gamma' P^3>,
      dc/dP = ((2P - 3P^2) t1 - t2 (I - 2P)) / t1^2.
  Returned gradients are symmetrised, so <G, D> is the directional
  derivative along any symmetric D.
"""
from __future__ import annotations

import numpy as np

from .canonical import initial_scalars, update_weights


def perturbation_gradient(h, nocc, w):
    eps, u = np.linalg.eigh(np.asarray(h, dtype=np.float64))
    n = len(eps)
    occ = np.arange(n) < nocc
    wt = u.T @ w @ u
    diff = eps[:, None] - eps[None, :]
    m = np.zeros((n, n))
    ov = occ[:, None] & ~occ[None, :]          # p occupied, q virtual
    m[ov] = 1.0 / diff[ov]
    vo = ~occ[:, None] & occ[None, :]          # p virtual, q occupied
    m[vo] = -1.0 / diff[vo]
    g = u @ (m * wt) @ u.T
    return 0.5 * (g + g.T)


def weight_derivatives(c, branch):
    """d(alpha, beta, gamma)/dc on the given branch (1: c >= 1/2)."""
    if branch:
        return 0.0, -1.0 / c ** 2, 1.0 / c ** 2
    q = (1.0 - c) ** 2
    return -1.0 / q, 2.0 / q, -1.0 / q


def branch_weights(c, branch):
    if branch:
        return 0.0, (1.0 + c) / c, -1.0 / c
    return (1.0 - 2.0 * c) / (1.0 - c), (1.0 + c) / (1.0 - c), -1.0 / (1.0 - c)


def fixed_pattern_forward(h, nocc, branches):
    """Canonical iterates with the branch of step k forced to branches[k].

    c_k is still recomputed from P_k (clamped to [0, 1]); returns the final P
    and a tape of (P, P2, P3, c, t1, t2, clamped) per step.
    """
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    theta, mu, lam, _, _, _ = initial_scalars(h, nocc)
    p = lam * (mu * np.eye(n) - h) + theta * np.eye(n)
    tape = []
    for br in branches:
        p2 = p @ p
        p3 = p2 @ p
        t1 = float(np.trace(p - p2))
        t2 = float(np.trace(p2 - p3))
        raw = 0.5 if t1 == 0.0 else t2 / t1
        c = min(max(raw, 0.0), 1.0)
        clamped = (t1 == 0.0) or (raw != c)
        tape.append((p, p2, p3, c, t1, t2, clamped))
        a, b, g = branch_weights(c, br)
        p = a * p + b * p2 + g * p3
    return p, tape


def loss(h, nocc, w, branches):
    p, _ = fixed_pattern_forward(h, nocc, branches)
    return float(np.sum(p * w))


def canonical_adjoint(h, nocc, w, branches):
    """dL/dH of L = tr(P_K W) through K canonical steps with fixed branches."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    eye = np.eye(n)
    _, tape = fixed_pattern_forward(h, nocc, branches)
    y = np.array(w, dtype=np.float64)
    for (p, p2, p3, c, t1, t2, clamped), br in zip(tape[::-1], branches[::-1]):
        a, b, g = branch_weights(c, br)
        m = y @ p
        mp = m @ p
        pm = p @ m
        pbar = a * y + b * (m + m.T) + g * (mp + mp.T + pm)
        if not clamped:
            da, db, dg = weight_derivatives(c, br)
            cbar = da * np.sum(y * p) + db * np.sum(y * p2) + dg * np.sum(y * p3)
            dc = ((2.0 * p - 3.0 * p2) * t1 - t2 * (eye - 2.0 * p)) / t1 ** 2
            pbar = pbar + cbar * dc
        y = 0.5 * (pbar + pbar.T)
    theta, mu, lam, h_min, h_max, which = initial_scalars(h, nocc)
    gbar = -lam * y + (lam * np.trace(y) / n) * eye
    lambar = mu * np.trace(y) - np.sum(y * h)
    diag = np.diag(h)
    off = np.sum(np.abs(h), axis=1) - np.abs(diag)
    sgn = np.sign(h)
    if which == 0:
        i = int(np.argmax(diag + off))
        dext = np.zeros((n, n))
        dext[i, :] = sgn[i, :]
        dext[i, i] = 1.0
        dlam = -theta / (h_max - mu) ** 2 * (dext - eye / n)
    else:
        i = int(np.argmin(diag - off))
        dext = np.zeros((n, n))
        dext[i, :] = -sgn[i, :]
        dext[i, i] = 1.0
        dlam = -(1.0 - theta) / (mu - h_min) ** 2 * (eye / n - dext)
    gbar = gbar + lambar * dlam
    return 0.5 * (gbar + gbar.T)
