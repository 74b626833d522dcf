"""Trace-resetting fourth-order purification (TRS4) and the one-step McWeeny
refinement, in FP64 (test infrastructure).

TRS4 is the purification the paper runs (Sec. 3, citing Niklasson, Tymczak
and Challacombe 2003).  Its polynomials, from that method's definition:

  initial guess   X0 = (h_max I - H) / (h_max - h_min), Gershgorin bounds,
                  so the spectrum of X0 lies in [0, 1] with the lowest levels
                  of H nearest 1;
  polynomials     F(X) = X^2 (4X - 3X^2),   G(X) = X^2 (I - X)^2;
  trace reset     gamma = (nocc - tr F) / tr G;
  update          0 <= gamma <= 6:  X <- F + gamma G   (then tr X = nocc)
                  gamma > 6:        X <- 2X - X^2      (raises the trace)
                  gamma < 0:        X <- X^2           (lowers the trace)
  energy, stop    E = tr(X H) and the stopping rule of Sec. 3, as in the
                  canonical module.

Reading where neither source fixes it: when tr G is exactly zero (X^2 = X,
so every branch returns X), gamma is taken as 0 on the in-range branch.

F + gamma G = X^2 T with T = (4 - 2 gamma) X + (gamma - 3) X^2 + gamma I, so
one TRS4 step costs two products, like a canonical step; the oracle forms F
and G as written, with plain products.

McWeeny refinement (Sec. 4.1): after purification has stopped, one step
P <- 3 P^2 - 2 P^3 in full FP64 (Sec. 2.3 gives the recurrence); the paper
reports that it recovers the energy of a low-precision run.
"""
from __future__ import annotations

import numpy as np

from .canonical import (STAGNATION_WINDOW, STOP_CONVERGED, STOP_MAX_ITER,
                        STOP_NONFINITE, STOP_STAGNATED, gershgorin)

GAMMA_MIN, GAMMA_MAX = 0.0, 6.0
BRANCH_SQUARE, BRANCH_RESET, BRANCH_RAISE = 0, 1, 2


def initial_guess(h):
    """X0 = (h_max I - H) / (h_max - h_min)."""
    h_min, h_max = gershgorin(h)
    n = h.shape[0]
    return (h_max * np.eye(n) - h) / (h_max - h_min)


def polynomials(x, matmul=np.matmul):
    """(X^2, F, G) with F = X^2 (4X - 3X^2), G = X^2 (I - X)^2."""
    n = x.shape[0]
    i = np.eye(n)
    x2 = matmul(x, x)
    f = matmul(x2, 4.0 * x - 3.0 * x2)
    g = matmul(x2, matmul(i - x, i - x))
    return x2, f, g


def reset_coefficient(nocc, tr_f, tr_g):
    """(gamma, branch): gamma = (nocc - tr F) / tr G and the branch it picks."""
    gamma = 0.0 if tr_g == 0.0 else (nocc - tr_f) / tr_g
    if gamma > GAMMA_MAX:
        return gamma, BRANCH_RAISE
    if gamma < GAMMA_MIN:
        return gamma, BRANCH_SQUARE
    return gamma, BRANCH_RESET


def step(x, nocc, matmul=np.matmul):
    """One TRS4 update; returns (X_new, gamma, branch, tr F, tr G)."""
    x2, f, g = polynomials(x, matmul)
    tr_f = float(np.trace(f))
    tr_g = float(np.trace(g))
    gamma, branch = reset_coefficient(nocc, tr_f, tr_g)
    if branch == BRANCH_RESET:
        x_new = f + gamma * g
    elif branch == BRANCH_RAISE:
        x_new = 2.0 * x - x2
    else:
        x_new = x2
    return x_new, gamma, branch, tr_f, tr_g


def purify(h, nocc, tol=1e-8, max_iter=200, matmul=np.matmul):
    """TRS4 purification; returns dict(P, E, iters, stop, history) with
    history[k] = (gamma_k, branch_k, trF_k, trG_k, E_{k+1})."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    if nocc == 0 or nocc == n:
        p = np.zeros((n, n)) if nocc == 0 else np.eye(n)
        return dict(P=p, E=float(np.trace(p @ h)), iters=0,
                    stop=STOP_CONVERGED, history=[])
    x = initial_guess(h)
    e_prev2 = None
    e_prev = float(np.sum(x * h))
    history = []
    stop = STOP_MAX_ITER
    for _ in range(max_iter):
        x, gamma, branch, tr_f, tr_g = step(x, nocc, matmul)
        e = float(np.sum(x * h))
        history.append((gamma, branch, tr_f, tr_g, e))
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
    return dict(P=x, E=e_prev, iters=len(history), stop=stop, history=history)


def eigen_simulate(h, nocc, tol=1e-8, max_iter=200):
    """TRS4 on the eigenvalues of X (scalar polynomials, FP64); returns
    dict(x, eps, E, iters, stop, history) like ``purify``."""
    eps = np.linalg.eigvalsh(h)
    h_min, h_max = gershgorin(h)
    x = (h_max - eps) / (h_max - h_min)
    e_prev2, e_prev = None, float(np.sum(x * eps))
    history = []
    stop = STOP_MAX_ITER
    for _ in range(max_iter):
        x2 = x * x
        f = x2 * (4.0 * x - 3.0 * x2)
        g = x2 * (1.0 - x) ** 2
        gamma, branch = reset_coefficient(nocc, float(np.sum(f)), float(np.sum(g)))
        if branch == BRANCH_RESET:
            x = f + gamma * g
        elif branch == BRANCH_RAISE:
            x = 2.0 * x - x2
        else:
            x = x2
        e = float(np.sum(x * eps))
        history.append((gamma, branch, float(np.sum(f)), float(np.sum(g)), e))
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
    return dict(x=x, eps=eps, E=e_prev, iters=len(history), stop=stop, history=history)


def mcweeny_refine(p, h):
    """One FP64 McWeeny step P' = 3P^2 - 2P^3; returns (P', tr(P' H))."""
    p2 = p @ p
    p_new = 3.0 * p2 - 2.0 * (p2 @ p)
    return p_new, float(np.sum(p_new * h))
