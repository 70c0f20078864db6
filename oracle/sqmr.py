"""SQMR (Freund & Nachtigal) with the multigrid preconditioner: paper Alg. 4.

Reading (variant): Alg. 4 is SQMR with the left preconditioner factor equal
to the V-cycle W and the right factor equal to the identity; its nu_j is the
quasi-residual ratio (theta in Freund & Nachtigal), nu_0 = 0 and d_0 = 0.
The initial guess x0 may be non-zero (a warm start); the V-cycle inside
always starts from zero.
Reading (convergence): stop at the first j with ||b - L x_j||_2 <=
rtol ||b||_2, the true residual recomputed every iteration, relative to
||b|| (Section 6 stops at relative residual 1e-8).
Reading (breakdown): sigma = 0 or rho = 0 ends the iteration with status
"breakdown"; a non-finite scalar ends it with "nonfinite"; b = 0 returns
x = 0.
"""
from __future__ import annotations

import math

import numpy as np

from .multigrid import Hierarchy, apply_L, vcycle
from .operator import from_vector, to_vector


def sqmr(apply_A, apply_W, b, x0, rtol=1e-8, maxit=200, on_iterate=None):
    """Alg. 4 on flat vectors.  Returns (x, info).

    `on_iterate(j, x_j, s_j)` is called after each iteration's update of x.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.linalg.norm(b))
    info = {"iters": 0, "status": "converged", "relres": []}
    if bnorm == 0.0:
        info["relres"].append(0.0)
        return np.zeros_like(b), info
    s = b - apply_A(x)
    info["relres"].append(float(np.linalg.norm(s)) / bnorm)
    if info["relres"][0] <= rtol:
        return x, info
    t = apply_W(s)
    q = t.copy()
    tau = float(np.linalg.norm(t))
    nu_prev = 0.0
    rho = float(np.dot(s, q))
    d = np.zeros_like(b)
    for j in range(1, maxit + 1):
        t = apply_A(q)
        sigma = float(np.dot(q, t))
        if not math.isfinite(sigma):
            info["status"] = "nonfinite"
            break
        if sigma == 0.0:
            info["status"] = "breakdown"
            break
        alpha = rho / sigma
        s = s - alpha * t
        t = apply_W(s)
        nu = float(np.linalg.norm(t)) / tau
        c = 1.0 / math.sqrt(1.0 + nu * nu)
        tau = tau * nu * c
        d = (c * c * nu_prev * nu_prev) * d + (c * c * alpha) * q
        x = x + d
        nu_prev = nu
        res = float(np.linalg.norm(b - apply_A(x))) / bnorm
        info["iters"] = j
        info["relres"].append(res)
        if on_iterate is not None:
            on_iterate(j, x, s)
        if not math.isfinite(res):
            info["status"] = "nonfinite"
            break
        if res <= rtol:
            info["status"] = "converged"
            return x, info
        if rho == 0.0:
            info["status"] = "breakdown"
            break
        rho_new = float(np.dot(s, t))
        beta = rho_new / rho
        q = t + beta * q
        rho = rho_new
    else:
        info["status"] = "maxit"
    return x, info


def mg_sqmr(H: Hierarchy, b, x0=None, rtol=1e-8, maxit=200, on_iterate=None, precondition=True):
    """MG-SQMR (Alg. 4) on state tuples: the system matrix is L, the
    preconditioner one V-cycle on L~.  `precondition=False` uses W = I."""
    dom = H.doms[0]
    bv = to_vector(dom, b)
    xv = np.zeros_like(bv) if x0 is None else to_vector(dom, x0)

    def apply_A(v):
        return to_vector(dom, apply_L(H, from_vector(dom, v)))

    def apply_W(v):
        if not precondition:
            return v.copy()
        return to_vector(dom, vcycle(H, from_vector(dom, v)))

    cb = None
    if on_iterate is not None:
        def cb(j, v, s):
            on_iterate(j, from_vector(dom, v))
    x, info = sqmr(apply_A, apply_W, bv, xv, rtol, maxit, cb)
    return from_vector(dom, x), info


def remove_pressure_mean(dom, x):
    """Subtract the mean of p over the active cells (the closed box leaves the
    pressure defined up to a constant)."""
    p = x[3]
    m = dom.active[3]
    mean = p[m].mean()
    return x[:3] + (np.where(m, p - mean, 0.0),)
