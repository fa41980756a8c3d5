"""Krylov solvers and the AL-Uzawa iteration (oracle; test infrastructure).

* Flexible CG (Notay 2000, one-term recurrence): with a fixed symmetric
  positive definite preconditioner it is plain PCG (Sec. 3.3 uses PCG for
  the inner solve).  beta_k = z_{k+1}.(r_{k+1} - r_k) / (z_k . r_k).
  Stop at ||r||_2 <= max(rtol ||r_0||_2, atol) (relative 1e-8 and absolute
  1e-10 in Sec. 5).
* AL-Uzawa (stOpEq-ALU): p = 0; b = g + D^T p; A^eps lambda = b;
  p_K -= eps^-1 (D lambda)_K / |K|, i.e. p <- p + eps^-1 B u with
  B = -div.  (The displayed update, read with B = -div, would add
  eps^-1 div u and grow the error; the step with the contraction factor
  eps/(eps + mu_0) of Lemma 3.1 is the standard augmented-Lagrangian one.)
"""
import numpy as np


class Breakdown(ArithmeticError):
    """Flexible CG cannot continue: z.r <= 0 or p.Ap <= 0 (the preconditioner
    or the operator is not positive definite on the Krylov space; the "NA"
    entries of the paper's tables)."""


def fcg(A, b, prec, rtol=1e-8, atol=1e-10, max_it=500, x0=None):
    """Returns (x, iterations, residual history); raises Breakdown."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    hist = [np.linalg.norm(r)]
    tol = max(rtol * hist[0], atol)
    if hist[0] <= tol:
        return x, 0, hist
    z = prec(r)
    p = z.copy()
    zr = z @ r
    it = 0
    while it < max_it:
        q = A @ p
        pq = p @ q
        if not (zr > 0.0 and pq > 0.0):
            raise Breakdown(f"z.r = {zr:.3e}, p.Ap = {pq:.3e} at iteration {it + 1}")
        alpha = zr / pq
        x += alpha * p
        r_new = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r_new))
        if hist[-1] <= tol:
            break
        z_new = prec(r_new)
        beta = (z_new @ (r_new - r)) / zr
        zr = z_new @ r_new
        p = z_new + beta * p
        r, z = r_new, z_new
    return x, it, hist


def uzawa(Aeps, D, area, g, eps_inv, inner, max_steps=50, tol=1e-10, flux_b=None):
    """AL-Uzawa.  inner(b) -> (lambda, its, hist).  Stops when
    ||p^n - p^{n-1}||_{L2} <= tol * max(1, ||p^n||_{L2}) or after max_steps
    (tol < 0: exactly max_steps).  flux_b: per-cell flux of prescribed
    normal boundary values (the constraint is D lambda + flux_b = 0).
    Returns (lambda, p0, list of (its, hist))."""
    p = np.zeros(D.shape[0])
    fb = np.zeros(D.shape[0]) if flux_b is None else flux_b
    g = g - eps_inv * (D.T @ (fb / area))
    log = []
    lam = None
    for n in range(max_steps):
        b = g + D.T @ p
        lam, its, hist = inner(b)
        log.append((its, hist))
        dp = -eps_inv * (D @ lam + fb) / area
        p = p + dp
        dn = np.sqrt(np.sum(area * dp ** 2))
        pn = np.sqrt(np.sum(area * p ** 2))
        if dn <= tol * max(1.0, pn):
            break
    return lam, p, log
