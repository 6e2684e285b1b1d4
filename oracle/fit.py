"""Constrained linear fitting of the cheap potential: the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg. The product package never imports it.

Follows "Constrained potential fitting" (Methods): the cheap potential is
linear in its spline coefficients, so its energies and forces are A c for a
design matrix A; soft data (A_S, y_S) is matched in the least-squares sense
while the hard data (A_H, y_H) must satisfy ||A_H c - y_H||^2 < alpha. The
augmented Lagrangian turns this into the unconstrained problem
min ||y_S - A_S c||^2 + lam ||y_H - A_H c||^2 at fixed lam, whose minimiser
solves the normal equations (gradient zero); lam is searched by increasing it
by decades until the hard constraint holds, then by interval bisection.

Free parameters u of the cheap model (clamped cubic B-splines):
  2-body: for each species pair za <= zb, c2[za][zb][n] = c2[zb][za][n] for
          n < nb2 - 3 (the last three vanish so that V2 reaches zero at its
          cutoff);
  3-body: for each centre species z, c3[z][p][q][s] = c3[z][q][p][s] for
          p <= q < nb3 - 3 and every s < nb3 (the last three along each leg
          vanish).
Columns are ordered 2-body first (za, zb, n), then 3-body (z, p, q, s), the
last index fastest.
"""
import numpy as np

from oracle import neighbors, uf3


def layout(model):
    """List of column descriptors: ("2", za, zb, n) or ("3", z, p, q, s)."""
    u = model["uf3"]
    ns = model["n_species"]
    nb2 = u["n_knots2"] + 2
    cols = []
    for za in range(ns):
        for zb in range(za, ns):
            for n in range(nb2 - 3):
                cols.append(("2", za, zb, n))
    if u["n_knots3"] > 0:
        nb3 = u["n_knots3"] + 2
        for z in range(ns):
            for p in range(nb3 - 3):
                for q in range(p, nb3 - 3):
                    for s in range(nb3):
                        cols.append(("3", z, p, q, s))
    return cols


def n_params(model):
    return len(layout(model))


def params_to_model(model, x):
    """The model with its cheap coefficients filled from the parameter vector
    x (the symmetric copies written out)."""
    u = dict(model["uf3"])
    ns = model["n_species"]
    nb2 = u["n_knots2"] + 2
    c2 = np.zeros((ns, ns, nb2))
    nb3 = u["n_knots3"] + 2 if u["n_knots3"] > 0 else 1
    c3 = np.zeros((ns, nb3, nb3, nb3))
    for v, col in zip(x, layout(model)):
        if col[0] == "2":
            _, za, zb, n = col
            c2[za, zb, n] = v
            c2[zb, za, n] = v
        else:
            _, z, p, q, s = col
            c3[z, p, q, s] = v
            c3[z, q, p, s] = v
    u["c2"], u["c3"] = c2, c3
    return dict(model, uf3=u)


def design(model, pos, species, L, periodic):
    """Design matrix of one configuration, (1 + 3n) x n_params: row 0 holds
    the total energy's derivatives by each parameter, row 1 + q n + i those
    of force component q on atom i. Column k is the cheap potential evaluated
    with the unit parameter vector e_k (the plain definition of a linear
    model's design matrix)."""
    pos = np.asarray(pos, np.float64)
    n = len(pos)
    r_list = max(model["uf3"]["rcut2"], model["uf3"]["rcut3"]) + 0.5
    offs, nbr = neighbors(pos, L, periodic, r_list)
    nd = n_params(model)
    A = np.zeros((1 + 3 * n, nd))
    for k in range(nd):
        e = np.zeros(nd)
        e[k] = 1.0
        m = params_to_model(model, e)
        ei, f = uf3(m, pos, species, L, periodic, offs, nbr)
        A[0, k] = ei.sum()
        A[1:, k] = f.T.reshape(-1)
    return A


def gram(A, y, w):
    """G = A^T diag(w) A and b = A^T diag(w) y."""
    Aw = A * w[:, None]
    return A.T @ Aw, Aw.T @ y


def solve_fixed(GS, bS, GH, bH, lam, ridge):
    """Minimiser of ||y_S - A_S c||^2 + lam ||y_H - A_H c||^2 + ridge ||c||^2:
    its gradient vanishes where (G_S + lam G_H + ridge I) c = b_S + lam b_H."""
    nd = len(bS)
    return np.linalg.solve(GS + lam * GH + ridge * np.eye(nd), bS + lam * bH)


def hard_residual(AH, yH, c, wH=None):
    r = AH @ c - yH
    if wH is None:
        return float(r @ r)
    return float(r @ (wH * r))


def constrained_fit(GS, bS, AH, yH, alpha, lam0=1.0, ridge=0.0, tol=None, max_decades=24,
                    max_bisect=200, wH=None):
    """The lambda search: solve at lam0, 10 lam0, 100 lam0, ... until the hard
    residual is at most alpha, then bisect between the last failing and the
    first passing lambda until the passing end's residual is within tol of
    alpha (tol = alpha/10 by default). Returns (c, info) with info = dict(lam,
    residual, n_solves, status, trace) and status 0 = converged, 1 = alpha not
    reached within max_decades (the solution with the smallest residual seen
    is returned), 2 = bisection limit reached (the passing end is returned).
    wH (optional) weights the hard rows: the residual is sum wH (A_H c - y_H)^2
    (per-atom energies from total-energy rows with wH = 1/n^2)."""
    if tol is None:
        tol = alpha / 10.0
    if wH is None:
        wH = np.ones(len(yH))
    GH, bH = gram(AH, yH, wH)
    trace = []

    def run(lam):
        c = solve_fixed(GS, bS, GH, bH, lam, ridge)
        r = hard_residual(AH, yH, c, wH)
        trace.append((lam, r))
        return c, r

    lam = lam0
    c, r = run(lam)
    best = (r, lam, c)
    dec = 0
    while r > alpha and dec < max_decades:
        lam_lo = lam
        lam = lam * 10.0
        dec += 1
        c, r = run(lam)
        if r < best[0]:
            best = (r, lam, c)
    if r > alpha:
        r, lam, c = best
        return c, dict(lam=lam, residual=r, n_solves=len(trace), status=1, trace=trace)
    if dec == 0:
        return c, dict(lam=lam, residual=r, n_solves=len(trace), status=0, trace=trace)
    lo, hi, c_hi, r_hi = lam_lo, lam, c, r
    status = 0
    it = 0
    while not (alpha - r_hi < tol):
        if it == max_bisect:
            status = 2
            break
        mid = 0.5 * (lo + hi)
        c, r = run(mid)
        if r <= alpha:
            hi, c_hi, r_hi = mid, c, r
        else:
            lo = mid
        it += 1
    return c_hi, dict(lam=hi, residual=r_hi, n_solves=len(trace), status=status, trace=trace)
