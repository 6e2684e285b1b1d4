"""Pins of the constrained-fit oracle against what the B-spline definition,
calculus and an independent constrained optimiser fix ("Constrained potential
fitting" and "Generation of synthetic data", Methods)."""
import numpy as np
import pytest
from scipy.interpolate import BSpline
from scipy.optimize import minimize

import oracle as O
from oracle import fit as OF
from gen import fitdata as FD
from gen.lattice import A_W


def _knots(n_pts, top):
    return np.concatenate([[0.0] * 3, np.linspace(0.0, top, n_pts), [top] * 3])


def _basis(n_pts, top, x, deriv=0):
    t = _knots(n_pts, top)
    nb = n_pts + 2
    out = np.zeros(nb)
    for k in range(nb):
        e = np.zeros(nb)
        e[k] = 1.0
        out[k] = BSpline(t, e, 3)(x, nu=deriv)
    return out


def _small_model(n_knots3=5):
    return FD.fit_model(n_knots2=12, n_knots3=n_knots3)


def test_layout_counts_and_roundtrip():
    m = _small_model()
    cols = OF.layout(m)
    assert len(cols) == 11 + 10 * 7
    # a model drawn with the generator's symmetry and vanishing tails is
    # exactly representable by its free parameters
    u = m["uf3"]
    x = np.array([u["c2"][c[1], c[2], c[3]] if c[0] == "2" else u["c3"][c[1], c[2], c[3], c[4]]
                  for c in cols])
    back = OF.params_to_model(m, x)["uf3"]
    assert np.array_equal(back["c2"], u["c2"])
    assert np.array_equal(back["c3"], u["c3"])


def _iso(pos):
    L = np.full(3, 100.0)
    return pos + 30.0, L, np.zeros(3, np.int32)


def test_dimer_rows_are_spline_values():
    m = _small_model()
    r = 2.71
    pos, L, per = _iso(np.array([[0.0, 0.0, 0.0], [r * 0.6, r * 0.8, 0.0]]))
    A = OF.design(m, pos, np.zeros(2, np.int32), L, per)
    B = _basis(12, 5.5, r)
    dB = _basis(12, 5.5, r, 1)
    n2 = 11
    assert np.allclose(A[0, :n2], B[:n2], rtol=0, atol=1e-14)
    assert np.all(A[:, n2:] == 0.0)
    u = np.array([0.6, 0.8, 0.0])
    # F_0 = V'(r) (x1 - x0)/r, F_1 = -F_0; rows 1 + q n + i
    for q in range(3):
        assert np.allclose(A[1 + q * 2 + 0, :n2], dB[:n2] * u[q], atol=1e-13)
        assert np.allclose(A[1 + q * 2 + 1, :n2], -dB[:n2] * u[q], atol=1e-13)


def test_equilateral_trimer_energy_row():
    m = _small_model()
    r = 2.9
    tri = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0], [r / 2, r * np.sqrt(3) / 2, 0.0]])
    pos, L, per = _iso(tri)
    A = OF.design(m, pos, np.zeros(3, np.int32), L, per)
    B2 = _basis(12, 5.5, r)
    Ba = _basis(5, 3.5, r)
    Bc = _basis(5, 7.0, r)
    for k, c in enumerate(OF.layout(m)):
        if c[0] == "2":
            want = 3.0 * B2[c[3]]
        else:
            _, z, p, q, s = c
            want = 3.0 * (2.0 if p < q else 1.0) * Ba[p] * Ba[q] * Bc[s]
        assert abs(A[0, k] - want) < 1e-13, (c, A[0, k], want)
    # no net force on an isolated cluster, column by column
    for q in range(3):
        assert np.abs(A[1 + q * 3: 1 + (q + 1) * 3].sum(0)).max() < 1e-13


def test_force_rows_are_minus_energy_gradient():
    m = _small_model()
    rng = np.random.default_rng(5)
    from gen.lattice import bcc_cubic
    pos0 = bcc_cubic(2, 2, 2)[:13] + rng.normal(0.0, 0.1, (13, 3))
    pos, L, per = _iso(pos0)
    sp = np.zeros(len(pos), np.int32)
    A = OF.design(m, pos, sp, L, per)
    h = 1e-5
    n = len(pos)
    for i, q in ((0, 0), (4, 1), (9, 2), (12, 0)):
        p1 = pos.copy()
        p1[i, q] += h
        p2 = pos.copy()
        p2[i, q] -= h
        g = (OF.design(m, p1, sp, L, per)[0] - OF.design(m, p2, sp, L, per)[0]) / (2 * h)
        scale = np.abs(g).max() + 1e-3
        assert np.abs(-g - A[1 + q * n + i]).max() < 1e-6 * scale, (i, q)


def test_design_times_parameters_is_the_potential():
    m = _small_model()
    snap = FD.thermal_snapshots(1, cells=3, sigma=0.1, seed=9)[0]
    sp = np.zeros(len(snap["pos"]), np.int32)
    A = OF.design(m, snap["pos"], sp, snap["L"], snap["periodic"])
    x = np.random.default_rng(2).normal(size=A.shape[1])
    mm = OF.params_to_model(m, x)
    offs, nbr = O.neighbors(snap["pos"], snap["L"], snap["periodic"], 6.0)
    e, f = O.uf3(mm, snap["pos"], sp, snap["L"], snap["periodic"], offs, nbr)
    pred = A @ x
    assert abs(pred[0] - e.sum()) < 1e-10 * max(1.0, abs(e.sum()))
    assert np.abs(pred[1:] - f.T.reshape(-1)).max() < 1e-10 * max(1.0, np.abs(f).max())


def _lsq_problem(seed, ns=60, nh=10, nd=6):
    r = np.random.default_rng(seed)
    AS = r.normal(size=(ns, nd))
    yS = r.normal(size=ns)
    AH = r.normal(size=(nh, nd))
    yH = r.normal(size=nh)
    w = r.uniform(0.5, 2.0, size=ns)
    return AS, yS, AH, yH, w


def test_fixed_lambda_solve_is_stacked_least_squares():
    AS, yS, AH, yH, w = _lsq_problem(1)
    GS, bS = OF.gram(AS, yS, w)
    GH, bH = OF.gram(AH, yH, np.ones(len(yH)))
    lam, ridge = 37.0, 1e-3
    c = OF.solve_fixed(GS, bS, GH, bH, lam, ridge)
    nd = AS.shape[1]
    M = np.vstack([AS * np.sqrt(w)[:, None], np.sqrt(lam) * AH, np.sqrt(ridge) * np.eye(nd)])
    v = np.concatenate([yS * np.sqrt(w), np.sqrt(lam) * yH, np.zeros(nd)])
    ref = np.linalg.lstsq(M, v, rcond=None)[0]
    assert np.abs(c - ref).max() < 1e-12 * np.abs(ref).max()


def test_constrained_fit_matches_independent_optimiser():
    AS, yS, AH, yH, w = _lsq_problem(3)
    w = np.ones_like(w)
    GS, bS = OF.gram(AS, yS, w)
    c_free = np.linalg.lstsq(AS, yS, rcond=None)[0]
    r_free = OF.hard_residual(AH, yH, c_free)
    r_min = OF.hard_residual(AH, yH, np.linalg.lstsq(AH, yH, rcond=None)[0])
    alpha = r_min + 0.3 * (r_free - r_min)
    c, info = OF.constrained_fit(GS, bS, AH, yH, alpha, lam0=1e-3, tol=alpha * 1e-9)
    assert info["status"] == 0
    assert alpha * (1 - 1e-9) < info["residual"] <= alpha
    # the residual falls as lambda grows
    tr = sorted(info["trace"])
    assert all(b[1] <= a[1] * (1 + 1e-12) for a, b in zip(tr, tr[1:]))

    def soft(x):
        d = AS @ x - yS
        return d @ d
    res = minimize(soft, c_free, jac=lambda x: 2 * AS.T @ (AS @ x - yS), method="SLSQP",
                   constraints=[dict(type="ineq", fun=lambda x: alpha - OF.hard_residual(AH, yH, x),
                                     jac=lambda x: -2 * AH.T @ (AH @ x - yH))],
                   options=dict(ftol=1e-12, maxiter=500))
    assert res.success
    assert abs(soft(c) - res.fun) < 1e-6 * res.fun
    assert np.abs(c - res.x).max() < 1e-6 * np.abs(res.x).max()


def test_constrained_fit_reports_unreachable_alpha():
    # more hard rows than parameters: the hard residual cannot fall below the
    # least-squares residual of the hard rows alone
    AS, yS, AH, yH, w = _lsq_problem(4, nh=20)
    GS, bS = OF.gram(AS, yS, w)
    r_min = OF.hard_residual(AH, yH, np.linalg.lstsq(AH, yH, rcond=None)[0])
    c, info = OF.constrained_fit(GS, bS, AH, yH, 0.5 * r_min, lam0=1.0, max_decades=12)
    assert info["status"] == 1
    assert info["residual"] >= r_min * (1 - 1e-9)
    assert info["residual"] == min(t[1] for t in info["trace"])


@pytest.mark.parametrize("frame", ["cubic", "110", "111"])
def test_strain_cells_are_perfect_bcc(frame):
    pos, L = FD._cell(frame)
    assert len(pos) == {"cubic": 250, "110": 180, "111": 216}[frame]
    assert np.all(L > 13.0)
    offs, nbr = O.neighbors(pos, L, np.ones(3, np.int32), 3.3)
    counts = np.diff(offs)
    assert np.all(counts == 14)   # 8 first + 6 second neighbours of bcc
    offs, _ = O.neighbors(pos, L, np.ones(3, np.int32), 0.9 * A_W)
    assert np.all(np.diff(offs) == 8)


def test_weighted_hard_rows_equal_scaled_rows():
    # weights w on the hard rows are the same problem as rows scaled by sqrt(w)
    AS, yS, AH, yH, w = _lsq_problem(6, nh=12)
    GS, bS = OF.gram(AS, yS, w)
    wH = np.random.default_rng(1).uniform(0.01, 3.0, size=len(yH))
    s = np.sqrt(wH)
    c_free = OF.solve_fixed(GS, bS, 0.0 * GS, 0.0 * bS, 0.0, 0.0)
    r_free = OF.hard_residual(AH, yH, c_free, wH)
    r_min = OF.hard_residual(AH * s[:, None], yH * s,
                             np.linalg.lstsq(AH * s[:, None], yH * s, rcond=None)[0])
    alpha = r_min + 0.3 * (r_free - r_min)
    c1, i1 = OF.constrained_fit(GS, bS, AH, yH, alpha, lam0=1e-2, wH=wH)
    c2, i2 = OF.constrained_fit(GS, bS, AH * s[:, None], yH * s, alpha, lam0=1e-2)
    assert i1["n_solves"] == i2["n_solves"] and i1["status"] == i2["status"] == 0
    assert abs(i1["lam"] - i2["lam"]) <= 1e-12 * i2["lam"]
    assert np.abs(c1 - c2).max() <= 1e-10 * np.abs(c2).max()
