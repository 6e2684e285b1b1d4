"""Pins of the FP64 oracle against facts fixed outside it.

Every check here compares the oracle with something it does not compute
itself: crystallographic shell counts, all-pairs enumeration, hand-derived
region fixtures, library special functions (scipy), closed forms (Racah's
formula for Gaunt coefficients, the spherical-harmonic addition theorem, the
Legendre form of the product basis), finite differences, symmetries and
exact limits of the mixing scheme.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps
from scipy.interpolate import BSpline

import oracle as O
from gen import workloads as W
from gen.lattice import bcc_cubic, A_W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ neighbours

def test_neighbors_cells_equal_all_pairs():
    for w in (W.tiny(), W.c1(), W.tiny(periodic=(1, 0, 1), vacuum=3.0, seed=7)):
        rl = O.r_list(w["model"])
        o1, n1 = O.neighbors(w["pos"], w["L"], w["periodic"], rl, method=0)
        o2, n2 = O.neighbors(w["pos"], w["L"], w["periodic"], rl, method=1)
        assert np.array_equal(o1, o2) and np.array_equal(n1, n2)


@pytest.mark.parametrize("r_list,count", [(2.9, 8), (3.3, 14), (4.6, 26), (5.3, 50),
                                           (5.6, 58), (6.2, 58), (6.4, 64), (6.7, 64)])
def test_bcc_shell_counts(r_list, count):
    # bcc shells: 8 @ a*sqrt3/2, 6 @ a, 12 @ a*sqrt2, 24 @ a*sqrt11/2, 8 @ a*sqrt3, 6 @ 2a
    pos = bcc_cubic(6, 6, 6)
    L = np.array([6 * A_W] * 3)
    offs, nbr = O.neighbors(pos, L, [1, 1, 1], r_list)
    assert np.all(np.diff(offs) == count)


def test_neighbor_rows_symmetric():
    w = W.c1()
    offs, nbr = O.neighbors(w["pos"], w["L"], w["periodic"], 6.0)
    pairs = set()
    for i in range(len(w["pos"])):
        for j in nbr[offs[i]:offs[i + 1]]:
            pairs.add((i, int(j)))
    assert all((j, i) in pairs for (i, j) in pairs)


# ----------------------------------------------------------- regions

def _region_fixture():
    with open(os.path.join(GOLD, "chain_regions.json")) as f:
        g = json.load(f)
    regs = [dict(type=r["type"], axis=r["axis"], follow_atom=r["follow_atom"],
                 center=np.array(r["center"], float), r_core=r["r_core"], r_blend=r["r_blend"])
            for r in g["regions"]]
    return g, regs


def test_chain_fixture_algorithms_1_to_3():
    g, regs = _region_fixture()
    pos = np.array(g["pos"], float)
    lam, flags = O.lambda_flags(pos, g["L"], g["periodic"], regs)
    offs, nbr = O.neighbors(pos, g["L"], g["periodic"], g["r_list"])
    flags = O.buffer_flags(pos, g["L"], g["periodic"], offs, nbr, g["r_buffer"], lam, flags)
    np.testing.assert_allclose(lam, g["lambda"], rtol=0, atol=1e-15)
    assert flags.tolist() == g["flags"]
    assert np.nonzero(flags & 5)[0].tolist() == g["S"]


def _closed_form_lambda(pos, L, per, regs):
    lam = np.zeros(len(pos))
    for r in regs:
        c = pos[r["follow_atom"]] if r["follow_atom"] >= 0 else r["center"]
        d = pos - c
        for k in range(3):
            if per[k]:
                d[:, k] -= L[k] * np.round(d[:, k] / L[k])
        if r["type"] == 1:
            d[:, r["axis"]] = 0
        dist = np.linalg.norm(d, axis=1)
        b = np.clip(1.0 - (dist - r["r_core"]) / r["r_blend"], 0.0, 1.0) if r["r_blend"] > 0 \
            else (dist < r["r_core"]).astype(float)
        lam = np.maximum(lam, b)
    return lam


def test_lambda_closed_form_random_regions():
    rng = np.random.default_rng(3)
    w = W.c2()
    L, per = w["L"], w["periodic"]
    regs = [W.sphere(rng.uniform(0, 50, 3), rng.uniform(2, 8), rng.uniform(0.5, 3)) for _ in range(4)]
    regs += [W.cylinder(rng.uniform(0, 50, 3), 1, 5.0, 2.0), W.sphere([0, 0, 0], 4.0, 0.0),
             W.sphere(None, 3.0, 2.0, follow_atom=17)]
    regs[-1]["center"] = np.zeros(3)
    lam, flags = O.lambda_flags(w["pos"], L, per, regs)
    ref = _closed_form_lambda(w["pos"], L, per, regs)
    np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-13)
    assert np.array_equal((flags & 1) != 0, lam > 0)
    assert np.array_equal((flags & 2) != 0, lam == 1.0)


def test_lambda_set_sizes_on_perfect_lattice():
    # sigma = 0 lattice: |{lambda > 0}| is the number of lattice points strictly
    # inside the outer sphere, |{lambda == 1}| inside the core sphere.
    pos = bcc_cubic(10, 10, 10)
    L = np.array([10 * A_W] * 3)
    c = np.array([5 * A_W + 0.01, 5 * A_W + 0.02, 5 * A_W + 0.03])
    lam, flags = O.lambda_flags(pos, L, [1, 1, 1], [W.sphere(c, 6.0, 2.0)])
    dd = np.linalg.norm(pos - c, axis=1)
    assert int((flags & 1).astype(bool).sum()) == int((dd < 8.0).sum())
    assert int(((flags & 2) != 0).sum()) == int((dd < 6.0).sum())


def test_buffer_brute_force_all_pairs():
    for w in (W.c1(), W.tiny(seed=99)):
        rl = O.r_list(w["model"])
        offs, nbr = O.neighbors(w["pos"], w["L"], w["periodic"], rl)
        lam, flags = O.lambda_flags(w["pos"], w["L"], w["periodic"], w["regions"])
        fb = O.buffer_flags(w["pos"], w["L"], w["periodic"], offs, nbr, w["r_buffer"], lam, flags)
        pos = w["pos"]
        d = pos[:, None, :] - pos[None, :, :]
        for k in range(3):
            if w["periodic"][k]:
                d[..., k] -= w["L"][k] * np.round(d[..., k] / w["L"][k])
        r2 = (d ** 2).sum(-1)
        np.fill_diagonal(r2, np.inf)
        inM = lam > 0
        ref = (~inM) & np.any((r2 < w["r_buffer"] ** 2) & inM[None, :], axis=1)
        assert np.array_equal((fb & 4) != 0, ref)
        assert not np.any(((fb & 4) != 0) & inM)


def _blend_ref(t, cubic):
    return 1.0 - 3.0 * t ** 2 + 2.0 * t ** 3 if cubic else 1.0 - t


def _seeded_brute(pos, L, per, seeds, regs, lam0):
    """The paper's Algorithms 1-2 for seeded regions over all pairs (no
    neighbour list), pure Python loops over the scatter loops as printed."""
    n = len(pos)
    d = pos[None, :, :] - pos[:, None, :]
    for k in range(3):
        if per[k]:
            d[..., k] -= L[k] * np.round(d[..., k] / L[k])
    r2 = (d ** 2).sum(-1)
    lam = lam0.copy()
    for r in regs:
        if r["type"] != 2:
            continue
        core = np.asarray(seeds, bool).copy()
        for i in range(n):
            if seeds[i]:
                for j in range(n):
                    if j != i and r2[i, j] < r["r_core"] ** 2:
                        core[j] = True
        lam[core] = 1.0
        for i in range(n):
            if core[i]:
                for j in range(n):
                    if j != i and r2[i, j] < r["r_blend"] ** 2:
                        lam[j] = max(lam[j], _blend_ref(math.sqrt(r2[i, j]) / r["r_blend"],
                                                        r.get("blend", 0)))
    return lam


def test_seeded_chain_closed_form():
    # atoms on a line 2 A apart, seed = atom 2; r_core 2.5 makes atoms 1-3
    # core; blend radius 5 measured to the nearest core atom: atoms 0 and 4
    # are 2 A from the core (t = 0.4), atom 5 is 4 A away (t = 0.8), atom 6
    # (6 A) gets nothing; buffer 3 A then takes atom 6 (2 A from atom 5)
    n = 9
    pos = np.zeros((n, 3))
    pos[:, 0] = 1.0 + 2.0 * np.arange(n)
    pos[:, 1:] = 5.0
    L, per = np.array([40.0, 10.0, 10.0]), [0, 0, 0]
    seeds = np.zeros(n, bool)
    seeds[2] = True
    offs, nbr = O.neighbors(pos, L, per, 7.0)
    for cubic in (0, 1):
        regs = [W.seeded(2.5, 5.0, blend=cubic)]
        lam, flags = O.lambda_flags(pos, L, per, regs)
        assert not lam.any()
        lam, flags = O.lambda_seeded(pos, L, per, offs, nbr, seeds, regs, lam)
        b4, b8 = _blend_ref(0.4, cubic), _blend_ref(0.8, cubic)
        np.testing.assert_allclose(lam, [b4, 1, 1, 1, b4, b8, 0, 0, 0], rtol=0, atol=1e-15)
        flags = O.buffer_flags(pos, L, per, offs, nbr, 3.0, lam, flags)
        assert flags.tolist() == [1, 3, 3, 3, 1, 1, 4, 0, 0]
    # the cubic values themselves: 1 - 3 t^2 + 2 t^3 at t = 0.4 and 0.8
    assert abs(_blend_ref(0.4, 1) - 0.648) < 1e-15 and abs(_blend_ref(0.8, 1) - 0.104) < 1e-15


def test_seeded_brute_force_random_cluster():
    rng = np.random.default_rng(11)
    n = 70
    L, per = np.array([11.0, 11.0, 11.0]), [1, 1, 0]
    pos = rng.uniform(0.0, 11.0, size=(n, 3))
    seeds = np.zeros(n, bool)
    seeds[rng.choice(n, 3, replace=False)] = True
    regs = [W.seeded(2.2, 3.0), W.seeded(1.5, 2.5, blend=1), W.sphere([2.0, 3.0, 4.0], 1.0, 1.5, blend=1)]
    offs, nbr = O.neighbors(pos, L, per, 4.0)
    lam0, _ = O.lambda_flags(pos, L, per, regs)
    lam, flags = O.lambda_seeded(pos, L, per, offs, nbr, seeds, regs, lam0)
    ref = _seeded_brute(pos, L, per, seeds, regs, lam0)
    np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-14)
    assert np.array_equal((flags & 1) != 0, lam > 0)
    assert np.array_equal((flags & 2) != 0, lam == 1.0)
    assert (lam[seeds] == 1.0).all()


def test_cubic_geometric_blend_closed_form():
    # atoms on a ray from a sphere's centre at known distances
    ds = np.array([0.5, 2.0, 2.6, 3.2, 3.8, 4.4, 5.0, 6.0])
    pos = np.zeros((len(ds), 3)) + 10.0
    pos[:, 0] += ds
    c = np.array([10.0, 10.0, 10.0])
    lam, _ = O.lambda_flags(pos, [30.0] * 3, [0, 0, 0], [W.sphere(c, 2.0, 3.0, blend=1)])
    t = np.clip((ds - 2.0) / 3.0, 0.0, 1.0)
    ref = np.where(ds < 2.0, 1.0, np.where(ds < 5.0, 1.0 - 3.0 * t ** 2 + 2.0 * t ** 3, 0.0))
    np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-14)


# ------------------------------------------------------ special functions

def test_radial_is_chebyshev_times_envelope():
    rc = 5.0
    for r in np.linspace(0.3, 4.99, 23):
        R, dR = O.radial(10, rc, r)
        x = 2 * r / rc - 1
        env = (1 - (r / rc) ** 2) ** 2
        ref = np.cos(np.arange(10) * np.arccos(x)) * env
        np.testing.assert_allclose(R, ref, atol=1e-13)
        h = 1e-6
        Rp, _ = O.radial(10, rc, r + h)
        Rm, _ = O.radial(10, rc, r - h)
        np.testing.assert_allclose(dR, (Rp - Rm) / (2 * h), atol=1e-7)


def _scipy_real_ylm(lmax, u):
    th = math.acos(max(-1.0, min(1.0, u[2])))
    ph = math.atan2(u[1], u[0])
    out = np.zeros((lmax + 1) ** 2)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            mu = abs(m)
            Yp = complex(sps.sph_harm_y(l, mu, th, ph))   # Condon-Shortley phase included
            Ym = complex(sps.sph_harm_y(l, -mu, th, ph))
            if m > 0:
                v = ((-1) ** mu * Yp + Ym) / math.sqrt(2)
            elif m < 0:
                v = ((-1) ** mu * Yp - Ym) / (1j * math.sqrt(2))
            else:
                v = Yp
            assert abs(v.imag) < 1e-12
            out[l * l + l + m] = v.real
    return out


def test_ylm_matches_scipy_and_gradient():
    rng = np.random.default_rng(1)
    for _ in range(20):
        v = rng.normal(size=3)
        u = v / np.linalg.norm(v)
        Y, g = O.ylm(5, u)
        np.testing.assert_allclose(Y, _scipy_real_ylm(5, u), atol=1e-12)
        # gradient of Y(r/|r|) with respect to r, projected as the oracle does
        r = np.linalg.norm(v)
        G = (g - np.outer((g @ u), u)) / r
        h = 1e-6
        for k in range(3):
            vp = v.copy(); vp[k] += h
            vm = v.copy(); vm[k] -= h
            fd = (O.ylm(5, vp / np.linalg.norm(vp))[0] - O.ylm(5, vm / np.linalg.norm(vm))[0]) / (2 * h)
            np.testing.assert_allclose(G[:, k], fd, atol=1e-7)


def test_ylm_addition_theorem_and_orthonormality():
    rng = np.random.default_rng(2)
    for _ in range(10):
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        Y, _ = O.ylm(6, u)
        for l in range(7):
            s = (Y[l * l:(l + 1) ** 2] ** 2).sum()
            assert abs(s - (2 * l + 1) / (4 * math.pi)) < 1e-13
    # orthonormality with an independent quadrature (Gauss-Legendre x uniform)
    x, wx = np.polynomial.legendre.leggauss(12)
    nph = 24
    M = np.zeros((36, 36))
    for zi, wi in zip(x, wx):
        for k in range(nph):
            ph = 2 * math.pi * k / nph
            st = math.sqrt(1 - zi * zi)
            Y, _ = O.ylm(5, np.array([st * math.cos(ph), st * math.sin(ph), zi]))
            M += wi * (2 * math.pi / nph) * np.outer(Y, Y)
    np.testing.assert_allclose(M, np.eye(36), atol=1e-13)


def _w3j(j1, j2, j3, m1, m2, m3):
    """Wigner 3j symbol from Racah's closed form."""
    if m1 + m2 + m3 != 0 or j3 > j1 + j2 or j3 < abs(j1 - j2):
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    f = math.factorial
    tri = f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3) / f(j1 + j2 + j3 + 1)
    pre = math.sqrt(tri * f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2) * f(j3 + m3) * f(j3 - m3))
    s = 0.0
    for k in range(0, j1 + j2 + j3 + 1):
        a = [k, j3 - j2 + k + m1, j3 - j1 + k - m2, j1 + j2 - j3 - k, j1 - k - m1, j2 - k + m2]
        if min(a) < 0:
            continue
        s += (-1) ** k / (f(a[0]) * f(a[1]) * f(a[2]) * f(a[3]) * f(a[4]) * f(a[5]))
    return (-1) ** (j1 - j2 - m3) * pre * s


def _U(l):
    """Real (no Condon-Shortley) from complex (with it) harmonics: Y^R = U Y^C."""
    U = np.zeros((2 * l + 1, 2 * l + 1), dtype=complex)
    for m in range(-l, l + 1):
        i = m + l
        mu = abs(m)
        if m > 0:
            U[i, mu + l] = (-1) ** mu / math.sqrt(2)
            U[i, -mu + l] = 1 / math.sqrt(2)
        elif m < 0:
            U[i, mu + l] = (-1) ** mu / (1j * math.sqrt(2))
            U[i, -mu + l] = -1 / (1j * math.sqrt(2))
        else:
            U[i, l] = 1.0
    return U


def _racah_real_gaunt(l1, l2, l3):
    """Real Gaunt block (l1, l2, l3) from Wigner 3j symbols and the complex ->
    real change of basis."""
    Gc = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1))
    pre = math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4 * math.pi)) \
        * _w3j(l1, l2, l3, 0, 0, 0)
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            for m3 in range(-l3, l3 + 1):
                Gc[m1 + l1, m2 + l2, m3 + l3] = pre * _w3j(l1, l2, l3, m1, m2, m3)
    Gr = np.einsum("ai,bj,ck,ijk->abc", _U(l1), _U(l2), _U(l3), Gc)
    assert np.abs(Gr.imag).max() < 1e-13
    return Gr.real


# every l-triple up to lmax 6, the largest degree the library accepts (the
# 1,023,800-atom workload runs lmax 5): a quadrature one order too short
# fails here at the top degrees first
def test_gaunt_matches_racah_closed_form():
    lmax = 6
    G = O.gaunt_table(lmax)
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for l3 in range(lmax + 1):
                Gr = _racah_real_gaunt(l1, l2, l3)
                sub = G[l1 * l1:(l1 + 1) ** 2, l2 * l2:(l2 + 1) ** 2, l3 * l3:(l3 + 1) ** 2]
                np.testing.assert_allclose(sub, Gr, atol=1e-13)


# ----------------------------------------------------- ACE-style potential

def _env(w, i, in_S=None):
    """Displacements from atom i to its S-neighbours within the expensive cutoff."""
    m = w["model"]
    rc = m["ace"]["rcut"]
    pos = w["pos"]
    d = pos - pos[i]
    for k in range(3):
        if w["periodic"][k]:
            d[:, k] -= w["L"][k] * np.round(d[:, k] / w["L"][k])
    r = np.linalg.norm(d, axis=1)
    sel = (r < rc) & (np.arange(len(pos)) != i)
    if in_S is not None:
        sel &= in_S
    return d[sel], r[sel], w["species"][sel]


def _np_radial(n_rad, rc, r):
    x = 2 * r / rc - 1
    T = np.polynomial.chebyshev.chebvander(x, n_rad - 1)
    return T * ((1 - (r / rc) ** 2) ** 2)[:, None]


def _model_with_orders(w, keep):
    import copy
    w2 = dict(w)
    m = copy.deepcopy(w["model"])
    a = m["ace"]
    if 1 not in keep:
        a["c1"] = a["c1"] * 0
    if 2 not in keep:
        a["c2"] = a["c2"] * 0
    if 3 not in keep:
        a["c3"] = a["c3"] * 0
    w2["model"] = m
    return w2


def test_order1_is_pair_potential():
    w = _model_with_orders(W.tiny(n_species=2, seed=5), {1})
    out = O.mixed(w, O.MODE_ALL_EXPENSIVE)
    a = w["model"]["ace"]
    for i in range(0, len(w["pos"]), 7):
        d, r, z = _env(w, i)
        R = _np_radial(a["n_rad"], a["rcut"], r)
        E = a["c0"][w["species"][i]]
        for j in range(len(r)):
            E += (a["c1"][w["species"][i], z[j] * a["n_rad"]:(z[j] + 1) * a["n_rad"]] * R[j]).sum() \
                / math.sqrt(4 * math.pi)
        assert abs(E - out["e_exp"][i]) < 1e-12


def test_order2_legendre_closed_form():
    # sum_m A_alm A_blm = (2l+1)/(4 pi) sum_{j,k} R_a(r_ij) R_b(r_ik) P_l(cos theta_jik)
    w = _model_with_orders(W.tiny(n_species=2, seed=6), {2})
    out = O.mixed(w, O.MODE_ALL_EXPENSIVE)
    a = w["model"]["ace"]
    nr, lmax = a["n_rad"], a["lmax"]
    nchan = w["model"]["n_species"] * nr
    for i in range(0, len(w["pos"]), 5):
        d, r, z = _env(w, i)
        u = d / r[:, None]
        R = _np_radial(nr, a["rcut"], r)
        phi = np.zeros((len(r), nchan))
        for j in range(len(r)):
            phi[j, z[j] * nr:(z[j] + 1) * nr] = R[j]
        cos = np.clip(u @ u.T, -1, 1)
        E = a["c0"][w["species"][i]]
        for l in range(lmax + 1):
            P = sps.eval_legendre(l, cos) * (2 * l + 1) / (4 * math.pi)
            Bab = phi.T @ P @ phi
            for aa in range(nchan):
                for bb in range(aa, nchan):
                    E += a["c2"][w["species"][i], l, aa, bb] * Bab[aa, bb]
        assert abs(E - out["e_exp"][i]) < 1e-11 * max(1.0, abs(E))


def _order3_sphere_integral(w, stride):
    # sum_m G Y Y Y over three atomic bases equals the sphere integral of the
    # product of three Legendre-weighted densities:
    # B = int dO prod_k [ (2l_k+1)/(4pi) sum_j R_{a_k}(r_j) P_{l_k}(u_j . O) ],
    # with a = (species of j, n): no harmonics and no Gaunt table involved.
    out = O.mixed(w, O.MODE_ALL_EXPENSIVE)
    a = w["model"]["ace"]
    ns = w["model"]["n_species"]
    nr, lmax = a["n_rad"], a["lmax"]
    L1 = lmax + 1
    K = ns * nr * L1
    x, wx = np.polynomial.legendre.leggauss(2 * lmax + 4)
    nph = 4 * lmax + 6
    dirs, wts = [], []
    for zi, wi in zip(x, wx):
        for k in range(nph):
            ph = 2 * math.pi * k / nph
            st = math.sqrt(1 - zi * zi)
            dirs.append([st * math.cos(ph), st * math.sin(ph), zi])
            wts.append(wi * 2 * math.pi / nph)
    dirs = np.array(dirs)
    wts = np.array(wts)
    checked = 0
    for i in range(0, len(w["pos"]), stride):
        d, r, z = _env(w, i)
        u = d / r[:, None]
        R = _np_radial(nr, a["rcut"], r)
        cos = u @ dirs.T
        P = [(2 * l + 1) / (4 * math.pi) * sps.eval_legendre(l, cos) for l in range(L1)]
        rho = np.zeros((K, len(dirs)))
        for zz in range(ns):
            sel = z == zz
            for n in range(nr):
                ch = zz * nr + n
                for l in range(L1):
                    rho[ch * L1 + l] = (R[sel, n][:, None] * P[l][sel]).sum(0)
        zi = w["species"][i]
        E = a["c0"][zi]
        for p in range(K):
            for q in range(p, K):
                rpq = wts * rho[p] * rho[q]
                for s in range(q, K):
                    l1, l2, l3 = p % L1, q % L1, s % L1
                    if (l1 + l2 + l3) % 2 or l3 > l1 + l2 or l3 < abs(l1 - l2):
                        continue
                    E += a["c3"][zi, p, q, s] * (rpq * rho[s]).sum()
        assert abs(E - out["e_exp"][i]) < 1e-11 * max(1.0, abs(E)), (i, E, out["e_exp"][i])
        checked += 1
    assert checked > 0


def test_order3_sphere_integral_form():
    _order3_sphere_integral(_model_with_orders(W.tiny(seed=8, lmax=2, n_rad=3), {3}), 9)


# the degree of the 1,023,800-atom workload (lmax 5) with two species, so that
# channel offsets by neighbour species and the top l-triples are both covered
def test_order3_sphere_integral_form_lmax5_two_species():
    w = _model_with_orders(W.tiny(seed=18, n_species=2, lmax=5, n_rad=2), {3})
    assert len(set(w["species"].tolist())) == 2
    _order3_sphere_integral(w, 13)


def _fd_forces(w, which, idx, h=1e-5, in_S=None):
    m = w["model"]
    rl = O.r_list(m)
    res = []
    for i in idx:
        row = []
        for k in range(3):
            Es = []
            for sgn in (1, -1):
                p = w["pos"].copy()
                p[i, k] += sgn * h
                offs, nbr = O.neighbors(p, w["L"], w["periodic"], rl)
                if which == "exp":
                    e, _ = O.ace(m, p, w["species"], w["L"], w["periodic"], offs, nbr, in_S=in_S)
                    if in_S is not None:
                        e = e[in_S]
                else:
                    e, _ = O.uf3(m, p, w["species"], w["L"], w["periodic"], offs, nbr, in_S=in_S)
                    if in_S is not None:
                        e = e[in_S]
                Es.append(e.sum())
            row.append(-(Es[0] - Es[1]) / (2 * h))
        res.append(row)
    return np.array(res)


@pytest.mark.parametrize("which", ["exp", "cheap"])
def test_forces_are_minus_gradient(which):
    w = W.tiny(n_species=2, seed=11)
    out = O.mixed(w, O.MODE_ALL_EXPENSIVE if which == "exp" else O.MODE_ALL_CHEAP)
    F = out["f_exp"] if which == "exp" else out["f_cheap"]
    idx = [0, 3, 20, 41]
    fd = _fd_forces(w, which, idx)
    scale = np.abs(F).max()
    np.testing.assert_allclose(F[idx], fd, atol=2e-8 * max(scale, 1.0))


def _masked_cheap_case():
    # 6^3 cells, a 3.5 A core (15 atoms) and a 3 A buffer: the first and
    # second shells of the core join the cheap buffer, the central atom lies
    # deeper and leaves the cheap subsystem
    w = W.tiny(seed=17, cells=6)
    w["regions"] = [W.sphere(w["L"] / 2.0, 3.5, 1.5)]
    w["r_buffer"] = 3.0
    return w


def test_cheap_buffer_brute_force_and_subset():
    # the cheap potential's buffer: lambda == 1 atoms strictly within r_buffer
    # of a lambda < 1 atom (all pairs); its subsystem is a proper subset here
    w = _masked_cheap_case()
    out = O.mixed(w, cheap_masked=True)
    lam, fl = out["lam"], out["flags"]
    pos = w["pos"]
    d = pos[:, None, :] - pos[None, :, :]
    for k in range(3):
        if w["periodic"][k]:
            d[..., k] -= w["L"][k] * np.round(d[..., k] / w["L"][k])
    r2 = (d ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    core = lam == 1.0
    ref = core & np.any((r2 < w["r_buffer"] ** 2) & ~core[None, :], axis=1)
    assert np.array_equal((fl & 8) != 0, ref)
    assert ref.any()
    in_Sc = ~core | ref
    assert 0 < in_Sc.sum() < len(pos)
    assert np.all(out["e_cheap"][~in_Sc] == 0.0) and np.all(out["f_cheap"][~in_Sc] == 0.0)


def test_masked_cheap_forces_gradient_and_locality():
    # Algorithm 4 for the cheap potential: with S_c frozen, F_cheap on S_c is
    # -grad of sum_{i in S_c} E_i^{S_c}; an atom whose 2 rc ball lies inside
    # S_c gets exactly the unmasked cheap force; no core at all = unmasked
    w = _masked_cheap_case()
    out = O.mixed(w, cheap_masked=True)
    in_Sc = (out["lam"] < 1.0) | ((out["flags"] & 8) != 0)
    idx = list(np.nonzero(in_Sc)[0][[0, 7, -1]])
    fd = _fd_forces(w, "cheap", idx, in_S=in_Sc)
    np.testing.assert_allclose(out["f_cheap"][idx], fd,
                               atol=2e-8 * max(np.abs(out["f_cheap"]).max(), 1.0))
    full = O.mixed(w)
    pos = w["pos"]
    rc = w["model"]["uf3"]["rcut2"]
    out_idx = np.nonzero(~in_Sc)[0]
    far = []
    for i in range(len(pos)):
        d = pos[out_idx] - pos[i]
        for k in range(3):
            if w["periodic"][k]:
                d[:, k] -= w["L"][k] * np.round(d[:, k] / w["L"][k])
        if len(out_idx) == 0 or np.linalg.norm(d, axis=1).min() >= 2.0 * rc:
            far.append(i)
    assert len(far) > 0
    assert np.array_equal(out["f_cheap"][far], full["f_cheap"][far])
    w0 = W.tiny(seed=17)
    w0["regions"] = [W.sphere(w0["L"] / 2.0, 0.0, 3.0)]  # blend only: lambda < 1 everywhere
    a, b = O.mixed(w0, cheap_masked=True), O.mixed(w0)
    assert np.array_equal(a["forces"], b["forces"]) and np.array_equal(a["e_cheap"], b["e_cheap"])


def test_subsystem_forces_are_gradient_of_subsystem_energy():
    # Algorithm 4 / Fig. 10: with S frozen, F_exp on S is -grad of sum_{i in S} E_i^S.
    w = W.tiny(seed=13)
    out = O.mixed(w)
    in_S = (out["flags"] & 5) != 0
    S = np.nonzero(in_S)[0]
    idx = list(S[[0, len(S) // 2, -1]])
    fd = _fd_forces(w, "exp", idx, in_S=in_S)
    np.testing.assert_allclose(out["f_exp"][idx], fd, atol=1e-7)
    assert np.all(out["f_exp"][~in_S] == 0)


def test_zero_net_force_and_translation():
    w = W.tiny(n_species=2, seed=17)
    for mode, key in ((O.MODE_ALL_EXPENSIVE, "f_exp"), (O.MODE_ALL_CHEAP, "f_cheap")):
        out = O.mixed(w, mode)
        assert np.abs(out[key].sum(0)).max() < 1e-11
        shift = np.array([0.37, -1.21, 2.05])
        w2 = dict(w)
        w2["pos"] = w["pos"] + shift
        for k in range(3):
            w2["pos"][:, k] %= w["L"][k]
        w2["regions"] = [dict(r, center=r["center"] + shift) for r in w["regions"]]
        out2 = O.mixed(w2, mode)
        np.testing.assert_allclose(out2[key], out[key], atol=1e-11)
    out = O.mixed(w)
    assert np.abs(out["f_exp"].sum(0)).max() < 1e-11   # subsystem net force


def test_rotation_and_permutation_of_cluster():
    w = W.tiny(n_species=2, seed=19, periodic=(0, 0, 0), vacuum=30.0)
    out = O.mixed(w, O.MODE_ALL_EXPENSIVE)
    outc = O.mixed(w, O.MODE_ALL_CHEAP)
    rng = np.random.default_rng(0)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    c = w["L"] / 2
    w2 = dict(w)
    w2["pos"] = (w["pos"] - c) @ q.T + c
    o2 = O.mixed(w2, O.MODE_ALL_EXPENSIVE)
    np.testing.assert_allclose(o2["e_exp"], out["e_exp"], atol=1e-11)
    np.testing.assert_allclose(o2["f_exp"], out["f_exp"] @ q.T, atol=1e-11)
    o2c = O.mixed(w2, O.MODE_ALL_CHEAP)
    np.testing.assert_allclose(o2c["e_cheap"], outc["e_cheap"], atol=1e-11)
    np.testing.assert_allclose(o2c["f_cheap"], outc["f_cheap"] @ q.T, atol=1e-11)
    perm = rng.permutation(len(w["pos"]))
    w3 = dict(w)
    w3["pos"] = w["pos"][perm]
    w3["species"] = w["species"][perm]
    o3 = O.mixed(w3, O.MODE_ALL_EXPENSIVE)
    np.testing.assert_allclose(o3["f_exp"], out["f_exp"][perm], atol=1e-11)


def test_mixing_limits_and_locality():
    w = W.c1()
    all_e = O.mixed(w, O.MODE_ALL_EXPENSIVE)
    all_c = O.mixed(w, O.MODE_ALL_CHEAP)
    # lambda == 1 everywhere: F = F_exp of the whole system, exactly
    w1 = dict(w, regions=[W.sphere(w["L"] / 2, 100.0, 1.0)])
    o1 = O.mixed(w1)
    assert np.all(o1["lam"] == 1.0)
    assert np.array_equal(o1["forces"], all_e["f_exp"])
    # lambda == 0 everywhere: F = F_cheap, exactly
    w0 = dict(w, regions=[W.sphere(w["L"] / 2, 0.1, 0.1)])
    o0 = O.mixed(w0)
    assert len(o0["S"]) == 0
    assert np.array_equal(o0["forces"], all_c["f_cheap"])
    # locality (buffer equation and the receptive-field remark): atoms with
    # lambda = 1 whose 2 r_c ball lies in S get the all-expensive force, and
    # atoms with lambda = 0 get exactly the cheap force.
    w5 = W.c2()
    o = O.mixed(w5)
    rc = w5["model"]["ace"]["rcut"]
    in_S = (o["flags"] & 5) != 0
    e_all = O.mixed(w5, O.MODE_ALL_EXPENSIVE, target=(o["lam"] == 1.0).astype(np.uint8))
    pos = w5["pos"]
    checked = 0
    for i in np.nonzero(o["lam"] == 1.0)[0]:
        d = pos - pos[i]
        d -= w5["L"] * np.round(d / w5["L"])
        ball = np.linalg.norm(d, axis=1) < 2 * rc
        if np.all(in_S[ball]):
            np.testing.assert_allclose(o["forces"][i], e_all["f_exp"][i], atol=1e-11)
            checked += 1
    assert checked > 10
    zero = o["lam"] == 0
    assert np.array_equal(o["forces"][zero], o["f_cheap"][zero])


# --------------------------------------------------------- UF3-style cheap

def test_bspline_matches_scipy_and_partition_of_unity():
    for n_pts, top in ((12, 5.0), (6, 3.5), (6, 7.0), (16, 5.5)):
        t = O.clamped_knots(n_pts, top)
        assert t[0] == t[3] == 0.0 and t[-1] == t[-4] == top
        nb = len(t) - 4
        for x in np.linspace(0.0, top * 0.9999, 37):
            B, dB = O.bspline(t, x)
            assert abs(B.sum() - 1.0) < 1e-14
            for k in range(nb):
                c = np.zeros(nb); c[k] = 1.0
                s = BSpline(t, c, 3, extrapolate=False)
                assert abs(s(x) - B[k]) < 1e-13
                assert abs(s.derivative()(x) - dB[k]) < 1e-11


def test_uf3_tensor_of_ones_counts_pairs_and_triplets():
    w = W.tiny(seed=23)
    import copy
    m = copy.deepcopy(w["model"])
    u = m["uf3"]
    u["c2"] = np.ones_like(u["c2"])
    u["c3"] = np.zeros_like(u["c3"])
    w2 = dict(w, model=m)
    rl = O.r_list(m)
    offs, nbr = O.neighbors(w["pos"], w["L"], w["periodic"], rl)
    e, _ = O.uf3(m, w["pos"], w["species"], w["L"], w["periodic"], offs, nbr)
    d, r = [], []
    for i in range(len(w["pos"])):
        _, ri, _ = _env(dict(w2, model=dict(m, ace=dict(m["ace"], rcut=u["rcut2"]))), i)
        assert abs(e[i] - 0.5 * len(ri)) < 1e-12
    u["c2"] = np.zeros_like(u["c2"])
    u["c3"] = np.ones_like(u["c3"])
    e, _ = O.uf3(m, w["pos"], w["species"], w["L"], w["periodic"], offs, nbr)
    for i in range(len(w["pos"])):
        _, ri, _ = _env(dict(w2, model=dict(m, ace=dict(m["ace"], rcut=u["rcut3"]))), i)
        k = len(ri)
        assert abs(e[i] - k * (k - 1) / 2) < 1e-11


# ---------------------------------------------------------- velocity Verlet

def test_vv_time_reversal_and_dt_squared_drift():
    w = W.tiny(seed=29, sigma=0.05)
    v0 = w["vel"] * 3.0
    p1, v1, _ = O.velocity_verlet(w, w["pos"], v0, 1.0, 20, mode=O.MODE_ALL_CHEAP)
    p2, v2, _ = O.velocity_verlet(w, p1, -v1, 1.0, 20, mode=O.MODE_ALL_CHEAP)
    d = p2 - w["pos"]
    d -= w["L"] * np.round(d / w["L"])
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + v0).max() < 1e-10

    def drift(dt, nsteps):
        es = []

        def cb(step, pos, vel, out):
            es.append(out["e_cheap"].sum() + O.kinetic(w, vel))
        out0 = O.mixed(w, O.MODE_ALL_CHEAP)
        e0 = out0["e_cheap"].sum() + O.kinetic(w, v0)
        O.velocity_verlet(w, w["pos"], v0, dt, nsteps, mode=O.MODE_ALL_CHEAP, callback=cb)
        return max(abs(e - e0) for e in es)
    d1 = drift(4.0, 10)
    d2 = drift(2.0, 20)
    assert 2.5 < d1 / d2 < 6.0   # energy error scales as dt^2 (ratio 4)


# ---------------------------------------------------------- Langevin thermostat

def _free_gas(seed=41, n_side=4, spacing=16.0):
    """W and He atoms on a simple cubic lattice whose spacing is several
    cutoffs: no potential acts, so only the thermostat changes velocities."""
    w = W.tiny(seed=seed, n_species=2)
    g = (np.arange(n_side) + 0.5) * spacing
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    n = len(pos)
    species = (np.arange(n) % 2).astype(np.int32)
    vel = W.maxwell(np.random.default_rng(seed), species, 300.0)
    return dict(w, pos=pos, L=np.full(3, n_side * spacing), species=species, vel=vel)


def test_langevin_friction_closed_form():
    # T = 0: a free atom's velocity decays geometrically. The opening kick of
    # step k carries the friction of step k-1, so the half-step velocity is
    # v0 (1 - dt/tau)^(k-1) and the closing kick takes another dt/(2 tau).
    w = _free_gas()
    dt, tau, k = 0.5, 7.0, 12
    xi = np.zeros((k, len(w["pos"]), 3))
    p, v, out = O.velocity_verlet(w, w["pos"], w["vel"], dt, k, mode=O.MODE_ALL_CHEAP,
                                  langevin=(0.0, tau, xi))
    assert np.all(out["lam"] == 0.0) and np.abs(out["e_cheap"]).max() == 0.0
    a = 1.0 - dt / tau
    half = [w["vel"] * a ** j for j in range(k)]
    assert np.allclose(v, half[-1] * (1.0 - 0.5 * dt / tau), rtol=1e-13, atol=0.0)
    x = w["pos"] + dt * np.sum(half, axis=0)
    d = p - x
    d -= w["L"] * np.round(d / w["L"])
    assert np.abs(d).max() < 1e-12


def test_langevin_equipartition_and_mass_scaling():
    # With no potential the scheme is a linear recurrence whose stationary
    # full-step velocity variance is exactly kB T / m (times kappa): for
    # h = dt/(2 tau) the half-step variance is s2/(1-h), s2 = kappa kB T/m, and
    # the closing kick maps it to s2 (1-h) + s2 h. Both species (masses 184
    # and 4) must sit at the bath temperature, started from 300 K.
    w = _free_gas(seed=43)
    dt, tau, T, k, burn = 1.0, 10.0, 900.0, 2400, 100
    n = len(w["pos"])
    xi = np.random.default_rng(7).normal(size=(k, n, 3))
    m = w["masses"][w["species"]]
    acc = np.zeros(n)
    cnt = [0]

    def cb(step, pos, vel, out):
        if step >= burn:
            acc[:] += (vel ** 2).sum(1)
            cnt[0] += 1
    O.velocity_verlet(w, w["pos"], w["vel"], dt, k, mode=O.MODE_ALL_CHEAP,
                      langevin=(T, tau, xi), callback=cb)
    t_est = acc / cnt[0] * m / (3.0 * W.KAPPA * W.KB)
    for s in (0, 1):
        ratio = t_est[w["species"] == s].mean() / T
        assert abs(ratio - 1.0) < 0.05, (s, ratio)


def test_langevin_acts_only_where_lambda_is_zero():
    # one mixed step: the opening kick and the drift use the initial forces,
    # so positions match NVE everywhere, velocities match bit for bit where
    # lambda > 0 at the force call, and differ on every lambda == 0 atom
    w = W.tiny(seed=47, n_species=2, sigma=0.05)
    n = len(w["pos"])
    xi = np.random.default_rng(3).normal(size=(1, n, 3))
    p0, v0, out0 = O.velocity_verlet(w, w["pos"], w["vel"], 1.0, 1)
    p1, v1, out1 = O.velocity_verlet(w, w["pos"], w["vel"], 1.0, 1,
                                     langevin=(300.0, 50.0, xi))
    assert np.array_equal(p0, p1)
    cheap = out0["lam"] == 0.0
    assert 0 < cheap.sum() < n
    assert np.array_equal(v0[~cheap], v1[~cheap])
    assert np.all(np.abs(v0[cheap] - v1[cheap]).max(1) > 0.0)
