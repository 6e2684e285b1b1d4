"""Python face of the FP64 CPU oracle (mlmix_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg. The product package never imports it.

Every function takes numpy arrays in natural (N, 3) row-major layout and the
workload dictionaries of gen.workloads, and returns numpy arrays.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmlmix_oracle.so")
_lib = None

MODE_MIXED, MODE_ALL_EXPENSIVE, MODE_ALL_CHEAP = 0, 1, 2


class _Ace(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_rad", ctypes.c_int32),
                ("lmax", ctypes.c_int32), ("order", ctypes.c_int32),
                ("rcut", ctypes.c_double),
                ("c0", ctypes.c_void_p), ("c1", ctypes.c_void_p),
                ("c2", ctypes.c_void_p), ("c3", ctypes.c_void_p)]


class _Uf3(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_knots2", ctypes.c_int32),
                ("n_knots3", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("rcut2", ctypes.c_double), ("rcut3", ctypes.c_double),
                ("c2", ctypes.c_void_p), ("c3", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.or_ace_site.restype = ctypes.c_double
        _lib.or_sum.restype = ctypes.c_double
        _lib.or_num_threads.restype = ctypes.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads():
    return int(lib().or_num_threads())


def set_threads(n):
    lib().or_set_threads(ctypes.c_int(int(n)))


# ---------------------------------------------------------------- geometry

def neighbors(pos, L, periodic, r_list, method=1):
    """CSR neighbour set {j != i : |d_ij|^2 < r_list^2}, rows ascending."""
    pos = _f64(pos)
    n = len(pos)
    L = _f64(L)
    per = _i32(periodic)
    offs = np.zeros(n + 1, dtype=np.int64)
    rc = lib().or_neighbors(ctypes.c_int(n), _p(pos), _p(L), _p(per), ctypes.c_double(r_list),
                            ctypes.c_int(method), _p(offs), None)
    assert rc == 0
    nbr = np.zeros(max(int(offs[-1]), 1), dtype=np.int32)
    rc = lib().or_neighbors(ctypes.c_int(n), _p(pos), _p(L), _p(per), ctypes.c_double(r_list),
                            ctypes.c_int(method), _p(offs), _p(nbr))
    assert rc == 0
    return offs, nbr[: offs[-1]]


def _regions_arrays(regions):
    k = len(regions)
    typ = np.array([r["type"] for r in regions], dtype=np.int32).reshape(k)
    ax = np.array([r.get("axis", 2) for r in regions], dtype=np.int32).reshape(k)
    fol = np.array([r.get("follow_atom", -1) for r in regions], dtype=np.int32).reshape(k)
    cen = np.array([r.get("center", np.zeros(3)) for r in regions], dtype=np.float64).reshape(k, 3)
    rc = np.array([r["r_core"] for r in regions], dtype=np.float64).reshape(k)
    rb = np.array([r["r_blend"] for r in regions], dtype=np.float64).reshape(k)
    bl = np.array([r.get("blend", 0) for r in regions], dtype=np.int32).reshape(k)
    return typ, ax, fol, cen, rc, rb, bl


def lambda_flags(pos, L, periodic, regions):
    """Geometric regions (types 0, 1); seeded regions (type 2) are skipped
    here and applied by lambda_seeded over the neighbour list."""
    pos = _f64(pos)
    n = len(pos)
    typ, ax, fol, cen, rc, rb, bl = _regions_arrays(regions)
    lam = np.zeros(n)
    flags = np.zeros(n, dtype=np.uint8)
    lib().or_lambda(ctypes.c_int(n), _p(pos), _p(_f64(L)), _p(_i32(periodic)),
                    ctypes.c_int(len(regions)), _p(typ), _p(ax), _p(fol), _p(cen),
                    _p(rc), _p(rb), _p(bl), _p(lam), _p(flags))
    return lam, flags


def lambda_seeded(pos, L, periodic, offs, nbr, seeds, regions, lam):
    """Seeded regions (Algorithms 1-2 over the neighbour list) on top of the
    geometric lambda; returns (lambda, flags)."""
    pos = _f64(pos)
    n = len(pos)
    typ, ax, fol, cen, rc, rb, bl = _regions_arrays(regions)
    lam = _f64(lam).copy()
    flags = np.zeros(n, dtype=np.uint8)
    seed = np.ascontiguousarray(np.asarray(seeds).astype(np.uint8))
    lib().or_lambda_seeded(ctypes.c_int(n), _p(pos), _p(_f64(L)), _p(_i32(periodic)),
                           _p(offs), _p(_i32(nbr)), _p(seed), ctypes.c_int(len(regions)),
                           _p(typ), _p(rc), _p(rb), _p(bl), _p(lam), _p(flags))
    return lam, flags


def cheap_buffer_flags(pos, L, periodic, offs, nbr, r_buffer, lam, flags):
    pos = _f64(pos)
    flags = flags.copy()
    lib().or_cheap_buffer(ctypes.c_int(len(pos)), _p(pos), _p(_f64(L)), _p(_i32(periodic)),
                          _p(offs), _p(_i32(nbr)), ctypes.c_double(r_buffer), _p(_f64(lam)),
                          _p(flags))
    return flags


def buffer_flags(pos, L, periodic, offs, nbr, r_buffer, lam, flags):
    pos = _f64(pos)
    flags = flags.copy()
    lib().or_buffer(ctypes.c_int(len(pos)), _p(pos), _p(_f64(L)), _p(_i32(periodic)),
                    _p(offs), _p(_i32(nbr)), ctypes.c_double(r_buffer), _p(_f64(lam)),
                    _p(flags))
    return flags


# --------------------------------------------------------------- potentials

def _ace_struct(model):
    a = model["ace"]
    keep = dict(c0=_f64(a["c0"]), c1=_f64(a["c1"]), c2=_f64(a["c2"]), c3=_f64(a["c3"]))
    s = _Ace(model["n_species"], a["n_rad"], a["lmax"], a["order"], a["rcut"],
             _p(keep["c0"]).value, _p(keep["c1"]).value, _p(keep["c2"]).value,
             _p(keep["c3"]).value)
    return s, keep


def _uf3_struct(model):
    u = model["uf3"]
    keep = dict(c2=_f64(u["c2"]), c3=_f64(u["c3"]))
    s = _Uf3(model["n_species"], u["n_knots2"], u["n_knots3"], 0, u["rcut2"], u["rcut3"],
             _p(keep["c2"]).value, _p(keep["c3"]).value)
    return s, keep


def ace(model, pos, species, L, periodic, offs, nbr, in_S=None, target=None, weights=None):
    """Site energies and forces of the ACE-style model on the subsystem S."""
    pos = _f64(pos)
    n = len(pos)
    s, keep = _ace_struct(model)
    e = np.zeros(n)
    f = np.zeros((n, 3))
    inS = None if in_S is None else np.ascontiguousarray(in_S, dtype=np.uint8)
    tg = None if target is None else np.ascontiguousarray(target, dtype=np.uint8)
    w = None if weights is None else _f64(weights)
    rc = lib().or_ace_eval(ctypes.byref(s), ctypes.c_int(n), _p(pos), _p(_i32(species)),
                           _p(_f64(L)), _p(_i32(periodic)), _p(offs), _p(_i32(nbr)),
                           _p(inS), _p(tg), _p(w), _p(e), _p(f))
    assert rc == 0
    return e, f


def ace_site(model, z, A):
    """E and dE/dA of one site for a given atomic-basis vector A[nchan][L2]."""
    s, keep = _ace_struct(model)
    A = _f64(A)
    dA = np.zeros_like(A)
    E = lib().or_ace_site(ctypes.byref(s), ctypes.c_int(z), _p(A), _p(dA))
    return E, dA


def uf3(model, pos, species, L, periodic, offs, nbr, target=None, in_S=None):
    """Cheap potential; with in_S only on that induced subsystem."""
    pos = _f64(pos)
    n = len(pos)
    s, keep = _uf3_struct(model)
    e = np.zeros(n)
    f = np.zeros((n, 3))
    tg = None if target is None else np.ascontiguousarray(target, dtype=np.uint8)
    inS = None if in_S is None else np.ascontiguousarray(in_S, dtype=np.uint8)
    rc = lib().or_uf3_eval(ctypes.byref(s), ctypes.c_int(n), _p(pos), _p(_i32(species)),
                           _p(_f64(L)), _p(_i32(periodic)), _p(offs), _p(_i32(nbr)),
                           _p(tg), _p(inS), _p(e), _p(f))
    assert rc == 0
    return e, f


# ---------------------------------------------------------- special functions

def ylm(lmax, u):
    u = _f64(u)
    L2 = (lmax + 1) ** 2
    Y = np.zeros(L2)
    g = np.zeros((L2, 3))
    lib().or_ylm(ctypes.c_int(lmax), _p(u), _p(Y), _p(g))
    return Y, g


def radial(n_rad, rc, r):
    R = np.zeros(n_rad)
    dR = np.zeros(n_rad)
    lib().or_radial(ctypes.c_int(n_rad), ctypes.c_double(rc), ctypes.c_double(r), _p(R), _p(dR))
    return R, dR


def gaunt_table(lmax):
    L2 = (lmax + 1) ** 2
    G = np.zeros((L2, L2, L2))
    lib().or_gaunt_table(ctypes.c_int(lmax), _p(G))
    return G


def clamped_knots(n_pts, top):
    t = np.zeros(n_pts + 6)
    lib().or_clamped_knots(ctypes.c_int(n_pts), ctypes.c_double(top), _p(t))
    return t


def bspline(t, x):
    t = _f64(t)
    nb = len(t) - 4
    B = np.zeros(nb)
    dB = np.zeros(nb)
    lib().or_bspline(_p(t), ctypes.c_int(len(t)), ctypes.c_double(x), _p(B), _p(dB))
    return B, dB


def csum(x):
    x = _f64(x)
    return float(lib().or_sum(ctypes.c_int(len(x)), _p(x)))


# ----------------------------------------------------------- whole pipeline

def r_list(model):
    return max(model["ace"]["rcut"], model["uf3"]["rcut2"],
               model["uf3"]["rcut3"] if model["uf3"]["n_knots3"] > 0 else 0.0) + model["skin"]


def mixed(w, mode=MODE_MIXED, pos=None, target=None, method=1, cheap_masked=False):
    """The whole mixed force evaluation for workload w.

    Returns dict(lam, flags, S, M, offs, nbr, e_exp, f_exp, e_cheap, f_cheap,
    forces). Modes: mixed; all-expensive (lambda = 1, S = every atom, cheap
    not evaluated); all-cheap (lambda = 0, S empty). cheap_masked (mixed
    mode): the cheap potential too sees only its induced subsystem
    S_c = {lambda < 1} plus its buffer (flags bit3), as Algorithm 4 masks each
    potential in turn.
    """
    pos = w["pos"] if pos is None else pos
    pos = _f64(pos)
    n = len(pos)
    model = w["model"]
    offs, nbr = neighbors(pos, w["L"], w["periodic"], r_list(model), method)
    if mode == MODE_MIXED:
        lam, flags = lambda_flags(pos, w["L"], w["periodic"], w["regions"])
        if any(r["type"] == 2 for r in w["regions"]):
            lam, flags = lambda_seeded(pos, w["L"], w["periodic"], offs, nbr, w["seeds"],
                                       w["regions"], lam)
        flags = buffer_flags(pos, w["L"], w["periodic"], offs, nbr, w["r_buffer"], lam, flags)
        if cheap_masked:
            flags = cheap_buffer_flags(pos, w["L"], w["periodic"], offs, nbr, w["r_buffer"], lam,
                                       flags)
    elif mode == MODE_ALL_EXPENSIVE:
        lam = np.ones(n)
        flags = np.full(n, 3, dtype=np.uint8)
    else:
        lam = np.zeros(n)
        flags = np.zeros(n, dtype=np.uint8)
    in_S = (flags & 5) != 0
    S = np.nonzero(in_S)[0].astype(np.int32)
    M = np.nonzero(flags & 1)[0].astype(np.int32)
    if mode != MODE_ALL_CHEAP and len(S):
        e_exp, f_exp = ace(model, pos, w["species"], w["L"], w["periodic"], offs, nbr,
                           in_S=in_S, target=target)
    else:
        e_exp, f_exp = np.zeros(n), np.zeros((n, 3))
    if mode != MODE_ALL_EXPENSIVE:
        in_Sc = None
        if cheap_masked and mode == MODE_MIXED:
            in_Sc = (lam < 1.0) | ((flags & 8) != 0)
        e_ch, f_ch = uf3(model, pos, w["species"], w["L"], w["periodic"], offs, nbr,
                         target=target, in_S=in_Sc)
    else:
        e_ch, f_ch = np.zeros(n), np.zeros((n, 3))
    forces = np.zeros((n, 3))
    lib().or_blend(ctypes.c_int(n), _p(lam), _p(f_exp), _p(f_ch), _p(forces))
    return dict(lam=lam, flags=flags, S=S, M=M, offs=offs, nbr=nbr, e_exp=e_exp,
                f_exp=f_exp, e_cheap=e_ch, f_cheap=f_ch, forces=forces)


def velocity_verlet(w, pos, vel, dt, nsteps, mode=MODE_MIXED, callback=None, cheap_masked=False,
                    langevin=None):
    """Velocity Verlet: v += dt/2 kappa F/m; x += dt v; wrap; F(x); v += dt/2 kappa F/m.

    langevin = (T in K, tau in fs, xi) adds a Langevin thermostat on the cheap
    region only (Methods, Si stretched bond and diffusion coefficients: a weak
    thermostat applied where the cheap potential alone acts). After each force
    evaluation an atom with lambda == 0 feels, besides its blended force, the
    friction -m v / tau and a random force whose variance over one step dt
    fixes the temperature, 2 m kB T / (tau dt) (both in mass-velocity units,
    divided by kappa for eV/A); v is the half-step velocity at that moment.
    xi[step] is an (n, 3) array of standard normals for the step's force call.
    """
    from gen.workloads import KAPPA, KB
    m = w["masses"][w["species"]][:, None]
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    out = mixed(w, mode, pos=pos, cheap_masked=cheap_masked)
    F = out["forces"]
    for step in range(nsteps):
        vel = vel + 0.5 * dt * KAPPA * F / m
        pos = pos + dt * vel
        for k in range(3):
            if w["periodic"][k]:
                Lk = w["L"][k]
                pos[:, k] = pos[:, k] - Lk * np.floor(pos[:, k] / Lk)
        out = mixed(w, mode, pos=pos, cheap_masked=cheap_masked)
        F = out["forces"]
        if langevin is not None:
            T, tau, xi = langevin
            cheap = (out["lam"] == 0.0)[:, None]
            friction = -m * vel / (KAPPA * tau)
            noise = np.sqrt(2.0 * m * KB * T / (KAPPA * tau * dt)) * np.asarray(xi[step], np.float64)
            F = np.where(cheap, F + (friction + noise), F)
            out = dict(out, forces=F)
        vel = vel + 0.5 * dt * KAPPA * F / m
        if callback:
            callback(step, pos, vel, out)
    return pos, vel, out


def kinetic(w, vel):
    from gen.workloads import KAPPA
    m = w["masses"][w["species"]]
    return csum(0.5 * m * (vel ** 2).sum(1)) / KAPPA
