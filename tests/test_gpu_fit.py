"""Constrained fit of the cheap potential on the device against the oracle:
design rows element by element, the weighted normal equations, the lambda
search, and the whole pipeline on labelled synthetic data."""
import numpy as np
import pytest

import oracle as O
from oracle import fit as OF
from gen import fitdata as FD
from gen import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _design_gpu(model_desc, cfg, species=None):
    import torch
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    from paper_2502_19081_amd.fit import CheapFit
    model = core.Model(model_desc, precision="fp64")
    fit = CheapFit(model)
    n = len(cfg["pos"])
    sp = np.zeros(n, np.int32) if species is None else species
    sy = core.System(model, n, cfg["L"], cfg["periodic"], cap=128)
    pos = _dev(cfg["pos"].T)
    spd = torch.from_numpy(sp).cuda()
    sy.compute(pos, spd, mode=B.MODE_ALL_CHEAP, force_rebuild=True)
    rows = fit.design(sy, pos, spd)
    sy.status()
    return rows.cpu().numpy(), fit


@pytest.mark.parametrize("case", ["thermal_250", "strained_250", "cluster_two_species"])
def test_design_rows_match_oracle(case):
    if case == "thermal_250":
        m = FD.fit_model()
        cfg = FD.thermal_snapshots(1, cells=5, sigma=0.12, seed=21)[0]
        sp = None
    elif case == "strained_250":
        m = FD.fit_model()
        cfg = FD.strained_cells(n_strain=3)[4]   # uniaxial [100], -0.5 %
        sp = None
    else:
        w = W.tiny(seed=23, n_species=2, periodic=(0, 0, 0), vacuum=4.0, sigma=0.1)
        m = w["model"]
        cfg = dict(pos=w["pos"], L=w["L"], periodic=w["periodic"])
        sp = w["species"]
    print(f"case fit design rows {case}, n={len(cfg['pos'])}", flush=True)
    A, fit = _design_gpu(m, cfg, sp)
    ref = OF.design(m, cfg["pos"], np.zeros(len(cfg["pos"]), np.int32) if sp is None else sp,
                    cfg["L"], cfg["periodic"])
    assert fit.nd == ref.shape[1]
    scale = np.abs(ref).max()
    err = np.abs(A - ref).max()
    print(f"  nd={fit.nd} max |dA| = {err:.3e} (scale {scale:.3e})", flush=True)
    assert err <= 1e-12 * scale


@pytest.mark.parametrize("n_rows", [1, 1000, 70001])
def test_gram_matches_oracle(n_rows):
    import torch
    from paper_2502_19081_amd import core
    from paper_2502_19081_amd.fit import CheapFit
    print(f"case fit gram, {n_rows} rows x 81", flush=True)
    fit = CheapFit(core.Model(FD.fit_model(), precision="fp64"))
    r = np.random.default_rng(n_rows)
    A = r.normal(size=(n_rows, fit.nd))
    y = r.normal(size=n_rows)
    w = r.uniform(0.1, 2.0, size=n_rows)
    G, b = fit.gram(_dev(A), _dev(y), _dev(w))
    # accumulation: a second call on the same rows doubles the sums
    G2, b2 = fit.gram(_dev(A), _dev(y), _dev(w), G.clone(), b.clone())
    Gr, br = OF.gram(A, y, w)
    G = G.cpu().numpy()
    assert np.array_equal(G, G.T)
    assert np.abs(G - Gr).max() <= 1e-13 * np.abs(Gr).max() * max(1.0, np.sqrt(n_rows) / 10)
    assert np.abs(b.cpu().numpy() - br).max() <= 1e-13 * np.abs(br).max() * max(1.0, np.sqrt(n_rows) / 10)
    assert np.array_equal(G2.cpu().numpy(), 2.0 * G)


def _problem(seed, ns=400, nh=30, nd=20):
    r = np.random.default_rng(seed)
    return r.normal(size=(ns, nd)), r.normal(size=ns), r.normal(size=(nh, nd)), r.normal(size=nh)


@pytest.mark.parametrize("case", ["bisection", "unreachable", "lambda0_passes"])
def test_search_matches_oracle(case):
    from paper_2502_19081_amd import core
    from paper_2502_19081_amd.fit import CheapFit
    import torch
    print(f"case fit lambda search {case}", flush=True)
    model = core.Model(FD.fit_model(), precision="fp64")
    fit = CheapFit(model)
    nd = fit.nd   # 81 parameters; the problem uses the first 20 and pins the rest with the ridge
    AS, yS, AH, yH = _problem(7, nh=12 if case != "unreachable" else 60)
    k = AS.shape[1]
    ASf = np.zeros((len(yS), nd))
    ASf[:, :k] = AS
    AHf = np.zeros((len(yH), nd))
    AHf[:, :k] = AH
    GS, bS = OF.gram(ASf, yS, np.ones(len(yS)))
    ridge = 1e-6
    c_free = OF.solve_fixed(GS, bS, np.zeros((nd, nd)), np.zeros(nd), 0.0, ridge)
    r_free = OF.hard_residual(AHf, yH, c_free)
    if case == "bisection":
        alpha, lam0 = 0.2 * r_free, 1e-3
    elif case == "unreachable":
        r_min = OF.hard_residual(AH, yH, np.linalg.lstsq(AH, yH, rcond=None)[0])
        alpha, lam0 = 0.5 * r_min, 1.0
    else:
        alpha, lam0 = 2.0 * r_free, 1e-3
    tol = alpha / 10.0
    ref_c, ref = OF.constrained_fit(GS, bS, AHf, yH, alpha, lam0=lam0, ridge=ridge, tol=tol,
                                    max_decades=12)
    u, info = fit.constrained(_dev(GS), _dev(bS), _dev(AHf), _dev(yH), alpha, tol=tol, lam0=lam0,
                              ridge=ridge, max_decades=12)
    print(f"  device {info} oracle lam {ref['lam']:.6e} res {ref['residual']:.6e} "
          f"solves {ref['n_solves']} status {ref['status']}", flush=True)
    assert info["status"] == ref["status"]
    assert info["n_solves"] == ref["n_solves"]
    if case == "unreachable":
        # the residual has reached its floor: which decade holds the smallest
        # value is decided by rounding, so only the floor is compared
        assert abs(info["residual"] - ref["residual"]) <= 1e-6 * ref["residual"]
        assert info["residual"] > alpha
        return
    assert abs(info["lam"] - ref["lam"]) <= 1e-12 * ref["lam"]
    assert abs(info["residual"] - ref["residual"]) <= 1e-9 * ref["residual"]
    u = u.cpu().numpy()
    assert np.abs(u - ref_c).max() <= 1e-8 * np.abs(ref_c).max()
    if case == "bisection":
        assert alpha - tol < info["residual"] <= alpha


def test_fit_pipeline_matches_oracle():
    # two thermal snapshots (soft: per-atom energy and forces) and ten strained
    # cells (hard: per-atom energies), labelled by the expensive potential
    import torch
    from paper_2502_19081_amd import core
    from paper_2502_19081_amd.fit import CheapFit, label_and_design
    print("case fit pipeline: 2 soft snapshots of 250 atoms, 10 strained cells of 250 atoms",
          flush=True)
    m = FD.fit_model()
    soft = FD.thermal_snapshots(2, cells=5, sigma=0.12, seed=31)
    hard = [c for c in FD.strained_cells(n_strain=5) if c["state"] in ("hydrostatic", "tetragonal shear")]
    model = core.Model(m, precision="fp64")
    fit = CheapFit(model)
    S = label_and_design(fit, soft)
    H = label_and_design(fit, hard)
    rows = torch.cat([r for (_, _, _, r) in S])
    y = torch.cat([torch.cat([e.reshape(1), f.reshape(-1)]) for (_, e, f, _) in S])
    w = torch.cat([torch.cat([torch.full((1,), 1.0 / n ** 2), torch.ones(3 * n)]) for (n, _, _, _) in S]).cuda().double()
    GS, bS = fit.gram(rows, y, w)
    # hard rows: total-energy rows weighted 1/n^2 (per-atom energy errors)
    AH = torch.stack([r[0] for (_, _, _, r) in H]).contiguous()
    yH = torch.stack([e for (_, e, _, _) in H])
    wH = torch.tensor([1.0 / n ** 2 for (n, _, _, _) in H], dtype=torch.float64).cuda()
    ridge = 1e-8 * float(torch.diagonal(GS).mean())
    u0, i0 = fit.constrained(GS, bS, AH, yH, 1e30, lam0=1e-12, ridge=ridge, wH=wH)
    r_free = i0["residual"]
    alpha = 1e-3 * r_free
    u, info = fit.constrained(GS, bS, AH, yH, alpha, lam0=1e-6, ridge=ridge, wH=wH)

    # the oracle: its own labels and design rows
    def lab(cfgs):
        out = []
        for c in cfgs:
            n = len(c["pos"])
            wk = dict(pos=c["pos"], species=np.zeros(n, np.int32), L=c["L"], periodic=c["periodic"],
                      regions=[], r_buffer=0.0, model=m, masses=np.array([183.84, 4.0]))
            o = O.mixed(wk, O.MODE_ALL_EXPENSIVE)
            A = OF.design(m, c["pos"], np.zeros(n, np.int32), c["L"], c["periodic"])
            out.append((n, o["e_exp"].sum(), o["forces"], A))
        return out
    So, Ho = lab(soft), lab(hard)
    Ar = np.vstack([A for (_, _, _, A) in So])
    yr = np.concatenate([np.concatenate([[e], f.T.reshape(-1)]) for (_, e, f, _) in So])
    wr = np.concatenate([np.concatenate([[1.0 / n ** 2], np.ones(3 * n)]) for (n, _, _, _) in So])
    GSr, bSr = OF.gram(Ar, yr, wr)
    AHr = np.stack([A[0] for (_, _, _, A) in Ho])
    yHr = np.array([e for (_, e, _, _) in Ho])
    wHr = np.array([1.0 / n ** 2 for (n, _, _, _) in Ho])
    assert np.abs(rows.cpu().numpy() - Ar).max() <= 1e-12 * np.abs(Ar).max()
    assert np.abs(y.cpu().numpy() - yr).max() <= 1e-9 * np.abs(yr).max()
    ur, ref = OF.constrained_fit(GSr, bSr, AHr, yHr, alpha, lam0=1e-6, ridge=ridge, wH=wHr)
    print(f"  device {info}; oracle lam {ref['lam']:.6e} res {ref['residual']:.6e} "
          f"solves {ref['n_solves']} status {ref['status']}; unconstrained residual {r_free:.3e}",
          flush=True)
    assert info["status"] == ref["status"] == 0
    assert alpha - alpha / 10 < info["residual"] <= alpha
    assert abs(info["lam"] / ref["lam"] - 1.0) < 1e-6
    # predictions of the two fits agree on the soft and the hard data
    pu = Ar @ u.cpu().numpy()
    pr = Ar @ ur
    assert np.abs(pu - pr).max() <= 1e-6 * np.abs(pr).max()


def test_batched_design_equals_single_calls():
    # 30 strained cells of three sizes (two launches of the batched call)
    import torch
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    from paper_2502_19081_amd.fit import CheapFit
    print("case fit design, 30 configurations in one batched call vs one call each", flush=True)
    model = core.Model(FD.fit_model(), precision="fp64")
    fit = CheapFit(model)
    cfgs = FD.strained_cells(n_strain=5)
    cfgs = cfgs[::1][:30]
    items = []
    for c in cfgs:
        n = len(c["pos"])
        sy = core.System(model, n, c["L"], c["periodic"], cap=128)
        pos = _dev(c["pos"].T)
        sp = torch.zeros(n, dtype=torch.int32, device="cuda")
        sy.compute(pos, sp, mode=B.MODE_ALL_CHEAP, force_rebuild=True)
        items.append((sy, pos, sp, torch.full((1 + 3 * n, fit.nd), float("nan"),
                                              dtype=torch.float64, device="cuda")))
    fit.design_many(items)
    for sy, pos, sp, out in items:
        ref = fit.design(sy, pos, sp)
        sy.status()
        assert torch.equal(out, ref)


def test_design_row_stride_and_empty_edge_cases():
    # ld wider than the parameter count leaves the padding columns untouched;
    # an empty row set leaves G and b as they were; no hard rows leaves the
    # unconstrained (ridge) solution at lambda0 with status 0
    import ctypes
    import torch
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    from paper_2502_19081_amd.core import _p, _stream
    from paper_2502_19081_amd.fit import CheapFit
    print("case fit edge cases: row stride, empty Gram, no hard rows", flush=True)
    model = core.Model(FD.fit_model(), precision="fp64")
    fit = CheapFit(model)
    c = FD.strained_cells(n_strain=3)[1]
    n = len(c["pos"])
    sy = core.System(model, n, c["L"], c["periodic"], cap=128)
    pos = _dev(c["pos"].T)
    sp = torch.zeros(n, dtype=torch.int32, device="cuda")
    sy.compute(pos, sp, mode=B.MODE_ALL_CHEAP, force_rebuild=True)
    ld = fit.nd + 7
    wide = torch.full((1 + 3 * n, ld), float("nan"), dtype=torch.float64, device="cuda")
    B.check(B.lib().mlmix_fit_design(model.handle, _stream(), _p(sy.ws), n, _p(pos), _p(sp),
                                     ctypes.byref(sy.box), _p(wide), ld))
    ref = fit.design(sy, pos, sp)
    sy.status()
    assert torch.equal(wide[:, :fit.nd], ref)
    assert torch.isnan(wide[:, fit.nd:]).all()

    G = torch.full((fit.nd, fit.nd), 2.0, dtype=torch.float64, device="cuda")
    b = torch.full((fit.nd,), 3.0, dtype=torch.float64, device="cuda")
    empty = torch.zeros(0, fit.nd, dtype=torch.float64, device="cuda")
    fit.gram(empty, None, None, G, b)
    assert bool((G == 2.0).all()) and bool((b == 3.0).all())

    r = np.random.default_rng(3)
    A = r.normal(size=(300, fit.nd))
    y = r.normal(size=300)
    GS, bS = OF.gram(A, y, np.ones(300))
    ridge = 1e-3
    u, info = fit.constrained(_dev(GS), _dev(bS), torch.zeros(0, fit.nd, dtype=torch.float64,
                                                               device="cuda"),
                              torch.zeros(0, dtype=torch.float64, device="cuda"), 1e-6,
                              lam0=1e-3, ridge=ridge)
    assert info["status"] == 0 and info["n_solves"] == 1 and info["residual"] == 0.0
    want = OF.solve_fixed(GS, bS, np.zeros_like(GS), np.zeros_like(bS), 0.0, ridge)
    assert np.abs(u.cpu().numpy() - want).max() <= 1e-10 * np.abs(want).max()
