"""The hand-written adjoint behind torch.autograd.Function: gradients of the
expensive site energies against central finite differences (h = 1e-4 A) on a
128-atom subset of the 54,000-atom screw-dislocation column, and against the
FP64 oracle's gradient of a randomly weighted sum of site energies."""
import numpy as np
import pytest

import oracle as O
from gen import workloads as W

pytestmark = pytest.mark.gpu


def _system(w, precision):
    from paper_2502_19081_amd import core
    model = core.Model(w["model"], precision=precision)
    return core.system_for(w, model=model, cap=128)


def test_adjoint_matches_finite_differences_c3_subset():
    import torch
    from paper_2502_19081_amd.autograd import expensive_energy
    w = W.c3()
    print(f"case c3 n={len(w['pos'])} FP64 finite differences, 128 atoms", flush=True)
    _, sy, pos, sp = _system(w, "fp64")
    p = pos.clone().requires_grad_(True)
    e = expensive_energy(p, sy, sp, w["r_buffer"])
    E = e.sum()
    E.backward()
    grad = p.grad.detach().cpu().numpy()
    flags = sy.flags.cpu().numpy()
    M = np.nonzero(flags & 1)[0]
    rng = np.random.default_rng(w["seed"] + 128)
    pick = rng.choice(M, size=128, replace=False)
    h = 1e-4
    errs = []
    for i in pick:
        for k in range(3):
            vals = []
            for sg in (1, -1):
                q = pos.clone()
                q[k, i] += sg * h
                ek = expensive_energy(q, sy, sp, w["r_buffer"])
                vals.append(ek.sum().item())
            fd = (vals[0] - vals[1]) / (2 * h)
            errs.append(abs(fd - grad[k, i]))
    print(f"  max |grad - FD| = {max(errs):.3e} eV/A", flush=True)
    assert max(errs) < 2e-5


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_adjoint_matches_oracle_weighted_gradient(precision, tol):
    import torch
    from paper_2502_19081_amd.autograd import expensive_energy
    w = W.c2()
    print(f"case c2 weighted adjoint {precision}", flush=True)
    _, sy, pos, sp = _system(w, precision)
    rng = np.random.default_rng(5)
    wts = rng.normal(size=len(w["pos"]))
    p = pos.clone().requires_grad_(True)
    e = expensive_energy(p, sy, sp, w["r_buffer"])
    (e * torch.from_numpy(wts).cuda()).sum().backward()
    g = p.grad.detach().cpu().numpy().T
    ref = O.mixed(w)
    in_S = (ref["flags"] & 5) != 0
    _, f_w = O.ace(w["model"], w["pos"], w["species"], w["L"], w["periodic"], ref["offs"], ref["nbr"],
                   in_S=in_S, weights=wts)
    err = np.abs(g - (-f_w)).max()
    print(f"  max |dG| = {err:.3e} (scale {np.abs(f_w).max():.3f})", flush=True)
    if precision == "fp64":
        assert err < tol * np.abs(f_w).max()
    else:
        assert err < tol
    np.testing.assert_allclose(e.detach().cpu().numpy()[in_S], ref["e_exp"][in_S],
                               atol=1e-9 if precision == "fp64" else 1e-3)


def test_adjoint_large_system_kernels_fp32():
    # above 65,536 atoms the forward keeps the finalisation kernel and the
    # backward runs the vector pair adjoint with two S atoms per wave
    # (lmax 5, 16 channels, 4 vacancy spheres in a 34^3-cell bcc crystal)
    import torch
    from paper_2502_19081_amd.autograd import expensive_energy
    w = W.c5(n=34, n_vac=4)
    n = len(w["pos"])
    assert n > 65536
    print(f"case weighted adjoint n={n} fp32 (large-system kernels)", flush=True)
    _, sy, pos, sp = _system(w, "fp32")
    rng = np.random.default_rng(6)
    wts = rng.normal(size=n)
    p = pos.clone().requires_grad_(True)
    e = expensive_energy(p, sy, sp, w["r_buffer"])
    (e * torch.from_numpy(wts).cuda()).sum().backward()
    g = p.grad.detach().cpu().numpy().T
    target = np.zeros(n, bool)
    target[:8] = True  # lists, lambda and S are global; few cheap forces needed
    ref = O.mixed(w, target=target)
    in_S = (ref["flags"] & 5) != 0
    _, f_w = O.ace(w["model"], w["pos"], w["species"], w["L"], w["periodic"], ref["offs"], ref["nbr"],
                   in_S=in_S, weights=wts)
    err = np.abs(g - (-f_w)).max()
    print(f"  |S| = {int(in_S.sum())}, max |dG| = {err:.3e} (scale {np.abs(f_w).max():.3f})",
          flush=True)
    assert err < 1e-4


def test_backward_refuses_stale_forward():
    import torch
    from paper_2502_19081_amd.autograd import expensive_energy
    w = W.c1()
    _, sy, pos, sp = _system(w, "fp64")
    p = pos.clone().requires_grad_(True)
    e = expensive_energy(p, sy, sp, w["r_buffer"])
    sy.compute(pos, sp, r_buffer=w["r_buffer"])
    with pytest.raises(RuntimeError):
        e.sum().backward()
