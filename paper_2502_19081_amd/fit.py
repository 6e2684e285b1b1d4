"""Constrained linear fitting of the cheap potential on the device (Methods,
"Constrained potential fitting"): design rows of labelled configurations,
weighted normal equations and the lambda search, each one call into the HIP
library. Argument marshalling only."""
import ctypes

import numpy as np
import torch

from paper_2502_19081_amd import binding as B
from paper_2502_19081_amd.core import System, _p, _stream

STATUS = {0: "converged", 1: "alpha not reached", 2: "bisection limit", 3: "non-positive pivot"}


class CheapFit:
    """Fits the free coefficients of `model`'s cheap potential (the
    coefficients the model was built with are ignored)."""

    def __init__(self, model, device="cuda"):
        self.model = model
        self.device = device
        nd = B._i32()
        B.check(B.lib().mlmix_fit_n_params(model.handle, ctypes.byref(nd)))
        self.nd = int(nd.value)

    def design(self, system, pos, species, out=None):
        """(1 + 3n, nd) float64 rows of one configuration: energy, then force
        component q of atom i at row 1 + q n + i. The workspace's last
        evaluation must have been on these positions."""
        n = system.n
        if out is None:
            out = torch.empty(1 + 3 * n, self.nd, dtype=torch.float64, device=self.device)
        assert out.shape == (1 + 3 * n, self.nd) and out.is_contiguous()
        B.check(B.lib().mlmix_fit_design(self.model.handle, _stream(), _p(system.ws), n, _p(pos),
                                         _p(species), ctypes.byref(system.box), _p(out), self.nd))
        return out

    def design_many(self, items):
        """Design rows of several configurations in one call, items =
        [(system, pos, species, out)] (one set of launches over all atoms)."""
        arr = (B.FitConfig * len(items))()
        for k, (sy, pos, sp, out) in enumerate(items):
            assert out.shape == (1 + 3 * sy.n, self.nd) and out.is_contiguous()
            arr[k].ws = sy.ws.data_ptr()
            arr[k].n_atoms = sy.n
            arr[k].pos = pos.data_ptr()
            arr[k].species = sp.data_ptr()
            arr[k].box = sy.box
            arr[k].rows = out.data_ptr()
        B.check(B.lib().mlmix_fit_design_batch(self.model.handle, _stream(), len(items), arr,
                                               self.nd))

    def work(self, n_rows):
        sz = ctypes.c_size_t()
        B.check(B.lib().mlmix_fit_work_size(int(n_rows), self.nd, ctypes.byref(sz)))
        return torch.empty(max(int(sz.value), 8), dtype=torch.uint8, device=self.device)

    def gram(self, rows, y=None, w=None, G=None, b=None):
        """G += rows^T diag(w) rows, b += rows^T diag(w) y (fresh zeros when
        G, b are None)."""
        assert rows.dtype == torch.float64 and rows.is_contiguous() and rows.shape[1] == self.nd
        if G is None:
            G = torch.zeros(self.nd, self.nd, dtype=torch.float64, device=self.device)
        if b is None:
            b = torch.zeros(self.nd, dtype=torch.float64, device=self.device)
        wk = self.work(rows.shape[0])
        B.check(B.lib().mlmix_fit_gram(self.model.handle, _stream(), _p(rows), rows.shape[0],
                                       self.nd, self.nd, _p(y), _p(w), _p(G), _p(b), _p(wk),
                                       wk.numel()))
        return G, b

    def constrained(self, GS, bS, AH, yH, alpha, tol=None, lam0=1.0, ridge=0.0, max_decades=24,
                    max_bisect=200, wH=None):
        """The lambda search; returns (u, info dict). wH weights the hard rows."""
        if tol is None:
            tol = alpha / 10.0
        AH = AH.contiguous()
        u = torch.zeros(self.nd, dtype=torch.float64, device=self.device)
        info = torch.zeros(6, dtype=torch.float64, device=self.device)
        wk = self.work(AH.shape[0])
        B.check(B.lib().mlmix_fit_constrained(self.model.handle, _stream(), self.nd, _p(GS), _p(bS),
                                              _p(AH), self.nd, AH.shape[0], _p(yH), _p(wH),
                                              float(alpha),
                                              float(tol), float(lam0), float(ridge),
                                              int(max_decades), int(max_bisect), _p(u), _p(info),
                                              _p(wk), wk.numel()))
        v = info.cpu().numpy()
        return u, dict(lam=float(v[0]), residual=float(v[1]), n_solves=int(v[2]),
                       status=int(v[3]), lam_lo=float(v[4]), decades=int(v[5]))


def label_and_design(fit, configs, cap=128):
    """Expensive-potential labels (total energy, forces) and design rows of
    each configuration (dicts with pos (n, 3), L, periodic, species
    optional). Returns a list of (n, energy, forces (3, n), rows) on the
    device."""
    out = []
    for c in configs:
        n = len(c["pos"])
        sy = System(fit.model, n, c["L"], c["periodic"], cap=cap, device=fit.device)
        pos = torch.from_numpy(np.ascontiguousarray(np.asarray(c["pos"], np.float64).T)).to(fit.device)
        sp = torch.from_numpy(np.asarray(c.get("species", np.zeros(n)), np.int32)).to(fit.device)
        r = sy.compute(pos, sp, mode=B.MODE_ALL_EXPENSIVE, force_rebuild=True)
        rows = fit.design(sy, pos, sp)
        sy.status()
        out.append((n, r["e_exp"].sum(), r["forces"].clone(), rows))
    return out
