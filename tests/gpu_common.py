"""Helpers shared by the GPU tests: run the HIP path on a workload and bring
the results to numpy in the oracle's (N, 3) layout."""
import numpy as np


def run_gpu(w, mode=0, precision=None, cap=128, force_rebuild=True, split=True, system=None,
            cheap_masked=False):
    import torch
    from paper_2502_19081_amd import core
    prec = precision or w.get("precision", "fp64")
    if system is None:
        model = core.Model(w["model"], precision=prec)
        _, sy, pos, sp = core.system_for(w, model=model, cap=cap)
        if "seeds" in w:
            sy.set_seeds(torch.from_numpy(np.asarray(w["seeds"]).astype(np.uint8)))
    else:
        sy, pos, sp = system
    out = sy.compute(pos, sp, r_buffer=w["r_buffer"], mode=mode, force_rebuild=force_rebuild,
                     split=split, cheap_masked=cheap_masked)
    bits, req, rc = sy.status(raise_on_error=False)
    torch.cuda.synchronize()
    assert rc == 0, f"device status {bits} (required cap {req})"
    res = {k: (v.cpu().numpy().T.copy() if v is not None and v.dim() == 2 else v.cpu().numpy())
           for k, v in out.items()}
    S, M = sy.index_sets()
    nbr, cnt = sy.neighbors()
    res["S"] = S.cpu().numpy()
    res["M"] = M.cpu().numpy()
    res["nbr"] = nbr.cpu().numpy()
    res["cnt"] = cnt.cpu().numpy()
    res["system"] = (sy, pos, sp)
    return res


def csr_rows(offs, nbr):
    return [nbr[offs[i]:offs[i + 1]] for i in range(len(offs) - 1)]


def assert_neighbors_equal(g, ref):
    rows = csr_rows(ref["offs"], ref["nbr"])
    assert np.array_equal(g["cnt"], np.diff(ref["offs"]).astype(np.int32))
    for i, r in enumerate(rows):
        c = g["cnt"][i]
        assert np.array_equal(g["nbr"][i, :c], r), f"row {i}"


def rel_force_err(F, Fref):
    return np.abs(F - Fref).max() / max(np.abs(Fref).max(), 1e-300)
