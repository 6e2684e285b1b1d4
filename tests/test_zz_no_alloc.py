"""The allocation-free entry point (mlmix_compute_noalloc): its workspace is
the library's static device scratch. Two calls in a row through the C ABI,
the second on a smaller system, each against mlmix_compute on a caller
workspace of the same row and S capacity (forced rebuild): identical bits
(the same kernels do the same arithmetic). A system too large for the
scratch is refused on the host."""
import ctypes

import numpy as np
import pytest

from gen import workloads as W
from gen.lattice import bcc_cubic, wrap

pytestmark = pytest.mark.gpu


def _small_cell_with_c2_model(w2, cells=10, sigma=0.08, seed=77):
    """A 2,000-atom bcc cube with the 8,193-atom cell's potentials and a
    sphere of the same radii at its centre."""
    rng = np.random.default_rng(seed)
    pos = bcc_cubic(cells, cells, cells)
    L = np.array([cells * W.A_W] * 3)
    pos = wrap(pos + rng.normal(0.0, sigma, size=pos.shape), L, [1, 1, 1])
    w = dict(w2)
    w.update(pos=pos, species=np.zeros(len(pos), dtype=np.int32), L=L,
             regions=[W.sphere(L / 2.0, 8.0, 2.0)])
    return w


def _noalloc(model, w, cap, s_cap, pos, sp, regions, out):
    import torch
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    box = core.make_box(w["L"], w["periodic"])
    used = ctypes.c_size_t()
    rc = B.lib().mlmix_compute_noalloc(
        model.handle, core._stream(), len(w["pos"]), cap, s_cap, core._p(pos), core._p(sp),
        ctypes.byref(box), core._p(regions), len(w["regions"]), float(w["r_buffer"]),
        B.MODE_MIXED, core._p(out["forces"]), core._p(out["e_exp"]), core._p(out["e_cheap"]),
        core._p(out["lam"]), core._p(out["flags"]), core._p(out["n_exp"]),
        core._p(out["status"]), ctypes.byref(used))
    return rc, used.value


def _outputs(n):
    import torch
    z = dict(dtype=torch.float64, device="cuda")
    return dict(forces=torch.full((3, n), np.nan, **z), e_exp=torch.full((n,), np.nan, **z),
                e_cheap=torch.full((n,), np.nan, **z), lam=torch.full((n,), np.nan, **z),
                flags=torch.full((n,), 255, dtype=torch.uint8, device="cuda"),
                n_exp=torch.full((2,), -1, dtype=torch.int32, device="cuda"),
                status=torch.full((2,), -1, dtype=torch.int32, device="cuda"))


def _reference(model, w, cap, s_cap):
    from paper_2502_19081_amd import core
    _, sy, pos, sp = core.system_for(w, model=model, cap=cap, s_cap=s_cap)
    out = sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    sy.status()
    return {k: v.clone() for k, v in out.items()}, pos, sp


def test_noalloc_matches_workspace_path_twice_second_smaller():
    import torch
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    w2 = W.c2()
    model = core.Model(w2["model"], precision="fp32")
    small = _small_cell_with_c2_model(w2)
    cases = [("c2 8,193 atoms, s_cap 2048", w2, 128, 2048),
             ("2,000-atom cube, s_cap = n", small, 128, 0)]
    for name, w, cap, s_cap in cases:
        n = len(w["pos"])
        print(f"case noalloc {name}", flush=True)
        ref, pos, sp = _reference(model, w, cap, s_cap)
        regions = core.pack_regions(w["regions"])
        out = _outputs(n)
        rc, used = _noalloc(model, w, cap, s_cap, pos, sp, regions, out)
        assert rc == 0, B.lib().mlmix_last_error().decode()
        assert 0 < used <= B.NOALLOC_SCRATCH_BYTES
        torch.cuda.synchronize()
        # no status bit and no overflowing row (the row count is kept only
        # for an overflowing row)
        assert out["status"].cpu().tolist() == [0, 0]
        for k in ("forces", "e_exp", "e_cheap", "lam", "flags", "n_exp"):
            a, b = out[k].cpu().numpy(), ref[k].cpu().numpy()
            assert np.array_equal(a, b), (name, k, np.abs(a.astype(float) - b.astype(float)).max())
        assert out["n_exp"][0].item() > 0


def test_noalloc_refuses_a_system_beyond_the_scratch():
    import torch
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    w2 = W.c2()
    model = core.Model(w2["model"], precision="fp32")
    print("case noalloc refuses 8,193 atoms with s_cap = n (beyond the scratch)", flush=True)
    pos = torch.from_numpy(np.ascontiguousarray(w2["pos"].T)).cuda()
    sp = torch.from_numpy(w2["species"]).cuda()
    out = _outputs(len(w2["pos"]))
    rc, used = _noalloc(model, w2, 256, 0, pos, sp, core.pack_regions(w2["regions"]), out)
    assert rc == -3  # MLMIX_E_WORKSPACE
    assert used > B.NOALLOC_SCRATCH_BYTES
    torch.cuda.synchronize()
    # nothing was launched: the outputs keep their fill
    assert out["n_exp"].cpu().tolist() == [-1, -1]
