"""A workspace whose S capacity (rows of the expensive potential's buffers)
is below |S|: the evaluation keeps the atoms past the capacity out of S,
raises MLMIX_STATUS_S_OVERFLOW and reports the required |S| in
n_expensive[0]; mlmix_status returns MLMIX_E_WORKSPACE. A workspace of
exactly the reported capacity then evaluates the same call without status
bits and with the same bits as a workspace sized for every atom.
"""
import numpy as np
import pytest

from gen import workloads as W

pytestmark = pytest.mark.gpu

E_WORKSPACE = -3


def test_s_capacity_overflow_reported_then_exact_capacity_matches():
    import torch
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    assert B.ERRORS[E_WORKSPACE] == "MLMIX_E_WORKSPACE"
    w = W.c2()
    model = core.Model(w["model"], precision="fp32")
    print("case c2 FP32 with s_cap 256 (|S| above it), then s_cap = |S| and s_cap = n",
          flush=True)
    _, sy, pos, sp = core.system_for(w, model=model, cap=128, s_cap=256)
    out = sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    bits, _, rc = sy.status(raise_on_error=False)
    n_s = int(out["n_exp"][0].item())
    assert bits & B.STATUS_S_OVERFLOW, bits
    assert rc == E_WORKSPACE, rc
    assert n_s > 256, n_s
    assert torch.isfinite(out["forces"]).all()

    res = []
    for s_cap in (n_s, 0):
        _, sy2, pos2, sp2 = core.system_for(w, model=model, cap=128, s_cap=s_cap)
        out2 = sy2.compute(pos2, sp2, r_buffer=w["r_buffer"], force_rebuild=True)
        bits2, _, rc2 = sy2.status(raise_on_error=False)
        assert bits2 == 0 and rc2 == 0, (s_cap, bits2, rc2)
        assert int(out2["n_exp"][0].item()) == n_s
        res.append(out2["forces"].cpu().numpy().copy())
    assert np.array_equal(res[0], res[1])
