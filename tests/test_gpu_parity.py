"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: neighbour rows, lambda, masks and the compacted index sets S and M are
bit-exact; FP64 forces agree to 1e-10 relative to the largest reference
force; FP32 forces to 1e-4 eV/A absolute; site energies to the same bounds.
"""
import numpy as np
import pytest

import oracle as O
from gen import workloads as W
from tests.gpu_common import run_gpu, assert_neighbors_equal, rel_force_err

pytestmark = pytest.mark.gpu

MODES = {"mixed": O.MODE_MIXED, "all_expensive": O.MODE_ALL_EXPENSIVE, "all_cheap": O.MODE_ALL_CHEAP}


def _check(w, mode, precision, ref=None, f_tol=None, cheap_masked=False):
    print(f"case {w['name']} seed={w['seed']} n={len(w['pos'])} mode={mode} prec={precision}"
          f"{' cheap masked' if cheap_masked else ''}", flush=True)
    ref = ref or O.mixed(w, MODES[mode], cheap_masked=cheap_masked)
    g = run_gpu(w, MODES[mode], precision=precision, cheap_masked=cheap_masked)
    assert_neighbors_equal(g, ref)
    assert np.array_equal(g["lam"], ref["lam"])
    # bit 7 is the seed marker the caller passes in (kept by the library)
    assert np.array_equal(g["flags"] & 0x7F, ref["flags"])
    assert np.array_equal(g["S"], ref["S"])
    assert np.array_equal(g["M"], ref["M"])
    assert g["n_exp"].tolist() == [len(ref["S"]), len(ref["M"])]
    if precision == "fp64":
        for key, rk in (("forces", "forces"), ("f_exp", "f_exp"), ("f_cheap", "f_cheap")):
            if np.abs(ref[rk]).max() > 0:
                assert rel_force_err(g[key], ref[rk]) < 1e-10, key
            else:
                assert np.abs(g[key]).max() == 0
        scale = max(1.0, np.abs(ref["e_exp"]).max(), np.abs(ref["e_cheap"]).max())
        assert np.abs(g["e_exp"] - ref["e_exp"]).max() < 1e-10 * scale
        assert np.abs(g["e_cheap"] - ref["e_cheap"]).max() < 1e-10 * scale
    else:
        tol = f_tol or 1e-4
        err = np.abs(g["forces"] - ref["forces"]).max()
        print(f"  fp32 max |dF| = {err:.3e} eV/A", flush=True)
        assert err < tol
        assert np.abs(g["e_exp"] - ref["e_exp"]).max() < 1e-3
        assert np.abs(g["e_cheap"] - ref["e_cheap"]).max() < 1e-3
    # atoms outside S carry no expensive force or energy
    outside = np.ones(len(w["pos"]), bool)
    outside[ref["S"]] = False
    assert np.all(g["f_exp"][outside] == 0) and np.all(g["e_exp"][outside] == 0)
    return g, ref


@pytest.mark.parametrize("mode", ["mixed", "all_expensive", "all_cheap"])
def test_c1_fp64(mode):
    _check(W.c1(), mode, "fp64")


@pytest.mark.parametrize("seed", [1, 2])
def test_tiny_two_species_order3_fp64(seed):
    w = W.tiny(seed=seed, n_species=2)
    _check(w, "mixed", "fp64")
    _check(w, "all_expensive", "fp64")


def test_tiny_nonperiodic_cylinder_fp64():
    w = W.tiny(seed=4, periodic=(1, 0, 0), vacuum=4.0, n_species=2)
    w["regions"] = [W.cylinder(w["L"] / 2, 0, 2.0, 1.5), W.sphere(None, 1.5, 1.0, follow_atom=3)]
    w["regions"][1]["center"] = np.zeros(3)
    _check(w, "mixed", "fp64")


@pytest.mark.parametrize("scale,rcut3,sigma", [(1.15, 3.2, 0.3), (0.8, 4.0, 0.3), (0.82, 4.2, 0.35)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_three_body_leg_counts(scale, rcut3, sigma, precision):
    """Strongly jittered bcc cells, stretched or compressed, with the 3-body
    cutoff set so that the per-atom counts of 3-body legs span 1-8 (stretched)
    or the mid twenties to about forty (compressed): the cheap kernel's two
    layouts of the leg pairs (offset blocks, and 64 pairs per round for the
    counts where blocks would take more rounds), including blocks that hold
    no pair, all carry atoms."""
    w = W.tiny(seed=7, n_species=2, cells=4, sigma=sigma)
    w["pos"] = w["pos"] * scale
    w["L"] = w["L"] * scale
    w["model"]["uf3"]["rcut3"] = rcut3
    d = w["pos"][None, :, :] - w["pos"][:, None, :]
    d -= w["L"] * np.round(d / w["L"])
    r2 = (d ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    n3 = (r2 < rcut3 ** 2).sum(1)
    s = 64 // np.maximum(n3, 1)
    blocks = -(-(n3 // 2) // s) <= -(-(n3 * (n3 // 2)) // 64)
    print(f"  legs {n3.min()}..{n3.max()}, {blocks.sum()} atoms in blocks, "
          f"{(~blocks).sum()} cyclic", flush=True)
    assert n3.max() <= 64
    if scale > 1:
        assert n3.min() <= 2 and n3.max() <= 8
    else:
        assert blocks.any() and (~blocks).any()
    _check(w, "all_cheap", precision)


def test_c2_fp32_mixed():
    _check(W.c2(), "mixed", "fp32")


def test_c2_fp64_mixed():
    _check(W.c2(), "mixed", "fp64")


def test_c2_fp32_all_expensive():
    _check(W.c2(), "all_expensive", "fp32")


@pytest.mark.parametrize("index,n_target", [(3, 2500), (5, 20000)])
def test_c4_replica_two_species_fp32(index, n_target):
    # the smallest and the largest replica size of the serving workload
    w = W.c4_replica(index, n_target=n_target)
    _check(w, "mixed", "fp32")


def test_repeat_is_bitwise_and_rebuild_decision():
    # deterministic accumulation: a second call (list reused, no rebuild)
    # reproduces the first bit for bit
    w = W.c2()
    g1 = run_gpu(w, 0, precision="fp32")
    sy, pos, sp = g1["system"]
    g2 = run_gpu(w, 0, precision="fp32", system=(sy, pos, sp), force_rebuild=False)
    assert np.array_equal(g1["forces"], g2["forces"])
    assert np.array_equal(g1["e_exp"], g2["e_exp"])


def test_buffer_paths_agree_with_oracle():
    # the buffer atoms come from the row kernel on a forced rebuild, from the
    # buffer pass when the list is kept, and from both when a displacement
    # triggers the rebuild: every path must give the oracle's masks and sets
    w = W.c2()
    print("case c2 buffer paths: forced, kept, displacement rebuild", flush=True)
    g1 = run_gpu(w, 0, precision="fp32")
    sy, pos, sp = g1["system"]
    g2 = run_gpu(w, 0, precision="fp32", system=(sy, pos, sp), force_rebuild=False)
    ref = O.mixed(w, O.MODE_MIXED)
    for g in (g1, g2):
        assert np.array_equal(g["flags"], ref["flags"])
        assert np.array_equal(g["S"], ref["S"])
        assert np.array_equal(g["M"], ref["M"])
    # move a few atoms by more than half the skin: the list is rebuilt
    import torch
    w3 = dict(w)
    p3 = w["pos"].copy()
    p3[::97] += 0.6
    p3 = W.wrap(p3, w["L"], w["periodic"])
    w3["pos"] = p3
    pos.copy_(torch.from_numpy(np.ascontiguousarray(p3.T)).to(pos.device))
    g3 = run_gpu(w3, 0, precision="fp32", system=(sy, pos, sp), force_rebuild=False)
    ref3 = O.mixed(w3, O.MODE_MIXED)
    assert_neighbors_equal(g3, ref3)
    assert np.array_equal(g3["flags"], ref3["flags"])
    assert np.array_equal(g3["S"], ref3["S"])
    assert np.array_equal(g3["M"], ref3["M"])



def test_basis_forms_agree():
    # the atomic basis of large systems (64-slot passes) and of small ones
    # (whole-row compaction) both match the oracle on the same cell
    import os
    w = W.c2()
    ref = O.mixed(w, O.MODE_MIXED)
    print("case c2 fp32: basis in 64-slot passes vs whole-row compaction", flush=True)
    os.environ["MLMIX_BASIS_CHUNKS"] = "1"
    try:
        g1 = run_gpu(w, 0, precision="fp32")
    finally:
        del os.environ["MLMIX_BASIS_CHUNKS"]
    g2 = run_gpu(w, 0, precision="fp32")
    for g in (g1, g2):
        assert np.abs(g["forces"] - ref["forces"]).max() < 1e-4
        assert np.abs(g["e_exp"] - ref["e_exp"]).max() < 1e-3


def _seeded_tiny(seed, blend):
    w = W.tiny(seed=seed, n_species=2)
    rng = np.random.default_rng(seed)
    seeds = np.zeros(len(w["pos"]), bool)
    seeds[rng.choice(len(seeds), 2, replace=False)] = True
    w["seeds"] = seeds
    w["regions"] = [W.seeded(2.9, 3.2, blend=blend), W.sphere(w["L"] / 4.0, 1.0, 1.5, blend=1)]
    return w


@pytest.mark.parametrize("blend", [0, 1])
def test_tiny_seeded_regions_fp64(blend):
    # the paper's seeded region fix (core around seed atoms, blend to the
    # nearest core atom; linear or cubic) beside a cubic geometric sphere
    _check(_seeded_tiny(21 + blend, blend), "mixed", "fp64")


def test_c2_seeded_region_fp32():
    w = W.c2()
    c = w["regions"][0]["center"]
    d = w["pos"] - c
    d -= w["L"] * np.round(d / w["L"])
    r = np.linalg.norm(d, axis=1)
    w["seeds"] = r < 2.0  # the atoms of the self-interstitial
    w["regions"] = [W.seeded(3.0, 5.0, blend=1)]
    g, ref = _check(w, "mixed", "fp32")
    assert 0 < len(ref["M"]) < len(w["pos"]) and np.array_equal(g["lam"], ref["lam"])


def test_tiny_cheap_masked_fp64():
    # Algorithm 4 for the cheap potential too: S_c = {lambda < 1} plus its
    # buffer (flags bit3); the core's central atom lies outside S_c
    w = W.tiny(seed=17, cells=6)
    w["regions"] = [W.sphere(w["L"] / 2.0, 3.5, 1.5)]
    w["r_buffer"] = 3.0
    g, ref = _check(w, "mixed", "fp64", cheap_masked=True)
    assert ((ref["flags"] & 8) != 0).any()
    in_Sc = (ref["lam"] < 1.0) | ((ref["flags"] & 8) != 0)
    assert not in_Sc.all() and np.all(g["e_cheap"][~in_Sc] == 0.0)


def test_c2_cheap_masked_fp32():
    _check(W.c2(), "mixed", "fp32", cheap_masked=True)



# ------------------------------------------------------- degenerate cases

def test_no_region_is_the_cheap_potential():
    # mixed mode without regions: lambda = 0, S empty (every expensive launch
    # sees |S| = 0), forces = the cheap forces exactly
    w = dict(W.tiny(seed=51, n_species=2, sigma=0.05), regions=[])
    g, ref = _check(w, "mixed", "fp64")
    assert len(ref["S"]) == 0 and np.all(g["lam"] == 0.0)
    cheap = O.mixed(w, O.MODE_ALL_CHEAP)
    assert rel_force_err(g["forces"], cheap["forces"]) < 1e-10


def test_region_covering_everything_is_the_expensive_potential():
    # a core sphere larger than the cell: lambda = 1 everywhere, forces = the
    # all-expensive forces
    w = W.tiny(seed=53, n_species=1, sigma=0.05)
    w = dict(w, regions=[W.sphere(w["L"] / 2.0, 100.0, 0.0)])
    g, ref = _check(w, "mixed", "fp64")
    assert np.all(g["lam"] == 1.0)
    full = O.mixed(w, O.MODE_ALL_EXPENSIVE)
    assert rel_force_err(g["forces"], full["forces"]) < 1e-10


def test_neighbour_overflow_is_reported_and_regrowth_recovers():
    import torch
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    w = W.c1()
    print("case c1 with nbr_cap 32 (rows hold 58): overflow, then the required capacity",
          flush=True)
    model = core.Model(w["model"], precision="fp64")
    _, sy, pos, sp = core.system_for(w, model=model, cap=32)
    sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    bits, req, rc = sy.status(raise_on_error=False)
    assert rc == -4 and bits & B.STATUS_NEIGH_OVERFLOW and req >= 58
    ref = O.mixed(w)
    assert req == int(np.diff(ref["offs"]).max())
    g = run_gpu(w, O.MODE_MIXED, precision="fp64", cap=req)
    assert rel_force_err(g["forces"], ref["forces"]) < 1e-10


def test_atom_outside_a_nonperiodic_box_is_reported():
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    w = W.tiny(seed=55, periodic=(0, 0, 0), vacuum=4.0, sigma=0.05)
    pos = w["pos"].copy()
    pos[3, 2] = w["L"][2] + 0.5   # beyond the box's upper z face
    w = dict(w, pos=pos)
    print("case non-periodic cell with one atom outside the box", flush=True)
    model = core.Model(w["model"], precision="fp64")
    _, sy, p, sp = core.system_for(w, model=model)
    sy.compute(p, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    bits, _, rc = sy.status(raise_on_error=False)
    assert rc == -5 and bits & B.STATUS_OUT_OF_BOX


def test_empty_system():
    import torch
    from paper_2502_19081_amd import core
    w = W.tiny(seed=57)
    print("case zero atoms: compute and an MD step are no-ops", flush=True)
    model = core.Model(w["model"], precision="fp64")
    sy = core.System(model, 0, w["L"], w["periodic"])
    pos = torch.zeros(3, 0, dtype=torch.float64, device="cuda")
    sp = torch.zeros(0, dtype=torch.int32, device="cuda")
    out = sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    vel = torch.zeros(3, 0, dtype=torch.float64, device="cuda")
    mass = torch.zeros(0, dtype=torch.float64, device="cuda")
    sy.vv_step(pos, vel, mass, sp, 1.0, r_buffer=w["r_buffer"])
    sy.status()
    assert out["forces"].numel() == 0 and out["n_exp"].cpu().tolist() == [0, 0]


_BIG = {}


def _sampled_reference(name):
    """A workload at its full size with the oracle's forces on a seeded
    sample: atoms in the blend shells, inside the regions and far from them
    (lambda, masks and lists are computed for every atom)."""
    if name not in _BIG:
        w = {"c3": W.c3, "c5": W.c5}[name]()
        lam, _ = O.lambda_flags(O._f64(w["pos"]), w["L"], w["periodic"], w["regions"])
        r = np.random.default_rng(2025)
        shell = np.nonzero((lam > 0) & (lam < 1))[0]
        core_ = np.nonzero(lam == 1)[0]
        far = np.nonzero(lam == 0)[0]
        sample = np.unique(np.concatenate([r.choice(shell, 24, replace=False),
                                           r.choice(core_, 8, replace=False),
                                           r.choice(far, 32, replace=False)]))
        target = np.zeros(len(w["pos"]), bool)
        target[sample] = True
        _BIG[name] = (w, sample, O.mixed(w, O.MODE_MIXED, target=target))
    return _BIG[name]


@pytest.mark.parametrize("name,precision", [("c3", "fp32"), ("c3", "fp64"), ("c5", "fp32"),
                                            ("c5", "fp64")])
def test_full_size_sampled(name, precision):
    """The dislocation slab (54,000 atoms) and the largest workload
    (1,023,800 atoms) at their full sizes, in the launch shapes of their
    benchmarks (on c5: uncapped side passes, chunked basis, 16-channel
    contraction, slot-parallel reverse slots): lists, lambda, masks and S/M
    bit-exact for all atoms; forces against the oracle on the sample; and,
    for every atom, the property that holds at any size: each pair gradient
    enters the gather of both of its atoms with opposite signs, so the cheap
    forces of all atoms and the expensive forces of S sum to zero up to the
    FP64 rounding of the sums."""
    w, sample, ref = _sampled_reference(name)
    print(f"case {name} full n={len(w['pos'])} sample={len(sample)} prec={precision}", flush=True)
    g = run_gpu(w, O.MODE_MIXED, precision=precision)
    cap = g["nbr"].shape[1]
    valid = np.arange(cap)[None, :] < g["cnt"][:, None]
    assert np.array_equal(g["cnt"], np.diff(ref["offs"]).astype(np.int32))
    assert np.array_equal(g["nbr"][valid], ref["nbr"])
    assert np.array_equal(g["lam"], ref["lam"])
    assert np.array_equal(g["flags"] & 0x7F, ref["flags"])
    assert np.array_equal(g["S"], ref["S"]) and np.array_equal(g["M"], ref["M"])
    for key in ("forces", "f_exp", "f_cheap"):
        d = np.abs(g[key][sample] - ref[key][sample]).max()
        scale = np.abs(ref[key][sample]).max()
        print(f"  {key}: max |dF| on the sample = {d:.3e} eV/A (max |F| {scale:.3f})", flush=True)
        if precision == "fp64":
            assert d < 1e-10 * max(scale, 1e-300), key
        else:
            assert d < 1e-4, key
    for key in ("f_cheap", "f_exp"):
        net = np.abs(g[key].sum(axis=0)).max()
        print(f"  {key}: |sum over atoms| = {net:.3e} eV/A", flush=True)
        assert net < 1e-6, key
    outside = np.ones(len(w["pos"]), bool)
    outside[ref["S"]] = False
    assert np.all(g["f_exp"][outside] == 0) and np.all(g["e_exp"][outside] == 0)
