"""FP64 velocity Verlet on the device: trajectory parity with the oracle's
integrator, time reversal, and the 1,000-step NVE run of the 54,000-atom
screw-dislocation column (pure-potential drift asserted, mixed drift
reported)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from gen import workloads as W

pytestmark = pytest.mark.gpu


def _setup(w, precision, cap=128):
    import torch
    from paper_2502_19081_amd import core
    model = core.Model(w["model"], precision=precision)
    _, sy, pos, sp = core.system_for(w, model=model, cap=cap)
    vel = torch.from_numpy(np.ascontiguousarray(w["vel"].T)).cuda()
    mass = torch.from_numpy(w["masses"][w["species"]]).cuda()
    return model, sy, pos, vel, mass, sp


def test_vv_trajectory_matches_oracle():
    import torch
    w = W.tiny(seed=31, n_species=2, sigma=0.05)
    w["vel"] = w["vel"] * 4.0
    print("case tiny VV parity, 10 steps FP64 mixed", flush=True)
    _, sy, pos, vel, mass, sp = _setup(w, "fp64")
    sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    for _ in range(10):
        sy.vv_step(pos, vel, mass, sp, 1.0, r_buffer=w["r_buffer"])
    sy.status()
    p_ref, v_ref, out = O.velocity_verlet(w, w["pos"], w["vel"], 1.0, 10)
    p = pos.cpu().numpy().T
    d = p - p_ref
    d -= w["L"] * np.round(d / w["L"])
    assert np.abs(d).max() < 1e-10
    assert np.abs(vel.cpu().numpy().T - v_ref).max() < 1e-10
    assert np.abs(sy.forces.cpu().numpy().T - out["forces"]).max() < 1e-9


def test_time_reversal_on_device():
    import torch
    w = W.c4_replica(2, n_target=2000)
    print("case c4 replica time reversal FP64, 200 + 200 steps", flush=True)
    _, sy, pos, vel, mass, sp = _setup(w, "fp64")
    p0 = pos.clone()
    v0 = vel.clone()
    sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    for _ in range(200):
        sy.vv_step(pos, vel, mass, sp, 0.2, r_buffer=w["r_buffer"], mode=2)
    vel.mul_(-1.0)
    for _ in range(200):
        sy.vv_step(pos, vel, mass, sp, 0.2, r_buffer=w["r_buffer"], mode=2)
    sy.status()
    d = (pos - p0).cpu().numpy().T
    d -= w["L"] * np.round(d / w["L"])
    assert np.abs(d).max() < 1e-8
    # the 10-80 eV He impact is chaotic: rounding grows over the 400 steps, so
    # velocities are bounded relative to the largest speed
    vmax = np.abs(v0.cpu().numpy()).max()
    assert np.abs((vel + v0).cpu().numpy()).max() < 1e-5 * vmax


def test_c3_nve_1000_steps():
    import torch
    from paper_2502_19081_amd import md
    w = W.c3()
    n = len(w["pos"])
    res = {}
    for name, mode, prec in (("all_cheap", 2, "fp64"), ("all_expensive", 1, "fp32"), ("mixed", 0, "fp32")):
        print(f"case c3 NVE 1000 steps dt 1 fs {name} {prec}", flush=True)
        model, sy, pos, vel, mass, sp = _setup(w, prec)
        snap = md.expensive_snapshot(model, w) if name == "mixed" else None
        rec = md.run_nve(sy, pos, vel, mass, sp, 1.0, 1000, r_buffer=w["r_buffer"], mode=mode,
                         every=100, snapshot=snap)
        rec = np.array(rec)
        if name == "all_cheap":
            etot = rec[:, 2] + rec[:, 3]
        elif name == "all_expensive":
            etot = rec[:, 1] + rec[:, 3]
        else:
            etot = rec[:, 4] + rec[:, 3]
        drift = (etot - etot[0]) / n
        temp = rec[:, 3] / (1.5 * n * 8.617333262e-5)
        res[name] = {"precision": prec, "energy_per_atom_drift_eV": drift.tolist(),
                     "temperature_K": temp.tolist(), "steps": rec[:, 0].tolist()}
        print(f"  max |dE|/N = {np.abs(drift).max():.3e} eV/atom, T {temp[0]:.0f} -> {temp[-1]:.0f} K",
              flush=True)
        if name != "mixed":
            assert np.abs(drift).max() < 2e-4
    from conftest import RESULTS_DIR
    os.makedirs(RESULTS_DIR, exist_ok=True)
    with open(os.path.join(RESULTS_DIR, "c3_nve_drift.json"), "w") as f:
        json.dump(res, f)


def test_vv_trajectory_seeded_matches_oracle():
    # seeded region (cubic blend) through 10 MD steps: the seed bits travel in
    # the flags array and the region follows the moving atoms
    import torch
    w = W.tiny(seed=33, n_species=2, sigma=0.05)
    w["vel"] = w["vel"] * 4.0
    seeds = np.zeros(len(w["pos"]), bool)
    seeds[[5, 40]] = True
    w["seeds"] = seeds
    w["regions"] = [W.seeded(2.9, 3.2, blend=1)]
    print("case tiny VV parity with a seeded region, 10 steps FP64 mixed", flush=True)
    _, sy, pos, vel, mass, sp = _setup(w, "fp64")
    sy.set_seeds(torch.from_numpy(seeds.astype(np.uint8)))
    sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    for _ in range(10):
        sy.vv_step(pos, vel, mass, sp, 1.0, r_buffer=w["r_buffer"])
    sy.status()
    p_ref, v_ref, out = O.velocity_verlet(w, w["pos"], w["vel"], 1.0, 10)
    p = pos.cpu().numpy().T
    d = p - p_ref
    d -= w["L"] * np.round(d / w["L"])
    assert np.abs(d).max() < 1e-10
    assert np.abs(vel.cpu().numpy().T - v_ref).max() < 1e-10
    # positions agree to rounding after 10 steps, so lambda to the same order
    assert np.abs(sy.lam.cpu().numpy() - out["lam"]).max() < 1e-9
    assert np.array_equal(sy.flags.cpu().numpy() & 0x7F, out["flags"])



def test_vv_langevin_cheap_region_matches_oracle():
    # thermostat on the lambda == 0 atoms, same normals on both sides
    import torch
    w = W.tiny(seed=35, n_species=2, sigma=0.05)
    w["vel"] = w["vel"] * 3.0
    n = len(w["pos"])
    T, tau, steps = 600.0, 20.0, 10
    xi = np.random.default_rng(11).normal(size=(steps, n, 3))
    print("case tiny VV parity with the cheap-region Langevin thermostat, 10 steps FP64",
          flush=True)
    _, sy, pos, vel, mass, sp = _setup(w, "fp64")
    sy.set_langevin(T, tau)
    sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    for k in range(steps):
        sy.vv_step(pos, vel, mass, sp, 1.0, r_buffer=w["r_buffer"],
                   xi=torch.from_numpy(np.ascontiguousarray(xi[k].T)).cuda())
    sy.status()
    p_ref, v_ref, out = O.velocity_verlet(w, w["pos"], w["vel"], 1.0, steps,
                                          langevin=(T, tau, xi))
    assert 0 < int((out["lam"] == 0.0).sum()) < n
    d = pos.cpu().numpy().T - p_ref
    d -= w["L"] * np.round(d / w["L"])
    assert np.abs(d).max() < 1e-10
    assert np.abs(vel.cpu().numpy().T - v_ref).max() < 1e-10
    assert np.abs(sy.forces.cpu().numpy().T - out["forces"]).max() < 1e-9


@pytest.mark.parametrize("case", ["off", "all_expensive"])
def test_langevin_without_cheap_atoms_is_nve(case):
    # a thermostat turned off again, or one in all-expensive mode (lambda = 1
    # everywhere), leaves the NVE trajectory bit for bit
    import torch
    w = W.tiny(seed=37, n_species=2, sigma=0.05)
    mode = 1 if case == "all_expensive" else 0
    print(f"case tiny VV with thermostat {case}, 5 steps FP64", flush=True)
    res = []
    for thermo in (False, True):
        _, sy, pos, vel, mass, sp = _setup(w, "fp64")
        if thermo:
            sy.set_langevin(300.0, 10.0)
            if case == "off":
                sy.set_langevin(300.0, 0.0)
        sy.compute(pos, sp, r_buffer=w["r_buffer"], mode=mode, force_rebuild=True)
        for _ in range(5):
            sy.vv_step(pos, vel, mass, sp, 1.0, r_buffer=w["r_buffer"], mode=mode)
        sy.status()
        res.append((pos.cpu().numpy(), vel.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("case", ["c2_fp32_rebuild", "tiny_fp64_skin", "tiny_seeded_cubic",
                                  "tiny_cheap_masked"])
def test_fused_steps_equal_single_steps(case):
    # n steps in one call (gather fused with the next opening kick and drift,
    # energy sums in the next binning kernel) = n single steps, bit for bit
    import torch
    masked = False
    seeds = None
    if case == "c2_fp32_rebuild":
        w = W.c2()
        vel0 = W.maxwell(np.random.default_rng(5), w["species"], 300.0)
        prec, rebuild, dt, steps = "fp32", True, 1.0, 6
    else:
        w = W.tiny(seed=41, n_species=2, sigma=0.05, cells=6 if case == "tiny_cheap_masked" else 3)
        vel0 = w["vel"] * 4.0
        prec, rebuild, dt, steps = "fp64", False, 1.0, 7
        if case == "tiny_seeded_cubic":
            seeds = np.zeros(len(w["pos"]), bool)
            seeds[[3, 30]] = True
            w = dict(w, regions=[W.seeded(2.9, 3.2, blend=1)])
        if case == "tiny_cheap_masked":
            masked = True
            w = dict(w, regions=[W.sphere(w["L"] / 2.0, 3.5, 1.5)], r_buffer=3.0)
    w = dict(w, vel=vel0)
    print(f"case fused multi-step VV {case}, {steps} steps", flush=True)
    res = []
    for fused in (False, True):
        _, sy, pos, vel, mass, sp = _setup(w, prec)
        if seeds is not None:
            sy.set_seeds(torch.from_numpy(seeds.astype(np.uint8)))
        sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True, cheap_masked=masked)
        if fused:
            en = sy.vv_steps(pos, vel, mass, sp, dt, steps, r_buffer=w["r_buffer"],
                             force_rebuild=rebuild, cheap_masked=masked).cpu().numpy()
        else:
            en = []
            for _ in range(steps):
                sy.vv_step(pos, vel, mass, sp, dt, r_buffer=w["r_buffer"], force_rebuild=rebuild,
                           cheap_masked=masked)
                en.append(sy.energies.cpu().numpy().copy())
            en = np.array(en)
        sy.status()
        res.append((pos.cpu().numpy(), vel.cpu().numpy(), sy.forces.cpu().numpy(), en,
                    sy.lam.cpu().numpy()))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_fused_steps_in_a_graph():
    # the fused call captured once and replayed = the same call launched eagerly
    import torch
    w = W.c4_replica(1, n_target=2000)
    print("case fused multi-step VV captured in a graph, c4 replica, 3 steps x 4 replays",
          flush=True)
    dt, steps = 0.2, 3
    _, sy, pos, vel, mass, sp = _setup(w, "fp32")
    sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    eager = []
    for _ in range(4):
        en = sy.vv_steps(pos, vel, mass, sp, dt, steps, r_buffer=w["r_buffer"], force_rebuild=True)
        torch.cuda.synchronize()
        eager.append((pos.cpu().numpy().copy(), en.cpu().numpy().copy()))
    _, sy2, pos2, vel2, mass2, sp2 = _setup(w, "fp32")
    sy2.compute(pos2, sp2, r_buffer=w["r_buffer"], force_rebuild=True)
    en2 = torch.zeros(steps, 3, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    p0, v0, f0 = pos2.clone(), vel2.clone(), sy2.forces.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            sy2.vv_steps(pos2, vel2, mass2, sp2, dt, steps, r_buffer=w["r_buffer"],
                         force_rebuild=True, energies=en2)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    pos2.copy_(p0)
    vel2.copy_(v0)
    sy2.forces.copy_(f0)
    for k in range(4):
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(pos2.cpu().numpy(), eager[k][0]), k
        assert np.array_equal(en2.cpu().numpy(), eager[k][1]), k
    sy2.status()
