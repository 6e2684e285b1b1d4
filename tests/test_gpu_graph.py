"""A velocity-Verlet step captured once in a HIP graph and replayed gives the
same bits as the same step launched eagerly, replay after replay, with other
eager work and synchronisations in between."""
import numpy as np
import pytest

from gen import workloads as W

pytestmark = pytest.mark.gpu


def _setup(w, model):
    import torch
    from paper_2502_19081_amd import core
    _, sy, pos, sp = core.system_for(w, model=model, cap=128)
    vel = torch.from_numpy(np.ascontiguousarray(w["vel"].T)).cuda()
    mass = torch.from_numpy(w["masses"][w["species"]]).cuda()
    sy.compute(pos, sp, r_buffer=w["r_buffer"], force_rebuild=True)
    return sy, pos, vel, mass, sp


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_replay_matches_eager(precision):
    import torch
    from paper_2502_19081_amd import core
    w = W.c4_replica(1, n_target=2000)
    print(f"case graph replay c4 replica n={len(w['pos'])} {precision}", flush=True)
    model = core.Model(w["model"], precision=precision)
    dt = 0.2
    steps = 6
    # eager reference trajectory
    sy, pos, vel, mass, sp = _setup(w, model)
    eager = []
    for _ in range(steps):
        sy.vv_step(pos, vel, mass, sp, dt, r_buffer=w["r_buffer"], force_rebuild=True)
        torch.cuda.synchronize()
        eager.append((pos.cpu().numpy().copy(), sy.forces.cpu().numpy().copy(),
                      sy.energies.cpu().numpy().copy()))
    sy.status()
    # graph: capture one step, replay
    sy2, pos2, vel2, mass2, sp2 = _setup(w, model)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        # the captured step must not run during capture: keep a copy of the
        # state and restore it after capture
        p0, v0, f0 = pos2.clone(), vel2.clone(), sy2.forces.clone()
        with torch.cuda.graph(g, stream=s):
            sy2.vv_step(pos2, vel2, mass2, sp2, dt, r_buffer=w["r_buffer"], force_rebuild=True)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    pos2.copy_(p0)
    vel2.copy_(v0)
    sy2.forces.copy_(f0)
    other = _setup(W.tiny(seed=3), core.Model(W.tiny(seed=3)["model"], precision="fp64"))
    for k in range(steps):
        g.replay()
        torch.cuda.synchronize()
        # unrelated eager work between replays
        other[0].compute(other[1], other[4], r_buffer=2.5, force_rebuild=True)
        torch.cuda.synchronize()
        assert np.array_equal(pos2.cpu().numpy(), eager[k][0]), k
        assert np.array_equal(sy2.forces.cpu().numpy(), eager[k][1]), k
        assert np.array_equal(sy2.energies.cpu().numpy(), eager[k][2]), k
    sy2.status()


def test_graph_replay_with_thermostat_matches_eager():
    # the cheap-region thermostat inside a captured step: the step reads the
    # normals from the workspace's buffer, refilled before every replay
    import torch
    from paper_2502_19081_amd import core
    w = W.c4_replica(2, n_target=2000)
    n = len(w["pos"])
    print(f"case graph replay with the Langevin thermostat, c4 replica n={n} fp64", flush=True)
    model = core.Model(w["model"], precision="fp64")
    dt, steps = 0.2, 5
    xi = [torch.from_numpy(np.random.default_rng(k).normal(size=(3, n))).cuda() for k in range(steps)]
    sy, pos, vel, mass, sp = _setup(w, model)
    sy.set_langevin(800.0, 50.0)
    eager = []
    for k in range(steps):
        sy.vv_step(pos, vel, mass, sp, dt, r_buffer=w["r_buffer"], force_rebuild=True, xi=xi[k])
        torch.cuda.synchronize()
        eager.append((pos.cpu().numpy().copy(), vel.cpu().numpy().copy()))
    sy.status()
    sy2, pos2, vel2, mass2, sp2 = _setup(w, model)
    sy2.set_langevin(800.0, 50.0)
    feed = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p0, v0, f0 = pos2.clone(), vel2.clone(), sy2.forces.clone()
        with torch.cuda.graph(g, stream=s):
            sy2.vv_step(pos2, vel2, mass2, sp2, dt, r_buffer=w["r_buffer"], force_rebuild=True,
                        xi=feed)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    pos2.copy_(p0)
    vel2.copy_(v0)
    sy2.forces.copy_(f0)
    for k in range(steps):
        feed.copy_(xi[k])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(pos2.cpu().numpy(), eager[k][0]), k
        assert np.array_equal(vel2.cpu().numpy(), eager[k][1]), k
    sy2.status()
    # the thermostat acted: the trajectory differs from plain NVE
    sy3, pos3, vel3, mass3, sp3 = _setup(w, model)
    for k in range(steps):
        sy3.vv_step(pos3, vel3, mass3, sp3, dt, r_buffer=w["r_buffer"], force_rebuild=True)
    assert not np.array_equal(vel3.cpu().numpy(), eager[-1][1])
