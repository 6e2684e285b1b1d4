"""Continuous batching of He-impact replicas: a replica gives the same bits
alone and in a changing mix; admission respects the HBM budget; a replica
with a non-finite position is evicted alone.

Each test runs in the tick modes of the server: one multi-stream HIP graph
per batch composition ("graph"), eager launches of every replica's step on
its own stream ("eager"), and one graph per replica captured at admission,
the active replicas' graphs launched each on its own stream
("replica_graphs"). The batch-graph mode is skipped: its capture end and
a later replay crashed in the host runtime (segmentation fault, no GPU fault
reported) after the library began to fork work onto a second stream; the
cause has not been shown, so the mode stays off until it is.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GRAPH_SKIP = pytest.mark.skip(
    reason="multi-replica graph capture/replay crashed in the host runtime (SIGSEGV in capture "
           "end, then in replay); cause not shown yet, so this mode stays off the GPU")
MODES = [pytest.param(True, id="graph", marks=GRAPH_SKIP), pytest.param(False, id="eager"),
         pytest.param("replica", id="replica_graphs")]


def _model():
    from gen import workloads as W
    from paper_2502_19081_amd import core
    return core.Model(W.c4_model(), precision="fp32")


def _rep(k, steps, arrival, n_target):
    from gen import workloads as W
    from paper_2502_19081_amd.serve import Replica
    return Replica(k, W.c4_replica(k, n_target=n_target), steps, 0.2, arrival)


@pytest.mark.parametrize("use_graph", MODES)
def test_alone_equals_in_mix(use_graph):
    from paper_2502_19081_amd.serve import Server
    model = _model()
    print(f"case serving alone vs mix (c4 replicas, 40 steps, graph={use_graph})", flush=True)
    alone = Server(model, max_slots=4, use_graph=use_graph)
    a = _rep(5, 40, 0.0, 3000)
    alone.submit(a)
    alone.run(clock=lambda: 0.0)
    mix = Server(model, max_slots=3, use_graph=use_graph)

    def clock():  # arrivals in tick units: the mix changes while replica 5 runs
        return float(len(mix.ticks))
    b = _rep(5, 40, 0.0, 3000)
    others = [_rep(1, 25, 0.0, 2000), _rep(2, 30, 5.0, 4500), _rep(3, 10, 12.0, 2500),
              _rep(4, 20, 20.0, 6000)]
    for r in [b] + others:
        mix.submit(r)
    mix.run(clock=clock)
    if use_graph:
        assert mix.recaptures >= 3
    assert max(n for n, _ in mix.ticks) == 3
    assert a.error is None and b.error is None
    for key in ("pos", "vel", "energies"):
        assert np.array_equal(a.result[key], b.result[key]), key


@pytest.mark.parametrize("use_graph", MODES)
def test_admission_by_hbm_budget(use_graph):
    from paper_2502_19081_amd.serve import Server
    model = _model()
    print(f"case serving admission by HBM budget (graph={use_graph})", flush=True)
    reps = [_rep(k, 5, 0.0, 2000) for k in range(6)]
    fp = max(r.footprint(model, 128) for r in reps)
    srv = Server(model, hbm_budget=int(2.5 * fp), max_slots=8, use_graph=use_graph)
    for r in reps:
        srv.submit(r)
    srv.run(clock=lambda: 0.0)
    assert len(srv.finished) == 6
    assert max(n for n, _ in srv.ticks) == 2


@pytest.mark.parametrize("use_graph", MODES)
def test_nonfinite_replica_is_evicted_alone(use_graph):
    from paper_2502_19081_amd.serve import Server
    model = _model()
    print(f"case serving eviction of a non-finite replica (graph={use_graph})", flush=True)
    srv = Server(model, max_slots=4, check_every=2, use_graph=use_graph)
    good = [_rep(k, 8, 0.0, 2000) for k in (7, 8)]
    bad = _rep(9, 8, 0.0, 2000)
    bad.w = dict(bad.w)
    p = bad.w["pos"].copy()
    p[10, 0] = np.nan
    bad.w["pos"] = p
    for r in good + [bad]:
        srv.submit(r)
    srv.run(clock=lambda: 0.0)
    assert [r.rid for r in srv.failed] == [9]
    assert sorted(r.rid for r in srv.finished) == [7, 8]
    assert all(r.error is None for r in srv.finished)


def test_replica_graphs_equal_eager_steps():
    # a replica served through its captured step gives the bits of the same
    # replica served with eager launches, beside another replica in both runs
    from paper_2502_19081_amd.serve import Server
    model = _model()
    print("case serving per-replica graphs vs eager (c4 replicas, 30 steps)", flush=True)
    out = {}
    for mode in (False, "replica"):
        srv = Server(model, max_slots=2, use_graph=mode)
        reps = [_rep(6, 30, 0.0, 3500), _rep(2, 20, 0.0, 2200)]
        for r in reps:
            srv.submit(r)
        srv.run(clock=lambda: 0.0)
        assert all(r.error is None for r in srv.finished)
        out[mode] = {r.rid: r.result for r in srv.finished}
        if mode == "replica":
            assert srv.recaptures == 2
    for rid in (6, 2):
        for key in ("pos", "vel", "energies"):
            assert np.array_equal(out[False][rid][key], out["replica"][rid][key]), (rid, key)


# ------------------------------------------------------------ batched server

def _tick_clock(srv):
    # arrivals in units of batch steps: the mix changes at known steps
    return lambda: float(srv._ticks_total)


def test_batch_server_alone_equals_in_changing_mix():
    from paper_2502_19081_amd.serve import BatchServer
    model = _model()
    print("case batched serving: a replica alone vs in a changing mix (bitwise)", flush=True)
    res = {}
    for name in ("alone", "mix"):
        srv = BatchServer(model, admit_every=4, check_every=7)
        reps = [_rep(5, 40, 0.0, 2500)]
        if name == "mix":
            reps += [_rep(1, 10, 0.0, 2000), _rep(2, 20, 5.0, 3000), _rep(3, 15, 12.0, 2200),
                     _rep(4, 6, 30.0, 2100)]
        for r in reps:
            srv.submit(r)
        srv.run(clock=_tick_clock(srv))
        assert not srv.failed and all(r.done == r.steps for r in srv.finished)
        a = [r for r in srv.finished if r.rid == 5][0]
        res[name] = a.result
        if name == "mix":
            assert srv.rebuilds >= 5
            rep = srv.report()
            assert rep["max_batch"] >= 3 and rep["replicas"] == 5
    for key in ("pos", "vel", "energies", "n_exp"):
        assert np.array_equal(res["alone"][key], res["mix"][key]), key


def test_batch_server_graph_equals_eager_and_admission_by_budget():
    from paper_2502_19081_amd.serve import BatchServer
    model = _model()
    print("case batched serving: graph = eager, HBM budget of 2.5 replicas", flush=True)
    out = {}
    for use_graph in (False, True):
        probe = BatchServer(model)
        fp = max(probe.footprint(_rep(k, 1, 0.0, 2000)) for k in range(4))
        srv = BatchServer(model, hbm_budget=int(2.5 * fp), use_graph=use_graph, admit_every=3)
        for k in range(4):
            srv.submit(_rep(k, 12 + 3 * k, 0.0, 2000))
        srv.run(clock=_tick_clock(srv))
        rep = srv.report()
        assert rep["replicas"] == 4 and rep["max_batch"] <= 2
        assert srv.peak_in_use <= srv.budget
        out[use_graph] = {r.rid: r.result for r in srv.finished}
    for rid in range(4):
        for key in ("pos", "vel", "energies"):
            assert np.array_equal(out[False][rid][key], out[True][rid][key]), (rid, key)


def test_batch_server_evicts_nonfinite_replica_alone():
    from paper_2502_19081_amd.serve import BatchServer
    model = _model()
    print("case batched serving: eviction of a non-finite replica", flush=True)
    srv = BatchServer(model, check_every=3)
    good = [_rep(k, 8, 0.0, 2000) for k in (7, 8)]
    bad = _rep(9, 8, 0.0, 2000)
    bad.w = dict(bad.w)
    p = bad.w["pos"].copy()
    p[10, 0] = np.nan
    bad.w["pos"] = p
    for r in good + [bad]:
        srv.submit(r)
    srv.run(clock=lambda: 0.0)
    assert [r.rid for r in srv.failed] == [9]
    assert sorted(r.rid for r in srv.finished) == [7, 8]
    for r in srv.finished:
        assert np.isfinite(r.result["pos"]).all()
