"""Benchmark of the mixed force evaluation on one MI355X.

One step = one velocity-Verlet MD step of the whole hot path on the device:
half kick + drift, neighbour-list rebuild (forced every step), lambda and
masks, buffer, compaction of S, expensive ACE-style forward + adjoint on S,
cheap UF3-style potential on every atom, gather + blend, half kick, FP64
energy sums. Inputs are resident in HBM before the timed region.

Prints ONE JSON line: mixed atom-steps/s (value), the all-expensive rate on
the same GPU and their ratio, the upper-bound speedup of the paper's cost
model, p50/p99 step latency, the force error against the FP64 CPU
reference, the roofline position of the dominant kernel and the CPU
baseline (the FP64 reference timed on this host).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_TFLOPS = 157.3
# the library is built without packed FP32 instructions: its FP32 vector code
# issues one FP32 FMA per lane per cycle, half the packed rate
FP32_VALU_UNPACKED_TFLOPS = 78.6
FP64_VALU_TFLOPS = 78.6
# dense matrix-core peaks (FP32 MFMA matches the FP32 vector peak)
MFMA_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "f32 (order-3 dense stage bf16)",
         "fp8": "f32 (order-3 dense stage fp8 e4m3)"}

WORKLOADS = {
    "c2": "c2: bcc W 16x16x16 cells + <111> dumbbell, 8193 atoms, sigma 0.08 A; "
          "ACE-style n_rad 12 lmax 4 order 3 rc 5.5; UF3-style 2-body 16 knots rc 5.5 + "
          "3-body 8x8x8 rc 3.5; sphere core 8 A + 2 A blend, buffer 5.5 A; FP32 potentials",
    "c1": "c1: bcc W 5x5x5 cells - vacancy, 249 atoms; ACE-style 8/3/2 rc 5; UF3 pair 12 knots; FP64",
    "c5": "c5: bcc W 80^3 cells - 200 vacancies, 1,023,800 atoms; ACE-style n_rad 16 lmax 5 "
          "order 3 rc 5.0; UF3-style 2-body 16 knots rc 5.5 + 3-body 6^3 rc 3.5; 200 spheres "
          "7 A core + 2 A blend at the vacancies, buffer 5 A",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only-mixed", action="store_true",
                    help="time the mixed step only (no all-expensive / all-cheap / latency runs); "
                         "used under a profiler so that every traced launch is a mixed-mode one")
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="consecutive MD steps captured in one HIP graph for the timed "
                         "region (1: one graph per step)")
    ap.add_argument("--seeded", action="store_true",
                    help="seeded region (the paper's fix: seeds at the defect, 6 A core, "
                         "2 A blend) instead of the workload's geometric regions")
    ap.add_argument("--cheap-masked", action="store_true",
                    help="the cheap potential on its own subsystem (lambda < 1 plus its "
                         "buffer) as Algorithm 4 masks each potential")
    ap.add_argument("--langevin", action="store_true",
                    help="Langevin thermostat (300 K, 2 ps) on the lambda == 0 atoms in every "
                         "step; the step's normals are drawn on the device inside the timed region")
    ap.add_argument("--dominant-only", action="store_true",
                    help="stop after timing the dominant kernel (phases 1-2) and print its "
                         "average; for a kernel trace of the same launches")
    ap.add_argument("--dominant", default=None,
                    help="take this stage as the dominant one instead of the largest in the "
                         "breakdown (for profiler runs)")
    ap.add_argument("--rebuild-every-step", action="store_true",
                    help="rebuild the neighbour list in every step of the timed runs instead of "
                         "keeping it while no atom has moved half the skin (the list policy of "
                         "the method; the other policy is timed too and reported beside it)")
    ap.add_argument("--single-stream", action="store_true",
                    help="keep every stage on the caller's stream (no fork of the cheap potential)")
    ap.add_argument("--fit", action="store_true",
                    help="the second workload instead: constrained linear fit of the cheap "
                         "potential to expensive-potential labels (thermal snapshots + strained "
                         "cells); prints its own JSON line")
    ap.add_argument("--fit-snapshots", type=int, default=20,
                    help="soft-constraint snapshots of the 2,000-atom cube for --fit")
    ap.add_argument("--probe", choices=["copy"], default=None,
                    help="copy: a plain 256 MiB device-to-device copy, 20 times (calibration of "
                         "the HBM byte counters)")
    return ap.parse_args()


def copy_probe():
    """A plain copy kernel of known size: reads and writes 256 MiB per launch."""
    import torch
    n = 64 << 20
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(20):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "copy", "bytes_read_per_launch": 4 * n,
                      "bytes_written_per_launch": 4 * n, "launches": 20}))


def measured_peaks():
    """Achievable peaks on this GPU: a 256 MiB device copy (bytes read plus
    written per second) and the FP32 matrix-core probe of the library."""
    import ctypes
    import torch
    from paper_2502_19081_amd import binding as B
    n = 64 << 20
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    hbm = 20 * 2 * 4 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
    sink = torch.zeros(2048, dtype=torch.float32, device="cuda")
    fl = ctypes.c_double()
    cur = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    B.check(B.lib().mlmix_probe_mfma_f32(cur, 2048, 256, ctypes.c_void_p(sink.data_ptr()),
                                         ctypes.byref(fl)))
    e0.record()
    B.check(B.lib().mlmix_probe_mfma_f32(cur, 2048, 4096, ctypes.c_void_p(sink.data_ptr()),
                                         ctypes.byref(fl)))
    e1.record()
    torch.cuda.synchronize()
    mfma = fl.value / (e0.elapsed_time(e1) * 1e-3) / 1e12
    return {"hbm_copy_GBps": hbm, "mfma_fp32_TFLOPs": mfma}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


KERNEL_SOURCES = {"ace_contract": ["paper_2502_19081_amd/csrc/o3.hip", "paper_2502_19081_amd/csrc/internal.h"],
                  "ace_pairgrad": ["paper_2502_19081_amd/csrc/ace.hip", "paper_2502_19081_amd/csrc/basis.h",
                                   "paper_2502_19081_amd/csrc/internal.h"],
                  "uf3": ["paper_2502_19081_amd/csrc/uf3.hip", "paper_2502_19081_amd/csrc/internal.h"]}


def measured_traffic(stage, cfg, prec):
    """HBM bytes per launch of a stage's kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy calibration),
    or None when there is none or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{stage}_{cfg}_{prec}_traffic.txt")
    if not os.path.exists(path) or stage not in KERNEL_SOURCES:
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[stage]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if kv.get("source_sha256") != h.hexdigest():
        return None
    return float(kv["traffic_bytes_per_launch"])


def make_workload(name):
    from gen import workloads as W
    return getattr(W, name)()


def pair_counts(w, nbr, cnt, S_mask):
    """Counts that scale the per-unit work: expensive pairs inside S within
    the expensive cutoff, cheap pairs within the 2-body cutoff, ordered
    cheap leg pairs within the 3-body cutoff, average list length."""
    pos = w["pos"]
    L = w["L"]
    per = w["periodic"].astype(bool)
    n = len(pos)
    rows = np.repeat(np.arange(n), cnt)
    cols = np.concatenate([nbr[i, :cnt[i]] for i in range(n)]) if n else np.zeros(0, int)
    d = pos[cols] - pos[rows]
    for k in range(3):
        if per[k]:
            d[:, k] -= L[k] * np.round(d[:, k] / L[k])
    r2 = (d ** 2).sum(1)
    m = w["model"]
    rce, rc2, rc3 = m["ace"]["rcut"], m["uf3"]["rcut2"], m["uf3"]["rcut3"]
    exp_pairs = int(np.sum(S_mask[rows] & S_mask[cols] & (r2 < rce ** 2)))
    cheap2 = int(np.sum(r2 < rc2 ** 2))
    k3 = np.bincount(rows[r2 < rc3 ** 2], minlength=n) if m["uf3"]["n_knots3"] > 0 else np.zeros(n, int)
    cheap3 = int(np.sum(k3 * (k3 - 1) // 2))  # unordered leg pairs
    return dict(exp_pairs=exp_pairs, cheap_pairs=cheap2, cheap_triplets=cheap3,
                list_pairs=int(cnt.sum()), n=n)


def fit_main(args):
    """Constrained linear fit of the cheap potential (Methods, "Constrained
    potential fitting" and "Generation of synthetic data"): soft data =
    energies and forces of thermal snapshots of a 2,000-atom bcc W cube, hard
    data = energies of 102 strained cells (six strain states x 17 strains in
    +-0.5 %), labelled by the expensive potential before the timed region.
    Timed: the design rows of every configuration, the weighted normal
    equations of the soft rows and the lambda search, on one stream; the
    search's result is read back at the end of each fit."""
    import torch
    from gen import fitdata as FD
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core
    from paper_2502_19081_amd.fit import CheapFit
    torch.cuda.set_device(0)
    dev = "cuda"
    m = FD.fit_model()
    model = core.Model(m, precision="fp64")
    fit = CheapFit(model, device=dev)
    nd = fit.nd
    soft = FD.thermal_snapshots(args.fit_snapshots)
    hard = FD.strained_cells()
    print(f"bench: fit, {len(soft)} soft snapshots, {len(hard)} strained cells, {nd} parameters",
          file=sys.stderr, flush=True)

    def prep(cfgs):
        out = []
        for c in cfgs:
            n = len(c["pos"])
            sy = core.System(model, n, c["L"], c["periodic"], cap=128, device=dev)
            pos = torch.from_numpy(np.ascontiguousarray(c["pos"].T)).to(dev)
            sp = torch.zeros(n, dtype=torch.int32, device=dev)
            r = sy.compute(pos, sp, mode=B.MODE_ALL_EXPENSIVE, force_rebuild=True)
            out.append((sy, pos, sp, n, r["e_exp"].sum().reshape(1), r["forces"].clone()))
            sy.status()
        return out
    S, H = prep(soft), prep(hard)
    offs = np.cumsum([0] + [1 + 3 * n for (_, _, _, n, _, _) in S])
    n_rows = int(offs[-1])
    rows = torch.empty(n_rows, nd, dtype=torch.float64, device=dev)
    y = torch.cat([torch.cat([e, f.reshape(-1)]) for (_, _, _, _, e, f) in S])
    w = torch.cat([torch.cat([torch.full((1,), 1.0 / n ** 2, dtype=torch.float64),
                              torch.ones(3 * n, dtype=torch.float64)])
                   for (_, _, _, n, _, _) in S]).to(dev)
    hoffs = np.cumsum([0] + [1 + 3 * n for (_, _, _, n, _, _) in H])
    hrows = torch.empty(int(hoffs[-1]), nd, dtype=torch.float64, device=dev)
    h_energy_rows = torch.from_numpy(hoffs[:-1].astype(np.int64)).to(dev)
    items = ([(sy, pos, sp, rows[o:o + 1 + 3 * n]) for (sy, pos, sp, n, _, _), o in zip(S, offs)] +
             [(sy, pos, sp, hrows[o:o + 1 + 3 * n]) for (sy, pos, sp, n, _, _), o in zip(H, hoffs)])
    yH = torch.cat([e for (_, _, _, _, e, _) in H])
    wH = torch.tensor([1.0 / n ** 2 for (_, _, _, n, _, _) in H], dtype=torch.float64, device=dev)
    G = torch.zeros(nd, nd, dtype=torch.float64, device=dev)
    bvec = torch.zeros(nd, dtype=torch.float64, device=dev)
    n_atoms = sum(n for (_, _, _, n, _, _) in S) + sum(n for (_, _, _, n, _, _) in H)

    AH = None

    def design_all():
        nonlocal AH
        fit.design_many(items)
        AH = hrows.index_select(0, h_energy_rows)

    def normal():
        G.zero_()
        bvec.zero_()
        fit.gram(rows, y, w, G, bvec)

    # alpha: three decades below the hard residual of the unconstrained fit
    design_all()
    normal()
    ridge = 1e-8 * float(torch.diagonal(G).mean())
    _, free = fit.constrained(G, bvec, AH, yH, 1e300, lam0=1e-12, ridge=ridge, wH=wH)
    alpha = 1e-3 * free["residual"]
    lam0 = 1e-6

    def once(ev=None):
        if ev:
            ev[0].record()
        design_all()
        if ev:
            ev[1].record()
        normal()
        if ev:
            ev[2].record()
        return fit.constrained(G, bvec, AH, yH, alpha, lam0=lam0, ridge=ridge, wH=wH)

    for _ in range(args.warmup):
        once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        u, info = once()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_fit = 1e3 * el / args.steps
    # stage split (events on the one stream)
    stage = np.zeros(3)
    for _ in range(max(3, args.steps // 4)):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        once(ev)
        ev[3].record()
        torch.cuda.synchronize()
        stage += [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
    stage /= max(3, args.steps // 4)
    # soft-data errors of the fitted cheap potential (per atom and per force component)
    pred = rows @ u
    err = (pred - y).cpu().numpy()
    e_rows = offs[:-1]
    e_err = np.array([err[o] / n for o, (_, _, _, n, _, _) in zip(e_rows, S)])
    f_mask = np.ones(n_rows, bool)
    f_mask[e_rows] = False
    print(f"bench: fit {ms_fit:.3f} ms (design {stage[0]:.3f}, normal equations {stage[1]:.3f}, "
          f"search {stage[2]:.3f}); lambda {info['lam']:.4e}, {info['n_solves']} solves",
          file=sys.stderr, flush=True)

    # roofline of the design-row stage (the dominant one): arithmetic of the
    # column-parallel accumulation, 8 flops per (pair, 2-body column), 16 per
    # (triplet centred on the atom, 3-body column) and 14 per (triplet in
    # which the atom is a leg, 3-body column); triplets with i as a leg are
    # twice the centred ones
    rc2, rc3 = m["uf3"]["rcut2"], m["uf3"]["rcut3"]
    n2c = m["uf3"]["n_knots2"] - 1
    n3c = nd - n2c
    pairs = trip = 0
    for (sy, pos, sp, n, _, _) in S + H:
        nb, cn = sy.neighbors()
        nb, cn = nb.cpu().numpy(), cn.cpu().numpy()
        P = pos.cpu().numpy().T
        rws = np.repeat(np.arange(n), cn)
        cls = np.concatenate([nb[i, :cn[i]] for i in range(n)])
        dd = P[cls] - P[rws]
        Lb = sy.box.L
        for k in range(3):
            dd[:, k] -= Lb[k] * np.round(dd[:, k] / Lb[k])
        r2 = (dd ** 2).sum(1)
        pairs += int((r2 < rc2 ** 2).sum())
        m3 = np.bincount(rws[r2 < rc3 ** 2], minlength=n)
        trip += int((m3 * (m3 - 1) // 2).sum())
    design_flops = 8.0 * n2c * pairs + (16.0 + 2 * 14.0) * n3c * trip
    gram_bytes = n_rows * (nd + 2) * 8
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's fit on a bounded sample: design rows of one soft
        # snapshot and of the 17 strains of one state, scaled to the whole
        # job by atom count; its Gram and search on the full matrices
        import oracle as O
        from oracle import fit as OF
        t0 = time.perf_counter()
        c = soft[0]
        OF.design(m, c["pos"], np.zeros(len(c["pos"]), np.int32), c["L"], c["periodic"])
        for c in hard[:17]:
            OF.design(m, c["pos"], np.zeros(len(c["pos"]), np.int32), c["L"], c["periodic"])
        t_design = time.perf_counter() - t0
        n_sample = len(soft[0]["pos"]) + sum(len(c["pos"]) for c in hard[:17])
        A_np, y_np, w_np = rows.cpu().numpy(), y.cpu().numpy(), w.cpu().numpy()
        t0 = time.perf_counter()
        GSr, bSr = OF.gram(A_np, y_np, w_np)
        OF.constrained_fit(GSr, bSr, AH.cpu().numpy(), yH.cpu().numpy(), alpha, lam0=lam0,
                           ridge=ridge, wH=wH.cpu().numpy())
        t_solve = time.perf_counter() - t0
        t_cpu = t_design * n_atoms / n_sample + t_solve
        cpu = {"value": t_cpu * 1e3, "unit": "ms per fit", "cores": O.num_threads(),
               "kind": "oracle",
               "sample": f"design rows of one {len(soft[0]['pos'])}-atom snapshot and 17 strained "
                         f"cells ({n_sample} atoms, {t_design:.1f} s) scaled by atom count to the "
                         f"{n_atoms} atoms of the job, plus the oracle's Gram and lambda search on "
                         f"the full matrices ({t_solve:.2f} s)"}
    res = {
        "metric": "constrained fit of the cheap potential: wall time per fit (design rows, "
                  "normal equations, lambda search)",
        "value": ms_fit, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_fit, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"constrained fit: {len(soft)} thermal snapshots of a 2,000-atom "
                               f"bcc W cube + {len(hard)} strained cells, {nd} parameters",
                   "soft_rows": n_rows, "hard_rows": len(H), "labelled_atoms": n_atoms,
                   "alpha": alpha, "ridge": ridge},
        "stage_ms": {"design": stage[0], "normal_equations": stage[1], "search": stage[2]},
        "lambda": info["lam"], "hard_residual": info["residual"], "status": info["status"],
        "n_solves": info["n_solves"], "unconstrained_hard_residual": free["residual"],
        "soft_energy_rmse_eV_per_atom": float(np.sqrt(np.mean(e_err ** 2))),
        "soft_force_rmse_eV_per_A": float(np.sqrt(np.mean(err[f_mask] ** 2))),
        "roofline": {"bound": "alu", "kernel": "design rows (k_fit_design, all configurations)",
                     "achieved": design_flops / (stage[0] * 1e-3) / 1e12,
                     "peak": FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": design_flops / (stage[0] * 1e-3) / 1e12 / FP64_VALU_TFLOPS,
                     "traffic": None, "algorithmic_per_stage": design_flops,
                     "pairs": pairs, "centred_triplets": trip,
                     "note": "stage time: one batched design call over all configurations"},
        "normal_equations_hbm": {"achieved": gram_bytes / (stage[1] * 1e-3) / 1e9,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": gram_bytes / (stage[1] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "algorithmic_bytes": gram_bytes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))


def replay_ms(model, sy, pos, sp, stage, reps):
    """Average duration (ms) of one stage's kernel: `reps` back-to-back
    launches on the state the last evaluation left in the workspace, two HIP
    events around them on the launch stream (the current stream). The pair
    adjoint writes the expensive site energies, the cheap potential the cheap
    ones."""
    import ctypes
    import torch
    from paper_2502_19081_amd import binding as B
    e_out = sy.e_exp if B.lib().mlmix_profile_stage_name(stage).decode() == "ace_pairgrad" \
        else sy.e_cheap
    cur = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = (model.handle, cur, ctypes.c_void_p(sy.ws.data_ptr()), sy.n,
            ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(sp.data_ptr()),
            ctypes.byref(sy.box), ctypes.c_void_p(e_out.data_ptr()), stage)
    B.check(B.lib().mlmix_profile_replay(*args, 10))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    B.check(B.lib().mlmix_profile_replay(*args, reps))
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def main():
    args = parse()
    if args.probe == "copy":
        copy_probe()
        return
    if args.fit:
        fit_main(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(multi-GPU sharding is designed, not built)"}))
        sys.exit(2)
    import torch
    from gen.workloads import KAPPA  # noqa: F401
    from paper_2502_19081_amd import binding as B
    from paper_2502_19081_amd import core

    cfg = args.config
    w = make_workload(cfg)
    if args.seeded:
        # the paper's seeded region fix in place of the geometric regions:
        # seeds = the atoms within 2 A of the first region's centre (the
        # defect), core = seeds and their neighbours within 6 A, 2 A linear
        # blend to the nearest core atom
        from gen.workloads import seeded
        c = w["regions"][0]["center"]
        d = w["pos"] - c
        per = np.asarray(w["periodic"], bool)
        d[:, per] -= w["L"][per] * np.round(d[:, per] / w["L"][per])
        w["seeds"] = np.linalg.norm(d, axis=1) < 2.0
        w["regions"] = [seeded(6.0, 2.0)]
    prec = args.precision or w.get("precision", "fp32")
    dev = "cuda:0"
    torch.cuda.set_device(0)
    n = len(w["pos"])
    print(f"bench: {cfg} n={n} precision={prec}", file=sys.stderr, flush=True)
    model = core.Model(w["model"], precision=prec)
    vel0 = w.get("vel")
    if vel0 is None:
        from gen.workloads import maxwell
        vel0 = maxwell(np.random.default_rng(w["seed"] + 17), w["species"], 300.0)
    mass = torch.from_numpy(w["masses"][w["species"]].astype(np.float64)).to(dev)

    def fresh(mode):
        _, sy, pos, sp = core.system_for(w, model=model, cap=128, device=dev)
        if "seeds" in w:
            sy.set_seeds(torch.from_numpy(w["seeds"].astype(np.uint8)))
        vel = torch.from_numpy(np.ascontiguousarray(vel0.T)).to(dev)
        if args.langevin:
            sy.set_langevin(300.0, 2000.0)
        sy.compute(pos, sp, r_buffer=w["r_buffer"], mode=mode, force_rebuild=True)
        return sy, pos, vel, sp

    dt = float(w.get("dt", 1.0))

    def step(sy, pos, vel, sp, mode, rebuild=True, single=False):
        sy.vv_step(pos, vel, mass, sp, dt, r_buffer=w["r_buffer"], mode=mode,
                   force_rebuild=rebuild, single_stream=args.single_stream or single,
                   cheap_masked=args.cheap_masked)

    en_buf = torch.zeros(max(args.graph_steps, 1), 3, dtype=torch.float64, device=dev)

    def steps_fused(sy, pos, vel, sp, mode, k, rebuild=True):
        # k steps in one call (the library fuses them up to 65,536 atoms);
        # with the thermostat every step needs its own normals
        if args.langevin or k == 1:
            for _ in range(k):
                step(sy, pos, vel, sp, mode, rebuild)
            return
        sy.vv_steps(pos, vel, mass, sp, dt, k, r_buffer=w["r_buffer"], mode=mode,
                    force_rebuild=rebuild, single_stream=args.single_stream,
                    cheap_masked=args.cheap_masked, energies=en_buf[:k])

    def run(mode, steps, warmup, stage_mask=0, latency=False, graph=False, rebuild=True,
            single=False):
        """Times `steps` steps. graph=True captures `chunk` consecutive steps
        (args.graph_steps when it divides `steps`, one step when latency is
        timed) in one HIP graph and replays it; otherwise the step's kernels
        are launched eagerly."""
        sy, pos, vel, sp = fresh(mode)
        for _ in range(warmup):
            step(sy, pos, vel, sp, mode, rebuild)
        sy.status()
        g = None
        chunk = 1
        if graph:
            if not latency and args.graph_steps > 1 and steps % args.graph_steps == 0:
                chunk = args.graph_steps
            g = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream()
            cs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cs):
                with torch.cuda.graph(g, stream=cs):
                    steps_fused(sy, pos, vel, sp, mode, chunk, rebuild)
            torch.cuda.current_stream().wait_stream(cs)
            for _ in range(3):
                g.replay()
        model.profile_read()
        model.profile_enable(stage_mask)
        builds0 = sy.list_builds()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat = []
        for _ in range(steps // chunk):
            ts = time.perf_counter()
            if g is not None:
                g.replay()
            else:
                step(sy, pos, vel, sp, mode, rebuild, single)
            if latency:
                torch.cuda.synchronize()
                lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        model.profile_enable(0)
        prof = model.profile_read()
        sy.status()
        run.builds = sy.list_builds() - builds0  # list builds inside the timed region
        return (t1 - t0), prof, lat, sy

    # 1. per-stage breakdown (every stage bracketed) to find the dominant
    # kernel: the steps run on one stream, so that each bracket holds its
    # stage alone on the GPU (and the dispatch gap before it), not the
    # cheap potential running beside it
    main_rebuild = args.rebuild_every_step
    n_break = max(10, args.steps // 4)
    _, prof_all, _, _ = run(B.MODE_MIXED, n_break, args.warmup,
                               stage_mask=(1 << B.N_STAGES) - 1, rebuild=main_rebuild,
                               single=True)
    build_frac = run.builds / n_break  # list builds per step in the breakdown
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in prof_all.items() if v[1]}
    # in the timed steps the reverse slots and the cheap potential run on the
    # second stream beside the expensive chain (the cheap potential has a
    # roofline line of its own): the dominant kernel is taken from that chain
    side = set() if args.single_stream else {"uf3", "reverse_slots"}
    dominant = max((k for k in stage_ms if k not in side),
                   key=lambda k: stage_ms[k] * prof_all[k][1])
    if args.dominant:
        dominant = args.dominant  # fixed for a profiler run, whose brackets shift the breakdown
    dom_bit = [B.lib().mlmix_profile_stage_name(i).decode() for i in range(B.N_STAGES)].index(dominant)

    print(f"bench: stage breakdown done, dominant {dominant}", file=sys.stderr, flush=True)

    # 2. the dominant kernel's duration: K eager steps with only that stage
    # timed by HIP events on its launch stream (for the matrix-core
    # contraction the kernel's own start/end events)
    el_eager, prof, _, _ = run(B.MODE_MIXED, args.steps, args.warmup, stage_mask=1 << dom_bit,
                               rebuild=main_rebuild)
    dom_ms, dom_cnt = prof[dominant]
    dom_avg_ms = dom_ms / max(dom_cnt, 1)
    dom_in_step_ms = dom_avg_ms
    dom_method = "stage bracketed by HIP events inside each of the K eager steps"
    # the state of one mixed step for the kernel replays below
    sy_r, pos_r, vel_r, sp_r = fresh(B.MODE_MIXED)
    step(sy_r, pos_r, vel_r, sp_r, B.MODE_MIXED)
    if dominant == "ace_contract" or (dominant == "ace_pairgrad" and prec != "fp64"):
        # the kernel's own duration: K back-to-back launches on the state of
        # a mixed step, two events around them on its stream (the in-step
        # bracket also holds the dispatch gap before the kernel)
        dom_avg_ms = replay_ms(model, sy_r, pos_r, sp_r, dom_bit, args.steps)
        dom_cnt = args.steps
        dom_method = ("K back-to-back launches on the state of a mixed step, HIP events on "
                      "the launch stream")
    if args.dominant_only:
        # the launches timed above, alone (for a kernel trace of exactly them)
        print(json.dumps({"kernel": dominant, "avg_ms": dom_avg_ms, "launches": dom_cnt,
                          "in_step_bracket_ms": dom_in_step_ms, "method": dom_method,
                          "config": cfg, "precision": prec}), flush=True)
        return

    # the cheap potential's own duration (second stream: it runs beside the
    # expensive chain in a step), K back-to-back uncapped launches
    uf3_bit = [B.lib().mlmix_profile_stage_name(i).decode() for i in range(B.N_STAGES)].index("uf3")
    uf3_ms = replay_ms(model, sy_r, pos_r, sp_r, uf3_bit, args.steps)

    # 3. timed region: K mixed steps replayed from one captured HIP graph
    el, _, _, _ = run(B.MODE_MIXED, args.steps, args.warmup, graph=True, rebuild=main_rebuild)
    timed_builds = run.builds
    ms_step = 1e3 * el / args.steps
    value = n * args.steps / el

    print(f"bench: mixed {ms_step:.4f} ms/step", file=sys.stderr, flush=True)

    # 4. all-expensive and all-cheap rates on the same GPU, same method
    rate_e = rate_c = None
    lat_ms = None
    rate_other = None
    other_builds = None
    if not args.only_mixed:
        el_e, _, _, _ = run(B.MODE_ALL_EXPENSIVE, args.steps, args.warmup, graph=True,
                            rebuild=main_rebuild)
        el_c, _, _, _ = run(B.MODE_ALL_CHEAP, args.steps, args.warmup, graph=True,
                            rebuild=main_rebuild)
        rate_e = n * args.steps / el_e
        rate_c = n * args.steps / el_c
        print(f"bench: all-expensive {1e3 * el_e / args.steps:.4f} ms/step, all-cheap "
              f"{1e3 * el_c / args.steps:.4f} ms/step", file=sys.stderr, flush=True)

        # 5. step latency (each replay waited for)
        _, _, lat, _ = run(B.MODE_MIXED, args.steps, 5, latency=True, graph=True,
                           rebuild=main_rebuild)
        lat_ms = np.array(lat) * 1e3
        # 6. the same mixed steps under the other list policy (rebuilt every
        # step, or kept while no atom has moved half the skin; lambda, the
        # buffer and both potentials are evaluated every step either way)
        el_s, _, _, sy_s = run(B.MODE_MIXED, args.steps, args.warmup, graph=True,
                               rebuild=not main_rebuild)
        rate_other = n * args.steps / el_s
        other_builds = run.builds
        print(f"bench: mixed with the other list policy {1e3 * el_s / args.steps:.4f} ms/step",
              file=sys.stderr, flush=True)

    # work counts of the initial configuration (for the roofline)
    sy, pos, vel, sp = fresh(B.MODE_MIXED)
    out = sy.compute(pos, sp, r_buffer=w["r_buffer"], mode=B.MODE_MIXED, force_rebuild=True,
                     cheap_masked=args.cheap_masked)
    torch.cuda.synchronize()
    nS, nM = [int(x) for x in out["n_exp"].cpu()]
    S_idx, _ = sy.index_sets()
    S_mask = np.zeros(n, bool)
    S_mask[S_idx.cpu().numpy()] = True
    nbr, cnt = sy.neighbors()
    pc = pair_counts(w, nbr.cpu().numpy(), cnt.cpu().numpy(), S_mask)
    fl = np.zeros(7)
    import ctypes
    B.check(B.lib().mlmix_model_flops(model.handle, fl.ctypes.data_as(ctypes.c_void_p)))
    gpu_forces = out["forces"].cpu().numpy().T.copy()

    tsz = 8 if prec == "fp64" else 4
    mw = w["model"]["ace"]
    nch = mw["n_rad"] * w["model"]["n_species"]
    KAt = (mw["lmax"] + 1) ** 2 * ((nch + 3) // 4 * 4)
    dp_stride = nch * sum(2 * l3 + 1 for l1 in range(mw["lmax"] + 1) for l2 in range(l1, mw["lmax"] + 1)
                          for l3 in range(l2 - l1, min(mw["lmax"], l1 + l2) + 1)
                          if (l1 + l2 + l3) % 2 == 0) if mw["order"] >= 3 else 0
    work = {
        # flops per launch
        "ace_contract": ("flops", fl[0] * nS),
        "ace_finalize": ("bytes", nS * (2 * KAt * tsz + dp_stride * tsz + 16)),
        "ace_basis": ("flops", fl[1] * pc["exp_pairs"]),
        # with the finalisation folded in (no finalisation launches), its
        # work per S atom too
        "ace_pairgrad": ("flops", fl[2] * pc["exp_pairs"]
                         + (fl[6] * nS if "ace_finalize" not in stage_ms else 0.0)),
        "uf3": ("flops", fl[3] * pc["cheap_pairs"] + fl[4] * pc["cheap_triplets"]),
        # HBM bytes per launch
        # per step: the displacement check (48 B per atom) unless every step
        # rebuilds, and a build's 24 B per atom + 8 B per list entry + 8 B per
        # atom in the fraction of steps that rebuilt
        "neighbours": ("bytes", build_frac * (24 * n + 8 * pc["list_pairs"] + 8 * n)
                       + (0 if main_rebuild else 48 * n)),
        "regions": ("bytes", 33 * n),
        "compaction": ("bytes", 9 * n + 4 * nS),
        "gather_blend": ("bytes", 44 * n + 8 * pc["list_pairs"] + 2 * 3 * tsz * pc["list_pairs"]
                         + 2 * 3 * tsz * pc["exp_pairs"]),
        "integrator": ("bytes", 2 * 88 * n),
        "energy_sums": ("bytes", 48 * n),
    }
    # every stage against its bound from the bracketed per-step times of the
    # breakdown (a bracket also holds the dispatch gap, so these achieved
    # figures are lower bounds; stages on the second stream overlap)
    stage_roof = {}
    for k, (kd, u) in work.items():
        t = stage_ms.get(k)
        if not t:
            continue
        if kd == "flops":
            pk = FP64_VALU_TFLOPS if prec == "fp64" else FP32_VALU_UNPACKED_TFLOPS
            if k == "ace_contract" and prec != "fp64" and w["model"]["n_species"] == 1:
                pk = MFMA_TFLOPS["fp32"]
            a_ = u / (t * 1e-3) / 1e12
            stage_roof[k] = {"unit": "TFLOP/s", "achieved": a_, "peak": pk, "frac": a_ / pk}
        else:
            a_ = u / (t * 1e-3) / 1e9
            stage_roof[k] = {"unit": "GB/s", "achieved": a_, "peak": HBM_PEAK_GBS,
                             "frac": a_ / HBM_PEAK_GBS}
    uf3_units = work["uf3"][1]
    uf3_peak = FP64_VALU_TFLOPS if prec == "fp64" else FP32_VALU_UNPACKED_TFLOPS
    uf3_roof = {"kernel": "uf3", "bound": "alu", "unit": "TFLOP/s",
                "achieved": uf3_units / (uf3_ms * 1e-3) / 1e12, "peak": uf3_peak,
                "frac": uf3_units / (uf3_ms * 1e-3) / 1e12 / uf3_peak, "avg_ms": uf3_ms,
                "launches": args.steps, "algorithmic_per_launch": uf3_units,
                "traffic": measured_traffic("uf3", cfg, prec),
                "timing": "K back-to-back uncapped launches on the state of a mixed step, HIP "
                          "events on the launch stream",
                "note": "second stream: in a step it runs beside the expensive chain; peak = "
                        "FP32 vector rate without packed instructions (the build disables them)"}
    traffic = measured_traffic(dominant, cfg, prec)
    kind, units = work[dominant]
    if kind == "flops":
        bound = "alu"
        peak = FP64_VALU_TFLOPS if prec == "fp64" else FP32_VALU_TFLOPS
        if dominant == "ace_contract" and prec != "fp64" and w["model"]["n_species"] == 1:
            # order-3 stages on the matrix cores: sparse stage FP32, dense
            # stage in the operand format; the peak is the time-weighted one
            # (all flops at their stage's peak)
            bound = "mfma"
            dense = fl[5] * nS
            peak = units / ((units - dense) / MFMA_TFLOPS["fp32"] + dense / MFMA_TFLOPS[prec])
        achieved = units / (dom_avg_ms * 1e-3) / 1e12
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic, "kernel": dominant,
                "avg_ms": dom_avg_ms, "launches": dom_cnt, "algorithmic_per_launch": units,
                "timing": dom_method, "in_step_bracket_ms": dom_in_step_ms}
    else:
        achieved = units / (dom_avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dominant,
                "avg_ms": dom_avg_ms, "launches": dom_cnt, "algorithmic_per_launch": units,
                "timing": dom_method, "in_step_bracket_ms": dom_in_step_ms}

    peaks = measured_peaks()
    roof["peak_measured"] = peaks
    if roof["unit"] == "GB/s":
        roof["frac_of_measured"] = roof["achieved"] / peaks["hbm_copy_GBps"]
    elif roof["bound"] == "mfma" and prec == "fp32":
        roof["frac_of_measured"] = roof["achieved"] / peaks["mfma_fp32_TFLOPs"]

    # 6. CPU baseline: the FP64 reference on this host, bounded sample of the
    # same workload (its first force call also gives the force error)
    cpu = None
    ferr = None
    if not args.no_cpu_baseline and n > 100000:
        # large cell: one mixed force call of the reference with forces
        # required on a ~4,000-atom cube around the first vacancy (every
        # site energy those forces depend on is evaluated)
        import oracle as O
        from gen.workloads import subvolume
        sub = subvolume(w, w["vacancy_centres"][0], 40.0)
        target = np.zeros(n, bool)
        target[sub] = True
        t0 = time.perf_counter()
        ref = O.mixed(w, O.MODE_MIXED, target=target, cheap_masked=args.cheap_masked)
        t_cpu = time.perf_counter() - t0
        ferr = float(np.abs(gpu_forces[sub] - ref["forces"][sub]).max())
        cpu = {"value": len(sub) / t_cpu, "unit": "atom-steps/s", "cores": O.num_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"one mixed FP64 force call of the same {cfg} cell with forces on the "
                         f"{len(sub)} atoms of a 40 A cube around a vacancy (neighbour list, "
                         f"lambda and buffer over the whole cell), rate = cube atoms / time"}
    elif not args.no_cpu_baseline:
        import oracle as O
        t0 = time.perf_counter()
        ref = O.mixed(w, O.MODE_MIXED, cheap_masked=args.cheap_masked)
        t_first = time.perf_counter() - t0
        ferr = float(np.abs(gpu_forces - ref["forces"]).max())
        n_cpu = max(1, int(args.cpu_seconds / max(t_first, 1e-3)))
        t0 = time.perf_counter()
        O.velocity_verlet(w, w["pos"], vel0, float(w.get("dt", 1.0)), n_cpu, mode=O.MODE_MIXED,
                          cheap_masked=args.cheap_masked)
        t_cpu = time.perf_counter() - t0
        # one thread, a shorter sample of the same steps
        cores = O.num_threads()
        O.set_threads(1)
        n1 = max(1, n_cpu // max(cores, 1))
        t0 = time.perf_counter()
        O.velocity_verlet(w, w["pos"], vel0, float(w.get("dt", 1.0)), n1, mode=O.MODE_MIXED,
                          cheap_masked=args.cheap_masked)
        t1 = time.perf_counter() - t0
        O.set_threads(cores)
        cpu = {"value": n * n_cpu / t_cpu, "unit": "atom-steps/s", "cores": cores,
               "kind": "oracle", "cpu_model": cpu_model(),
               "value_1_thread": n * n1 / t1,
               "sample": f"{n_cpu} velocity-Verlet steps of the same {cfg} workload in mixed mode "
                         f"(plus one initial force call), FP64, neighbour list rebuilt every step; "
                         f"{n1} steps on one thread for value_1_thread"}

    s_ul = None
    if rate_e:
        S_CE = rate_c / rate_e
        s_ul = n * S_CE / (nS * S_CE + n)
    res = {
        "metric": "mixed atom-steps/s vs all-expensive at stated force error; p99 step latency",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[cfg], "n_atoms": n, "mode": "mixed",
                   "regions": "seeded (6 A core, 2 A blend)" if args.seeded else "geometric",
                   "cheap": "masked to its subsystem" if args.cheap_masked else "every atom",
                   "thermostat": ("Langevin 300 K, 2 ps, lambda == 0 atoms" if args.langevin
                                  else "none (NVE)"),
                   "precision": prec,
                   "neighbour_rebuild": ("every step" if main_rebuild else
                                         "when an atom has moved more than half the 1 A skin "
                                         "since the last build (checked on the device every "
                                         "step)"),
                   "list_builds_in_timed_steps": timed_builds, "n_S": nS, "n_lambda_pos": nM,
                   "launch": (f"{args.graph_steps} consecutive steps per captured HIP graph "
                              f"({'one step per call' if args.langevin else 'one fused multi-step call'}), "
                              "replayed" if args.steps % args.graph_steps == 0 and args.graph_steps > 1
                              else "one captured HIP graph per step, replayed")},
        "eager_atom_steps_per_s": n * args.steps / el_eager,
        "all_expensive_atom_steps_per_s": rate_e,
        "all_cheap_atom_steps_per_s": rate_c,
        "mixed_over_all_expensive": value / rate_e if rate_e else None,
        ("rebuild_every_step_atom_steps_per_s" if not main_rebuild
         else "skin_list_atom_steps_per_s"): rate_other,
        "other_policy_list_builds": other_builds,
        "S_UL": s_ul,
        "force_err_max_eV_per_A": ferr,
        "p50_step_ms": float(np.percentile(lat_ms, 50)) if lat_ms is not None else None,
        "p99_step_ms": float(np.percentile(lat_ms, 99)) if lat_ms is not None else None,
        "stage_ms_per_step": {k: round(v, 5) for k, v in stage_ms.items()},
        "stage_timing": "every stage bracketed by HIP events in mixed steps run on one stream "
                        "(each stage alone on the GPU; a bracket also holds the dispatch gap)",
        "stage_roofline": stage_roof,
        "roofline": roof,
        "second_stream_roofline": uf3_roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
