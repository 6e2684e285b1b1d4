"""NVE molecular dynamics on the device with the mixed forces (FP64
velocity Verlet, `mlmix_vv_step`), and the energy bookkeeping of mixed runs.

Total energy is undefined under force mixing (the paper's discussion of
energy conservation); a mixed run's drift is measured as kinetic energy plus
the expensive potential's energy of the whole system, evaluated on snapshots
(the supplementary drift protocol), and a pure run's as kinetic plus its own
potential energy every step.
"""
import numpy as np
import torch

from . import binding as B
from . import core


def run_nve(sy, pos, vel, mass, species, dt, steps, r_buffer=0.0, mode=B.MODE_MIXED,
            every=10, force_rebuild=False, snapshot=None):
    """Advance `steps` velocity-Verlet steps. Returns a list of
    (step, sum e_exp, sum e_cheap, kinetic[, snapshot energy]) every `every`
    steps (the first entry is the initial state). `snapshot(pos)` may return
    an extra energy (for example the all-expensive energy of the positions)."""
    out = sy.compute(pos, species, r_buffer=r_buffer, mode=mode, force_rebuild=True)
    e = sy.energy_reduce(vel, mass).cpu().numpy()
    rec = [(0, *e.tolist(), *( [snapshot(pos)] if snapshot else []))]
    for s in range(1, steps + 1):
        sy.vv_step(pos, vel, mass, species, dt, r_buffer=r_buffer, mode=mode,
                   force_rebuild=force_rebuild)
        if s % every == 0:
            e = sy.energies.cpu().numpy()
            rec.append((s, *e.tolist(), *([snapshot(pos)] if snapshot else [])))
    sy.status()
    return rec


def expensive_snapshot(model, w, device="cuda"):
    """Energy of the whole system under the expensive potential alone (a
    separate workspace, all-expensive mode), for mixed-run drift."""
    _, sy, _, sp = core.system_for(w, model=model, device=device)

    def f(pos):
        sy.compute(pos, sp, mode=B.MODE_ALL_EXPENSIVE, force_rebuild=True, energy_only=True)
        return float(sy.energy_reduce().cpu().numpy()[0])
    return f
