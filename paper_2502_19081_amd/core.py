"""Python face of the HIP library: a Model (the two potentials' tables on the
device) and a System (one workspace: the neighbour list and intermediates of
one set of atoms). Torch tensors carry device memory and streams only; all
arithmetic runs in libmlmix.so.
"""
import ctypes

import numpy as np
import torch

from . import binding as B


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_box(L, periodic):
    b = B.Box()
    for k in range(3):
        b.L[k] = float(L[k])
        b.periodic[k] = int(periodic[k])
    return b


def pack_regions(regions, device="cuda"):
    """Region dictionaries (type, axis, follow_atom, center, r_core, r_blend,
    optional blend: 0 linear, 1 cubic) -> a device byte tensor of
    mlmix_region structs. Seeded regions (type 2) need only r_core, r_blend
    and blend."""
    n = max(len(regions), 1)
    arr = (B.Region * n)()
    for k, r in enumerate(regions):
        arr[k].type = int(r["type"])
        arr[k].axis = int(r.get("axis", 2))
        arr[k].follow_atom = int(r.get("follow_atom", -1))
        arr[k].blend = int(r.get("blend", 0))
        c = r.get("center", None)
        for q in range(3):
            arr[k].center[q] = float(c[q]) if c is not None else 0.0
        arr[k].r_core = float(r["r_core"])
        arr[k].r_blend = float(r["r_blend"])
    raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


class Model:
    """Device tables of the ACE-style and UF3-style potentials."""

    def __init__(self, model, precision="fp64"):
        a, u = model["ace"], model["uf3"]
        self._keep = [np.ascontiguousarray(x, dtype=np.float64) for x in
                      (a["c0"], a["c1"], a["c2"], a["c3"], u["c2"], u["c3"])]
        c0, c1, c2, c3, u2, u3 = self._keep
        d = B.ModelDesc()
        d.n_species = int(model["n_species"])
        d.precision = {"fp64": B.FP64, "fp32": B.FP32, "bf16": B.BF16_CONTRACT,
                       "fp8": B.FP8_CONTRACT}[precision]
        d.skin = float(model["skin"])
        d.ace_n_rad, d.ace_lmax, d.ace_order = int(a["n_rad"]), int(a["lmax"]), int(a["order"])
        d.ace_rcut = float(a["rcut"])
        d.ace_c0, d.ace_c1, d.ace_c2 = c0.ctypes.data, c1.ctypes.data, c2.ctypes.data
        d.ace_c3 = c3.ctypes.data if a["order"] >= 3 else None
        d.uf3_n_knots2, d.uf3_n_knots3 = int(u["n_knots2"]), int(u["n_knots3"])
        d.uf3_rcut2, d.uf3_rcut3 = float(u["rcut2"]), float(u["rcut3"])
        d.uf3_c2 = u2.ctypes.data
        d.uf3_c3 = u3.ctypes.data if u["n_knots3"] > 0 else None
        self.precision = precision
        self.n_species = d.n_species
        h = ctypes.c_void_p()
        B.check(B.lib().mlmix_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.r_list = B.lib().mlmix_list_radius(h)

    def profile_enable(self, stage_mask):
        """Bracket the selected stages (bit i = stage i) with HIP events."""
        B.check(B.lib().mlmix_profile_enable(self.handle, int(stage_mask)))

    def profile_read(self):
        """{stage name: (milliseconds, launches)} since the last read."""
        ms = (ctypes.c_double * B.N_STAGES)()
        cnt = (ctypes.c_int64 * B.N_STAGES)()
        B.check(B.lib().mlmix_profile_read(self.handle, ms, cnt))
        return {B.lib().mlmix_profile_stage_name(i).decode(): (ms[i], cnt[i])
                for i in range(B.N_STAGES)}

    def close(self):
        if self.handle:
            B.lib().mlmix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    """One workspace: n atoms in an orthorhombic box with a neighbour-row
    capacity `cap`. Outputs are allocated once and reused between calls."""

    def __init__(self, model, n, L, periodic, cap=128, device="cuda", s_cap=0):
        self.model = model
        self.n = int(n)
        self.cap = int(cap)
        self.s_cap = int(s_cap)  # rows of the expensive potential's buffers (0: n)
        self.box = make_box(L, periodic)
        self.device = device
        sz = ctypes.c_size_t()
        B.check(B.lib().mlmix_workspace_size(model.handle, self.n, self.cap, self.s_cap,
                                             ctypes.byref(self.box), ctypes.byref(sz)))
        self.ws_bytes = int(sz.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        B.check(B.lib().mlmix_workspace_init(model.handle, _stream(), _p(self.ws), self.ws_bytes,
                                             self.n, self.cap, self.s_cap, ctypes.byref(self.box)))
        z = dict(dtype=torch.float64, device=device)
        self.forces = torch.zeros(3, self.n, **z)
        self.e_exp = torch.zeros(self.n, **z)
        self.e_cheap = torch.zeros(self.n, **z)
        self.lam = torch.zeros(self.n, **z)
        self.flags = torch.zeros(self.n, dtype=torch.uint8, device=device)
        self.n_exp = torch.zeros(2, dtype=torch.int32, device=device)
        self.energies = torch.zeros(3, **z)
        self.regions = pack_regions([], device)
        self.n_regions = 0
        self.generation = 0  # bumped by every evaluation on this workspace
        self.langevin = None
        self.xi = None
        self.xi_gen = None

    def set_regions(self, regions):
        self.regions = pack_regions(regions, self.device)
        self.n_regions = len(regions)

    def set_seeds(self, seeds):
        """Seed atoms of the seeded regions (bool/uint8 (n,), any device), or
        None. Each later evaluation passes them as MLMIX_FLAG_SEED bits of the
        flags array with MLMIX_SEEDED set."""
        if seeds is None:
            self.seed_bits = None
            return
        s = torch.as_tensor(seeds).to(self.device).reshape(self.n)
        self.seed_bits = (s != 0).to(torch.uint8) * B.FLAG_SEED

    def _seed_mode(self):
        if getattr(self, "seed_bits", None) is None:
            return 0
        self.flags.copy_(self.seed_bits)
        return B.SEEDED

    def set_langevin(self, temperature, damping_fs, generator=None):
        """Langevin thermostat on the atoms with lambda == 0 inside vv_step
        (temperature in K, damping time in fs; damping_fs <= 0 turns it off).
        The standard normals live in self.xi (3, n): vv_step refills them from
        `generator` before each step unless it is given xi itself."""
        on = damping_fs > 0.0
        if on and getattr(self, "xi", None) is None:
            self.xi = torch.zeros(3, self.n, dtype=torch.float64, device=self.device)
        self.langevin = (float(temperature), float(damping_fs)) if on else None
        self.xi_gen = generator
        B.check(B.lib().mlmix_set_langevin(self.model.handle, _p(self.ws), self.n,
                                           float(temperature), float(damping_fs),
                                           _p(self.xi) if on else None))

    def compute(self, pos, species, r_buffer=0.0, mode=B.MODE_MIXED, force_rebuild=False,
                split=False, energy_only=False, single_stream=False, cheap_masked=False):
        """pos: (3, n) float64 device tensor; species: (n,) int32 device tensor.
        single_stream: keep every stage on the current stream (no fork onto
        the workspace's second stream). cheap_masked: the cheap potential on
        its own subsystem only (MLMIX_CHEAP_MASKED)."""
        assert pos.shape == (3, self.n) and pos.dtype == torch.float64 and pos.is_contiguous()
        assert species.shape == (self.n,) and species.dtype == torch.int32
        flags = (mode | (B.FORCE_REBUILD if force_rebuild else 0) |
                 (B.ENERGY_ONLY if energy_only else 0) | (B.SINGLE_STREAM if single_stream else 0))
        flags |= self._seed_mode() | (B.CHEAP_MASKED if cheap_masked else 0)
        self.generation += 1
        fe = fc = None
        if split:
            fe = torch.zeros(3, self.n, dtype=torch.float64, device=self.device)
            fc = torch.zeros(3, self.n, dtype=torch.float64, device=self.device)
        B.check(B.lib().mlmix_compute(self.model.handle, _stream(), _p(self.ws), self.n, _p(pos),
                                      _p(species), ctypes.byref(self.box), _p(self.regions),
                                      self.n_regions, float(r_buffer), flags,
                                      None if energy_only else _p(self.forces), _p(self.e_exp),
                                      _p(self.e_cheap), _p(self.lam), _p(self.flags),
                                      _p(self.n_exp), _p(fe), _p(fc)))
        out = dict(forces=self.forces, e_exp=self.e_exp, e_cheap=self.e_cheap, lam=self.lam,
                   flags=self.flags, n_exp=self.n_exp)
        if split:
            out["f_exp"], out["f_cheap"] = fe, fc
        return out

    def backward(self, pos, species, grad_e, grad_pos):
        B.check(B.lib().mlmix_backward(self.model.handle, _stream(), _p(self.ws), self.n, _p(pos),
                                       _p(species), ctypes.byref(self.box), _p(grad_e),
                                       _p(grad_pos)))
        return grad_pos

    def vv_step(self, pos, vel, mass, species, dt, r_buffer=0.0, mode=B.MODE_MIXED,
                force_rebuild=False, energies=True, single_stream=False, cheap_masked=False,
                xi=None):
        """One velocity-Verlet step. With a thermostat set, xi ((3, n) float64)
        gives this step's normals; otherwise they are drawn here."""
        self.generation += 1
        if getattr(self, "langevin", None) is not None:
            if xi is not None:
                self.xi.copy_(xi)
            else:
                self.xi.normal_(generator=self.xi_gen)
        flags = mode | (B.FORCE_REBUILD if force_rebuild else 0) | (B.SINGLE_STREAM if single_stream else 0)
        flags |= self._seed_mode() | (B.CHEAP_MASKED if cheap_masked else 0)
        B.check(B.lib().mlmix_vv_step(self.model.handle, _stream(), _p(self.ws), self.n, _p(pos),
                                      _p(vel), _p(mass), _p(species), float(dt),
                                      ctypes.byref(self.box), _p(self.regions), self.n_regions,
                                      float(r_buffer), flags, _p(self.forces), _p(self.e_exp),
                                      _p(self.e_cheap), _p(self.lam), _p(self.flags),
                                      _p(self.n_exp), _p(self.energies) if energies else None))

    def vv_steps(self, pos, vel, mass, species, dt, n_steps, r_buffer=0.0, mode=B.MODE_MIXED,
                 force_rebuild=False, single_stream=False, cheap_masked=False, energies=None):
        """n_steps velocity-Verlet steps in one call (fused up to 65,536
        atoms); returns the (n_steps, 3) energy sums of every step. Not with
        the thermostat."""
        self.generation += n_steps
        flags = mode | (B.FORCE_REBUILD if force_rebuild else 0) | (B.SINGLE_STREAM if single_stream else 0)
        flags |= self._seed_mode() | (B.CHEAP_MASKED if cheap_masked else 0)
        if energies is None:
            energies = torch.zeros(n_steps, 3, dtype=torch.float64, device=self.device)
        B.check(B.lib().mlmix_vv_steps(self.model.handle, _stream(), _p(self.ws), self.n, _p(pos),
                                       _p(vel), _p(mass), _p(species), float(dt), int(n_steps),
                                       ctypes.byref(self.box), _p(self.regions), self.n_regions,
                                       float(r_buffer), flags, _p(self.forces), _p(self.e_exp),
                                       _p(self.e_cheap), _p(self.lam), _p(self.flags),
                                       _p(self.n_exp), _p(energies)))
        self.energies.copy_(energies[-1])
        return energies

    def energy_reduce(self, vel=None, mass=None):
        B.check(B.lib().mlmix_energy_reduce(self.model.handle, _stream(), _p(self.ws), self.n,
                                            _p(self.e_exp), _p(self.e_cheap), _p(vel), _p(mass),
                                            _p(self.energies)))
        return self.energies

    def status(self, raise_on_error=True):
        bits = ctypes.c_int32()
        req = ctypes.c_int32()
        rc = B.lib().mlmix_status(self.model.handle, _stream(), _p(self.ws), ctypes.byref(bits),
                                  ctypes.byref(req))
        if raise_on_error:
            B.check(rc)
        return int(bits.value), int(req.value), rc

    def list_builds(self):
        """Neighbour-list builds since the workspace was set up."""
        b = ctypes.c_int32()
        B.check(B.lib().mlmix_list_builds(self.model.handle, _stream(), _p(self.ws),
                                          ctypes.byref(b)))
        return int(b.value)

    def neighbors(self):
        nbr = torch.empty(self.n, self.cap, dtype=torch.int32, device=self.device)
        cnt = torch.empty(self.n, dtype=torch.int32, device=self.device)
        B.check(B.lib().mlmix_get_neighbors(self.model.handle, _stream(), _p(self.ws), self.n,
                                            _p(nbr), _p(cnt)))
        return nbr, cnt

    def index_sets(self):
        S = torch.empty(self.n, dtype=torch.int32, device=self.device)
        M = torch.empty(self.n, dtype=torch.int32, device=self.device)
        B.check(B.lib().mlmix_get_index_sets(self.model.handle, _stream(), _p(self.ws), self.n,
                                             _p(S), _p(M)))
        ns, nm = [int(x) for x in self.n_exp.cpu()]
        return S[:ns], M[:nm]


def system_for(w, model=None, cap=128, device="cuda", s_cap=0):
    """Model + System + device inputs for a workload dictionary of
    gen.workloads."""
    if model is None:
        model = Model(w["model"], precision=w.get("precision", "fp64"))
    n = len(w["pos"])
    sys_ = System(model, n, w["L"], w["periodic"], cap=cap, device=device, s_cap=s_cap)
    sys_.set_regions(w["regions"])
    pos = torch.from_numpy(np.ascontiguousarray(w["pos"].T)).to(device)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(device)
    return model, sys_, pos, species


class Batch:
    """Several independent systems sharing one model, evaluated and integrated
    together: one launch per kernel for the whole batch (mlmix_batch_*).

    systems: list of dicts with n (atoms), L, periodic and regions (region
    dictionaries as for System.set_regions; follow_atom counts from the
    system's first atom). The batch arrays hold the systems side by side:
    positions (3, n_total) SoA, per-atom arrays (n_total,); `offsets[k]` is
    the first atom of system k."""

    def __init__(self, model, systems, cap=128, s_cap=0, device="cuda"):
        self.model = model
        self.device = device
        self.cap = int(cap)
        self.s_cap = int(s_cap)
        self.nseg = len(systems)
        segs = (B.Segment * max(self.nseg, 1))()
        regions = []
        off = 0
        self.offsets = []
        self.sizes = []
        for k, sy in enumerate(systems):
            n = int(sy["n"])
            segs[k].offset = off
            segs[k].n_atoms = n
            segs[k].box = make_box(sy["L"], sy["periodic"])
            segs[k].region_offset = len(regions)
            segs[k].n_regions = len(sy.get("regions", []))
            regions.extend(sy.get("regions", []))
            self.offsets.append(off)
            self.sizes.append(n)
            off += n
        self.n = off
        self.segs = segs
        self.n_regions = len(regions)
        self.regions = pack_regions(regions, device)
        sz = ctypes.c_size_t()
        B.check(B.lib().mlmix_batch_workspace_size(model.handle, self.nseg, segs, self.cap,
                                                   self.s_cap, ctypes.byref(sz)))
        self.ws_bytes = int(sz.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        B.check(B.lib().mlmix_batch_init(model.handle, _stream(), _p(self.ws), self.ws_bytes,
                                         self.nseg, segs, self.cap, self.s_cap))
        z = dict(dtype=torch.float64, device=device)
        self.forces = torch.zeros(3, self.n, **z)
        self.e_exp = torch.zeros(self.n, **z)
        self.e_cheap = torch.zeros(self.n, **z)
        self.lam = torch.zeros(self.n, **z)
        self.flags = torch.zeros(self.n, dtype=torch.uint8, device=device)
        self.n_exp = torch.zeros(self.nseg, 2, dtype=torch.int32, device=device)
        self.energies = torch.zeros(self.nseg, 3, **z)

    def _flags(self, mode, force_rebuild, single_stream, cheap_masked):
        return (mode | (B.FORCE_REBUILD if force_rebuild else 0) |
                (B.SINGLE_STREAM if single_stream else 0) | (B.CHEAP_MASKED if cheap_masked else 0))

    def compute(self, pos, species, r_buffer=0.0, mode=B.MODE_MIXED, force_rebuild=False,
                single_stream=False, cheap_masked=False):
        assert pos.shape == (3, self.n) and pos.dtype == torch.float64 and pos.is_contiguous()
        assert species.shape == (self.n,) and species.dtype == torch.int32
        B.check(B.lib().mlmix_batch_compute(
            self.model.handle, _stream(), _p(self.ws), self.n, _p(pos), _p(species),
            _p(self.regions), self.n_regions, float(r_buffer),
            self._flags(mode, force_rebuild, single_stream, cheap_masked), _p(self.forces),
            _p(self.e_exp), _p(self.e_cheap), _p(self.lam), _p(self.flags), _p(self.n_exp),
            _p(self.energies)))
        return dict(forces=self.forces, e_exp=self.e_exp, e_cheap=self.e_cheap, lam=self.lam,
                    flags=self.flags, n_exp=self.n_exp, energies=self.energies)

    def vv_steps(self, pos, vel, mass, species, dt, n_steps, r_buffer=0.0, mode=B.MODE_MIXED,
                 force_rebuild=False, single_stream=False, cheap_masked=False, energies=None):
        """n_steps velocity-Verlet steps of every system; returns the
        (n_steps, n_systems, 3) energy sums (expensive, cheap, kinetic).
        Each system keeps its neighbour list until one of its own atoms
        moved half the skin (force_rebuild: every list every step)."""
        if energies is None:
            energies = torch.zeros(n_steps, self.nseg, 3, dtype=torch.float64,
                                   device=self.device)
        B.check(B.lib().mlmix_batch_vv_steps(
            self.model.handle, _stream(), _p(self.ws), self.n, _p(pos), _p(vel), _p(mass),
            _p(species), float(dt), int(n_steps), _p(self.regions), self.n_regions,
            float(r_buffer), self._flags(mode, force_rebuild, single_stream, cheap_masked),
            _p(self.forces), _p(self.e_exp), _p(self.e_cheap), _p(self.lam), _p(self.flags),
            _p(self.n_exp), _p(energies)))
        return energies

    def status(self, raise_on_error=True):
        """(per-system status bits, required row capacity, return code)."""
        bits = (ctypes.c_int32 * max(self.nseg, 1))()
        req = ctypes.c_int32()
        rc = B.lib().mlmix_batch_status(self.model.handle, _stream(), _p(self.ws), bits,
                                        ctypes.byref(req))
        if raise_on_error:
            B.check(rc)
        return [int(bits[k]) for k in range(self.nseg)], int(req.value), rc


    def carry_lists_from(self, old, seg_map):
        """Takes over the neighbour-list state of the systems this batch keeps
        from the batch `old` (seg_map[k]: old index of system k, or -1)."""
        m = (ctypes.c_int32 * max(self.nseg, 1))(*[int(v) for v in seg_map])
        B.check(B.lib().mlmix_batch_carry_lists(self.model.handle, _stream(), _p(self.ws),
                                                _p(old.ws), m))

    def list_builds(self):
        """Calls since the batch was set up in which some system's neighbour
        list was rebuilt."""
        b = ctypes.c_int32()
        B.check(B.lib().mlmix_list_builds(self.model.handle, _stream(), _p(self.ws),
                                          ctypes.byref(b)))
        return int(b.value)
    def slice(self, k):
        """Atom range of system k in the batch arrays."""
        return slice(self.offsets[k], self.offsets[k] + self.sizes[k])
