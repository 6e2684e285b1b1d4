"""ctypes declarations of the C ABI in include/mlmix.h (argument marshalling
only; every step of the computation runs in the HIP library).

Loading fails loudly when libmlmix.so has not been built: there is no
fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlmix.so")

MLMIX_OK = 0
ERRORS = {-1: "MLMIX_E_ARG", -2: "MLMIX_E_HIP", -3: "MLMIX_E_WORKSPACE",
          -4: "MLMIX_E_NEIGH_OVERFLOW", -5: "MLMIX_E_BOX", -6: "MLMIX_E_NONFINITE",
          -7: "MLMIX_E_STATE", -8: "MLMIX_E_HOST"}
FP64, FP32, BF16_CONTRACT, FP8_CONTRACT = 0, 1, 2, 3
MODE_MIXED, MODE_ALL_EXPENSIVE, MODE_ALL_CHEAP = 0, 1, 2
FORCE_REBUILD = 0x100
ENERGY_ONLY = 0x200
SINGLE_STREAM = 0x400
SEEDED = 0x800
FLAG_SEED = 0x80
CHEAP_MASKED = 0x1000
N_STAGES = 12
NOALLOC_SCRATCH_BYTES = 64 << 20
STATUS_NEIGH_OVERFLOW, STATUS_OUT_OF_BOX, STATUS_NONFINITE, STATUS_TRIPLET_OVERFLOW, STATUS_BAD_SPECIES = 1, 2, 4, 8, 16
STATUS_CELL_OVERFLOW, STATUS_SEEDED_REGIONS, STATUS_S_OVERFLOW = 32, 64, 128


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("skin", ctypes.c_double),
                ("ace_n_rad", ctypes.c_int32), ("ace_lmax", ctypes.c_int32),
                ("ace_order", ctypes.c_int32), ("ace_pad", ctypes.c_int32),
                ("ace_rcut", ctypes.c_double),
                ("ace_c0", ctypes.c_void_p), ("ace_c1", ctypes.c_void_p),
                ("ace_c2", ctypes.c_void_p), ("ace_c3", ctypes.c_void_p),
                ("uf3_n_knots2", ctypes.c_int32), ("uf3_n_knots3", ctypes.c_int32),
                ("uf3_rcut2", ctypes.c_double), ("uf3_rcut3", ctypes.c_double),
                ("uf3_c2", ctypes.c_void_p), ("uf3_c3", ctypes.c_void_p)]


class Box(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("periodic", ctypes.c_int32 * 3),
                ("pad", ctypes.c_int32)]


class FitConfig(ctypes.Structure):
    _fields_ = [("ws", ctypes.c_void_p), ("n_atoms", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("pos", ctypes.c_void_p), ("species", ctypes.c_void_p), ("box", Box),
                ("rows", ctypes.c_void_p)]


class Segment(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int32), ("n_atoms", ctypes.c_int32), ("box", Box),
                ("region_offset", ctypes.c_int32), ("n_regions", ctypes.c_int32)]


class Region(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("axis", ctypes.c_int32),
                ("follow_atom", ctypes.c_int32), ("blend", ctypes.c_int32),
                ("center", ctypes.c_double * 3), ("r_core", ctypes.c_double),
                ("r_blend", ctypes.c_double)]


assert ctypes.sizeof(Region) == 56
assert ctypes.sizeof(Segment) == 56

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_d = ctypes.c_double
_sz = ctypes.c_size_t

SIGNATURES = {
    "mlmix_create": (ctypes.c_int, [ctypes.POINTER(ModelDesc), ctypes.POINTER(_vp)]),
    "mlmix_destroy": (ctypes.c_int, [_vp]),
    "mlmix_list_radius": (ctypes.c_double, [_vp]),
    "mlmix_workspace_size": (ctypes.c_int, [_vp, _i32, _i32, _i32, ctypes.POINTER(Box),
                                            ctypes.POINTER(_sz)]),
    "mlmix_workspace_init": (ctypes.c_int, [_vp, _vp, _vp, _sz, _i32, _i32, _i32,
                                            ctypes.POINTER(Box)]),
    "mlmix_compute": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, ctypes.POINTER(Box), _vp, _i32, _d,
                                     _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mlmix_compute_noalloc": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _vp, _vp,
                                             ctypes.POINTER(Box), _vp, _i32, _d, _u32, _vp, _vp,
                                             _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_sz)]),
    "mlmix_backward": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, ctypes.POINTER(Box), _vp, _vp]),
    "mlmix_vv_step": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _d, ctypes.POINTER(Box),
                                     _vp, _i32, _d, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mlmix_set_langevin": (ctypes.c_int, [_vp, _vp, _i32, _d, _d, _vp]),
    "mlmix_vv_steps": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _d, _i32,
                                      ctypes.POINTER(Box), _vp, _i32, _d, _u32, _vp, _vp, _vp,
                                      _vp, _vp, _vp, _vp]),
    "mlmix_energy_reduce": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "mlmix_batch_workspace_size": (ctypes.c_int, [_vp, _i32, _vp, _i32, _i32,
                                                  ctypes.POINTER(_sz)]),
    "mlmix_batch_init": (ctypes.c_int, [_vp, _vp, _vp, _sz, _i32, _vp, _i32, _i32]),
    "mlmix_batch_compute": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _i32, _d, _u32,
                                           _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mlmix_batch_vv_steps": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _d, _i32,
                                            _vp, _i32, _d, _u32, _vp, _vp, _vp, _vp, _vp, _vp,
                                            _vp]),
    "mlmix_batch_status": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_i32)]),
    "mlmix_status": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "mlmix_list_builds": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_i32)]),
    "mlmix_get_neighbors": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "mlmix_get_index_sets": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "mlmix_model_flops": (ctypes.c_int, [_vp, _vp]),
    "mlmix_batch_carry_lists": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "mlmix_gaunt_table": (ctypes.c_int, [_i32, _vp]),
    "mlmix_fit_n_params": (ctypes.c_int, [_vp, ctypes.POINTER(_i32)]),
    "mlmix_fit_design": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, ctypes.POINTER(Box), _vp,
                                        _i32]),
    "mlmix_fit_design_batch": (ctypes.c_int, [_vp, _vp, _i32, _vp, _i32]),
    "mlmix_fit_work_size": (ctypes.c_int, [ctypes.c_int64, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    "mlmix_fit_gram": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, _i32, _i32, _vp, _vp, _vp,
                                      _vp, _vp, ctypes.c_size_t]),
    "mlmix_fit_constrained": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _i32, _i32, _vp, _vp, _d,
                                             _d, _d, _d, _i32, _i32, _vp, _vp, _vp,
                                             ctypes.c_size_t]),
    "mlmix_profile_enable": (ctypes.c_int, [_vp, _u32]),
    "mlmix_profile_replay": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, ctypes.POINTER(Box),
                                            _vp, _i32, _i32]),
    "mlmix_probe_mfma_f32": (ctypes.c_int, [_vp, _i32, _i32, _vp, ctypes.POINTER(_d)]),
    "mlmix_profile_read": (ctypes.c_int, [_vp, _vp, _vp]),
    "mlmix_profile_stage_name": (ctypes.c_char_p, [_i32]),
    "mlmix_last_error": (ctypes.c_char_p, []),
}

_lib = None


class MlmixError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def check(rc):
    if rc != MLMIX_OK:
        raise MlmixError(rc, lib().mlmix_last_error().decode())
    return rc
