"""ctypes declarations of libvplmc.so (include/vplmc.h).  Argument marshalling
only: every step of the method runs in the library's HIP kernels.  There is
no fallback: if the library is missing the import of a caller fails."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvplmc.so")

c_f32p = ctypes.c_void_p   # device pointers travel as integers


class Points(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32)] + [(k, ctypes.c_void_p) for k in (
        "px", "py", "pz", "nx", "ny", "nz", "kd_r", "kd_g", "kd_b", "ks", "phong_e", "vx", "vy", "vz")]


class Lights(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32)] + [(k, ctypes.c_void_p) for k in (
        "x", "y", "z", "nx", "ny", "nz", "ir", "ig", "ib")]


class Cut(ctypes.Structure):
    _fields_ = [("n_clusters", ctypes.c_int32), ("offsets", ctypes.c_void_p), ("members", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("pass1_ppm", ctypes.c_int32), ("pass2_ppm", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("flags", ctypes.c_int32), ("tol", ctypes.c_float),
                ("alpha0", ctypes.c_float), ("beta0", ctypes.c_float), ("gamma", ctypes.c_float),
                ("r_min", ctypes.c_float), ("ray_eps", ctypes.c_float), ("lam", ctypes.c_float),
                ("pass2_mix", ctypes.c_float)]


class Coarsen(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int32), ("pixels", ctypes.c_int32), ("left", ctypes.c_void_p),
                ("right", ctypes.c_void_p), ("n_max", ctypes.c_void_p), ("bound", ctypes.c_double),
                ("reserved", ctypes.c_int32)]


class LightTree(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int32), ("perm", ctypes.c_void_p), ("left", ctypes.c_void_p),
                ("right", ctypes.c_void_p)]


class Tune(ctypes.Structure):
    _fields_ = [("adm_queue", ctypes.c_int32), ("adm_threads", ctypes.c_int32), ("eval_threads", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class SliceInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("q", ctypes.c_int32), ("N1", ctypes.c_int32),
                ("N2", ctypes.c_int32), ("adm_in_lds", ctypes.c_int32), ("q_pad", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("off1", ctypes.c_int64), ("off2", ctypes.c_int64),
                ("off_omega", ctypes.c_int64), ("off_col", ctypes.c_int64), ("off_row", ctypes.c_int64),
                ("off_colptr", ctypes.c_int64), ("off_x", ctypes.c_int64), ("off_y", ctypes.c_int64)]


OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
FIXED_ITERS, LEARNED, FEATURES, GIVEN_INIT, NO_NONNEG, ALS = 1, 2, 4, 8, 16, 32
SLICE_ALL_ZERO, SLICE_NOT_CONVERGED, SLICE_SHORTFALL, SLICE_FALLBACK = 1, 2, 4, 8
REGIONS = ["LIGHTS", "REP", "BBOX", "OMEGA1", "VAL1", "OMEGA2", "VAL2", "WEIGHTS", "COLMIN", "COLMAX",
           "COLCNT", "ROW_PTR", "CSR_COL", "CSR_VAL", "COL_PTR", "CSC_ROW", "CSC_VAL", "X", "Y", "SLICE_SCALE",
           "FEATURES", "LOGITS", "COLUMNS", "NODE_EPS", "LEAF_DRAWS", "NODE_MEMBERS"]
R = {name: k for k, name in enumerate(REGIONS)}

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
SIG = {
    "vplmc_version": (I32, []),
    "vplmc_last_error": (ctypes.c_char_p, []),
    "vplmc_default_params": (I32, [ctypes.POINTER(Params)]),
    "vplmc_create": (I32, [I32, P, ctypes.POINTER(P)]),
    "vplmc_destroy": (I32, [P]),
    "vplmc_set_stream": (I32, [P, P]),
    "vplmc_set_occluders": (I32, [P, I32, P, P, P, P]),
    "vplmc_set_triangles": (I32, [P, I32, P]),
    "vplmc_bvh_build": (I32, [I32, P, P, P, P, I32, P, P, P, ctypes.POINTER(I32)]),
    "vplmc_sbvh_build": (I32, [I32, P, I32, P, P, I32, P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "vplmc_plan_create": (I32, [I32, P, P, P, I32, ctypes.POINTER(Params), ctypes.POINTER(P)]),
    "vplmc_plan_create_coarse": (I32, [I32, P, P, ctypes.POINTER(Coarsen), ctypes.POINTER(Params),
                                       ctypes.POINTER(P)]),
    "vplmc_plan_destroy": (I32, [P]),
    "vplmc_workspace_size": (I32, [P, ctypes.POINTER(ctypes.c_size_t)]),
    "vplmc_plan_slice": (I32, [P, I32, ctypes.POINTER(SliceInfo)]),
    "vplmc_plan_region": (I32, [P, I32, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "vplmc_render": (I32, [P, P, ctypes.POINTER(Points), ctypes.POINTER(Lights), ctypes.POINTER(Cut), P, P,
                           ctypes.POINTER(Params), P, ctypes.c_size_t, P]),
    "vplmc_render_static": (I32, [P, P, ctypes.POINTER(Points), ctypes.POINTER(Lights), ctypes.POINTER(Cut), P, P,
                                  ctypes.POINTER(Params), P]),
    "vplmc_read_stats": (I32, [P, P, P, P, P, P, P]),
    "vplmc_read_counts": (I32, [P, P, P, P, P, P]),
    "vplmc_read_totals": (I32, [P, P, P, P]),
    "vplmc_check_inputs": (I32, [P, P, I32, I32, ctypes.POINTER(Cut), P, P, ctypes.POINTER(I64)]),
    "vplmc_cluster_table": (I32, [P, ctypes.POINTER(Lights), ctypes.POINTER(Cut), U64, P, P, P]),
    "vplmc_eval_pairs": (I32, [P, ctypes.POINTER(Points), ctypes.POINTER(Lights), I64, P, P,
                               ctypes.POINTER(Params), P]),
    "vplmc_brute_force": (I32, [P, ctypes.POINTER(Points), ctypes.POINTER(Lights), I32, P,
                                ctypes.POINTER(Params), P]),
    "vplmc_philox4x64": (I32, [P, U64, U64, P, I64, P]),
    "vplmc_lightcut_plan_create": (I32, [ctypes.POINTER(LightTree), I32, I32, ctypes.POINTER(P)]),
    "vplmc_lightcut_plan_destroy": (I32, [P]),
    "vplmc_lightcut_workspace_size": (I32, [P, ctypes.POINTER(ctypes.c_size_t)]),
    "vplmc_lightcut": (I32, [P, P, ctypes.POINTER(Points), ctypes.POINTER(Lights), P, ctypes.c_double,
                             ctypes.c_float, U64, P, ctypes.c_size_t, P, P, P, P, P, P]),
    "vplmc_stage_pass2": (I32, [P, P, ctypes.POINTER(Params), P, ctypes.c_size_t]),
    "vplmc_stage_adm": (I32, [P, P, ctypes.POINTER(Params), P, I32, P, ctypes.c_size_t, P]),
    "vplmc_stage_reduce": (I32, [P, P, P, I32, P, ctypes.c_size_t, P]),
    "vplmc_full_matrix": (I32, [P, P, ctypes.POINTER(Points), P, I32, P, P, ctypes.POINTER(Params), I32, I32, P]),
    "vplmc_mlp_param_count": (I32, []),
    "vplmc_set_proposal": (I32, [P, P]),
    "vplmc_mlp_forward": (I32, [P, P, I64, P, P]),
    "vplmc_mlp_scratch_size": (I32, [I64, ctypes.POINTER(ctypes.c_size_t)]),
    "vplmc_mlp_grad": (I32, [P, P, I64, P, P, P, ctypes.c_size_t, P]),
    "vplmc_mlp_adam": (I32, [P, P, P, P, P, I32, ctypes.c_float]),
    "vplmc_mlp_train_step": (I32, [P, P, P, P, I32, ctypes.c_float, I64, P, P, I32, P, P, ctypes.c_size_t, P]),
    "vplmc_proposal_targets": (I32, [P, P, ctypes.POINTER(Points), P, P, P, ctypes.POINTER(Params), P,
                                     ctypes.c_size_t, P]),
    "vplmc_profile_begin": (I32, [P, I32]),
    "vplmc_profile_end": (I32, [P, P, P]),
    "vplmc_plan_get_tune": (I32, [P, P]),
    "vplmc_plan_set_tune": (I32, [P, P]),
    "vplmc_autotune": (I32, [P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P, I32, P]),
    "vplmc_graph_create": (I32, [P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P, P]),
    "vplmc_graph_launch": (I32, [P, P]),
    "vplmc_graph_destroy": (I32, [P]),
}
N_PHASES = 11
PHASES = ["setup", "cluster", "coarsen", "pass1", "eval1", "weights", "pass2", "eval2", "sort", "adm", "reduce"]

_lib = None


class VplmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vplmc error {code}: {msg}")
        self.code = code


def load():
    """Load libvplmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_12567_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIG.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(rc):
    if rc != 0:
        raise VplmcError(rc, load().vplmc_last_error().decode())
    return rc
