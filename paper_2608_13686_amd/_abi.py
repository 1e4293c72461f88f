"""ctypes mirror of ``include/sfhk.h`` and loader of ``libsfhk.so``."""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsfhk.so")

MAX_GTO = 64
FP64, MIXED = 0, 1
ALIGN_FIXED, ALIGN_COS2M = 0, 1
FS_Q, FS_P, FS_M, FS_S, FS_CRE, FS_CIM, FS_FLIPS = 0, 3, 6, 42, 43, 44, 45
FS_MMAX, FS_NEAR, FS_COUNT = 46, 47, 48

STATUS = {0: "SFHK_OK", 1: "SFHK_E_INVALID", 2: "SFHK_E_NOMEM", 3: "SFHK_E_DEVICE",
          4: "SFHK_E_BUSY", 5: "SFHK_E_UNSUPPORTED"}

EXPORTS = ["sfhk_abi_version", "sfhk_last_error", "sfhk_problem_steps", "sfhk_workspace_bytes",
           "sfhk_footprint_bytes", "sfhk_propagate_static",
           "sfhk_sample_initial", "sfhk_propagate", "sfhk_dipole", "sfhk_spectrum",
           "sfhk_plan_workspace_bytes", "sfhk_plan_create", "sfhk_plan_run", "sfhk_plan_capture",
           "sfhk_plan_replay", "sfhk_plan_destroy", "sfhk_plan_kernel_ms", "sfhk_request_bytes", "sfhk_request_layout",
           "sfhk_request_table_bytes", "sfhk_request_init", "sfhk_serve_window",
           "sfhk_request_run", "sfhk_request_finalize", "sfhk_gabor", "sfhk_return_steps",
           "sfhk_fft_log2_len", "sfhk_spectrum_fft_work_bytes", "sfhk_spectrum_fft",
           "sfhk_acceleration"]


class Center(C.Structure):
    _fields_ = [("Zinf", C.c_double), ("dZ", C.c_double), ("alpha", C.c_double),
                ("eps2", C.c_double)]


class Gto(C.Structure):
    _fields_ = [("center", C.c_int32), ("l", C.c_int32), ("a", C.c_double), ("c", C.c_double)]


class Target(C.Structure):
    _fields_ = [("R", C.c_double), ("Ip", C.c_double), ("ctr", Center * 2),
                ("n_gto", C.c_int32), ("reserved", C.c_int32), ("gto", C.POINTER(Gto))]


class Laser(C.Structure):
    _fields_ = [("lambda_nm", C.c_double), ("intensity_wcm2", C.c_double),
                ("n_cycles", C.c_double), ("cep", C.c_double)]


class Align(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int32), ("theta", C.c_double),
                ("phi", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("tgt", Target), ("las", Laser), ("al", Align), ("dt", C.c_double),
                ("gamma_cs", C.c_double), ("w_cut", C.c_double), ("sigma_perp", C.c_double),
                ("n_steps", C.c_int32), ("ionization", C.c_int32), ("c_max", C.c_double)]


class Ensemble(C.Structure):
    _fields_ = [("capacity", C.c_uint64), ("k0", C.c_void_p), ("prob", C.c_void_p),
                ("qx", C.c_void_p), ("qy", C.c_void_p), ("qz", C.c_void_p),
                ("px", C.c_void_p), ("py", C.c_void_p), ("pz", C.c_void_p),
                ("w", C.c_void_p), ("nx", C.c_void_p), ("ny", C.c_void_p), ("nz", C.c_void_p),
                ("dph", C.c_void_p), ("order", C.c_void_p), ("live_start", C.c_void_p), ("live_count", C.c_void_p),
                ("pack_start", C.c_void_p)]


IONIZATION = {"first_order": 0, "saddle": 1, "saddle_modified": 2}


class Tuning(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("waves_per_cu", C.c_int32),
                ("step_unroll", C.c_int32), ("traj_per_lane", C.c_int32),
                ("lanes_per_traj", C.c_int32)]


_lib = None


def lib():
    """The loaded C library.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(hipcc for gfx950) first")
        L = C.CDLL(LIB_PATH)
        u64p = C.POINTER(C.c_uint64)
        P = C.POINTER(Problem)
        L.sfhk_abi_version.restype = C.c_int32
        L.sfhk_last_error.restype = C.c_char_p
        L.sfhk_problem_steps.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]
        L.sfhk_problem_steps.restype = C.c_int
        L.sfhk_workspace_bytes.argtypes = [P, C.c_int32, C.c_uint64]
        L.sfhk_workspace_bytes.restype = C.c_size_t
        L.sfhk_sample_initial.argtypes = [P, C.c_int32, u64p, u64p, u64p, C.POINTER(Ensemble),
                                          C.c_void_p, C.c_size_t, C.c_void_p]
        L.sfhk_sample_initial.restype = C.c_int
        L.sfhk_footprint_bytes.argtypes = [P, C.c_uint64, C.c_int32]
        L.sfhk_footprint_bytes.restype = C.c_size_t
        L.sfhk_propagate.argtypes = [P, C.c_int32, C.POINTER(Ensemble), C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_size_t, C.c_void_p]
        L.sfhk_propagate.restype = C.c_int
        L.sfhk_propagate_static.argtypes = [P, C.c_int32, C.POINTER(Ensemble), C.c_int32,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                            C.c_int32, C.c_void_p]
        L.sfhk_propagate_static.restype = C.c_int
        L.sfhk_dipole.argtypes = [P, C.c_int32, C.c_void_p, u64p, C.c_void_p, C.c_void_p]
        L.sfhk_dipole.restype = C.c_int
        L.sfhk_spectrum.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double,
                                    C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]
        L.sfhk_spectrum.restype = C.c_int
        L.sfhk_fft_log2_len.argtypes = [C.c_int32]
        L.sfhk_fft_log2_len.restype = C.c_int32
        L.sfhk_spectrum_fft_work_bytes.argtypes = [C.c_int32]
        L.sfhk_spectrum_fft_work_bytes.restype = C.c_size_t
        L.sfhk_spectrum_fft.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double,
                                        C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p]
        L.sfhk_spectrum_fft.restype = C.c_int
        L.sfhk_acceleration.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double,
                                        C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]
        L.sfhk_acceleration.restype = C.c_int
        L.sfhk_plan_workspace_bytes.argtypes = [P, C.c_int32, u64p]
        L.sfhk_plan_workspace_bytes.restype = C.c_size_t
        L.sfhk_plan_create.argtypes = [P, C.c_int32, u64p, u64p, u64p, C.c_int32,
                                       C.POINTER(Tuning), C.c_double, C.c_int32,
                                       C.POINTER(Ensemble), C.c_void_p, C.c_size_t, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.POINTER(C.c_void_p)]
        L.sfhk_plan_create.restype = C.c_int
        for f in ("sfhk_plan_run", "sfhk_plan_capture", "sfhk_plan_replay"):
            getattr(L, f).argtypes = [C.c_void_p, C.c_void_p]
            getattr(L, f).restype = C.c_int
        L.sfhk_plan_kernel_ms.argtypes = [C.c_void_p, C.POINTER(C.c_float)]
        L.sfhk_plan_kernel_ms.restype = C.c_int
        L.sfhk_plan_destroy.argtypes = [C.c_void_p]
        L.sfhk_plan_destroy.restype = None
        L.sfhk_request_bytes.argtypes = [P, C.c_uint64, C.c_int32]
        L.sfhk_request_bytes.restype = C.c_size_t
        L.sfhk_request_layout.argtypes = [P, C.c_uint64, C.c_int32, C.POINTER(C.c_size_t)]
        L.sfhk_request_layout.restype = C.c_int
        L.sfhk_request_table_bytes.argtypes = [C.c_int32]
        L.sfhk_request_table_bytes.restype = C.c_size_t
        L.sfhk_request_init.argtypes = [P, C.c_uint64, C.c_uint64, C.c_uint64, C.c_double,
                                        C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                        C.c_int32, C.c_int32, C.c_void_p]
        L.sfhk_request_init.restype = C.c_int
        i32p = C.POINTER(C.c_int32)
        L.sfhk_serve_window.argtypes = [C.c_void_p, C.c_int32, C.c_int32, i32p, u64p, i32p,
                                        i32p, C.c_int32, C.c_int32, C.c_void_p]
        L.sfhk_serve_window.restype = C.c_int
        L.sfhk_request_run.argtypes = [P, C.c_uint64, C.c_int32, C.c_void_p, C.c_size_t,
                                       C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
        L.sfhk_request_run.restype = C.c_int
        L.sfhk_request_finalize.argtypes = [P, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                            C.c_void_p]
        L.sfhk_request_finalize.restype = C.c_int
        L.sfhk_gabor.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double,
                                 C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]
        L.sfhk_gabor.restype = C.c_int
        L.sfhk_return_steps.argtypes = [P, C.c_int32, C.POINTER(Ensemble), C.c_double,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                        C.c_void_p]
        L.sfhk_return_steps.restype = C.c_int
        _lib = L
    return _lib


class SfhkError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().sfhk_last_error().decode()
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status, where):
    if status != 0:
        raise SfhkError(status, where)


def make_problems(dicts):
    """ctypes array of sfhk_problem from workload dictionaries; the GTO arrays
    are attached to the returned object so that they outlive the call."""
    arr = (Problem * len(dicts))()
    keep = []
    for P, d in zip(arr, dicts):
        las, tgt, al = d["laser"], d["target"], d["align"]
        P.las = Laser(las["lambda_nm"], las["intensity_wcm2"], las["n_cycles"], las["cep"])
        gt = (Gto * len(tgt["gto"]))(*[Gto(int(c), int(l), a, cc) for (c, l, a, cc) in tgt["gto"]])
        keep.append(gt)
        P.tgt.R = tgt["R"]
        P.tgt.Ip = tgt["Ip"]
        for i, c in enumerate(tgt["centers"]):
            P.tgt.ctr[i] = Center(c["Zinf"], c["dZ"], c["alpha"], c["eps2"])
        P.tgt.n_gto = len(tgt["gto"])
        P.tgt.gto = C.cast(gt, C.POINTER(Gto))
        P.al = Align(ALIGN_FIXED if al["kind"] == "fixed" else ALIGN_COS2M, int(al.get("m", 0)),
                     al.get("theta", 0.0), al.get("phi", 0.0))
        P.dt = d["dt"]
        P.gamma_cs = d["gamma"]
        P.w_cut = d["w_cut"]
        P.sigma_perp = d["sigma_perp"]
        P.n_steps = int(d.get("n_steps", 0))
        P.c_max = float(d.get("c_max", 0.0))
        P.ionization = IONIZATION[d.get("ionization", "first_order")]
    arr._keep = keep
    return arr


def u64_array(values):
    vals = [int(v) for v in values]
    return (C.c_uint64 * len(vals))(*vals)
