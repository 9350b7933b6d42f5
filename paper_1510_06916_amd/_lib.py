"""ctypes declarations of include/nxgraph.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnxgraph.so")

NXG_OK, NXG_EINVAL, NXG_ENOMEM, NXG_EDEVICE, NXG_ENOTCONV, NXG_EUNSUPPORTED = range(6)
STATUS_NAMES = {0: "NXG_OK", 1: "NXG_EINVAL", 2: "NXG_ENOMEM", 3: "NXG_EDEVICE",
                4: "NXG_ENOTCONV", 5: "NXG_EUNSUPPORTED"}

NXG_BUILD_KEEP_PERM = 0x1
NXG_BUILD_TRANSPOSE = 0x2
NXG_BUILD_SYMMETRIZE = 0x4
NXG_BUILD_DEDUP = 0x8
NXG_BUILD_RELABEL = 0x10
NXG_BUILD_SCATTER = 0x20
NXG_BUILD_DEGREE = 0x40
NXG_BUILD_HOST_STREAM = 0x80
NXG_BUILD_PAIRS = 0x100
NXG_BUILD_SHUFFLE_SCHEDULE = 0x200

NXG_PAGERANK, NXG_PAGERANK_WEIGHTED, NXG_BFS, NXG_WCC, NXG_SCC = range(5)
NXG_F32, NXG_F64, NXG_I32 = range(3)
NXG_RUN_WARM_START = 0x1
NXG_RUN_PERSISTENT = 0x2
NXG_RUN_CAPTURE = 0x4
NXG_RUN_SCATTER = 0x8
NXG_RUN_MPU = 0x10
NXG_ORDER_DST, NXG_ORDER_SRC = 0, 1


class BuildDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("d_src", ctypes.c_void_p),
                ("d_dst", ctypes.c_void_p), ("d_weight", ctypes.c_void_p),
                ("interval", ctypes.c_int32), ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("value_bytes", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("order", ctypes.c_int32)]


class DsssInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("interval", ctypes.c_int32),
                ("P", ctypes.c_int32), ("tile", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("n_chunks", ctypes.c_int64),
                ("n_words", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("max_tile_edges", ctypes.c_int64), ("has_perm", ctypes.c_int32),
                ("has_weights", ctypes.c_int32), ("has_transpose", ctypes.c_int32),
                ("order", ctypes.c_int32), ("relabeled", ctypes.c_int32),
                ("n_kept", ctypes.c_int32), ("pairs", ctypes.c_int32)]


class RunDesc(ctypes.Structure):
    _fields_ = [("program", ctypes.c_int), ("dtype", ctypes.c_int), ("batch", ctypes.c_int32),
                ("damping", ctypes.c_double), ("max_iters", ctypes.c_int32),
                ("tol", ctypes.c_double), ("d_teleport", ctypes.c_void_p),
                ("roots", ctypes.c_void_p), ("d_values", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("d_seeds", ctypes.c_void_p),
                ("piece_chunks", ctypes.c_int32), ("d_stats", ctypes.c_void_p),
                ("vertex_budget", ctypes.c_int64)]


class RunStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("residual", ctypes.c_double), ("max_level", ctypes.c_int32),
                ("changed_rounds", ctypes.c_int32), ("reached_edges", ctypes.c_int64),
                ("device_ms", ctypes.c_double), ("streamed_chunks", ctypes.c_int64),
                ("resident_intervals", ctypes.c_int32), ("host_read_bytes", ctypes.c_int64),
                ("host_write_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AdjointDesc(ctypes.Structure):
    _fields_ = [("damping", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("d_xstar", ctypes.c_void_p),
                ("d_gx", ctypes.c_void_p), ("d_lambda", ctypes.c_void_p),
                ("d_gw", ctypes.c_void_p), ("d_gt", ctypes.c_void_p)]


class TuneResult(ctypes.Structure):
    _fields_ = [("interval", ctypes.c_int32), ("tile", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("order", ctypes.c_int32), ("piece_chunks", ctypes.c_int32),
                ("ms_per_iter", ctypes.c_double), ("candidates", ctypes.c_int32),
                ("relabel", ctypes.c_int32), ("pairs", ctypes.c_int32), ("width", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                           ctypes.c_void_p)

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "nxg_set_allocator": (ctypes.c_int, [ALLOC_FN, FREE_FN, ctypes.c_void_p]),
    "nxg_last_error": (ctypes.c_char_p, []),
    "nxg_abi_version": (ctypes.c_int, []),
    "nxg_dsss_build": (ctypes.c_int, [ctypes.POINTER(BuildDesc), ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "nxg_dsss_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nxg_dsss_info_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(DsssInfo)]),
    "nxg_dsss_vertex_map": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nxg_dsss_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "nxg_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RunDesc), ctypes.c_void_p,
                               ctypes.POINTER(RunStats)]),
    "nxg_dsss_set_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nxg_multi_build": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(BuildDesc), ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "nxg_multi_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RunDesc),
                                     ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                     ctypes.POINTER(RunStats)]),
    "nxg_multi_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nxg_copy_probe": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double)]),
    "nxg_read_probe": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double)]),
    "nxg_tune": (ctypes.c_int, [ctypes.POINTER(BuildDesc), ctypes.c_int, ctypes.c_int, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.POINTER(TuneResult)]),
    "nxg_pagerank_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AdjointDesc),
                                            ctypes.c_void_p, ctypes.POINTER(RunStats)]),
    "nxg_run_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RunDesc), ctypes.c_void_p,
                                       ctypes.POINTER(RunStats)]),
    "nxg_noalloc_scratch_bytes": (ctypes.c_size_t, []),
}

_lib = None


def lib():
    """Loads libnxgraph.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnxgraph.so is not built: run paper_1510_06916_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class NxgError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().nxg_last_error().decode()
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status, where, allow=()):
    if status != NXG_OK and status not in allow:
        raise NxgError(status, where)
    return status
