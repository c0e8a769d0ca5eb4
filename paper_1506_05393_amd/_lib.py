"""ctypes declarations of libmrf's C ABI (include/libmrf.h).

Argument marshalling only: every step of the method runs in the HIP library.
Importing this module fails loudly when libmrf.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrf.so")

MRF_OK = 0
MRF_F32, MRF_BF16, MRF_F32_ROWS = 0, 1, 2
STATUS = {0: "MRF_OK", 1: "MRF_ERR_INVALID", 2: "MRF_ERR_OOM", 3: "MRF_ERR_DEVICE",
          4: "MRF_ERR_NOT_READY", 5: "MRF_ERR_REJECTED", 6: "MRF_ERR_UNSUPPORTED",
          7: "MRF_ERR_CANCELLED"}


class MRFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SequenceDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("fa_deg", C.POINTER(C.c_double)),
                ("phase_deg", C.POINTER(C.c_double)), ("tr_ms", C.POINTER(C.c_double)),
                ("te_ms", C.POINTER(C.c_double)), ("inversion", C.c_int32),
                ("ti_ms", C.c_double), ("smooth", C.c_int32)]


class Axis(C.Structure):
    _fields_ = [("n", C.c_int32), ("v", C.POINTER(C.c_double))]


class GridDesc(C.Structure):
    _fields_ = [("t1_ms", Axis), ("t2_ms", Axis), ("df_hz", Axis), ("b1", Axis)]


class DictView(C.Structure):
    _fields_ = [("dtype", C.c_int), ("n_tr", C.c_int32), ("n_entries", C.c_int64),
                ("ld", C.c_int64), ("re", C.c_void_p), ("im", C.c_void_p),
                ("norm", C.c_void_p), ("entry_base", C.c_int64)]


class ResultView(C.Structure):
    _fields_ = [("idx", C.c_void_p), ("cc", C.c_void_p), ("margin", C.c_void_p),
                ("pd_re", C.c_void_p), ("pd_im", C.c_void_p), ("n_sim", C.c_void_p)]


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("mrf_status_str", C.c_char_p, [C.c_int]),
    ("mrf_last_error", C.c_char_p, []),
    ("mrf_version", C.c_char_p, []),
    ("mrf_context_create", C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    ("mrf_context_destroy", C.c_int, [C.c_void_p]),
    ("mrf_sequence_create", C.c_int, [C.c_void_p, C.POINTER(SequenceDesc), C.POINTER(C.c_void_p)]),
    ("mrf_sequence_destroy", C.c_int, [C.c_void_p]),
    ("mrf_grid_size", C.c_int64, [C.POINTER(GridDesc)]),
    ("mrf_simulate_dictionary", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(GridDesc), C.c_int32, C.c_int64, C.c_int64, C.c_int,
      C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
    ("mrf_simulate_dictionary_pair", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(GridDesc), C.c_int32, C.c_int64, C.c_int64, C.c_void_p,
      C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("mrf_cc_map", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(GridDesc), C.c_int32, C.c_void_p, C.c_int32, C.c_int64,
      C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    ("mrf_smooth_signals", C.c_int,
     [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int64, C.c_int32,
      C.c_int32, C.c_void_p]),
    ("mrf_simulate_signals", C.c_int,
     [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
      C.c_void_p]),
    ("mrf_match_workspace", C.c_int,
     [C.c_void_p, C.POINTER(DictView), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    ("mrf_match_bruteforce", C.c_int,
     [C.c_void_p, C.POINTER(DictView), C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_void_p,
      C.POINTER(GridDesc), ResultView, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
      C.c_void_p]),
    ("mrf_zoom_schedule_finest_objective", C.c_int, [C.c_void_p, C.c_int32]),
    ("mrf_zoom_schedule_multistart", C.c_int,
     [C.POINTER(GridDesc), C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    ("mrf_static_scratch_bytes", C.c_size_t, []),
    ("mrf_match_bruteforce_noalloc", C.c_int,
     [C.c_void_p, C.POINTER(DictView), C.c_void_p, C.c_int32, C.c_int64, C.c_int32, ResultView,
      C.c_void_p, C.c_void_p, C.c_void_p]),
    ("mrf_probe_mfma", C.c_int,
     [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.c_void_p]),
    ("mrf_probe_mfma_varied", C.c_int,
     [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.c_void_p]),
    ("mrf_probe_write", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_uint32, C.c_void_p]),
    ("mrf_profile_enable", C.c_int, [C.c_void_p, C.c_int32]),
    ("mrf_profile_read", C.c_int,
     [C.c_void_p, C.c_char_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
]


def load():
    """Load libmrf.so and declare every exported symbol (raises if missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libmrf.so is not built ({LIB_PATH}); run "
                              "python -c 'import __graft_entry__; __graft_entry__.build()'")
        lib = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_names():
    return [s[0] for s in _SIGS]


def check(status: int):
    if status != MRF_OK:
        msg = load().mrf_last_error().decode(errors="replace")
        raise MRFError(status, msg)


ZOOM_MAX_STAGES, ZOOM_MAX_STARTS = 32, 16


class ZoomStage(C.Structure):
    _fields_ = [("kind", C.c_int32), ("axis0", C.c_int32), ("axis1", C.c_int32),
                ("step0", C.c_int32), ("step1", C.c_int32), ("window", C.c_int32),
                ("hop", C.c_double), ("objective", C.c_int32)]


OBJ_CC, OBJ_DIST = 0, 1


class ZoomSchedule(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("stages", ZoomStage * ZOOM_MAX_STAGES),
                ("n_outer", C.c_int32), ("outer", ZoomStage * ZOOM_MAX_STAGES),
                ("outer_max", C.c_int32), ("n_starts", C.c_int32),
                ("starts", (C.c_int32 * 4) * ZOOM_MAX_STARTS), ("pruned", C.c_int32),
                ("prior_half", C.c_int32 * 4)]


_SIGS += [
    ("mrf_zoom_schedule_paper", C.c_int,
     [C.POINTER(GridDesc), C.c_void_p, C.POINTER(ZoomSchedule)]),
    ("mrf_zoom_schedule_local", C.c_int,
     [C.POINTER(GridDesc), C.c_int32, C.POINTER(ZoomSchedule)]),
    ("mrf_zoom_schedule_prior", C.c_int,
     [C.POINTER(GridDesc), C.POINTER(C.c_double), C.POINTER(ZoomSchedule)]),
    ("mrf_zoom_workspace", C.c_int,
     [C.c_void_p, C.POINTER(GridDesc), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    ("mrf_zoom_search", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(GridDesc), C.POINTER(ZoomSchedule), C.c_void_p,
      C.c_int32, C.c_int64, C.c_int32, C.c_void_p, ResultView, C.c_void_p, C.c_size_t,
      C.c_void_p]),
    ("mrf_zoom_search_ragged", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(GridDesc), C.POINTER(ZoomSchedule), C.c_void_p,
      C.c_int32, C.c_int64, C.c_int32, C.c_void_p, ResultView, C.c_void_p, C.c_size_t,
      C.c_void_p]),
    ("mrf_zoom_search_dict", C.c_int,
     [C.c_void_p, C.POINTER(DictView), C.POINTER(GridDesc), C.POINTER(ZoomSchedule), C.c_void_p,
      C.c_int32, C.c_int64, C.c_int32, C.c_void_p, ResultView, C.c_void_p, C.c_size_t,
      C.c_void_p]),
    ("mrf_zoom_search_lattice", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(GridDesc), C.POINTER(ZoomSchedule), C.c_void_p,
      C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_int32, ResultView, C.c_void_p,
      C.c_size_t, C.c_void_p]),
    ("mrf_zoom_search_from", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(GridDesc), C.POINTER(ZoomSchedule), C.c_void_p,
      C.c_int32, C.c_int64, C.c_int32, C.c_void_p, ResultView, C.c_void_p, C.c_size_t,
      C.c_void_p]),
]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_inflight", C.c_int32),
                ("n_streams", C.c_int32), ("max_batch_vox", C.c_int32),
                ("fake_device", C.c_int32), ("fake_ns_per_byte", C.c_double),
                ("fake_fail_ticket", C.c_uint64), ("refine_bf16", C.c_int32),
                ("batch_window_ms", C.c_double)]


class Request(C.Structure):
    _fields_ = [("mode", C.c_int32), ("slot", C.c_int32), ("n_tr", C.c_int32),
                ("n_vox", C.c_int32), ("vox", C.c_void_p), ("ld_vox", C.c_int64),
                ("out", ResultView)]


class ServerStats(C.Structure):
    _fields_ = [("budget_bytes", C.c_size_t), ("resident_bytes", C.c_size_t),
                ("reserved_bytes", C.c_size_t), ("peak_reserved_bytes", C.c_size_t),
                ("arena_peak_bytes", C.c_size_t), ("submitted", C.c_int64),
                ("rejected", C.c_int64), ("done", C.c_int64), ("failed", C.c_int64),
                ("cancelled", C.c_int64), ("batches", C.c_int64),
                ("max_batch_requests", C.c_int64), ("peak_inflight", C.c_int32),
                ("admitted", C.c_int64), ("mode_batches", C.c_int64 * 2),
                ("mode_requests", C.c_int64 * 2), ("mixed_length_batches", C.c_int64 * 2)]


SERVE_BRUTE, SERVE_ZOOM = 0, 1
REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}

_SIGS += [
    ("mrf_server_create", C.c_int,
     [C.c_void_p, C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]),
    ("mrf_server_register", C.c_int,
     [C.c_void_p, C.c_void_p, C.POINTER(GridDesc), C.c_int, C.POINTER(C.c_int32), C.c_int32,
      C.POINTER(C.c_int32)]),
    ("mrf_serve_submit", C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    ("mrf_serve_poll", C.c_int,
     [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double),
      C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("mrf_serve_cancel", C.c_int, [C.c_void_p, C.c_uint64]),
    ("mrf_server_stats_read", C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    ("mrf_server_destroy", C.c_int, [C.c_void_p]),
]
