"""ctypes declarations of the C ABI in ``include/swccl.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswccl.so")

ABI_VERSION = 7  # the SWCCL_ABI_VERSION these declarations follow

# status codes
SW_OK, SW_ERR_ARG, SW_ERR_SIZE, SW_ERR_WORKSPACE, SW_ERR_DEVICE, SW_ERR_STATE, SW_ERR_UNSUPPORTED, SW_ERR_HOST_MEMORY = range(8)
SW_SPIN_ISING_I8, SW_SPIN_POTTS_U8 = 0, 1
SW_F_KEEP_SPINS, SW_F_SIZES, SW_F_REVERSE_TILES, SW_F_BATCH_FUSED = 1, 2, 4, 8
CCL_BONDS_PERIODIC, CCL_BONDS_OPEN, CCL_SITES_OPEN = 0, 1, 2
CCL_NOALLOC_SCRATCH_BYTES = 64 << 20
TILE_HEIGHTS = (16, 32, 64, 128)  # sw_params.tile_h (0: 64)
MERGE_WAVES = (4, 8, 16)          # sw_params.merge_waves (0: 8)
SW_PHASE_TILE, SW_PHASE_MERGE, SW_PHASE_FLIP = 0, 1, 2
SW_HIST_ACTIVE, SW_HIST_NCLUST, SW_HIST_MAXCL, SW_HIST_NSAT, SW_HIST_COUNTS, SW_HIST_LEN = 0, 1, 2, 3, 4, 12
SW3_REC_ACTIVE, SW3_REC_NCLUST, SW3_REC_NSAT, SW3_REC_COUNTS, SW3_REC_LEN = 0, 1, 2, 3, 11


class SwParams(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_int32),
        ("H", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("spin_kind", ctypes.c_int32),
        ("K", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("tile_h", ctypes.c_int32),
        ("merge_waves", ctypes.c_int32),
        ("p_flip", ctypes.c_double),
        ("few_b", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class SwBuffers(ctypes.Structure):
    _fields_ = [
        ("spins", ctypes.c_void_p),
        ("labels", ctypes.c_void_p),
        ("bonds", ctypes.c_void_p),
        ("roots", ctypes.c_void_p),
        ("sizes", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class SwObs(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_uint64),
        ("threshold", ctypes.c_uint64),
        ("n_sat", ctypes.c_int64),
        ("magnet", ctypes.c_int64),
        ("counts", ctypes.c_int64 * 8),
        ("n_active_bonds", ctypes.c_int64),
        ("n_clusters", ctypes.c_int64),
        ("max_cluster", ctypes.c_int64),
        ("digest_spins", ctypes.c_uint64),
        ("digest_labels", ctypes.c_uint64),
        ("digest_bonds", ctypes.c_uint64),
    ]


class Sw3Params(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32),
        ("Ly", ctypes.c_int32),
        ("Lz", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("spin_kind", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("K", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint32),
        ("reserved", ctypes.c_int32),
    ]


class CclServerParams(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("sizes", ctypes.c_int32),
        ("max_inflight", ctypes.c_int32),
        ("n_streams", ctypes.c_int32),
        ("batch_px", ctypes.c_int32),
    ]


class SwccLError(RuntimeError):
    """A non-zero sw_status from the library (``status``)."""

    def __init__(self, message: str, status: int = 0):
        super().__init__(message)
        self.status = int(status)


_lib = None

# name -> (restype, argtypes); every function declared in include/swccl.h
SIGNATURES = {
    "swccl_abi_version": (ctypes.c_int32, []),
    "sw_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "sw_last_error": (ctypes.c_char_p, []),
    "sw_threshold": (ctypes.c_uint64, [ctypes.c_double]),
    "sw_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SwParams)]),
    "sw_init": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(SwParams),
                                 ctypes.POINTER(SwBuffers), ctypes.c_void_p]),
    "sw_sweep": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "sw_sweep_phase": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "sw_sweep_history": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sw_observables": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(SwObs), ctypes.c_void_p]),
    "sw_get_t": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "sw_set_t": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64]),
    "sw_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "swb_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SwParams), ctypes.c_int32]),
    "swb_init": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(SwParams),
                                  ctypes.POINTER(SwBuffers), ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]),
    "swb_sweep": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "swb_sweep_graph": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "swb_observables": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(SwObs), ctypes.c_void_p]),
    "swb_get_t": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "swb_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "ccl_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "ccl_workspace_bytes_tiled": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_int32]),
    "ccl_label_tiled": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p]),
    "ccl_server_footprint": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(CclServerParams)]),
    "ccl_server_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(CclServerParams),
                                           ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "ccl_server_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_size_t, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "ccl_server_flush": (ctypes.c_int32, [ctypes.c_void_p]),
    "ccl_server_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "ccl_server_result": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "ccl_server_release": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "ccl_server_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "ccl_label": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "sw3_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Sw3Params)]),
    "sw3_init_spins": (ctypes.c_int32, [ctypes.POINTER(Sw3Params), ctypes.c_void_p, ctypes.c_void_p]),
    "sw3_sweep": (ctypes.c_int32, [ctypes.POINTER(Sw3Params), ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p]),
    "ccl3_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "ccl3_label": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "ccl_label_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
}


def lib():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
            )
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.swccl_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI {L.swccl_abi_version()}, expected {ABI_VERSION}: rebuild it")
        _lib = L
    return _lib


def check(status: int, what: str) -> None:
    if status != SW_OK:
        L = lib()
        msg = L.sw_status_string(status).decode()
        extra = L.sw_last_error().decode() if status == SW_ERR_DEVICE else ""
        raise SwccLError(f"{what}: {msg} ({status}) {extra}".strip(), status)
