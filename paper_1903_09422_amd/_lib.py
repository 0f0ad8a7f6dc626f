"""ctypes declarations of libkadabra.so (the C ABI in include/kadabra.h).

There is no fallback: if the native library is missing, importing the
binding's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# KADABRA_LIB names another build of the same library (for example one with
# host-side sanitizers); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("KADABRA_LIB") or os.path.join(HERE, "libkadabra.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ERANGE, ECANCELED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
                ESTATE: "ESTATE", ERANGE: "ERANGE", ECANCELED: "ECANCELED"}

# every symbol declared in include/kadabra.h
EXPORTS = (
    "kadabra_create_graph", "kadabra_set_param", "kadabra_get_param", "kadabra_set_stream",
    "kadabra_run", "kadabra_run_static", "kadabra_get_checkpoint", "kadabra_resume", "kadabra_get_scores", "kadabra_get_scores_device", "kadabra_get_decisions",
    "kadabra_get_balance", "kadabra_eval_stop_fg", "kadabra_cancel", "kadabra_destroy_graph", "kadabra_last_error",
    "kadabra_version", "kadabra_autotune", "kadabra_batch_create", "kadabra_batch_set_param",
    "kadabra_batch_get_param", "kadabra_batch_set_stream", "kadabra_batch_add", "kadabra_batch_run",
    "kadabra_batch_autotune", "kadabra_batch_get_scores", "kadabra_batch_clear",
    "kadabra_batch_destroy", "kadabra_server_create", "kadabra_server_set_param",
    "kadabra_server_get_param", "kadabra_server_submit", "kadabra_server_wait",
    "kadabra_server_result", "kadabra_server_release", "kadabra_server_info_get",
    "kadabra_server_destroy",
)
VOID_FUNCS = ("kadabra_destroy_graph", "kadabra_batch_destroy", "kadabra_server_destroy",
              "kadabra_last_error")


class KadabraError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "tau", "omega", "vd_bound", "epochs", "decision", "v_exp", "e_scan", "e_bt",
        "path_interior", "disconnected")] + [
        ("log_inv_delta", C.c_double), ("ms_sampling", C.c_double), ("ms_total", C.c_double),
        ("ms_sample_kernels", C.c_double), ("sample_launches", C.c_int64)] + [
        (k, C.c_int64) for k in ("first_samples", "plan_tau", "first_v_exp", "first_e_scan",
                                 "first_e_bt", "first_path_interior", "first_disconnected",
                                 "v_written")]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Checkpoint(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n", "tau", "epochs", "omega", "check_interval")] + [
        ("eps", C.c_double), ("delta", C.c_double), ("seed", C.c_uint64), ("work", C.c_int64 * 6)]


class ServerInfo(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "submitted", "completed", "failed", "active", "pending", "bytes_in_use",
        "budget_bytes", "peak_active")] + [
        (k, C.c_double) for k in ("p50_ms", "p99_ms", "max_ms", "mean_queue_ms")]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> C.CDLL:
    """Load libkadabra.so and declare its signatures (raises if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"native library {LIB_PATH} is not built; run "
                           "`python -c 'import __graft_entry__ as g; g.build()'` first")
    # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7.  If
    # torch is importable it is loaded first, and the library's dependency on
    # the same soname then resolves to torch's copy (otherwise torch would
    # later load a second runtime that sees no device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
    L.kadabra_create_graph.argtypes = [C.c_int32, C.c_int64, vp, vp, C.POINTER(vp)]
    L.kadabra_set_param.argtypes = [vp, C.c_char_p, C.c_int64]
    L.kadabra_get_param.argtypes = [vp, C.c_char_p, i64p]
    L.kadabra_set_stream.argtypes = [vp, vp]
    L.kadabra_run.argtypes = [vp, C.c_double, C.c_double, C.c_uint64]
    L.kadabra_run_static.argtypes = [vp, C.c_double, C.c_double, C.c_uint64, vp, C.POINTER(Stats)]
    L.kadabra_get_checkpoint.argtypes = [vp, C.POINTER(Checkpoint), vp]
    L.kadabra_resume.argtypes = [vp, C.POINTER(Checkpoint), vp]
    L.kadabra_get_scores.argtypes = [vp, vp, vp, C.POINTER(Stats)]
    L.kadabra_get_scores_device.argtypes = [vp, vp, vp]
    L.kadabra_get_decisions.argtypes = [vp, vp, C.c_int64, i64p]
    L.kadabra_get_balance.argtypes = [vp, vp, vp, vp]
    L.kadabra_eval_stop_fg.argtypes = [C.c_int32, vp, C.c_int64, C.c_int64, C.c_double, vp, vp]
    L.kadabra_cancel.argtypes = [vp]
    L.kadabra_destroy_graph.argtypes = [vp]
    L.kadabra_destroy_graph.restype = None
    L.kadabra_last_error.argtypes = []
    L.kadabra_last_error.restype = C.c_char_p
    L.kadabra_version.argtypes = []
    L.kadabra_autotune.argtypes = [vp, C.c_double, C.c_double, C.c_int64]
    L.kadabra_batch_create.argtypes = [C.POINTER(vp)]
    L.kadabra_batch_set_param.argtypes = [vp, C.c_char_p, C.c_int64]
    L.kadabra_batch_get_param.argtypes = [vp, C.c_char_p, i64p]
    L.kadabra_batch_set_stream.argtypes = [vp, vp]
    L.kadabra_batch_add.argtypes = [vp, vp, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                    C.POINTER(C.c_int32)]
    L.kadabra_batch_run.argtypes = [vp]
    L.kadabra_batch_autotune.argtypes = [vp, C.c_int64]
    L.kadabra_batch_get_scores.argtypes = [vp, C.c_int32, vp, vp, C.POINTER(Stats)]
    L.kadabra_batch_clear.argtypes = [vp]
    L.kadabra_batch_destroy.argtypes = [vp]
    L.kadabra_batch_destroy.restype = None
    L.kadabra_server_create.argtypes = [vp, C.c_int32, C.c_int64, C.c_int32, C.POINTER(vp)]
    L.kadabra_server_set_param.argtypes = [vp, C.c_char_p, C.c_int64]
    L.kadabra_server_get_param.argtypes = [vp, C.c_char_p, i64p]
    L.kadabra_server_submit.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                        i64p]
    L.kadabra_server_wait.argtypes = [vp, C.c_int64, C.c_double, C.POINTER(C.c_int32)]
    L.kadabra_server_result.argtypes = [vp, C.c_int64, vp, vp, C.POINTER(Stats),
                                        C.POINTER(C.c_double)]
    L.kadabra_server_release.argtypes = [vp, C.c_int64]
    L.kadabra_server_info_get.argtypes = [vp, C.POINTER(ServerInfo), C.c_int32]
    L.kadabra_server_destroy.argtypes = [vp]
    L.kadabra_server_destroy.restype = None
    for name in EXPORTS:
        if name not in VOID_FUNCS:
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status: int) -> None:
    if status != OK:
        msg = lib().kadabra_last_error().decode(errors="replace")
        raise KadabraError(status, msg)
