"""ctypes wrapper of the plain CPU oracle (kadabra_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg; never by the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kadabra_oracle.c")
# ORACLE_LIB names another build of the oracle (for example one with
# sanitizers); by default the in-tree build is loaded.
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fPIC", "-shared", "-pthread"]


SAN_LIB = os.path.join(os.path.dirname(_HERE), "_build", "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer"]


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no contraction).  With
    sanitize, an AddressSanitizer + UndefinedBehaviorSanitizer build goes to
    _build/liboracle_san.so (load it with ORACLE_LIB and gcc's libasan and
    libubsan preloaded)."""
    if sanitize:
        os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
        flags = [f for f in CFLAGS if f != "-O2"] + SAN_FLAGS
        subprocess.check_call(["gcc", *flags, _SRC, "-o", SAN_LIB, "-lm"])
        return SAN_LIB
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "tau", "omega", "vd", "epochs", "v_exp", "e_scan", "v_new", "e_pred", "e_bt",
        "path_interior", "disconnected", "rescaled_levels")] + [("L", C.c_double)] + [
        (k, C.c_int64) for k in ("first_samples", "plan_tau", "first_v_exp", "first_e_scan",
                                 "first_e_bt", "first_path_interior", "first_disconnected")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SampleInfo(C.Structure):
    _fields_ = [("s", C.c_int32), ("t", C.c_int32), ("d", C.c_int32), ("meet_size", C.c_int32),
                ("meet_vertex", C.c_int32), ("meet_shift", C.c_int32), ("meet_total", C.c_uint64),
                ("sigma_w", C.c_uint64 * 4), ("side_x_last", C.c_int32),
                ("sigma_scale", C.c_int32)]

    @property
    def sigma(self) -> int:
        """Sum over the meeting set of m_s m_t (sigma_st / 2^sigma_scale)."""
        return sum(int(self.sigma_w[k]) << (64 * k) for k in range(4))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_uniform64.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32]
        L.oracle_uniform64.restype = C.c_uint64
        L.oracle_pair.argtypes = [C.c_uint64, C.c_uint64, C.c_int32, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]
        L.oracle_pairs.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int32, i32p, i32p]
        L.oracle_components.argtypes = [C.c_int32, i32p, i32p, i32p]
        L.oracle_components.restype = C.c_int32
        L.oracle_vd_bound.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32]
        L.oracle_vd_bound.restype = C.c_int32
        L.oracle_omega.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.oracle_omega.restype = C.c_int64
        L.oracle_log_inv_delta.argtypes = [C.c_int32, C.c_double]
        L.oracle_log_inv_delta.restype = C.c_double
        L.oracle_fg.argtypes = [C.c_int32, C.c_int64, C.c_int64, C.c_double,
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_fg_batch.argtypes = [C.c_int64, i32p, C.c_int64, C.c_int64, C.c_double, f64p, f64p]
        L.oracle_check_stop.argtypes = [C.c_int32, i32p, C.c_int64, C.c_int64, C.c_double,
                                        C.c_double]
        L.oracle_check_stop.restype = C.c_int
        L.oracle_setup.argtypes = [C.c_int32, i32p, i32p, C.c_double, C.c_double, i32p,
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]
        L.oracle_run_threads.argtypes = [C.c_int32, i32p, i32p, C.c_double, C.c_double, C.c_uint64,
                                         C.c_int64, C.c_int32, i32p, C.POINTER(Stats),
                                         np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS"), C.c_int64]
        L.oracle_run.argtypes = [C.c_int32, i32p, i32p, C.c_double, C.c_double, C.c_uint64,
                                 C.c_int64, C.c_int64, i32p, C.POINTER(Stats),
                                 np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS"), C.c_int64]
        L.oracle_check_stop_v.argtypes = [C.c_int32, i32p, C.c_int64, C.c_int64, f64p, f64p,
                                          C.c_double]
        L.oracle_check_stop_v.restype = C.c_int
        L.oracle_first_phase_samples.argtypes = [C.c_int64]
        L.oracle_first_phase_samples.restype = C.c_int64
        L.oracle_plan_lfg.argtypes = [C.c_double, C.c_int64, C.c_int64, C.c_double,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_plan_sum.argtypes = [C.c_int32, i32p, C.c_int64, C.c_int64, C.c_int64, C.c_double]
        L.oracle_plan_sum.restype = C.c_double
        L.oracle_plan.argtypes = [C.c_int32, i32p, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                  C.c_double, f64p, f64p]
        L.oracle_plan.restype = C.c_int64
        L.oracle_run_balanced.argtypes = [
            C.c_int32, i32p, i32p, C.c_double, C.c_double, C.c_uint64, C.c_int64, C.c_int64,
            C.c_int64, i32p, C.POINTER(Stats), np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS"),
            C.c_int64, f64p, f64p, i32p]
        L.oracle_sample.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_uint64, C.c_uint64, i32p,
                                    C.POINTER(SampleInfo)]
        L.oracle_sample.restype = C.c_int32
        L.oracle_sample_pair.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_uint64, C.c_int32,
                                         C.c_int32, C.c_uint64, C.c_int64, C.c_int32, i32p, i32p,
                                         C.POINTER(SampleInfo)]
        L.oracle_sample_pair.restype = C.c_int32
        L.oracle_accumulate.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_uint64, C.c_uint64,
                                        C.c_uint64, i64p]
        L.oracle_accumulate.restype = C.c_int64
        L.oracle_brandes.argtypes = [C.c_int32, i32p, i32p, f64p]
        L.oracle_bfs_sigma.argtypes = [C.c_int32, i32p, i32p, C.c_int32, i32p, f64p]
        _lib = L
    return _lib


def _csr(g):
    return (int(g.n), np.ascontiguousarray(g.row_ptr, dtype=np.int32),
            np.ascontiguousarray(g.col, dtype=np.int32))


def philox4x32_10(ctr, key) -> tuple:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(c, k, out)
    return tuple(int(x) for x in out)


def uniform64(seed: int, i: int, j: int) -> int:
    return int(lib().oracle_uniform64(seed, i, j))


def pair(seed: int, i: int, n: int) -> tuple:
    s, t = C.c_int32(), C.c_int32()
    lib().oracle_pair(seed, i, n, C.byref(s), C.byref(t))
    return s.value, t.value


def pairs(seed: int, i0: int, count: int, n: int) -> tuple:
    s = np.zeros(count, dtype=np.int32)
    t = np.zeros(count, dtype=np.int32)
    lib().oracle_pairs(seed, i0, count, n, s, t)
    return s, t


def components(g) -> tuple:
    n, rp, col = _csr(g)
    comp = np.zeros(n, dtype=np.int32)
    k = lib().oracle_components(n, rp, col, comp)
    return k, comp


def setup(g, eps: float, delta: float) -> dict:
    n, rp, col = _csr(g)
    comp = np.zeros(n, dtype=np.int32)
    vd, om, L = C.c_int32(), C.c_int64(), C.c_double()
    rc = lib().oracle_setup(n, rp, col, eps, delta, comp, C.byref(vd), C.byref(om), C.byref(L))
    if rc != 0:
        raise ValueError("oracle_setup rejected its input")
    return {"comp": comp, "vd": vd.value, "omega": om.value, "L": L.value}


def omega(vd: int, eps: float, delta: float) -> int:
    return int(lib().oracle_omega(vd, eps, delta))


def log_inv_delta(n: int, delta: float) -> float:
    return float(lib().oracle_log_inv_delta(n, delta))


def fg(c: int, tau: int, omega_: int, L: float) -> tuple:
    f, g = C.c_double(), C.c_double()
    lib().oracle_fg(c, tau, omega_, L, C.byref(f), C.byref(g))
    return f.value, g.value


def fg_batch(counts, tau: int, omega_: int, L: float) -> tuple:
    """fg of every counter at one (tau, omega, L): two float64 arrays."""
    c = np.ascontiguousarray(counts, dtype=np.int32)
    f = np.empty(c.size, dtype=np.float64)
    g = np.empty(c.size, dtype=np.float64)
    lib().oracle_fg_batch(c.size, c, tau, omega_, L, f, g)
    return f, g


def check_stop(counts, tau: int, omega_: int, L: float, eps: float) -> bool:
    c = np.ascontiguousarray(counts, dtype=np.int32)
    return bool(lib().oracle_check_stop(c.size, c, tau, omega_, L, eps))


def check_stop_v(counts, tau: int, omega_: int, LL, LU, eps: float) -> bool:
    """The stopping rule with per-vertex log(1/delta_L(v)), log(1/delta_U(v))."""
    c = np.ascontiguousarray(counts, dtype=np.int32)
    LL = np.ascontiguousarray(LL, dtype=np.float64)
    LU = np.ascontiguousarray(LU, dtype=np.float64)
    return bool(lib().oracle_check_stop_v(c.size, c, tau, omega_, LL, LU, eps))


# First-phase sample m is sample index FIRST_PHASE_BASE + m (a stream the
# adaptive loop never reaches).
FIRST_PHASE_BASE = 1 << 63


def first_phase_samples(omega_: int) -> int:
    return int(lib().oracle_first_phase_samples(omega_))


def plan_lfg(b: float, t: int, omega_: int, eps: float) -> tuple:
    """Largest log(1/delta_L), log(1/delta_U) with f, g <= eps at (b, t)."""
    lf, lg = C.c_double(), C.c_double()
    lib().oracle_plan_lfg(b, t, omega_, eps, C.byref(lf), C.byref(lg))
    return lf.value, lg.value


def plan_sum(c1, m1: int, t: int, omega_: int, eps: float) -> float:
    c = np.ascontiguousarray(c1, dtype=np.int32)
    return float(lib().oracle_plan_sum(c.size, c, m1, t, omega_, eps))


def plan(c1, m1: int, omega_: int, eps: float, delta: float, L: float) -> tuple:
    """(t*, LL, LU) of the balancing rule; t* = 0: no plan, uniform L."""
    c = np.ascontiguousarray(c1, dtype=np.int32)
    LL = np.zeros(c.size)
    LU = np.zeros(c.size)
    t = lib().oracle_plan(c.size, c, m1, omega_, eps, delta, L, LL, LU)
    return int(t), LL, LU


@dataclass
class RunResult:
    tau: int
    counts: np.ndarray
    stats: dict
    decisions: np.ndarray  # per boundary: 0 = continue, 1 = stop rule met, 2 = omega reached
    LL: np.ndarray = None  # balanced runs: log(1/delta_L(v)), log(1/delta_U(v)), first-phase counts
    LU: np.ndarray = None
    c1: np.ndarray = None

    @property
    def scores(self) -> np.ndarray:
        return self.counts.astype(np.float64) / float(self.tau)


def run(g, eps: float, delta: float, seed: int, check_interval: int,
        sample_cap: int = -1, first_samples: int = 0) -> RunResult:
    """The adaptive loop.  first_samples: 0 = uniform constants; -1 = balanced
    with the default first phase; > 0 = balanced with that many samples."""
    n, rp, col = _csr(g)
    counts = np.zeros(n, dtype=np.int32)
    st = Stats()
    dec = np.full(1 << 16, -1, dtype=np.int8)
    LL, LU = np.zeros(n), np.zeros(n)
    c1 = np.zeros(n, dtype=np.int32)
    rc = lib().oracle_run_balanced(n, rp, col, eps, delta, seed, check_interval, sample_cap,
                                   first_samples, counts, C.byref(st), dec, dec.size, LL, LU, c1)
    if rc != 0:
        raise ValueError(f"oracle_run failed ({rc})")
    ne = min(int(st.epochs), dec.size)
    r = RunResult(tau=int(st.tau), counts=counts, stats=st.as_dict(), decisions=dec[:ne].copy())
    if first_samples != 0:
        r.LL, r.LU, r.c1 = LL, LU, c1
    return r


def run_threads(g, eps: float, delta: float, seed: int, check_interval: int, threads: int) -> RunResult:
    """The adaptive loop on `threads` host threads (per-thread counter frames
    of each epoch's samples, split by index, added at every boundary)."""
    n, rp, col = _csr(g)
    counts = np.zeros(n, dtype=np.int32)
    st = Stats()
    dec = np.full(1 << 16, -1, dtype=np.int8)
    rc = lib().oracle_run_threads(n, rp, col, eps, delta, seed, check_interval, threads, counts,
                                  C.byref(st), dec, dec.size)
    if rc != 0:
        raise ValueError(f"oracle_run_threads failed ({rc})")
    ne = min(int(st.epochs), dec.size)
    return RunResult(tau=int(st.tau), counts=counts, stats=st.as_dict(), decisions=dec[:ne].copy())


def sample(g, comp, seed: int, i: int):
    """One sample: (interior vertices in path order or None, SampleInfo)."""
    n, rp, col = _csr(g)
    out = np.zeros(max(n, 1), dtype=np.int32)
    info = SampleInfo()
    k = lib().oracle_sample(n, rp, col, np.ascontiguousarray(comp, dtype=np.int32), seed, i,
                            out, C.byref(info))
    if k == -2:
        raise MemoryError
    return (None if k < 0 else out[:k].copy()), info


def sample_pair(g, comp, seed: int, s: int, t: int, i0: int, count: int):
    """count samples (indices i0 ...) at the fixed pair (s, t): (interior
    vertices per sample as a (count, d - 1) array, meeting vertex per sample,
    SampleInfo of the first sample)."""
    n, rp, col = _csr(g)
    stride = max(n, 1)
    paths = np.zeros((count, stride), dtype=np.int32)
    meet = np.zeros(count, dtype=np.int32)
    info = SampleInfo()
    k = lib().oracle_sample_pair(n, rp, col, np.ascontiguousarray(comp, dtype=np.int32), seed,
                                 s, t, i0, count, stride, paths, meet, C.byref(info))
    if k == -2:
        raise MemoryError
    if k < 0:
        raise ValueError(f"pair ({s}, {t}) not connected or bad stride ({k})")
    return paths[:, :k].copy(), meet, info


def accumulate(g, comp, seed: int, i0: int, i1: int) -> tuple:
    n, rp, col = _csr(g)
    acc = np.zeros(n, dtype=np.int64)
    k = lib().oracle_accumulate(n, rp, col, np.ascontiguousarray(comp, dtype=np.int32), seed,
                                i0, i1, acc)
    return int(k), acc


def brandes(g) -> np.ndarray:
    n, rp, col = _csr(g)
    bc = np.zeros(n, dtype=np.float64)
    lib().oracle_brandes(n, rp, col, bc)
    return bc


def bfs_sigma(g, s: int) -> tuple:
    n, rp, col = _csr(g)
    dist = np.zeros(n, dtype=np.int32)
    sig = np.zeros(n, dtype=np.float64)
    lib().oracle_bfs_sigma(n, rp, col, s, dist, sig)
    return dist, sig
