"""KADABRA adaptive-sampling betweenness centrality on MI355X (gfx950).

Thin Python binding over the C ABI of libkadabra.so (include/kadabra.h):
argument marshalling only; every step of the sampling path runs in the
library's HIP kernels.  PyTorch is optional and used only to hand over
device memory and streams.

    from paper_1903_09422_amd import Graph, graphs
    g = Graph.from_csr(graphs.rmat(18))
    g.set_param("check_interval", 16384)
    g.run(eps=0.01, delta=0.1, seed=1)
    res = g.result()          # tau, counts, scores, stats, decisions
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from ._lib import EXPORTS, Checkpoint, KadabraError, ServerInfo, Stats, check, lib  # noqa: F401

__all__ = ["Graph", "Batch", "Server", "RunResult", "KadabraError", "eval_stop_fg", "lib"]


@dataclass
class RunResult:
    tau: int
    counts: np.ndarray    # int32[n]
    scores: np.ndarray    # float64[n], counts / tau, computed on the device
    stats: dict
    decisions: np.ndarray  # int8 per boundary: 0 continue, 1 stop rule met, 2 omega


class Graph:
    """A graph resident on the device plus its sampling state (one handle)."""

    def __init__(self, n: int, row_ptr, col):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        if rp.shape != (n + 1,):
            raise ValueError("row_ptr must have n + 1 entries")
        self.n = int(n)
        h = C.c_void_p()
        check(lib().kadabra_create_graph(self.n, int(cl.size), rp.ctypes.data, cl.ctypes.data,
                                         C.byref(h)))
        self._h = h
        self._stream_ref = None

    @classmethod
    def from_csr(cls, csr) -> "Graph":
        return cls(csr.n, csr.row_ptr, csr.col)

    # -- parameters -------------------------------------------------------
    def set_param(self, key: str, value: int) -> None:
        check(lib().kadabra_set_param(self._h, key.encode(), int(value)))

    def get_param(self, key: str) -> int:
        v = C.c_int64()
        check(lib().kadabra_get_param(self._h, key.encode(), C.byref(v)))
        return int(v.value)

    def set_stream(self, stream) -> None:
        """Issue all work on a HIP stream: a torch.cuda.Stream, a raw handle
        (int), or None for the library's own stream."""
        if stream is None:
            ptr = None
        elif isinstance(stream, int):
            ptr = stream
        else:
            ptr = int(stream.cuda_stream)
        self._stream_ref = stream
        check(lib().kadabra_set_stream(self._h, ptr))

    # -- running ------------------------------------------------------------
    def run(self, eps: float, delta: float, seed: int) -> None:
        check(lib().kadabra_run(self._h, float(eps), float(delta), int(seed)))

    def run_static(self, eps: float, delta: float, seed: int, counts_dev) -> dict:
        """kadabra_run_static: the run with all device state in the library's
        static array (no allocation).  counts_dev: a device int32[n] tensor
        (or a raw device address) that receives the counters.  Returns the
        statistics."""
        ptr = counts_dev if isinstance(counts_dev, int) else int(counts_dev.data_ptr())
        st = Stats()
        check(lib().kadabra_run_static(self._h, float(eps), float(delta), int(seed), ptr, C.byref(st)))
        return st.as_dict()

    def checkpoint(self):
        """(Checkpoint, counters) of the last run when it stopped at a
        boundary ("stop_after_epochs" or cancel)."""
        ck = Checkpoint()
        counts = np.empty(self.n, dtype=np.int32)
        check(lib().kadabra_get_checkpoint(self._h, C.byref(ck), counts.ctypes.data))
        return ck, counts

    def resume(self, ck, counts) -> None:
        """Continue a run from a checkpoint to completion (kadabra_resume)."""
        c = np.ascontiguousarray(counts, dtype=np.int32)
        check(lib().kadabra_resume(self._h, C.byref(ck), c.ctypes.data))

    def cancel(self) -> None:
        check(lib().kadabra_cancel(self._h))

    def result(self) -> RunResult:
        scores = np.empty(self.n, dtype=np.float64)
        counts = np.empty(self.n, dtype=np.int32)
        st = Stats()
        check(lib().kadabra_get_scores(self._h, scores.ctypes.data, counts.ctypes.data,
                                       C.byref(st)))
        cnt = C.c_int64()
        check(lib().kadabra_get_decisions(self._h, None, 0, C.byref(cnt)))
        dec = np.empty(max(int(cnt.value), 1), dtype=np.int8)
        check(lib().kadabra_get_decisions(self._h, dec.ctypes.data, dec.size, C.byref(cnt)))
        return RunResult(tau=int(st.tau), counts=counts, scores=scores, stats=st.as_dict(),
                         decisions=dec[: int(cnt.value)].copy())

    def balance(self) -> tuple:
        """The last run's per-vertex constants: (log(1/delta_L), log(1/delta_U),
        first-phase counters); uniform L and zeros without "balance"."""
        LL = np.empty(self.n, dtype=np.float64)
        LU = np.empty(self.n, dtype=np.float64)
        c1 = np.empty(self.n, dtype=np.int32)
        check(lib().kadabra_get_balance(self._h, LL.ctypes.data, LU.ctypes.data, c1.ctypes.data))
        return LL, LU, c1

    def autotune(self, eps: float, delta: float, trial_samples: int = 8192) -> dict:
        """Pick the fastest mapping (team, slots, probe, epochs per launch) on a trial prefix;
        results never depend on it.  Returns the chosen parameters."""
        check(lib().kadabra_autotune(self._h, float(eps), float(delta), int(trial_samples)))
        return {k: self.get_param(k) for k in ("team", "slots", "probe_min", "epochs_per_launch")}

    def stats(self) -> dict:
        st = Stats()
        check(lib().kadabra_get_scores(self._h, None, None, C.byref(st)))
        return st.as_dict()

    def result_device(self, scores=None, counts=None) -> None:
        """Write scores (float64[n]) and/or counts (int32[n]) into device
        tensors on the handle's stream (no host round trip)."""
        sp = None if scores is None else int(scores.data_ptr())
        cp = None if counts is None else int(counts.data_ptr())
        for t, dt in ((scores, "float64"), (counts, "int32")):
            if t is not None and (not t.is_cuda or str(t.dtype) != f"torch.{dt}" or
                                  t.numel() != self.n or not t.is_contiguous()):
                raise ValueError(f"expected a contiguous CUDA {dt} tensor of {self.n} elements")
        check(lib().kadabra_get_scores_device(self._h, sp, cp))

    # -- lifetime -------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().kadabra_destroy_graph(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many queries (graph, eps, delta, seed, check interval) run in shared
    launches; each result equals the query's own Graph.run result."""

    def __init__(self):
        h = C.c_void_p()
        check(lib().kadabra_batch_create(C.byref(h)))
        self._h = h
        self._graphs = []  # keep graph handles alive while queries reference them
        self._stream_ref = None

    def set_param(self, key: str, value: int) -> None:
        check(lib().kadabra_batch_set_param(self._h, key.encode(), int(value)))

    def get_param(self, key: str) -> int:
        v = C.c_int64()
        check(lib().kadabra_batch_get_param(self._h, key.encode(), C.byref(v)))
        return int(v.value)

    def set_stream(self, stream) -> None:
        ptr = None if stream is None else (stream if isinstance(stream, int) else int(stream.cuda_stream))
        self._stream_ref = stream
        check(lib().kadabra_batch_set_stream(self._h, ptr))

    def add(self, graph: Graph, eps: float, delta: float, seed: int, check_interval: int) -> int:
        idx = C.c_int32()
        check(lib().kadabra_batch_add(self._h, graph._h, float(eps), float(delta), int(seed),
                                      int(check_interval), C.byref(idx)))
        self._graphs.append(graph)
        return int(idx.value)

    def run(self) -> None:
        check(lib().kadabra_batch_run(self._h))

    def autotune(self, trial_samples: int = 4096) -> dict:
        check(lib().kadabra_batch_autotune(self._h, int(trial_samples)))
        return {k: self.get_param(k) for k in ("team", "slots", "probe_min", "epochs_per_launch")}

    def result(self, index: int) -> RunResult:
        if not 0 <= index < len(self._graphs):  # let the library report the bad index
            check(lib().kadabra_batch_get_scores(self._h, int(index), None, None, None))
        n = self._graphs[index].n
        scores = np.empty(n, dtype=np.float64)
        counts = np.empty(n, dtype=np.int32)
        st = Stats()
        check(lib().kadabra_batch_get_scores(self._h, int(index), scores.ctypes.data,
                                             counts.ctypes.data, C.byref(st)))
        return RunResult(tau=int(st.tau), counts=counts, scores=scores, stats=st.as_dict(),
                         decisions=np.empty(0, dtype=np.int8))

    def stats(self, index: int) -> dict:
        st = Stats()
        check(lib().kadabra_batch_get_scores(self._h, int(index), None, None, C.byref(st)))
        return st.as_dict()

    def clear(self) -> None:
        check(lib().kadabra_batch_clear(self._h))
        self._graphs = []

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().kadabra_batch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous batching over resident graphs: submit() returns a ticket at
    once; a native worker admits waiting queries at every round boundary
    while their device memory fits the budget.  Each result equals the
    query's own Graph.run result."""

    def __init__(self, graphs, hbm_budget_bytes: int = 0, max_active: int = 0):
        self._graphs = list(graphs)  # the server references their device CSR
        arr = (C.c_void_p * len(self._graphs))(*[g._h.value for g in self._graphs])
        h = C.c_void_p()
        check(lib().kadabra_server_create(arr, len(self._graphs), int(hbm_budget_bytes),
                                          int(max_active), C.byref(h)))
        self._h = h
        self._graph_of = {}  # ticket -> graph index (sizes the result buffers)

    def set_param(self, key: str, value: int) -> None:
        check(lib().kadabra_server_set_param(self._h, key.encode(), int(value)))

    def get_param(self, key: str) -> int:
        v = C.c_int64()
        check(lib().kadabra_server_get_param(self._h, key.encode(), C.byref(v)))
        return int(v.value)

    def submit(self, graph_index: int, eps: float, delta: float, seed: int,
               check_interval: int) -> int:
        t = C.c_int64()
        check(lib().kadabra_server_submit(self._h, int(graph_index), float(eps), float(delta),
                                          int(seed), int(check_interval), C.byref(t)))
        self._graph_of[int(t.value)] = int(graph_index)
        return int(t.value)

    def wait(self, ticket: int, timeout: float = -1.0) -> bool:
        done = C.c_int32()
        check(lib().kadabra_server_wait(self._h, int(ticket), float(timeout), C.byref(done)))
        return bool(done.value)

    def result(self, ticket: int, graph_index: int = None, scores: bool = True):
        """(RunResult, latency in ms) of a final query."""
        if graph_index is None:
            graph_index = self._graph_of.get(int(ticket), 0)  # an unknown ticket: the library reports it
        n = self._graphs[graph_index].n
        sc = np.empty(n, dtype=np.float64) if scores else None
        counts = np.empty(n, dtype=np.int32)
        st = Stats()
        lat = C.c_double()
        check(lib().kadabra_server_result(self._h, int(ticket),
                                          sc.ctypes.data if sc is not None else None,
                                          counts.ctypes.data, C.byref(st), C.byref(lat)))
        return RunResult(tau=int(st.tau), counts=counts, scores=sc, stats=st.as_dict(),
                         decisions=np.empty(0, dtype=np.int8)), float(lat.value)

    def release(self, ticket: int) -> None:
        check(lib().kadabra_server_release(self._h, int(ticket)))
        self._graph_of.pop(int(ticket), None)

    def info(self, reset: bool = False) -> dict:
        inf = ServerInfo()
        check(lib().kadabra_server_info_get(self._h, C.byref(inf), 1 if reset else 0))
        return inf.as_dict()

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().kadabra_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_stop_fg(counts, tau: int, omega: int, L: float):
    """Device evaluation of the stopping-rule functions (f, g) per counter."""
    c = np.ascontiguousarray(counts, dtype=np.int32)
    f = np.empty(c.size, dtype=np.float64)
    g = np.empty(c.size, dtype=np.float64)
    check(lib().kadabra_eval_stop_fg(c.size, c.ctypes.data, int(tau), int(omega), float(L),
                                     f.ctypes.data, g.ctypes.data))
    return f, g
