"""Streaming server binding (cwt_server_* / cwt_stream_* of include/cwt.h)."""
import ctypes

import numpy as np

from . import _lib


def now_ns():
    """CLOCK_MONOTONIC nanoseconds, the clock of the stream time stamps."""
    return int(_lib.load().cwt_now_ns())


class Server:
    """Batching stream server with an HBM budget (device memory of rings + workspaces).

    stream: the torch stream every device operation of the server goes on (a
    new default-priority torch stream when None).  memory: "torch" (rings and
    batch buffers from torch's caching allocator, the default), a
    TorchDeviceMemory, or None (HIP's stream-ordered pool)."""

    def __init__(self, hbm_budget_bytes, max_batch=256, deadline_us=500, max_pending=64,
                 max_session_windows=4, stream=None, memory="torch"):
        import torch

        from . import TorchDeviceMemory
        lib = _lib.load()
        self._lib = lib
        o = _lib.ServerOpts()
        lib.cwt_server_opts_init(ctypes.byref(o))
        o.max_batch, o.deadline_us, o.max_pending = int(max_batch), int(deadline_us), int(max_pending)
        o.max_session_windows = int(max_session_windows)
        self.stream = torch.cuda.Stream() if stream is None else stream
        self.memory = TorchDeviceMemory() if memory == "torch" else memory
        if self.memory is not None:
            self.memory.fill(o)
        h = ctypes.c_void_p()
        self._ptr = None
        _lib.check(lib.cwt_server_create(ctypes.byref(h), int(hbm_budget_bytes), ctypes.byref(o),
                                         ctypes.c_void_p(self.stream.cuda_stream)))
        self._ptr = h
        self.sessions = []

    def open(self, plan, C, hop):
        """Open a session on a band-power plan (window = plan.n samples)."""
        return Session(self, plan, C, hop)

    def flush(self):
        _lib.check(self._lib.cwt_server_flush(self._ptr))

    def stats(self):
        st = _lib.ServerStats()
        _lib.check(self._lib.cwt_server_get_stats(self._ptr, ctypes.byref(st)))
        return {n: int(getattr(st, n)) for n, _ in _lib.ServerStats._fields_}

    def close(self):
        if self._ptr:
            for s in list(self.sessions):
                s.close()
            self._lib.cwt_server_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Session:
    def __init__(self, server, plan, C, hop):
        self.server = server
        self.plan = plan  # keeps the plan alive
        self.C, self.hop = int(C), int(hop)
        self.n_bands = plan.n_bands
        h = ctypes.c_void_p()
        self._ptr = None
        _lib.check(server._lib.cwt_stream_open(server._ptr, plan.handle, self.C, self.hop,
                                               ctypes.byref(h)))
        self._ptr = h
        server.sessions.append(self)
        self._bp = np.empty((self.C, self.n_bands), dtype=np.float32)

    def push(self, samples, t_arrival_ns=0):
        """samples: [C, m] float32 host array.  Returns False on backpressure (CWT_E_AGAIN)."""
        a = np.ascontiguousarray(samples, dtype=np.float32)
        if a.ndim != 2 or a.shape[0] != self.C:
            raise ValueError("samples must be [C, m]")
        rc = self.server._lib.cwt_stream_push(self._ptr, a.ctypes.data_as(
            ctypes.POINTER(ctypes.c_float)), a.shape[1], int(t_arrival_ns))
        if rc == _lib.CWT_E_AGAIN:
            return False
        _lib.check(rc)
        return True

    def poll(self):
        """(bp [C, B], hop_idx, t_push_ns, t_done_ns) of the oldest result, or None."""
        hi, tp, td = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        rc = self.server._lib.cwt_stream_poll(
            self._ptr, self._bp.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            ctypes.byref(hi), ctypes.byref(tp), ctypes.byref(td))
        if rc == _lib.CWT_E_AGAIN:
            return None
        _lib.check(rc)
        return self._bp.copy(), int(hi.value), int(tp.value), int(td.value)

    def close(self):
        if self._ptr:
            self.server._lib.cwt_stream_close(self._ptr)
            self._ptr = None
            if self in self.server.sessions:
                self.server.sessions.remove(self)
