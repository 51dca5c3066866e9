"""Python side of the serving loop: argument marshalling for the library's
apax_server_* calls, and a Poisson load driver.

The loop itself (FIFO, admission by HBM budget, slots with resident codec
state, persistent batch launches per admitted group, event-polled
completions, latency stamps) runs in libapax.so.  This module keeps the
tensors of in-flight requests alive and turns completions into dicts.
Each request is ordered after the work enqueued on torch's current stream
before it was submitted (APAX_REQ_AFTER): the server's slot streams wait on
an event recorded there at submit.
"""
from __future__ import annotations

import ctypes as C
import time

import torch

from . import apax as A


class Server:
    def __init__(self, budget_bytes: int = 64 << 30, slots: int = 4, max_group: int = 64,
                 ws_bytes: int = 16 << 20, tune: dict | None = None, device="cuda"):
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        torch.cuda.set_device(dev)
        t = A.Tune()
        for k, v in (tune or {}).items():
            setattr(t, k, int(v))
        h = C.c_void_p()
        A._check(A.lib.apax_server_create(int(budget_bytes), int(slots), int(max_group), int(ws_bytes),
                                          C.byref(t), C.byref(h)), "apax_server_create")
        self.handle = h
        self._live = {}     # id -> objects kept alive until completion
        self._buf = (A.Completion * 1024)()

    # -- submission
    def submit(self, req: A.Request, keep) -> int:
        req.flags |= A.REQ_AFTER
        req.after = torch.cuda.current_stream(self.device).cuda_stream
        rid = C.c_uint64()
        A._check(A.lib.apax_server_submit(self.handle, C.byref(req), C.byref(rid)), "apax_server_submit")
        self._live[rid.value] = keep
        return rid.value

    def submit_encode(self, x: torch.Tensor, params: dict, out: torch.Tensor, nbytes: torch.Tensor,
                      tag: int = 0) -> int:
        """Encode x into out; the stream length goes to nbytes[0] (device int64)."""
        assert x.is_cuda and x.is_contiguous() and out.dtype == torch.uint8
        q = A.Request()
        q.op = A.OP_ENCODE
        q.item.p = A.make_params(x.dtype, tuple(x.shape), params)
        q.item.d_in = x.data_ptr() if x.numel() else None
        q.item.d_out = out.data_ptr()
        q.item.cap = out.numel()
        q.item.d_nbytes = nbytes.data_ptr()
        q.tag = int(tag)
        return self.submit(q, (x, out, nbytes))

    def submit_decode(self, stream_buf: torch.Tensor, nbytes: int, hdr: bytes, y: torch.Tensor,
                      tag: int = 0) -> int:
        """Decode nbytes of stream_buf (64-byte header hdr, host copy) into y."""
        hb = (C.c_uint8 * 64).from_buffer_copy(bytes(hdr[:64]))
        q = A.Request()
        q.op = A.OP_DECODE
        q.item.d_in = stream_buf.data_ptr()
        q.item.d_out = y.data_ptr() if y.numel() else None
        q.item.in_bytes = int(nbytes)
        q.item.cap = y.numel() * y.element_size()
        q.item.h_hdr = C.cast(hb, C.c_void_p)
        q.tag = int(tag)
        return self.submit(q, (stream_buf, y))

    # -- completion
    def poll(self) -> list:
        n = C.c_uint32()
        A._check(A.lib.apax_server_poll(self.handle, self._buf, len(self._buf), C.byref(n)),
                 "apax_server_poll")
        out = []
        for i in range(n.value):
            c = self._buf[i]
            self._live.pop(c.id, None)
            out.append({"id": c.id, "tag": c.tag, "status": c.status, "slot": c.slot,
                        "latency_s": c.latency_s})
        return out

    def stats(self) -> dict:
        q, u, g = C.c_uint64(), C.c_uint64(), C.c_uint64()
        A._check(A.lib.apax_server_stats(self.handle, C.byref(q), C.byref(u), C.byref(g)),
                 "apax_server_stats")
        return {"queued": q.value, "in_flight_bytes": u.value, "groups": g.value}

    def in_flight(self) -> int:
        return len(self._live)

    def close(self):
        if self.handle:
            A.lib.apax_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def drive(server: Server, jobs, arrivals, on_done=None, deadline_s: float | None = None) -> dict:
    """Open-loop load: job k is submitted at arrivals[k] seconds after the
    start (jobs[k]() performs the submit and returns its payload bytes);
    completions are polled continuously.  Returns latency percentiles and
    sustained throughput (payload bytes / (last completion - first arrival))."""
    order = sorted(range(len(jobs)), key=lambda k: arrivals[k])
    lat = {}
    payload = 0
    tags = {}
    t0 = time.perf_counter()
    nxt = 0
    t_last = 0.0
    while len(lat) < len(jobs):
        now = time.perf_counter() - t0
        while nxt < len(order) and arrivals[order[nxt]] <= now:
            k = order[nxt]
            rid, nb = jobs[k]()
            tags[rid] = k
            payload += nb
            nxt += 1
        for c in server.poll():
            k = tags.pop(c["id"])
            lat[k] = c["latency_s"]
            t_last = time.perf_counter() - t0
            if c["status"] != 0:
                raise A.ApaxError(c["status"], f"served request {k}")
            if on_done:
                on_done(k, c)
        if deadline_s is not None and now > deadline_s:
            raise TimeoutError(f"{len(lat)} of {len(jobs)} requests done after {now:.1f} s")
        if nxt < len(order) and server.in_flight() == 0:
            wait = arrivals[order[nxt]] - (time.perf_counter() - t0)
            if wait > 2e-4:
                time.sleep(wait - 1e-4)
    ls = sorted(lat.values())

    def pct(p):
        return ls[min(len(ls) - 1, max(0, int(-(-p * len(ls) // 100)) - 1))] if ls else 0.0
    first = min(arrivals) if len(arrivals) else 0.0
    span = max(1e-9, t_last - first)
    return {"requests": len(jobs), "bytes": payload, "seconds": span, "GBps": payload / span / 1e9,
            "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "max_ms": 1e3 * (ls[-1] if ls else 0.0),
            "groups": server.stats()["groups"]}
