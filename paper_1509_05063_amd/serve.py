"""Serving loop for Lippmann–Schwinger solves on one GPU (Python face of the
library's ls_server_* calls).

Requests name a scatterer (a workload configuration) and an incidence angle.
The native server keeps operators resident in HBM (set-up once: nodes,
near-field weights, equivalent-source matrices and the FFT'd Green's
kernels), admits them under a byte budget (least recently used idle operators
are evicted when a new one does not fit), and batches requests on the same
operator as extra right-hand sides of one solve.  Batching is continuous:
while an operator's solve runs, new requests for it queue up and form its next
batch; solves on different operators run at the same time in their own worker
threads and HIP streams.  This module only registers scatterers, submits,
polls and keeps latency records.

Results are deterministic per right-hand side (the batched solve advances
every right-hand side independently and freezes the ones that have
converged), so a request gets the same answer alone or inside any batch.
"""
import ctypes as C
import time

import numpy as np

from . import binding
from .inputs import n2_function


class Request:
    __slots__ = ("ticket", "key", "cfg", "alpha", "arrival", "done", "latency", "result", "stats", "batch", "N",
                 "status")

    def __init__(self, ticket, key, cfg, alpha, arrival):
        self.ticket, self.key, self.cfg, self.alpha, self.arrival = ticket, key, cfg, alpha, arrival
        self.done = self.latency = self.result = self.stats = None
        self.batch = 0
        self.N = 0
        self.status = None


class Server:
    """budget_bytes: HBM allowed for resident operators plus solver memory.
    max_batch: right-hand sides per solve.  workers: concurrent solves."""

    def __init__(self, budget_bytes, max_batch=16, workers=4, tol=1e-7, restart=60, inner_tol=1e-4,
                 keep_results=True, max_iter=4000, max_outer=30, ortho=binding.LS_ORTHO_CGS2):
        L = binding.lib()
        self.tol, self.restart, self.inner_tol = tol, restart, inner_tol
        self.keep_results = keep_results
        opts = binding.ServerOpts(int(max_batch), int(workers), float(tol), int(max_iter), int(restart),
                                  binding.LS_SOLVE_FP32_REFINE, float(inner_tol), int(max_outer), int(ortho))
        self._srv = C.c_void_p()
        binding._check(L.ls_server_create(C.c_size_t(int(budget_bytes)), C.byref(opts), C.byref(self._srv)),
                       "ls_server_create")
        self._ids = {}            # scatterer key -> server key
        self._keep = []           # callbacks and structs the server refers to
        self.tickets = {}

    def _register(self, key, cfg):
        if key in self._ids:
            return self._ids[key]
        sid = len(self._ids)
        g, p = binding.geometry_from(cfg), binding.params_from(cfg)
        cb = binding._n2_callback(n2_function(cfg))
        self._keep.append((g, p, cb))
        binding._check(binding.lib().ls_server_add_operator(self._srv, sid, C.byref(g), cb, None,
                                                            float(cfg["kappa"]), C.byref(p)),
                       "ls_server_add_operator")
        self._ids[key] = sid
        return sid

    # ------------------------------------------------------------ client API
    def submit(self, key, cfg, alpha, arrival=None):
        sid = self._register(key, cfg)
        t = C.c_int64()
        binding._check(binding.lib().ls_server_submit(self._srv, sid, float(alpha), C.byref(t)), "ls_server_submit")
        r = Request(t.value, key, cfg, alpha, time.perf_counter() if arrival is None else arrival)
        self.tickets[t.value] = r
        return t.value

    def poll(self, ticket):
        """The finished request, or None while it is pending."""
        r = self.tickets[ticket]
        if r.done is not None:
            return r
        L = binding.lib()
        info = binding.RequestInfo()
        rc = L.ls_server_poll(self._srv, ticket, None, 0, C.byref(info))
        if rc == binding.LS_ENOTREADY:
            return None
        if self.keep_results and rc in (binding.LS_OK, binding.LS_ENOCONV):
            buf = np.empty(info.N, complex)
            L.ls_server_poll(self._srv, ticket, buf.ctypes.data, 2 * info.N, C.byref(info))
            r.result = buf
        s = info.stats
        r.stats = {"iterations": s.iterations, "outer": s.outer, "converged": s.converged,
                   "rel_residual": s.rel_residual, "seconds": s.seconds}
        r.status, r.batch, r.N = rc, info.batch, info.N
        r.latency = info.t_done - info.t_submit
        r.done = r.arrival + r.latency
        L.ls_server_release(self._srv, ticket)
        return r

    def drain(self):
        pending = [t for t, r in self.tickets.items() if r.done is None]
        while pending:
            pending = [t for t in pending if self.poll(t) is None]
            if pending:
                time.sleep(0.002)

    def points(self, key):
        n = C.c_int64()
        L = binding.lib()
        binding._check(L.ls_server_points(self._srv, self._ids[key], None, 0, C.byref(n)), "ls_server_points")
        xy = np.empty((n.value, 2))
        binding._check(L.ls_server_points(self._srv, self._ids[key], xy.ctypes.data, 2 * n.value, C.byref(n)),
                       "ls_server_points")
        return xy

    def info(self):
        i = binding.ServerInfo()
        binding._check(binding.lib().ls_server_stats(self._srv, C.byref(i)), "ls_server_stats")
        return {"resident_bytes": i.resident_bytes, "resident_ops": i.resident_ops, "queued": i.queued,
                "running": i.running, "evictions": i.evictions}

    @property
    def evictions(self):
        return self.info()["evictions"]

    def close(self):
        if self._srv:
            binding.lib().ls_server_destroy(self._srv)
            self._srv = None


def latency_stats(reqs):
    lat = np.array([r.done - r.arrival for r in reqs])
    return {"n": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_batch": float(np.mean([r.batch for r in reqs]))}


def replay(server, trace, time_scale=1.0):
    """Submit (arrival_s, key, cfg, alpha) tuples at their arrival times;
    returns the requests once all have finished and the wall time."""
    t0 = time.perf_counter()
    tickets = []
    for (ta, key, cfg, alpha) in trace:
        now = time.perf_counter() - t0
        if ta * time_scale > now:
            time.sleep(ta * time_scale - now)
        tickets.append(server.submit(key, cfg, alpha, arrival=t0 + ta * time_scale))
    server.drain()
    wall = time.perf_counter() - t0
    return [server.tickets[t] for t in tickets], wall
