"""Serving loop for Lippmann–Schwinger solves on one GPU.

Requests name a scatterer (a workload configuration) and an incidence
angle.  The server keeps operators resident in HBM (set-up once: nodes,
near-field weights, equivalent-source matrices and the FFT'd Green's kernels),
admits them under a byte budget (least recently used idle operators are
evicted when a new one does not fit), and batches requests on the same
operator as extra right-hand sides of one solve.  Batching is continuous:
while an operator's solve runs, new requests for it queue up and form its
next batch; solves on different operators run at the same time in their own
worker threads and HIP streams.  All arithmetic happens in the C ABI
(ls_solve); this module only schedules.

Results are deterministic per right-hand side: a request gets the same
answer alone or inside any batch (the batched solve advances every
right-hand side independently and freezes the ones that have converged).
"""
import collections
import math
import threading
import time

import numpy as np

from . import binding
from .inputs import n2_function, plane_wave


class Request:
    __slots__ = ("ticket", "key", "cfg", "alpha", "arrival", "start", "done", "result", "stats", "batch")

    def __init__(self, ticket, key, cfg, alpha, arrival):
        self.ticket, self.key, self.cfg, self.alpha, self.arrival = ticket, key, cfg, alpha, arrival
        self.start = self.done = None
        self.result = None
        self.stats = None
        self.batch = 0


class Server:
    """budget_bytes: HBM allowed for resident operators plus solver memory.
    max_batch: right-hand sides per solve.  workers: concurrent solves."""

    def __init__(self, budget_bytes, max_batch=16, workers=4, tol=1e-7, restart=60, inner_tol=1e-4,
                 keep_results=True):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.tol, self.restart, self.inner_tol = tol, restart, inner_tol
        self.keep_results = keep_results
        self.lock = threading.Condition()
        self.queues = collections.OrderedDict()       # key -> deque of Request
        self.ops = collections.OrderedDict()          # key -> binding.Operator (LRU order)
        self.busy = set()                             # keys with a solve in flight
        self.tickets = {}
        self.next_ticket = 0
        self.stop = False
        self.evictions = 0
        self.threads = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(workers)]
        for t in self.threads:
            t.start()

    # ------------------------------------------------------------ client API
    def submit(self, key, cfg, alpha, arrival=None):
        with self.lock:
            t = self.next_ticket
            self.next_ticket += 1
            r = Request(t, key, cfg, alpha, time.perf_counter() if arrival is None else arrival)
            self.tickets[t] = r
            self.queues.setdefault(key, collections.deque()).append(r)
            self.lock.notify_all()
            return t

    def poll(self, ticket):
        """The finished request, or None while it is pending."""
        with self.lock:
            r = self.tickets[ticket]
            return r if r.done is not None else None

    def drain(self):
        with self.lock:
            while any(r.done is None for r in self.tickets.values()):
                self.lock.wait(0.05)

    def close(self):
        with self.lock:
            self.stop = True
            self.lock.notify_all()
        for t in self.threads:
            t.join()
        for op in self.ops.values():
            op.close()
        self.ops.clear()

    # ------------------------------------------------------------- internals
    def _resident(self):
        return sum(op.resident_bytes() for op in self.ops.values())

    @staticmethod
    def _solve_bytes(N, nrhs, restart):
        # Krylov basis + work vectors (complex double) + FP32 copies + apply workspace (estimate)
        return 16 * N * nrhs * (restart + 7) + 16 * N * nrhs + (64 << 20) * nrhs

    def _admit(self, key, n_est):
        """Make room for operator `key` (lock held): evict idle operators in
        least-recently-used order until it and one more solve fit the budget.
        False when the remaining operators are all busy (the caller waits)."""
        need = self._solve_bytes(n_est, self.max_batch, self.restart)
        while True:
            op_bytes = 0 if key in self.ops else int(n_est * 8000)   # resident estimate per unknown
            if self._resident() + op_bytes + need * (len(self.busy) + 1) <= self.budget:
                return True
            victim = next((k for k in self.ops if k not in self.busy and k != key), None)
            if victim is None:
                # nothing left to evict: run alone if no other solve is in flight
                return not (self.busy - {key})
            self.ops.pop(victim).close()
            self.evictions += 1

    def _pick(self):
        for key, q in self.queues.items():
            if q and key not in self.busy:
                return key
        return None

    def _worker(self, wid):
        torch = self.torch
        stream = torch.cuda.Stream()
        while True:
            with self.lock:
                key = None
                while not self.stop:
                    key = self._pick()
                    if key is not None:
                        break
                    self.lock.wait(0.05)
                if self.stop:
                    return
                q = self.queues[key]
                cfg = q[0].cfg
                n_est = self.ops[key].N if key in self.ops else _estimate_points(cfg)
                if not self._admit(key, n_est):
                    self.lock.wait(0.05)
                    continue
                batch = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
                self.busy.add(key)
                op = self.ops.get(key)
                if op is not None:
                    self.ops.move_to_end(key)
            t0 = time.perf_counter()
            for r in batch:
                r.start = t0
            if op is None:
                op = binding.Operator(cfg, n2_function(cfg))
                with self.lock:
                    self.ops[key] = op
            xy, _ = op.points()
            with torch.cuda.stream(stream):
                F = torch.tensor(np.stack([plane_wave(cfg, xy, r.alpha) for r in batch]),
                                 dtype=torch.complex128, device="cuda")
                X = torch.empty_like(F)
                st = op.solve(F, X, tol=self.tol, restart=self.restart, max_iter=4000,
                              mode=binding.LS_SOLVE_FP32_REFINE, inner_tol=self.inner_tol, max_outer=30,
                              stream=stream, raise_on_noconv=False)
                stream.synchronize()
                host = X.cpu().numpy() if self.keep_results else None
            t1 = time.perf_counter()
            with self.lock:
                for k, r in enumerate(batch):
                    r.done = t1
                    r.stats = st
                    r.batch = len(batch)
                    if host is not None:
                        r.result = host[k]
                self.busy.discard(key)
                self.lock.notify_all()


def _estimate_points(cfg):
    """Rough node count of a configuration (for admission before set-up)."""
    a = cfg["shape"]["a"]
    area = math.pi * (1 + a * a / 2)
    s_b = cfg["pou"]["s_b"]
    b = cfg["band"]
    return int(area * s_b * s_b / cfg["h"] ** 2 + b["N1"] * (b["N2"] + 1))


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
