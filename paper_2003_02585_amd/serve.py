"""Serving loop: continuous batching of Helmholtz solve requests over the
libhdsw C-ABI.

Each request names an operator key (grid size, subdomain size, medium,
points per wavelength) and carries R point sources.  The server

  * keeps one factored context per key on the device (the factor cache),
    in least-recently-used order, and evicts idle contexts when a new key
    does not fit the HBM budget;
  * admits the columns of queued requests into free column slots of their
    context as slots and memory free up (column-granular continuous
    batching): a request may start with part of its columns;
  * keeps one refinement iteration (x += M^{-1} r, then the FP64 residual,
    M^{-1} the diagonal-sweeping DDM) in flight on every context with
    occupied slots, each context on its own stream so that the iterations
    of different keys overlap on the device; a context whose iteration has
    finished is serviced at once, without waiting for the others;
  * takes every column whose relative residual reached the tolerance out of
    its slot, and completes a request when its last column leaves.

A column's arithmetic does not depend on the other columns of its context,
so every result is the same alone and in the mix.  Metrics: throughput
(requests/s, RHS-solves/s), latency and admission wait (p50/p99), cache hit
rate, evictions and peak bytes held.

The executor is pluggable: HipExecutor drives the library on the GPU;
tests drive the same Server with a host-only stub to check the scheduling
logic.
"""

import argparse
import collections
import json
import time

import numpy as np

from . import workloads as wl


class Request:
    __slots__ = ("rid", "arrival", "key", "positions", "R", "next_col", "cols_done",
                 "admitted", "done", "hit", "iters", "rel", "failed", "result")

    def __init__(self, rid, arrival, key, positions):
        self.rid = rid
        self.arrival = arrival
        self.key = key
        self.positions = np.asarray(positions, dtype=np.float64)
        self.R = len(self.positions)
        self.next_col = 0          # next column to admit
        self.cols_done = 0
        self.admitted = None       # time the first column joined a context
        self.done = None
        self.hit = None            # False: the request's admission factored a new context
        self.iters = [0] * self.R
        self.rel = [np.nan] * self.R
        self.failed = False
        self.result = None

    @property
    def pending(self):
        return self.R - self.next_col


class CtxState:
    """Server-side view of one cached context."""

    def __init__(self, key, handle, nbytes, cap):
        self.key = key
        self.handle = handle
        self.nbytes = nbytes
        self.cap = cap
        self.slots = {}            # slot -> (request, column)
        self.iters = {}            # slot -> iterations so far

    @property
    def nact(self):
        return len(self.slots)


# --------------------------------------------------------------- executors
class HipExecutor:
    """Runs contexts of libhdsw on the GPU, one torch stream per context."""

    def __init__(self, cap_max=32, tol=1e-10, precision=None, add_chunk=8):
        import torch
        from . import hdsw
        self.torch = torch
        self.H = hdsw
        self.cap_max = cap_max
        self.tol = tol
        self.precision = hdsw.HDSW_MIXED if precision is None else precision
        self.add_chunk = add_chunk
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self._sink = None
        self._pool = None

    def now(self):
        return time.perf_counter()

    def idle_until(self, t):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)

    def start_create(self, key, free_bytes, slot_bytes=None):
        """Set up the context of `key` within `free_bytes` (host work and the
        factor storage, on the calling thread) and start its factorization
        and slot reservation on a worker thread, on the context's own
        stream, so that other contexts keep running meanwhile.  Returns a
        token for poll_create, or None if the factors do not fit."""
        H, torch = self.H, self.torch
        kap, h, P, W, rounds = wl.serve_kappa(key)
        stream = torch.cuda.Stream(device=self.dev)
        opt = H.hdsw_default_options(precision=self.precision, rounds=rounds, tol=self.tol,
                                     hbm_budget=int(max(free_bytes, 1)))
        try:
            ctx = H.hdsw_setup(kap, h, P, W, opt, stream=stream.cuda_stream)
        except H.HdswError as e:
            if e.status == H.HDSW_ENOMEM:
                return None
            raise
        if self._pool is None:
            import concurrent.futures
            self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=1)
        fut = self._pool.submit(self._factor_reserve, ctx, free_bytes, slot_bytes)
        return dict(fut=fut, handle=dict(ctx=ctx, stream=stream, N=kap.shape[-1], h=h))

    def _factor_reserve(self, ctx, free_bytes, slot_bytes):
        H = self.H
        try:
            H.hdsw_factor(ctx)
            H.hdsw_batch_reserve(ctx, 1)
            fb, _, ws1 = H.hdsw_query(ctx)
            sb = free_bytes if slot_bytes is None else min(slot_bytes, free_bytes)
            fit = max(1, (sb - fb) // max(ws1, 1)) if free_bytes - fb >= ws1 else 0
            cap = int(min(self.cap_max, fit))
            while cap > 1:
                # the estimate leaves out the context's small set-up arrays:
                # step down when the library's own budget check refuses
                try:
                    H.hdsw_batch_reserve(ctx, cap)
                    break
                except H.HdswError as e:
                    if e.status != H.HDSW_ENOMEM:
                        raise
                    cap -= max(1, cap // 8)
            if cap < 1:
                raise H.HdswError(H.HDSW_ENOMEM, "no column fits")
            if cap == 1:
                H.hdsw_batch_reserve(ctx, 1)
            fb, _, ws = H.hdsw_query(ctx)
            return int(fb + ws), cap
        except H.HdswError as e:
            H.hdsw_destroy(ctx)
            if e.status == H.HDSW_ENOMEM:
                return None
            raise

    def poll_create(self, tok):
        """None while the factorization runs; then (handle, bytes, capacity),
        or False if it did not fit."""
        if not tok["fut"].done():
            return None
        r = tok["fut"].result()
        if r is None:
            return False
        return tok["handle"], r[0], r[1]

    def sources(self, N, h, positions):
        """The request's input: Gaussian point sources (sigma = 2h) at the
        given positions, [R][N][N] complex128 on the device, formed on the
        current stream as the outer product of per-axis factors (the client
        side of the loop; no arithmetic of the method)."""
        torch = self.torch
        sigma = 2 * h
        gx = np.stack([wl.gaussian_axis(N, h, p[0], sigma) for p in positions])
        gy = np.stack([wl.gaussian_axis(N, h, p[1], sigma) for p in positions])
        gx = torch.from_numpy(gx).to(self.dev)
        gy = torch.from_numpy(gy).to(self.dev)
        f = (gx[:, None, :] * gy[:, :, None]) / wl.gaussian_mass(2, sigma)
        return f.to(torch.complex128).contiguous()

    def add(self, handle, req, c0, n):
        """Build the sources of columns c0..c0+n of `req` on the context's
        stream and add them; returns the slot ids."""
        torch, H = self.torch, self.H
        slots = []
        with torch.cuda.stream(handle["stream"]):
            for a in range(c0, c0 + n, self.add_chunk):
                b = min(a + self.add_chunk, c0 + n)
                f = self.sources(handle["N"], handle["h"], req.positions[a:b])
                slots += H.hdsw_batch_add(handle["ctx"], f, b - a)
        return slots

    def step(self, handle):
        self.H.hdsw_batch_step(handle["ctx"])

    def ready(self, handle):
        return self.H.hdsw_batch_ready(handle["ctx"])

    def pause(self):
        time.sleep(2e-5)

    def wait(self, handle, cap):
        return self.H.hdsw_batch_wait(handle["ctx"], cap)

    def take(self, handle, slot, out=None):
        """Copy the slot's solution (into `out`, a [N][N] complex128 device
        tensor, or into a reused buffer) and free the slot."""
        torch = self.torch
        if out is None:
            N = handle["N"]
            if self._sink is None or self._sink.numel() < N * N:
                self._sink = torch.empty(N * N, dtype=torch.complex128, device=self.dev)
            out = self._sink[:N * N].view(N, N)
        self.H.hdsw_batch_take(handle["ctx"], slot, out)

    def result_buffer(self, handle, R):
        # no fill kernel: every interior value is written by take, on the
        # context's stream
        N = handle["N"]
        return self.torch.empty((R, N, N), dtype=self.torch.complex128, device=self.dev)

    def destroy(self, handle):
        self.H.hdsw_destroy(handle["ctx"])


# ------------------------------------------------------------------ server
class Server:
    def __init__(self, executor, budget_bytes, tol=1e-10, max_iter=30, keep_results=False,
                 progress=None, age_limit=2.0, ctx_share=0.5):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.tol = tol
        self.max_iter = max_iter
        self.keep = keep_results
        self.ctxs = collections.OrderedDict()    # key -> CtxState, LRU first
        self.used = 0
        self.peak = 0
        self.created = 0
        self.evictions = 0
        self.steps = 0
        self.progress = progress      # print a line every `progress` completed requests
        self.age_limit = age_limit    # seconds before a request's key is factored first
        self.blocked_key = None
        self.pending = None           # (key, token, bytes held) of the running factorization
        self.ctxs_first = {}          # key -> hit flag of its first request (a miss)
        self.ctx_share = ctx_share    # largest budget share of one context's slots

    # context cache ---------------------------------------------------
    def _evict_one(self):
        for key, cs in self.ctxs.items():
            if cs.nact == 0:
                self.ex.destroy(cs.handle)
                self.used -= cs.nbytes
                del self.ctxs[key]
                self.evictions += 1
                return True
        return False

    def _start_create(self, key):
        """Start factoring `key`, evicting idle contexts (least recently
        used first) until its factors fit; the whole free budget is held
        for it until it is done."""
        while True:
            free = self.budget - self.used
            tok = self.ex.start_create(key, free, min(free, int(self.ctx_share * self.budget)))
            if tok is not None:
                self.pending = (key, tok, free)
                self.used += free
                return True
            if not self._evict_one():
                return False

    def _finish_create(self, now):
        """Poll the pending factorization; returns True if it ended."""
        key, tok, held = self.pending
        r = self.ex.poll_create(tok)
        if r is None:
            return False
        self.pending = None
        self.used -= held
        if r is False:
            # the factorization's own workspaces did not fit: free an idle
            # context and try again, or give up on the key
            if not self._evict_one():
                self.blocked_key = key
            return True
        handle, nbytes, cap = r
        cs = CtxState(key, handle, nbytes, cap)
        self.ctxs[key] = cs
        self.used += nbytes
        self.peak = max(self.peak, self.used)
        self.created += 1
        return True

    # admission -------------------------------------------------------
    def _join(self, cs, req, now):
        n = min(cs.cap - cs.nact, req.pending)
        if n <= 0:
            return
        if req.admitted is None:
            req.admitted = now
            if self.keep:
                req.result = self.ex.result_buffer(cs.handle, req.R)
        slots = self.ex.add(cs.handle, req, req.next_col, n)
        for j, s in enumerate(slots):
            cs.slots[s] = (req, req.next_col + j)
            cs.iters[s] = 0
        req.next_col += n

    def _admit(self, queue, now, inflight):
        """Cache-aware admission.  (1) Queued requests join the contexts of
        their keys, first come first served, while slots are free.  (2) One
        factorization at a time runs beside the other contexts' iterations:
        for the key of the oldest request that has waited longer than
        age_limit, else for the key with the most waiting columns (ties:
        oldest request).  Returns True while a factorization is pending."""
        if self.pending is not None:
            self._finish_create(now)
        for req in queue:
            cs = self.ctxs.get(req.key)
            if cs is None:
                continue
            if req.hit is None:
                # the first request of a new key triggered its
                # factorization (a miss); later ones reuse it
                req.hit = self.ctxs_first.pop(req.key, True)
            self.ctxs.move_to_end(req.key)
            if req.key not in inflight:
                self._join(cs, req, now)
        queue[:] = [r for r in queue if r.pending > 0]
        waiting = [r for r in queue if r.key not in self.ctxs]
        if self.pending is None and waiting:
            old = [r for r in waiting if now - r.arrival > self.age_limit]
            if old:
                key = min(old, key=lambda r: (r.arrival, r.rid)).key
            else:
                agg = {}
                for r in waiting:
                    a = agg.setdefault(r.key, [0, r.arrival, r.rid])
                    a[0] += r.pending
                key = max(agg, key=lambda k: (agg[k][0], -agg[k][1], -agg[k][2]))
            if self._start_create(key):
                self.blocked_key = None
                self.ctxs_first[key] = False
            else:
                self.blocked_key = key
        return self.pending is not None

    def _retire(self, cs, now):
        """Read the finished step's residuals and take converged columns;
        returns the number of requests completed."""
        rel = self.ex.wait(cs.handle, cs.cap)
        done = 0
        for s in list(cs.slots):
            if rel[s] < 0:
                continue
            req, j = cs.slots[s]
            cs.iters[s] += 1
            conv = rel[s] <= self.tol
            if conv or cs.iters[s] >= self.max_iter:
                out = req.result[j] if req.result is not None else None
                self.ex.take(cs.handle, s, out)
                req.iters[j] = cs.iters[s]
                req.rel[j] = float(rel[s])
                req.failed |= not conv
                req.cols_done += 1
                del cs.slots[s]
                del cs.iters[s]
                if req.cols_done == req.R:
                    req.done = now
                    done += 1
        return done

    # main loop -------------------------------------------------------
    def run(self, requests):
        reqs = [r if isinstance(r, Request) else Request(**r) for r in requests]
        arrivals = collections.deque(sorted(reqs, key=lambda r: (r.arrival, r.rid)))
        queue = []
        inflight = collections.OrderedDict()     # key -> CtxState with a step running
        t0 = self.ex.now()
        finished = 0
        while finished < len(reqs):
            now = self.ex.now() - t0
            while arrivals and arrivals[0].arrival <= now:
                queue.append(arrivals.popleft())
            more = self._admit(queue, now, inflight) if queue else False
            for key, cs in self.ctxs.items():
                if cs.nact > 0 and key not in inflight:
                    self.ex.step(cs.handle)
                    inflight[key] = cs
                    self.steps += 1
            if not inflight:
                if more:
                    self.ex.pause()          # a factorization is running
                elif queue:
                    # nothing runs and the chosen key cannot get memory even
                    # with every idle context evicted: it never fits
                    bad = self.blocked_key if self.blocked_key is not None else queue[0].key
                    for r in [r for r in queue if r.key == bad and r.next_col == 0]:
                        queue.remove(r)
                        r.failed = True
                        r.done = now
                        finished += 1
                elif arrivals:
                    self.ex.idle_until(t0 + arrivals[0].arrival)
                continue
            progressed = False
            for key in list(inflight):
                cs = inflight[key]
                if self.ex.ready(cs.handle):
                    del inflight[key]
                    done = self._retire(cs, self.ex.now() - t0)
                    if self.progress and done and \
                            (finished + done) // self.progress > finished // self.progress:
                        print(f"served {finished + done}/{len(reqs)} requests at "
                              f"{self.ex.now() - t0:.1f} s", flush=True)
                    finished += done
                    progressed = True
            if not progressed:
                self.ex.pause()
        self.wall = self.ex.now() - t0
        return reqs

    def close(self):
        if self.pending is not None:
            while self.ex.poll_create(self.pending[1]) is None:
                self.ex.pause()
            r = self.ex.poll_create(self.pending[1])
            if r:
                self.ex.destroy(r[0])
            self.pending = None
        for cs in self.ctxs.values():
            self.ex.destroy(cs.handle)
        self.ctxs.clear()
        self.used = 0


def metrics(server, reqs):
    ok = [r for r in reqs if not r.failed]
    lat = np.array([r.done - r.arrival for r in ok]) if ok else np.zeros(1)
    wait = np.array([r.admitted - r.arrival for r in ok]) if ok else np.zeros(1)
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs) if reqs else 0.0
    cols = sum(r.R for r in ok)
    hits = [r.hit for r in reqs if r.hit is not None]
    return dict(
        requests=len(reqs), failed=len(reqs) - len(ok), rhs=cols,
        wall_s=round(span, 4),
        requests_per_s=round(len(ok) / span, 3) if span > 0 else None,
        rhs_solves_per_s=round(cols / span, 2) if span > 0 else None,
        latency_p50_ms=round(1e3 * float(np.percentile(lat, 50)), 3),
        latency_p99_ms=round(1e3 * float(np.percentile(lat, 99)), 3),
        admission_wait_p50_ms=round(1e3 * float(np.percentile(wait, 50)), 3),
        admission_wait_p99_ms=round(1e3 * float(np.percentile(wait, 99)), 3),
        cache_hit_rate=round(float(np.mean(hits)), 4) if hits else None,
        contexts_created=server.created, evictions=server.evictions,
        peak_bytes=server.peak, steps=server.steps,
        iters_mean=round(float(np.mean([i for r in ok for i in r.iters])), 3) if ok else None,
        rel_residual_max=float(max(x for r in ok for x in r.rel)) if ok else None,
    )


def main(argv=None):
    ap = argparse.ArgumentParser(description="continuous-batching serving run")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate-frac", type=float, nargs="*", default=[0.5, 0.8, 1.0],
                    help="arrival rates as fractions of the measured capacity")
    ap.add_argument("--budget-gb", type=float, nargs="*", default=[16.0, 64.0])
    ap.add_argument("--cap", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=wl.SEED_BASE + 5)
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the serving loop needs a GPU")
    for gb in a.budget_gb:
        budget = int(gb * 1e9)
        ex = HipExecutor(cap_max=a.cap, tol=a.tol)
        # capacity: the whole stream at time 0 (closed loop)
        srv = Server(ex, budget, tol=a.tol, progress=50)
        reqs = srv.run(wl.request_stream(a.requests, None, seed=a.seed))
        m = metrics(srv, reqs)
        srv.close()
        cap_rps = m["requests_per_s"]
        print(json.dumps(dict(mode="closed", budget_gb=gb, **m)), flush=True)
        for fr in a.rate_frac:
            srv = Server(ex, budget, tol=a.tol, progress=50)
            reqs = srv.run(wl.request_stream(a.requests, fr * cap_rps, seed=a.seed))
            m = metrics(srv, reqs)
            srv.close()
            print(json.dumps(dict(mode="poisson", budget_gb=gb, rate_frac=fr,
                                  rate_rps=round(fr * cap_rps, 3), **m)), flush=True)


if __name__ == "__main__":
    main()
