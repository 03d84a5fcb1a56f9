"""Scheduling logic of the serving loop on the host: admission by HBM
budget, LRU eviction of idle contexts, column-granular continuous batching,
asynchronous servicing of contexts, failure of requests that can never fit.
The executor is a stub with a virtual clock; no device is touched."""

import numpy as np
import pytest

from paper_2003_02585_amd import serve
from paper_2003_02585_amd import workloads as wl


class StubExecutor:
    """Virtual device: a context of key (N, n_a, yi, ppw) takes
    factor_cost(N) to create, N^2 * col_bytes per slot plus N^2 * fac_bytes
    of factors, and a step costs step_cost(N) whatever the column count.
    Column j of a request converges after conv_iters(key) steps."""

    def __init__(self, cap_max=4, col_bytes=1.0, fac_bytes=2.0):
        self.t = 0.0
        self.cap_max = cap_max
        self.col_bytes = col_bytes
        self.fac_bytes = fac_bytes
        self.live = {}
        self.next_id = 0
        self.taken = []
        self.adds = []
        self.created = []
        self.pending = []
        self.max_concurrent_steps = 0

    # model
    @staticmethod
    def conv_iters(key):
        return 3 if key[2] is None else 5

    @staticmethod
    def step_cost(N):
        return 1e-3 * (N / 256) ** 2

    def now(self):
        return self.t

    def idle_until(self, t):
        self.t = max(self.t, t)

    def pause(self):
        busy = [h["finish"] for h in self.live.values() if h["finish"] is not None]
        busy += [tok["ready"] for tok in self.pending]
        self.t = max(self.t, min(busy)) if busy else self.t + 1e-5

    def start_create(self, key, free, slot_bytes=None):
        # factors must fit at set-up; the factorization then runs in the
        # background for factor_cost(N) of virtual time
        N = key[0]
        fb = self.fac_bytes * N * N
        per = self.col_bytes * N * N
        sb = free if slot_bytes is None else min(free, slot_bytes)
        cap = 0
        if free - fb >= per:
            cap = int(min(self.cap_max, max(1, (sb - fb) // per)))
        if cap < 1:
            return None
        assert not self.pending, "one factorization at a time"
        tok = dict(key=key, cap=cap, nbytes=int(fb + cap * per),
                   ready=self.t + 1e-3 * (N / 256) ** 2)
        self.pending.append(tok)
        self.created.append(key)
        return tok

    def poll_create(self, tok):
        if self.t < tok["ready"]:
            return None
        if tok in self.pending:
            self.pending.remove(tok)
            hid = self.next_id
            self.next_id += 1
            tok["h"] = dict(id=hid, key=tok["key"], cap=tok["cap"], slots={}, finish=None,
                            stepped=set())
            self.live[hid] = tok["h"]
        return tok["h"], tok["nbytes"], tok["cap"]

    def add(self, h, req, c0, n):
        free = [s for s in range(h["cap"]) if s not in h["slots"]]
        assert len(free) >= n
        out = []
        for j in range(n):
            s = free[j]
            h["slots"][s] = dict(req=req.rid, col=c0 + j, it=0)
            out.append(s)
        self.adds.append((req.rid, c0, n))
        return out

    def step(self, h):
        assert h["finish"] is None, "step while a step is in flight"
        h["finish"] = self.t + self.step_cost(h["key"][0])
        h["stepped"] = set(h["slots"])
        n = sum(1 for x in self.live.values() if x["finish"] is not None)
        self.max_concurrent_steps = max(self.max_concurrent_steps, n)

    def ready(self, h):
        return h["finish"] is not None and self.t >= h["finish"]

    def wait(self, h, cap):
        self.t = max(self.t, h["finish"])
        h["finish"] = None
        rel = np.full(cap, -1.0)
        need = self.conv_iters(h["key"])
        for s in h["stepped"]:
            st = h["slots"][s]
            st["it"] += 1
            rel[s] = 0.1 ** st["it"] if st["it"] < need else 1e-12
        return rel

    def take(self, h, s, out=None):
        st = h["slots"].pop(s)
        self.taken.append((st["req"], st["col"], st["it"]))

    def result_buffer(self, h, R):
        return None

    def destroy(self, h):
        assert not h["slots"], "destroying a context with occupied slots"
        del self.live[h["id"]]


def _reqs(spec):
    """spec: list of (arrival, key, R)."""
    out = []
    for i, (t, key, R) in enumerate(spec):
        out.append(dict(rid=i, arrival=t, key=key, positions=np.full((R, 2), 0.5)))
    return out


K256 = (256, 64, None, 10)
K512 = (512, 64, None, 10)
K512L = (512, 64, 0.37, 10)
K1024 = (1024, 128, None, 8)


def _check_complete(ex, reqs):
    # every column of every request is taken exactly once, after exactly
    # the stub's convergence count
    got = sorted((r, c) for r, c, _ in ex.taken)
    want = sorted((r.rid, c) for r in reqs if not r.failed for c in range(r.R))
    assert got == want
    for r in reqs:
        if r.failed:
            continue
        assert r.admitted >= r.arrival - 1e-12
        assert r.done >= r.admitted
        assert all(it == StubExecutor.conv_iters(r.key) for it in r.iters)


def test_all_requests_complete_and_columns_taken_once():
    spec = [(0.0, K256, 3), (0.0, K512, 2), (0.001, K256, 4), (0.002, K512L, 1),
            (0.004, K256, 2), (0.03, K1024, 3)]
    ex = StubExecutor(cap_max=4)
    srv = serve.Server(ex, budget_bytes=1e9, tol=1e-10)
    reqs = srv.run(_reqs(spec))
    _check_complete(ex, reqs)
    m = serve.metrics(srv, reqs)
    assert m["failed"] == 0 and m["rhs"] == 15
    # K256 requested three times: one miss, two hits (the later arrivals
    # find its context)
    hits = [r.hit for r in reqs]
    assert hits == [False, False, True, False, True, False]
    assert m["cache_hit_rate"] == pytest.approx(2 / 6, abs=1e-4)
    assert srv.evictions == 0 and srv.created == 4


def test_request_larger_than_capacity_is_admitted_column_by_column():
    ex = StubExecutor(cap_max=3)
    srv = serve.Server(ex, budget_bytes=1e9)
    reqs = srv.run(_reqs([(0.0, K256, 8)]))
    _check_complete(ex, reqs)
    # columns joined in groups no larger than the capacity, in order
    assert [a for a in ex.adds] == [(0, 0, 3), (0, 3, 3), (0, 6, 2)]


def test_budget_is_respected_and_idle_contexts_evicted():
    # budget holds one 512 context (factors 2*512^2, one slot 512^2) but not two
    budget = 3.5 * 512 * 512
    spec = [(0.0, K512, 1), (0.0, K512L, 1), (0.0, K256, 1), (0.05, K512, 1)]
    ex = StubExecutor(cap_max=1)
    srv = serve.Server(ex, budget_bytes=budget)
    reqs = srv.run(_reqs(spec))
    _check_complete(ex, reqs)
    assert srv.peak <= budget
    assert srv.evictions >= 2
    # the second 512 key waited for the first to retire and be evicted
    assert reqs[1].admitted >= reqs[0].done


def test_blocked_request_is_not_starved_by_later_new_keys():
    # after K512L is blocked on memory, later requests may join K512 (which
    # exists) but must not create new contexts ahead of K512L, although the
    # K256 context would fit in what is left
    budget = 5.0 * 512 * 512
    spec = [(0.0, K512, 1), (0.0, K512L, 1), (0.0, K256, 1), (0.0, K512, 1)]
    ex = StubExecutor(cap_max=2)
    srv = serve.Server(ex, budget_bytes=budget, ctx_share=1.0)
    reqs = srv.run(_reqs(spec))
    _check_complete(ex, reqs)
    assert ex.created.index(K512L) < ex.created.index(K256)
    # the two K512 requests share the first context and join it together
    assert ex.created[0] == K512 and reqs[3].admitted == reqs[0].admitted


def test_request_that_never_fits_fails_without_hanging():
    ex = StubExecutor(cap_max=2)
    srv = serve.Server(ex, budget_bytes=3.5 * 256 * 256)    # no 512 context fits
    reqs = srv.run(_reqs([(0.0, K512, 2), (0.0, K256, 1)]))
    assert reqs[0].failed and not reqs[1].failed
    m = serve.metrics(srv, reqs)
    assert m["failed"] == 1 and m["rhs"] == 1


def test_contexts_are_serviced_asynchronously():
    # a small key's request does not wait for the steps of a large key: its
    # latency is its own steps, far below one large step
    spec = [(0.0, K1024, 2), (0.0, K256, 1)]
    ex = StubExecutor(cap_max=4)
    srv = serve.Server(ex, budget_bytes=1e9)
    reqs = srv.run(_reqs(spec))
    _check_complete(ex, reqs)
    small, big = reqs[1], reqs[0]
    assert ex.max_concurrent_steps == 2
    lat_small = small.done - small.arrival
    assert lat_small < 3 * StubExecutor.step_cost(256) + 0.02      # own steps + factors
    assert lat_small < StubExecutor.step_cost(1024) * 3


def test_cache_aware_admission_prefers_the_most_waiting_columns():
    # with everything queued at once and room for one context at a time,
    # the key with the most waiting columns is factored first, and each key
    # is factored once
    budget = 4.0 * 512 * 512
    spec = [(0.0, K512L, 1), (0.0, K512, 2), (0.0, K512L, 1), (0.0, K512, 3),
            (0.0, K512L, 1)]
    ex = StubExecutor(cap_max=8)
    srv = serve.Server(ex, budget_bytes=budget, ctx_share=1.0)
    reqs = srv.run(_reqs(spec))
    _check_complete(ex, reqs)
    assert ex.created == [K512, K512L]
    assert srv.created == 2 and srv.evictions == 1


def test_old_requests_are_factored_first():
    # past the age limit the oldest waiting request's key goes first
    budget = 4.0 * 512 * 512
    spec = [(0.0, K512L, 1), (0.0, K512, 2), (0.0, K512, 3)]
    ex = StubExecutor(cap_max=8)
    srv = serve.Server(ex, budget_bytes=budget, ctx_share=1.0, age_limit=-1.0)
    reqs = srv.run(_reqs(spec))
    _check_complete(ex, reqs)
    assert ex.created == [K512L, K512]


def test_request_stream_recipe():
    a = wl.request_stream(200, 5.0, seed=wl.SEED_BASE + 5)
    b = wl.request_stream(200, 10.0, seed=wl.SEED_BASE + 5)
    # same requests at another rate: same content, arrival times halved
    assert [r["key"] for r in a] == [r["key"] for r in b]
    assert np.allclose([r["arrival"] for r in a], [2 * r["arrival"] for r in b])
    assert all(np.array_equal(x["positions"], y["positions"]) for x, y in zip(a, b))
    keys = {r["key"] for r in a}
    for N, n_a, yi, ppw in keys:
        assert N in wl.SERVE_SIZES and n_a in wl.SERVE_SUBDOMAINS and ppw in wl.SERVE_PPW
        assert N % n_a == 0
        if yi is not None:
            # the interface lies on no subdomain boundary
            assert abs(yi * N / n_a - round(yi * N / n_a)) > 1e-6
    R = [len(r["positions"]) for r in a]
    assert min(R) >= 1 and max(R) <= wl.SERVE_RMAX
    frac_const = np.mean([r["key"][2] is None for r in a])
    assert 0.35 < frac_const < 0.65
    gaps = np.diff([r["arrival"] for r in a])
    assert abs(np.mean(gaps) - 0.2) < 0.05


def test_stub_sources_match_workload_sources():
    # the serving path builds sources as an outer product of per-axis
    # Gaussians; on the host that equals the workload generator bitwise
    N, h = 64, 1.0 / 64
    p = (0.31, 0.72)
    gx = wl.gaussian_axis(N, h, p[0], 2 * h)
    gy = wl.gaussian_axis(N, h, p[1], 2 * h)
    f = (gx[None, :] * gy[:, None]) / wl.gaussian_mass(2, 2 * h)
    assert np.array_equal(f, wl.gaussian_source((N, N), h, p, 2 * h))


def test_factorization_runs_beside_other_contexts():
    # a large key is factored while a small key's iterations go on: the
    # small request finishes long before the large factorization ends
    K2048 = (2048, 128, None, 10)
    spec = [(0.0, K512, 1), (0.0005, K2048, 1)]
    ex = StubExecutor(cap_max=4)
    srv = serve.Server(ex, budget_bytes=1e9)
    reqs = srv.run(_reqs(spec))
    _check_complete(ex, reqs)
    small, big = reqs
    factor_big = 1e-3 * (2048 / 256) ** 2
    assert small.done < 0.02 < factor_big
    assert big.done > factor_big
