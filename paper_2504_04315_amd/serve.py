"""Thin binding of the serving form (include/npm_serve.h) and a load generator.

The server keeps many guiding sessions resident and batches their requests
continuously into persistent kernels; this module only marshals arguments.
`run_load` drives it with Poisson arrivals of query batches (sizes
log-uniform) and a training batch after every few queries per session, and
reports latency percentiles and aggregate throughput.
"""
import ctypes as C
import math
import threading
import time

import numpy as np

from . import npm as B
from . import workload as W

_P, _i64, _u64, _u32, _i32 = C.c_void_p, C.c_int64, C.c_uint64, C.c_uint32, C.c_int32


class npm_server_config(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("max_sessions", C.c_int32),
                ("round_vertices", C.c_int32), ("plain_path", C.c_int32), ("reserved", C.c_int32)]


class npm_request_info(C.Structure):
    _fields_ = [("submit_us", C.c_double), ("launch_us", C.c_double), ("done_us", C.c_double),
                ("round", C.c_int64), ("n", C.c_int64), ("kind", C.c_int32),
                ("session", C.c_int32)]


class npm_server_stats(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("requests_done", C.c_int64), ("vertices_done", C.c_int64),
                ("sessions", C.c_int64), ("bytes_in_use", C.c_int64), ("busy_us", C.c_double)]


SIGNATURES = {
    "npm_server_create": [_P, _P],
    "npm_server_destroy": [_P],
    "npm_session_create": [_P, _P, _P],
    "npm_session_destroy": [_P, _i32],
    "npm_session_ctx": [_P, _i32, _P],
    "npm_submit_query": [_P, _i32, _i64, _P, _P, _u64, _u32, _P, _P, _P, _P, _P],
    "npm_submit_train": [_P, _i32, _i64, _P, _P, _P, _P, _P, _P],
    "npm_wait": [_P, _u64, _i64],
    "npm_drain": [_P],
    "npm_server_hold": [_P, _i32],
    "npm_request_info_get": [_P, _u64, _P],
    "npm_server_stats_get": [_P, _P],
}

_bound = False


def lib():
    global _bound
    L = B.lib()
    if not _bound:
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        _bound = True
    return L


class Server:
    def __init__(self, budget_bytes=200 << 30, max_sessions=64, round_vertices=1 << 20,
                 plain_path=False):
        cfg = npm_server_config(budget_bytes, max_sessions, round_vertices, int(plain_path), 0)
        self._h = C.c_void_p()
        B.check(lib().npm_server_create(C.byref(cfg), C.byref(self._h)))

    def close(self):
        if self._h:
            B.check(lib().npm_server_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def create_session(self, cfg):
        sid = C.c_int32()
        B.check(lib().npm_session_create(self._h, C.byref(cfg), C.byref(sid)))
        return sid.value

    def destroy_session(self, sid):
        B.check(lib().npm_session_destroy(self._h, sid))

    def session_state(self, sid, n_params, which=B.STATE_PARAMS):
        """Host copy of a session's state buffer (synchronises the device)."""
        return session_ctx_state(self, sid, n_params, which)

    def submit_query(self, sid, pos, dir=None, seed=0, stream_id=0, lobes=None, pdf=None,
                     sdir=None, spdf=None):
        req = C.c_uint64()
        B.check(lib().npm_submit_query(self._h, sid, pos.shape[1], B._ptr(pos), B._ptr(dir), seed,
                                       stream_id, B._ptr(lobes), B._ptr(pdf), B._ptr(sdir),
                                       B._ptr(spdf), C.byref(req)))
        return req.value

    def submit_train(self, sid, pos, dir, radiance, pdf, stats=None):
        req = C.c_uint64()
        B.check(lib().npm_submit_train(self._h, sid, pos.shape[1], B._ptr(pos), B._ptr(dir),
                                       B._ptr(radiance), B._ptr(pdf), B._ptr(stats),
                                       C.byref(req)))
        return req.value

    def wait(self, req, timeout_us=-1):
        B.check(lib().npm_wait(self._h, req, timeout_us))

    def hold(self, on=True):
        """While held the server forms no round; release to run what queued."""
        B.check(lib().npm_server_hold(self._h, int(on)))

    def drain(self):
        B.check(lib().npm_drain(self._h))

    def info(self, req):
        out = npm_request_info()
        B.check(lib().npm_request_info_get(self._h, req, C.byref(out)))
        return out

    def stats(self):
        out = npm_server_stats()
        B.check(lib().npm_server_stats_get(self._h, C.byref(out)))
        return out


def session_ctx_state(server, sid, n_params, which=B.STATE_PARAMS):
    """Host copy of a session's state (through its context)."""
    ctx = C.c_void_p()
    B.check(lib().npm_session_ctx(server._h, sid, C.byref(ctx)))
    a = np.empty(n_params, dtype=np.float32)
    B.check(B.lib().npm_get_state(ctx, which, a.ctypes.data_as(C.c_void_p), a.size))
    return a


# ---------------------------------------------------------------------------
# Load generator
# ---------------------------------------------------------------------------
def plan_requests(n_sessions, per_session, rate_hz, min_log2=10, max_log2=18, train_every=4,
                  seed=0):
    """Arrival schedule: per session a Poisson stream of query batches with
    sizes log-uniform in [2^min, 2^max], and a training batch (same size law)
    after every `train_every` queries.  Returns a list of dicts sorted by time."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_sessions):
        t = 0.0
        nq = 0
        for i in range(per_session):
            t += rng.exponential(1.0 / rate_hz)
            n = int(round(2.0 ** rng.uniform(min_log2, max_log2)))
            nq += 1
            out.append(dict(t=t, session=s, kind=0, n=n))
            if nq % train_every == 0:
                n2 = int(round(2.0 ** rng.uniform(min_log2, max_log2)))
                out.append(dict(t=t, session=s, kind=1, n=n2))
    out.sort(key=lambda r: (r["t"], r["session"], r["kind"]))
    return out


def make_request_buffers(plan, n_pools=4, pool_size=1 << 18, base_seed=500):
    """Device input/output tensors for every planned request, made before the
    timed run so the submission loop does no allocation or host work.  Inputs
    are contiguous slices of a few seeded surface batches (one per session
    group, with the field's phase varied)."""
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pools = []
    for i in range(n_pools):
        b = W.make_batch("surface", pool_size, seed=base_seed + i, phase=0.3 * i, tris_seed=i)
        pools.append([t(b.pos), t(b.dir), t(b.radiance), t(b.pdf)])
    rng = np.random.default_rng(base_seed)
    for r in plan:
        P = pools[r["session"] % n_pools]
        n = r["n"]
        o = int(rng.integers(0, pool_size - n + 1))
        r["pos"] = P[0][:, o:o + n].contiguous()
        r["dir"] = P[1][:, o:o + n].contiguous()
        if r["kind"] == 0:
            r["lobes"] = torch.empty((4, 8, n), device="cuda")
            r["pdf"] = torch.empty(n, device="cuda")
            r["sdir"] = torch.empty((3, n), device="cuda")
            r["spdf"] = torch.empty(n, device="cuda")
        else:
            r["rad"] = P[2][o:o + n].contiguous()
            r["spdfin"] = P[3][o:o + n].contiguous()
            r["stats"] = torch.zeros(2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    return plan


def submit(server, sids, r, seed=7):
    if r["kind"] == 0:
        return server.submit_query(sids[r["session"]], r["pos"], r["dir"], seed=seed,
                                   stream_id=r["session"], lobes=r["lobes"], pdf=r["pdf"],
                                   sdir=r["sdir"], spdf=r["spdf"])
    return server.submit_train(sids[r["session"]], r["pos"], r["dir"], r["rad"], r["spdfin"],
                               stats=r["stats"])


def run_load(server, sids, plan, time_scale=1.0):
    """Submits the plan at its arrival times (scaled), waits for everything,
    and returns latency and throughput figures."""
    t0 = time.perf_counter()
    reqs = []
    for r in plan:
        delay = r["t"] * time_scale - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        reqs.append(submit(server, sids, r))
    server.drain()
    t1 = time.perf_counter()
    lat_q, lat_t, verts = [], [], 0
    first, last = math.inf, 0.0
    for rid, r in zip(reqs, plan):
        inf = server.info(rid)
        lat = (inf.done_us - inf.submit_us) / 1e3
        (lat_q if r["kind"] == 0 else lat_t).append(lat)
        verts += r["n"]
        first = min(first, inf.submit_us)
        last = max(last, inf.done_us)
    span_s = (last - first) / 1e6

    def pct(v):
        return dict(p50=float(np.percentile(v, 50)), p99=float(np.percentile(v, 99))) if v else None
    return dict(requests=len(plan), vertices=verts, wall_s=t1 - t0, span_s=span_s,
                vertices_per_s=verts / span_s,
                query_vertices=sum(r["n"] for r in plan if r["kind"] == 0),
                train_vertices=sum(r["n"] for r in plan if r["kind"] == 1),
                latency_ms=pct(lat_q + lat_t), query_latency_ms=pct(lat_q),
                train_latency_ms=pct(lat_t), rounds=server.stats().rounds)
