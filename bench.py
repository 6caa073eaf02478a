"""Benchmark of the NPM hot path on one MI355X.

Workload: the production-size plain FP32 configuration -- a 16-level hashed
grid (2^19 entries per level, F = 2, resolutions 16..2048), MLP
32-64-64-64-32 decoding K = 8 vMF lobes, batches of 2^20 path vertices on a
synthetic triangle set with directions and Exp(1)-noisy radiance from an
analytic 8-lobe vMF field.  One step is one pass of the whole hot path over
the batch: npm_query (encode + MLP + mappings + pdf at dir + one sample and
its pdf per vertex) followed by npm_train_step (forward, KL gradient,
backward, grid scatter, weight gradients, Adam over all parameters).  The
default run also reports the serving form, the paper's own network on its
batch sizes, NPM-product, the learned BSDF-selection probability (on the
paper's network, staged and fused), and the FP64 oracle on the host cores.

Prints one JSON line.  `value` is vertices per second through a full step
(query + train on the same batch), inputs resident in HBM.  The roofline
entry is for the kernel with the largest share of the timed region, from the
library's own HIP events on the stream the kernels run on; the CPU baseline
is the FP64 oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vertex queries/s (encode+MLP+vMF sample/pdf), train vertices/s, p99 latency"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}

# Algorithmic work per vertex of each fused kernel on the production config
# (16 levels x 8 corners x F = 2): streams in/out, element-granular grid
# gathers, 8-byte read-modify-write per FP32 atomic, and MLP FLOPs
# (2 x 12,288 weights per pass; training runs forward, delta chain and
# weight gradient = 3 passes).
GATHER_B = 16 * 8 * 2 * 4       # 16 levels x 8 corners x 2 features x 4 B
ATOMIC_B = 2 * GATHER_B          # 256 FP32 atomics, read + write
ACT_B = 3 * 64 * 4               # hidden activations of one vertex
MLP_F = 2 * 12288                # FLOPs of one pass over the 12,288 weights
WORK = {
    # fused: streams + gathers + atomics only, intermediates stay on chip
    # except the tile kernel's dG (32 FP32 per vertex), which the aggregated
    # scatter reads back; the visiting order adds 4 B per vertex to each
    "fused_query": dict(bytes=24 + 4 + GATHER_B + 160, flops=MLP_F),
    # ordered query: 160-byte staged slot read, inverse order, outputs written
    "query_unstage": dict(bytes=160 + 4 + 148, flops=0),
    "fused_backward": dict(bytes=32 + 4 + GATHER_B + 32 * 4, flops=3 * MLP_F),
    "fused_scatter": dict(bytes=12 + 4 + 32 * 4 + ATOMIC_B, flops=0),
    # counting sort: positions read twice, two counter atomics, perm (and
    # for queries its inverse) written
    "spatial_sort": dict(bytes=2 * 12 + 2 * 8 + 4, flops=0),
    # staged: each kernel's own streams (feature-major intermediates)
    "staged_encode": dict(bytes=12 + GATHER_B + 32 * 4, flops=0),
    "staged_mlp_fwd": dict(bytes=32 * 4 + 32 * 4, flops=MLP_F),
    "staged_mlp_fwd_train": dict(bytes=32 * 4 + ACT_B + 32 * 4, flops=MLP_F),
    "staged_head": dict(bytes=32 * 4 + 12 + 148, flops=0),
    "staged_loss_grad": dict(bytes=32 * 4 + 12 + 8 + 32 * 4, flops=0),
    "staged_mlp_bwd": dict(bytes=32 * 4 + ACT_B + ACT_B + 32 * 4, flops=MLP_F),
    "staged_mlp_dw": dict(bytes=2 * (ACT_B + 32 * 4 + 32 * 4), flops=MLP_F),
    "staged_scatter": dict(bytes=12 + 32 * 4 + ATOMIC_B, flops=0),
}
# Binned scatter of the production grid's hashed levels in a spatially
# ordered batch: levels 6-15 (D >= 100), 2^19 entries x F = 2 each, in slices
# of 8,192 entries: 640 bins; chunks of 1,024 vertices; one 16-byte item (the
# key, the x fraction, 2 FP32 values) per pair of x-neighbour corners and
# level.  Levels 0-5 keep the windowed scatter.
L_BINNED, L_WINDOW, T_HASH = 10, 6, 1 << 19
BIN_ITEM_B = 16
BIN_ITEMS_B = L_BINNED * 4 * BIN_ITEM_B           # 640 B per vertex
BIN_COUNTERS_B = 4 * 640 / 1024                   # one counter per bin and chunk
BIN_WORK = {
    # positions, dG of the binned levels; counters written
    "bin_count": dict(bytes=16 + L_BINNED * 2 * 4 + BIN_COUNTERS_B, flops=0),
    # two read + write passes over the counters
    "bin_scan": dict(bytes=4 * BIN_COUNTERS_B, flops=0),
    # positions, dG, the chunk's counter pairs, items written
    "bin_place": dict(bytes=16 + L_BINNED * 2 * 4 + 2 * BIN_COUNTERS_B + BIN_ITEMS_B, flops=0),
    # items read; the hashed tables' gradient read and written once per batch
    # (its per-vertex share at 2^20 vertices is added in main)
    "bin_reduce": dict(bytes=BIN_ITEMS_B, flops=0),
}
# with those levels binned the windowed scatter covers levels 0-5
FUSED_SCATTER_DENSE_B = 12 + 4 + 32 * 4 + 2 * 8 * 2 * 4 * L_WINDOW
ADAM_BYTES_PER_PARAM = 32      # read p, g, m, v; write p, m, v, g
# FP32 global atomics with random addresses, one 64-byte line per request,
# measured on the MI355X by a probe kernel: 21.1 G requests/s for the chip
ATOMIC_REQ_CEILING = 21.1e9


def kernel_sources_sha():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2504_04315_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--mode", choices=["fused", "staged"], default="fused")
    p.add_argument("--precision", choices=["fp32", "bf16"], default="fp32")
    p.add_argument("--n", type=int, default=1 << 20)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-serving", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target CPU time of the oracle baseline sample")
    p.add_argument("--profile", action="store_true",
                   help="few steps, no CPU baseline, for rocprofv3 runs")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 1 GiB device copy (counter calibration)")
    p.add_argument("--only", choices=["selection", "serving"],
                   help="run one extra leg alone (a short version, for rocprofv3 runs) and "
                        "print its JSON instead of the step benchmark")
    return p.parse_args()


def cpu_baseline(netcfg, batch, params, seconds):
    """The FP64 oracle, as it stands, on the host cores.  Query (OpenMP over
    vertices) and training step (the backward over one contiguous vertex
    range per thread, then Adam over every parameter), each timed with all
    cores and with one thread, on bounded samples of the bench's 2^20-vertex
    batch, and on cfg1's whole 16,384-vertex batch; the headline value is
    the all-core rate of a whole step (query + training) on the bench batch."""
    from oracle import oracle as O
    from paper_2504_04315_amd import workload as W
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    old = O.set_threads(threads)

    def onet(c):
        return O.Net(c.n_levels, c.feat, c.base_res, c.max_res, c.log2_table, c.dense_only,
                     c.n_hidden, c.width, c.n_lobes)

    def t_query(on, b, p, m):
        sub = b.subset(np.arange(m))
        t0 = time.perf_counter()
        O.query(on, sub.pos, p, dirs=sub.dir, seed=1, stream=0)
        return (time.perf_counter() - t0) / m

    def t_backward(on, b, p, m):
        sub = b.subset(np.arange(m))
        t0 = time.perf_counter()
        O.backward(on, sub.pos, sub.dir, sub.radiance, sub.pdf, p, n_total=b.n, with_abs=False)
        return (time.perf_counter() - t0) / m

    def t_adam(p):
        q, g, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p), np.zeros_like(p)
        t0 = time.perf_counter()
        O.adam(q, g, m, v, 1, 1e-2)
        return time.perf_counter() - t0

    def legs(on, b, p, budget, th):
        """Per-vertex query and backward times on samples sized to the budget."""
        O.set_threads(th)
        q0 = t_query(on, b, p, min(b.n, 4096 * th))
        b0 = t_backward(on, b, p, min(b.n, 1024 * th))
        mq = int(min(b.n, max(4096, 0.2 * budget / q0)))
        mb = int(min(b.n, max(1024, 0.8 * budget / b0)))
        return (t_query(on, b, p, mq), mq), (t_backward(on, b, p, mb), mb)

    out = {"unit": "vertices/s", "kind": "oracle", "cores": threads}
    on2 = onet(netcfg)
    ta2 = t_adam(params)
    rows = {}
    for th in (threads, 1):
        (q, mq), (bw, mb) = legs(on2, batch, params, seconds * (0.7 if th > 1 else 0.2), th)
        rows[th] = dict(query_vertices_per_s=1.0 / q, train_vertices_per_s=1.0 / (bw + ta2 / batch.n),
                        query_sample=mq, train_sample=mb,
                        backward_threads=O.backward_threads(on2, mb, False))
    b1 = W.make_batch("cube", W.N_CFG1, seed=1)
    on1 = onet(W.CFG1)
    rng = np.random.default_rng(1)
    p1 = np.zeros(on1.n_params)
    p1[:on1.grid_params] = rng.normal(0, 1e-2, on1.grid_params)
    for i, (o, k) in enumerate(on1.layer_shape):
        a = math.sqrt(6.0 / (o + k))
        p1[on1.layer_offset[i]:on1.layer_offset[i] + o * k] = rng.uniform(-a, a, o * k)
    ta1 = t_adam(p1)
    cfg1 = {}
    for th in (threads, 1):
        O.set_threads(th)
        q = t_query(on1, b1, p1, b1.n)
        bw = t_backward(on1, b1, p1, b1.n)
        cfg1[str(th)] = dict(query_vertices_per_s=1.0 / q,
                             train_vertices_per_s=1.0 / (bw + ta1 / b1.n),
                             backward_threads=O.backward_threads(on1, b1.n, False))
    O.set_threads(old)
    a = rows[threads]
    out["value"] = 1.0 / (1.0 / a["query_vertices_per_s"] + 1.0 / a["train_vertices_per_s"])
    out["sample"] = (f"the 2^20-vertex bench batch: query of {a['query_sample']} vertices and "
                     f"backward of {a['train_sample']} ({threads} OpenMP threads; the backward "
                     f"ran on {a['backward_threads']}), Adam over all {params.size} parameters "
                     f"(one thread, {ta2:.2f} s); per-vertex times summed and inverted; one-thread "
                     f"rates from smaller samples; cfg1 whole (16,384 vertices)")
    out["cfg2"] = {str(k): v for k, v in rows.items()}
    out["cfg1"] = cfg1
    out["query_vertices_per_s"] = a["query_vertices_per_s"]
    out["train_vertices_per_s"] = a["train_vertices_per_s"]
    return out


def serving_bench(n_sessions=32, per_session=6, load=0.7, sweep=(0.3, 0.9)):
    """The serving form on its workload: n_sessions guiding sessions (16-level
    FP16 hash grid, T = 2^17, MLP 32-64-64-64-32), each a Poisson stream of
    query batches with sizes log-uniform in 2^10..2^18 and a training batch
    after every 4 queries.  First the saturation throughput (everything
    submitted at once), the plan's queries alone and its training batches
    alone at saturation (the query and the training rates), then the mixed
    plan offered at `load` times its saturation rate (the reported latency)
    and at the `sweep` loads; both for the shared persistent kernels (BF16)
    and the per-session plain FP32 path."""
    from paper_2504_04315_amd import npm as B
    from paper_2504_04315_amd import serve as S
    from paper_2504_04315_amd import workload as W
    from dataclasses import replace
    mean_n = (2.0 ** 18 - 2.0 ** 10) / math.log(2.0 ** 8)
    out = {"sessions": n_sessions, "requests_per_session": None, "offered_load": load}
    for name, plain in (("shared_bf16", False), ("plain_fp32", True)):
        srv = S.Server(budget_bytes=200 << 30, max_sessions=n_sessions, round_vertices=1 << 20,
                       plain_path=plain)
        sids = [srv.create_session(B.make_config(replace(W.CFG5, seed=100 + i)))
                for i in range(n_sessions)]
        plan = S.plan_requests(n_sessions, per_session, rate_hz=1e9, train_every=4, seed=1)
        out["requests_per_session"] = len(plan) / n_sessions
        S.make_request_buffers(plan)
        for r in plan:                  # warm the kernels once
            r["t"] = 0.0
        S.run_load(srv, sids, plan[:n_sessions])
        sat = S.run_load(srv, sids, plan)
        # each kind alone at saturation: the query and the training rates
        sat_q = S.run_load(srv, sids, [r for r in plan if r["kind"] == 0])
        sat_t = S.run_load(srv, sids, [r for r in plan if r["kind"] == 1])
        def offered(f, seed):
            rate = f * sat["vertices_per_s"] / (n_sessions * mean_n * 1.25)
            plan2 = S.plan_requests(n_sessions, per_session, rate_hz=rate, train_every=4,
                                    seed=seed)
            S.make_request_buffers(plan2)
            return S.run_load(srv, sids, plan2)
        res = offered(load, 2)
        out[name] = {"saturation_vertices_per_s": sat["vertices_per_s"],
                     "saturation_latency_ms": sat["latency_ms"],
                     "query_only_vertices_per_s": sat_q["vertices_per_s"],
                     "train_only_vertices_per_s": sat_t["vertices_per_s"],
                     "offered_vertices_per_s": load * sat["vertices_per_s"],
                     "vertices_per_s": res["vertices_per_s"], "latency_ms": res["latency_ms"],
                     "query_latency_ms": res["query_latency_ms"],
                     "train_latency_ms": res["train_latency_ms"], "rounds": res["rounds"],
                     "sweep": {}}
        for k, f in enumerate(sweep):
            r = offered(f, 3 + k)
            out[name]["sweep"][str(f)] = {"vertices_per_s": r["vertices_per_s"],
                                          "latency_ms": r["latency_ms"]}
        srv.close()
    return out


def _median_ms(fn, reps, warm):
    """Median HIP-event time of fn(i) on the current stream over reps calls,
    after warm untimed ones."""
    import torch
    for i in range(warm):
        fn(i)
    ms = []
    for i in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn(100 + i)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return float(np.median(ms))


def _time_forms(net, nq, nt, seeds, reps, warm, product=False):
    """Median HIP-event times of fused queries of nq vertices (dir given;
    lobes, pdf, sample, sample pdf) and training steps of nt vertices, FP32
    and the precision form, on surface batches of the workload."""
    import torch
    from paper_2504_04315_amd import npm as B
    from paper_2504_04315_amd import workload as W
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    qb = W.make_batch("surface", nq, seed=seeds[0])
    tb = W.make_batch("surface", nt, seed=seeds[1])
    qa = [t(qb.pos), t(qb.dir)]
    ta = [t(tb.pos), t(tb.dir), t(tb.radiance), t(tb.pdf)]
    qx = t(W.make_aux(qb, seeds[0])) if product else None
    tx = t(W.make_aux(tb, seeds[1])) if product else None
    out = {}
    for prec in ("fp32", "bf16"):
        m = B.NPM(B.make_config(net, exec_mode=B.EXEC_FUSED, precision=prec))
        o = dict(lobes=torch.empty((4, 8, nq), device="cuda"), pdf=torch.empty(nq, device="cuda"),
                 sample_dir=torch.empty((3, nq), device="cuda"),
                 sample_pdf=torch.empty(nq, device="cuda"))

        timed = lambda fn: _median_ms(fn, reps, warm)
        lib = B.lib()
        q_ms = timed(lambda i: B.check(lib.npm_query_aux(
            m.handle, nq, B._ptr(qa[0]), B._ptr(qx), B._ptr(qa[1]), i, 0, B._ptr(o["lobes"]),
            B._ptr(o["pdf"]), B._ptr(o["sample_dir"]), B._ptr(o["sample_pdf"]), B._stream())))
        t_ms = timed(lambda i: m.train_step(*ta, aux=tx))
        out[prec] = {"query_ms": q_ms, "train_ms": t_ms,
                     "query_vertices_per_s": nq / (q_ms / 1e3),
                     "train_vertices_per_s": nt / (t_ms / 1e3)}
        m.close()
    return out


def paper_config_bench(reps=20, warm=5):
    """The paper's own network (8 dense levels 8..86 x F=4, MLP 32-64-64-32,
    lr 5e-3) on its own batch sizes: queries of one 1280x720 wavefront
    (921,600 vertices) and training steps of 2^18 vertices.  The paper's
    figures (about 3 ms and 10 ms on an RTX 3070) are context: another GPU."""
    from paper_2504_04315_amd import workload as W
    out = {"network": "8 dense levels 8..86 x F=4, MLP 32-64-64-32, K=8",
           "query_batch": W.N_PAPER_QUERY, "train_batch": W.N_PAPER_TRAIN,
           "paper": {"query_ms": 3.0, "train_ms": 10.0, "hardware": "RTX 3070"}}
    out.update(_time_forms(W.PAPER, W.N_PAPER_QUERY, W.N_PAPER_TRAIN, (71, 72), reps, warm))
    return out


def product_bench(reps=20, warm=5):
    """NPM-product (Sec. 4.3) at the production size: the 16-level hash grid
    with omega_o, normal (4 SH bands each) and roughness after G(x) -- 65
    inputs -- on 2^20-vertex queries and training steps."""
    from paper_2504_04315_amd import workload as W
    out = {"network": "16-level hash grid T=2^19 F=2 + SH4(omega_o) + SH4(normal) + roughness, "
                      "MLP 65-64-64-64-32, K=8", "query_batch": 1 << 20, "train_batch": 1 << 20}
    out.update(_time_forms(W.CFG2P, 1 << 20, 1 << 20, (81, 82), reps, warm, product=True))
    return out


def selection_bench(reps=20, warm=5):
    """The learned BSDF-selection probability (the Sec. 6.3 extension) on the
    paper's network with its extra output: queries of one 1280x720 wavefront
    returning the selection probability, and training steps of 2^18 vertices
    with the selection term, on the staged FP32 path, the fused FP32 path and
    the fused precision form; the same network without the output on the same
    path gives the extension's cost; per-kernel times of the fused FP32
    selection training step."""
    import torch
    from paper_2504_04315_amd import npm as B
    from paper_2504_04315_amd import workload as W
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nq, nt = W.N_PAPER_QUERY, W.N_PAPER_TRAIN
    qb = W.make_batch("surface", nq, seed=73)
    tb = W.make_batch("surface", nt, seed=74)
    qa = [t(qb.pos), t(qb.dir)]
    ta = [t(tb.pos), t(tb.dir), t(tb.radiance), t(tb.pdf)]
    bsdf = t(W.make_bsdf(tb, 74))
    lib = B.lib()
    out = {"network": "8 dense levels 8..86 x F=4, MLP 32-64-64-33 (32 lobe outputs + the "
                      "selection logit), K=8", "query_batch": nq, "train_batch": nt}
    forms = (("staged", B.EXEC_STAGED, "fp32"), ("fused", B.EXEC_FUSED, "fp32"),
             ("fused_bf16", B.EXEC_FUSED, "bf16"))
    for form, mode, prec in forms:
        res = {}
        for label, net in (("selection", W.PAPERS), ("without_output", W.PAPER)):
            m = B.NPM(B.make_config(net, exec_mode=mode, precision=prec))
            o = [torch.empty((4, 8, nq), device="cuda"), torch.empty(nq, device="cuda"),
                 torch.empty((3, nq), device="cuda"), torch.empty(nq, device="cuda")]
            sel = torch.empty(nq, device="cuda")
            if label == "selection":
                q = lambda i: B.check(lib.npm_query_select(
                    m.handle, nq, B._ptr(qa[0]), None, B._ptr(qa[1]), i, 0, *map(B._ptr, o),
                    B._ptr(sel), B._stream()))
                tr = lambda i: m.train_step_select(*ta, bsdf)
            else:
                q = lambda i: B.check(lib.npm_query_aux(
                    m.handle, nq, B._ptr(qa[0]), None, B._ptr(qa[1]), i, 0, *map(B._ptr, o),
                    B._stream()))
                tr = lambda i: m.train_step(*ta)
            q_ms, t_ms = _median_ms(q, reps, warm), _median_ms(tr, reps, warm)
            res[label] = {"query_ms": q_ms, "train_ms": t_ms,
                          "query_vertices_per_s": nq / (q_ms / 1e3),
                          "train_vertices_per_s": nt / (t_ms / 1e3)}
            if label == "selection" and form == "fused":
                m.set_timing(True)
                m.reset_timing()
                for i in range(reps):
                    tr(i)
                torch.cuda.synchronize()
                res[label]["train_kernels_ms"] = {k: round(v[1] / v[0], 4)
                                                  for k, v in m.kernel_times().items() if v[0]}
                m.set_timing(False)
            m.close()
        w, s0 = res["selection"], res["without_output"]
        res["cost"] = {"query": round(w["query_ms"] / s0["query_ms"] - 1.0, 4),
                       "train": round(w["train_ms"] / s0["train_ms"] - 1.0, 4)}
        out[form] = res
    return out


def load_profile(kind, workload, sha):
    """A counter summary under profiles/ (traffic_* or counters_*), if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}.json")
    if not os.path.exists(path):
        return {}
    d = json.load(open(path))
    return d if d.get("source_sha") == sha else {}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library runs "
              "the hot path on one GPU and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2504_04315_amd import npm as B
    from paper_2504_04315_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.only:
        torch.cuda.set_device(0)
        if args.only == "selection":
            leg = selection_bench(reps=3, warm=1)
        else:
            leg = serving_bench(n_sessions=8, per_session=4, sweep=())
        print(json.dumps({"leg": args.only, args.only: leg}), flush=True)
        return
    torch.cuda.set_device(0)
    netcfg = W.CFG2 if args.precision == "fp32" else W.CFG3
    n = args.n
    mode = B.EXEC_FUSED if args.mode == "fused" else B.EXEC_STAGED
    model = B.NPM(B.make_config(netcfg, exec_mode=mode))
    batch = W.make_batch("surface", n, seed=2)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pos, dirs, rad, pdf = t(batch.pos), t(batch.dir), t(batch.radiance), t(batch.pdf)
    outs = dict(lobes=torch.empty((4, 8, n), device="cuda"), pdf=torch.empty(n, device="cuda"),
                sdir=torch.empty((3, n), device="cuda"), spdf=torch.empty(n, device="cuda"))
    stats = torch.zeros(2, dtype=torch.float64, device="cuda")
    lib = B.lib()
    params0 = model.get_state().astype(np.float64) if not (args.no_cpu_baseline or args.profile) else None

    def query(seed):
        B.check(lib.npm_query(model.handle, n, B._ptr(pos), B._ptr(dirs), seed, 0,
                              B._ptr(outs["lobes"]), B._ptr(outs["pdf"]), B._ptr(outs["sdir"]),
                              B._ptr(outs["spdf"]), B._stream()))

    def train():
        B.check(lib.npm_train_step(model.handle, n, B._ptr(pos), B._ptr(dirs), B._ptr(rad),
                                   B._ptr(pdf), B._ptr(stats), B._stream()))

    steps = 3 if args.profile else args.steps
    warm = 1 if args.profile else args.warmup
    for i in range(warm):
        query(i)
        train()
    torch.cuda.synchronize()
    print(f"warmup done ({warm} steps)", file=sys.stderr, flush=True)

    # ---- timed region: K full steps, each bracketed by events
    model.set_timing(True)
    model.reset_timing()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        query(100 + i)
        ev[3 * i + 1].record()
        train()
        ev[3 * i + 2].record()
        ev[3 * i + 3].record()
    ev[3 * steps].record()
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[3 * steps])
    step_ms, q_ms, t_ms = [], [], []
    prev = ev[0]
    for i in range(steps):
        q_ms.append(prev.elapsed_time(ev[3 * i + 1]))
        t_ms.append(ev[3 * i + 1].elapsed_time(ev[3 * i + 2]))
        step_ms.append(prev.elapsed_time(ev[3 * i + 3]))
        prev = ev[3 * i + 3]
    kt = model.kernel_times()
    model.set_timing(False)
    ms_per_step = total_ms / steps
    print(f"timed {steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    # ---- achievable rates of this device (after the timed region; not in a
    # profiled run, whose kernel list it would join)
    peaks = None if args.profile else B.measure_peaks(reps=3)
    if peaks is not None:
        print("achievable: " + ", ".join(f"{k} {v:.0f}" for k, v in peaks.items()),
              file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel
    sha = kernel_sources_sha()
    traffic = load_profile("traffic", f"cfg2_{args.precision}_{args.mode}", sha)
    measured = load_profile("counters", f"cfg2_{args.precision}_{args.mode}", sha)
    np_params = model.n_params
    work = dict(WORK)
    if "bin_reduce" in kt:
        work.update(BIN_WORK)
        work["bin_reduce"] = dict(bytes=BIN_ITEMS_B + 2 * L_BINNED * T_HASH * 2 * 4 / n, flops=0)
        work["fused_scatter"] = dict(bytes=FUSED_SCATTER_DENSE_B, flops=0)
    rows = {}
    for name, (launches, tot) in kt.items():
        if launches == 0:
            continue
        avg_s = tot / launches / 1e3
        if name in work:
            w = work[name]
            rows[name] = dict(avg_ms=avg_s * 1e3, launches=launches,
                              gbs=w["bytes"] * n / avg_s / 1e9,
                              tflops=w["flops"] * n / avg_s / 1e12)
        elif name == "adam":
            rows[name] = dict(avg_ms=avg_s * 1e3, launches=launches,
                              gbs=ADAM_BYTES_PER_PARAM * np_params / avg_s / 1e9, tflops=0.0)
        else:
            rows[name] = dict(avg_ms=avg_s * 1e3, launches=launches, gbs=None, tflops=None)
    known = [k for k in kt if k in work or k == "adam"]
    dom = max(known, key=lambda k: kt[k][1])
    r = rows[dom]
    dtype = args.precision if args.precision == "bf16" else "f32"
    peak_tf = PEAK_TFLOPS[dtype]
    if dom == "adam" or dom not in work or r["tflops"] / peak_tf < r["gbs"] / HBM_PEAK_GBS:
        bound, achieved, peak, unit = "hbm", r["gbs"], HBM_PEAK_GBS, "GB/s"
        per_launch = (work[dom]["bytes"] * n if dom in work else ADAM_BYTES_PER_PARAM * np_params)
    else:
        bound, achieved, peak, unit = "mfma", r["tflops"], peak_tf, "TFLOP/s"
        per_launch = work[dom]["flops"] * n
    tr = traffic.get("kernels", {}).get(dom)
    roof = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "kernel": dom,
            "kernel_avg_ms": round(r["avg_ms"], 4), "algorithmic_per_launch": per_launch,
            # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters
            # (copy-calibrated), null when the kernels changed since
            "traffic": None if tr is None else tr["fetch_bytes"] + tr["write_bytes"],
            "traffic_fetch_write": (None if tr is None else [tr["fetch_bytes"], tr["write_bytes"]])}
    if peaks is not None:
        # the same kernel against what this device reaches with a plain kernel
        # of the bounding kind (matrix instructions alone, or the better of a
        # 2 GiB read stream and a 1 GiB copy)
        ach = (peaks["mfma_bf16_tflops" if dtype == "bf16" else "mfma_f32_tflops"]
               if bound == "mfma" else max(peaks["hbm_copy_gbs"], peaks["hbm_read_gbs"]))
        roof["achievable_peak"] = round(ach, 2)
        roof["frac_of_achievable"] = round(achieved / ach, 4)
    mc = measured.get("kernels", {}).get(dom)
    if mc is not None:
        # counter evidence beside the time-derived fraction (rocprofv3 --pmc):
        # MFMA, VALU and LDS busy fractions of the SIMDs, the L2 hit rate
        roof["measured"] = {k: round(v, 4) for k, v in mc.items()
                            if k in ("mfma_busy", "valu_busy", "lds_busy", "l2_hit")}
    if tr is not None and tr.get("atomic_requests"):
        # the FP32 grid-gradient atomics are executed at the memory side, one
        # request per 64-byte line and wave instruction; their rate, not the
        # bytes, bounds the scatter (ceiling from a random-address probe)
        rate = tr["atomic_requests"] / (r["avg_ms"] / 1e3)
        roof["atomics"] = {"requests_per_launch": tr["atomic_requests"],
                           "requests_per_s": round(rate), "ceiling_per_s": ATOMIC_REQ_CEILING,
                           "frac": round(rate / ATOMIC_REQ_CEILING, 4)}
    line = {
        "metric": METRIC,
        "value": n / (ms_per_step / 1e3),
        "unit": "vertices/s",
        "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"cfg2 production size: 2^20 vertices on a synthetic triangle set, "
                               f"16-level hash grid T=2^19 F=2 (16..2048), MLP 32-64-64-64-32, "
                               f"K=8; step = query + train step",
                   "n": n, "precision": args.precision, "exec": args.mode},
        "query_vertices_per_s": n / (np.median(q_ms) / 1e3),
        "train_vertices_per_s": n / (np.median(t_ms) / 1e3),
        "step_latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                            "p99": float(np.percentile(step_ms, 99))},
        "query_latency_ms": {"p50": float(np.percentile(q_ms, 50)),
                             "p99": float(np.percentile(q_ms, 99))},
        "train_latency_ms": {"p50": float(np.percentile(t_ms, 50)),
                             "p99": float(np.percentile(t_ms, 99))},
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in rows.items()},
        "roofline": roof,
        "loss_last_step": float(stats[0].item()),
    }
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if peaks is not None:
        line["achievable_peaks"] = {k: round(v, 1) for k, v in peaks.items()}
    if not (args.no_serving or args.profile):
        print("serving ...", file=sys.stderr, flush=True)
        line["serving"] = serving_bench()
        line["p99_latency_ms"] = line["serving"]["shared_bf16"]["latency_ms"]["p99"]
    if not (args.no_serving or args.profile):
        print("paper configuration ...", file=sys.stderr, flush=True)
        line["paper_config"] = paper_config_bench()
        print("NPM-product ...", file=sys.stderr, flush=True)
        line["product"] = product_bench()
        print("learned selection probability ...", file=sys.stderr, flush=True)
        line["selection"] = selection_bench()
    if not (args.no_cpu_baseline or args.profile):
        print("cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(netcfg, batch, params0, args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    model.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
