"""Benchmark: observed-entry SGLD updates/s of the PSGLD sampler on one MI355X.

Workload (default): the large recommender-shaped sparse Gaussian MF,
I = 480,000 rows, J = 17,800 columns, 100M observed ratings (90M training,
10M held out), Zipf(1.1) column popularity and lognormal row activity, fit
K = 100, B = 64, T = 1000 iterations with burn-in 500 and moments kept every
10th post-burn-in iteration.  A step is one PSGLD iteration (one part).

The timed region is one psgld_step call of K iterations from t = 0 (the
chain's state after the warmup is rolled back), with the data resident in
HBM.  value = training entries visited / elapsed seconds.  The sampler
kernel's average launch duration is the same events' elapsed time over the
iterations (one launch each, back to back); the roofline fraction divides the
mean algorithmic bytes of those iterations by it.  A second pass replays the
same iterations with HIP events around every launch, for the averages before
and after burn-in.  A third pass runs the workload's whole chain (T
iterations from t = 0, moments and held-out sums after burn-in) and reports
its held-out RMSE beside the FP64 oracle's stored full run, so the rate is
quoted at a held-out RMSE matched to the oracle's.  The FP64 oracle is timed
on the host's cores on a bounded sample (cpu_baseline), with all threads and
with one.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "observed-entry SGLD updates/s at matched held-out RMSE; served-job p50/p99"
# The paper's own figures for the same metric and workload shape (another
# GPU: a GeForce GT 750M), as lower bounds of observed-entry updates/s:
# Poisson NMF 1024 x 1024, K = 32, B = 32, 10,000 samples in under 15 s
# (Section 4.2.1); the 256 x 256, K = 8, B = 8 spectrum, 10,000 samples in
# 3.5 s (Section 4.2.2, stood in for by synthetic Poisson NMF data).
PAPER_UPDATES_PER_S = {"paper_poisson_1024": 10_000 * 1024 * 1024 / 32 / 15.0,
                       "paper_spectrum_256": 10_000 * 256 * 256 / 8 / 3.5}
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "bf16v": 2500.0}
# Stored bytes of a dense cell's training value per precision (bf16v: the
# values themselves stored in BF16).
VALUE_BYTES = {"f32": 4, "bf16": 4, "bf16v": 2}


class HipEvents:
    """hipEvent timing on a given stream, through the HIP runtime's C API."""

    def __init__(self):
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]

    def create(self, n):
        evs = []
        for _ in range(n):
            e = C.c_void_p()
            assert self.hip.hipEventCreate(C.byref(e)) == 0
            evs.append(e)
        return evs

    def record(self, ev, stream):
        assert self.hip.hipEventRecord(ev, C.c_void_p(stream)) == 0

    def elapsed_ms(self, a, b):
        assert self.hip.hipEventSynchronize(b) == 0
        ms = C.c_float()
        assert self.hip.hipEventElapsedTime(C.byref(ms), a, b) == 0
        return float(ms.value)

    def sync(self):
        assert self.hip.hipDeviceSynchronize() == 0


# The library's default placement of the blocks of a dense load: a block
# runs on the dense kernels when it has at most 128 rows, at least 256
# columns, K <= 64 and a training density above 0.3 (contiguous pieces);
# every other block runs as coordinates.
DENSE_MAX_ROWS, DENSE_MIN_COLS, DENSE_MAX_K, DENSE_THRESHOLD = 128, 256, 64, 0.3


def block_placement(wl):
    """(dense, cnt, rows, cols): which blocks (b, c) run on the dense kernels,
    the training entries of every block and the sizes of the pieces."""
    rp, cp = pkg_pieces(wl, "row"), pkg_pieces(wl, "col")
    rows, cols = np.bincount(rp, minlength=wl.B), np.bincount(cp, minlength=wl.B)
    cnt = np.zeros((wl.B, wl.B), dtype=np.int64)
    np.add.at(cnt, (rp[wl.row], cp[wl.col]), 1)
    size = rows[:, None].astype(np.float64) * cols[None, :]
    dense = ((rows[:, None] <= DENSE_MAX_ROWS) & (cols[None, :] >= DENSE_MIN_COLS) & (wl.K <= DENSE_MAX_K)
             & (cnt > DENSE_THRESHOLD * size))
    return dense, cnt, rows, cols


def part_work(wl, dense, cnt, rows, cols):
    """Per part p: cells of its dense-kernel blocks (all cells, masked or
    not: the dense kernels stream every cell) and training entries of its
    blocks that run as coordinates."""
    cells = np.zeros(wl.B, dtype=np.int64)
    entries = np.zeros(wl.B, dtype=np.int64)
    for p in range(wl.B):
        for b in range(wl.B):
            c = (b + p) % wl.B
            if dense[b, c]:
                cells[p] += int(rows[b]) * int(cols[c])
            else:
                entries[p] += int(cnt[b, c])
    return cells, entries


def algorithmic_cost(wl, cells_p, entries_p, ho_p, t, p, value_bytes=4):
    """(bytes, flops) one iteration must move and compute at minimum: each
    training entry of the part's coordinate blocks read once (4-byte index +
    4-byte value), each cell of its dense blocks read once (its value in the
    stored precision, value_bytes, + one bit of training mask), every factor
    element read and written once in
    FP32, the FP64 sums of x and x^2 read and written at kept iterations, one
    FP64 read-modify-write per held-out cell of the part after burn-in; 6K
    flops per dense cell for mu = W H, G_H = W^T E and G_W = E H^T.  p is the
    part of iteration t."""
    b = (value_bytes + 0.125) * cells_p[p] + 8 * entries_p[p] + 8 * (wl.I + wl.J) * wl.K
    if t >= wl.burn_in:
        b += 16 * ho_p[p]
        if (t - wl.burn_in) % wl.thin == 0:
            b += 32 * (wl.I + wl.J) * wl.K
    return b, 6 * wl.K * cells_p[p]


# Sources of each kernel family: a traffic measurement stored in
# profiles/traffic.json applies only while these files are unchanged.
KERNEL_SOURCES = {
    "sparse": ["sparse.hip", "internal.hpp", "noise.hpp", "model.hpp"],
    "dense": ["dense.hip", "internal.hpp", "noise.hpp", "model.hpp"],
}


def source_digest(kind):
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1506_01418_amd", "csrc")
    for name in KERNEL_SOURCES[kind]:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(key, kind):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters stored in
    profiles/traffic.json (each scaled by the copy-kernel reference), or None
    when there is no measurement or the kernel's sources changed since."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    run = data.get("runs", {}).get(key)
    if not run or run.get("source_sha256") != source_digest(kind):
        return None
    ref = data["copy_reference"]
    return 1024.0 * (run["FETCH_SIZE_KiB"] * ref["fetch_scale"] + run["WRITE_SIZE_KiB"] * ref["write_scale"])


def stored_oracle_rmse(wl):
    """The FP64 oracle's held-out RMSE after the same whole run, as stored in
    tests/golden/heldout_rmse.json (written from the oracle alone), or None."""
    path = os.path.join(ROOT, "tests", "golden", "heldout_rmse.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f).get(wl.name)
    if not ref or (ref["T"], ref["burn_in"], ref["thin"], ref["n_heldout"]) != (wl.T, wl.burn_in, wl.thin,
                                                                                 len(wl.hval)):
        return None
    return ref["heldout_rmse"]


def stored_oracle_trace(wl, every):
    """Mean training log-likelihood of the oracle's whole run over the trace
    points of its second half, from tests/golden/ll_trace.json, or None."""
    path = os.path.join(ROOT, "tests", "golden", "ll_trace.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f).get(wl.name)
    if not ref or ref["T"] != wl.T or ref["every"] != every:
        return None
    return float(np.mean([p[1] for p in ref["points"] if p[0] > wl.T // 2]))


def make_workload(name):
    try:
        return workloads.by_name(name)
    except KeyError as e:
        raise SystemExit(str(e))


def cpu_baseline(wl, seconds, part_order="cyclic", row_piece=None, col_piece=None, iters=0, single_iters=1):
    """The oracle on the host: iterations from t = 0 with all its threads
    until `seconds` of oracle time have passed (at least two iterations, or
    exactly `iters`), then `single_iters` more on one thread.  Bucketing the
    entries (once per chain) is not timed."""
    import oracle
    threads = oracle.threads(int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1))
    cfg = oracle.Config(**wl.fit_kwargs())
    cfg.part_order = part_order
    ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol,
                      row_piece=row_piece, col_piece=col_piece)
    n_p = ch.part_sizes()
    ch._prepared()

    def timed(n_max, budget):
        done, dt, ent = 0, 0.0, 0
        while done < n_max and (done < 2 or dt < budget):
            t = ch.t
            t0 = time.perf_counter()
            ch.run(1)
            dt += time.perf_counter() - t0
            ent += int(n_p[ch.part_at(t)])
            done += 1
        return done, dt, ent

    done, dt, ent = timed(iters if iters > 0 else 10 ** 9, seconds if iters <= 0 else float("inf"))
    oracle.threads(1)
    d1, dt1, ent1 = timed(max(single_iters, 1), 0.0)
    oracle.threads(threads)
    return {"value": ent / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "single_thread_value": ent1 / dt1,
            "sample": f"{done} iterations from t=0 of the same workload on {threads} threads "
                      f"({dt:.1f} s of oracle time), then {d1} on one thread ({dt1:.1f} s); FP64 C, "
                      f"threads over the blocks of a part and the rows/columns of the update"}


def serve_main(args):
    """Serving stream: jobs arrive as a Poisson process (rate 0: all at once),
    are admitted FIFO under the HBM budget and stepped together; latency is
    finish minus arrival on the host clock.  value = training-entry updates of
    all jobs / makespan (first arrival to last finish)."""
    import paper_1506_01418_amd as pkg

    t_gen = time.perf_counter()
    jobs = [workloads.serving_job(j, T=args.job_iters, burn_in=args.job_iters // 2) for j in range(args.jobs)]
    arrivals = workloads.job_arrivals(args.jobs, args.rate)
    print(f"[bench] {args.jobs} jobs generated in {time.perf_counter() - t_gen:.1f} s "
          f"({sum(wl.nnz for wl in jobs)} training entries, {sum(wl.dense is not None for wl in jobs)} dense)",
          file=sys.stderr, flush=True)
    srv = pkg.Server(int(args.budget_gib * (1 << 30)), max_active=args.max_active,
                     iters_per_tick=args.iters_per_tick, persistent=args.persistent)
    # warm-up: one small job through the whole path (kernel loading, allocator)
    wid = srv.submit(workloads.serving_job(10_000, T=args.iters_per_tick, burn_in=0), args.iters_per_tick)
    while srv.tick()[:2] != (0, 0):
        pass
    srv.release(wid)
    ids, finish, rejected = {}, {}, []
    nxt, t0 = 0, time.perf_counter()
    ticks, max_running = 0, 0
    while len(finish) < args.jobs:
        now = time.perf_counter() - t0
        while nxt < args.jobs and arrivals[nxt] <= now:
            wl = jobs[nxt]
            try:
                ids[srv.submit(wl, args.job_iters, dense=wl.dense is not None)] = nxt
            except pkg.PsgldError:
                rejected.append(nxt)       # needs more device memory than the whole budget
                finish[nxt] = None
            nxt += 1
        running, queued, retired = srv.tick()
        ticks += 1
        max_running = max(max_running, running)
        if retired:
            now = time.perf_counter() - t0
            for jid, j in list(ids.items()):
                st = srv.info(jid)["state"]
                if st in (pkg.PSGLD_JOB_DONE, pkg.PSGLD_JOB_FAILED):
                    if st == pkg.PSGLD_JOB_FAILED:
                        raise SystemExit(f"job {j} failed: {srv.error(jid)}")
                    finish[j] = now
                    srv.release(jid)
                    del ids[jid]
        if running == 0 and queued == 0 and nxt < args.jobs:
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
    srv.close()
    served = [j for j in range(args.jobs) if finish[j] is not None]
    lat = np.array([finish[j] - arrivals[j] for j in served])
    makespan = max(finish[j] for j in served) - float(arrivals[0])
    updates = float(sum(jobs[j].nnz * args.job_iters for j in served))
    value = updates / makespan
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
    print(f"[bench] serve: {len(served)} jobs ({len(rejected)} over the budget) in {makespan:.2f} s, "
          f"p50 {p50 * 1e3:.1f} ms, p99 {p99 * 1e3:.1f} ms, "
          f"{value:.4g} updates/s, {ticks} ticks, at most {max_running} running", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.job_iters,
        "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serve_c5_{args.jobs}jobs", "jobs": args.jobs, "rate_per_s": args.rate,
                   "hbm_budget_gib": args.budget_gib, "iters_per_job": args.job_iters,
                   "iters_per_tick": args.iters_per_tick, "max_active": args.max_active,
                   "persistent": bool(args.persistent),
                   "parallelism": "single-gpu"},
        "serving": {"p50_ms": p50 * 1e3, "p99_ms": p99 * 1e3, "jobs_per_s": len(served) / makespan,
                    "rejected_over_budget": len(rejected),
                    "makespan_s": makespan, "ticks": ticks, "max_running": max_running},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sparse_ratings_480k")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle time on all threads for the CPU baseline")
    ap.add_argument("--cpu-single-iters", type=int, default=1,
                    help="oracle iterations on one thread for the CPU baseline")
    ap.add_argument("--no-full-chain", action="store_true",
                    help="skip the whole-chain pass (held-out RMSE after T iterations)")
    ap.add_argument("--trace-every", type=int, default=0,
                    help="mixing trace: a whole-chain pass recording the training log-likelihood every this "
                         "many iterations against the sampler's time (0: off)")
    ap.add_argument("--cpu-iters", type=int, default=0, help="exact oracle iterations instead (0: by time)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", choices=["f32", "bf16", "bf16v"], default="f32",
                    help="dense-block kernels: FP32 operands, BF16 operands, or BF16 operands with the "
                         "training values also stored in BF16")
    ap.add_argument("--quads-per-lane", type=int, default=0,
                    help="with --entries-per-group: use that schedule and kernel variant without tuning")
    ap.add_argument("--entries-per-group", type=int, default=0,
                    help="fix the sparse schedule's entries per group instead of tuning it")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with one 256 MiB device-to-device copy kernel (torch), the reference "
                         "for scaling HBM traffic counters")
    ap.add_argument("--jobs", type=int, default=200, help="serve_c5: number of jobs")
    ap.add_argument("--rate", type=float, default=20.0, help="serve_c5: arrivals per second (0: all at once)")
    ap.add_argument("--budget-gib", type=float, default=8.0, help="serve_c5: HBM budget of the running jobs")
    ap.add_argument("--iters-per-tick", type=int, default=25, help="serve_c5: iterations per job per tick")
    ap.add_argument("--max-active", type=int, default=64, help="serve_c5: running jobs at most")
    ap.add_argument("--job-iters", type=int, default=500, help="serve_c5: iterations per job")
    ap.add_argument("--persistent", action="store_true",
                    help="run iterations in cooperative single launches (coordinate-stored contexts)")
    ap.add_argument("--graph-iters", type=int, default=-1,
                    help="iterations per captured graph (<0: no capture, the default; 0: whole cycles)")
    ap.add_argument("--coo", action="store_true", help="load a dense workload as coordinates")
    ap.add_argument("--balanced", action="store_true",
                    help="row and column pieces balancing training entries (psgld_balanced_pieces)")
    ap.add_argument("--part-order", choices=["cyclic", "random"], default="cyclic",
                    help="cyclic parts, or parts drawn with probability |part| / N")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve_c5":
        serve_main(args)
        return

    import paper_1506_01418_amd as pkg

    t_gen = time.perf_counter()
    wl = make_workload(args.workload)
    print(f"[bench] workload {wl.name}: I={wl.I} J={wl.J} nnz={wl.nnz} K={wl.K} B={wl.B} "
          f"({time.perf_counter() - t_gen:.1f} s to generate)", file=sys.stderr, flush=True)

    ev = HipEvents()
    dense = wl.dense is not None and not args.coo
    prec = {"f32": pkg.PSGLD_FP32, "bf16": pkg.PSGLD_BF16_DENSE, "bf16v": pkg.PSGLD_BF16_DENSE_VALUES}[args.precision]
    t_load = time.perf_counter()
    pieces = {}
    if args.balanced and not dense:
        rp, cp = pkg.balanced_pieces_for(wl.row, wl.col, wl.I, wl.J, wl.B)
        pieces = {"row_piece": rp, "col_piece": cp}
    s = pkg.PSGLD.from_workload(wl, dense=dense, precision=prec, graph_iters=args.graph_iters,
                                persistent=args.persistent, part_order=args.part_order, **pieces)
    print(f"[bench] loaded in {time.perf_counter() - t_load:.1f} s", file=sys.stderr, flush=True)
    stream = s.stream()
    n_p, N = s.part_sizes()
    if dense:
        placed, cnt, rows, cols = block_placement(wl)
        cells_p, entries_p = part_work(wl, placed, cnt, rows, cols)
        # the blocks' entries per part agree with the library's part sizes
        assert np.array_equal([sum(int(cnt[b, (b + p) % wl.B]) for b in range(wl.B)) for p in range(wl.B)], n_p)
    else:
        placed = np.zeros((wl.B, wl.B), dtype=bool)
        cells_p, entries_p = np.zeros(wl.B, dtype=np.int64), np.asarray(n_p, dtype=np.int64)
    runs_dense, runs_sparse = bool(placed.any()), not bool(placed.all())
    chosen, sched_info = None, (None, None, None)
    if runs_sparse:
        t_tune = time.perf_counter()
        if args.entries_per_group > 0 and args.quads_per_lane > 0:
            # a fixed schedule (profiling runs: the tuner's timings are perturbed there)
            s.set_schedule(args.entries_per_group, args.quads_per_lane)
            chosen, how = args.entries_per_group, "fixed"
        else:
            cands = (args.entries_per_group,) if args.entries_per_group > 0 else (16, 32, 64, 128)
            chosen, how = s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=cands, iters=wl.B), "tuned"
        sched_info = s.schedule_info()
        print(f"[bench] {how} schedule: {chosen} entries per group, {sched_info[1]} quads per lane, "
              f"{sched_info[2]} lanes per group ({time.perf_counter() - t_tune:.1f} s)", file=sys.stderr, flush=True)
    rpc = pieces.get("row_piece", pkg_pieces(wl, "row"))
    cpc = pieces.get("col_piece", pkg_pieces(wl, "col"))
    ho_part = (np.asarray(cpc)[wl.hcol] - np.asarray(rpc)[wl.hrow]) % wl.B
    ho_p = np.bincount(ho_part, minlength=wl.B)
    state0 = s.get_state()

    # warmup, then roll the chain back to t = 0
    s.step(args.warmup, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    s.sync()
    s.set_state(state0)
    ev.sync()

    # pass 1: whole-job throughput, one call of K iterations
    e0, e1 = ev.create(2)
    ev.record(e0, stream)
    s.step(args.steps, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    ev.record(e1, stream)
    elapsed_ms = ev.elapsed_ms(e0, e1)
    s.sync()
    ev.sync()
    parts = [s.part_at(t) for t in range(args.steps)]
    entries = int(sum(n_p[p] for p in parts))
    value = entries / (elapsed_ms * 1e-3)
    rmse = s.heldout_rmse() if args.steps > wl.burn_in and len(wl.hrow) else None
    print(f"[bench] pass 1: {args.steps} iterations in {elapsed_ms:.3f} ms, "
          f"{value:.4g} updates/s, held-out RMSE {rmse}", file=sys.stderr, flush=True)

    # pass 2: the same iterations again, HIP events around every launch
    s.set_state(state0)
    ev.sync()
    evs = ev.create(2 * args.steps)
    for t in range(args.steps):
        ev.record(evs[2 * t], stream)
        s.step(1, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        ev.record(evs[2 * t + 1], stream)
    durs = np.array([ev.elapsed_ms(evs[2 * t], evs[2 * t + 1]) for t in range(args.steps)])
    s.sync()
    rmse2 = s.heldout_rmse() if args.steps > wl.burn_in and len(wl.hrow) else None
    loglik = s.log_likelihood()
    # the kernel's average launch duration: the timed region's HIP events over
    # its iterations (back-to-back launches, so within a few tenths of a
    # microsecond of the traced kernel time); events around every launch add
    # their own gaps and are kept for the split at burn-in
    avg_ms = elapsed_ms / args.steps
    pre = durs[: min(args.steps, wl.burn_in)]
    post = durs[min(args.steps, wl.burn_in):]
    print(f"[bench] launch average before burn-in {pre.mean() * 1e3:.2f} us"
          + (f", after {post.mean() * 1e3:.2f} us" if len(post) else ""), file=sys.stderr, flush=True)
    vb = VALUE_BYTES[args.precision] if dense else 4
    bf = np.array([algorithmic_cost(wl, cells_p, entries_p, ho_p, t, parts[t], vb) for t in range(args.steps)],
                  dtype=np.float64)
    alg, flops = bf[:, 0], bf[:, 1]
    t_hbm = alg.mean() / (HBM_PEAK_GBS * 1e9)
    t_mfma = flops.mean() / (MFMA_PEAK_TFLOPS[args.precision] * 1e12)
    if t_mfma > t_hbm:
        achieved = float(flops.mean()) / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_PEAK_TFLOPS[args.precision],
                "unit": "TFLOP/s", "frac": achieved / MFMA_PEAK_TFLOPS[args.precision]}
    else:
        achieved = float(alg.mean()) / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS}
    if runs_dense and not runs_sparse:
        kernel, traffic = ("dense iteration (dense_tile_kernel + dense_w_update_kernel)",
                           measured_traffic(f"{wl.name}:{args.precision}", "dense"))
    elif runs_dense:
        kernel, traffic = "dense iteration and sparse_iter_kernel", None
    else:
        kernel, traffic = "sparse_iter_kernel", measured_traffic(wl.name, "sparse")
    roof.update({"traffic": traffic, "kernel": kernel, "avg_launch_us": avg_ms * 1e3,
                 "event_bracketed_launch_us": float(durs.mean()) * 1e3,
                 "alg_bytes_per_launch": float(alg.mean())})
    if runs_dense:
        roof["flops_per_launch"] = float(flops.mean())
        # beside the HBM fraction: how busy the products keep the matrix cores
        roof["mfma_frac"] = float(flops.mean()) / (avg_ms * 1e-3) / (MFMA_PEAK_TFLOPS[args.precision] * 1e12)
        roof["hbm_frac"] = float(alg.mean()) / (avg_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
    print(f"[bench] pass 2: iteration avg {float(durs.mean()) * 1e3:.2f} us with events around each launch; "
          f"timed region {avg_ms * 1e3:.2f} us per iteration, roofline {roof['achieved']:.1f} "
          f"{roof['unit']} ({roof['bound']}), RMSE {rmse2}", file=sys.stderr, flush=True)

    # pass 3: the whole chain (T iterations from t = 0, moments and held-out
    # sums after burn-in), whose held-out RMSE is compared with the oracle's
    chain = None
    if not args.no_full_chain and len(wl.hrow) and wl.T > wl.burn_in:
        s.set_state(state0)
        ev.sync()
        e2, e3 = ev.create(2)
        ev.record(e2, stream)
        s.step(wl.T, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        ev.record(e3, stream)
        chain_ms = ev.elapsed_ms(e2, e3)
        s.sync()
        chain_rmse = s.heldout_rmse()
        chain_entries = int(sum(n_p[s.part_at(t)] for t in range(wl.T)))
        ref = stored_oracle_rmse(wl)
        chain = {"T": wl.T, "burn_in": wl.burn_in, "thin": wl.thin, "ms": chain_ms,
                 "updates_per_s": chain_entries / (chain_ms * 1e-3), "heldout_rmse": chain_rmse,
                 "oracle_heldout_rmse": ref,
                 "rmse_rel_diff": None if ref is None else abs(chain_rmse - ref) / ref}
        print(f"[bench] pass 3: whole chain of {wl.T} iterations in {chain_ms:.2f} ms "
              f"({chain['updates_per_s']:.4g} updates/s), held-out RMSE {chain_rmse:.6f}"
              f" (oracle {ref})", file=sys.stderr, flush=True)
    # pass 4: the mixing indicator of the paper's synthetic experiments, the
    # log-likelihood of the chain's state against time (Section 4.2.1)
    trace = None
    if args.trace_every > 0:
        s.set_state(state0)
        ev.sync()
        points, sampler_ms, t = [[0, 0.0, s.log_likelihood()]], 0.0, 0
        while t < wl.T:
            n = min(args.trace_every, wl.T - t)
            ea, eb = ev.create(2)
            ev.record(ea, stream)
            s.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
            ev.record(eb, stream)
            sampler_ms += ev.elapsed_ms(ea, eb)
            t += n
            points.append([t, sampler_ms, s.log_likelihood()])
        ref = stored_oracle_trace(wl, args.trace_every)
        half = [p[2] for p in points if p[0] > wl.T // 2]
        trace = {"every": args.trace_every, "T": wl.T, "sampler_ms": sampler_ms, "points": points,
                 "loglik_mean_second_half": float(np.mean(half)) if half else None,
                 "oracle_loglik_mean_second_half": ref}
        print(f"[bench] pass 4: trace of {len(points)} log-likelihoods over {wl.T} iterations "
              f"({sampler_ms:.1f} ms of sampling), second-half mean {trace['loglik_mean_second_half']:.6g} "
              f"(oracle {ref})", file=sys.stderr, flush=True)
    s.close()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds, args.part_order, pieces.get("row_piece"), pieces.get("col_piece"),
                           iters=args.cpu_iters, single_iters=args.cpu_single_iters)
        print(f"[bench] oracle: {cpu['value']:.4g} updates/s on {cpu['cores']} threads, "
              f"{cpu['single_thread_value']:.4g} on one", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed_ms / args.steps,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": value / PAPER_UPDATES_PER_S[wl.name] if wl.name in PAPER_UPDATES_PER_S else None,
        "dtype": "bf16+f32" if runs_dense and args.precision in ("bf16", "bf16v") else "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "I": wl.I, "J": wl.J, "nnz_train": wl.nnz,
                   "nnz_heldout": int(len(wl.hrow)), "K": wl.K, "B": wl.B, "beta": wl.beta,
                   "timed_iterations": args.steps, "T": wl.T, "burn_in": wl.burn_in, "thin": wl.thin,
                   "heldout_rmse": chain["heldout_rmse"] if chain else rmse,
                   "oracle_heldout_rmse": chain["oracle_heldout_rmse"] if chain else None,
                   "whole_chain": chain, "train_loglik_end": loglik, "entries_per_group": chosen,
                   "quads_per_lane": sched_info[1], "lanes_per_group": sched_info[2], "dense": runs_dense,
                   "dense_blocks": int(placed.sum()),
                   "precision": args.precision if runs_dense else "f32", "parallelism": "single-gpu",
                   "part_order": args.part_order, "balanced_pieces": bool(pieces),
                   "launch": "persistent" if args.persistent and not runs_dense else
                             ("graph" if args.graph_iters >= 0 else "per-iteration")},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if trace:
        out["mixing_trace"] = trace
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        import torch
        # the fill kernel of torch.ones only writes; the reference is the neg
        # dispatch after it, so the two must not be averaged together
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)      # an elementwise kernel: 256 MiB read, 256 MiB written
        torch.cuda.synchronize()
        print("[bench] calibration copy (the neg kernel, after a fill): 268435456 bytes read and written",
              file=sys.stderr, flush=True)


def pkg_pieces(wl, which):
    n = wl.I if which == "row" else wl.J
    return np.concatenate([np.full(len(a), b) for b, a in enumerate(np.array_split(np.arange(n), wl.B))])


if __name__ == "__main__":
    main()
