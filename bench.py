#!/usr/bin/env python3
"""Benchmark of the FP64 ILU(0)-preconditioned BiCGSTAB hot path on one MI355X.

Workload (default): the large single-instance grid, X = Y = 1, eps = 0.01,
4096 x 4096 interior unknowns, upwind and centered schemes, manufactured
forcing, zero initial guess, relative residual 1e-10.  With Neumann data on
x = X and y = Y (the boundary mix the workload names) ILU(0)-BiCGSTAB does not
converge at eps = 0.01 -- the Neumann-closed operator is exponentially
ill-conditioned -- so time-to-tolerance is measured with Dirichlet data on all
four sides (labelled "dirichlet substitute" in the config), and the Neumann
variant is run for a fixed window of passes to report its status and
bandwidth.

One step = the whole hot path for both schemes: assemble, ilu0 and the solve
to tolerance, upwind then centered.  `value` is the mean time to relative
residual 1e-10 per solve (device time from r0 to the stop, inputs resident in
HBM).  The per-kernel roofline numbers are timed with HIP events on the
library's stream; the CPU baseline runs the oracle on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--n 4096] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
RING_NAMES = {0: "deep", 1: "compact"}   # adr_sweep_ring


def kernel_bytes(precision="fp64", tables=True):
    """Bytes per unknown of each kernel with perfect reuse of neighbours.
    tables=False: the algorithmic bytes of the five-diagonal method (L sweep
    q, lw, ls in, y out: 32; U sweep y, E, N, invd in, z out: 40; stencil
    product with its dot 64; a pass 392 in FP64) -- the figures the roofline
    is priced on.  tables=True: what the kernels actually read, S, W, E, N
    coming from per-column / per-row tables of a few KB (24, 24, 32; a pass
    280)."""
    f = 4 if precision == "fp32_factors" else 8          # bytes of a stored factor
    if tables:
        ls = 8 + 8 + 8 if precision == "fp64" else 8 + 2 * f + 8   # q, invd (FP64) | q, lw, ls; y out
        us = 8 + f + 8                                              # y, invd in; z out
        sp = 8 + 8 + 8 + 8                                          # x, C, r^ in; v out
    else:
        ls = 8 + 2 * f + 8                                          # q, lw, ls in; y out
        us = 8 + 3 * f + 8                                          # y, E, N, invd in; z out
        sp = 8 + 40 + 8 + 8                                         # x, S, W, C, E, N, r^ in; v out
    # pass: p update 32, two L and two U sweeps, two stencil products with a
    # dot, s update 24, x / r update 64
    return {"lsweep": ls, "usweep": us, "spmv_dot": sp, "iteration": 32 + 2 * (ls + us) + 2 * sp + 24 + 64,
            "spmv": 56}   # the stand-alone stencil product reads the five diagonals


BYTES = kernel_bytes("fp64", tables=True)
BYTES_DIA = kernel_bytes("fp64", tables=False)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxit", type=int, default=20000)
    ap.add_argument("--variant-maxit", type=int, default=14000, help="pass limit of the mixed-precision variants")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--rows", type=int, default=0, help="sweep strip height (0 = automatic)")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--neumann-window", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--no-variants", dest="variants", action="store_false")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--workload", choices=("single", "batch", "warmstart", "network", "kernels", "large", "traffic"),
                    default="single")
    ap.add_argument("--pmc-fetch", default="", help="traffic: rocprofv3 output folder of the FETCH_SIZE pass")
    ap.add_argument("--pmc-write", default="", help="traffic: rocprofv3 output folder of the WRITE_SIZE pass")
    ap.add_argument("--instances-out", default="", help="batch: write the per-instance outcomes to this JSON file")
    ap.add_argument("--pmc-net-fetch", default="", help="traffic: FETCH_SIZE folder of --workload network")
    ap.add_argument("--pmc-net-write", default="", help="traffic: WRITE_SIZE folder of --workload network")
    ap.add_argument("--large-maxit", type=int, default=10000, help="large: pass limit of the Dirichlet solves")
    ap.add_argument("--heldout", type=int, default=1000, help="warmstart: held-out instances")
    ap.add_argument("--single-sample", type=int, default=128,
                    help="warmstart: instances also timed one at a time")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-precision", default="fp32_factors")
    ap.add_argument("--batch-maxit", type=int, default=2000)
    ap.add_argument("--sequential-sample", type=int, default=0,
                    help="solve only this many instances one at a time for the comparison (0 = all)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_us(prob, fns, reps):
    """Mean device time (us) per call of each of `fns`, called in turn `reps`
    times (L sweep then U sweep, as in the solve, so the U sweep reads the
    vector the L sweep has just written): the library records HIP events on
    the problem's stream around the launches of each single-step call (a
    whole-loop event pair would also count the host's turnaround between
    these synchronous calls)."""
    for fn in fns.values():
        fn()
    total = dict.fromkeys(fns, 0.0)
    for _ in range(reps):
        for name, fn in fns.items():
            fn()
            total[name] += prob.last_call_ms
    return {name: t * 1e3 / reps for name, t in total.items()}


def code_text(path):
    """A C/C++ source without its comments and with its white space collapsed:
    what the compiler reads of it, so that editing a comment leaves counters
    taken on the same code valid."""
    with open(path, encoding="utf-8") as fh:
        s = fh.read()
    out, i, n = [], 0, len(s)
    while i < n:
        c = s[i]
        if c in "\"'":                     # string or character literal, kept whole
            j = i + 1
            while j < n and s[j] != c:
                j += 2 if s[j] == "\\" else 1
            out.append(s[i:j + 1])
            i = j + 1
        elif s.startswith("//", i):
            j = s.find("\n", i)
            i = n if j < 0 else j
        elif s.startswith("/*", i):
            j = s.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def sweep_source_hash():
    h = hashlib.sha256()
    for f in ("adr_sweeps.hip", "adr_kernels.hip", "adr_device.h", "adr_internal.h"):
        h.update(code_text(os.path.join(ROOT, "paper_1308_5215_amd", "csrc", f)).encode())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            t = json.load(fh)
        e = t.get(workload, {}).get(kernel)
        if not e or e.get("source_hash") != sweep_source_hash():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def host_cpu():
    """Model name of the host CPU that runs the oracle (Linux), else ""."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _oracle_pass_seconds(job):
    """Worker (own process): seconds per BiCGSTAB pass of the CPU oracle on one
    instance of the batch, over a fixed window of passes (tol 0)."""
    eps, X, Y, n, scheme, bc, field, passes, precision = job
    from oracle import core as orc
    P = orc.assemble(eps, X, Y, n, n, scheme, bc, field=field, amp=0.1)
    F = orc.ilu0(P)
    if precision == "fp32_factors":
        F = orc.round_factors_f32(F)
    t = time.perf_counter()
    r = orc.bicgstab(P, F, tol=0.0, maxit=passes)
    return (time.perf_counter() - t) / max(r.iters, 1), n * n


def run_batch(args):
    """Batched workload: many uneven instances (grid n x n, n in 128..1024 step
    32, eps log-uniform in [1e-3, 1], X, Y in [0.5, 2], scheme and boundary
    type with p = 1/2, forcing = manufactured + Gaussian random field of length
    0.1 and amplitude 0.1 max|f|), FP32 preconditioner with FP64 Krylov, one
    launch per step for the whole batch.  Compared with the same instances
    solved one at a time by the single-instance path."""
    import numpy as np
    import torch
    import paper_1308_5215_amd as adr
    from synthetic import fields

    torch.cuda.set_device(0)
    inst = fields.batch_instances(args.batch_count, seed=1308)
    t0 = time.perf_counter()
    flds = [fields.gaussian_random_field(d["n"], d["n"], d["X"] / (d["n"] + 1), d["Y"] / (d["n"] + 1),
                                         length=0.1, seed=1308, instance=k).ravel() for k, d in enumerate(inst)]
    log("fields: %.1f s" % (time.perf_counter() - t0))
    flat = torch.from_numpy(np.concatenate(flds)).cuda()
    cols = dict(eps=[d["eps"] for d in inst], X=[d["X"] for d in inst], Y=[d["Y"] for d in inst],
                nx=[d["n"] for d in inst], ny=[d["n"] for d in inst], scheme=[d["scheme"] for d in inst],
                bc=[d["bc"] for d in inst])
    N = [d["n"] * d["n"] for d in inst]

    def batch_once():
        b = adr.assemble_batch(cols["eps"], cols["X"], cols["Y"], cols["nx"], cols["ny"], cols["scheme"],
                               cols["bc"], field=flat, amp=0.1)
        b.ilu0(args.batch_precision)
        rows, ms = b.autotune()
        ring = b.sweep_ring
        res = b.solve(tol=args.tol, maxit=args.batch_maxit)
        return b, (rows, ring), ms, res

    log("batch warmup")
    for _ in range(args.warmup):
        batch_once()
    torch.cuda.synchronize()
    log("batch timed: %d step(s)" % args.steps)
    times, t0 = [], time.perf_counter()
    for _ in range(args.steps):
        b, rows, ms_apply, res = batch_once()
        times.append(res.solve_ms)
        log("  batch solve %.1f ms, rows %d, %s ring (autotuned, %.2f ms per M^-1)" %
            (res.solve_ms, rows[0], RING_NAMES.get(rows[1], str(rows[1])), ms_apply))
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    st = np.asarray(res.status)
    its = np.asarray(res.iters)
    counts = {int(k): int((st == k).sum()) for k in np.unique(st)}
    # the instance classifier's expectation against the outcome
    expect = np.array([adr.classify(d["eps"], d["X"], d["Y"], d["n"], d["n"], d["scheme"], d["bc"], args.tol).expect_fail
                       for d in inst])
    failed = st != adr.OK
    confusion = {"expected_fail_failed": int((expect & failed).sum()),
                 "expected_fail_converged": int((expect & ~failed).sum()),
                 "expected_ok_failed": int((~expect & failed).sum()),
                 "expected_ok_converged": int((~expect & ~failed).sum())}
    log("  classifier vs outcome: %s" % confusion)
    per_instance = [dict(k=k, n=d["n"], eps=round(d["eps"], 6), X=round(d["X"], 4), Y=round(d["Y"], 4),
                         scheme=d["scheme"], bc=d["bc"], status=int(st[k]), iters=int(its[k]),
                         restarts=int(res.restarts[k]), expect_fail=bool(expect[k]))
                    for k, d in enumerate(inst)]
    tr_ok = np.asarray(res.true_relres)[~failed]
    work = float(sum(N[k] * its[k] for k in range(len(inst))))
    batch_s = float(np.mean(times)) / 1e3
    xb = [v.clone() for v in b.split(res.x)]
    del b

    # the same instances one at a time
    sample = range(len(inst)) if args.sequential_sample <= 0 else \
        np.linspace(0, len(inst) - 1, args.sequential_sample).round().astype(int)
    seq_ms, seq_work, maxdiff = 0.0, 0.0, 0.0
    log("sequential: %d instance(s)" % len(sample))
    for k in sample:
        d = inst[k]
        prob = adr.assemble(d["eps"], d["X"], d["Y"], d["n"], d["n"], d["scheme"], d["bc"],
                            field=flat[sum(N[:k]):sum(N[:k + 1])], amp=0.1)
        prob.ilu0(args.batch_precision)
        r1 = prob.solve(tol=args.tol, maxit=args.batch_maxit)
        seq_ms += r1.solve_ms
        seq_work += N[k] * r1.iters
        if r1.status == 0 and st[k] == 0:
            maxdiff = max(maxdiff, float((r1.x - xb[k]).abs().max() / xb[k].abs().max().clamp_min(1e-300)))
        del prob, r1
    scale = len(inst) / len(sample)
    seq_s = seq_ms * scale / 1e3

    # the CPU oracle, one instance per core: seconds per unknown-pass from a
    # fixed window of passes on a sample of the instances, applied to the
    # batch's own unknown-passes
    cpu = None
    if args.cpu_baseline:
        import multiprocessing as mp
        cores = max(1, min(16, os.cpu_count() or 1))
        pick = np.linspace(0, len(inst) - 1, 16).round().astype(int)
        jobs = [(inst[k]["eps"], inst[k]["X"], inst[k]["Y"], inst[k]["n"], inst[k]["scheme"], inst[k]["bc"],
                 flds[k], 10, args.batch_precision) for k in pick]
        log("cpu baseline (oracle): %d instances x 10 passes on %d processes" % (len(jobs), cores))
        with mp.get_context("spawn").Pool(cores) as pool:
            got = pool.map(_oracle_pass_seconds, jobs)
        rate = sum(t for t, _ in got) / sum(m for _, m in got)     # s per unknown-pass, one core
        single = rate * work
        cpu = dict(value=round(single / cores, 2), unit="s", cores=cores, kind="oracle",
                   single_core_s=round(single, 1), host=host_cpu(),
                   sample="10 BiCGSTAB passes of the FP64 oracle (%s factors) on each of %d instances spread "
                          "over the batch, one process per core: %.1f ns per unknown-pass on one core, applied to "
                          "the batch's %.3g unknown-passes and divided over %d cores (load balance assumed)"
                          % ("FP32-rounded" if args.batch_precision == "fp32_factors" else "FP64",
                             len(jobs), rate * 1e9, work, cores))
        log("  %.1f ns per unknown-pass -> %.0f s on one core, %.0f s on %d" % (rate * 1e9, single, single / cores,
                                                                              cores))
    out = {
        "metric": "time to rel-resid 1e-10, batched instances (FP32 preconditioner, FP64 Krylov)",
        "value": round(batch_s, 4), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%d instances, n in 128..1024 step 32, eps log-uniform [1e-3,1], X,Y in [0.5,2], "
                               "random scheme/bc, manufactured f + GRF (length 0.1, amp 0.1 max|f|)" % len(inst),
                   "precision": args.batch_precision, "tol": args.tol, "maxit": args.batch_maxit,
                   "total_unknowns": int(sum(N)), "seed": 1308},
        "statuses": counts,
        "classifier_vs_outcome": confusion,
        "restarts_total": int(np.sum(res.restarts)),
        "true_relres_max_of_ok": float(tr_ok.max()) if tr_ok.size else None,
        "unknown_passes_per_s": round(work / batch_s, 1),
        "hbm_gbs_algorithmic": round(kernel_bytes(args.batch_precision)["iteration"] * work / batch_s / 1e9, 1),
        "sequential": {"solve_s": round(seq_s, 3), "instances_timed": len(sample),
                       "extrapolated": len(sample) != len(inst),
                       "speedup_batched": round(seq_s / batch_s, 2) if batch_s > 0 else None,
                       "max_rel_diff_vs_batched": maxdiff},
        "sweep_rows": rows[0],
        "sweep_ring": RING_NAMES.get(rows[1], str(rows[1])),
        "cpu_baseline": cpu,
    }
    if args.instances_out:
        with open(args.instances_out, "w") as fh:
            json.dump(per_instance, fh)
    print(json.dumps(out), flush=True)


def network_roofline(weights, reps=10):
    """Forward pass and one training step of the warm-start network on a batch
    of 64 instances at 258 x 258 nodes (random inputs in the ten field
    channels), timed with events on the current stream."""
    import torch
    import paper_1308_5215_amd as adr

    n = 256
    net = adr.WarmStartNet(n + 2, n + 2, 64)
    net.set_params(weights)
    # network throughput: inference and one training step of a batch of 64
    # instances.  Algorithmic work of the six 3x3 layers (10 -> 32 -> ... ->
    # 32 -> 1 channels; the zero channels the kernels pad to are not counted):
    # 2 * 9 * sum(cin * cout) flop per node, and per node the bytes a
    # layer-by-layer forward pass must move: each layer reads its input
    # (10 channels, then 32, bfloat16) and writes its output (32 bfloat16
    # channels, the last one FP32 u).  At 120 flop/B the pass sits below the
    # bf16 ridge (2.5 PFLOP/s / 8 TB/s = 312 flop/B): it is HBM-bound.
    H = n + 2
    B = 64
    xin = torch.zeros((B, H, H, 32), dtype=torch.bfloat16, device="cuda")
    xin[..., :10] = torch.randn((B, H, H, 10), device="cuda").to(torch.bfloat16)
    u = torch.empty((B, H, H), dtype=torch.float32, device="cuda")
    tgt = torch.zeros((B, n, n), dtype=torch.float32, device="cuda")
    cio = [(10, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]
    fwd_flop = 2.0 * B * H * H * 9 * sum(ci * co for ci, co in cio)
    fwd_bytes = float(B * H * H * (10 * 2 + 5 * 32 * 2 + 5 * 32 * 2 + 4))
    stream = torch.cuda.current_stream()
    net.forward(xin, out=u)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        net.forward(xin, out=u)
    e1.record(stream)
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    # training: forward + input gradients of layers 2..6 + weight gradients of all six
    step_flop = 2 * fwd_flop + 2.0 * B * H * H * 9 * sum(ci * co for ci, co in cio[1:])
    net2 = adr.WarmStartNet(H, H, B)
    net2.set_params(weights)
    net2.train_step(xin, tgt, lr=0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        net2.train_step(xin, tgt, lr=0.0)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t1) * 1e3 / 5
    fwd_tflops = fwd_flop / (fwd_ms * 1e-3) / 1e12
    traffic = None
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            e = json.load(fh).get("network_258_b64")
        if e and e.get("source_hash") == network_source_hash():
            traffic = float(e["bytes_per_forward"])
    except (OSError, ValueError):
        pass
    return dict(bound="hbm", kernel="k_conv (6-layer forward, batch 64, 258x258)",
                achieved=round(fwd_bytes / (fwd_ms * 1e-3) / 1e9, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(fwd_bytes / (fwd_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4), traffic=traffic,
                algorithmic_bytes=fwd_bytes, algorithmic_flop=fwd_flop,
                flop_per_byte=round(fwd_flop / fwd_bytes, 1),
                tflops=round(fwd_tflops, 1), frac_of_bf16_peak=round(fwd_tflops / 2500.0, 4),
                forward_ms=round(fwd_ms, 3), train_step_ms=round(step_ms, 3),
                train_step_tflops=round(step_flop / (step_ms * 1e-3) / 1e12, 1))


def run_network(args):
    """The warm-start network alone: forward pass and training step of a batch
    of 64 instances at 258 x 258 with the committed weights (the per-layer
    profile of the network is taken on this workload)."""
    import numpy as np
    import torch
    from paper_1308_5215_amd import train_warmstart as tw

    torch.cuda.set_device(0)
    r = network_roofline(np.load(tw.DEFAULT_WEIGHTS, allow_pickle=False), reps=args.steps * 10)
    out = {"metric": "warm-start network forward pass, batch 64 at 258x258", "value": r["forward_ms"] / 1e3,
           "unit": "s", "n_gpus": 1, "steps": args.steps * 10, "warmup": 1, "ms_per_step": r["forward_ms"],
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": "6 x conv3x3, 10->32->...->32->1, GELU, bf16 activations and weights, fp32 "
                                  "accumulate; batch 64, 258 x 258 nodes"},
           "roofline": r}
    log("  network: forward %.3f ms (%.0f GB/s, %.0f TFLOP/s), training step %.2f ms" %
        (r["forward_ms"], r["achieved"], r["tflops"], r["train_step_ms"]))
    print(json.dumps(out), flush=True)


def run_warmstart(args):
    """Learned initial guess: held-out 256 x 256 instances (seeds 100000...,
    eps log-uniform in [1e-3, 1], X, Y in [0.5, 2], Dirichlet or Neumann outer
    sides, upwind or centered convection, manufactured f + Gaussian random
    field) solved to relative residual
    1e-10 from the zero guess and from the trained network's guess (committed
    weights; the guess time counts against it).  FP64 throughout."""
    import numpy as np
    import torch
    from multiprocessing import Pool
    import paper_1308_5215_amd as adr
    from paper_1308_5215_amd import train_warmstart as tw

    torch.cuda.set_device(0)
    n = 256
    net = adr.WarmStartNet(n + 2, n + 2, 64)
    net.set_params(np.load(tw.DEFAULT_WEIGHTS, allow_pickle=False))
    seeds = list(range(tw.HELDOUT_SEED0, tw.HELDOUT_SEED0 + args.heldout))
    t0 = time.perf_counter()
    with Pool(16) as pool:
        ev = tw.evaluate(net, seeds, n, args.tol, 3000, pool=pool, log=log, single=args.single_sample)
    wall = time.perf_counter() - t0
    s = ev["summary"]
    k = max(s["single_instances"], 1)
    mfma = network_roofline(np.load(tw.DEFAULT_WEIGHTS, allow_pickle=False))
    log("  network: forward %.2f ms (%.0f GB/s, %.0f TFLOP/s), training step %.2f ms" %
        (mfma["forward_ms"], mfma["achieved"], mfma["tflops"], mfma["train_step_ms"]))
    out = {
        "metric": "time to rel-resid 1e-10 per instance from the learned guess (single-instance solves)",
        "value": round(s["single_warm_ms"] / k / 1e3, 5), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(wall * 1e3, 1), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "learned warm start, %d held-out instances 256x256 (seeds %d..), eps log-uniform "
                               "[1e-3,1], X,Y in [0.5,2], Dirichlet/Neumann p=1/2, upwind/centered p=1/2, "
                               "manufactured f + GRF (length 0.1, amp 0.1 max|f|)" % (len(seeds), seeds[0]),
                   "network": "6 x conv3x3, 10->32->...->32->1, GELU, bf16 weights, fp32 accumulate",
                   "well_posed": "instance classifier: expected to converge, Neumann g_y <= %g, wrong-sign "
                                 "couplings only with cell Peclet <= %g" % (tw.G_Y_MAX, tw.PE_MAX),
                   "weights": os.path.relpath(tw.DEFAULT_WEIGHTS, ROOT), "tol": args.tol},
        "zero_guess_s": round(s["single_zero_ms"] / k / 1e3, 5),
        "summary": s,
        "roofline": mfma,
    }
    print(json.dumps(out), flush=True)


def run_large(args):
    """Convection-dominated large grid: X = 2, Y = 1, eps = 1e-3, 8192 x 8192
    (67M unknowns), upwind and centered, FP32-stored ILU(0) factors with FP64
    BiCGSTAB, graph-replayed iteration.  With Dirichlet data on all sides the
    solve runs to relative residual 1e-10 (or the pass limit); the mixed
    boundary (Neumann on x = X and y = Y) is run for a fixed window of passes
    and reported by status and bandwidth.  Per-kernel algorithmic bandwidth is
    timed with HIP events for FP32 and FP64 factors."""
    import numpy as np
    import torch
    import paper_1308_5215_amd as adr

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = 8192 if args.n == 4096 else args.n
    N = n * n
    X, Y, eps = 2.0, 1.0, 1e-3
    solves, windows = {}, {}
    bytes_pass = {p: kernel_bytes(p)["iteration"] for p in ("fp32_factors", "fp64")}
    for sc in ("upwind", "centered"):
        prob = adr.assemble(eps, X, Y, n, n, sc, "dirichlet")
        try:
            prob.ilu0("fp32_factors")
        except adr.AdrError as e:   # a zero or non-finite pivot: no preconditioner for this case
            solves[sc] = dict(status=int(e.status), error=str(e))
            log("  dirichlet %s: %s" % (sc, e))
            del prob
            continue
        res = prob.solve(tol=args.tol, maxit=args.large_maxit)
        ms_it = res.solve_ms / max(res.iters, 1)
        c = adr.classify(eps, X, Y, n, n, sc, "dirichlet")
        solves[sc] = dict(status=int(res.status), iters=int(res.iters), restarts=int(res.restarts),
                          solve_s=round(res.solve_ms / 1e3, 3),
                          ms_per_iter=round(ms_it, 3), true_relres=res.true_relres,
                          max_error=prob.max_error(res.x),
                          last_relres=float(res.hist_l2[-1] / res.bnorm) if res.bnorm > 0 else None,
                          algorithmic_gbs=round(bytes_pass["fp32_factors"] * N / (ms_it * 1e-3) / 1e9, 1),
                          pe_x=round(c.pe_x, 3), neg_offdiag=int(c.neg_offdiag), expected_to_fail=c.expect_fail)
        log("  dirichlet %s: status %d passes %d restarts %d %.2f s (%.2f ms/pass) true relres %.2e max error %.3e" %
            (sc, res.status, res.iters, res.restarts, res.solve_ms / 1e3, ms_it, res.true_relres,
             solves[sc]["max_error"]))
        del prob, res
        prob = adr.assemble(eps, X, Y, n, n, sc, "neumann")
        try:
            prob.ilu0("fp32_factors")
        except adr.AdrError as e:
            windows[sc] = dict(status=int(e.status), error=str(e))
            log("  neumann %s: %s" % (sc, e))
            del prob
            continue
        res = prob.solve(tol=args.tol, maxit=args.neumann_window)
        ms_it = res.solve_ms / max(res.iters, 1)
        windows[sc] = dict(status=int(res.status), iters=int(res.iters), solve_ms=round(res.solve_ms, 2),
                           restarts=int(res.restarts), true_relres=res.true_relres,
                           algorithmic_gbs=round(bytes_pass["fp32_factors"] * N / (ms_it * 1e-3) / 1e9, 1),
                           last_relres=float(res.hist_l2[-1] / res.bnorm) if res.bnorm > 0 else None)
        log("  neumann %s: status %d after %d passes" % (sc, res.status, res.iters))
        del prob, res
    # per-kernel bandwidth
    kernels = {}
    q = torch.randn(N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(q)
    z = torch.empty_like(q)
    for prec, kb in (("fp32_factors", kernel_bytes("fp32_factors")), ("fp64", kernel_bytes("fp64"))):
        prob = adr.assemble(eps, X, Y, n, n, "centered", "dirichlet")
        prob.ilu0(prec)
        kernels[prec] = {}
        times = kernel_us(prob, {"lsweep": lambda: prob.lsolve(q, out=y), "usweep": lambda: prob.usolve(y, out=z),
                                 "spmv": lambda: prob.spmv(q, out=z)}, args.kernel_reps)
        for name, us in times.items():
            gbs = kb[name] * N / (us * 1e-6) / 1e9
            kernels[prec][name] = dict(avg_us=round(us, 1), bytes_per_unknown=kb[name], gbs=round(gbs, 1),
                                       frac=round(gbs / PEAK_HBM_GBS, 4))
            log("  %s %s: %.1f us %.0f GB/s" % (prec, name, us, gbs))
        del prob
    conv = [v["solve_s"] for v in solves.values() if v["status"] == 0]
    out = {
        "metric": "time to rel-resid 1e-10 & HBM GB/s, convection-dominated 8192^2 (FP32 factors, FP64 Krylov)",
        "value": round(float(np.mean(conv)), 4) if conv else None, "unit": "s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "advection-diffusion %dx%d, X=2, Y=1, eps=1e-3, upwind+centered, FP32 ILU(0) "
                               "factors + FP64 BiCGSTAB; Dirichlet on all sides for time-to-tolerance, Neumann on "
                               "x=X,y=Y for a %d-pass window" % (n, n, args.neumann_window),
                   "tol": args.tol, "maxit": args.large_maxit},
        "dirichlet": solves, "mixed_bc_window": windows, "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


# Algorithmic bytes per unknown of every kernel of a pass (FP64; the five-
# diagonal figures, and what the kernels read with the stencil tables).
PASS_KERNELS = {
    # name: (bytes with the diagonals, bytes with the tables, what moves)
    "lsweep": (32, 24, "q, lw, ls in, y out (tables: q, invd in, y out)"),
    "usweep": (40, 24, "y, E, N, invd in, z out (tables: y, invd in, z out)"),
    "pass_p": (32, 32, "p, r, v in, p out"),
    "pass_v": (64, 32, "p^, S, W, C, E, N, r^ in, v out (tables: p^, C, r^ in, v out)"),
    "pass_s": (24, 24, "r, v in, s out"),
    "pass_t": (64, 32, "z, S, W, C, E, N, s in, t out (tables: z, C, s in, t out)"),
    "pass_xr": (64, 64, "x, p^, z, t, s, r^ in, x, r out"),
    "spmv": (56, 56, "x, S, W, C, E, N in, v out (stand-alone, diagonals)"),
}


def kernel_key(name):
    """Short name of a library kernel from its demangled name, else None."""
    import re
    m = re.search(r"k_sweep_ws<\s*\d+,\s*(\d)", name)
    if m:
        return "lsweep" if m.group(1) == "0" else "usweep"
    for key, pat in (("pass_xr", "k_pass_xr("), ("pass_p", "k_pass_p("), ("pass_v", "k_pass_v<"),
                     ("pass_s", "k_pass_s("), ("pass_t", "k_pass_t<"), ("spmv", "k_spmv("),
                     ("copy", "k_stream_copy(")):
        if pat in name:
            return key
    return None


def run_kernels(args):
    """Each hot-path kernel under the counters: the two sweeps and the
    stand-alone stencil product `--kernel-reps` launches each on the n x n grid
    (centered scheme, FP64 factors), then `--kernel-reps` passes of a solve
    (the in-loop kernels), then the library's streaming copy of 1 GiB each way
    as the calibration for hardware counters.  For counter runs:
        rocprofv3 --pmc FETCH_SIZE -d DIR -o run --output-format csv -- python bench.py --workload kernels
    and then `python bench.py --workload traffic --pmc-fetch DIR --pmc-write DIR2`.
    """
    import torch
    import paper_1308_5215_amd as adr

    torch.cuda.set_device(0)
    n = args.n
    N = n * n
    prob = adr.assemble(args.eps, 1.0, 1.0, n, n, "centered", "dirichlet")
    if args.rows:
        prob.set_sweep_rows(args.rows)
    prob.ilu0(args.precision)
    q = torch.randn(N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(q)
    z = torch.empty_like(q)
    out = {}
    for name, fn in (("lsweep", lambda: prob.lsolve(q, out=y)), ("usweep", lambda: prob.usolve(y, out=z)),
                     ("spmv", lambda: prob.spmv(q, out=z))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.kernel_reps):
            fn()
        torch.cuda.synchronize()
        out[name] = round((time.perf_counter() - t0) * 1e6 / args.kernel_reps, 1)
        log("  %s: %.1f us per launch (host clock)" % (name, out[name]))
    # the in-loop kernels: passes of a solve that cannot stop early
    res = prob.solve(tol=1e-30, maxit=args.kernel_reps)
    log("  solve: %d passes, %.1f ms" % (res.iters, res.solve_ms))
    # the library's streaming copy, 1 GiB each way
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(args.kernel_reps):
        adr.stream_copy(a, b)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "kernels", "n": n, "reps": args.kernel_reps, "us_per_launch": out,
                      "solve_passes": res.iters, "copy_bytes_each_way": a.numel() * 8,
                      "sweep_rows": args.rows or "auto", "precision": args.precision}), flush=True)


def read_pmc(folder, counter):
    """Per-kernel counter values (one list entry per dispatch) from a
    rocprofv3 --pmc CSV output folder."""
    import csv
    import glob
    vals = {}
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no *counter_collection.csv under %s" % folder)
    per_dispatch = {}
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                key = kernel_key(row.get("Kernel_Name", ""))
                if key is None:
                    continue
                d = (f, row.get("Dispatch_Id"))
                per_dispatch.setdefault((key, d), 0.0)
                per_dispatch[(key, d)] += float(row["Counter_Value"])
    for (key, _), v in per_dispatch.items():
        vals.setdefault(key, []).append(v)
    return vals


def network_source_hash():
    h = hashlib.sha256()
    h.update(code_text(os.path.join(ROOT, "paper_1308_5215_amd", "csrc", "adr_cnn.hip")).encode())
    return h.hexdigest()[:16]


def read_forward_pmc(folder, counter):
    """Counter totals of each six-layer forward pass (five k_conv<32, 0>
    dispatches followed by one k_conv<16, 1>) in a rocprofv3 --pmc folder of
    `--workload network`."""
    import csv
    import glob
    disp = {}
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                name = row.get("Kernel_Name", "")
                kind = "h" if "k_conv<32, 0>" in name else ("o" if "k_conv<16, 1>" in name else "x")
                d = disp.setdefault((f, int(row["Dispatch_Id"])), [kind, 0.0])
                d[1] += float(row["Counter_Value"])
    seq = [disp[k] for k in sorted(disp)]
    return [sum(v for _, v in seq[i:i + 6]) for i in range(len(seq) - 5)
            if [k for k, _ in seq[i:i + 6]] == ["h"] * 5 + ["o"]]


def run_traffic(args):
    """HBM bytes per launch of every hot-path kernel from two rocprofv3
    counter passes of `--workload kernels` (FETCH_SIZE, then WRITE_SIZE, KiB
    per dispatch), each scaled by what the same counter reads for the
    library's streaming copy of 1 GiB each way; written to
    profiles/traffic.json with the hash of the kernel sources.  With
    --pmc-net-fetch / --pmc-net-write (the same two passes of `--workload
    network`), also the bytes of one forward pass of the warm-start network,
    scaled by the same factors."""
    import statistics
    fetch = read_pmc(args.pmc_fetch, "FETCH_SIZE")
    write = read_pmc(args.pmc_write, "WRITE_SIZE")

    def working(v):
        # a solve's graph chunk also launches passes after the stop, which
        # return at entry: keep the dispatches that did the kernel's work
        top = max(v)
        return [x for x in v if x >= 0.5 * top]

    fetch = {k: working(v) for k, v in fetch.items()}
    write = {k: working(v) for k, v in write.items()}
    gib = float(1 << 30)
    ff = gib / (statistics.median(fetch["copy"]) * 1024.0)
    wf = gib / (statistics.median(write["copy"]) * 1024.0)
    N = args.n * args.n
    h = sweep_source_hash()
    res = {}
    lines = []
    for key, (dia, tab, what) in PASS_KERNELS.items():
        if key not in fetch or key not in write:
            continue
        fb = statistics.median(fetch[key]) * 1024.0 * ff
        wb = statistics.median(write[key]) * 1024.0 * wf
        res[key] = dict(bytes_per_launch=round(fb + wb), fetch_bytes=round(fb), write_bytes=round(wb),
                        algorithmic_bytes=dia * N, algorithmic_bytes_tables=tab * N,
                        bytes_per_unknown=round((fb + wb) / N, 2), dispatches=len(fetch[key]), source_hash=h)
        lines.append("%-8s FETCH %10.1f KiB x %.3f  WRITE %10.1f KiB x %.3f -> %8.1f MB per launch = %5.1f B/unknown "
                     "(algorithmic %d, tables %d: %s)" % (key, statistics.median(fetch[key]), ff,
                                                         statistics.median(write[key]), wf, (fb + wb) / 1e6,
                                                         (fb + wb) / N, dia, tab, what))
    out = {"n%d" % args.n: res,
           "calibration": {"kernel": "adr::k_stream_copy", "bytes_each_way": int(gib),
                           "fetch_factor": ff, "write_factor": wf}}
    if args.pmc_net_fetch and args.pmc_net_write:
        nf = statistics.median(read_forward_pmc(args.pmc_net_fetch, "FETCH_SIZE")) * 1024.0 * ff
        nw = statistics.median(read_forward_pmc(args.pmc_net_write, "WRITE_SIZE")) * 1024.0 * wf
        nodes = 64 * 258 * 258
        out["network_258_b64"] = dict(bytes_per_forward=round(nf + nw), fetch_bytes=round(nf), write_bytes=round(nw),
                                      algorithmic_bytes=nodes * (10 * 2 + 5 * 32 * 2 + 5 * 32 * 2 + 4),
                                      bytes_per_node=round((nf + nw) / nodes, 2), source_hash=network_source_hash())
        lines.append("network  FETCH %.1f MB  WRITE %.1f MB per forward pass (64 x 258 x 258 nodes) = %.1f B per node "
                     "(algorithmic 664)" % (nf / 1e6, nw / 1e6, (nf + nw) / nodes))
    path = os.path.join(ROOT, "profiles", "traffic.json")
    old = {}
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
    old.update(out)
    with open(path, "w") as fh:
        json.dump(old, fh, indent=1)
    print("calibration: the streaming copy (1 GiB each way) reads FETCH_SIZE %.0f KiB and WRITE_SIZE %.0f KiB "
          "per dispatch: factors %.3f and %.3f" % (statistics.median(fetch["copy"]), statistics.median(write["copy"]),
                                                   ff, wf))
    print("\n".join(lines))


def copy_reference_gbs(dev, reps=5):
    """Bandwidth of the library's plain streaming copy kernel (1 GiB read and
    1 GiB written), timed with events on the current stream: the practical
    HBM ceiling beside the 8 TB/s peak."""
    import torch
    import paper_1308_5215_amd as adr
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    adr.stream_copy(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        adr.stream_copy(a, b)
    e1.record()
    e1.synchronize()
    gbs = 2 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def solve_record(prob, res, extra=None):
    """Status, passes, restarts, true relative residual and discretisation
    error (max |U - u_exact| over the grid, adr_max_error) of one solve."""
    d = dict(status=int(res.status), iters=int(res.iters), restarts=int(res.restarts),
             solve_s=round(res.solve_ms / 1e3, 4), true_relres=float(res.true_relres),
             max_error=prob.max_error(res.x))
    if extra:
        d.update(extra)
    return d


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "warmstart":
        return run_warmstart(args)
    if args.workload == "network":
        return run_network(args)
    if args.workload == "kernels":
        return run_kernels(args)
    if args.workload == "traffic":
        return run_traffic(args)
    if args.workload == "large":
        return run_large(args)
    import numpy as np
    import torch
    import paper_1308_5215_amd as adr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    N = n * n
    schemes = ("upwind", "centered")
    tables_used = []

    def hot_path(scheme, bc="dirichlet", maxit=args.maxit, precision=args.precision):
        prob = adr.assemble(args.eps, 1.0, 1.0, n, n, scheme, bc)
        if args.rows:
            prob.set_sweep_rows(args.rows)
        prob.ilu0(precision)
        res = prob.solve(tol=args.tol, maxit=maxit)
        tables_used.append(prob.stencil_tables)
        return prob, res

    log("warmup: %d step(s)" % args.warmup)
    for _ in range(args.warmup):
        for sc in schemes:
            hot_path(sc)
    torch.cuda.synchronize()

    log("timed: %d step(s)" % args.steps)
    solves = []
    t0 = time.perf_counter()
    for step in range(args.steps):
        for sc in schemes:
            prob, res = hot_path(sc)
            solves.append(dict(scheme=sc, status=res.status, iters=res.iters, restarts=res.restarts,
                               solve_ms=res.solve_ms, true_relres=res.true_relres))
            log("  step %d %s: status %d passes %d restarts %d solve %.1f ms true relres %.2e" %
                (step, sc, res.status, res.iters, res.restarts, res.solve_ms, res.true_relres))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / max(args.steps, 1)
    ok = [s for s in solves if s["status"] == adr.OK]
    # value: mean time to tolerance over the solves that reached it on the true
    # residual (ADR_OK); a solve that did not is reported, never averaged in
    solve_s = float(np.mean([s["solve_ms"] for s in ok])) / 1e3 if ok else None
    iters = {sc: [s["iters"] for s in solves if s["scheme"] == sc] for sc in schemes}
    mean_iters = float(np.mean([s["iters"] for s in solves]))
    ms_per_iter = float(np.mean([s["solve_ms"] / max(s["iters"], 1) for s in solves]))
    if not all(tables_used):
        raise RuntimeError("the solves did not use the stencil tables; the byte model below assumes them")
    algo_gbs = BYTES["iteration"] * N / (ms_per_iter * 1e-3) / 1e9
    dia_gbs = BYTES_DIA["iteration"] * N / (ms_per_iter * 1e-3) / 1e9

    # ---- discretisation error and true residual of each FP64 form ----
    forms = {}
    for sc in schemes:
        prob, res = hot_path(sc)
        forms["fp64_" + sc] = solve_record(prob, res)
        log("  fp64 %s: max error %.4e true relres %.2e" % (sc, forms["fp64_" + sc]["max_error"], res.true_relres))
        if sc == "centered":
            xref = res.x.clone()
            ref_rec = forms["fp64_" + sc]
        del prob, res

    # ---- per-kernel timing with HIP events on the library's stream ----
    log("kernel timing")
    prob, _ = hot_path("centered", maxit=1)
    q = torch.randn(N, dtype=torch.float64, device=dev)
    y = torch.empty_like(q)
    z = torch.empty_like(q)
    kern = {}
    times = kernel_us(prob, {"lsweep": lambda: prob.lsolve(q, out=y), "usweep": lambda: prob.usolve(y, out=z),
                             "spmv": lambda: prob.spmv(q, out=z)}, args.kernel_reps)
    for name, us in times.items():
        b = BYTES_DIA[name] * N
        kern[name] = dict(avg_us=us, algorithmic_bytes=b, gbs=b / (us * 1e-6) / 1e9,
                          bytes_per_unknown=BYTES_DIA[name], bytes_per_unknown_read=BYTES[name],
                          gbs_bytes_read=BYTES[name] * N / (us * 1e-6) / 1e9)
        log("  %s: %.1f us  %.0f GB/s of %d B/unknown (%.0f GB/s of the %d B it reads)" %
            (name, us, kern[name]["gbs"], BYTES_DIA[name], kern[name]["gbs_bytes_read"], BYTES[name]))
    dom = max(("lsweep", "usweep"), key=lambda k: kern[k]["avg_us"])
    traffic = traffic_for(dom, "n%d" % n)
    del prob
    copy_gbs = copy_reference_gbs(dev)
    log("  streaming copy kernel: %.0f GB/s" % copy_gbs)
    roofline = dict(bound="hbm", kernel=dom, achieved=round(kern[dom]["gbs"], 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(kern[dom]["gbs"] / PEAK_HBM_GBS, 4), traffic=traffic,
                    bytes_per_unknown=BYTES_DIA[dom], unknowns_per_launch=N,
                    bytes_per_unknown_read=BYTES[dom],
                    frac_of_bytes_read=round(kern[dom]["gbs_bytes_read"] / PEAK_HBM_GBS, 4))

    # ---- mixed precision: FP32-stored factors (FP64 or FP32 sweeps) ----
    variants = {}
    if args.variants:
        log("mixed-precision variants")
        e64 = ref_rec["max_error"]
        for prec in ("fp32_factors", "fp32_sweeps"):
            prob, res = hot_path("centered", maxit=args.variant_maxit, precision=prec)
            d = float((res.x - xref).abs().max() / xref.abs().max())
            rec = solve_record(prob, res, dict(
                speedup_vs_fp64=round(ref_rec["solve_s"] / (res.solve_ms / 1e3), 3) if res.solve_ms > 0 else None,
                max_rel_diff_vs_fp64=d, fp64_iters=ref_rec["iters"]))
            rec["max_error_within_1pct_of_fp64"] = bool(abs(rec["max_error"] - e64) <= 0.01 * e64)
            variants[prec] = rec
            log("  %s: status %d passes %d restarts %d (fp64 %d) %.2f s true relres %.2e max error %.4e "
                "(fp64 %.4e) max-rel-diff %.2e" % (prec, res.status, res.iters, res.restarts, ref_rec["iters"],
                                                  res.solve_ms / 1e3, res.true_relres, rec["max_error"], e64, d))
            del prob, res

    # ---- the Neumann variant over a fixed window of passes ----
    log("neumann window: %d passes" % args.neumann_window)
    neu = {}
    for sc in schemes:
        c = adr.classify(args.eps, 1.0, 1.0, n, n, sc, "neumann")
        _, res = hot_path(sc, bc="neumann", maxit=args.neumann_window)
        neu[sc] = dict(status=int(res.status), iters=int(res.iters), restarts=int(res.restarts),
                       solve_ms=round(res.solve_ms, 2), true_relres=float(res.true_relres),
                       algorithmic_gbs=round(BYTES["iteration"] * N * res.iters / (res.solve_ms * 1e-3) / 1e9, 1)
                       if res.solve_ms > 0 and res.iters > 0 else None,
                       last_relres=float(res.hist_l2[-1] / res.bnorm) if res.bnorm > 0 else None,
                       g_y=round(c.g_y, 2), expected_to_fail=c.expect_fail)
        log("  %s: status %d passes %d (g_y %.1f, expected to fail: %s)" % (sc, res.status, res.iters, c.g_y,
                                                                          c.expect_fail))

    # ---- CPU baseline: the oracle on a bounded sample ----
    cpu = None
    if args.cpu_baseline:
        log("cpu baseline (oracle), ~%.0f s" % args.cpu_seconds)
        from oracle import core as orc
        P = orc.assemble(args.eps, 1.0, 1.0, n, n, orc.CENTERED, orc.DIRICHLET)
        F = orc.ilu0(P)
        k = 1
        t_pass = None
        while True:
            c0 = time.perf_counter()
            orc.bicgstab(P, F, tol=args.tol, maxit=k)
            dt = time.perf_counter() - c0
            t_pass = dt / k
            if dt * 2 > args.cpu_seconds or k >= 64:
                break
            k = max(k + 1, int(args.cpu_seconds / 2 / max(t_pass, 1e-9)))
        est = t_pass * mean_iters
        cpu = dict(value=round(est, 2), unit="s", cores=1, kind="oracle", host=host_cpu(),
                   sample="%d BiCGSTAB passes of the single-threaded FP64 oracle on the %dx%d centered grid "
                          "(%.3f s per pass), extrapolated to the GPU's mean pass count %.0f" %
                          (k, n, n, t_pass, mean_iters, ))
        log("  %.3f s per pass -> %.1f s to tolerance (extrapolated)" % (t_pass, est))

    out = {
        # the headline metric: time to tolerance of the plain FP64 solve, with the
        # achieved HBM GB/s and the mixed-precision variant alongside
        "metric": "time to rel-resid 1e-10 & HBM GB/s: plain FP64 vs mixed/batched/warm-start",
        "value": round(solve_s, 4) if solve_s is not None else None,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32_sweeps" else "f64",
        "data": "synthetic",
        "config": {"workload": "advection-diffusion %dx%d, X=Y=1, eps=%g, upwind+centered, "
                               "Dirichlet substitute for the Neumann mix (which does not converge)" % (n, n, args.eps),
                   "nx": n, "ny": n, "eps": args.eps, "tol": args.tol, "precision": args.precision,
                   "sweep_rows": args.rows or "auto",
                   "stop": "||r||_2 < tol ||b||_2 on the recursive residual, confirmed on the true residual "
                           "b - A x (restart from x otherwise, up to 8 times)"},
        "solves_ok": "%d of %d" % (len(ok), len(solves)),
        "iters": iters,
        "ms_per_iter": round(ms_per_iter, 4),
        "bytes_per_unknown_per_pass": BYTES_DIA["iteration"],
        "bytes_per_unknown_per_pass_read": BYTES["iteration"],
        "hbm_gbs_algorithmic": round(dia_gbs, 1),
        "hbm_frac_algorithmic": round(dia_gbs / PEAK_HBM_GBS, 4),
        "hbm_gbs_bytes_read": round(algo_gbs, 1),
        "copy_kernel_gbs": round(copy_gbs, 1),
        "hbm_frac_of_copy_algorithmic": round(dia_gbs / copy_gbs, 4),
        "roofline_frac_of_copy": round(kern[dom]["gbs"] / copy_gbs, 4),
        "kernels": {k: {kk: round(vv, 2) for kk, vv in v.items()} for k, v in kern.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "mixed_precision": variants,
        "neumann_window": neu,
        "solves": solves,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
