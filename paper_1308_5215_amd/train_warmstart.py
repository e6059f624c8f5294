"""Train and evaluate the learned initial guess (include/adr_cnn.h).

Training data are converged FP64 solutions that the batched solver itself
produces for seeded instances (eps log-uniform in [1e-3, 1], X and Y uniform
in [0.5, 2], Dirichlet or Neumann outer sides with p = 1/2, upwind or
centered convection with p = 1/2, forcing f_man + 0.1 max|f_man| times a
Gaussian random field); only instances whose solve ends with status OK and
that the instance classifier (adr_classify: cell Peclet numbers, the Neumann
growth factor, the sign of the diagonal; Section 6.3) expects to be well
posed are kept.  The network is trained on the GPU by the library's own
forward/backward kernels with Adam.  Evaluation solves held-out instances
twice, from zero and from the network's guess (with the zero-guess
fallback), to the same tolerance, and reports iterations and time per
scheme.

    python paper_1308_5215_amd/train_warmstart.py --train 20000 --out weights.npy
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1308_5215_amd as adr  # noqa: E402
from synthetic.fields import gaussian_random_field  # noqa: E402
from synthetic.warmstart import initial_params, warmstart_instance  # noqa: E402

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_256.npy")
TRAIN_SEED0, HELDOUT_SEED0 = 0, 100000
AMP = 0.1
# Training and the evaluation's well-posed set take the instances that the
# instance classifier (adr_classify) expects to converge, whose Neumann
# closure amplifies by at most e^5 (g_y <= G_Y_MAX) and whose wrong-sign
# couplings, if any, come with cell Peclet numbers of at most PE_MAX.  Beyond
# these the discrete solution grows by orders of magnitude (the convection
# term differenced against the flow, or a Neumann side amplifying the
# forcing): measured on training seeds 0..767, every converged instance
# inside the rule stays below 1.9 in magnitude (the exact u is below 1.27)
# while converged instances outside it reach 3.9e3.
G_Y_MAX, PE_MAX = 5.0, 4.0


def well_posed(d, tol):
    """The instance classifier's verdict on instance d, as above."""
    c = adr.classify(d["eps"], d["X"], d["Y"], d["n"], d["n"], d["scheme"], d["bc"], tol)
    return (not c.expect_fail and (d["bc"] == 0 or c.g_y <= G_Y_MAX)
            and (c.neg_offdiag == 0 or max(c.pe_x, c.pe_y) <= PE_MAX))


def _field(d):
    n = d["n"]
    return gaussian_random_field(n, n, d["X"] / (n + 1), d["Y"] / (n + 1), length=0.1, seed=d["field_seed"])


def make_batch(seeds, n, pool=None):
    """Assemble the instances of `seeds` as one batch on the GPU."""
    import torch
    inst = [warmstart_instance(s, n=n) for s in seeds]
    fields = pool.map(_field, inst, chunksize=8) if pool is not None else [_field(d) for d in inst]
    fd = torch.from_numpy(np.concatenate([f.ravel() for f in fields])).cuda()
    cnt = len(inst)
    batch = adr.assemble_batch([d["eps"] for d in inst], [d["X"] for d in inst], [d["Y"] for d in inst],
                               [n] * cnt, [n] * cnt, [d["scheme"] for d in inst], [d["bc"] for d in inst],
                               field=fd, amp=AMP)
    del fd
    return batch, inst


def generate(seeds, n, tol, maxit, chunk=256, pool=None, log=print):
    """Converged solutions of the seeded instances: (inputs bf16 [K, n+2, n+2, 32],
    targets f32 [K, n, n], per-seed record)."""
    import torch
    H = n + 2
    inputs = torch.empty((len(seeds), H, H, 32), dtype=torch.bfloat16, device="cuda")
    targets = torch.empty((len(seeds), n, n), dtype=torch.float32, device="cuda")
    kept, rec = 0, []
    t0 = time.time()
    for c0 in range(0, len(seeds), chunk):
        cs = seeds[c0:c0 + chunk]
        batch, inst = make_batch(cs, n, pool)
        batch.ilu0("fp64")
        res = batch.solve(tol=tol, maxit=maxit)
        feats = batch.features()
        for k, xk in enumerate(batch.split(res.x)):
            wp = well_posed(inst[k], tol)
            rec.append(dict(seed=int(cs[k]), status=int(res.status[k]), iters=int(res.iters[k]),
                            scheme=inst[k]["scheme"], well_posed=wp))
            if res.status[k] == adr.OK and wp:
                inputs[kept].copy_(feats[k])
                targets[kept].copy_(xk.view(n, n))
                kept += 1
        del feats, res
        batch.close()
        log("generated %d/%d instances (%d converged) in %.1f s" % (
            min(c0 + chunk, len(seeds)), len(seeds), kept, time.time() - t0))
    return inputs[:kept], targets[:kept], rec


def train(net, inputs, targets, epochs, batch, lr, seed=0, log=print, time_limit=None):
    """Adam on contiguous minibatches visited in a seeded random order each
    epoch, with a cosine learning-rate decay; returns the per-epoch mean loss."""
    K = inputs.shape[0]
    nb = K // batch
    rng = np.random.default_rng(seed)
    total = epochs * nb
    step, hist = 0, []
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(nb)
        acc = 0.0
        for b in order:
            cur = lr * 0.5 * (1.0 + np.cos(np.pi * step / max(total, 1)))
            acc += net.train_step(inputs[b * batch:(b + 1) * batch], targets[b * batch:(b + 1) * batch], lr=cur)
            step += 1
        hist.append(acc / max(nb, 1))
        log("epoch %d/%d: mean loss %.4e (%.1f s)" % (ep + 1, epochs, hist[-1], time.time() - t0))
        if time_limit is not None and time.time() - t0 > time_limit:
            log("stopping at the time limit")
            break
    return hist


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t) * 1e3


def evaluate(net, seeds, n, tol, maxit, chunk=256, pool=None, log=print, single=32):
    """Held-out comparison of the zero guess and the network's guess.

    Per chunk: every instance is solved from both guesses (iterations and
    statuses); then the instances that converged both ways and that the
    classifier expects to be well posed are assembled again as one batch and
    both solves are timed on it (the network's time
    includes the input fields, inference and the fallback test).  The first
    `single` of those are also timed one instance at a time."""
    import torch
    out = dict(seeds=[], zero_iters=[], warm_iters=[], zero_status=[], warm_status=[], used=[], well_posed=[],
               scheme=[], max_rel_diff=[], zero_ms=0.0, warm_ms=0.0, guess_ms=0.0, single_zero_ms=[],
               single_warm_ms=[])
    ok_all = []
    for c0 in range(0, len(seeds), chunk):
        cs = seeds[c0:c0 + chunk]
        batch, inst = make_batch(cs, n, pool)
        batch.ilu0("fp64")
        z = batch.solve(tol=tol, maxit=maxit)
        x0, used = batch.warm_start(net)
        w = batch.solve(tol=tol, maxit=maxit, x0=x0)
        wp = [well_posed(d, tol) for d in inst]
        for a, b in zip(batch.split(z.x), batch.split(w.x)):
            den = float(torch.max(torch.abs(a)))
            out["max_rel_diff"].append(float(torch.max(torch.abs(a - b))) / den if den > 0 else 0.0)
        out["well_posed"] += wp
        out["scheme"] += [d["scheme"] for d in inst]
        out["seeds"] += [int(s) for s in cs]
        out["zero_iters"] += z.iters.tolist()
        out["warm_iters"] += w.iters.tolist()
        out["zero_status"] += z.status.tolist()
        out["warm_status"] += w.status.tolist()
        out["used"] += used.astype(int).tolist()
        batch.close()
        ok = [s for k, s in enumerate(cs) if z.status[k] == adr.OK and w.status[k] == adr.OK and wp[k]]
        ok_all += ok
        if ok:
            batch, _ = make_batch(ok, n, pool)
            batch.ilu0("fp64")
            _, tz = _timed(lambda: batch.solve(tol=tol, maxit=maxit))
            (x0, _), tg = _timed(lambda: batch.warm_start(net))
            _, ts = _timed(lambda: batch.solve(tol=tol, maxit=maxit, x0=x0))
            out["zero_ms"] += tz
            out["guess_ms"] += tg
            out["warm_ms"] += tg + ts
            batch.close()
        log("evaluated %d/%d" % (min(c0 + chunk, len(seeds)), len(seeds)))
    for s in ok_all[:single]:
        batch, _ = make_batch([s], n, None)
        batch.ilu0("fp64")
        batch.solve(tol=tol, maxit=maxit)            # warm-up (graph capture)
        _, tz = _timed(lambda: batch.solve(tol=tol, maxit=maxit))
        (x0, _), tg = _timed(lambda: batch.warm_start(net))
        _, ts = _timed(lambda: batch.solve(tol=tol, maxit=maxit, x0=x0))
        out["single_zero_ms"].append(tz)
        out["single_warm_ms"].append(tg + ts)
        batch.close()
    zi, wi = np.array(out["zero_iters"]), np.array(out["warm_iters"])
    conv = (np.array(out["zero_status"]) == 0) & (np.array(out["warm_status"]) == 0)
    both = conv & np.array(out["well_posed"], dtype=bool)
    sch = np.array(out["scheme"])

    def per_scheme(sc):
        m = both & (sch == sc)
        return dict(instances=int((sch == sc).sum()), well_posed_converged=int(m.sum()),
                    mean_zero_iters=float(zi[m].mean()) if m.any() else None,
                    mean_warm_iters=float(wi[m].mean()) if m.any() else None,
                    iters_saved_frac=float(1.0 - wi[m].sum() / zi[m].sum()) if m.any() else None)
    sz, sw = float(np.sum(out["single_zero_ms"])), float(np.sum(out["single_warm_ms"]))
    out["summary"] = dict(
        instances=len(seeds), both_converged=int(conv.sum()), well_posed_converged=int(both.sum()),
        guess_used=int(np.sum(out["used"])),
        guess_used_well_posed=int(np.sum(np.array(out["used"])[both])),
        all_converged_iters_saved_frac=float(1.0 - wi[conv].sum() / zi[conv].sum()) if conv.any() else None,
        mean_zero_iters=float(zi[both].mean()) if both.any() else None,
        mean_warm_iters=float(wi[both].mean()) if both.any() else None,
        iters_saved_frac=float(1.0 - wi[both].sum() / zi[both].sum()) if both.any() else None,
        batched_zero_ms=out["zero_ms"], batched_warm_ms=out["warm_ms"], batched_guess_ms=out["guess_ms"],
        batched_time_saved_frac=float(1.0 - out["warm_ms"] / out["zero_ms"]) if out["zero_ms"] > 0 else None,
        single_instances=len(out["single_zero_ms"]), single_zero_ms=sz, single_warm_ms=sw,
        single_time_saved_frac=float(1.0 - sw / sz) if sz > 0 else None,
        status_changed=int(np.sum(np.array(out["zero_status"]) != np.array(out["warm_status"]))),
        max_rel_diff_well_posed=float(np.max(np.array(out["max_rel_diff"])[both])) if both.any() else None,
        upwind=per_scheme(0), centered=per_scheme(1),
    )
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--train", type=int, default=20000, help="training seeds (0, 1, ...)")
    ap.add_argument("--heldout", type=int, default=1000, help="held-out seeds (100000, ...)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxit", type=int, default=1500)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--train-time", type=float, default=None, help="stop training after this many seconds")
    ap.add_argument("--init", default=None, help="start from these weights (.npy) instead of a seeded init")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--report", default=None, help="write a JSON report here")
    a = ap.parse_args(argv)
    import torch

    def log(msg):
        print(msg, flush=True)

    pool = Pool(a.workers) if a.workers > 1 else None
    report = dict(args=vars(a))
    net = adr.WarmStartNet(a.n + 2, a.n + 2, max(a.batch, 64))
    p0 = np.load(a.init) if a.init else initial_params(0)
    net.set_params(p0)
    if a.train > 0:
        t = time.time()
        inputs, targets, rec = generate(list(range(TRAIN_SEED0, TRAIN_SEED0 + a.train)), a.n, a.tol, a.maxit,
                                        pool=pool, log=log)
        report["generate_s"] = time.time() - t
        report["train_instances"] = int(inputs.shape[0])
        report["train_converged"] = int(sum(1 for r in rec if r["status"] == 0))
        report["train_iters_mean"] = float(np.mean([r["iters"] for r in rec if r["status"] == 0]))
        t = time.time()
        report["loss"] = train(net, inputs, targets, a.epochs, a.batch, a.lr, log=log, time_limit=a.train_time)
        torch.cuda.synchronize()
        report["train_s"] = time.time() - t
        del inputs, targets
        torch.cuda.empty_cache()
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.save(a.out, net.get_params())
        log("saved %s" % a.out)
    if a.heldout > 0:
        ev = evaluate(net, list(range(HELDOUT_SEED0, HELDOUT_SEED0 + a.heldout)), a.n, a.tol, 2 * a.maxit,
                      pool=pool, log=log)
        report["heldout"] = ev["summary"]
        report["heldout_detail"] = {k: ev[k] for k in ("seeds", "zero_iters", "warm_iters", "zero_status",
                                                        "warm_status", "used", "scheme", "well_posed")}
        log(json.dumps(ev["summary"]))
    if a.report:
        with open(a.report, "w") as f:
            json.dump(report, f)
    if pool is not None:
        pool.close()
    return report


if __name__ == "__main__":
    main()
