"""Learned warm start for personalized CPAA: training on CPAA outputs and
evaluation against plain CPAA.

    python -m paper_2112_01743_amd.warmstart --out result.json [--n 1000000 ...]

Training graph: Chung-Lu, n vertices, average degree 16, exponent 2.1
(seed 2112004).  Targets are plain CPAA solves (cpaa_solve_batched, 256
sources per call, certified to 1e-6 L1) of random training sources; the
network (cpaa_model_*) is trained on them with Adam.  Evaluation: an unseen
graph from the same generator (seed 2112005) and held-out random sources,
each solved (a) plainly and (b) from the network's guess by CPAA on the
residual; plain CPAA is both the fallback and the judge (the two results
must agree within the sum of their certified bounds).  Reports Chebyshev
terms, solves/s with and without the network's inference, and how often the
guess was rejected.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def save_checkpoint(path: str, model, meta: dict) -> None:
    """Parameters, Adam moments and step in an .npz (no pickled objects)."""
    w, m, v, step = model.get_state()
    np.savez(path, params=w, adam_m=m, adam_v=v, step=np.array([step], dtype=np.int64),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_checkpoint(path: str, model) -> dict:
    with np.load(path, allow_pickle=False) as z:
        model.set_state(z["params"], z["adam_m"], z["adam_v"], int(z["step"][0]))
        return json.loads(bytes(z["meta"]).decode())


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def train(plan, model, g, train_sources, *, chunk=256, batch=8, epochs=1, lr=3e-2,
          lr_final=3e-3, tol=1e-6, seed=0):
    """Targets per chunk of sources come from plain batched CPAA; each chunk is
    visited `epochs` times in shuffled minibatches."""
    import torch
    import graphgen as gg
    rng = gg.philox(seed)
    steps_total = epochs * int(np.ceil(len(train_sources) / batch))
    step = 0
    losses = []
    t_solve = t_train = 0.0
    for c0 in range(0, len(train_sources), chunk):
        src = np.asarray(train_sources[c0:c0 + chunk])
        P = torch.zeros((len(src), g.n), dtype=torch.float64, device="cuda")
        P[torch.arange(len(src)), torch.as_tensor(src, device="cuda")] = 1.0
        t0 = time.perf_counter()
        T, reps = plan.solve_batched(P, tol)
        torch.cuda.synchronize()
        t_solve += time.perf_counter() - t0
        if not all(r["certified"] for r in reps):
            raise RuntimeError("a training target was not certified")
        del P
        t0 = time.perf_counter()
        for _ in range(epochs):
            order = rng.permutation(len(src))
            for b0 in range(0, len(src), batch):
                idx = order[b0:b0 + batch]
                frac = step / max(1, steps_total - 1)
                lr_now = lr * (lr_final / lr) ** frac
                loss, _ = model.train_step(src[idx], T[idx], lr_now)
                losses.append(loss)
                step += 1
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t0
        _log(f"trained on sources {c0}..{c0 + len(src)}: L1 {np.mean(losses[-len(src)//batch:]):.4f}")
        del T
    return {"steps": step, "target_solve_s": t_solve, "train_s": t_train,
            "l1_first": float(np.mean(losses[:16])), "l1_last": float(np.mean(losses[-16:]))}


def evaluate(plan, model, g, sources, *, tol=1e-6, chunk=256):
    import torch
    out = {"plain_terms": [], "warm_terms": [], "fallback": 0, "x0_l1": [], "x0_resid_ratio": [],
           "plain_s": 0.0, "warm_s": 0.0, "predict_s": 0.0, "agree_max": 0.0}
    for c0 in range(0, len(sources), chunk):
        src = np.asarray(sources[c0:c0 + chunk])
        P = torch.zeros((len(src), g.n), dtype=torch.float64, device="cuda")
        P[torch.arange(len(src)), torch.as_tensor(src, device="cuda")] = 1.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xp, rp = plan.solve_batched(P, tol)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X0 = model.predict(src)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        Xw, rw = plan.solve_batched(P, tol, X0=X0)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        out["plain_s"] += t1 - t0
        out["predict_s"] += t2 - t1
        out["warm_s"] += t3 - t2
        out["plain_terms"] += [r["terms"] + r["refine_terms"] for r in rp]
        out["warm_terms"] += [r["terms"] + r["refine_terms"] for r in rw]
        out["fallback"] += sum(r["fallback_used"] for r in rw)
        diff = (Xw - Xp).abs().sum(dim=1).cpu().numpy()
        bounds = np.array([a["cert_bound"] + b["cert_bound"] for a, b in zip(rw, rp)])
        certified = np.all(rw["certified"] == 1) and np.all(rp["certified"] == 1)
        if not (np.all(diff <= bounds) and certified):
            raise RuntimeError("warm-started and plain results disagree beyond their bounds")
        out["agree_max"] = max(out["agree_max"], float(diff.max()))
        out["x0_l1"] += (X0 - Xp).abs().sum(dim=1).cpu().numpy().tolist()
        del P, Xp, Xw, X0
    n = len(sources)
    return {
        "sources": n,
        "plain_terms_mean": float(np.mean(out["plain_terms"])),
        "warm_terms_mean": float(np.mean(out["warm_terms"])),
        "fallback_rate": out["fallback"] / n,
        "x0_l1_mean": float(np.mean(out["x0_l1"])),
        "plain_solves_per_s": n / out["plain_s"],
        "warm_solves_per_s_incl_inference": n / (out["warm_s"] + out["predict_s"]),
        "warm_solves_per_s_excl_inference": n / out["warm_s"],
        "inference_ms_per_source": 1e3 * out["predict_s"] / n,
        "max_warm_vs_plain_l1": out["agree_max"],
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--avg-deg", type=float, default=16.0)
    ap.add_argument("--train-sources", type=int, default=2048)
    ap.add_argument("--eval-sources", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=3e-2)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    torch.cuda.init()          # torch's HIP context first, then the library's plans
    import graphgen as gg
    from paper_2112_01743_amd import Plan
    from paper_2112_01743_amd.binding import Model

    c = 0.85
    t0 = time.perf_counter()
    g_tr = gg.chung_lu(args.n, args.avg_deg, 2.1, seed=2112004, dmax=50000)
    g_ev = gg.chung_lu(args.n, args.avg_deg, 2.1, seed=2112005, dmax=50000)
    _log(f"graphs n={g_tr.n} nnz={g_tr.nnz}/{g_ev.nnz} ({time.perf_counter() - t0:.1f} s)")
    plan_tr = Plan.from_graph(g_tr, c)
    model = Model(plan_tr, gg.mpnn_init(2112004))
    tr_src = gg.random_sources(g_tr.n, args.train_sources, seed=2112004)
    stats = train(plan_tr, model, g_tr, tr_src, batch=args.batch, epochs=args.epochs, lr=args.lr,
                  tol=args.tol)
    _log(f"training {stats}")
    if args.checkpoint:
        save_checkpoint(args.checkpoint, model, {"graph_seed": 2112004, **stats})
    w, m, v, step = model.get_state()
    plan_ev = Plan.from_graph(g_ev, c)
    model_ev = Model(plan_ev, gg.mpnn_init(0))
    model_ev.set_state(w, m, v, step)
    ev_src = gg.random_sources(g_ev.n, args.eval_sources, seed=2112005)
    res = evaluate(plan_ev, model_ev, g_ev, ev_src, tol=args.tol)
    res.update(workload="warm start on unseen Chung-Lu graph", n=g_ev.n, nnz=g_ev.nnz,
               train=stats, tol_l1=args.tol)
    line = json.dumps(res)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
