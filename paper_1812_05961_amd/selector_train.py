"""Training harness of the variant selector.

  collect   for corpus tensors (synth.selector_tensor: 3-5 modes, log-uniform
            dims and nonzero counts, Zipf skew per mode, ranks 8-64), time
            every candidate of every mode on the GPU (exhaustive), one JSON
            line per (tensor, mode): statistics, candidates, times, and which
            candidate the fallback rule picks;
  train     network inputs from the recorded statistics (cpd_select_features),
            the network trained on the GPU (cpd_mlp_train) to predict the
            standardised log(ns per nonzero) of each candidate;
  evaluate  per held-out (tensor, mode): time of the network's choice over the
            fastest candidate, the fallback's, and the library default's (the
            tree rooted at the mode that cpd_als builds, default tile).

The target times are whole cpd_mttkrp calls (output zeroing and per-call
copies included) with factors padded to the rank, FP32 gathers.

    python -m paper_1812_05961_amd.selector_train collect --seeds 0:100 --out corpus.jsonl
    python -m paper_1812_05961_amd.selector_train train --corpus c1.jsonl c2.jsonl --out params.json
"""
from __future__ import annotations

import argparse
import gzip
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(HERE, "selector_params.json")
HIDDEN = 64


def _log(msg):
    print("[selector] " + msg, flush=True)


def _open(path, mode="rt"):
    return gzip.open(path, mode) if path.endswith(".gz") else open(path, mode)


# ---------------------------------------------------------------------------
# exhaustive timing


def time_call(fn, target_ms=0.5, max_batch=64):
    """Median over batches of the mean time (ms) of back-to-back calls of fn
    on the current stream, after one warm-up call; the batch size aims at
    target_ms of work, slow calls get one batch of one."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    e0.record()
    fn()
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1)
    k = int(min(max_batch, max(1, round(target_ms / max(t, 1e-3)))))
    nb = 3 if t < 20.0 else 1
    res = []
    for _ in range(nb):
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        e1.synchronize()
        res.append(e0.elapsed_time(e1) / k)
    return float(np.median(res))


def rooted_index(cands, dims, mode):
    """Index of the library's own default for a mode's MTTKRP: the tree cpd_als
    builds (the mode, then the rest by descending length) with the ROW
    kernel's default tile of 128 leaves (the LANE default 256 when the ROW
    kernel does not fit the tree)."""
    order = [mode] + sorted((m for m in range(len(dims)) if m != mode), key=lambda m: (-dims[m], m))
    for kernel, tile in (("row", 128), ("lane", 256)):
        for i, d in enumerate(cands):
            if d["order"] == order and d["kernel"] == kernel and d["tile_nnz"] == tile:
                return i
    raise ValueError("the rooted default is not among the candidates")


def time_tensor(x, rank, seed):
    """Exhaustive timing of every candidate of every mode of one tensor."""
    import torch

    from . import cpd
    N = x.nmodes
    inds = x.inds.to(torch.int32)
    st = cpd.tensor_stats(inds, x.dims)
    g = torch.Generator(device="cuda").manual_seed(seed)
    facs = [torch.rand((d, rank), device="cuda", generator=g) for d in x.dims]
    trees = {}
    recs = []
    try:
        for mode in range(N):
            cands = cpd.select_candidates(st, rank, mode)
            heur = cpd.select_heuristic(st, rank, mode).as_dict(N)
            cd = [c.as_dict(N) for c in cands]
            out = torch.empty((x.dims[mode], rank), device="cuda")
            ms = []
            for d in cd:
                key = tuple(d["order"])
                if key not in trees:
                    trees[key] = cpd.csf_build(inds, x.vals, x.dims, list(key))
                tree = trees[key]

                def fn(tree=tree, d=d, mode=mode, out=out):
                    cpd.mttkrp(tree, facs, mode, out=out, rank=rank, variant=d["variant"],
                               kernel=d["kernel"], tile_nnz=d["tile_nnz"])
                ms.append(time_call(fn))
            recs.append(dict(mode=mode, rank=rank, cands=cd, ms=ms, heur=cd.index(heur),
                             rooted=rooted_index(cd, x.dims, mode)))
    finally:
        for t in trees.values():
            t.free()
    return st.as_dict(), recs


def collect(seeds, max_nnz, out_path, time_limit=None):
    import torch

    from . import cpd, synth
    cpd.lib()
    t_start = time.perf_counter()
    done = set()
    if os.path.exists(out_path):
        with _open(out_path) as f:
            for line in f:
                done.add(json.loads(line)["seed"])
    with open(out_path, "a") as fo:
        for seed in seeds:
            if seed in done:
                continue
            if time_limit and time.perf_counter() - t_start > time_limit:
                _log("time limit reached before seed %d" % seed)
                break
            t0 = time.perf_counter()
            x = synth.selector_tensor(seed, device="cuda", max_nnz=max_nnz)
            spec = synth.selector_spec(seed, max_nnz)
            t1 = time.perf_counter()
            st, recs = time_tensor(x, spec["rank"], seed)
            for r in recs:
                r.update(seed=seed, stats=st, spec=spec)
                fo.write(json.dumps(r) + "\n")
            fo.flush()
            ncand = sum(len(r["cands"]) for r in recs)
            best = [min(r["ms"]) for r in recs]
            _log("seed %d: %d modes, nnz %d, rank %d: gen %.2f s, timing %.2f s, %d candidates, "
                 "best ms %s" % (seed, x.nmodes, x.nnz, spec["rank"], t1 - t0,
                                 time.perf_counter() - t1, ncand,
                                 ",".join("%.3f" % b for b in best)))
            del x
            torch.cuda.empty_cache()


def load_corpus(paths):
    recs = []
    for p in paths:
        with _open(p) as f:
            for line in f:
                recs.append(json.loads(line))
    return recs


# ---------------------------------------------------------------------------
# features, training, evaluation


def case_features(rec):
    from . import cpd
    s = rec["stats"]
    st = cpd.make_stats(s["dims"], s["nnz"], s["top1"], s["distinct"], s["alpha"], s["sample"])
    cands = [cpd.make_choice(d) for d in rec["cands"]]
    return cpd.select_features(st, rec["rank"], rec["mode"], cands)


def case_targets(rec):
    """log(ns per nonzero) of each candidate."""
    nnz = rec["stats"]["nnz"]
    return np.log(np.asarray(rec["ms"], dtype=np.float64) * 1e6 / nnz)


def build_matrix(recs):
    X = np.concatenate([case_features(r) for r in recs]).astype(np.float32)
    y = np.concatenate([case_targets(r) for r in recs])
    return X, y


def train(recs, epochs=300, batch=256, lr=1e-3, seed=1, hidden=HIDDEN):
    import torch

    from . import cpd
    X, y = build_matrix(recs)
    mu, sd = float(y.mean()), float(y.std())
    yn = ((y - mu) / sd).astype(np.float32)
    p = cpd.mlp_init(cpd.SEL_NFEAT, hidden, seed)
    trace = cpd.mlp_train(p, cpd.SEL_NFEAT, hidden, torch.from_numpy(X).cuda(),
                          torch.from_numpy(yn).cuda(), epochs, batch, lr, seed)
    torch.cuda.synchronize()
    return p, dict(y_mean=mu, y_std=sd, loss_trace=trace, samples=int(X.shape[0]))


def predict(params, recs, hidden=HIDDEN):
    import torch

    from . import cpd
    out = []
    for r in recs:
        F = torch.from_numpy(case_features(r)).cuda()
        out.append(cpd.mlp_forward(params, cpd.SEL_NFEAT, hidden, F).cpu().numpy())
    return out


def evaluate(recs, preds):
    """Ratios t(choice) / t(best) for the network, the fallback rule and the
    library's own default (the rooted tree cpd_als builds, default tile)."""
    net, heur, rooted = [], [], []
    for r, p in zip(recs, preds):
        ms = np.asarray(r["ms"])
        best = ms.min()
        net.append(ms[int(np.argmin(p))] / best)
        heur.append(ms[r["heur"]] / best)
        rooted.append(ms[r["rooted"]] / best)
    net, heur, rooted = np.array(net), np.array(heur), np.array(rooted)

    def summ(a):
        return dict(geomean=float(np.exp(np.log(a).mean())), mean=float(a.mean()),
                    median=float(np.median(a)), p90=float(np.quantile(a, 0.9)),
                    max=float(a.max()), within_10pct=float((a <= 1.10).mean()))
    return dict(cases=len(recs), network=summ(net), heuristic=summ(heur), rooted_default=summ(rooted),
                speedup_over_heuristic_geomean=float(np.exp(np.log(heur / net).mean())),
                speedup_over_rooted_default_geomean=float(np.exp(np.log(rooted / net).mean())))


def save_params(path, params, meta):
    from . import cpd
    d = dict(n_in=cpd.SEL_NFEAT, hidden=meta.get("hidden", HIDDEN),
             params=[float(v) for v in params.cpu().numpy()])
    d.update({k: v for k, v in meta.items() if k != "hidden"})
    with open(path, "w") as f:
        json.dump(d, f)


def load_params(path=PARAMS_PATH, device="cuda"):
    """(params tensor on the device, hidden) of a trained network."""
    import torch

    from . import cpd
    with open(path) as f:
        d = json.load(f)
    if d["n_in"] != cpd.SEL_NFEAT:
        raise ValueError("network built for %d inputs, the library has %d" % (d["n_in"], cpd.SEL_NFEAT))
    p = torch.tensor(d["params"], dtype=torch.float32, device=device)
    if p.numel() != cpd.mlp_param_count(d["n_in"], d["hidden"]):
        raise ValueError("parameter count does not match the shape")
    return p, d["hidden"]


def _seed_range(s):
    a, b = s.split(":")
    return range(int(a), int(b))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--seeds", required=True, help="a:b")
    c.add_argument("--max-nnz", type=float, default=5e7)
    c.add_argument("--out", required=True)
    c.add_argument("--time-limit", type=float, default=None, help="seconds")
    t = sub.add_parser("train")
    t.add_argument("--corpus", nargs="+", required=True)
    t.add_argument("--train-seeds", default="0:1600")
    t.add_argument("--eval-seeds", default="1600:2000")
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=1)
    t.add_argument("--out", default=PARAMS_PATH)
    t.add_argument("--report", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        collect(_seed_range(a.seeds), a.max_nnz, a.out, a.time_limit)
        return
    recs = load_corpus(a.corpus)
    tr_s, ev_s = set(_seed_range(a.train_seeds)), set(_seed_range(a.eval_seeds))
    tr = [r for r in recs if r["seed"] in tr_s]
    ev = [r for r in recs if r["seed"] in ev_s]
    _log("corpus: %d cases (%d train, %d held-out)" % (len(recs), len(tr), len(ev)))
    t0 = time.perf_counter()
    params, meta = train(tr, a.epochs, a.batch, a.lr, a.seed)
    _log("trained in %.1f s; loss %.4f -> %.4f" % (time.perf_counter() - t0, meta["loss_trace"][0],
                                                  meta["loss_trace"][-1]))
    rep = dict(train=evaluate(tr, predict(params, tr)), heldout=evaluate(ev, predict(params, ev)),
               train_tensors=len({r["seed"] for r in tr}), heldout_tensors=len({r["seed"] for r in ev}),
               epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, samples=meta["samples"])
    meta.update(hidden=HIDDEN, report=rep)
    save_params(a.out, params, meta)
    _log(json.dumps(rep))
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
