"""Learned form of the target-dimension search (a method extension, not in
the paper): generate instances, label them with the plain certified fit,
train the predictor MLP with the library's own kernels, and evaluate the
learned search against plain bisection.

Every GPU computation here goes through the C ABI (sketch features, MLP
forward/backward/Adam, fits).  Instances are drawn on the host by
``gen.power_law`` in parallel worker processes while the GPU labels the
previous ones.

Command line (runs on a GPU host):
  python -m paper_1609_05388_amd.learned label --start 0 --stop 4096 --out labels.npz
  python -m paper_1609_05388_amd.learned label --held-out --start 0 --stop 512 --out held.npz
  python -m paper_1609_05388_amd.learned train --labels labels.npz --held held.npz --out predictor.npz
  python -m paper_1609_05388_amd.learned evaluate --predictor predictor.npz --start 0 --stop 64
"""
import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import gen

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
PREDICTOR = os.path.join(DATA_DIR, "predictor.npz")
TAU = 0.9
IN_USED = 67


def instance(index, held_out=False):
    """(params, X float32) of one learned-form instance."""
    pr = gen.instance_params(index, held_out)
    X = gen.power_law(pr["n"], pr["d"], pr["rank"], pr["alpha"], noise=0.01, seed=pr["seed"])
    return pr, X


def _instance_worker(args):
    index, held_out = args
    return instance(index, held_out)


_THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def instances(indices, held_out=False, workers=None):
    """Yield (index, params, X) in order, drawn by a pool of worker processes
    (single-threaded BLAS each, leaving host cores to the process that drives
    the GPU)."""
    workers = workers or min(8, max(1, (os.cpu_count() or 2) // 2))
    saved = {k: os.environ.get(k) for k in _THREAD_VARS}
    for k in _THREAD_VARS:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        pool = ctx.Pool(workers)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    with pool:
        for index, (pr, X) in zip(indices, pool.imap(_instance_worker, [(i, held_out) for i in indices],
                                                     chunksize=1)):
            yield index, pr, X


def target(r, d):
    """Regression target: ln(r / d)."""
    return np.log(np.asarray(r, np.float64) / np.asarray(d, np.float64))


def predicted_r(y, d):
    """r from a predicted ln(r / d): ceil(d exp(y)) clamped to [1, d]."""
    return int(min(d, max(1, int(np.ceil(d * np.exp(min(float(y), 0.0)))))))


def _save_labels(rows, held_out, out_path):
    cols = list(zip(*rows))
    tmp = out_path + ".tmp.npz"
    np.savez(tmp, index=np.array(cols[0]), n=np.array(cols[1]), d=np.array(cols[2]),
             alpha=np.array(cols[3]), rank=np.array(cols[4]), eps=np.array(cols[5]), r=np.array(cols[6]),
             certificates=np.array(cols[7]), fit_ms=np.array(cols[8]), max_distortion=np.array(cols[9]),
             certified=np.array(cols[10]), feat=np.stack(cols[11]).astype(np.float32), held_out=held_out)
    os.replace(tmp, out_path)


def label(indices, held_out, out_path, log_every=25, save_every=256):
    """Label instances with the plain certified fit (BF16 split screen: same
    decisions as the FP32 one); the label file is rewritten every
    ``save_every`` instances so partial progress survives."""
    import torch
    from . import adagio
    adagio.load()
    rows = []
    t0 = time.time()
    for k, (index, pr, X) in enumerate(instances(list(indices), held_out)):
        Xd = torch.from_numpy(X).cuda()
        feat = adagio.sketch_features(Xd, pr["eps"], gen.JL_SEED)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        fit = adagio.fit(Xd, pr["eps"], gen.JL_SEED, screen="bf16x3")
        torch.cuda.synchronize()
        fit_ms = (time.perf_counter() - ta) * 1e3
        rows.append((index, pr["n"], pr["d"], pr["alpha"], pr["rank"], pr["eps"], fit["r"],
                     fit["stats"]["n_certificates"], fit_ms, fit["cert"]["max_distortion"],
                     fit["cert"]["certified"], feat.cpu().numpy()))
        if (k + 1) % log_every == 0:
            print("labelled %d/%d (last: n=%d d=%d eps=%.3f r*=%d, %.0f ms) %.0f s"
                  % (k + 1, len(indices), pr["n"], pr["d"], pr["eps"], fit["r"], fit_ms, time.time() - t0),
                  flush=True)
        if (k + 1) % save_every == 0:
            _save_labels(rows, held_out, out_path)
        del Xd
    _save_labels(rows, held_out, out_path)
    print("wrote %s (%d instances, %.0f s)" % (out_path, len(rows), time.time() - t0), flush=True)


def init_params(count, seed=0):
    """He-uniform weights, zero biases, in the library's parameter layout
    (W1[256][80] (first 67 columns used), b1, W2, b2, W3, b3, w4, b4)."""
    rng = np.random.default_rng(seed)
    H, K = 256, 80
    p = np.zeros(count, np.float32)
    o = 0
    W1 = np.zeros((H, K), np.float32)
    W1[:, :IN_USED] = rng.uniform(-1, 1, (H, IN_USED)) * np.sqrt(6.0 / IN_USED)
    p[o:o + H * K] = W1.ravel()
    o += H * K + H
    for _ in range(2):
        p[o:o + H * H] = (rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)).ravel()
        o += H * H + H
    p[o:o + H] = rng.uniform(-1, 1, H) * np.sqrt(6.0 / H)
    return p


def train(labels, held, out_path, epochs=400, batch=256, lr=1e-3, seed=0, log_every=50):
    import torch
    from . import adagio
    adagio.load()
    tr, ho = np.load(labels), np.load(held)
    X = torch.from_numpy(tr["feat"]).cuda()
    y = torch.from_numpy(target(tr["r"], tr["d"]).astype(np.float32)).cuda()
    Xh = torch.from_numpy(ho["feat"]).cuda()
    yh = target(ho["r"], ho["d"])
    count = adagio.mlp_param_count()
    params = torch.from_numpy(init_params(count, seed)).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    rng = np.random.default_rng(seed + 1)
    N = X.shape[0]
    step = 0
    hist = []
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(N)).cuda()
        losses = []
        for b0 in range(0, N - batch + 1, batch):
            idx = order[b0:b0 + batch]
            step += 1
            losses.append(adagio.mlp_train_step(params, m, v, step, lr, X[idx].contiguous(), y[idx].contiguous(), TAU))
        if (ep + 1) % log_every == 0 or ep == epochs - 1:
            train_loss = float(torch.stack(losses).mean())
            pred = adagio.mlp_forward(params, Xh).cpu().numpy().astype(np.float64)
            u = yh - pred
            ho_loss = float(np.mean(np.maximum(TAU * u, (TAU - 1) * u)))
            over = float(np.mean(pred >= yh))
            hist.append((ep + 1, train_loss, ho_loss, over))
            print("epoch %d: train pinball %.4f, held-out pinball %.4f, held-out prediction >= target %.3f"
                  % (ep + 1, train_loss, ho_loss, over), flush=True)
    np.savez(out_path, params=params.cpu().numpy(), tau=TAU, epochs=epochs, batch=batch, lr=lr,
             history=np.array(hist))
    print("wrote", out_path, flush=True)


def load_predictor(path=PREDICTOR, device="cuda"):
    import torch
    return torch.from_numpy(np.load(path)["params"].astype(np.float32)).to(device)


def evaluate(predictor_path, indices, held_out=True, log_every=8):
    """Plain bisection vs learned search on instances: returns a list of dicts.
    The fits keep the library's workspace across calls (as a loop of fits
    should: a workspace made and freed per call adds its streams' and buffers'
    set-up to every fit); each fit is timed after a warm-up fit of the same
    search on the same instance."""
    import torch
    from . import adagio
    adagio.load()
    P = load_predictor(predictor_path)
    res = []
    adagio.keep_workspace(True)
    try:
        for k, (index, pr, X) in enumerate(instances(list(indices), held_out)):
            res.append(_evaluate_one(adagio, P, index, pr, X))
            if (k + 1) % log_every == 0:
                print("evaluated %d/%d" % (k + 1, len(indices)), flush=True)
    finally:
        adagio.keep_workspace(False)
    return res


def _evaluate_one(adagio, P, index, pr, X):
    """Both searches on one instance (a warm-up fit, then the timed one)."""
    import torch
    Xd = torch.from_numpy(X).cuda()
    out = {}
    for mode in ("bisect", "learned"):
        adagio.fit(Xd, pr["eps"], gen.JL_SEED, screen="bf16x3", search=mode, predictor=P)  # warm buffers
        torch.cuda.synchronize()
        ta = time.perf_counter()
        f = adagio.fit(Xd, pr["eps"], gen.JL_SEED, screen="bf16x3", search=mode, predictor=P)
        torch.cuda.synchronize()
        out[mode] = {"r": f["r"], "ms": (time.perf_counter() - ta) * 1e3,
                     "certificates": f["stats"]["n_certificates"], "fallback": f["stats"]["n_fallback"],
                     "r_predicted": f["stats"]["r_predicted"], "certified": f["cert"]["certified"],
                     "max_distortion": f["cert"]["max_distortion"], "bound_rest": f["cert"]["bound_rest"],
                     "proven_within_eps": proven_within(f["cert"], pr["eps"])}
    out.update(index=index, n=pr["n"], d=pr["d"], eps=pr["eps"])
    return out


def proven_within(cert, eps):
    """The certificate proves max distortion <= eps: its exact maximum when
    complete, else its proven bound over all pairs (near-isometries)."""
    if cert["certified"] == 1:
        return bool(cert["max_distortion"] <= eps)
    return bool(cert["bound_rest"] <= eps)


def summarize(res):
    b = [r["bisect"] for r in res]
    l = [r["learned"] for r in res]
    return {
        "instances": len(res),
        "mean_certificates_plain": float(np.mean([x["certificates"] for x in b])),
        "mean_certificates_learned": float(np.mean([x["certificates"] for x in l])),
        "fit_ms_plain": float(np.sum([x["ms"] for x in b])),
        "fit_ms_learned": float(np.sum([x["ms"] for x in l])),
        "speedup": float(np.sum([x["ms"] for x in b]) / np.sum([x["ms"] for x in l])),
        "fallback_rate": float(np.mean([x["fallback"] for x in l])),
        "mean_r_ratio_learned_over_plain": float(np.mean([x["r"] / y["r"] for x, y in zip(l, b)])),
        "all_proven_within_eps": bool(all(x["proven_within_eps"] for x in l + b)),
        "complete_certificates": float(np.mean([x["certified"] == 1 for x in l])),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("label")
    a.add_argument("--start", type=int, default=0)
    a.add_argument("--stop", type=int, default=4096)
    a.add_argument("--held-out", action="store_true")
    a.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--labels", nargs="+", required=True)
    t.add_argument("--held", nargs="+", required=True)
    t.add_argument("--out", default=PREDICTOR)
    t.add_argument("--epochs", type=int, default=400)
    e = sub.add_parser("evaluate")
    e.add_argument("--predictor", default=PREDICTOR)
    e.add_argument("--start", type=int, default=0)
    e.add_argument("--stop", type=int, default=64)
    e.add_argument("--out", help="write the per-instance results and the summary (JSON)")
    args = ap.parse_args(argv)
    if args.cmd == "label":
        label(range(args.start, args.stop), args.held_out, args.out)
    elif args.cmd == "train":
        lab = merge(args.labels, "/tmp/_labels_merged.npz")
        held = merge(args.held, "/tmp/_held_merged.npz")
        train(lab, held, args.out, epochs=args.epochs)
    else:
        import json
        res = evaluate(args.predictor, range(args.start, args.stop))
        summ = summarize(res)
        if args.out:
            with open(args.out, "w") as f:
                json.dump({"summary": summ, "instances": res}, f)
        print(json.dumps(summ))


def merge(paths, out):
    """Concatenate label files (same keys) into one npz."""
    if len(paths) == 1:
        return paths[0]
    parts = [np.load(p) for p in paths]
    keys = [k for k in parts[0].files if k != "held_out"]
    np.savez(out, held_out=parts[0]["held_out"], **{k: np.concatenate([p[k] for p in parts]) for k in keys})
    return out


if __name__ == "__main__":
    main()
