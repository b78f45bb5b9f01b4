#!/usr/bin/env python3
"""Benchmark of the ADAGIO fit on one MI355X.

A step is one whole fit (centring, FP64 covariance, Jacobi eigensolve, then
the bisection over r with one exact all-pairs certificate per probe) of the
MNIST-shaped synthetic cloud: n = 60000 points in d = 784 dimensions,
eps = 0.1, the input already resident in HBM.

Printed on one line (JSON):
  value       pairs certified per second of fit: n(n-1)/2 / fit time (the
              fit proves the bound for every pair of the cloud; the pair
              evaluations of its screens, n(n-1)/2 per certificate, are
              reported beside it as fit.pair_evaluations_per_s)
  ms_per_step the fit time (the paper's headline quantity: time to an
              embedding whose max distortion is certified <= eps)
  roofline    the all-pairs screen kernel (FP32 MFMA): algorithmic flops
              n(n-1)/2 * 2 (d' + r) per launch (d' = non-constant
              coordinates; 2r when the point Gram is cached) over its
              average launch time from HIP events on the library's stream
  cpu_baseline the FP64 oracle's certificate on this host, on a bounded row
              block of the same workload, in the same unit
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP8_MFMA_TFLOPS = 5000.0
PEAK_BF16_MFMA_TFLOPS = 2500.0
PAIRS_KERNEL_SRC = [os.path.join(ROOT, "paper_1609_05388_amd", "csrc", f) for f in ("k_pairs.hip", "pairs_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pairs_f32_mnist60k_traffic.txt")
MFMA_FILE = os.path.join(ROOT, "profiles", "pairs_f32_mnist60k_mfma_util.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the screen kernel's sources (the traffic figures go stale when they change)."""
    h = hashlib.sha256()
    for path in PAIRS_KERNEL_SRC:
        h.update(open(path, "rb").read())
    return h.hexdigest()


def traffic_per_launch(kind):
    """HBM bytes per screen launch of one kind ("fill": the point-Gram fill
    of a fit; "cached": its certificates' screens) from the committed
    rocprofv3 counter runs, or None when absent or taken on other kernel
    sources."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != source_hash():
        return None
    return rec.get("hbm_bytes_per_launch", {}).get(kind)


def mfma_util(kind):
    """Mean MFMA utilisation (percent, rocprofv3 MfmaUtil) of the screen
    launches of one kind from the committed counter run, or None when absent
    or taken on other kernel sources."""
    try:
        rec = json.load(open(MFMA_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != source_hash():
        return None
    return rec.get("kinds", {}).get(kind, {}).get("mean_mfma_util_pct")


TRAFFIC_KERNEL = "adg::k_pairs_f32<0"
FULL_KERNEL = "adg::k_pairs_f32<0, false>"     # point Gram computed (the fit's cache fill)
CACHED_KERNEL = "adg::k_pairs_f32<0, true>"    # point Gram loaded
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 1 << 30


def per_kernel(path):
    """Counter bytes (KiB x 1024) per dispatch in dispatch order, by kernel name."""
    agg = collections.defaultdict(list)
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
    for r in rows:
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
    return agg


def pick(agg, key):
    return [v for k, vs in agg.items() if key in k for v in vs]


def summarize_traffic(d):
    """HBM bytes per screen launch from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE) of one plain fit and of the 1 GiB copy calibration, each
    counter scaled by the factor that maps its copy reading to 1 GiB.  The
    fit's first screen launch computes and stores the point Gram ("full"),
    the others load it ("cached")."""
    out = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        copy = pick(per_kernel(os.path.join(d, "copy_%s_counter_collection.csv" % c)), COPY_KERNEL)
        agg = per_kernel(os.path.join(d, "fit_%s_counter_collection.csv" % c))
        fill, cached = pick(agg, FULL_KERNEL), pick(agg, CACHED_KERNEL)
        factor = COPY_BYTES / (sum(copy) / len(copy))
        out[c] = {"copy_counter_bytes": sum(copy) / len(copy), "factor": factor,
                  "fill_launch_bytes": sum(fill) / len(fill) * factor,
                  "cached_launch_bytes": (sum(cached) / len(cached) * factor) if cached else None,
                  "launches": len(fill) + len(cached)}
    hb = {"fill": out["FETCH_SIZE"]["fill_launch_bytes"] + out["WRITE_SIZE"]["fill_launch_bytes"]}
    if out["FETCH_SIZE"]["cached_launch_bytes"] is not None:
        hb["cached"] = out["FETCH_SIZE"]["cached_launch_bytes"] + out["WRITE_SIZE"]["cached_launch_bytes"]
    rec = {
        "kernel": TRAFFIC_KERNEL,
        "kernel_source_sha256": source_hash(),
        "hbm_bytes_per_launch": hb,
        "fetch": out["FETCH_SIZE"], "write": out["WRITE_SIZE"],
        "commands": [
            "cd /tmp && TMPDIR=/tmp rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pmc -o copy_FETCH_SIZE -- python3 <repo>/bench.py --calib-copy-mib 1024",
            "cd /tmp && TMPDIR=/tmp rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pmc -o fit_FETCH_SIZE -- python3 <repo>/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-oracle-parity --no-extra-eps --no-forms --no-large --no-knn --no-witness --no-ceiling --learned-instances 0",
            "(the same two with WRITE_SIZE)",
            "python3 <repo>/bench.py --summarize-traffic <out>/pmc",
        ],
        "note": "counter bytes are KiB x 1024 per dispatch; one fit certifying every probe in full (so every "
                "launch is whole): its k_pairs_f32<0, false> launch (the point-Gram fill, no images) and the "
                "mean of its k_pairs_f32<0, true> launches (point Gram loaded, image Gram computed); each counter "
                "is scaled by the factor that maps its reading for a plain 1 GiB copy to 1 GiB",
    }
    print(json.dumps(rec, indent=1))


def host_cpu():
    """The host's CPU model and core counts (lscpu) and the CPUs this
    process may run on."""
    import subprocess
    info = {"model": None, "physical_cores": None, "logical_cpus": None}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name")
        sockets, cps = int(kv.get("Socket(s)", "0") or 0), int(kv.get("Core(s) per socket", "0") or 0)
        info["physical_cores"] = sockets * cps or None
        info["logical_cpus"] = int(kv.get("CPU(s)", "0") or 0) or None
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:
        info["cpus_available"] = len(os.sched_getaffinity(0))
    except OSError:
        info["cpus_available"] = os.cpu_count()
    return info


def rows_for_pairs(n, goal):
    """Smallest m such that rows [0, m) x all j > i hold at least goal pairs."""
    m, acc = 0, 0
    while m < n and acc < goal:
        acc += n - 1 - m
        m += 1
    return max(m, 1)


def cpu_baseline(X, Pi, target_s, n_probes):
    """The oracle, as it stands, on this host: its certificate (C, FP64,
    OpenMP over the host's threads) on rows [0, m) x all j > i of the same
    cloud at the fitted map, m chosen for ~target_s of work, the same on one
    thread for a shorter row block, and its PCA (centre, covariance, eigh).
    In the metric's unit: an oracle fit runs its PCA once and certifies all
    n(n-1)/2 pairs once per probe of its bisection (n_probes of them), so its
    pairs certified per second of fit are n(n-1)/2 / (t_pca + n_probes *
    n(n-1)/2 / pair rate)."""
    import numpy as np
    from oracle import certificate, embedding, pca as opca
    X64 = X.astype(np.float64)
    Y = embedding.embed(X64, Pi)
    n = X.shape[0]
    npairs = n * (n - 1) // 2
    threads = certificate.threads()
    c = certificate.certify(X64, Y, rows=(0, 64))                  # warm-up and rate estimate
    t0 = time.perf_counter()
    c = certificate.certify(X64, Y, rows=(0, 64))
    rate0 = c["n_pairs"] / max(time.perf_counter() - t0, 1e-9)
    m = rows_for_pairs(n, rate0 * target_s)
    t0 = time.perf_counter()
    c = certificate.certify(X64, Y, rows=(0, m))
    dt = time.perf_counter() - t0
    rate = c["n_pairs"] / dt
    # one thread, on a block of ~target_s / 4 of work
    m1 = rows_for_pairs(n, rate / max(threads, 1) * target_s / 4)
    certificate.set_threads(1)
    try:
        t0 = time.perf_counter()
        c1 = certificate.certify(X64, Y, rows=(0, m1))
        dt1 = time.perf_counter() - t0
    finally:
        certificate.set_threads(threads)
    rate1 = c1["n_pairs"] / dt1
    t0 = time.perf_counter()
    opca.pca(X)
    t_pca = time.perf_counter() - t0
    est_fit = t_pca + n_probes * npairs / rate
    return {"value": npairs / est_fit, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "host": host_cpu(), "threads": threads,
            "pair_evaluations_per_s": rate, "pair_evaluations_per_s_1thread": rate1,
            "t_pca_s": t_pca, "certificates_per_fit": n_probes, "est_oracle_fit_s": est_fit,
            "sample": "eq.(3) certificate by FP64 direct differences (oracle/certificate.c, OpenMP, %d threads) "
                      "over rows [0,%d) x all j>i of the same cloud at the fitted r (%d pairs, %.1f s); one thread "
                      "over rows [0,%d) (%d pairs, %.1f s); the oracle's PCA (numpy centre, covariance, eigh) "
                      "%.2f s; value = n(n-1)/2 / (PCA + %d full certificates at the sampled rate)"
                      % (threads, m, c["n_pairs"], dt, m1, c1["n_pairs"], dt1, t_pca, n_probes)}


def oracle_parity(X, plain, forms, torch):
    """The oracle's full eq. (3) certificate of the plain fit's final map
    (every pair, FP64 direct differences) and the error against it of the
    maximum each form certified; a form whose map differs from the plain
    fit's is certified by the oracle separately."""
    import numpy as np
    from oracle import certificate, embedding
    X64 = X.astype(np.float64)
    cache = {}

    def oracle_of(Pi):
        key = Pi.cpu().numpy().tobytes()
        if key not in cache:
            t0 = time.perf_counter()
            w = certificate.certify(X64, embedding.embed(X64, Pi.cpu().numpy().astype(np.float64)))
            cache[key] = (w, time.perf_counter() - t0)
        return cache[key]

    def entry(o):
        w, sec = oracle_of(o["Pi"])
        c = o["cert"]
        gap = w["max"] - w["runner_up"]
        return {"r": o["r"], "max_distortion": c["max_distortion"], "oracle_max": w["max"],
                "abs_err": abs(c["max_distortion"] - w["max"]),
                "argmax": [c["i"], c["j"]], "oracle_argmax": [w["i"], w["j"]],
                "oracle_runner_up_gap": gap,
                "same_argmax": bool((c["i"], c["j"]) == (w["i"], w["j"])), "oracle_s": sec,
                "oracle_pairs": w["n_pairs"]}

    out = {"threads": certificate.threads(), "plain_f32": entry(plain)}
    for name, o in forms.items():
        out[name] = entry(o)
    return out


def c4_oracle_sample(X, Pi, cert, n_blocks, block=1024, seed=4096):
    """The oracle on the large cloud's fitted map, where a full certificate
    (2e10 pairs) is out of reach: every pair of the argmax's and runner-up's
    rows (both directions), the 2048 x 2048 row block holding the argmax
    pair, and n_blocks random block x block row-block pairs."""
    import numpy as np
    from oracle import certificate
    n = X.shape[0]
    t0 = time.perf_counter()
    X64 = X.astype(np.float64)
    Y = X64 @ Pi.astype(np.float64).T
    t_embed = time.perf_counter() - t0
    t0 = time.perf_counter()
    allr = np.arange(n)
    rows = sorted({cert["i"], cert["j"], cert["i2"], cert["j2"]} - {-1})
    pairs, row_best = 0, -1.0
    for row in rows:
        for a, b in ((allr, [row]), ([row], allr)):
            o = certificate.certify_cross(X64, Y, a, b)
            pairs += o["n_pairs"]
            row_best = max(row_best, o["max"])
    a0 = min(max(cert["i"] - 1024, 0), n - 2048)
    b0 = min(max(cert["j"] - 1024, 0), n - 2048)
    blk = certificate.certify_cross(X64, Y, np.arange(a0, a0 + 2048), np.arange(b0, b0 + 2048))
    pairs += blk["n_pairs"]
    rng = np.random.default_rng(seed)
    top = max(row_best, blk["max"])
    for _ in range(n_blocks):
        a, b = np.sort(rng.integers(0, n - block, 2))
        o = certificate.certify_cross(X64, Y, np.arange(a, a + block), np.arange(b, b + block))
        pairs += o["n_pairs"]
        top = max(top, o["max"])
    dt = time.perf_counter() - t0
    return {"pairs": pairs, "seconds": dt, "embed_s": t_embed, "threads": certificate.threads(),
            "rows": rows, "random_blocks": n_blocks, "block_rows": block,
            "largest_sampled": top, "argmax_rows_largest": row_best,
            "argmax_block_max": blk["max"], "argmax_block_argmax": [blk["i"], blk["j"]],
            "reproduces_certified_max": bool(abs(row_best - cert["max_distortion"]) <= 1e-12
                                             and (blk["i"], blk["j"]) == (cert["i"], cert["j"])),
            "none_above_certified": bool(top <= cert["max_distortion"] + 1e-12),
            "sample": "oracle/certificate.c on the fitted map: every pair of rows %s against all rows, the 2048 x "
                      "2048 row block holding the argmax pair, %d random %d x %d row-block pairs"
                      % (rows, n_blocks, block, block)}


def nonconstant_columns(X):
    """Coordinates that are not constant over the cloud: the point Gram's
    algorithmic width (a constant coordinate centres to exact zeros and adds
    nothing to any distance; the library's screens leave it out)."""
    return int((X.max(axis=0) != X.min(axis=0)).sum())


def screen_flops(npairs, d, cols, gram):
    """Algorithmic flops of one screen launch: both Grams (2(d + cols) per
    pair, d = non-constant coordinates), or the image Gram only (2 cols) when
    the point Gram came from the cache; cols = the image columns the screen
    ran over (r, or d when a map of more rows went through the Gram factor)."""
    return npairs * 2.0 * (cols if gram == 2 else d + cols)


def split_probes(st):
    """A fit's logged probes as (screened, rigorous, refuted) lists of
    (r, delta, screen_ms, gram, cols): the first n_screened probes that ran a
    screen were FP8 screens; gram 3 and 4 mark probes refuted by a witness
    pair."""
    fp8, rig, ref = [], [], []
    for p in zip(st["probe_r"], st["probe_delta"], st["probe_screen_ms"], st["probe_gram"], st["probe_cols"]):
        if p[3] in (3, 4):
            ref.append(p)
        elif len(fp8) < st["n_screened"]:
            fp8.append(p)
        else:
            rig.append(p)
    return fp8, rig, ref


def timed_fits(adagio, torch, Xd, eps, seed, steps, **kw):
    adagio.fit(Xd, eps, seed, **kw)             # buffers and first-call set-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [adagio.fit(Xd, eps, seed, **kw) for _ in range(steps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, outs


def fp8_form(adagio, gen, torch, Xd, eps, steps, plain_s, plain, npairs, d):
    """Fit whose bisection decides on FP8 screens, then certifies its result
    with the BF16 split screen."""
    fs, outs = timed_fits(adagio, torch, Xd, eps, gen.JL_SEED, steps, screen="fp8")
    o = outs[-1]
    st = o["stats"]
    scr, _, ref = split_probes(st)
    fl = sum(screen_flops(npairs, d, c, g) for _, _, _, g, c in scr)
    ms = sum(t for _, _, t, _, _ in scr)
    return o, {"fit_ms": fs * 1e3, "speedup_vs_plain": plain_s / fs, "r": o["r"],
            "max_distortion": o["cert"]["max_distortion"], "certified": o["cert"]["certified"],
            "abs_err_vs_plain_f32_fit": abs(o["cert"]["max_distortion"] - plain["cert"]["max_distortion"]),
            "same_map_as_plain": bool(o["r"] == plain["r"] and torch.equal(o["Pi"], plain["Pi"])),
            "screens": st["n_screened"], "certificates": st["n_certificates"] - st["n_screened"],
            "refuted_probes": st["n_refuted"],
            "screen_probes": [[r, dl] for r, dl, _, _, _ in scr],
            "screen_avg_launch_ms": ms / max(1, len(scr)),
            "screen_fp8_mfma_tflops": fl / max(ms, 1e-9) / 1e9,
            "screen_fp8_mfma_frac": fl / max(ms, 1e-9) / 1e9 / PEAK_FP8_MFMA_TFLOPS}


def learned_form(adagio, gen, torch, Xd, eps, steps, plain_s, plain):
    """Fit from the trained predictor's r (certified, bisection fallback),
    with exact PCA and with the randomized PCA for the predicted s, on the
    MNIST-shaped cloud: outside the predictor's training range (n <= 20000),
    so r there says nothing about the learned form's accuracy."""
    from paper_1609_05388_amd import learned
    if not os.path.exists(learned.PREDICTOR):
        return None
    P = learned.load_predictor(learned.PREDICTOR)
    fs, outs = timed_fits(adagio, torch, Xd, eps, gen.JL_SEED, steps, search="learned", predictor=P)
    o = outs[-1]
    rs, routs = timed_fits(adagio, torch, Xd, eps, gen.JL_SEED, steps, search="learned", predictor=P,
                           pca="randomized", pca_iters=2)
    ro = routs[-1]
    return {"fit_ms": fs * 1e3, "speedup_vs_plain": plain_s / fs, "r": o["r"], "r_plain": plain["r"],
            "r_predicted": o["stats"]["r_predicted"], "fallback": o["stats"]["n_fallback"],
            "certificates": o["stats"]["n_certificates"], "max_distortion": o["cert"]["max_distortion"],
            "certified": o["cert"]["certified"],
            "with_randomized_pca": {"fit_ms": rs * 1e3, "speedup_vs_plain": plain_s / rs, "r": ro["r"],
                                    "max_distortion": ro["cert"]["max_distortion"],
                                    "certified": ro["cert"]["certified"]}}


def learned_heldout(adagio, gen, torch, count):
    """The learned form where it is defined: the first `count` held-out
    instances of the learned-form workload (n in [1000, 20000], d in
    {128, 256, 784, 2048}, power-law spectra, eps in [0.05, 0.3]; never seen
    in training).  Per instance plain bisection, the learned search
    (certified prediction, bisection fallback) and the learned search with
    downward refinement, each run once as a warm-up (which sizes the kept
    workspace's buffers for that search, as the 512-instance evaluation does)
    and then timed twice, the faster time counting (a single timing of a fit
    of a few ms picks up host-side stalls of tens of ms now and then; FP32
    screen)."""
    import numpy as np
    from paper_1609_05388_amd import learned
    if not os.path.exists(learned.PREDICTOR):
        return None
    P = learned.load_predictor(learned.PREDICTOR)
    modes = (("plain", {}), ("learned", {"search": "learned", "predictor": P}),
             ("learned_refine", {"search": "learned", "predictor": P, "refine": True}),
             ("learned_refine_within4", {"search": "learned", "predictor": P, "refine": "within4"}))
    rows = []
    t0 = time.perf_counter()
    for index, pr, X in learned.instances(list(range(count)), held_out=True):
        Xd = torch.from_numpy(X).cuda()
        row = {"index": index, "n": pr["n"], "d": pr["d"], "eps": pr["eps"]}
        for name, kw in modes:
            adagio.fit(Xd, pr["eps"], gen.JL_SEED, **kw)
            best = None
            for _ in range(2):
                torch.cuda.synchronize()
                ta = time.perf_counter()
                o = adagio.fit(Xd, pr["eps"], gen.JL_SEED, **kw)
                torch.cuda.synchronize()
                t = (time.perf_counter() - ta) * 1e3
                best = t if best is None else min(best, t)
            c = o["cert"]
            row[name] = {"ms": best, "r": o["r"],
                         "certificates": o["stats"]["n_certificates"], "fallback": o["stats"]["n_fallback"],
                         "r_predicted": o["stats"]["r_predicted"],
                         "proven": bool(c["max_distortion"] <= pr["eps"] if c["certified"] == 1
                                        else c["bound_rest"] <= pr["eps"]),
                         "t_pca_ms": o["stats"]["t_pca_ms"]}
        rows.append(row)
        del Xd
    out = {"instances": len(rows), "seconds": time.perf_counter() - t0, "screen": "f32",
           "d_counts": {str(d): sum(1 for r in rows if r["d"] == d) for d in (128, 256, 784, 2048)},
           "workload": "held-out learned-form instances 0..%d (n U{1000..20000}, d in {128, 256, 784, 2048}, "
                       "power-law spectrum exponent U[0.5, 2] at rank U{10..200}, noise 0.01, eps U[0.05, 0.3])"
                       % (count - 1)}
    plain_ms = sum(r["plain"]["ms"] for r in rows)
    for name, _ in modes:
        ms = sum(r[name]["ms"] for r in rows)
        out[name] = {"fit_ms_total": ms, "speedup_vs_plain": plain_ms / ms,
                     "mean_certificates": float(np.mean([r[name]["certificates"] for r in rows])),
                     "mean_pca_ms": float(np.mean([r[name]["t_pca_ms"] for r in rows])),
                     "fallback_rate": float(np.mean([r[name]["fallback"] for r in rows])),
                     "mean_r_over_plain": float(np.mean([r[name]["r"] / r["plain"]["r"] for r in rows])),
                     "max_r_over_plain": float(max(r[name]["r"] / r["plain"]["r"] for r in rows)),
                     "same_r_as_plain": float(np.mean([r[name]["r"] == r["plain"]["r"] for r in rows])),
                     "all_proven_within_eps": bool(all(r[name]["proven"] for r in rows))}
    log("learned held-out (%d instances): learned %.2fx (r %.3f), refined %.2fx (r %.3f), "
        "refined within 4%% %.2fx (r %.3f)" % (
            len(rows), out["learned"]["speedup_vs_plain"], out["learned"]["mean_r_over_plain"],
            out["learned_refine"]["speedup_vs_plain"], out["learned_refine"]["mean_r_over_plain"],
            out["learned_refine_within4"]["speedup_vs_plain"], out["learned_refine_within4"]["mean_r_over_plain"]))
    out["per_instance"] = [[r["index"], r["n"], r["d"], round(r["eps"], 4), r["plain"]["r"], r["learned"]["r"],
                            r["learned_refine"]["r"], r["learned_refine_within4"]["r"], round(r["plain"]["ms"], 2),
                            round(r["learned"]["ms"], 2), round(r["learned_refine"]["ms"], 2),
                            round(r["learned_refine_within4"]["ms"], 2)] for r in rows]
    out["per_instance_columns"] = ["index", "n", "d", "eps", "r_plain", "r_learned", "r_refined",
                                   "r_refined_within4", "ms_plain", "ms_learned", "ms_refined",
                                   "ms_refined_within4"]
    return out


def large_form(adagio, gen, torch, eps, oracle_blocks):
    """Precision form at scale: the power-law cloud n=200000, d=4096 (rank 512,
    sigma_i = 1/i, noise 0.01), fit with FP8-screened bisection and a BF16
    split certificate of the result; the plain FP32 certificate of the same
    map is timed once beside it."""
    t0 = time.perf_counter()
    X = gen.power_law(200000, 4096, 512, 1.0, noise=0.01)
    gen_s = time.perf_counter() - t0
    dx = nonconstant_columns(X)
    Xd = torch.from_numpy(X).cuda()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    o = adagio.fit(Xd, eps, gen.JL_SEED, screen="fp8")
    torch.cuda.synchronize()
    fit_ms = (time.perf_counter() - ta) * 1e3
    st = o["stats"]
    n, d = Xd.shape
    npairs = n * (n - 1) // 2
    scr = list(zip(st["probe_r"], st["probe_delta"], st["probe_screen_ms"], st["probe_gram"]))
    fp8, rig, ref = split_probes(st)
    fl = sum(screen_flops(npairs, dx, c, g) for _, _, _, g, c in fp8)
    ms = sum(t for _, _, t, _, _ in fp8)
    bfl = sum(screen_flops(npairs, dx, c, g) for _, _, _, g, c in rig)
    bms = sum(t for _, _, t, _, _ in rig)
    same_r = [dl for r, dl, _, _, _ in fp8 if r == o["r"]]
    plain = adagio.certify_map(Xd, o["Pi"].contiguous(), screen="f32", with_stats=True)
    pst = plain.pop("stats")
    torch.cuda.synchronize()
    tr = time.perf_counter()
    ro = adagio.fit(Xd, eps, gen.JL_SEED, screen="fp8", pca="randomized", pca_iters=2)
    torch.cuda.synchronize()
    rand = {"fit_ms": (time.perf_counter() - tr) * 1e3, "r": ro["r"], "max_distortion": ro["cert"]["max_distortion"],
            "certified": ro["cert"]["certified"], "power_iterations": 2, "oversampling": 10}
    del Xd
    torch.cuda.empty_cache()
    sample = None
    if oracle_blocks >= 0:
        log("large: oracle sample of the fitted map")
        sample = c4_oracle_sample(X, o["Pi"].cpu().numpy(), o["cert"], oracle_blocks)
        log("large: oracle checked %d pairs in %.1f s, largest %.9f, reproduces the max: %s"
            % (sample["pairs"], sample["seconds"], sample["largest_sampled"], sample["reproduces_certified_max"]))
    del X
    return {
        "workload": "power-law cloud n=200000, d=4096, rank 512, sigma_i=1/i, noise 0.01, eps=%g" % eps,
        "oracle_sample": sample,
        "generate_s": gen_s, "fit_ms": fit_ms, "t_pca_ms": st["t_pca_ms"], "eig_sweeps": st["eig_sweeps"],
        "r": o["r"], "max_distortion": o["cert"]["max_distortion"], "certified": o["cert"]["certified"],
        "argmax": [o["cert"]["i"], o["cert"]["j"]],
        "fp8_screens": len(fp8), "bf16x3_certificates": len(rig), "refuted_probes": len(ref),
        "fp8_screen_avg_ms": ms / max(1, len(fp8)),
        "fp8_screen_tflops": fl / max(ms, 1e-9) / 1e9,
        "fp8_screen_frac_of_fp8_peak": fl / max(ms, 1e-9) / 1e9 / PEAK_FP8_MFMA_TFLOPS,
        "bf16x3_screen_avg_ms": bms / max(1, len(rig)),
        "bf16x3_screen_useful_tflops": bfl / max(bms, 1e-9) / 1e9,
        "fp8_error_vs_certificate_at_r": (abs(same_r[-1] - o["cert"]["max_distortion"]) if same_r else None),
        "fp32_certificate_of_same_map": {"ms": pst["t_total_ms"], "screen_ms": pst["t_screen_ms"],
                                         "screen_tflops": npairs * 2.0 * (dx + o["r"]) / pst["t_screen_ms"] / 1e9,
                                         "max_distortion": plain["max_distortion"],
                                         "certified": plain["certified"]},
        "probes": [[r, dl, "refuted" if g in (3, 4) else "screened"] for r, dl, _, g in scr],
        "with_randomized_pca": rand,
    }


def knn_form(adagio, gen, torch, rs=(128, 64, 32, 24, 20, 16, 12, 8, 4)):
    """Sec. 4.6's image retrieval on the SIFT-shaped workload (201 objects, a
    402,000 x 128 database of 4 photos x 500 descriptors each, 20,100 query
    descriptors of one photo per object): at each target dimension r the
    ADAGIO map of the database and, beside it, the PCA-only map (both from
    the PCA of the database; r = 128 = no reduction), the embedding of
    database and queries, exact 10-NN of every query, the
    majority vote per query photo and its accuracy; also the 30-NN graph of
    50,000 database rows.  The screen's roofline is taken at r = 128."""
    import numpy as np
    D, dl, Q, qi = gen.sift_shaped()
    nb = int(qi.max()) + 1
    per_q = len(Q) // nb
    Dd, Qd = torch.from_numpy(D).cuda(), torch.from_numpy(Q).cuda()
    dld = torch.from_numpy(dl).cuda()
    lam, Vt = adagio.pca(Dd)
    adagio.knn(Qd, Dd, 10)                       # warm-up of the workspace
    rows = []
    roof = None
    for r, fam in [(r, f) for r in rs for f in (("none",) if r >= D.shape[1] else ("adagio", "pca"))]:
        if fam == "none":
            YD, YQ = Dd, Qd
        else:
            Pi = adagio.project_family(Vt, r, fam, gen.JL_SEED)
            YD, YQ = adagio.embed(Dd, Pi), adagio.embed(Qd, Pi)
        torch.cuda.synchronize()
        best = None
        for _ in range(2):
            ta = time.perf_counter()
            idx, dist, st = adagio.knn(YQ, YD, 10)
            torch.cuda.synchronize()
            t = (time.perf_counter() - ta) * 1e3
            if best is None or t < best[0]:
                best = (t, st)
        pred = adagio.knn_vote(idx, dld, nb, per_q).cpu().numpy()
        acc = float((pred == np.arange(nb)).mean())
        t, st = best
        rows.append({"r": r, "map": fam, "knn_ms": t, "screen_ms": st["t_screen_ms"], "finish_ms": st["t_finish_ms"],
                     "fallback_ms": st["t_fallback_ms"], "n_fallback": st["n_fallback"], "accuracy": acc,
                     "correct": int((pred == np.arange(nb)).sum()), "splits": st["splits"]})
        log("knn r=%d %s: %.2f ms (screen %.2f), accuracy %.3f, fallbacks %d" % (r, fam, t, st["t_screen_ms"], acc,
                                                                                 st["n_fallback"]))
        if r == rs[0]:
            fl = 2.0 * D.shape[1] * len(Q) * len(D)
            roof = {"kernel": "k_knn_screen", "m": D.shape[1], "flops_per_launch": fl,
                    "avg_launch_ms": st["t_screen_ms"], "tflops": fl / st["t_screen_ms"] / 1e9,
                    "frac": fl / st["t_screen_ms"] / 1e9 / PEAK_FP32_MFMA_TFLOPS}
    graph = []
    G = Dd[:50000].contiguous()
    for r in (128, 24):
        Y = G if r >= D.shape[1] else adagio.embed(G, adagio.project_axes(Vt, r, gen.JL_SEED))
        adagio.knn(Y, Y, 30, exclude_self=True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        _, _, st = adagio.knn(Y, Y, 30, exclude_self=True)
        torch.cuda.synchronize()
        graph.append({"r": r, "n": 50000, "k": 30, "ms": (time.perf_counter() - ta) * 1e3,
                      "screen_ms": st["t_screen_ms"], "n_fallback": st["n_fallback"]})
    del Dd, Qd, G
    torch.cuda.empty_cache()
    return {"workload": "SIFT-shaped retrieval: 201 objects, database 402000 x 128, 20100 queries, k=10",
            "per_r": rows, "screen_roofline_r128": roof, "knn_graph": graph}


def summarize_mfma(d):
    """MFMA utilisation of the screen kernel from one rocprofv3 --pmc run of
    one plain fit certifying every probe in full (derived counters MfmaUtil =
    SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs) and MfmaFlopsF32 =
    512 x SQ_INSTS_VALU_MFMA_MOPS_F32), per launch kind, beside the
    algorithmic flops of the same launches."""
    rows = sorted(csv.DictReader(open(os.path.join(d, "fit_mfma_counter_collection.csv"))),
                  key=lambda r: int(r["Dispatch_Id"]))
    per = collections.defaultdict(dict)
    for r in rows:
        per[(int(r["Dispatch_Id"]), r["Kernel_Name"])][r["Counter_Name"]] = float(r["Counter_Value"])
    fit = [json.loads(l) for l in open(os.path.join(d, "fit_mfma.log")) if l.startswith("{")][-1]
    n, dx = fit["config"]["n"], fit["config"]["d_nonconstant"]
    npairs = n * (n - 1) // 2
    rs = [p[0] for p in fit["fit"]["probes"]]
    cols = [p[3] if len(p) > 3 else p[0] for p in fit["fit"]["probes"]]   # the screens' image columns
    out = {}
    for kind, key in (("fill", FULL_KERNEL), ("cached", CACHED_KERNEL)):
        ds = [v for (i, k), v in sorted(per.items()) if key in k]
        if kind == "cached":      # each fit's screens in probe order (the run may hold several fits)
            alg = [npairs * 2.0 * cols[i % len(cols)] for i in range(len(ds))]
        else:
            alg = [npairs * 2.0 * dx for _ in ds]
        util = [v["MfmaUtil"] for v in ds]
        hw = [v["MfmaFlopsF32"] for v in ds]
        out[kind] = {"launches": len(ds), "mfma_util_pct": util, "mean_mfma_util_pct": sum(util) / len(util),
                     "hw_mfma_flops": hw, "algorithmic_flops": alg[:len(hw)],
                     "algorithmic_over_hw": sum(alg[:len(hw)]) / sum(hw)}
    rec = {
        "kernel": TRAFFIC_KERNEL,
        "kernel_source_sha256": source_hash(),
        "workload": fit["config"]["workload"], "probes_r": rs, "probes_screen_cols": cols,
        "kinds": out,
        "commands": [
            "cd /tmp && TMPDIR=/tmp rocprofv3 --pmc MfmaUtil MfmaFlopsF32 --output-format csv -d <out>/mfma -o fit_mfma -- python3 <repo>/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-oracle-parity --no-extra-eps --no-forms --no-large --no-knn --no-witness --no-ceiling --learned-instances 0 > <out>/mfma/fit_mfma.log",
            "python3 <repo>/bench.py --summarize-mfma <out>/mfma",
        ],
        "note": "MfmaUtil: percent of the dispatch's GPU-active cycles during which the SIMDs' MFMA units were busy "
                "(SQ_VALU_MFMA_BUSY_CYCLES summed over SIMDs / (GRBM_GUI_ACTIVE x 1024)); MfmaFlopsF32: FP32 MFMA "
                "flops executed (MOPS x 512), which include the padded rows and columns and the masked halves of "
                "the diagonal tiles that the algorithmic count leaves out",
    }
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--n", type=int, default=60000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-parity", action="store_true",
                    help="skip the oracle's full certificate of the fitted map (about 45 s on 16 threads)")
    ap.add_argument("--c4-oracle-blocks", type=int, default=16,
                    help="random 1024 x 1024 row-block pairs the oracle checks on the large cloud (-1: none)")
    ap.add_argument("--no-extra-eps", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision-form fits")
    ap.add_argument("--no-large", action="store_true", help="skip the n=200000, d=4096 precision-form fit")
    ap.add_argument("--no-knn", action="store_true", help="skip the kNN retrieval application")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the MFMA-only kernels that measure the matrix cores' attainable rate")
    ap.add_argument("--learned-instances", type=int, default=64,
                    help="held-out learned-form instances for the learned search's gain (0: none)")
    ap.add_argument("--no-witness", action="store_true",
                    help="plain fits certify every probe in full (every screen launch whole: the counter runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--summarize-mfma", metavar="PMC_DIR",
                    help="print the MFMA-utilisation summary of a rocprofv3 MfmaUtil/MfmaFlopsF32 run")
    ap.add_argument("--summarize-traffic", metavar="PMC_DIR",
                    help="print the traffic summary of rocprofv3 --pmc runs in PMC_DIR and exit")
    args = ap.parse_args()

    if args.summarize_mfma:
        summarize_mfma(args.summarize_mfma)
        return
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1609_05388_amd import adagio, gen

    if args.calib_copy_mib:
        nel = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written per copy" % (nel * 4, nel * 4))
        return

    adagio.load()
    # a loop of fits keeps the library's workspace across calls (the opt-in
    # adagio_keep_workspace; the library default allocates per call: timed
    # below beside it)
    adagio.keep_workspace(True)
    log("generating MNIST-shaped cloud n=%d" % args.n)
    X = gen.mnist_shaped(n=args.n)
    n, d = X.shape
    dx = nonconstant_columns(X)
    Xd = torch.from_numpy(X).cuda()
    torch.cuda.synchronize()

    wit = not args.no_witness
    for w in range(args.warmup):
        out = adagio.fit(Xd, args.eps, gen.JL_SEED, witness=wit)
        log("warmup %d: r=%d fit %.1f ms" % (w, out["r"], out["stats"]["t_total_ms"]))
    torch.cuda.synchronize()

    outs = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        outs.append(adagio.fit(Xd, args.eps, gen.JL_SEED, witness=wit))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fit_s = (t1 - t0) / args.steps
    last = outs[-1]
    st = last["stats"]
    npairs = n * (n - 1) // 2
    ncert = st["n_certificates"]
    value = npairs / fit_s
    log("fit %.1f ms/step: r=%d, %d certificates, %d probes refuted, delta=%.6f, pca %.1f ms, search %.1f ms, "
        "screen %.1f ms" % (fit_s * 1e3, last["r"], ncert, st["n_refuted"], last["cert"]["max_distortion"],
                            st["t_pca_ms"], st["t_search_ms"], st["t_screen_ms"]))

    # the same fits with the library default: every call allocates its
    # workspace (the 7.2 GB point-Gram cache among it) and frees it
    adagio.keep_workspace(False)
    pc_s, pc_outs = timed_fits(adagio, torch, Xd, args.eps, gen.JL_SEED, args.steps, witness=wit)
    adagio.keep_workspace(True)
    per_call = {"fit_ms": pc_s * 1e3, "slowdown_vs_kept_workspace": pc_s / fit_s,
                "same_result": bool(pc_outs[-1]["r"] == last["r"] and torch.equal(pc_outs[-1]["Pi"], last["Pi"])
                                    and pc_outs[-1]["cert"] == last["cert"])}
    log("per-call workspace: fit %.1f ms" % (pc_s * 1e3))

    # the same fit certifying every probe in full (no witness pool, no early stop)
    without_witness = None
    if wit:
        nw_s, nw_outs = timed_fits(adagio, torch, Xd, args.eps, gen.JL_SEED, args.steps, witness=False)
        nw = nw_outs[-1]
        without_witness = {"fit_ms": nw_s * 1e3, "certificates": nw["stats"]["n_certificates"],
                           "same_result": bool(nw["r"] == last["r"] and torch.equal(nw["Pi"], last["Pi"])
                                               and nw["cert"] == last["cert"]),
                           "pair_evaluations_per_s": npairs * nw["stats"]["n_certificates"] / nw_s}
        log("without witnesses: fit %.1f ms, %d certificates" % (nw_s * 1e3, without_witness["certificates"]))

    # roofline of the screen kernel over the launches of the timed steps.  A
    # fit fills the point-Gram cache once (2 d' flops per pair, d' non-constant
    # coordinates; on a second stream during the PCA); its certificates load it
    # and compute the image Gram (2r flops per pair).  Without the cache a
    # screen computes both (2(d' + r)).
    kinds = {"fill": [0.0, 0.0, 0], "full": [0.0, 0.0, 0], "cached": [0.0, 0.0, 0]}
    for o in outs:
        s = o["stats"]
        if s["t_gram_ms"] > 0:  # the point-Gram fill: 2 d' flops per pair, overlapping the PCA
            kinds["fill"][0] += npairs * 2.0 * dx
            kinds["fill"][1] += s["t_gram_ms"]
            kinds["fill"][2] += 1
        for c, t, g in zip(s["probe_cols"], s["probe_screen_ms"], s["probe_gram"]):
            if g in (3, 4):     # refuted by a witness pair: no screen, or one stopped early
                continue
            k = "cached" if g == 2 else "full"
            kinds[k][0] += screen_flops(npairs, dx, c, g)
            kinds[k][1] += t
            kinds[k][2] += 1
    launch_kinds = {}
    for k, (fl, ms, nl) in kinds.items():
        if nl:
            launch_kinds[k] = {"launches": nl, "avg_launch_ms": ms / nl, "flops_per_launch": fl / nl,
                               "tflops": fl / ms / 1e9, "frac": fl / ms / 1e9 / PEAK_FP32_MFMA_TFLOPS}
    dom = max(launch_kinds, key=lambda k: kinds[k][1])
    traffic = traffic_per_launch(dom)
    roofline = {"bound": "mfma", "achieved": launch_kinds[dom]["tflops"], "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": launch_kinds[dom]["frac"], "traffic": traffic,
                "mfma_util_rocprof_pct": mfma_util(dom),
                "kernel": "k_pairs_f32<0, %s> (all-pairs screen), %s launches" % ("true" if dom == "cached" else "false",
                                                                                    dom),
                "launches": launch_kinds[dom]["launches"], "avg_launch_ms": launch_kinds[dom]["avg_launch_ms"],
                "flops_per_launch": launch_kinds[dom]["flops_per_launch"], "launch_kinds": launch_kinds}

    # precision form: BF16 split screen, same exact certificate
    forms = {}
    form_outs = {}
    if not args.no_forms:
        torch.cuda.synchronize()
        bf = adagio.fit(Xd, args.eps, gen.JL_SEED, screen="bf16x3")  # warm-up of its buffers
        torch.cuda.synchronize()
        tb = time.perf_counter()
        bouts = [adagio.fit(Xd, args.eps, gen.JL_SEED, screen="bf16x3") for _ in range(args.steps)]
        torch.cuda.synchronize()
        bf_s = (time.perf_counter() - tb) / args.steps
        bl = bouts[-1]
        bflops, bms, bn = 0.0, 0.0, 0
        for o in bouts:
            for c, t, g in zip(o["stats"]["probe_cols"], o["stats"]["probe_screen_ms"], o["stats"]["probe_gram"]):
                if g in (3, 4):
                    continue
                bflops += screen_flops(npairs, dx, c, g)
                bms += t
                bn += 1
        forms["bf16x3"] = {
            "fit_ms": bf_s * 1e3, "speedup_vs_plain": fit_s / bf_s, "r": bl["r"],
            "max_distortion": bl["cert"]["max_distortion"], "certified": bl["cert"]["certified"],
            "abs_err_vs_plain_f32_fit": abs(bl["cert"]["max_distortion"] - last["cert"]["max_distortion"]),
            "same_map_as_plain": bool(bl["r"] == last["r"] and torch.equal(bl["Pi"], last["Pi"])),
            "screen_avg_launch_ms": bms / bn,
            "screen_useful_tflops": bflops / bms / 1e9,
            "screen_bf16_mfma_tflops": 3.0 * bflops / bms / 1e9,
            "screen_bf16_mfma_frac": 3.0 * bflops / bms / 1e9 / PEAK_BF16_MFMA_TFLOPS,
            "rescored_pairs": bl["stats"]["n_rescored"], "flagged_tiles": bl["stats"]["n_flagged_tiles"]}
        log("bf16x3 fit %.1f ms (%.2fx), screen %.2f ms/launch" % (bf_s * 1e3, fit_s / bf_s, bms / bn))
        fp8_last, forms["fp8"] = fp8_form(adagio, gen, torch, Xd, args.eps, args.steps, fit_s, last, npairs, dx)
        form_outs = {"bf16x3": bl, "fp8": fp8_last}
        log("fp8 fit %.1f ms (%.2fx)" % (forms["fp8"]["fit_ms"], forms["fp8"]["speedup_vs_plain"]))
        rs, routs = timed_fits(adagio, torch, Xd, args.eps, gen.JL_SEED, args.steps, pca="randomized", pca_iters=2)
        ro = routs[-1]
        forms["randomized_pca"] = {"fit_ms": rs * 1e3, "speedup_vs_plain": fit_s / rs, "r": ro["r"],
                                   "r_exact_pca": last["r"], "max_distortion": ro["cert"]["max_distortion"],
                                   "certified": ro["cert"]["certified"], "power_iterations": 2,
                                   "oversampling": 10}
        log("randomized-PCA fit %.1f ms (%.2fx), r=%d" % (rs * 1e3, fit_s / rs, ro["r"]))
        lf = learned_form(adagio, gen, torch, Xd, args.eps, args.steps, fit_s, last)
        if lf:
            forms["learned_out_of_distribution"] = lf
            log("learned fit (out of distribution) %.1f ms (%.2fx)" % (lf["fit_ms"], lf["speedup_vs_plain"]))
        if args.learned_instances > 0:
            lh = learned_heldout(adagio, gen, torch, args.learned_instances)
            if lh:
                forms["learned_heldout"] = lh

    parity = None
    if not args.no_oracle_parity:
        log("oracle: full eq. (3) certificate of the fit's map (%d pairs)" % npairs)
        parity = oracle_parity(X, last, form_outs, torch)
        for k in form_outs:
            forms[k]["abs_err_vs_oracle"] = parity[k]["abs_err"]
        log("oracle max %.9f in %.1f s; |err| plain %.2e%s" % (
            parity["plain_f32"]["oracle_max"], parity["plain_f32"]["oracle_s"], parity["plain_f32"]["abs_err"],
            "".join(", %s %.2e" % (k, parity[k]["abs_err"]) for k in form_outs)))

    extra = {}
    if not args.no_extra_eps:
        for e in (0.05, 0.2):
            if abs(e - args.eps) < 1e-12:
                continue
            torch.cuda.synchronize()
            ta = time.perf_counter()
            o = adagio.fit(Xd, e, gen.JL_SEED)
            torch.cuda.synchronize()
            extra[str(e)] = {"r": o["r"], "fit_ms": (time.perf_counter() - ta) * 1e3,
                             "max_distortion": o["cert"]["max_distortion"],
                             "certificates": o["stats"]["n_certificates"]}

    # The stand-in has 549 always-zero coordinates; real MNIST's 60000 training
    # images have 67.  The same fit on a cloud with 67 constant coordinates
    # shows what the constant-coordinate splits are worth there.
    border67 = None
    if not args.no_extra_eps:
        X67 = gen.mnist_shaped(n=n, active=d - 67)
        X67d = torch.from_numpy(X67).cuda()
        adagio.fit(X67d, args.eps, gen.JL_SEED)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        o = adagio.fit(X67d, args.eps, gen.JL_SEED)
        torch.cuda.synchronize()
        border67 = {"constant_coordinates": d - nonconstant_columns(X67), "fit_ms": (time.perf_counter() - ta) * 1e3,
                    "r": o["r"], "t_pca_ms": o["stats"]["t_pca_ms"], "certificates": o["stats"]["n_certificates"],
                    "max_distortion": o["cert"]["max_distortion"], "certified": o["cert"]["certified"]}
        log("67 constant coordinates: fit %.1f ms, r=%d" % (border67["fit_ms"], o["r"]))
        del X67d

    # Table 3 (Sec. 4.4) / Fig. 6 (Sec. 4.3) analogue: the smallest certified r of each map family per eps
    tradeoff = {}
    if not args.no_extra_eps:
        for fam in ("adagio", "pca", "jl"):
            tradeoff[fam] = {}
            for e in (0.05, 0.1, 0.2):
                torch.cuda.synchronize()
                ta = time.perf_counter()
                o = adagio.fit(Xd, e, gen.JL_SEED, family=fam)
                torch.cuda.synchronize()
                tradeoff[fam][str(e)] = {"r": o["r"], "fit_ms": (time.perf_counter() - ta) * 1e3,
                                         "max_distortion": o["cert"]["max_distortion"],
                                         "certified": o["cert"]["certified"]}
        log("tradeoff r: " + ", ".join("%s %s" % (f, [v["r"] for v in tradeoff[f].values()]) for f in tradeoff))

    large = None
    if not args.no_large:
        log("precision form at n=200000, d=4096")
        large = large_form(adagio, gen, torch, args.eps, args.c4_oracle_blocks)
        log("large: fp8 fit %.0f ms, r=%d, delta=%.6f" % (large["fit_ms"], large["r"], large["max_distortion"]))

    knn = None
    if not args.no_knn:
        log("kNN retrieval on the SIFT-shaped workload")
        knn = knn_form(adagio, gen, torch)

    # The matrix cores' attainable rate: kernels of independent MFMAs only,
    # under which the shader clock settles below the 2.4 GHz that the
    # published peaks assume; context for the fractions of peak above.
    ceil = None
    if not args.no_ceiling:
        ceil = {k: adagio.mfma_ceiling(k) for k in ("fp32", "bf16", "fp8")}
        for k, v in ceil.items():
            v["frac_of_peak"] = v["tflops"] / {"fp32": PEAK_FP32_MFMA_TFLOPS, "bf16": PEAK_BF16_MFMA_TFLOPS,
                                               "fp8": PEAK_FP8_MFMA_TFLOPS}[k]
        roofline["attainable"] = ceil["fp32"]["tflops"]
        roofline["frac_of_attainable"] = roofline["achieved"] / ceil["fp32"]["tflops"]
        if "bf16x3" in forms:
            f = forms["bf16x3"]
            f["screen_bf16_mfma_frac_of_attainable"] = f["screen_bf16_mfma_tflops"] / ceil["bf16"]["tflops"]
        if "fp8" in forms:
            f = forms["fp8"]
            f["screen_fp8_mfma_frac_of_attainable"] = f["screen_fp8_mfma_tflops"] / ceil["fp8"]["tflops"]
        if large:
            large["fp8_screen_frac_of_attainable"] = large["fp8_screen_tflops"] / ceil["fp8"]["tflops"]
            large["bf16x3_screen_mfma_frac_of_attainable"] = (3.0 * large["bf16x3_screen_useful_tflops"]
                                                              / ceil["bf16"]["tflops"])
        log("MFMA-only ceilings: " + ", ".join("%s %.0f TFLOP/s (%.2f of peak, %.2f GHz)"
                                               % (k, v["tflops"], v["frac_of_peak"], v["clock_ghz"])
                                               for k, v in ceil.items()))

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample (~%.0f s)" % args.cpu_seconds)
        cpu = cpu_baseline(X, last["Pi"].cpu().numpy().astype(np.float64), args.cpu_seconds, len(st["probe_r"]))

    rec = {
        "metric": "fit time to certified max-distortion <= eps; pairs certified per second of fit",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fit_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "MNIST-shaped synthetic cloud (rank-50 mixture of 10 classes, 70%% fixed "
                               "zero mask), n=%d, d=%d, eps=%g, plain FP32 screen, bisection search"
                               % (n, d, args.eps),
                   "n": n, "d": d, "d_nonconstant": dx, "eps": args.eps, "seed": gen.JL_SEED, "data_seed": gen.DATA_SEED,
                   "parallelism": "single GPU", "workspace": "kept across calls"},
        "fit": {"r": last["r"], "s": last["s"], "k": last["k"], "certificates": ncert,
                "max_distortion": last["cert"]["max_distortion"], "certified": last["cert"]["certified"],
                "argmax": [last["cert"]["i"], last["cert"]["j"]], "t_pca_ms": st["t_pca_ms"],
                "t_search_ms": st["t_search_ms"], "t_screen_ms": st["t_screen_ms"],
                "t_rescore_ms": st["t_rescore_ms"], "eig_sweeps": st["eig_sweeps"],
                "rescored_pairs": st["n_rescored"], "flagged_tiles": st["n_flagged_tiles"],
                "refuted_probes": st["n_refuted"], "pair_evaluations_per_s": npairs * ncert / fit_s,
                "probes": [[r, dl, {3: "refuted by the pool", 4: "screen stopped early"}.get(g, "certified"), c]
                           for r, dl, g, c in zip(st["probe_r"], st["probe_delta"], st["probe_gram"],
                                                  st["probe_cols"])],
                "without_witness_pool": without_witness,
                "workspace": "kept across calls (adagio_keep_workspace(1), opted in for the loop of fits)",
                "with_per_call_workspace": per_call},
        "other_eps": extra,
        "mnist_like_67_constant_coordinates": border67,
        "tradeoff_min_r": tradeoff,
        "forms": forms,
        "large_precision_form": large,
        "knn_application": knn,
        "roofline": roofline,
        "mfma_ceilings": ceil,
        "cpu_baseline": cpu,
        "oracle_parity": parity,
        "paper_context": "paper: <10 s for 60,000 x 784 MNIST on an i5-3317U laptop (abstract); not this workload",
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
