"""Learned form on the GPU: the predictor's own BF16 MFMA forward/backward
kernels against the FP64 oracle MLP, the Adam step, the sketch features, the
learned search (every prediction certified, bisection fallback), and what the
trained predictor gains over plain bisection on held-out instances."""
import os

import numpy as np
import pytest
import torch

from oracle import certificate, embedding
from oracle import mlp as omlp
from oracle import sketch as osketch
from paper_1609_05388_amd import gen, learned

pytestmark = pytest.mark.gpu


def bf16_round(a):
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)


def setup(seed=0, B=64):
    count = omlp.layout()[1]
    p = learned.init_params(count, seed).astype(np.float32)
    rng = np.random.default_rng(seed + 5)
    X = np.zeros((B, 80), np.float32)
    X[:, :67] = rng.normal(0, 1, (B, 67))
    y = rng.normal(-1.5, 0.6, B).astype(np.float32)
    return p, X, y


def test_param_count_matches_oracle_layout(gpu_lib):
    assert gpu_lib.mlp_param_count() == omlp.layout()[1]


def test_mlp_forward_matches_oracle(gpu_lib):
    p, X, y = setup(1)
    out = gpu_lib.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    # oracle on the BF16 values of weights and inputs (biases stay FP32)
    pb = p.astype(np.float64).copy()
    off, _ = omlp.layout()
    for name in ("W1", "W2", "W3", "w4"):
        o, s = off[name]
        pb[o:o + s] = bf16_round(p[o:o + s])
    want, _ = omlp.forward(pb, bf16_round(X), round_act=bf16_round)
    err = np.abs(out - want).max() / (np.abs(want).max() + 1e-12)
    assert err < 2e-2, err


def test_mlp_gradient_matches_oracle(gpu_lib):
    """Per tensor: cosine >= 0.999 and relative L2 error <= 2e-2 against the
    FP64 chain rule on the same BF16 weights and inputs.  The oracle rounds
    the hidden activations to BF16 where the kernels do, so both sides take
    the same ReLU decisions; the remaining difference is the BF16 rounding of
    back-propagated errors used as MFMA operands."""
    p, X, y = setup(2, B=128)
    g, loss = gpu_lib.mlp_grad(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), 0.9)
    g = g.cpu().numpy().astype(np.float64)
    pb = p.astype(np.float64).copy()
    off, _ = omlp.layout()
    for name in ("W1", "W2", "W3", "w4"):
        o, s = off[name]
        pb[o:o + s] = bf16_round(p[o:o + s])
    L, G = omlp.grad(pb, bf16_round(X), y.astype(np.float64), 0.9, round_act=bf16_round)
    assert abs(float(loss.cpu()) - L) <= 2e-2 * abs(L)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4"):
        o, s = off[name]
        a, b = g[o:o + s], G[o:o + s]
        if np.linalg.norm(b) == 0:
            assert np.linalg.norm(a) == 0
            continue
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert cos >= 0.999 and rel <= 2e-2, (name, cos, rel)


def test_adam_first_step_and_descent(gpu_lib):
    """From zero moments, Adam's first step is -lr * sign(g) (|g| >> eps), and
    repeated steps lower the loss on a fixed batch."""
    p, X, y = setup(3, B=64)
    P = torch.from_numpy(p).cuda()
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    g, _ = gpu_lib.mlp_grad(P, Xd, yd, 0.9)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    P1 = P.clone()
    loss0 = gpu_lib.mlp_train_step(P1, m, v, 1, 1e-3, Xd, yd, 0.9)
    d = (P1 - P).cpu().numpy()
    gn = g.cpu().numpy()
    big = np.abs(gn) > 1e-5
    assert np.allclose(d[big], -1e-3 * np.sign(gn[big]), rtol=1e-3, atol=1e-7)
    losses = [float(loss0.cpu())]
    for step in range(2, 60):
        losses.append(float(gpu_lib.mlp_train_step(P1, m, v, step, 1e-3, Xd, yd, 0.9).cpu()))
    assert losses[-1] < 0.5 * losses[0]


@pytest.mark.parametrize("n,d", [(300, 40), (2000, 784)])
def test_sketch_features_match_oracle(gpu_lib, n, d):
    X = gen.low_rank_pixels(n=n, d=d, rank=12, seed=n)
    f = gpu_lib.sketch_features(torch.from_numpy(X).cuda(), 0.12, gen.JL_SEED).cpu().numpy()
    want = osketch.sketch_features(X, 0.12, gen.JL_SEED)
    # the smallest sketch eigenvalues are at rounding level: compare where
    # sigma_i / ||sigma|| >= 1e-5, and the scalar features exactly
    ok = want[:64] > np.log(1e-5) / 4
    assert np.abs(f[:64][ok] - want[:64][ok]).max() < 1e-4
    assert np.abs(f[64:] - want[64:]).max() < 1e-6


def test_learned_search_certified_with_fallback(gpu_lib):
    """A predictor that always says r = 1 forces the fallback: the result is
    bisection on (1, d], certified and within eps."""
    X = torch.from_numpy(gen.low_rank_pixels(n=600, d=120, rank=10, seed=5)).cuda()
    count = gpu_lib.mlp_param_count()
    P = torch.zeros(count, dtype=torch.float32, device="cuda")
    off, _ = omlp.layout()
    P[off["b4"][0]] = -50.0          # ln(r / d) = -50 -> r = 1
    f = gpu_lib.fit(X, 0.1, 7, search="learned", predictor=P)
    assert f["stats"]["r_predicted"] == 1 and f["stats"]["n_fallback"] == 1
    assert f["cert"]["certified"] == 1 and f["cert"]["max_distortion"] <= 0.1
    plain = gpu_lib.fit(X, 0.1, 7)
    assert f["r"] >= 1 and f["cert"]["max_distortion"] <= 0.1
    # a predictor that says r = plain r* certifies with one certificate
    P[off["b4"][0]] = float(np.log(plain["r"] / 120.0)) - 1e-6
    g = gpu_lib.fit(X, 0.1, 7, search="learned", predictor=P)
    assert g["stats"]["r_predicted"] == plain["r"]
    assert g["stats"]["n_certificates"] == 1 and g["stats"]["n_fallback"] == 0
    assert g["r"] == plain["r"] and torch.equal(g["Pi"], plain["Pi"])


@pytest.mark.skipif(not os.path.exists(learned.PREDICTOR), reason="no trained predictor committed")
def test_trained_predictor_gains_over_bisection(gpu_lib):
    """Held-out instances: every fit's certificate proves max distortion <=
    eps (its exact maximum, or for a near-isometry its proven bound), and the
    learned search needs fewer certificates and less fit time than plain
    bisection."""
    res = learned.evaluate(learned.PREDICTOR, range(0, 12), held_out=True, log_every=100)
    s = learned.summarize(res)
    print(s)
    assert s["all_proven_within_eps"]
    assert s["mean_certificates_learned"] < s["mean_certificates_plain"]
    assert s["speedup"] > 1.0


def test_learned_search_refined_downward(gpu_lib):
    """refine=True: a prediction far above the needed r certifies, then the
    search probes downward and bisects, so the result is bisection-minimal:
    certified within eps, and the map at r - 1 fails (an FP64 oracle
    certificate of the library's own map at r - 1 exceeds eps)."""
    X = gen.low_rank_pixels(n=600, d=120, rank=10, seed=5)
    Xd = torch.from_numpy(X).cuda()
    count = gpu_lib.mlp_param_count()
    P = torch.zeros(count, dtype=torch.float32, device="cuda")
    off, _ = omlp.layout()
    P[off["b4"][0]] = float(np.log(100.0 / 120.0))   # r = 100, far above r*
    plain = gpu_lib.fit(Xd, 0.1, 7)
    coarse = gpu_lib.fit(Xd, 0.1, 7, search="learned", predictor=P)
    f = gpu_lib.fit(Xd, 0.1, 7, search="learned", predictor=P, refine=True)
    assert coarse["r"] == 100 and f["stats"]["r_predicted"] == 100 and f["stats"]["n_fallback"] == 0
    assert f["cert"]["certified"] == 1 and f["cert"]["max_distortion"] <= 0.1
    assert f["r"] < 100
    below = gpu_lib.project(Xd, f["r"] - 1, 7).cpu().numpy().astype(np.float64)
    want = certificate.certify(X, embedding.embed(X, below))
    assert want["max"] > 0.1
    print("refined r %d, plain r %d" % (f["r"], plain["r"]))


def test_learned_search_refined_within_4_percent(gpu_lib):
    """refine="within4": the same downward search, but its bisection stops
    once the largest failing probe below the returned r is within r / 25 of
    it (or next to it); the result is certified within eps, lies between the
    bisection-minimal r and the prediction, and takes no more certificates
    than refine=True."""
    X = gen.low_rank_pixels(n=600, d=120, rank=10, seed=5)
    Xd = torch.from_numpy(X).cuda()
    count = gpu_lib.mlp_param_count()
    P = torch.zeros(count, dtype=torch.float32, device="cuda")
    off, _ = omlp.layout()
    P[off["b4"][0]] = float(np.log(100.0 / 120.0))   # r = 100, far above r*
    print("learned search, refine within 4%", flush=True)
    f = gpu_lib.fit(Xd, 0.1, 7, search="learned", predictor=P, refine="within4")
    full = gpu_lib.fit(Xd, 0.1, 7, search="learned", predictor=P, refine=True)
    assert f["cert"]["certified"] == 1 and f["cert"]["max_distortion"] <= 0.1
    assert f["stats"]["n_fallback"] == 0 and full["r"] <= f["r"] < 100
    st = f["stats"]
    failed = [r for r, dl in zip(st["probe_r"], st["probe_delta"]) if dl > 0.1 and r < f["r"]]
    gap = f["r"] - max(failed)
    assert failed and (gap <= 1 or gap * 25 <= f["r"])
    assert st["n_certificates"] <= full["stats"]["n_certificates"]
