"""Learned pruning on the GPU, through the C ABI: the MLP's forward pass,
gradient and Adam step against the FP64 NumPy oracle, the feature/target
dump against the oracle's per-mask errors, and the pruned search.

Tolerances.  The GEMM operands are BF16 (8 significant bits) with FP32
accumulation, so the forward pass is compared twice: tightly (1e-3) with
the oracle fed the same BF16-rounded operands, which pins the MFMA lane
layout, and loosely against the unrounded FP64 oracle.  The gradient is
compared per parameter block in relative norm (backward operands are BF16
as well).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp
from synth_feeders import make_feeder

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def okr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2510_19608_amd as okr
    okr.lib()
    return okr


F, H = 32, 256
KEYS = ("W1", "b1", "W2", "b2", "w3", "b3")


def flat(p):
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in KEYS]).astype(np.float32)


def unflat(v):
    v = np.asarray(v, np.float64)
    sizes = dict(W1=(H, F), b1=(H,), W2=(H, H), b2=(H,), w3=(H,), b3=(1,))
    out, o = {}, 0
    for k in KEYS:
        n = int(np.prod(sizes[k]))
        out[k] = v[o:o + n].reshape(sizes[k])
        o += n
    return out


def bf16(a):
    import torch
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def forward_bf16(p, X):
    """The oracle's forward pass with the kernels' BF16 rounding points."""
    Z1 = bf16(X) @ bf16(p["W1"]).T + p["b1"]
    H1 = bf16(mlp.gelu(Z1))
    Z2 = H1 @ bf16(p["W2"]).T + p["b2"]
    return mlp.gelu(Z2) @ p["w3"] + p["b3"][0]


def problem(seed, B):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(F, H, seed)
    p["b1"] = rng.normal(0, 0.1, H)
    p["b2"] = rng.normal(0, 0.1, H)
    p["b3"] = np.array([-5.0])
    p = unflat(flat(p))  # the FP32 values the GPU sees
    X = rng.normal(0, 1, (B, F))
    X[:, 20:] = 0.0  # padded feature columns, as in the search
    X = np.asarray(X, np.float32).astype(np.float64)
    t = rng.normal(-6, 2, B).astype(np.float32).astype(np.float64)
    return p, X, t


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("B", [64, 320])
def test_forward_matches_oracle(okr, B):
    import torch
    _say(f"surrogate forward B={B}")
    p, X, _ = problem(1, B)
    y = torch.empty(B, dtype=torch.float32, device="cuda")
    work = torch.empty(okr.okr_surrogate_workspace(B), dtype=torch.uint8, device="cuda")
    okr.okr_surrogate_forward(dev(flat(p)), dev(X), y, work)
    got = y.cpu().numpy().astype(np.float64)
    tight = forward_bf16(p, X)
    np.testing.assert_allclose(got, tight, rtol=0, atol=1e-3 * (1 + np.abs(tight)).max())
    exact, _ = mlp.forward(p, X)
    assert np.abs(got - exact).max() <= 0.05 * (1 + np.abs(exact).max())


@pytest.mark.parametrize("B", [128, 512])
def test_gradient_matches_oracle(okr, B):
    import torch
    _say(f"surrogate gradient B={B}")
    p, X, t = problem(2, B)
    grads = torch.empty(okr.SURR_PARAMS, dtype=torch.float32, device="cuda")
    work = torch.empty(okr.okr_surrogate_workspace(B), dtype=torch.uint8, device="cuda")
    loss = okr.okr_surrogate_grad(dev(flat(p)), dev(X), dev(t), grads, work)
    assert abs(loss - mlp.loss(p, X, t)) <= 1e-2 * mlp.loss(p, X, t)
    got = unflat(grads.cpu().numpy())
    ref = mlp.grads(p, X, t)
    for k in KEYS:
        g, r = got[k], ref[k]
        if k == "W1":  # columns of the zero feature padding have zero gradient
            assert np.abs(g[:, 20:]).max() == 0.0
            g, r = g[:, :20], r[:, :20]
        rel = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
        assert rel < 2e-2, f"{k}: relative error {rel:.3g}"


def test_adam_step_matches_oracle(okr):
    """One epoch of one batch = one Adam step from zero moments."""
    import torch
    _say("surrogate adam step")
    B, lr = 256, 1e-3
    p, X, t = problem(3, B)
    p0 = flat(p)
    grads = torch.empty(okr.SURR_PARAMS, dtype=torch.float32, device="cuda")
    work = torch.empty(okr.okr_surrogate_workspace(B), dtype=torch.uint8, device="cuda")
    okr.okr_surrogate_grad(dev(p0), dev(X), dev(t), grads, work)
    g = unflat(grads.cpu().numpy())
    params = dev(p0)
    loss = okr.okr_train_surrogate(dev(X), dev(t), 1, B, lr, 0, params, work)
    assert loss.shape == (1,) and np.isfinite(loss).all()
    zeros = {k: np.zeros_like(v) for k, v in p.items()}
    want, _, _ = mlp.adam_step(dict(p), g, dict(zeros), {k: v.copy() for k, v in zeros.items()}, 1, lr)
    got = params.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, flat(want).astype(np.float64), rtol=0, atol=lr * 1e-3 + 1e-6)


def test_features_and_targets(okr):
    """Targets of the exhaustive run are ln(e_loc + 1e-12) of the oracle's
    per-mask errors; feature 0 is the mask's reduced fraction."""
    import torch
    _say("surrogate features c1 seed 0")
    f = make_feeder("c1", 0, e_bar=3e-4)
    R = okr.Reducer(f)
    try:
        R.run(replan=False, want_features=True)
        torch.cuda.synchronize()
        k = R.result()["segments"][0]["k"]
        Xf = R.features.cpu().numpy()
        t = R.targets.cpu().numpy().astype(np.float64)
    finally:
        R.close()
    V, I, _, _ = oracle.powerflow(f)
    ref = oracle.score_masks(f, V, I, np.ones(f["n"], np.uint8), 0, np.arange(1 << k))
    e = ref["e_loc"]
    np.testing.assert_allclose(np.exp(t) - 1e-12, e, rtol=1e-5, atol=1e-9)
    pop = np.array([bin(m).count("1") for m in range(1 << k)])
    np.testing.assert_array_equal(Xf[:, 0], (pop / k).astype(np.float32))
    assert np.all(Xf[:, 16:] == 0.0)
    assert np.isfinite(Xf).all()


def test_training_reduces_loss(okr):
    import torch
    from paper_2510_19608_amd import surrogate
    _say("surrogate training on c1 seeds 0-3")
    feeders = [make_feeder("c1", s, e_bar=3e-4) for s in range(4)]
    X, t, _ = surrogate.collect(feeders)
    params, loss = surrogate.train(X, t, epochs=8, batch=1024, lr=1e-3, seed=0)
    assert np.isfinite(loss).all()
    assert loss[-1] < 0.7 * loss[0], loss
    y = surrogate.predict(params, X)
    mse = float(((y - t) ** 2).mean().item())
    assert mse < 2.0 * loss[-1] + 1e-3


@pytest.mark.parametrize("seed", [0, 2, 5])
def test_full_topk_equals_exhaustive(okr, seed):
    """top_k = 2^k rescoring covers every mask, so the pruned search must make
    the exhaustive decision whatever the network predicts."""
    from paper_2510_19608_amd import surrogate
    _say(f"surrogate top_k=4096 c1 seed={seed}")
    f = make_feeder("c1", seed, e_bar=3e-4)
    V, I, _, _ = oracle.powerflow(f)
    keep, dec, st = oracle.search(f, V, I)
    params = surrogate.init_params(seed)
    out = okr.reduce_feeder(f, surrogate=params, top_k=1 << 12)
    assert [s["mask"] for s in out["segments"]] == [d["mask"] for d in dec]
    np.testing.assert_array_equal(out["kept"], keep)
    for s, d in zip(out["segments"], dec):
        assert abs(s["e_loc"] - d["e_loc"]) < 1e-9


@pytest.mark.parametrize("seed", [1, 4])
def test_small_topk_is_feasible(okr, seed):
    """With an untrained network and a small top_k the decision may lose
    reduction, but it is feasible (oracle error within the margin) or the
    full enumeration's."""
    from paper_2510_19608_amd import surrogate
    _say(f"surrogate top_k=16 c1 seed={seed}")
    f = make_feeder("c1", seed, e_bar=3e-4)
    V, I, _, _ = oracle.powerflow(f)
    keep, dec, st = oracle.search(f, V, I)
    params = surrogate.init_params(100 + seed)
    out = okr.reduce_feeder(f, surrogate=params, top_k=16)
    s = out["segments"][0]
    ref = oracle.score_masks(f, V, I, np.ones(f["n"], np.uint8), 0, np.array([s["mask"]]))
    assert ref["feasible"][0]
    assert s["popcount"] <= dec[0]["popcount"]
    assert abs(s["e_loc"] - ref["e_loc"][0]) < 1e-9


def test_trained_network_gains_over_untrained(okr):
    """What training buys: on 32 held-out 30-bus feeders at a binding bound,
    the pruned search (top 32 of 4,096 masks rescored exactly, full
    enumeration as fallback) with the network trained on the exhaustive
    search's own dumps decides more segments correctly from the top-k alone
    (no fallback) than the same search with an untrained network, and agrees
    with the exhaustive decision on most of them.  Each network's
    predicted-feasible test uses its own calibrated margin (99.9% quantile of
    its over-prediction on the training rows)."""
    from paper_2510_19608_amd import surrogate
    _say("surrogate: trained vs untrained on held-out c1 seeds 100-131")
    train_feeders = [make_feeder("c1", s) for s in range(16)] + [make_feeder("c2", s) for s in (101, 102)]
    X, t, _ = surrogate.collect(train_feeders)
    trained, loss = surrogate.train(X, t, epochs=6, batch=4096, lr=1e-3, seed=0)
    untrained = surrogate.init_params(7, b3=float(t.mean().item()))
    m_tr = surrogate.calibrate(trained, X, t, 0.999)
    m_un = surrogate.calibrate(untrained, X, t, 0.999)
    held = [make_feeder("c1", s, e_bar=3e-4) for s in range(100, 132)]
    stats = {}
    for name, params, margin in (("trained", trained, m_tr), ("untrained", untrained, m_un)):
        ok_topk = agree = fallback = deficit = 0
        for f in held:
            ex = okr.reduce_feeder(f, want_vhat=False)
            out = okr.reduce_feeder(f, want_vhat=False, surrogate=params, top_k=32, surrogate_margin=margin)
            a, b = out["segments"][0], ex["segments"][0]
            fb = a["n_scored"] > a["n_refined"]
            agree += a["mask"] == b["mask"]
            fallback += fb
            ok_topk += (a["mask"] == b["mask"]) and not fb
            deficit += b["popcount"] - a["popcount"]
        stats[name] = dict(ok_topk=ok_topk, agree=agree, fallback=fallback, deficit=deficit)
    _say(f"  margins {m_tr:.3f} / {m_un:.3f}: {stats}")
    tr, un = stats["trained"], stats["untrained"]
    assert tr["ok_topk"] >= un["ok_topk"] + 4, stats
    assert tr["fallback"] < un["fallback"], stats
    assert tr["agree"] >= 26, stats
