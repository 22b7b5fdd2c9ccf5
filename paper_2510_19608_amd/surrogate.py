"""Learned pruning for the segment search: data collection, training and
evaluation of the ranking MLP (F=32 -> 256 -> 256 -> 1, GELU) through the C ABI.

Every numerical step runs in libokr's kernels: feature extraction and the
FP64 targets come out of an exhaustive search (okr_result.features /
.targets), training is okr_train_surrogate (BF16 MFMA forward/backward,
FP32 Adam), and the pruned search is okr_reduce_feeder with ``top_k`` and
the trained parameters.  This module only allocates device buffers and
draws the initial weights.
"""
from __future__ import annotations

import math

import numpy as np

from .binding import (SURR_FEATURES, SURR_HIDDEN, SURR_PARAMS, Reducer, okr_surrogate_forward,
                      okr_surrogate_workspace, okr_train_surrogate)

F, H = SURR_FEATURES, SURR_HIDDEN
OFF_W1 = 0
OFF_B1 = OFF_W1 + H * F
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H


def init_params(seed=0, device="cuda:0", b3=0.0):
    """He-normal weights, zero biases, output bias ``b3`` (the target mean is a
    good start); one FP32 device vector in the library's layout."""
    import torch
    rng = np.random.default_rng(seed)
    p = np.zeros(SURR_PARAMS, np.float32)
    p[OFF_W1:OFF_B1] = rng.normal(0.0, math.sqrt(2.0 / F), H * F)
    p[OFF_W2:OFF_B2] = rng.normal(0.0, math.sqrt(2.0 / H), H * H)
    p[OFF_W3:OFF_B3] = rng.normal(0.0, math.sqrt(1.0 / H), H)
    p[OFF_B3] = b3
    return torch.from_numpy(p).to(device)


def collect(feeders, device="cuda:0", **margin_kw):
    """Run the exhaustive FP64 search on each feeder dict and return the
    per-mask features X [N][32] and targets t [N] (device FP32), plus the
    per-feeder decisions.  Feeders whose base network is out of band are
    skipped (their searches make no decisions)."""
    import torch
    Xs, ts, decisions = [], [], []
    for f in feeders:
        R = Reducer(f, device=device, **margin_kw)
        try:
            R.run(replan=False, want_features=True)
            torch.cuda.synchronize(R.device)
            res = R.result()
            if res["warnings"]:
                continue
            Xs.append(R.features.clone())
            ts.append(R.targets.clone())
            decisions.append([s["mask"] for s in res["segments"]])
        finally:
            R.close()
    return torch.cat(Xs), torch.cat(ts), decisions


def train(X, t, epochs=6, batch=4096, lr=1e-3, seed=0, params=None):
    """Adam on mean-squared error over whole batches of (X, t); rows beyond the
    last whole batch of each shuffled pass are not used.  Returns (params,
    per-epoch mean loss)."""
    import torch
    n = (X.shape[0] // batch) * batch
    if n == 0:
        raise ValueError(f"need at least one batch of {batch} rows, have {X.shape[0]}")
    if params is None:
        params = init_params(seed, X.device, b3=float(t.mean().item()))
    work = torch.empty(okr_surrogate_workspace(batch), dtype=torch.uint8, device=X.device)
    loss = okr_train_surrogate(X, t, epochs, batch, lr, seed, params, work)
    return params, loss


def calibrate(params, X, t, q=0.99):
    """The network's over-prediction at quantile q on (X, t): the ln-error
    slack that keeps a fraction q of masks ranked as predicted feasible when
    they are (okr_margins.surrogate_margin).  Computed with the library's own
    forward pass; the quantile is taken on the host from the residuals."""
    import numpy as np
    y = predict(params, X)
    r = (y - t).float().cpu().numpy()
    return float(max(0.0, np.quantile(r, q)))


def predict(params, X, batch=65536):
    """Surrogate predictions for every row of X (device), in chunks."""
    import torch
    n = X.shape[0]
    pad = (-n) % 64
    Xp = torch.cat([X, X.new_zeros((pad, F))]) if pad else X
    y = torch.empty(Xp.shape[0], dtype=torch.float32, device=X.device)
    step = min(batch, Xp.shape[0])
    work = torch.empty(okr_surrogate_workspace(step), dtype=torch.uint8, device=X.device)
    for a in range(0, Xp.shape[0], step):
        b = min(a + step, Xp.shape[0])
        okr_surrogate_forward(params, Xp[a:b], y[a:b], work)
    return y[:n]
