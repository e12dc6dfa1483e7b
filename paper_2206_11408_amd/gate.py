"""Training driver for the learned skip gate (an extension beyond the paper).

1. ``collect_log``: FINGER searches with feature logging; every screened
   edge yields its features and (exact d2, bound ub2).
2. ``finger_gate_targets`` turns the log into targets t = cos(q_res, d_res).
3. ``train``: minibatch Adam on the mean squared error, forward/backward and
   the update all in the library's kernels (bf16 operands, float32
   accumulation); torch only holds buffers and draws the batch order.
4. ``calibrate``: eps_gate = mean |t - f(x)| on held-out rows, the analogue
   of Algorithm 2's correction term, computed by the library
   (``finger_gate_calibrate``), then ``finger_gate_attach``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from . import api


def collect_log(tables: api.Tables, queries: torch.Tensor, ef: int, k: int = 10,
                capacity: int = 1 << 22, entry: int = -1):
    """Run FINGER search over ``queries`` with logging.  Returns
    (features [rows, 2r+4], (d2, ub2) [rows, 2], rows screened in total)."""
    r = tables.info()["rank"]
    feats = torch.empty((capacity, 2 * r + 4), dtype=torch.float32, device=queries.device)
    targs = torch.empty((capacity, 2), dtype=torch.float32, device=queries.device)
    count = torch.zeros(1, dtype=torch.int64, device=queries.device)
    p = api.search_params(mode=L.MODE_FINGER, k=k, ef=ef, entry=entry, log=(feats, targs, count))
    api.finger_search(tables, queries, p)
    total = int(count.item())
    rows = min(total, capacity)
    return feats[:rows], targs[:rows], total


def init_weights(in_dim: int, hidden: int, seed: int = 0) -> np.ndarray:
    """He-uniform weights and zero biases in the C ABI's layout."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (hidden, in_dim)) * np.sqrt(6.0 / in_dim)
    W2 = rng.uniform(-1, 1, (hidden, hidden)) * np.sqrt(6.0 / hidden)
    W3 = rng.uniform(-1, 1, hidden) * np.sqrt(6.0 / hidden)
    return np.concatenate([W1.ravel(), np.zeros(hidden), W2.ravel(), np.zeros(hidden), W3,
                           [0.0]]).astype(np.float32)


def train(X: torch.Tensor, t: torch.Tensor, hidden: int = 64, epochs: int = 2, batch: int = 4096,
          lr: float = 1e-3, seed: int = 0, weights: np.ndarray | None = None, log=None):
    """Minibatch Adam on mean squared error.  Returns (weights float32 numpy,
    per-epoch mean training loss)."""
    in_dim = X.shape[1]
    dev = X.device
    w = torch.as_tensor(weights if weights is not None else init_weights(in_dim, hidden, seed),
                        dtype=torch.float32, device=dev).contiguous()
    g = torch.empty_like(w)
    m1 = torch.zeros_like(w)
    m2 = torch.zeros_like(w)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws = torch.empty(max(256, api.finger_mlp_backward_workspace_size(in_dim, hidden, batch)),
                     dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    n = X.shape[0]
    step = 0
    hist = []
    for ep in range(epochs):
        order = torch.randperm(n, generator=gen, device=dev)
        losses = []
        for s in range(0, n - batch + 1, batch):
            idx = order[s:s + batch]
            xb = X.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            api.finger_mlp_backward(w, in_dim, hidden, xb, tb, g, loss, workspace=ws)
            step += 1
            api.finger_adam_step(w, g, m1, m2, lr=lr, step=step)
            if (step % 64) == 0:
                losses.append(float(loss.item()))
        hist.append(float(np.mean(losses)) if losses else float("nan"))
        if log:
            log(f"gate epoch {ep}: loss {hist[-1]:.5f} ({step} steps)")
    return w.cpu().numpy(), hist


def calibrate(weights: np.ndarray, X: torch.Tensor, t: torch.Tensor, hidden: int) -> float:
    """eps_gate = mean |t - f(x)| over the given rows (finger_gate_calibrate)."""
    w = torch.as_tensor(weights, dtype=torch.float32, device=X.device)
    return api.finger_gate_calibrate(w, X.shape[1], hidden, X.contiguous(), t.contiguous())


def fit_gate(tables: api.Tables, train_queries: torch.Tensor, ef: int, hidden: int = 64,
             epochs: int = 2, batch: int = 4096, lr: float = 1e-3, capacity: int = 1 << 22,
             val_frac: float = 0.1, seed: int = 0, log=None) -> dict:
    """Log, train, calibrate and attach a gate to ``tables``."""
    X, Y, total = collect_log(tables, train_queries, ef, capacity=capacity)
    r = tables.info()["rank"]
    t = api.finger_gate_targets(X, Y, X.shape[0], r)
    n = X.shape[0]
    nval = max(1, int(n * val_frac))
    w, hist = train(X[nval:], t[nval:], hidden, epochs, batch, lr, seed, log=log)
    eps_gate = calibrate(w, X[:nval], t[:nval], hidden)
    api.finger_gate_attach(tables, w, X.shape[1], hidden, eps_gate)
    return {"weights": w, "eps_gate": eps_gate, "loss": hist, "rows": n, "screened": total}
