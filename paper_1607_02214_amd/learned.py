"""Learned Riemann guess: harvest interface records from sweeps, train the
network on them, and switch a context to the learned guess.  Orchestration
over the C ABI only: the harvest runs in the sweep kernels, training in the
BF16 matrix-core kernels (ppmlr_mlp_train_step)."""
from __future__ import annotations

from . import inputs
from . import ppmlr


def harvest(ctx, u, steps, cfl, capacity, stream=None):
    """Advance `u` by `steps` steps with the plain guess while every selected
    face appends a record; returns (records [n, 28] device tensor, number of
    records offered)."""
    import torch
    rec = torch.empty((int(capacity), ppmlr.RECORD_FLOATS), dtype=torch.float32, device=u.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=u.device)
    ctx.set_harvest(rec, cnt)
    ctx.set_guess(ppmlr.GUESS_HARVEST, stream=stream)
    try:
        ctx.advance(u, steps, cfl, stream=stream)
        offered = int(cnt.item())
    finally:
        ctx.set_guess(ppmlr.GUESS_PLAIN, stream=stream)
        ctx.set_harvest(None)
    return rec[:min(offered, int(capacity))], offered


def train(records, steps, batch=4096, lr=1e-3, seed=0, log_every=0, log=None):
    """Adam on the mean-squared error of the two targets over consecutive
    batches of the record buffer (cycled); returns (theta, [(step, loss)])."""
    import torch
    n = int(records.shape[0])
    if n < 1:
        raise ValueError("no records to train on")
    batch = min(int(batch), n)
    theta = torch.from_numpy(inputs.mlp_init(seed)).to(records.device)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    mlp = ppmlr.MLP(batch)
    loss = torch.zeros(1, dtype=torch.float32, device=records.device)
    nb = n // batch
    X = records[:, 0:14]
    Y = records[:, 14:16]
    history = []
    for t in range(1, int(steps) + 1):
        b = (t - 1) % nb
        mlp.train_step(theta, m, v, X[b * batch:(b + 1) * batch], Y[b * batch:(b + 1) * batch], t, lr=lr, loss=loss)
        if log_every and (t % log_every == 0 or t == 1):
            history.append((t, float(loss.item())))
            if log:
                log(f"[train] step {t} loss {history[-1][1]:.4e}")
    return theta, history
