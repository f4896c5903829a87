"""Learned Riemann guess: harvest interface records from sweeps, train the
network on them, and switch a context to the learned guess.  Orchestration
over the C ABI only: the harvest runs in the sweep kernels, training in the
BF16 matrix-core kernels (ppmlr_mlp_train_step)."""
from __future__ import annotations

from . import inputs
from . import ppmlr


def canonical_order(records):
    """The rows of a record buffer in lexicographic order of their values
    (first column most significant).  The waves of a sweep append records in
    an order that depends on their scheduling; this order depends on the
    record set only, so that training on it is reproducible."""
    import torch
    perm = torch.arange(records.shape[0], device=records.device)
    for c in range(records.shape[1] - 1, -1, -1):       # least significant first, stable
        perm = perm[torch.sort(records[perm, c], stable=True).indices]
    return records[perm]


def harvest(ctx, u, steps, cfl, capacity, stream=None):
    """Advance `u` by `steps` steps with the plain guess while every selected
    face appends a record; returns (records [n, 28] device tensor in
    canonical order, number of records offered)."""
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
    return canonical_order(rec[:min(offered, int(capacity))]), offered


def train(records, steps, batch=4096, lr=1e-3, seed=0, log_every=0, log=None):
    """Adam on the mean-squared error of the two targets over consecutive
    batches (cycled) of a permutation of the records drawn from `seed`, which
    also seeds the initial parameters; returns (theta, [(step, loss)])."""
    import torch
    n = int(records.shape[0])
    if n < 1:
        raise ValueError("no records to train on")
    batch = min(int(batch), n)
    theta = torch.from_numpy(inputs.mlp_init(seed)).to(records.device)
    gen = torch.Generator(device=records.device)
    gen.manual_seed(int(seed))
    records = records[torch.randperm(n, generator=gen, device=records.device)]
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
