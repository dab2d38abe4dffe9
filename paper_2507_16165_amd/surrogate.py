"""Training driver of the sweep surrogate.

Every numeric step runs in the library's kernels: labels by the FP64
integrator (bh_surrogate_labels), forward/backward/Adam on the matrix cores
(bh_surrogate_train_step), validation and the trust map (bh_surrogate_infer,
bh_surrogate_build_trust).  This module draws the seeded samples, batches and
shuffles them (torch indexing), and schedules the learning rate.

Training set (units of M, sky at 1000 M): escape side b log-uniform in
[3 sqrt(3) + 0.05, 1000], r0 uniform in [10, 200], b <= 0.85 r0 (renders see
b <= 0.76 r0); capture side b uniform in [0, 3 sqrt(3) - 0.05] so that the
capture logit sees both classes.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import api, inputs

B_CRIT = 3.0 * math.sqrt(3.0)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (output layer scaled by 0.1), zero biases, in the
    flat order of bh.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (fi, fo) in enumerate([(2, 128), (128, 128), (128, 128), (128, 2)]):
        lim = math.sqrt(6.0 / fi) * (0.1 if k == 3 else 1.0)
        parts.append(rng.uniform(-lim, lim, (fi, fo)).astype(np.float32).ravel())
        parts.append(np.zeros(fo, np.float32))
    return np.concatenate(parts)


def generate(sur: api.Surrogate, n_escape: int, n_capture: int, seed: int, device="cuda"):
    """Labelled samples {b, r0, phi, cap} as device tensors."""
    import torch

    bs, rs = [], []
    have = 0
    rnd = 0
    while have < n_escape:
        b, r0 = inputs.surrogate_samples(int(2.5 * (n_escape - have)) + 1024, seed * 1000 + rnd,
                                         B_CRIT + 0.05, 1000.0)
        bs.append(b)
        rs.append(r0)
        have += b.size
        rnd += 1
    b = np.concatenate(bs)
    r0 = np.concatenate(rs)
    bc, rc = inputs.capture_samples(n_capture, seed * 1000 + 999, B_CRIT - 0.05)
    b = torch.from_numpy(np.concatenate([b, bc])).to(device)
    r0 = torch.from_numpy(np.concatenate([r0, rc])).to(device)
    phi, cap = sur.labels(b, r0)
    torch.cuda.synchronize()
    valid = torch.isfinite(phi) | (cap == 1)          # drop pairs with no such ray
    esc = torch.isfinite(phi)
    keep_esc = torch.nonzero(esc & valid).squeeze(1)[:n_escape]
    keep_cap = torch.nonzero((cap == 1) & valid).squeeze(1)
    idx = torch.cat([keep_esc, keep_cap])
    return {"b": b[idx].contiguous(), "r0": r0[idx].contiguous(), "phi": phi[idx].contiguous(),
            "cap": cap[idx].contiguous()}


def train(sur: api.Surrogate, data: dict, epochs: int, batch: int = 4096, lr_max: float = 3e-3,
          lr_min: float = 2e-5, seed: int = 0, log=None, time_limit: float | None = None):
    """Adam with a cosine learning-rate schedule; returns the mean loss per epoch."""
    import torch

    n = data["b"].numel()
    steps_per_epoch = n // batch
    total = max(1, epochs * steps_per_epoch)
    g = torch.Generator(device=data["b"].device)
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=data["b"].device)
    hist = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=data["b"].device)
        acc = torch.zeros(1, dtype=torch.float64, device=data["b"].device)
        for k in range(steps_per_epoch):
            idx = perm[k * batch:(k + 1) * batch]
            lr = lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * step / total))
            sur.train_step(data["b"][idx].contiguous(), data["r0"][idx].contiguous(),
                           data["phi"][idx].contiguous(), data["cap"][idx].contiguous(), lr, loss)
            acc += loss
            step += 1
        hist.append(float(acc.item()) / max(1, steps_per_epoch))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.3e} ({time.time() - t0:.1f} s)")
        if time_limit is not None and time.time() - t0 > time_limit:
            break
    return hist


def evaluate(sur: api.Surrogate, data: dict) -> dict:
    """Exit-azimuth errors of escaping samples and capture-logit agreement."""
    import torch

    y, phi = sur.infer(data["b"], data["r0"])
    esc = torch.isfinite(data["phi"])
    err = (phi - data["phi"]).abs()[esc]
    cap_ok = ((y[:, 1] >= 0) == (data["cap"] == 1)).float().mean()
    out = {"n": int(esc.sum().item()), "max_err": float(err.max().item()),
           "p99_err": float(torch.quantile(err.float()[:1 << 20], 0.99).item()),
           "mean_err": float(err.mean().item()), "capture_agreement": float(cap_ok.item())}
    bb = data["b"][esc]
    for lo, hi in ((10, 30), (30, 100), (100, 1000)):
        e = err[(bb >= lo) & (bb < hi)].float()
        if e.numel():
            out[f"p99_err_b{lo}_{hi}"] = float(torch.quantile(e[:1 << 20], 0.99).item())
            out[f"max_err_b{lo}_{hi}"] = float(e.max().item())
    return out


def fit(n_escape=4_000_000, n_capture=1_000_000, n_val=1_000_000, epochs=40, batch=4096,
        max_err=5e-5, min_count=5, seed=4, val_seed=40, log=None, time_limit=None,
        max_batch=4096):
    """The whole pipeline: labels, training, validation, trust map.  Returns
    (surrogate, report)."""
    sur = api.Surrogate(init_params(seed), max_batch=max_batch)
    t0 = time.time()
    data = generate(sur, n_escape, n_capture, seed)
    val = generate(sur, n_val, n_val // 4, val_seed)
    t1 = time.time()
    hist = train(sur, data, epochs, batch=batch, seed=seed, log=log, time_limit=time_limit)
    t2 = time.time()
    ev = evaluate(sur, val)
    esc = val["phi"].isfinite()
    sur.build_trust(val["b"][esc].contiguous(), val["r0"][esc].contiguous(),
                    val["phi"][esc].contiguous(), max_err, min_count)
    trust = sur.trust()
    report = {"train_samples": int(data["b"].numel()), "val_samples": int(val["b"].numel()),
              "label_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2), "epochs": len(hist),
              "final_loss": hist[-1] if hist else None, "val": ev,
              "trusted_bins": int(trust.sum()), "trust_max_err": max_err}
    return sur, report


def save(sur: api.Surrogate, path: str, step: int = 0) -> None:
    np.savez(path, params=sur.get(0), m=sur.get(2), v=sur.get(3), trust=sur.trust(),
             step=np.int64(step))


def load(path: str, max_batch: int = 4096) -> api.Surrogate:
    z = np.load(path, allow_pickle=False)
    sur = api.Surrogate(z["params"], max_batch=max_batch)
    sur.set(z["params"], z["m"], z["v"], int(z["step"]))
    sur.set_trust(z["trust"])
    return sur
