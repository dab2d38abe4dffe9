"""FP64 reference of the surrogate network (numpy).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's
checks, never by the product path; shares no code with the GPU kernels.

What it computes (the learned extension of the tracer; the paper's Eq. (1)
and initial conditions give the labels, see bh_ref.c):
  - inputs (b/M, r0/M) of an ingoing ray from r0 with impact parameter b;
  - features  f1 = sign(d) ln(1 + |d|/0.05) / 5,  d = b/M - 3 sqrt(3),
              f2 = (r0/M - 105) / 95;
  - network   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2),
              h3 = relu(h2 W3 + b3), y = h3 W4 + b4   (2 -> 128 -> 128 -> 128 -> 2);
  - outputs   y0: scaled deflection residual, y1: capture logit;
  - exit azimuth  phi_exit = sweep1(b, r0, R) + S(b) y0, with sweep1 the
    first-order weak-field sweep and S(b) = 12 (M/b)^2 its residual scale;
  - loss      L = (1/B) sum_i [ e_i (y0_i - t_i)^2 + 0.1 BCE(y1_i, c_i) ],
              t = (phi_exit_true - sweep1) / S, e_i = 1 for escaping rays with
              b >= 10 M (the regression domain: closer to the critical value the
              residual is too steep for bf16 activations to meet 1e-4 rad, and
              the trust map keeps such rays on the integrator anyway),
              c_i = 1 for captured rays;
  - Adam (Kingma & Ba 2015) on FP32 master weights; the network runs on the
    bf16-rounded copy.
  - quantize=True: the network as it is stored between layers -- the hidden
    activations h1, h2, h3, the output gradient dL/dy and the back-propagated
    gradients dL/dz3, dL/dz2, dL/dz1 each rounded to bf16 (ties to even)
    where the matrix-core network keeps them; every sum is still FP64.  With
    quantize=False (the default) nothing but the weights is rounded.
All lengths in units of M (the method is scale-free in M).
"""
from __future__ import annotations

import math

import numpy as np

B_CRIT = 3.0 * math.sqrt(3.0)
R_SKY = 1000.0
BAND_SCALE = 0.05
BCE_WEIGHT = 0.1
HIDDEN = 128
SHAPES = [(2, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, 2)]


# -- features, baseline, targets ---------------------------------------------

def features(b, r0):
    b = np.asarray(b, np.float64)
    r0 = np.asarray(r0, np.float64)
    d = b - B_CRIT
    f1 = np.sign(d) * np.log1p(np.abs(d) / BAND_SCALE) / 5.0
    f2 = (r0 - 105.0) / 95.0
    return np.stack([f1, f2], -1)


def residual_scale(b):
    return 12.0 / np.asarray(b, np.float64) ** 2


def sweep_first_order(b, r0, r_sky=R_SKY):
    """pi - a(r_sky) - a(r0), a(r) = asin(clip(b/r - (1/b)(2 - b^2/r^2), -1, 1)):
    the sweep of the first-order solution u = sin(phi)/b + (1 + cos^2 phi)/b^2
    (M = 1) between its two crossings of radius r0 and r_sky."""
    b = np.asarray(b, np.float64)

    def a(r):
        return np.arcsin(np.clip(b / r - (2.0 - b * b / (r * r)) / b, -1.0, 1.0))

    return math.pi - a(r_sky) - a(np.asarray(r0, np.float64))


REGRESSION_B_MIN = 10.0


def regression_mask(b, phi_exit):
    """Samples that carry the squared-error term: escaped, b >= 10 M."""
    return np.isfinite(np.asarray(phi_exit, np.float64)) & (np.asarray(b) >= REGRESSION_B_MIN)


def targets(b, r0, phi_exit):
    return (np.asarray(phi_exit) - sweep_first_order(b, r0)) / residual_scale(b)


def predict_exit(b, r0, y0):
    return sweep_first_order(b, r0) + residual_scale(b) * np.asarray(y0)


# -- parameters ---------------------------------------------------------------

def init_params(seed: int):
    """He-uniform weights (last layer scaled by 0.1), zero biases, float32."""
    rng = np.random.default_rng(seed)
    params = []
    for k, (fi, fo) in enumerate(SHAPES):
        lim = math.sqrt(6.0 / fi) * (0.1 if k == 3 else 1.0)
        params.append(rng.uniform(-lim, lim, (fi, fo)).astype(np.float32))
        params.append(np.zeros(fo, np.float32))
    return params


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32."""
    x = np.ascontiguousarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(x), x, out)


# -- network ------------------------------------------------------------------

def _q(x, quantize):
    """x rounded to bf16 (through float32) when quantize, else x itself."""
    return bf16_round(np.asarray(x, np.float64).astype(np.float32)).astype(np.float64) if quantize else x


def forward(params, x, quantize=False):
    """Returns (y, cache); params: [W1, b1, ..., W4, b4] (any float dtype,
    evaluated in float64); quantize: hidden activations rounded to bf16."""
    W = [np.asarray(p, np.float64) for p in params]
    h0 = np.asarray(x, np.float64)
    z1 = h0 @ W[0] + W[1]
    h1 = _q(np.maximum(z1, 0.0), quantize)
    z2 = h1 @ W[2] + W[3]
    h2 = _q(np.maximum(z2, 0.0), quantize)
    z3 = h2 @ W[4] + W[5]
    h3 = _q(np.maximum(z3, 0.0), quantize)
    y = h3 @ W[6] + W[7]
    return y, (h0, z1, h1, z2, h2, z3, h3)


def loss_and_dy(y, t, escaped, captured):
    """Loss and its gradient with respect to y (both (B, 2))."""
    y = np.asarray(y, np.float64)
    B = y.shape[0]
    e = np.asarray(escaped, np.float64)
    c = np.asarray(captured, np.float64)
    t = np.where(e > 0, np.asarray(t, np.float64), 0.0)
    r = y[:, 0] - t
    z = y[:, 1]
    bce = np.maximum(z, 0.0) - z * c + np.log1p(np.exp(-np.abs(z)))
    L = np.sum(e * r * r + BCE_WEIGHT * bce) / B
    dy = np.zeros_like(y)
    dy[:, 0] = 2.0 * e * r / B
    dy[:, 1] = BCE_WEIGHT * (1.0 / (1.0 + np.exp(-z)) - c) / B
    return L, dy


def backward(params, cache, dy, quantize=False):
    """Gradients [dW1, db1, ..., dW4, db4] (float64) of sum(dy * y);
    quantize: dy and the back-propagated dz rounded to bf16 (the ReLU masks
    then come from the stored activations, h > 0)."""
    W = [np.asarray(p, np.float64) for p in params]
    h0, z1, h1, z2, h2, z3, h3 = cache
    m1, m2, m3 = (h1 > 0, h2 > 0, h3 > 0) if quantize else (z1 > 0, z2 > 0, z3 > 0)
    dy = _q(np.asarray(dy, np.float64), quantize)
    g = [None] * 8
    g[6] = h3.T @ dy
    g[7] = dy.sum(0)
    dz3 = _q((dy @ W[6].T) * m3, quantize)
    g[4] = h2.T @ dz3
    g[5] = dz3.sum(0)
    dz2 = _q((dz3 @ W[4].T) * m2, quantize)
    g[2] = h1.T @ dz2
    g[3] = dz2.sum(0)
    dz1 = _q((dz2 @ W[2].T) * m1, quantize)
    g[0] = h0.T @ dz1
    g[1] = dz1.sum(0)
    return g


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        g = np.asarray(g, np.float64)
        mm = beta1 * np.asarray(mm, np.float64) + (1 - beta1) * g
        vv = beta2 * np.asarray(vv, np.float64) + (1 - beta2) * g * g
        mh = mm / (1 - beta1 ** step)
        vh = vv / (1 - beta2 ** step)
        out_p.append(np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
