"""Learned warm start for the eigenvalue MLE.  Test infrastructure only.

Algorithm 1 starts its eigenvalue loop at lambda^0 = 1/E.  The warm start
replaces that start by a small network's prediction from the two axes'
spectra; the solver then finishes from it (the optimum does not depend on the
start).  The paper does not fix this component; the reading implemented here:

* Features of an axis pair (c, g): each axis' log-spectrum resampled to
  B = 512 bins.  Bin b sits at the 0-based fractional index
  t_b = (b + 1/2) r / B - 1/2, clamped to [0, r - 1], and takes the linear
  interpolation of log E between the neighbouring indices.  Both curves are
  shifted by s = max(log E_c,0, log E_g,0).  Four scalars follow:
  log r_c, log r_g, log d_c, log d_g (d = the axes' dimensions).
  Total 2 B + 4 = 1028 inputs.
* Network: three linear layers 1028 -> 256 -> 256 -> 1024 with SiLU
  (x sigmoid(x)) after the first two.  Parameters are one flat FP32 vector:
  W1 (256 x 1028), b1, W2 (256 x 256), b2, W3 (1024 x 256), b3, row-major.
* Outputs: two 512-bin curves y_c, y_g of log(lambda_i E_i), resampled the
  same way as the features (targets come from solved problems).
* Back to eigenvalues: index i sits at bin coordinate
  u_i = (i + 1/2) B / r - 1/2, clamped to [0, B - 1]; lambda_i =
  exp(linear interpolation of y at u_i) / E_i.  The solver then moves the
  start to its gauge and clips it to the box.
* Loss: mean over unmasked entries of (y - target)^2 (mask = per-entry weight).
* Optimiser: AdamW (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay
  applied as p -= lr (m_hat / (sqrt(v_hat) + eps) + wd p)).

Everything here is FP64 NumPy written from those definitions.  The network
also runs in a BF16-weight mode (``low=True``): the two operands of every
matrix product, forward and backward, are rounded to BF16 (from their FP32
value, nearest even) and the products summed in full precision; parameters,
biases, activations and the optimiser stay in full precision.
"""
from __future__ import annotations

import math

import numpy as np

BINS = 512
D_IN = 2 * BINS + 4
D_H = 256
D_OUT = 2 * BINS
SHAPES = [("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
          ("W3", (D_OUT, D_H)), ("b3", (D_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def resample(values, bins=BINS):
    """Linear interpolation of ``values`` (length r) at t_b = (b + 1/2) r / bins - 1/2."""
    values = np.asarray(values, dtype=np.float64)
    r = values.size
    t = np.clip((np.arange(bins) + 0.5) * r / bins - 0.5, 0.0, r - 1)
    lo = np.floor(t).astype(np.int64)
    hi = np.minimum(lo + 1, r - 1)
    f = t - lo
    return values[lo] * (1.0 - f) + values[hi] * f


def features(Ec, Eg, dc, dg):
    lc, lg = np.log(np.asarray(Ec, np.float64)), np.log(np.asarray(Eg, np.float64))
    s = max(lc[0], lg[0])
    return np.concatenate([resample(lc) - s, resample(lg) - s,
                           [math.log(lc.size), math.log(lg.size), math.log(dc), math.log(dg)]])


def targets(Ec, lam_c, Eg, lam_g):
    return np.concatenate([resample(np.log(np.asarray(lam_c) * np.asarray(Ec))),
                           resample(np.log(np.asarray(lam_g) * np.asarray(Eg)))])


def _curve_at(y, r):
    """Linear interpolation of a bins-long curve at u_i = (i + 1/2) bins / r - 1/2."""
    bins = y.size
    u = np.clip((np.arange(r) + 0.5) * bins / r - 0.5, 0.0, bins - 1)
    lo = np.floor(u).astype(np.int64)
    hi = np.minimum(lo + 1, bins - 1)
    f = u - lo
    return y[lo] * (1.0 - f) + y[hi] * f


def apply(curves, Ec, Eg):
    """Warm-start eigenvalues (lambda_c, lambda_g) from the network's two curves."""
    curves = np.asarray(curves, dtype=np.float64)
    Ec, Eg = np.asarray(Ec, np.float64), np.asarray(Eg, np.float64)
    return (np.exp(_curve_at(curves[:BINS], Ec.size)) / Ec,
            np.exp(_curve_at(curves[BINS:], Eg.size)) / Eg)


def bf16(x):
    """Operands of the BF16-weight mode: a value as FP32, then rounded to the
    nearest BF16 (8 significant bits, ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    hi, lo = b >> 16, b & 0xFFFF
    up = (lo > 0x8000) | ((lo == 0x8000) & ((hi & 1) == 1))
    hi = (hi + up.astype(np.uint64)) & 0xFFFF
    return (hi << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(a, b, low):
    """a @ b, with both operands rounded to BF16 in the BF16-weight mode."""
    return bf16(a) @ bf16(b) if low else a @ b


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, cache=False, low=False):
    """The network; low=True is the BF16-weight mode (every product's operands
    rounded to BF16, the rest in full precision)."""
    P = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    Z1 = _mm(X, P["W1"].T, low) + P["b1"]
    H1 = silu(Z1)
    Z2 = _mm(H1, P["W2"].T, low) + P["b2"]
    H2 = silu(Z2)
    Y = _mm(H2, P["W3"].T, low) + P["b3"]
    if cache:
        return Y, (X, Z1, H1, Z2, H2)
    return Y


def loss(theta, X, T, mask=None, low=False):
    Y = forward(theta, X, low=low)
    M = np.ones_like(Y) if mask is None else np.asarray(mask, np.float64)
    return float(np.sum(M * (Y - T) ** 2) / np.sum(M))


def loss_and_grad(theta, X, T, mask=None, low=False):
    """Loss and its gradient with respect to the flat parameter vector (chain
    rule); low=True rounds the operands of every product, forward and
    backward, to BF16."""
    P = unpack(theta)
    Y, (X, Z1, H1, Z2, H2) = forward(theta, X, cache=True, low=low)
    M = np.ones_like(Y) if mask is None else np.asarray(mask, np.float64)
    msum = np.sum(M)
    L = float(np.sum(M * (Y - T) ** 2) / msum)
    dY = 2.0 * M * (Y - T) / msum
    g = {"W3": _mm(dY.T, H2, low), "b3": dY.sum(axis=0)}
    dZ2 = _mm(dY, P["W3"], low) * silu_grad(Z2)
    g["W2"] = _mm(dZ2.T, H1, low)
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = _mm(dZ2, P["W2"], low) * silu_grad(Z1)
    g["W1"] = _mm(dZ1.T, X, low)
    g["b1"] = dZ1.sum(axis=0)
    return L, pack(g)


def adamw_step(theta, m, v, grad, step, lr, wd, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v
