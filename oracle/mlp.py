"""Surrogate network of the homogenisation map (oracle; test infrastructure only).

The surrogate is not part of the paper: it learns the map from one macro Gauss
point's record (temperature T, moisture c, exposure time t, eight property
factors) to the homogenised C_bar, K_bar, D_bar that the RVE solve of Sec. 2
produces.  T, c and t enter the paper's model only through the degradation
factor (1 - omega) = exp(-gamma(c) alpha(T) t) of Sec. 4 (Eq. Eq_Model_final1),
so the network sees the record through that law: its ten features are
log(1 - omega), (1 - omega) and the eight factors.

Network (one ensemble member): features -> 256 -> 256 -> 256 -> 36, GELU on the
hidden layers (exact form z * Phi(z), Phi the standard normal CDF), identity
output.  The physical outputs are the 21 upper-triangle entries of C_bar
(row-major, Voigt order 11, 22, 33, 12, 23, 31), then K_bar and D_bar as
(xx, yy, zz, xy, yz, zx).  The network predicts them in a per-block encoding:
for each block (C, K, D) the log of its Frobenius norm and the block divided by
that norm (21 + 1, 6 + 1, 6 + 1 = 36 numbers); decoding rescales the predicted
direction to unit norm.  Relative errors of a block then do not grow where the
block is small (heavily degraded matrix).  Features and encoded outputs are
standardised (per column mean and population standard deviation of the training
set).

Flat parameter layout of one member (row-major [out][in] matrices):
    W1 [256][10], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256],
    W4 [36][256], b4 [36]                             (143,652 numbers)

Arithmetic is FP64 here.  With quant=True the values the GPU kernels round to
bfloat16 are rounded at the same points (round to nearest even from the FP32
value): the standardised inputs, every weight matrix, the hidden activations,
the output gradient and the hidden pre-activation gradients.  The backward
pass treats each rounding as the identity (straight-through), which is what the
kernels compute.  With quant=False it is the plain network, whose gradient the
tests check by finite differences.

Training: mean squared error on the standardised encoded outputs over the rows
and the 36 columns; Adam (Kingma and Ba, ICLR 2015) with bias correction.

Ensemble: the prediction is the member mean in physical units; the
disagreement of a point is the largest over the C, K, D blocks of
||s||_F / ||mean||_F, with s the sample standard deviation over members and
||.||_F the Frobenius norm of the full symmetric matrix (off-diagonal entries
counted twice).
"""
from __future__ import annotations

import math

import numpy as np

from . import materials as mats

N_FEAT = 10
HIDDEN = 256
N_OUT = 36          # encoded outputs of the network
N_PHYS = 33         # physical outputs
LAYERS = ((N_FEAT, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, N_OUT))
# Frobenius weights of the output blocks (full symmetric matrix from the stored entries)
_CW = np.array([1.0 if a == b else 2.0 for a in range(6) for b in range(a, 6)])
_SW = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
OUT_WEIGHTS = np.concatenate([_CW, _SW, _SW])
BLOCKS = (slice(0, 21), slice(21, 27), slice(27, 33))


def n_params(layers=LAYERS):
    return sum(o * i + o for i, o in layers)


def unpack(flat, layers=LAYERS):
    """Flat vector -> list of (W [out][in], b [out])."""
    flat = np.asarray(flat, dtype=np.float64)
    out, k = [], 0
    for i, o in layers:
        W = flat[k:k + o * i].reshape(o, i)
        k += o * i
        b = flat[k:k + o]
        k += o
        out.append((W, b))
    if k != flat.size:
        raise ValueError("flat vector has the wrong length")
    return out


def pack(Wb):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in Wb])


# ------------------------------------------------------------------ rounding
def bf16(x):
    """Round to the nearest bfloat16 (ties to even) via the FP32 value; returns float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, quant):
    return bf16(x) if quant else np.asarray(x, dtype=np.float64)


# ------------------------------------------------------------------ activation
_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


# ------------------------------------------------------------------ features
def features(params, c_sat=1.5):
    """[n, 11] records -> [n, 10] features: log(1-omega), (1-omega), 8 factors (Sec. 4 law)."""
    p = np.atleast_2d(np.asarray(params, dtype=np.float64))
    t_days = p[:, 2] * mats.DAYS_PER_YEAR
    log_keep = -mats.gamma_of_c(p[:, 1], c_sat) * mats.alpha_of_T(p[:, 0]) * t_days
    return np.concatenate([log_keep[:, None], np.exp(log_keep)[:, None], p[:, 3:11]], axis=1)


def column_stats(A):
    """Per-column mean and population standard deviation (1 where a column is constant)."""
    A = np.asarray(A, dtype=np.float64)
    mu = A.mean(axis=0)
    sd = np.sqrt(((A - mu) ** 2).mean(axis=0))
    sd = np.where(sd > 0.0, sd, 1.0)
    return mu, sd


def targets(C, K, D):
    """Physical outputs [n, 33]."""
    return np.concatenate([np.asarray(C, float), np.asarray(K, float), np.asarray(D, float)], axis=1)


def encode(Y):
    """[n, 33] physical -> [n, 36]: per block log ||y||_F, then y / ||y||_F."""
    Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
    out = []
    for blk in BLOCKS:
        nrm = np.sqrt((OUT_WEIGHTS[blk] * Y[:, blk] ** 2).sum(axis=1))
        out += [np.log(nrm)[:, None], Y[:, blk] / nrm[:, None]]
    return np.concatenate(out, axis=1)


def decode(T):
    """[n, 36] encoded -> [n, 33] physical: exp(log norm) times the direction rescaled to unit norm."""
    T = np.atleast_2d(np.asarray(T, dtype=np.float64))
    out, k = [], 0
    for blk in BLOCKS:
        w = blk.stop - blk.start
        d = T[:, k + 1:k + 1 + w]
        dn = np.sqrt((OUT_WEIGHTS[blk] * d ** 2).sum(axis=1))
        out.append(np.exp(T[:, k])[:, None] * d / dn[:, None])
        k += 1 + w
    return np.concatenate(out, axis=1)


def standardise(A, mu, sd, quant):
    """(A - mu) / sd, held in FP32 (and rounded to bfloat16 when quant) as the kernels hold it."""
    z = ((np.asarray(A, dtype=np.float64) - mu) / sd).astype(np.float32).astype(np.float64)
    return _q(z, quant)


# ------------------------------------------------------------------ network
def forward(flat, xhat, quant=True):
    """Standardised encoded output [n, 36] and the cache the backward pass needs."""
    Wb = unpack(flat)
    a = np.asarray(xhat, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(Wb):
        Wq = _q(W, quant)
        z = a @ Wq.T + b
        cache.append((a, Wq, z))
        if li < len(Wb) - 1:
            a = _q(gelu(z), quant)
        else:
            a = z
    return a, cache


def loss_grad(flat, xhat, that, quant=True):
    """Mean squared error on standardised outputs and its gradient (flat layout)."""
    y, cache = forward(flat, xhat, quant)
    n = y.shape[0]
    diff = y - that
    loss = float(np.sum(diff * diff) / (n * N_OUT))
    g = _q(2.0 * diff / (n * N_OUT), quant)
    grads = [None] * len(cache)
    for li in range(len(cache) - 1, -1, -1):
        a_in, Wq, _ = cache[li]
        grads[li] = (g.T @ a_in, g.sum(axis=0))
        if li > 0:
            z_prev = cache[li - 1][2]
            g = _q((g @ Wq) * gelu_grad(z_prev), quant)
    return loss, pack(grads)


def adam_step(w, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict(members, x_mu, x_sd, y_mu, y_sd, params, c_sat=1.5, quant=True):
    """Ensemble mean in physical units [n, 33] and the disagreement [n].

    y_mu, y_sd standardise the encoded outputs (36 columns)."""
    xhat = standardise(features(params, c_sat), x_mu, x_sd, quant)
    outs = []
    for flat in members:
        y, _ = forward(flat, xhat, quant)
        outs.append(decode(y_mu + y_sd * y))
    Y = np.stack(outs)                                   # [M, n, 33]
    mean = Y.mean(axis=0)
    if len(members) > 1:
        s2 = Y.var(axis=0, ddof=1)
    else:
        s2 = np.zeros_like(mean)
    dis = np.zeros(mean.shape[0])
    for blk in BLOCKS:
        w = OUT_WEIGHTS[blk]
        num = np.sqrt((w * s2[:, blk]).sum(axis=1))
        den = np.sqrt((w * mean[:, blk] ** 2).sum(axis=1))
        dis = np.maximum(dis, num / den)
    return mean, dis


def block_errors(pred, ref):
    """Per point, the largest over C, K, D of ||pred - ref||_F / ||ref||_F (full symmetric matrices)."""
    pred = np.atleast_2d(pred)
    ref = np.atleast_2d(ref)
    err = np.zeros(pred.shape[0])
    for blk in BLOCKS:
        w = OUT_WEIGHTS[blk]
        num = np.sqrt((w * (pred[:, blk] - ref[:, blk]) ** 2).sum(axis=1))
        den = np.sqrt((w * ref[:, blk] ** 2).sum(axis=1))
        err = np.maximum(err, num / den)
    return err
