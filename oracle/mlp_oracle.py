"""Plain FP64 CPU oracle of the learned selection weights.

TEST INFRASTRUCTURE ONLY: imported by the test suite and the smoke check,
never by the product path.  Plain numpy in float64, written out step by step
so that each line can be checked by eye; it imports nothing from the HIP
package.

What it computes (the weights must stay positive and fixed before the chains
start, so that the Gibbs kernel keeps pi invariant and the coupled estimator
stays unbiased: Proposition 1, Theorem 1, Assumption 1; the floor is the one
of the score weights, Section "Score-Weighted Update Gibbs Sampler"):

  base logits: c_i = tau_w (s_i - s_max), the log-weights of the softmax
    part of the paper's score weights (s_i = sum_j d_j a_j, tau_w =
    log(100 n) / (s_max - s_min), 0 if all scores are equal);
  features x_i (8 per clone), from the design and the outcomes only:
    x0 = #positive pools of i / 8          x1 = #negative pools of i / 8
    x2 = mean size of its positive pools / 64 (0 if none)
    x3 = mean size of its negative pools / 64 (0 if none)
    x4 = smallest size of its positive pools / 64 (0 if none)
    x5 = c_i / 16, the normalised score     x6 = 10 fp      x7 = 10 fn
  network: f = W3 relu(W2 relu(W1 x + b1) + b2) + b3, widths 8-64-64-1,
    4801 parameters, used through their BF16 roundings (round to nearest,
    ties to even), the FP32 master copy being what the optimiser updates;
    the logits are c + f, so a network that outputs 0 gives back the
    score weights exactly;
  weights: w = (1 - alpha) softmax(c + f) + alpha / n;
  training target per instance: t_i ~ exp(beta c_i) (u_i + eps)^gamma with
    u = clip(v, 0, 1) for a per-clone signal v taken from the method's own
    outputs (its marginals, or the per-update scales SE_j sqrt(w_j) of its
    standard errors, over their maximum), normalised over the instance
    (beta = 1, gamma = 0 is the score softmax itself); the loss is
    the mean over instances of KL(t || softmax(c + f)); the optimiser is
    AdamW (Loshchilov and Hutter, decoupled weight decay) on every
    parameter.

Parameter layout (flat, 4801): W1 [64][8] (out, in), b1 [64], W2 [64][64],
b2 [64], W3 [64], b3 [1].
"""

from __future__ import annotations

import numpy as np

from . import oracle as O

F, H = 8, 64
SIZES = (("W1", H * F), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H), ("b3", 1))
N_PARAMS = sum(s for _, s in SIZES)   # 4801


def split(theta):
    """Views (W1, b1, W2, b2, W3, b3) of a flat parameter vector."""
    out, at = [], 0
    for name, size in SIZES:
        v = theta[at:at + size]
        at += size
        if name == "W1":
            v = v.reshape(H, F)
        elif name == "W2":
            v = v.reshape(H, H)
        out.append(v)
    return out


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32.  bfloat16 keeps the sign, the 8 exponent bits and the top 7
    fraction bits of a float32: the low 16 bits are dropped, and the kept
    part goes up by one unit when they exceed half a unit, or equal half a
    unit while the kept part is odd (a carry into the exponent is the
    correct result)."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    low = u & np.uint64(0xFFFF)
    kept = u - low
    odd = (kept >> np.uint64(16)) & np.uint64(1)
    up = (low > 0x8000) | ((low == 0x8000) & (odd == 1))
    r = kept + np.where(up, np.uint64(0x10000), np.uint64(0))
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)


def base_logits(inst):
    """c_i = tau_w (s_i - s_max) with the paper's tau_w (0 if all equal)."""
    s, _ = O.score_weights(inst)
    smin, smax = float(np.min(s)), float(np.max(s))
    tau = np.log(100.0 * inst.n) / (smax - smin) if smax > smin else 0.0
    return tau * (s - smax)


def features(inst):
    """[n, 8] float64 features of every clone (see the module docstring)."""
    n, m = inst.n, inst.m
    rp, pi, y = inst.row_ptr, inst.pool_idx, inst.y
    size = np.zeros(m, np.int64)
    for j in pi:
        size[j] += 1
    c = base_logits(inst)
    X = np.zeros((n, F))
    for i in range(n):
        pools = pi[rp[i]:rp[i + 1]]
        pos = [int(size[j]) for j in pools if y[j] == 1]
        neg = [int(size[j]) for j in pools if y[j] == 0]
        X[i, 0] = len(pos) / 8.0
        X[i, 1] = len(neg) / 8.0
        X[i, 2] = (sum(pos) / len(pos)) / 64.0 if pos else 0.0
        X[i, 3] = (sum(neg) / len(neg)) / 64.0 if neg else 0.0
        X[i, 4] = min(pos) / 64.0 if pos else 0.0
        X[i, 5] = c[i] / 16.0
        X[i, 6] = 10.0 * inst.fp
        X[i, 7] = 10.0 * inst.fn
    return X


def forward(theta_bf16, X):
    """Logits g [rows] and the intermediate values, in float64, from the
    BF16-rounded parameters (given as a flat float array)."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(v, np.float64) for v in split(np.asarray(theta_bf16))]
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    g = h2 @ W3 + b3[0]
    return g, dict(z1=z1, h1=h1, z2=z2, h2=h2)


def targets(signal, base, seg_ptr, beta, gamma, eps):
    """t per instance segment: exp(beta c) (u + eps)^gamma / sum, with
    u = clip(signal, 0, 1) and c the base logits."""
    u = np.clip(np.asarray(signal, np.float64), 0.0, 1.0)
    raw = np.exp(beta * np.asarray(base, np.float64)) * (u + eps) ** gamma
    t = np.empty_like(raw)
    for a, b in zip(seg_ptr[:-1], seg_ptr[1:]):
        t[a:b] = raw[a:b] / raw[a:b].sum()
    return t


def loss_and_dg(f, base, t, seg_ptr):
    """Mean over segments of KL(t || softmax(c + f)) and its gradient in the
    network output f: (softmax(c + f) - t) / #segments on each segment (t
    sums to 1 on it)."""
    S = len(seg_ptr) - 1
    loss = 0.0
    g = np.asarray(base, np.float64) + np.asarray(f, np.float64)
    dg = np.zeros_like(g)
    for a, b in zip(seg_ptr[:-1], seg_ptr[1:]):
        ga = g[a:b]
        mx = ga.max()
        e = np.exp(ga - mx)
        Z = e.sum()
        p = e / Z
        logp = ga - mx - np.log(Z)
        ts = t[a:b]
        loss += float(np.sum(ts * (np.log(ts) - logp)))
        dg[a:b] = (p - ts) / S
    return loss / S, dg


def backward(theta_bf16, X, dg):
    """Gradient of sum_i dg_i g_i with respect to the flat parameters
    (through the BF16 values, i.e. the straight-through gradient that the
    FP32 master copy receives)."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(v, np.float64) for v in split(np.asarray(theta_bf16))]
    X = np.asarray(X, np.float64)
    g, c = forward(theta_bf16, X)
    dg = np.asarray(dg, np.float64)
    dW3 = c["h2"].T @ dg
    db3 = np.array([dg.sum()])
    dz2 = np.outer(dg, W3) * (c["z2"] > 0)
    dW2 = dz2.T @ c["h1"]
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (c["z1"] > 0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, db3])


def adamw_step(theta, m, v, grad, step, lr, beta1, beta2, eps, wd):
    """One AdamW step (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta - lr * (mhat / (np.sqrt(vhat) + eps) + wd * theta)
    return theta, m, v


def selection_weights(f, base, alpha=0.5):
    """w = (1 - alpha) softmax(c + f) + alpha / n."""
    g = np.asarray(base, np.float64) + np.asarray(f, np.float64)
    e = np.exp(g - g.max())
    return (1.0 - alpha) * e / e.sum() + alpha / len(g)
