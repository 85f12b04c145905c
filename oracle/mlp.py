"""Oracle for the learned Metropolis proposal (test infrastructure only).

The paper's sampler proposes single-bit flips (Sec. "Heuristic Metropolis
simulator").  The learned proposal is a flip-mask distribution from a small
MLP f: {0,1}^n -> R^n (n -> H -> H -> n, ReLU), mixed with the single-bit
flip at weight eps, and corrected by Metropolis-Hastings with the exact
amplitude ratio, so the chain's stationary law is the paper's P(x):

  pi_j(x) = clip(sigmoid(f(x)_j), pi_min, pi_max)
  q(y|x)  = eps [|m| = 1] / n + (1 - eps) prod_j pi_j(x)^{m_j} (1 - pi_j(x))^{1 - m_j},  m = x ^ y
  accept iff U < (P(y) q(x|y)) / (P(x) q(y|x)).

Features: s_j = 1 - 2 x_j.  Precision mirrors the GPU's BF16 matrix-core path:
weights, inputs, activations and back-propagated gradients are rounded to
bfloat16 (round to nearest even) where they enter a product; every sum is
FP32 (the oracle sums in float64 and rounds, which bounds the difference to
the GPU's summation order).  `exact=True` runs everything in float64 without
rounding, for the finite-difference pin of the backward pass.

Loss: binary cross-entropy with logits against target flip bits t,
L = mean_{b, j} softplus(l_bj) - t_bj l_bj.  Optimiser: Adam
(beta1 0.9, beta2 0.999, eps 1e-8), FP32 master weights.
"""
from __future__ import annotations

import numpy as np

PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def bf16(a):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), np.float32(np.nan), out).astype(np.float32)


def features(x, n):
    x = np.asarray(x, dtype=np.uint64)
    bits = ((x[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.float32)
    return 1.0 - 2.0 * bits


def bits_of(x, n):
    x = np.asarray(x, dtype=np.uint64)
    return ((x[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.float32)


def pack(params):
    return np.concatenate([np.asarray(params[k], np.float32).ravel() for k in PARAM_ORDER])


def unpack(flat, n, H):
    shapes = {"W1": (H, n), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (n, H), "b3": (n,)}
    out, off = {}, 0
    for k in PARAM_ORDER:
        size = int(np.prod(shapes[k]))
        out[k] = np.asarray(flat[off: off + size], np.float32).reshape(shapes[k]).copy()
        off += size
    return out


class MLPRef:
    def __init__(self, params, n, H):
        self.n, self.H = n, H
        self.p = {k: np.asarray(v, np.float32).copy() for k, v in params.items()}
        self.m = {k: np.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: np.zeros_like(v) for k, v in self.p.items()}
        self.t = 0

    # ---- forward ----
    def forward(self, x, exact=False):
        """Logits [B, n] and the cache for backward."""
        p = self.p
        rnd = (lambda a: np.asarray(a, np.float64)) if exact else (lambda a: bf16(a).astype(np.float64))
        dt = np.float64
        a0 = rnd(features(x, self.n))
        z1 = a0 @ rnd(p["W1"]).T + p["b1"].astype(dt)
        if not exact:
            z1 = z1.astype(np.float32).astype(dt)
        h1 = np.maximum(z1, 0.0)
        a1 = rnd(h1.astype(np.float32)) if not exact else h1
        z2 = a1 @ rnd(p["W2"]).T + p["b2"].astype(dt)
        if not exact:
            z2 = z2.astype(np.float32).astype(dt)
        h2 = np.maximum(z2, 0.0)
        a2 = rnd(h2.astype(np.float32)) if not exact else h2
        l = a2 @ rnd(p["W3"]).T + p["b3"].astype(dt)
        if not exact:
            l = l.astype(np.float32)
        cache = dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, l=np.asarray(l, np.float64))
        return np.asarray(l), cache

    # ---- loss and backward ----
    def loss_and_grad(self, x, target, exact=False):
        """BCE-with-logits loss and gradients of every parameter (same shapes)."""
        p = self.p
        rnd = (lambda a: np.asarray(a, np.float64)) if exact else (lambda a: bf16(a).astype(np.float64))
        l, c = self.forward(x, exact)
        l = np.asarray(l, np.float64)
        t = bits_of(target, self.n).astype(np.float64)
        B = l.shape[0]
        loss = float(np.mean(np.logaddexp(0.0, l) - t * l))
        sig = 1.0 / (1.0 + np.exp(-l))
        g = (sig - t) / (B * self.n)
        if not exact:
            g = g.astype(np.float32).astype(np.float64)
        grads = {}
        gb = rnd(g.astype(np.float32)) if not exact else g
        grads["W3"] = gb.T @ c["a2"]
        grads["b3"] = g.sum(axis=0)
        dA2 = gb @ rnd(p["W3"])
        dZ2 = dA2 * (c["z2"] > 0)
        if not exact:
            dZ2 = dZ2.astype(np.float32).astype(np.float64)
        gz2 = rnd(dZ2.astype(np.float32)) if not exact else dZ2
        grads["W2"] = gz2.T @ c["a1"]
        grads["b2"] = dZ2.sum(axis=0)
        dA1 = gz2 @ rnd(p["W2"])
        dZ1 = dA1 * (c["z1"] > 0)
        if not exact:
            dZ1 = dZ1.astype(np.float32).astype(np.float64)
        gz1 = rnd(dZ1.astype(np.float32)) if not exact else dZ1
        grads["W1"] = gz1.T @ c["a0"]
        grads["b1"] = dZ1.sum(axis=0)
        dt = np.float64 if exact else np.float32
        return loss, {k: np.asarray(v, dt) for k, v in grads.items()}

    def loss(self, x, target, exact=False):
        l, _ = self.forward(x, exact)
        l = np.asarray(l, np.float64)
        t = bits_of(target, self.n).astype(np.float64)
        return float(np.mean(np.logaddexp(0.0, l) - t * l))

    def adam_step(self, grads, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        for k in PARAM_ORDER:
            g = np.asarray(grads[k], np.float32)
            self.m[k] = (beta1 * self.m[k] + (1 - beta1) * g).astype(np.float32)
            self.v[k] = (beta2 * self.v[k] + (1 - beta2) * g * g).astype(np.float32)
            mh = self.m[k] / (1 - beta1 ** self.t)
            vh = self.v[k] / (1 - beta2 ** self.t)
            self.p[k] = (self.p[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)

    # ---- proposal ----
    def flip_probs(self, x, pi_min, pi_max):
        l, _ = self.forward(x)
        l = np.asarray(l, np.float32)
        pi = (np.float32(1.0) / (np.float32(1.0) + np.exp(-l))).astype(np.float32)
        return np.clip(pi, np.float32(pi_min), np.float32(pi_max)).astype(np.float32)


def log_q(pi, m_bits, eps, n):
    """log q(y|x) for flip mask m (bits [n]) under flip probabilities pi [n]:
    q = eps [|m| = 1] / n + (1 - eps) prod_j pi_j^{m_j} (1 - pi_j)^{1 - m_j},
    evaluated as a log-sum-exp of the two terms' logs (a zero term is -inf),
    so that a product far below the smallest double keeps its exact log."""
    pi = pi.astype(np.float64)
    eps = float(eps)
    lp = float(np.where(m_bits > 0, np.log(pi), np.log1p(-pi)).sum())
    a = np.log(eps / n) if (int(m_bits.sum()) == 1 and eps > 0.0) else -np.inf
    b = np.log1p(-eps) + lp if eps < 1.0 else -np.inf
    return float(np.logaddexp(a, b))


def learned_chain(terms, mlp: MLPRef, x0, u_mix, jstream, u_bits, ustream, eps, pi_min, pi_max,
                  tie=1e-5):
    """Reference chain with the learned proposal.

    terms: an oracle Terms object (amplitudes by its exact evaluation).
    Random inputs per chain c and step t: u_mix[c,t] (< eps: single flip at
    jstream[c,t]), u_bits[c,t,j] (flip j iff u_bits < pi_j(x)), ustream[c,t].
    Returns (trace, accepted, flips, first_near_tie_step per chain): a near tie
    is |u_bits - pi| < tie or |U - r| < tie * r, where two correct
    implementations may decide differently after rounding."""
    n = mlp.n
    C, T = jstream.shape
    trace = np.zeros((C, T), np.uint64)
    acc = np.zeros((C, T), np.uint8)
    flips = np.zeros((C, T), np.uint32)
    first_tie = np.full(C, T, np.int64)
    for c in range(C):
        x = int(x0[c])
        ax = terms.amplitudes(np.array([x], np.uint64))[0]
        for t in range(T):
            pi_x = mlp.flip_probs(np.array([x], np.uint64), pi_min, pi_max)[0]
            if u_mix[c, t] < eps:
                m = np.zeros(n, np.float32)
                m[int(jstream[c, t])] = 1
            else:
                if np.min(np.abs(u_bits[c, t, :n] - pi_x)) < tie and first_tie[c] == T:
                    first_tie[c] = t
                m = (u_bits[c, t, :n] < pi_x).astype(np.float32)
            mask = int(sum(1 << j for j in range(n) if m[j]))
            flips[c, t] = int(m.sum())
            if mask == 0:
                trace[c, t] = x
                acc[c, t] = 1
                continue
            y = x ^ mask
            pi_y = mlp.flip_probs(np.array([y], np.uint64), pi_min, pi_max)[0]
            ay = terms.amplitudes(np.array([y], np.uint64))[0]
            r = (abs(ay) ** 2 / abs(ax) ** 2) * np.exp(log_q(pi_y, m, eps, n) - log_q(pi_x, m, eps, n))
            U = ustream[c, t]
            if abs(U - r) < tie * max(r, 1e-300) and first_tie[c] == T:
                first_tie[c] = t
            if U < r:
                x, ax = y, ay
                acc[c, t] = 1
            trace[c, t] = x
    return trace, acc, flips, first_tie
