"""ORACLE -- test infrastructure. The learned scatter-mode selector in FP64.

What the library's selector computes, written from its definitions for
checking only:

* the 12 per-partition features (vertex and edge counts of the partition and
  its active part, the partition's message ratio r^p = M^p / E^p from message
  generation, Sec. 3.1.2, bin fill, degree skew, iteration, the global active
  edge fraction, and the log ratio of the two byte counts compared by Eq. 1,
  Sec. 3.2);
* the network 12 -> 64 -> 64 -> 1 with ReLU, evaluated in FP64 on weights
  rounded to bf16 (round to nearest even) and on FP32 standardisation
  constants; and as the per-iteration selection evaluates it, with the input
  of each hidden layer rounded to bf16 (forward_infer), and which samples
  hold a value so close to a bf16 rounding midpoint that an FP32 difference
  could round it the other way (infer_ambiguous);
* the regret-weighted binary cross-entropy (label: partition-centric was
  faster; weight: |t_SC - t_PC|) and its exact gradient with respect to the
  bf16 weights, by hand-written backpropagation;
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP64 masters.

Parameter order: W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3.
"""
from __future__ import annotations

import math
from typing import Dict, Iterable, Tuple

import numpy as np

N_IN, N_H = 12, 64
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1   # 5057
OFF_W1, OFF_B1 = 0, N_H * N_IN
OFF_W2 = OFF_B1 + N_H
OFF_B2 = OFF_W2 + N_H * N_H
OFF_W3 = OFF_B2 + N_H
OFF_B3 = OFF_W3 + N_H


# ---------------------------------------------------------------------------
# bf16
# ---------------------------------------------------------------------------
def bf16_round(x) -> np.ndarray:
    """Rounds float32 values to the nearest bf16 value (ties to even) and
    returns them as float64. NaN stays NaN."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    t = np.asarray(theta, dtype=np.float64)
    return {
        "W1": t[OFF_W1:OFF_B1].reshape(N_H, N_IN),
        "b1": t[OFF_B1:OFF_W2],
        "W2": t[OFF_W2:OFF_B2].reshape(N_H, N_H),
        "b2": t[OFF_B2:OFF_W3],
        "w3": t[OFF_W3:OFF_B3],
        "b3": t[OFF_B3],
    }


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------
def partition_stats(offsets, cols, q: int):
    """E^p, M^p (messages when every vertex is active: one per vertex and
    neighbouring partition), non-empty bins of row p, and max out-degree of
    each index-range partition of q vertices."""
    n = len(offsets) - 1
    k = max(1, -(-n // q))
    Ep = [0] * k
    Mp = [0] * k
    rows = [set() for _ in range(k)]
    maxd = [0] * k
    for v in range(n):
        p = v // q
        a, b = int(offsets[v]), int(offsets[v + 1])
        Ep[p] += b - a
        maxd[p] = max(maxd[p], b - a)
        parts = {int(cols[e]) // q for e in range(a, b)}
        Mp[p] += len(parts)
        rows[p] |= parts
    return Ep, Mp, [len(r) for r in rows], maxd


def features(offsets, cols, q: int, frontier: Iterable[int], it: int, s_i: int = 4,
             s_v: int = 4) -> np.ndarray:
    """k x 12 FP64 features of the frontier `frontier` at iteration `it`."""
    n = len(offsets) - 1
    m = int(offsets[-1])
    k = max(1, -(-n // q))
    Ep, Mp, nzb, maxd = partition_stats(offsets, cols, q)
    Va = [0] * k
    Ea = [0] * k
    for v in set(int(x) for x in frontier):
        Va[v // q] += 1
        Ea[v // q] += int(offsets[v + 1]) - int(offsets[v])
    frac = sum(Ea) / m if m else 0.0
    out = np.zeros((k, N_IN))
    for p in range(k):
        nv = min(q, n - p * q)
        E, M = Ep[p], Mp[p]
        mean_deg = E / nv
        cost_pc = (M + E) * s_i + 2.0 * M * s_v + k * s_i
        cost_sc = (2.0 * s_v * M * Ea[p] / E if E else 0.0) + (3.0 * Ea[p] + Va[p]) * s_i
        out[p] = [
            math.log1p(Va[p]), math.log1p(Ea[p]), math.log1p(E), math.log1p(M),
            M / E if E else 0.0,
            Va[p] / nv,
            Ea[p] / E if E else 0.0,
            nzb[p] / k,
            math.log(maxd[p] / mean_deg) if E else 0.0,
            math.log1p(it),
            frac,
            math.log(cost_pc / cost_sc) if cost_sc > 0 else 0.0,
        ]
    return out


def standardisation(X) -> Tuple[np.ndarray, np.ndarray]:
    """Mean and 1 / max(population std, 1e-6) of each feature column."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = np.sqrt(((X - mu) ** 2).mean(axis=0))
    return mu, 1.0 / np.maximum(sd, 1e-6)


# ---------------------------------------------------------------------------
# Network, loss, gradient
# ---------------------------------------------------------------------------
def _layers(theta_bf16, mean, inv_std, X):
    P = unpack(theta_bf16)
    Xh = (np.asarray(X, dtype=np.float64) - np.asarray(mean, np.float64)) * np.asarray(inv_std, np.float64)
    Z1 = Xh @ P["W1"].T + P["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ P["W2"].T + P["b2"]
    H2 = np.maximum(Z2, 0.0)
    z = H2 @ P["w3"] + P["b3"]
    return P, Xh, Z1, H1, Z2, H2, z


def forward(theta_bf16, mean, inv_std, X) -> np.ndarray:
    """Logits of the samples X (n x 12 raw features)."""
    return _layers(theta_bf16, mean, inv_std, X)[-1]


def forward_infer(theta_bf16, mean, inv_std, X) -> np.ndarray:
    """Logits as the per-iteration mode selection evaluates the network: the
    input of each hidden layer is rounded to bf16 (ties to even) -- the
    standardised features (taken to FP32 first, as the device computes them;
    b1 multiplies an exact 1) and the first hidden layer after its ReLU.
    Products and sums in FP64."""
    P = unpack(theta_bf16)
    xs = (np.asarray(X, dtype=np.float64) - np.asarray(mean, np.float64)) * np.asarray(inv_std, np.float64)
    Xh = bf16_round(xs.astype(np.float32))
    H1 = bf16_round(np.maximum(Xh @ P["W1"].T + P["b1"], 0.0).astype(np.float32))
    H2 = np.maximum(H1 @ P["W2"].T + P["b2"], 0.0)
    return H2 @ P["w3"] + P["b3"]


def infer_ambiguous(theta_bf16, mean, inv_std, X, rel_x: float = 1e-5, rel_h: float = 1e-6) -> np.ndarray:
    """Per sample: True if one of the values forward_infer rounds to bf16 lies
    so close to a rounding midpoint that another evaluation could round it
    the other way: a standardised feature within rel_x of the magnitudes it
    is made of (plus rel_x absolute on the raw feature: features computed in
    FP32 agree to a few 1e-6), a first-layer sum within rel_h of the sum of
    its terms' magnitudes (13 FP32 additions err by at most 13 * 2^-24 of
    that). Elsewhere every rounding is the same on both sides and the logits
    differ by FP32 summation only."""
    P = unpack(theta_bf16)
    Xr = np.asarray(X, dtype=np.float64)
    mu, iv = np.asarray(mean, np.float64), np.asarray(inv_std, np.float64)
    xs = (Xr - mu) * iv
    e0 = rel_x * (np.abs(Xr) + np.abs(mu) + 1.0) * np.abs(iv)

    def flips(v, e):
        lo = bf16_round((v - e).astype(np.float32))
        hi = bf16_round((v + e).astype(np.float32))
        return lo != hi

    amb = np.any(flips(xs, e0), axis=1)
    Xh = bf16_round(xs.astype(np.float32))
    pre = Xh @ P["W1"].T + P["b1"]
    e1 = rel_h * (np.abs(Xh) @ np.abs(P["W1"]).T + np.abs(P["b1"]))
    amb |= np.any(flips(np.maximum(pre, 0.0), e1) & (pre + e1 > 0), axis=1)
    return amb


def loss_and_grad(theta_bf16, mean, inv_std, X, t_sc, t_pc):
    """L = sum_n c_n l_n / sum_n c_n with c_n = |t_SC - t_PC|,
    y_n = [t_PC < t_SC], l_n = softplus(z_n) - y_n z_n; and dL/dtheta."""
    P, Xh, Z1, H1, Z2, H2, z = _layers(theta_bf16, mean, inv_std, X)
    t_sc = np.asarray(t_sc, np.float64)
    t_pc = np.asarray(t_pc, np.float64)
    c = np.abs(t_sc - t_pc)
    y = (t_pc < t_sc).astype(np.float64)
    C = c.sum()
    if C == 0:
        return 0.0, np.zeros(N_PARAMS)
    softplus = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    L = float((c * (softplus - y * z)).sum() / C)
    g = c * (1.0 / (1.0 + np.exp(-z)) - y) / C          # dL/dz
    D2 = np.outer(g, P["w3"]) * (Z2 > 0)                 # dL/dZ2
    D1 = (D2 @ P["W2"]) * (Z1 > 0)                       # dL/dZ1
    grad = np.zeros(N_PARAMS)
    grad[OFF_W1:OFF_B1] = (D1.T @ Xh).ravel()
    grad[OFF_B1:OFF_W2] = D1.sum(axis=0)
    grad[OFF_W2:OFF_B2] = (D2.T @ H1).ravel()
    grad[OFF_B2:OFF_W3] = D2.sum(axis=0)
    grad[OFF_W3:OFF_B3] = H2.T @ g
    grad[OFF_B3] = g.sum()
    return L, grad


def adam_step(master, m, v, grad, step: int, lr: float):
    """One Adam step; returns the new (master, m, v)."""
    m = 0.9 * np.asarray(m, np.float64) + 0.1 * grad
    v = 0.999 * np.asarray(v, np.float64) + 0.001 * grad * grad
    mh = m / (1.0 - 0.9 ** step)
    vh = v / (1.0 - 0.999 ** step)
    return np.asarray(master, np.float64) - lr * mh / (np.sqrt(vh) + 1e-8), m, v
