"""FP64 reference of the warm-start message-passing network.  TEST INFRASTRUCTURE ONLY.

The paper has no learned component; this network is the warm start that the
GPU library trains on CPAA outputs (inputs: log-degree and a one-hot source;
output: a probability vector x0 used as the CPAA starting guess).  Readings
(not in the paper): aggregation uses the paper's transition matrix
(M = P H = A D^{-1} H, the same neighbour weighting as Alg. 1's inner loop),
ReLU activations, a softmax over the graph's vertices of the score (so a
score of log d gives the degree-proportional stationary vector exactly).  Training minimises the cross-entropy -sum_u pi_u log x0_u
(the natural objective of a softmax output; its score gradient is
x0 sum(pi) - pi); the L1 distance sum_u |x0_u - pi_u| is the reported error.

    H^0      = [log d, 1{u = s}]                      (n x 2)
    M^l      = A D^{-1} H^l
    Z^l      = H^l W_self^l + M^l W_nbr^l + b^l      (n x hidden)
    H^{l+1}  = relu(Z^l)
    score    = H^L w_out + b_out
    x0       = exp(score - max score) / sum(exp(score - max score))
    loss     = -sum_u pi_u log x0_u          (error measure: sum_u |x0_u - pi_u|)

``bf16=True`` reproduces the GPU kernels' precision: weights, H and M are
rounded to bfloat16 (round to nearest even) before every product, products
accumulate in FP32 (here: FP64, which differs from FP32 only in rounding).

Parity status: forward/backward pinned by central finite differences and by
closed forms on tiny graphs (tests/test_oracle_mpnn.py); learning quality is
"parity unpinned" (no reference result exists).
"""
from __future__ import annotations

import numpy as np

from .cpaa_ref import adjacency

__all__ = ["bf16_round", "mpnn_features", "mpnn_forward", "mpnn_loss", "mpnn_l1",
           "mpnn_backward", "param_names", "adam_step"]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rnd = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rnd) & 0xFFFF0000).astype(np.uint32)
    out = u.view(np.float32).astype(np.float64)
    nonfinite = ~np.isfinite(f)
    out[nonfinite] = f[nonfinite]
    return out


def param_names(layers: int) -> list[str]:
    names = []
    for l in range(layers):
        names += [f"w_self{l}", f"w_nbr{l}", f"b{l}"]
    return names + ["w_out", "b_out"]


def mpnn_features(g, source: int) -> np.ndarray:
    d = np.diff(np.asarray(g.row_ptr, dtype=np.int64)).astype(np.float64)
    h0 = np.zeros((g.n, 2))
    h0[:, 0] = np.log(d)
    h0[source, 1] = 1.0
    return h0


def mpnn_forward(g, params: dict, source: int, layers: int = 3, bf16: bool = False):
    """Returns (x0, cache) for one source."""
    A = adjacency(g)
    d = np.diff(np.asarray(g.row_ptr, dtype=np.int64)).astype(np.float64)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    H = r(mpnn_features(g, source))
    cache = {"H": [H], "M": [], "Z": [], "d": d, "A": A}
    for l in range(layers):
        M = r(A @ (H / d[:, None]))
        Z = H @ r(params[f"w_self{l}"]) + M @ r(params[f"w_nbr{l}"]) + params[f"b{l}"]
        H = r(np.maximum(Z, 0.0))
        cache["M"].append(M)
        cache["Z"].append(Z)
        cache["H"].append(H)
    score = H @ r(params["w_out"]) + params["b_out"][0]
    y = np.exp(score - score.max())
    x0 = y / y.sum()
    cache.update(score=score, y=y, x0=x0)
    return x0, cache


def mpnn_loss(x0: np.ndarray, target: np.ndarray) -> float:
    """Cross-entropy -sum_u pi_u log x0_u (the training objective)."""
    return float(-(target * np.log(x0)).sum())


def mpnn_l1(x0: np.ndarray, target: np.ndarray) -> float:
    """L1 distance of the guess to the target (the reported error)."""
    return float(np.abs(x0 - target).sum())


def mpnn_backward(params: dict, cache: dict, target: np.ndarray, layers: int = 3,
                  bf16: bool = False) -> dict:
    """Gradient of the cross-entropy loss with respect to every parameter (FP64).

    Weights enter the forward pass as their (optionally bf16-rounded) values;
    the gradient is taken with respect to those values (straight-through).
    """
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    A, d = cache["A"], cache["d"]
    x0, score = cache["x0"], cache["score"]
    # d/ds_u of -sum_v pi_v log softmax(s)_v = x0_u sum(pi) - pi_u
    gs = x0 * target.sum() - target
    grads = {}
    HL = cache["H"][layers]
    grads["w_out"] = HL.T @ gs
    grads["b_out"] = np.array([gs.sum()])
    dH = np.outer(gs, r(params["w_out"]))
    for l in reversed(range(layers)):
        Z, H, M = cache["Z"][l], cache["H"][l], cache["M"][l]
        dZ = dH * (Z > 0.0)
        grads[f"w_self{l}"] = H.T @ dZ
        grads[f"w_nbr{l}"] = M.T @ dZ
        grads[f"b{l}"] = dZ.sum(axis=0)
        if l > 0:
            dM = dZ @ r(params[f"w_nbr{l}"]).T
            # M = A D^{-1} H  =>  dH += D^{-1} A^T dM, and A is symmetric
            dH = dZ @ r(params[f"w_self{l}"]).T + (A @ dM) / d[:, None]
    return grads


def adam_step(w: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1) in FP64.

    ``step`` counts updates already taken; the bias corrections use step + 1.
    Returns (w', m', v')."""
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    t = step + 1
    m_hat = m / (1.0 - b1**t)
    v_hat = v / (1.0 - b2**t)
    return np.asarray(w, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
