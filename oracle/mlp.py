"""FP64 oracle: the descriptor-MLP potential (not in the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per atom, features G (24, from ``oracle.descriptor``) are standardised,
g = (G - mu) / sd, zero-padded to 32, and mapped by a 32-64-64-1 network
with SiLU activations (silu(z) = z / (1 + exp(-z))):

  z1 = W1 g + b1,  h1 = silu(z1)
  z2 = W2 h1 + b2, h2 = silu(z2)
  y  = w3 . h2 + b3,   E_i = e_mean + e_sd * y

Weights are used exactly as given (the device keeps them in bfloat16; the
tests pass the same bf16-rounded values here in FP64).  The input gradient
dE_i/dG, the weight gradients of the standardised-energy loss
L = mean_i (y_i - t_i)^2 and one Adam step are written out by hand.
"""
from __future__ import annotations

import numpy as np

NIN, NPAD, NH = 24, 32, 64


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def standardise(G, mu, sd):
    g = np.zeros((G.shape[0], NPAD))
    g[:, :NIN] = (G - mu[None, :]) / sd[None, :]
    return g


def forward(params, g):
    """Returns y (N,) and the cache for backward."""
    z1 = g @ params["W1"].T + params["b1"]
    h1 = silu(z1)
    z2 = h1 @ params["W2"].T + params["b2"]
    h2 = silu(z2)
    y = h2 @ params["w3"] + params["b3"][0]
    return y, (g, z1, h1, z2, h2)


def input_grad(params, cache):
    """dy_i/dg_i (N, 32)."""
    g, z1, h1, z2, h2 = cache
    d2 = params["w3"][None, :] * dsilu(z2)
    d1 = (d2 @ params["W2"]) * dsilu(z1)
    return d1 @ params["W1"]


def energy_and_feature_grad(params, G, mu, sd, e_mean, e_sd):
    """Per-atom energies E_i and dE_i/dG_i (N, 24)."""
    g = standardise(G, mu, sd)
    y, cache = forward(params, g)
    dy = input_grad(params, cache)[:, :NIN]
    return e_mean + e_sd * y, dy * (e_sd / sd[None, :])


def loss_and_grads(params, g, t):
    """L = mean (y - t)^2 and dL/dparams."""
    y, (g, z1, h1, z2, h2) = forward(params, g)
    n = g.shape[0]
    r = y - t
    L = float(np.mean(r * r))
    dy = 2.0 * r / n
    grads = {}
    grads["w3"] = h2.T @ dy
    grads["b3"] = np.array([dy.sum()])
    d2 = dy[:, None] * params["w3"][None, :] * dsilu(z2)
    grads["W2"] = d2.T @ h1
    grads["b2"] = d2.sum(axis=0)
    d1 = (d2 @ params["W2"]) * dsilu(z1)
    grads["W1"] = d1.T @ g
    grads["b1"] = d1.sum(axis=0)
    return L, grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); state holds m, v and step t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    new = {}
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] * grads[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        new[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return new


def linear_fit(G, e):
    """Least-squares e ~ a . G + c (the method without the network)."""
    A = np.concatenate([G, np.ones((G.shape[0], 1))], axis=1)
    coef, *_ = np.linalg.lstsq(A, e, rcond=None)
    return coef[:-1], float(coef[-1])
