"""FP64 reference of the learned control variate's network (test infrastructure only).

Network r_theta (coarse final field -> prediction of the level correction Y):
    conv 3x3, 1 -> 16 channels, circular padding, ReLU
    conv 3x3, 16 -> 16, circular padding, ReLU
    conv 3x3, 16 -> 16, circular padding, ReLU
    global average pool -> 16
    dense 16 -> 64, ReLU
    dense 64 -> 1
Loss: mean squared error over the batch, L = mean_b (r_b - y_b)^2.

The convolution is a cross-correlation: out[o, y, x] = b[o] + sum_{c, dy, dx} W[o, c, dy+1, dx+1]
in[c, (y+dy) mod n, (x+dx) mod n].  Forward and backward are written out plainly with numpy
(no autograd); the tests pin the backward pass with finite differences.
"""
from __future__ import annotations

import numpy as np

SHAPES = {
    "W1": (16, 1, 3, 3), "b1": (16,),
    "W2": (16, 16, 3, 3), "b2": (16,),
    "W3": (16, 16, 3, 3), "b3": (16,),
    "U1": (64, 16), "c1": (64,),
    "U2": (1, 64), "c2": (1,),
}
ORDER = ["W1", "b1", "W2", "b2", "W3", "b3", "U1", "c1", "U2", "c2"]


def n_params() -> int:
    return int(sum(np.prod(SHAPES[k]) for k in ORDER))


def init_params(seed: int = 0) -> dict:
    """He-style initialisation from a seeded numpy generator."""
    rng = np.random.default_rng(seed)
    p = {}
    for k in ORDER:
        s = SHAPES[k]
        if k.startswith(("W", "U")):
            fan_in = int(np.prod(s[1:]))
            p[k] = rng.standard_normal(s) * np.sqrt(2.0 / fan_in)
        else:
            p[k] = np.zeros(s)
    return p


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in ORDER])


def unflatten(v: np.ndarray) -> dict:
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = v[o:o + n].reshape(SHAPES[k]).astype(np.float64)
        o += n
    return out


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x [B, C, n, n] -> [B, O, n, n], circular 3x3 cross-correlation."""
    out = np.zeros((x.shape[0], W.shape[0], x.shape[2], x.shape[3]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            xs = np.roll(x, shift=(-dy, -dx), axis=(2, 3))      # xs[.., y, x] = x[.., y+dy, x+dx]
            out += np.einsum("oc,bcyx->boyx", W[:, :, dy + 1, dx + 1], xs)
    return out + b[None, :, None, None]


def conv_backward(x: np.ndarray, W: np.ndarray, dout: np.ndarray):
    """Gradients of conv() with respect to x, W and b."""
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    for dy in (-1, 0, 1):
        for dx_ in (-1, 0, 1):
            xs = np.roll(x, shift=(-dy, -dx_), axis=(2, 3))
            dW[:, :, dy + 1, dx_ + 1] = np.einsum("boyx,bcyx->oc", dout, xs)
            contrib = np.einsum("oc,boyx->bcyx", W[:, :, dy + 1, dx_ + 1], dout)
            dx += np.roll(contrib, shift=(dy, dx_), axis=(2, 3))
    db = dout.sum(axis=(0, 2, 3))
    return dx, dW, db


def forward(p: dict, x: np.ndarray, keep: bool = False):
    """x [B, n, n] -> r [B] (and the activations when keep)."""
    a0 = x[:, None, :, :].astype(np.float64)
    z1 = conv(a0, p["W1"], p["b1"]); a1 = np.maximum(z1, 0)
    z2 = conv(a1, p["W2"], p["b2"]); a2 = np.maximum(z2, 0)
    z3 = conv(a2, p["W3"], p["b3"]); a3 = np.maximum(z3, 0)
    g = a3.mean(axis=(2, 3))
    h1 = g @ p["U1"].T + p["c1"]; a4 = np.maximum(h1, 0)
    r = (a4 @ p["U2"].T + p["c2"])[:, 0]
    if keep:
        return r, dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, g=g, h1=h1, a4=a4)
    return r


def loss_and_grad(p: dict, x: np.ndarray, y: np.ndarray):
    r, A = forward(p, x, keep=True)
    B = len(y)
    loss = float(np.mean((r - y) ** 2))
    dr = 2.0 * (r - y) / B
    g = {}
    g["U2"] = dr[None, :] @ A["a4"]
    g["c2"] = np.array([dr.sum()])
    da4 = dr[:, None] * p["U2"][0][None, :]
    dh1 = da4 * (A["h1"] > 0)
    g["U1"] = dh1.T @ A["g"]
    g["c1"] = dh1.sum(axis=0)
    dg = dh1 @ p["U1"]
    n2 = A["a3"].shape[2] * A["a3"].shape[3]
    da3 = np.broadcast_to(dg[:, :, None, None] / n2, A["a3"].shape)
    dz3 = da3 * (A["z3"] > 0)
    da2, g["W3"], g["b3"] = conv_backward(A["a2"], p["W3"], dz3)
    dz2 = da2 * (A["z2"] > 0)
    da1, g["W2"], g["b2"] = conv_backward(A["a1"], p["W2"], dz2)
    dz1 = da1 * (A["z1"] > 0)
    _, g["W1"], g["b1"] = conv_backward(A["a0"], p["W1"], dz1)
    return loss, g


def adam_step(p: dict, g: dict, state: dict, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """Adam (Kingma & Ba 2015) with bias correction, in place."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in ORDER:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
