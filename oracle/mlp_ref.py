"""Reference (float64, numpy) of the packing cost model: a 16-64-64-1
multilayer perceptron with ReLU, trained by mean squared error and Adam.

TEST INFRASTRUCTURE ONLY: used by the test suite to check the library's GPU
forward, backward and Adam kernels. It shares no code with the library.

Parameter vector (same layout as the library):
  x_mean[16] x_std[16] W1[64][16] b1[64] W2[64][64] b2[64] W3[64] b3 y_mean y_std
The input is log(1 + x) standardised with (x_mean, x_std); the output y is in
standardised units, y * y_std + y_mean is the prediction of log(time).
Loss: mean over samples of (y - (t - y_mean)/y_std)^2. Gradients of the
standardisation entries are zero (they are fixed, not trained).
"""
from __future__ import annotations

import numpy as np

F, H1, H2 = 16, 64, 64
OXM, OXS = 0, 16
OW1 = 32
OB1 = OW1 + H1 * F
OW2 = OB1 + H1
OB2 = OW2 + H2 * H1
OW3 = OB2 + H2
OB3 = OW3 + H2
OYM = OB3 + 1
OYS = OYM + 1
NP = OYS + 1


def unpack(p):
    p = np.asarray(p, np.float64)
    return dict(xm=p[OXM:OXS], xs=p[OXS:OW1], W1=p[OW1:OB1].reshape(H1, F),
                b1=p[OB1:OW2], W2=p[OW2:OB2].reshape(H2, H1), b2=p[OB2:OW3],
                W3=p[OW3:OB3], b3=p[OB3], ym=p[OYM], ys=p[OYS])


def forward(p, x):
    """Returns (prediction of log time, cache for backward)."""
    q = unpack(p)
    u = (np.log1p(np.asarray(x, np.float64)) - q["xm"]) / q["xs"]
    z1 = u @ q["W1"].T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ q["W3"] + q["b3"]
    return y * q["ys"] + q["ym"], (u, z1, h1, z2, h2, y)


def loss(p, x, t):
    q = unpack(p)
    _, (u, z1, h1, z2, h2, y) = forward(p, x)
    ts = (np.asarray(t, np.float64) - q["ym"]) / q["ys"]
    return float(np.mean((y - ts) ** 2))


def loss_grad(p, x, t):
    """Loss and its gradient by reverse-mode differentiation of the network."""
    q = unpack(p)
    n = x.shape[0]
    _, (u, z1, h1, z2, h2, y) = forward(p, x)
    ts = (np.asarray(t, np.float64) - q["ym"]) / q["ys"]
    err = y - ts
    L = float(np.mean(err ** 2))
    dy = 2.0 * err / n                       # dL/dy
    g = np.zeros(NP)
    g[OW3:OB3] = dy @ h2
    g[OB3] = dy.sum()
    dz2 = np.outer(dy, q["W3"]) * (z2 > 0)   # dL/dz2
    g[OW2:OB2] = (dz2.T @ h1).ravel()
    g[OB2:OW3] = dz2.sum(0)
    dz1 = (dz2 @ q["W2"]) * (z1 > 0)
    g[OW1:OB1] = (dz1.T @ u).ravel()
    g[OB1:OW2] = dz1.sum(0)
    return L, g


def adam(p, x, t, epochs, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Full-batch Adam on the trainable entries (W1 .. b3)."""
    p = np.array(p, np.float64)
    m = np.zeros(NP)
    v = np.zeros(NP)
    sl = slice(OW1, OB3 + 1)
    for k in range(1, epochs + 1):
        _, g = loss_grad(p, x, t)
        m[sl] = b1 * m[sl] + (1 - b1) * g[sl]
        v[sl] = b2 * v[sl] + (1 - b2) * g[sl] ** 2
        mh = m[sl] / (1 - b1 ** k)
        vh = v[sl] / (1 - b2 ** k)
        p[sl] -= lr * mh / (np.sqrt(vh) + eps)
    return p


def init(x, t, seed=0):
    """Standardisation from the data and small random weights (the library
    uses its own generator; tests that compare the two pass parameters)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NP)
    lx = np.log1p(np.asarray(x, np.float64))
    p[OXM:OXS] = lx.mean(0)
    sd = lx.std(0)
    p[OXS:OW1] = np.where(sd > 1e-6, sd, 1.0)
    p[OW1:OB1] = rng.uniform(-1, 1, H1 * F) * np.sqrt(6.0 / F)
    p[OW2:OB2] = rng.uniform(-1, 1, H2 * H1) * np.sqrt(6.0 / H1)
    p[OW3:OB3] = rng.uniform(-1, 1, H2) * np.sqrt(6.0 / H2)
    p[OYM] = float(np.mean(t))
    sdt = float(np.std(t))
    p[OYS] = sdt if sdt > 1e-6 else 1.0
    return p
