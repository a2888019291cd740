"""O3: FP64 reference of the learned inverse-square-root initial guess -- test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg may import
this module.  It shares no code with the HIP path.

The network (an addition to the paper's method: it supplies the initial guess of the
inverse square root that Alg. 2 line 5 needs) maps a normalised input z = (u - m)/s
through  h1 = W1 z + b1,  a1 = h1^2,  h2 = W2 a1 + b2,  a2 = h2^2,  y = W3 . a2 + b3
with 16 hidden units per layer, so y is a degree-4 polynomial of u.  The training loss is
the mean squared relative error  (y sqrt(u) - 1)^2.

Parameter vector layout (321 values): W1[16], b1[16], W2[16][16] (row = output unit),
b2[16], W3[16], b3.
"""
from __future__ import annotations

import numpy as np

H = 16
NPARAM = H + H + H * H + H + H + 1


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = t[o:o + H]; o += H
    b1 = t[o:o + H]; o += H
    W2 = t[o:o + H * H].reshape(H, H); o += H * H
    b2 = t[o:o + H]; o += H
    W3 = t[o:o + H]; o += H
    b3 = t[o]
    return W1, b1, W2, b2, W3, b3


def forward(theta, u, m, s):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z = (np.asarray(u, dtype=np.float64) - m) / s
    h1 = np.outer(z, W1) + b1
    a1 = h1 * h1
    h2 = a1 @ W2.T + b2
    a2 = h2 * h2
    return a2 @ W3 + b3


def loss(theta, u, m, s):
    y = forward(theta, u, m, s)
    r = y * np.sqrt(u) - 1.0
    return float(np.mean(r * r))


def grad(theta, u, m, s):
    """Analytic gradient of loss() by the chain rule, layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    u = np.asarray(u, dtype=np.float64)
    B = u.size
    z = (u - m) / s
    h1 = np.outer(z, W1) + b1
    a1 = h1 * h1
    h2 = a1 @ W2.T + b2
    a2 = h2 * h2
    y = a2 @ W3 + b3
    su = np.sqrt(u)
    dy = 2.0 * (y * su - 1.0) * su / B
    gW3 = a2.T @ dy
    gb3 = dy.sum()
    da2 = np.outer(dy, W3)
    dh2 = da2 * 2.0 * h2
    gW2 = dh2.T @ a1
    gb2 = dh2.sum(axis=0)
    da1 = dh2 @ W2
    dh1 = da1 * 2.0 * h1
    gW1 = dh1.T @ z
    gb1 = dh1.sum(axis=0)
    return np.concatenate([gW1, gb1, gW2.ravel(), gb2, gW3, [gb3]])


def fd_grad(theta, u, m, s, eps=1e-6):
    """Central finite differences of loss() (pins grad())."""
    t = np.asarray(theta, dtype=np.float64).copy()
    g = np.empty_like(t)
    for i in range(t.size):
        old = t[i]
        t[i] = old + eps
        lp = loss(t, u, m, s)
        t[i] = old - eps
        lm = loss(t, u, m, s)
        t[i] = old
        g[i] = (lp - lm) / (2 * eps)
    return g


def to_poly(theta, m, s):
    """Power-basis coefficients c0..c4 of y(u), expanded layer by layer in exact
    polynomial arithmetic (numpy.polynomial), then composed with z = (u - m)/s."""
    P = np.polynomial.polynomial
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    zpoly = np.array([-m / s, 1.0 / s])          # z as a polynomial of u
    y = np.zeros(1)
    a1 = [P.polymul(P.polyadd(W1[k] * zpoly, [b1[k]]), P.polyadd(W1[k] * zpoly, [b1[k]])) for k in range(H)]
    for j in range(H):
        h2 = np.array([b2[j]])
        for k in range(H):
            h2 = P.polyadd(h2, W2[j, k] * a1[k])
        y = P.polyadd(y, W3[j] * P.polymul(h2, h2))
    y = P.polyadd(y, [b3])
    out = np.zeros(5)
    out[:len(y)] = y[:5]
    return out
