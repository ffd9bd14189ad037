"""CPU reference for the learned-temperature network (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use this module; the
GPU library never calls it.

The paper runs Jet with a fixed schedule of temperatures (Section 4.1 and the temperature study of
Section 7).  The learned part replaces the schedule by a small network that maps 16 statistics of
the current level and round to a temperature in [0, 1]:

    16 inputs -> 64 ReLU -> 64 ReLU -> 1 -> sigmoid,   5,313 parameters,

trained by mean squared error against the temperature that a sweep found best, with Adam
(beta1 = 0.9, beta2 = 0.999, eps = 1e-8).  This module is the plain definition: dense matrix
products, the chain rule written out layer by layer, and Adam's update as published (Kingma and
Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015, Algorithm 1).  It runs in any numpy
floating type: float32 to compare with the GPU kernels, float64 for the central-difference check
of the gradient.

Flat parameter layout (shared with the GPU library by convention only, no code is shared):
    W1[64][16] (row = hidden unit, column = input), b1[64],
    W2[64][64] (row = output unit, column = input unit), b2[64],
    w3[64], b3[1].
Feature standardisation: x_std = (x - mean) / std per input, applied before the first layer.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 16, 64
NPARAM = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1  # 5313


def unpack(theta):
    """Views (W1, b1, W2, b2, w3, b3) into the flat parameter vector."""
    o = 0
    W1 = theta[o:o + N_H * N_IN].reshape(N_H, N_IN)
    o += N_H * N_IN
    b1 = theta[o:o + N_H]
    o += N_H
    W2 = theta[o:o + N_H * N_H].reshape(N_H, N_H)
    o += N_H * N_H
    b2 = theta[o:o + N_H]
    o += N_H
    w3 = theta[o:o + N_H]
    o += N_H
    b3 = theta[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def standardise(X, mean, std):
    return (X - mean) / std


def forward(theta, X):
    """Returns (tau[B], cache) for standardised inputs X[B][16]."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0)
    z3 = h2 @ w3 + b3[0]
    y = 1 / (1 + np.exp(-z3))
    return y, (X, z1, h1, z2, h2, y)


def loss(theta, X, t):
    """Mean squared error over the batch."""
    y, _ = forward(theta, X)
    return np.mean((y - t) ** 2)


def grad(theta, X, t):
    """(loss, dL/dtheta) by the chain rule, layer by layer."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    y, (X, z1, h1, z2, h2, _) = forward(theta, X)
    B = X.shape[0]
    one = theta.dtype.type(1)
    dy = (2 * (y - t) / B).astype(theta.dtype)       # dL/dy
    d3 = dy * y * (one - y)                           # dL/dz3 (sigmoid' = y (1 - y))
    d2 = np.outer(d3, w3) * (z2 > 0)                  # dL/dz2
    d1 = (d2 @ W2) * (z1 > 0)                         # dL/dz1
    g = np.zeros_like(theta)
    gW1, gb1, gW2, gb2, gw3, gb3 = unpack(g)
    gW1[...] = d1.T @ X
    gb1[...] = d1.sum(axis=0)
    gW2[...] = d2.T @ h1
    gb2[...] = d2.sum(axis=0)
    gw3[...] = h2.T @ d3
    gb3[...] = d3.sum()
    return np.mean((y - t) ** 2), g


def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place (step counts from 1).  The bias corrections 1 / (1 - beta^step)
    are formed in double and rounded to the parameters' type."""
    dt = theta.dtype.type
    c1 = dt(1.0 / (1.0 - beta1 ** step))
    c2 = dt(1.0 / (1.0 - beta2 ** step))
    m[...] = dt(beta1) * m + dt(1 - beta1) * g
    v[...] = dt(beta2) * v + dt(1 - beta2) * g * g
    theta[...] = theta - dt(lr) * (m * c1) / (np.sqrt(v * c2) + dt(eps))


def central_difference(theta64, X64, t64, h=1e-6):
    """dL/dtheta by symmetric differences in float64 (slow; for checking grad only)."""
    g = np.zeros_like(theta64)
    for i in range(theta64.size):
        a = theta64.copy()
        b = theta64.copy()
        a[i] += h
        b[i] -= h
        g[i] = (loss(a, X64, t64) - loss(b, X64, t64)) / (2 * h)
    return g


def level_features(stats, eps, level, levels, n_finest, rnd, rounds, prev_gain, dtype=np.float64):
    """The 16 network inputs of one temperature round, from the level statistics ``stats`` (the 16
    exact integers of ``oracle.level_stats``: n, m, pins, largest net, k, W, Lmax, largest block
    weight, cut nets, metric, sum of net weights, boundary vertices, weight of the cut nets,
    ceil(W/k), 0, 0).  Written from the definitions of the inputs, one per line:

        0  log2 n                     8  level / (levels - 1), 0 on a single level
        1  log2 m                     9  log2(n_finest / n): how far the level is coarsened
        2  log2 pins                 10  largest block weight / Lmax - 1 (imbalance)
        3  mean net size pins / m    11  cut nets / m
        4  log2 largest net          12  metric / sum of net weights
        5  mean degree pins / n      13  boundary vertices / n
        6  log2 k                    14  round / (rounds - 1), 0 for a single round
        7  eps                       15  previous round's relative metric decrease

    Level 0 is the finest level.  Arithmetic in float64, rounded to ``dtype`` at the end.
    """
    n, m, p, big, k = (float(stats[i]) for i in range(5))
    lmax, heaviest, cut, metric, wsum, boundary = (float(stats[i]) for i in (6, 7, 8, 9, 10, 11))
    f = np.empty(16, dtype=np.float64)
    f[0] = np.log2(n)
    f[1] = np.log2(m)
    f[2] = np.log2(p)
    f[3] = p / m
    f[4] = np.log2(big)
    f[5] = p / n
    f[6] = np.log2(k)
    f[7] = eps
    f[8] = level / (levels - 1) if levels > 1 else 0.0
    f[9] = np.log2(n_finest / n)
    f[10] = heaviest / lmax - 1.0
    f[11] = cut / m
    f[12] = metric / wsum
    f[13] = boundary / n
    f[14] = rnd / (rounds - 1) if rounds > 1 else 0.0
    f[15] = prev_gain
    return f.astype(dtype)
