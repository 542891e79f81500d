"""CPU FP64 reference of the learned form's network and features.

TEST INFRASTRUCTURE ONLY (imported by tests and the smoke check, never by the
product package).  Plain numpy, written from the definitions:

* features of an instance (site, E): the centre's species one-hot, then for
  the first seven neighbour shells of the fcc lattice (ideal radii
  a*sqrt(k/2), k = 1..7) the number of Ni and Au sites assigned to the shell
  (each LIZ site goes to the ideal shell nearest in radius; sites nearer to
  the eighth shell are not counted) divided by the shell's size
  (12, 6, 24, 12, 24, 8, 48), then Re E and Im E: 18 inputs;
* network: 18 -> 256 -> 256 -> 256 -> 1024, SiLU (x * sigmoid(x)) after the
  three hidden layers, linear output; weights W_l [out][in], biases b_l;
* the products of the GPU path take bf16-rounded operands (weights and
  layer inputs, round to nearest even) with wide accumulation;
  `round_bf16=True` reproduces that, `False` is the plain FP64 network used
  for the finite-difference check;
* backward: exact derivatives of the forward above, the bf16 rounding taken
  as the identity (straight-through);
* AdamW (Loshchilov and Hutter): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  w -= lr (m / (1-b1^t) / (sqrt(v / (1-b2^t)) + eps) + wd w).
"""

from __future__ import annotations

import numpy as np

LAYERS = (18, 256, 256, 256, 1024)
SHELL_SIZE = (12, 6, 24, 12, 24, 8, 48)


def param_count() -> int:
    return sum(o * i + o for i, o in zip(LAYERS[:-1], LAYERS[1:]))


def unpack(theta):
    """Views (W_l, b_l) into the flat parameter vector [W1 b1 W2 b2 W3 b3 W4 b4]."""
    out, off = [], 0
    for i, o in zip(LAYERS[:-1], LAYERS[1:]):
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, round_bf16=True):
    """Outputs [n, 1024] and the per-layer cache (inputs, pre-activations)."""
    h = np.asarray(X, dtype=np.float64)
    cache = []
    layers = unpack(np.asarray(theta, dtype=np.float64))
    for l, (W, b) in enumerate(layers):
        hin = bf16(h) if round_bf16 else h
        Wr = bf16(W) if round_bf16 else W
        z = hin @ Wr.T + b
        cache.append((hin, Wr, z))
        h = silu(z) if l + 1 < len(layers) else z
    return h, cache


def backward(theta, cache, dY):
    """Gradient of sum(dY * outputs) with respect to the flat parameters."""
    layers = unpack(np.asarray(theta, dtype=np.float64))
    grads = [None] * len(layers)
    g = np.asarray(dY, dtype=np.float64)
    for l in range(len(layers) - 1, -1, -1):
        hin, Wr, z = cache[l]
        if l + 1 < len(layers):
            g = g * dsilu(z)
        grads[l] = (g.T @ hin, g.sum(axis=0))
        g = g @ Wr
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adamw(theta, m, v, g, lr, b1, b2, eps, wd, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v


def features(liz_off, pos, species, energies, e_idx, a):
    """[n_inst, 18] features of each instance from its LIZ (relative
    positions, centre first) and energy."""
    n = len(liz_off) - 1
    F = np.zeros((n, 18))
    radii = a * np.sqrt(np.arange(1, 9) / 2.0)
    for i in range(n):
        s, e = int(liz_off[i]), int(liz_off[i + 1])
        F[i, int(species[s])] = 1.0
        counts = np.zeros((7, 2))
        for j in range(s + 1, e):
            r = np.linalg.norm(pos[j])
            k = int(np.argmin(np.abs(radii - r)))  # nearest ideal shell, 0-based (shell k+1)
            if k < 7:
                counts[k, int(species[j])] += 1.0
        F[i, 2:16] = (counts / np.asarray(SHELL_SIZE, dtype=np.float64)[:, None]).ravel()
        E = energies[e_idx[i]]
        F[i, 16] = E.real
        F[i, 17] = E.imag
    return F
