"""Pins of the learned form's CPU reference (oracle/mlp.py): finite
differences for the backward, closed forms for SiLU, bf16 rounding and AdamW,
and the fcc shell structure for the features."""

import numpy as np
import pytest

import inputs
import oracle
from oracle import mlp


def test_param_count():
    # 18*256 + 256 + 2*(256*256 + 256) + 256*1024 + 1024
    assert mlp.param_count() == 399616


def test_silu_derivative_closed_form():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    num = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(num - mlp.dsilu(z))) < 1e-9
    assert mlp.silu(0.0) == 0.0 and abs(mlp.dsilu(0.0) - 0.5) < 1e-15


def test_bf16_rounding():
    # exact values, a tie to even each way, and the definition on random data
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0                   # tie -> even (1.0)
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6   # tie -> even (mantissa ...10)
    assert mlp.bf16(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    rng = np.random.default_rng(3)
    x = rng.standard_normal(10000).astype(np.float32).astype(np.float64)
    r = mlp.bf16(x)
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    ulp = 2.0 ** (np.floor(np.log2(np.abs(x))) - 7)
    assert np.all(np.abs(r - x) <= ulp / 2)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(7)
    theta = inputs.mlp_init(seed=11)
    X = rng.standard_normal((3, 18))
    dY = rng.standard_normal((3, 1024))
    _, cache = mlp.forward(theta, X, round_bf16=False)
    g = mlp.backward(theta, cache, dY)
    # sample parameters in every layer (weights and biases)
    offs, off = [], 0
    for i, o in zip(mlp.LAYERS[:-1], mlp.LAYERS[1:]):
        offs += list(rng.integers(off, off + o * i, 6)) + list(rng.integers(off + o * i, off + o * i + o, 3))
        off += o * i + o
    h = 1e-6
    for p in offs:
        tp = theta.copy()
        tp[p] += h
        tm = theta.copy()
        tm[p] -= h
        fp = np.sum(dY * mlp.forward(tp, X, round_bf16=False)[0])
        fm = np.sum(dY * mlp.forward(tm, X, round_bf16=False)[0])
        num = (fp - fm) / (2 * h)
        assert abs(num - g[p]) <= 1e-6 * max(1.0, abs(num)), (p, num, g[p])


def test_adamw_first_step_closed_form():
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, wd, eps = 1e-3, 1e-2, 1e-8
    t1, m, v = mlp.adamw(theta, np.zeros(50), np.zeros(50), g, lr, 0.9, 0.999, eps, wd, 1)
    # first step: bias-corrected m = g, v = g^2
    assert np.allclose(t1, theta - lr * (g / (np.abs(g) + eps) + wd * theta), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_fcc_shells():
    # a 135-atom LIZ of the fcc lattice: every one of the 7 shells is full, so
    # the per-species fractions of each shell add up to exactly 1
    w = inputs.subset(inputs.config2(), [0, 1, 40, 8191])
    liz_off, pos, spec = oracle.liz_batch(w)
    F = mlp.features(liz_off, pos, spec, w.energies, w.e_idx, inputs.A_LAT)
    assert F.shape == (4, 18)
    for i in range(4):
        assert F[i, 0] + F[i, 1] == 1.0
        assert F[i, spec[liz_off[i]]] == 1.0
        shells = F[i, 2:16].reshape(7, 2).sum(axis=1)
        assert np.allclose(shells, 1.0, rtol=0, atol=1e-12)
        E = w.energies[w.e_idx[i]]
        assert F[i, 16] == E.real and F[i, 17] == E.imag
    # a pure-Ni crystal: all Ni fractions 1, all Au fractions 0
    spec0 = np.zeros_like(spec)
    F0 = mlp.features(liz_off, pos, spec0, w.energies, w.e_idx, inputs.A_LAT)
    assert np.all(F0[:, 2:16:2] == 1.0) and np.all(F0[:, 3:16:2] == 0.0)


def test_features_count_only_seven_shells():
    # the cutoff 1.9a reaches shell 7 exactly (135 atoms); a larger cutoff adds
    # atoms nearer to shell 8 that must not be counted
    w = inputs.subset(inputs.config2(), [3])
    w.rc = np.full_like(w.rc, 2.05 * inputs.A_LAT)
    liz_off, pos, spec = oracle.liz_batch(w)
    # shell 8 (r = 2a) is half the 28-bohr box: its 6 sites are 3 minimum images
    assert liz_off[1] - liz_off[0] == 138
    F = mlp.features(liz_off, pos, spec, w.energies, w.e_idx, inputs.A_LAT)
    assert np.allclose(F[0, 2:16].reshape(7, 2).sum(axis=1), 1.0, rtol=0, atol=1e-12)
