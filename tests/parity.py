"""Comparison helpers of the GPU parity tests (no GPU code, no arithmetic of
the method beyond what the oracle provides).

Two measures per instance, both against the oracle:
  rel_F  = ||tau - tau_ref||_F / ||tau_ref||_F  (the stated tolerance);
  x_err  = max |X - X_ref| / max |X_ref| with X = tau00 diag(t_0)^{-1} =
           [M^{-1}]_{00}, elementwise and scale-free.  The f-channel entries of
           t_0 are orders of magnitude below the s-channel ones, so an f column
           of [M^{-1}]_{00} can be far off while tau00 still passes rel_F; the
           elementwise X check sees it.
"""

from __future__ import annotations

import numpy as np

import oracle


def rel_f(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    num = np.linalg.norm((got - ref).reshape(got.shape[0], -1), axis=1)
    den = np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)
    return num / den


def l_of(kk: int) -> np.ndarray:
    return np.floor(np.sqrt(np.arange(kk)) + 1e-9).astype(int)


def t0_of(w) -> np.ndarray:
    """Single-site t of each instance's centre, [n_inst, kk] (the oracle's t)."""
    kk = w.kk
    lv = l_of(kk)
    out = np.empty((w.n_inst, kk), np.complex128)
    for i in range(w.n_inst):
        e = int(w.e_idx[i])
        s = int(w.atom_species[w.centre[i]])
        out[i] = oracle.tmat(w.lmax, w.energies[e], w.delta[s, e])[lv]
    return out


def x_err(got, ref, t0) -> np.ndarray:
    """Per instance: max |X - X_ref| / max |X_ref|, X = tau00 diag(t0)^{-1};
    columns whose t0 vanishes are left out."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    out = np.zeros(got.shape[0])
    for i in range(got.shape[0]):
        keep = np.abs(t0[i]) > 0
        if not np.any(keep):
            continue
        xg = got[i][:, keep] / t0[i][None, keep]
        xr = ref[i][:, keep] / t0[i][None, keep]
        out[i] = np.abs(xg - xr).max() / np.abs(xr).max()
    return out


def check_tau(got, ref, w, tol: float, what: str = ""):
    """Asserts rel_F <= tol and x_err <= tol on every instance of workload w;
    returns (rel_F, x_err) per instance."""
    rf = rel_f(got, ref)
    xe = x_err(got, ref, t0_of(w))
    print(f"{what} rel_F max {rf.max():.2e}  [M^-1]00 elementwise max {xe.max():.2e}")
    assert rf.max() <= tol, (what, "rel_F", rf.max(), int(np.argmax(rf)))
    assert xe.max() <= tol, (what, "[M^-1]00 elementwise", xe.max(), int(np.argmax(xe)))
    return rf, xe


_ORACLE = {}


def oracle_cached(key: str, w):
    """Oracle tau00 and info of workload w, computed once per test session
    under `key` (shared by the GPU test modules)."""
    if key not in _ORACLE:
        _ORACLE[key] = oracle.tau00_workload(w)
    return _ORACLE[key]


def config2_two_sites():
    """Every contour energy of two sites of the benchmark workload (the first
    Ni and the first Au centre), N = 2160: 64 instances."""
    import inputs

    w2 = inputs.config2()
    ni = int(np.flatnonzero(w2.atom_species == 0)[0])
    au = int(np.flatnonzero(w2.atom_species == 1)[0])
    return inputs.subset(w2, np.concatenate([ni * 32 + np.arange(32), au * 32 + np.arange(32)]))


def config4_sample(n: int = 32):
    """n instances of the ragged workload spread over its 1024 (N 1184..2400)."""
    import inputs

    return inputs.subset(inputs.config4(n_inst=1024), np.linspace(0, 1023, n).astype(int))


def config3_sample():
    """8 instances of the lmax = 4 benchmark systems (N = 3375): both contour
    ends and mid-contour on eight sites."""
    import inputs

    return inputs.subset(inputs.config3(), [0, 31, 16 + 32 * 9, 1 + 32 * 40, 30 + 32 * 101, 8 + 32 * 150,
                                           24 + 32 * 200, 31 + 32 * 255])
