"""Pins of the oracle's spin-canted tau00 (rank 2 kk n_liz, paper Sec. 2.1).

Reading (the paper gives only the rank): site i carries a unit moment
direction e_i and, in its own spin frame, t = diag(t_up, t_dn); in the global
frame t_i = tbar 1 + dt (e_i . sigma); the propagator is spin-independent.
Each check compares the oracle with something its spin code does not
produce: the already-pinned non-canted oracle on special cases (collinear,
antiparallel, non-magnetic), the covariance of tau under a global spin
rotation (SU(2) matrices built here from the axis and angle), a 2 x 2 closed
form for the lmax = 0 dimer (Pauli matrices written out here), the transpose
relation that the symmetry of the propagator forces, and LAPACK on the
oracle's own M.
"""

import numpy as np
import pytest

import inputs
import oracle

SX = np.array([[0, 1], [1, 0]], complex)
SY = np.array([[0, -1j], [1j, 0]])
SZ = np.array([[1, 0], [0, -1]], complex)


def _w(n_sites=3, n_e=4, lmax=3, moments=None, seed=0):
    """Spin-canted config-1-like workload: sites 0..n_sites-1, energies spread
    over the 16-point contour (both ends included)."""
    w1 = inputs.config1()
    up, dn = inputs.spin_phase_shift_tables(w1.energies, lmax)
    mom = inputs.canted_moments(w1.atom_pos.shape[0], seed) if moments is None else moments
    ew = np.linspace(0, 15, n_e).astype(int)
    idx = np.array([s * 16 + e for s in range(n_sites) for e in ew])
    w = inputs.subset(w1, idx)
    import dataclasses

    return dataclasses.replace(w, lmax=lmax, delta=up, delta_dn=dn, atom_moment=mom)


def _nc(w, delta, species=None):
    liz_off, pos, spec = oracle.liz_batch(w)
    if species is not None:
        spec = species
    return oracle.tau00_batch(w.lmax, liz_off, pos, spec, w.energies, w.e_idx, delta)


def _blocks(t, kk):
    return t[:, :kk, :kk], t[:, :kk, kk:], t[:, kk:, :kk], t[:, kk:, kk:]


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_collinear_is_two_plain_solves():
    n_at = inputs.config1().atom_pos.shape[0]
    w = _w(moments=np.tile([0.0, 0.0, 1.0], (n_at, 1)))
    tau, info = oracle.tau00_spin_workload(w)
    assert np.all(info == 0)
    kk = w.kk
    uu, ud, du, dd = _blocks(tau, kk)
    assert np.all(ud == 0) and np.all(du == 0)
    ref_u, _ = _nc(w, w.delta)
    ref_d, _ = _nc(w, w.delta_dn)
    assert _rel(uu, ref_u) <= 1e-13
    assert _rel(dd, ref_d) <= 1e-13


def test_antiparallel_sites_swap_the_spin_channels():
    # moments +z or -z at random: a -z site sees the up/down phase shifts
    # exchanged, i.e. the plain solve with extra species carrying the swapped
    # tables
    rng = np.random.default_rng(5)
    n_at = inputs.config1().atom_pos.shape[0]
    sign = rng.choice([-1.0, 1.0], n_at)
    w = _w(moments=np.stack([np.zeros(n_at), np.zeros(n_at), sign], axis=1))
    tau, info = oracle.tau00_spin_workload(w)
    assert np.all(info == 0)
    kk = w.kk
    liz_off, pos, spec = oracle.liz_batch(w)
    sgn = oracle.liz_moments(w)[:, 2]
    spec2 = np.where(sgn > 0, spec, spec + 2).astype(np.int32)
    up_ext = np.concatenate([w.delta, w.delta_dn])
    dn_ext = np.concatenate([w.delta_dn, w.delta])
    ref_u, _ = _nc(w, up_ext, spec2)
    ref_d, _ = _nc(w, dn_ext, spec2)
    uu, ud, du, dd = _blocks(tau, kk)
    assert np.all(ud == 0) and np.all(du == 0)
    assert _rel(uu, ref_u) <= 1e-13
    assert _rel(dd, ref_d) <= 1e-13


def test_nonmagnetic_is_plain_tau_times_identity():
    w = _w()
    w.delta_dn = w.delta.copy()
    tau, info = oracle.tau00_spin_workload(w)
    assert np.all(info == 0)
    ref, _ = _nc(w, w.delta)
    uu, ud, du, dd = _blocks(tau, w.kk)
    assert _rel(uu, ref) <= 1e-13 and _rel(dd, ref) <= 1e-13
    assert np.abs(ud).max() <= 1e-15 * np.abs(ref).max() and np.abs(du).max() <= 1e-15 * np.abs(ref).max()


def _su2(axis, ang):
    n = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.cos(ang / 2) * np.eye(2) - 1j * np.sin(ang / 2) * (n[0] * SX + n[1] * SY + n[2] * SZ)


def _so3(axis, ang):
    n = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def test_global_spin_rotation_covariance():
    axis, ang = [0.3, -0.8, 0.5], 1.1
    U, R = _su2(axis, ang), _so3(axis, ang)
    # the pair (U, R) represents the same rotation on spin and on vectors
    a = np.array([0.2, 0.7, -0.4])
    sa = a[0] * SX + a[1] * SY + a[2] * SZ
    ra = R @ a
    assert np.allclose(U @ sa @ U.conj().T, ra[0] * SX + ra[1] * SY + ra[2] * SZ, atol=1e-15)
    w = _w()
    tau, info = oracle.tau00_spin_workload(w)
    w2 = _w(moments=w.atom_moment @ R.T)
    tau2, info2 = oracle.tau00_spin_workload(w2)
    assert np.all(info == 0) and np.all(info2 == 0)
    big = np.kron(U, np.eye(w.kk))
    pred = big @ tau @ big.conj().T
    assert _rel(tau2, pred) <= 1e-13
    # and the rotation does something: the blocks really change
    assert _rel(tau2, tau) > 1e-3


def test_dimer_lmax0_closed_form():
    # two sites, lmax = 0: M = [[1, -t_A g], [-t_B g, 1]] with 2 x 2 spin
    # blocks, so tau00 = (1 - g^2 t_A t_B)^{-1} t_A
    E = 0.25 + 0.1j
    du = np.array([[[0.3 + 0.02j]], [[-0.7 + 0.05j]]])
    dd = np.array([[[0.1 + 0.01j]], [[-0.5 + 0.04j]]])
    R = np.array([[0, 0, 0], [2.0, -3.0, 1.5]])
    eA = np.array([np.sin(0.4) * np.cos(1.0), np.sin(0.4) * np.sin(1.0), np.cos(0.4)])
    eB = np.array([np.sin(1.9) * np.cos(-2.2), np.sin(1.9) * np.sin(-2.2), np.cos(1.9)])
    tau, info = oracle.tau00_spin_batch(0, [0, 2], R, [0, 1], np.stack([eA, eB]), [E], [0], du, dd)
    assert info[0] == 0

    def t2(s, e):
        tu = oracle.tmat(0, E, du[s, 0])[0]
        td = oracle.tmat(0, E, dd[s, 0])[0]
        return 0.5 * (tu + td) * np.eye(2) + 0.5 * (tu - td) * (e[0] * SX + e[1] * SY + e[2] * SZ)

    g = -np.exp(1j * np.sqrt(E) * np.linalg.norm(R[1])) / np.linalg.norm(R[1])
    tA, tB = t2(0, eA), t2(1, eB)
    ref = np.linalg.solve(np.eye(2) - g * g * tA @ tB, tA)
    assert np.abs(tau[0] - ref).max() <= 1e-15 * np.abs(ref).max()
    # one-site LIZ: tau00 = t_0
    tau1, _ = oracle.tau00_spin_batch(0, [0, 1], R[:1], [0], eA[None], [E], [0], du, dd)
    assert np.abs(tau1[0] - tA).max() <= 1e-16 * np.abs(tA).max()


def test_transpose_flips_the_y_components():
    # t_i^T is t_i with e_y -> -e_y (sigma_y^T = -sigma_y, sigma_x,z symmetric)
    # and the propagator is symmetric (G^{ji}_{L'L} = G^{ij}_{LL'}), so
    # (t^{-1} - G)^{-1} transposes into the same with every e_y negated
    w = _w()
    tau, info = oracle.tau00_spin_workload(w)
    mom = w.atom_moment * np.array([1.0, -1.0, 1.0])
    tau2, info2 = oracle.tau00_spin_workload(_w(moments=mom))
    assert np.all(info == 0) and np.all(info2 == 0)
    assert _rel(tau2, tau.transpose(0, 2, 1)) <= 1e-13


def test_matches_lapack_on_its_matrix():
    w = _w(n_sites=2, n_e=2)
    tau, info = oracle.tau00_spin_workload(w)
    liz_off, pos, spec = oracle.liz_batch(w)
    mom = oracle.liz_moments(w)
    kk = w.kk
    for i in range(w.n_inst):
        a, b = liz_off[i], liz_off[i + 1]
        e = int(w.e_idx[i])
        M, st = oracle.build_m_spin(w.lmax, pos[a:b], spec[a:b], mom[a:b], w.energies[e], w.delta[:, e],
                                    w.delta_dn[:, e])
        assert st == 0 and M.shape[0] == 2 * kk * (b - a)
        X = np.linalg.solve(M, np.eye(M.shape[0], 2 * kk))[:2 * kk]
        lv = np.floor(np.sqrt(np.arange(kk)) + 1e-9).astype(int)
        tu = oracle.tmat(w.lmax, w.energies[e], w.delta[spec[a], e])[lv]
        td = oracle.tmat(w.lmax, w.energies[e], w.delta_dn[spec[a], e])[lv]
        ez = mom[a]
        t0 = np.zeros((2 * kk, 2 * kk), complex)
        for L in range(kk):
            blk = 0.5 * (tu[L] + td[L]) * np.eye(2) + 0.5 * (tu[L] - td[L]) * (ez[0] * SX + ez[1] * SY + ez[2] * SZ)
            for s in range(2):
                for sp in range(2):
                    t0[kk * s + L, kk * sp + L] = blk[s, sp]
        ref = X @ t0
        assert _rel(tau[i], ref) <= 1e-12


@pytest.mark.parametrize("lmax", [3, 4])
def test_canted_workload_shapes(lmax):
    w = inputs.config_canted(lmax=lmax)
    assert w.spin and w.n_inst == 8192
    assert np.allclose(np.linalg.norm(w.atom_moment, axis=1), 1.0)
    assert np.degrees(np.arccos(w.atom_moment[:, 2])).max() <= 60.0
    # rank 2 kk n_liz of the 135-atom LIZ: 4320 (lmax 3), 6750 (lmax 4)
    assert 2 * w.kk * 135 == {3: 4320, 4: 6750}[lmax]
    assert w.delta.shape == w.delta_dn.shape and not np.allclose(w.delta, w.delta_dn)
