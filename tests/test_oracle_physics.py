"""Pins of the oracle's t-matrix, structure constants, KKR matrix, LU and tau00.

Every check compares the oracle with a fact that does not depend on its code:
closed forms, the free-particle propagator itself (addition theorem), the
optical theorem and the Born limit, LAPACK through numpy/scipy, and the
symmetries the Dyson equation forces on tau00 (paper Sec. 2.1-2.2).
"""

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp
from scipy.special import spherical_jn, spherical_yn

import inputs
import oracle


def _lvec(lmax):
    return np.array([int(np.floor(np.sqrt(L) + 1e-9)) for L in range((lmax + 1) ** 2)])


def _mvec(lmax):
    l = _lvec(lmax)
    return np.arange((lmax + 1) ** 2) - l * l - l


# ------------------------------------------------------------ t-matrix
def test_optical_theorem_real_energy():
    # For real E > 0 and real phase shifts, Im(1/t_l) = kappa.
    for E in [0.05, 0.3, 0.65]:
        d = inputs.square_well_delta(np.array([E]), 4, 1.4)[0]
        assert np.all(np.abs(d.imag) < 1e-12)
        t = oracle.tmat(4, E, d)
        np.testing.assert_allclose((1 / t).imag, np.sqrt(E), rtol=1e-13)


@pytest.mark.parametrize("E", [0.3 + 0.0j, 0.2 + 0.3j, -0.4 + 0.05j])
def test_born_limit(E):
    # Weak well: t_l -> int_0^rmt j_l(k r) V j_l(k r) r^2 dr = -V0 int j_l^2 r^2 dr.
    v0 = 1e-6
    kap = np.sqrt(complex(E))
    d = inputs.square_well_delta(np.array([E]), 3, v0)[0]
    t = oracle.tmat(3, E, d)
    for l in range(4):
        re = quad(lambda r: (spherical_jn(l, kap * r) ** 2 * r * r).real, 0, inputs.R_MT, epsabs=0, epsrel=1e-13)[0]
        im = quad(lambda r: (spherical_jn(l, kap * r) ** 2 * r * r).imag, 0, inputs.R_MT, epsabs=0, epsrel=1e-13)[0]
        born = -v0 * (re + 1j * im)
        assert abs(t[l] - born) <= 5e-6 * abs(born)


def test_zero_well_gives_zero_t():
    # no well: the two terms of the matching numerator cancel (to rounding)
    d = inputs.square_well_delta(inputs.contour_energies(8), 3, 0.0)
    assert np.abs(d).max() < 1e-14
    assert np.all(oracle.tmat(3, 0.3 + 0.1j, np.zeros(4, complex)) == 0)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_generator_phase_shift_vs_radial_integration(l):
    # Integrate u'' = (l(l+1)/r^2 + V - E) u through the well and beyond, then
    # match u/r = A [cos d j_l(k r) - sin d y_l(k r)] at two outer radii.
    E, v0, rmt = 0.4, 1.4, inputs.R_MT
    k = np.sqrt(E)

    def rhs(r, y):
        V = -v0 if r < rmt else 0.0
        return [y[1], (l * (l + 1) / r ** 2 + V - E) * y[0]]

    r0 = 1e-3
    y0 = [r0 ** (l + 1), (l + 1) * r0 ** l]
    r1, r2 = rmt + 1.0, rmt + 2.0
    sol = solve_ivp(rhs, [r0, r2], y0, method="DOP853", rtol=1e-12, atol=1e-14 * r0 ** (l + 1),
                    dense_output=True, t_eval=[r1, r2], first_step=1e-4)
    R1, R2 = sol.y[0, 0] / r1, sol.y[0, 1] / r2
    # [j1 -y1; j2 -y2] [A cos d; A sin d] = [R1; R2]
    mat = np.array([[spherical_jn(l, k * r1), -spherical_yn(l, k * r1)],
                    [spherical_jn(l, k * r2), -spherical_yn(l, k * r2)]])
    c, s = np.linalg.solve(mat, [R1, R2])
    tan_ref = s / c
    d = inputs.square_well_delta(np.array([E]), 3, v0)[0, l].real
    assert abs(np.tan(d) - tan_ref) <= 1e-7 * max(1.0, abs(tan_ref))


# ------------------------------------------------- structure constants
@pytest.mark.parametrize("E", [0.3 + 0.2j, -0.49 + 0.013j, 0.69 + 0.013j])
def test_g00_closed_form_and_reciprocity(E):
    lmax = 3
    C, _ = oracle.gaunt(lmax)
    kap = np.sqrt(E)
    rng = np.random.default_rng(3)
    l = _lvec(lmax)
    for _ in range(5):
        R = rng.normal(size=3) * 5
        G = oracle.structure_constants(lmax, kap, R, C)
        Gm = oracle.structure_constants(lmax, kap, -R, C)
        r = np.linalg.norm(R)
        assert abs(G[0, 0] + np.exp(1j * kap * r) / r) <= 1e-14 * abs(G[0, 0])
        # reciprocity: G^{ji}_{L'L} = G^{ij}_{LL'}
        np.testing.assert_allclose(Gm.T, G, rtol=0, atol=1e-14 * np.abs(G).max())
        # parity: G(-R) = (-1)^{l+l'} G(R)
        sgn = (-1.0) ** (l[:, None] + l[None, :])
        np.testing.assert_allclose(Gm, sgn * G, rtol=0, atol=1e-14 * np.abs(G).max())


@pytest.mark.parametrize("E", [0.3 + 0.2j, -0.4 + 0.05j, 0.65 + 0.013j])
def test_addition_theorem_brute_force(E):
    # G0(R_i + r, R_j + r') = sum_LL' j_l(k r) Y_L(r) G^{ij}_{LL'} j_l'(k r') Y_L'(r')
    # with G0(x, x') = -exp(i k |x - x'|) / (4 pi |x - x'|).
    lmax = 8
    C, _ = oracle.gaunt(lmax)
    kap = np.sqrt(E)
    rng = np.random.default_rng(11)
    l = _lvec(lmax)
    for _ in range(4):
        Rij = np.array([3.5, -3.5, 0.0]) + rng.normal(0, 0.3, 3)
        G = oracle.structure_constants(lmax, kap, Rij, C)
        r = rng.normal(0, 0.08, 3)
        rp = rng.normal(0, 0.08, 3)
        a = spherical_jn(l, kap * np.linalg.norm(r)) * oracle.ylm(lmax, r)
        b = spherical_jn(l, kap * np.linalg.norm(rp)) * oracle.ylm(lmax, rp)
        d = np.linalg.norm(Rij + r - rp)
        ref = -np.exp(1j * kap * d) / (4 * np.pi * d)
        assert abs(a @ G @ b - ref) <= 1e-12 * abs(ref)


# ------------------------------------------------------------ LU
@pytest.mark.parametrize("n", [1, 7, 50, 160])
def test_lu_matches_lapack(n):
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    B = rng.normal(size=(n, 3)) + 1j * rng.normal(size=(n, 3))
    LU, ipiv, info = oracle.lu_factor(A)
    assert info == 0
    X = oracle.lu_solve(LU, ipiv, B)
    np.testing.assert_allclose(X, np.linalg.solve(A, B), rtol=0, atol=1e-11 * np.abs(X).max())
    # same pivot rows as LAPACK zgetrf (|Re| + |Im| rule)
    import scipy.linalg as sl

    _, piv = sl.lu_factor(A)
    np.testing.assert_array_equal(ipiv, piv)
    # backward error at roundoff
    res = np.linalg.norm(A @ X - B) / (np.linalg.norm(A) * np.linalg.norm(X))
    assert res < 1e-15 * n


def test_lu_zero_pivot_reported():
    A = np.eye(5, dtype=complex)
    A[:, 2] = 0
    _, _, info = oracle.lu_factor(A)
    assert info == 3


# ------------------------------------------------------------ tau00
def _delta_e(w, e):
    return w.delta[:, e, :]


@pytest.fixture(scope="module")
def cfg1():
    w = inputs.config1()
    liz_off, pos, spec = oracle.liz_batch(w)
    return w, liz_off, pos, spec


def test_one_atom_liz_gives_t(cfg1):
    w = cfg1[0]
    for e in [0, 7, 15]:
        tau, info = oracle.tau00_batch(3, [0, 1], np.zeros((1, 3)), [1], w.energies, [e], w.delta)
        t = oracle.tmat(3, w.energies[e], w.delta[1, e])
        assert info[0] == 0
        np.testing.assert_allclose(tau[0], np.diag(t[_lvec(3)]), rtol=0, atol=1e-15)


def test_zero_t_gives_identity_and_zero_tau(cfg1):
    w, liz_off, pos, spec = cfg1
    d0 = np.zeros_like(w.delta)
    M, st = oracle.build_m(3, pos[:13], spec[:13], w.energies[3], d0[:, 3, :])
    assert st == 0 and np.array_equal(M, np.eye(M.shape[0]))
    tau, info = oracle.tau00_batch(3, liz_off[:2], pos, spec, w.energies, w.e_idx[:1], d0)
    assert info[0] == 0 and np.all(tau == 0)


def test_dimer_closed_form():
    # lmax = 0 dimer: tau00 = t_A / (1 - t_A t_B g^2), g = -exp(i k R) / R
    E = 0.25 + 0.1j
    kap = np.sqrt(E)
    delta = np.array([[[0.3 + 0.02j]], [[-0.7 + 0.05j]]])  # [species][energy][l]
    R = np.array([[0, 0, 0], [2.0, -3.0, 1.5]])
    tau, info = oracle.tau00_batch(0, [0, 2], R, [0, 1], [E], [0], delta)
    tA = oracle.tmat(0, E, delta[0, 0])[0]
    tB = oracle.tmat(0, E, delta[1, 0])[0]
    r = np.linalg.norm(R[1])
    g = -np.exp(1j * kap * r) / r
    ref = tA / (1 - tA * tB * g * g)
    assert info[0] == 0 and abs(tau[0, 0, 0] - ref) <= 1e-15 * abs(ref)


def test_tau_matches_lapack_solve_and_schur(cfg1):
    w, liz_off, pos, spec = cfg1
    C, _ = oracle.gaunt(3)
    for i in [0, 17, 40, 127]:
        a, b = liz_off[i], liz_off[i + 1]
        e = w.e_idx[i]
        M, st = oracle.build_m(3, pos[a:b], spec[a:b], w.energies[e], _delta_e(w, e), C)
        assert st == 0
        tau, info = oracle.tau00_batch(3, [0, b - a], pos[a:b], spec[a:b], w.energies, [e], w.delta)
        t0 = oracle.tmat(3, w.energies[e], w.delta[spec[a], e])[_lvec(3)]
        E0 = np.zeros((M.shape[0], 16), complex)
        E0[:16, :16] = np.eye(16)
        ref = np.linalg.solve(M, E0)[:16] * t0[None, :]
        np.testing.assert_allclose(tau[0], ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        ts, infs = oracle.tau00_schur(3, pos[a:b], spec[a:b], w.energies[e], _delta_e(w, e), C)
        assert infs == 0
        np.testing.assert_allclose(ts, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        # tau00 is complex symmetric (t^{-1} - G is)
        np.testing.assert_allclose(tau[0], tau[0].T, rtol=0, atol=1e-13 * np.abs(ref).max())


def _liz_case(r_c=1.0, e=5, n_liz_species=None, seed=0):
    pos, box = inputs.fcc_supercell(4)
    rel, idx = oracle.liz(pos, box, 0, r_c * inputs.A_LAT)
    rng = np.random.default_rng(seed)
    spec = rng.integers(0, 2, rel.shape[0]).astype(np.int32) if n_liz_species is None else n_liz_species
    return rel, spec


def _tau_one(lmax, rel, spec, E, delta):
    tau, info = oracle.tau00_batch(lmax, [0, rel.shape[0]], rel, spec, [E], [0], delta)
    assert info[0] == 0
    return tau[0]


def test_permutation_and_removal():
    E = 0.2 + 0.15j
    rel, spec = _liz_case()
    delta = inputs.phase_shift_table([E], 3)
    delta3 = np.concatenate([delta, np.zeros_like(delta[:1])])  # species 2: t = 0
    ref = _tau_one(3, rel, spec, E, delta)
    perm = np.concatenate([[0], 1 + np.random.default_rng(5).permutation(rel.shape[0] - 1)])
    np.testing.assert_allclose(_tau_one(3, rel[perm], spec[perm], E, delta), ref, rtol=0,
                               atol=1e-13 * np.abs(ref).max())
    # a site with t = 0 is the same as that site absent
    extra = np.vstack([rel, [[5.1, 4.3, -2.2]]])
    spx = np.concatenate([spec, [2]]).astype(np.int32)
    np.testing.assert_allclose(_tau_one(3, extra, spx, E, delta3), ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_mirror_covariance():
    E = 0.2 + 0.15j
    lmax = 3
    rel, spec = _liz_case(seed=2)
    rel = rel + np.random.default_rng(9).normal(0, 0.1, rel.shape) * (np.arange(rel.shape[0]) > 0)[:, None]
    delta = inputs.phase_shift_table([E], lmax)
    ref = _tau_one(lmax, rel, spec, E, delta)
    l, m = _lvec(lmax), _mvec(lmax)
    Ds = {0: np.where(m < 0, -1.0, 1.0) * (-1.0) ** np.abs(m),
          1: np.where(m < 0, -1.0, 1.0),
          2: (-1.0) ** (l + np.abs(m))}
    for ax, D in Ds.items():
        r2 = rel.copy()
        r2[:, ax] *= -1
        got = _tau_one(lmax, r2, spec, E, delta)
        np.testing.assert_allclose(got, D[:, None] * ref * D[None, :], rtol=0, atol=1e-13 * np.abs(ref).max())


def test_cubic_symmetry_pure_species():
    E = 0.2 + 0.15j
    lmax = 3
    rel, _ = _liz_case(r_c=1.0)
    spec = np.zeros(rel.shape[0], np.int32)
    tau = _tau_one(lmax, rel, spec, E, inputs.phase_shift_table([E], lmax))
    scale = np.abs(tau).max()
    l, m = _lvec(lmax), _mvec(lmax)
    even = (l % 2 == 0)
    assert np.abs(tau[np.ix_(even, ~even)]).max() < 1e-14 * scale
    assert np.abs(tau[0, 4:9]).max() < 1e-14 * scale          # s-d
    p = tau[1:4, 1:4]
    np.testing.assert_allclose(p, p[0, 0] * np.eye(3), rtol=0, atol=1e-14 * scale)
    d = tau[4:9, 4:9]
    np.testing.assert_allclose(d - np.diag(np.diag(d)), 0, atol=1e-14 * scale)
    t2g = np.diag(d)[[0, 1, 3]]   # m = -2, -1, 1
    eg = np.diag(d)[[2, 4]]       # m = 0, 2
    np.testing.assert_allclose(t2g, t2g[0], rtol=1e-13)
    np.testing.assert_allclose(eg, eg[0], rtol=1e-13)
    assert abs(t2g[0] - eg[0]) > 1e-6 * scale


def test_refined_residual_and_error_codes(cfg1):
    w, liz_off, pos, spec = cfg1
    a, b = liz_off[0], liz_off[1]
    e = 0  # left contour end: the worst-conditioned energy
    M, _ = oracle.build_m(3, pos[a:b], spec[a:b], w.energies[e], _delta_e(w, e))
    LU, ipiv, info = oracle.lu_factor(M)
    E0 = np.zeros((M.shape[0], 16), complex)
    E0[:16] = np.eye(16)
    X = oracle.lu_solve(LU, ipiv, E0)
    res = np.linalg.norm(M @ X - E0) / (np.linalg.norm(M) * np.linalg.norm(X))
    assert res < 1e-15
    # NaN phase shift -> -1 ; coincident sites -> -2
    dn = w.delta.copy()
    dn[0, e, 1] = np.nan
    _, info = oracle.tau00_batch(3, [0, b - a], pos[a:b], spec[a:b], w.energies, [e], dn)
    assert info[0] == -1
    pc = pos[a:b].copy()
    pc[3] = pc[2]
    tau, info = oracle.tau00_batch(3, [0, b - a], pc, spec[a:b], w.energies, [e], w.delta)
    assert info[0] == -2 and np.all(np.isnan(tau))


# ------------------------------------------------------------ LIZ (a1)
def _golden_sizes():
    import os

    rows, ranks = [], []
    with open(os.path.join(os.path.dirname(__file__), "golden", "fcc_liz_sizes.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "rank":
                ranks.append(tuple(int(v) for v in line[1:]))
            else:
                rows.append((float(line[0]), int(line[1])))
    return rows, ranks


def test_liz_sizes_match_paper_and_fcc_shells():
    rows, ranks = _golden_sizes()
    pos, box = inputs.fcc_supercell(6)
    for rc, n in rows:
        rel, idx = oracle.liz(pos, box, 77, rc * inputs.A_LAT)
        assert rel.shape[0] == n, (rc, rel.shape[0], n)
        d = np.linalg.norm(rel, axis=1)
        assert idx[0] == 77 and d[0] == 0 and np.all(np.diff(d) >= 0)
    for rank, n_liz, lmax, canted in ranks:
        assert rank == (1 + canted) * n_liz * (lmax + 1) ** 2


def test_liz_minimum_image_brute_force():
    w = inputs.config4(n_inst=6)
    for c, rc in zip(w.centre, w.rc):
        rel, idx = oracle.liz(w.atom_pos, w.box, int(c), float(rc))
        shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]) * w.box
        dd = w.atom_pos[None, :, :] + shifts[:, None, :] - w.atom_pos[c]
        dist = np.linalg.norm(dd, axis=2).min(axis=0)
        members = set(np.nonzero(dist <= rc)[0].tolist())
        assert set(idx.tolist()) == members
        np.testing.assert_allclose(np.linalg.norm(rel, axis=1), dist[idx], rtol=0, atol=1e-12)
