"""Pins of the oracle's block row of tau, ln det M, Lloyd's multiple-scattering
integrated density of states and the contour quadrature.

tau = (t^{-1} - g0)^{-1} (paper Sec. 2.1, eq. Dyson_equation) equals
M^{-1} t with M = 1 - t g0, so its block row through the central site is
tau^{0j} = [M^{-1}]_{0j} t_j; these blocks (with the diagonal ones) enter the
Green's function of eq. Green_KKR.  ln det M is the multiple-scattering term
of Lloyd's formula for the integrated density of states, the energy integral
of eq. Density.  Every check compares the oracle with something that does
not depend on its code: LAPACK through numpy, closed forms, the reciprocity
tau = tau^T the Dyson equation forces (t and g0 are complex symmetric), the
derivative identity d ln det M / dE = tr(M^{-1} dM/dE), and exact integrals
of polynomials along the contour.
"""

import numpy as np
import pytest

import inputs
import oracle


def _lvec(kk):
    return np.floor(np.sqrt(np.arange(kk)) + 1e-9).astype(int)


def _tiny(idx):
    return inputs.subset(inputs.config1(), idx)


def _M(w, i, lmax=None):
    lmax = w.lmax if lmax is None else lmax
    liz_off, pos, spec = oracle.liz_batch(w)
    a, b = liz_off[i], liz_off[i + 1]
    e = int(w.e_idx[i])
    M, st = oracle.build_m(lmax, pos[a:b], spec[a:b], w.energies[e], w.delta[:, e, :])
    assert st == 0
    return M, spec[a:b]


def _t_blocks(w, i, spec):
    e = int(w.e_idx[i])
    lv = _lvec(w.kk)
    return np.concatenate([oracle.tmat(w.lmax, w.energies[e], w.delta[s, e])[lv] for s in spec])


# ------------------------------------------------------------ block row
@pytest.mark.parametrize("i", [0, 7, 15, 64, 127])
def test_tau_row_matches_lapack_inverse_rows(i):
    w = _tiny([i])
    rows, info = oracle.tau_row_workload(w)
    assert info[0] == 0
    M, spec = _M(w, 0)
    kk = w.kk
    Minv_rows = np.linalg.solve(M.T, np.eye(M.shape[0], kk)).T  # rows 0..kk-1 of M^-1
    ref = Minv_rows * _t_blocks(w, 0, spec)[None, :]
    assert np.abs(rows[0] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_tau_row_central_block_is_tau00():
    w = _tiny(np.arange(0, 128, 9))
    rows, info = oracle.tau_row_workload(w)
    tau, tinfo = oracle.tau00_workload(w)
    assert np.all(info == 0) and np.all(tinfo == 0)
    kk = w.kk
    for q in range(w.n_inst):
        d = rows[q][:, :kk] - tau[q]
        assert np.abs(d).max() <= 1e-14 * np.abs(tau[q]).max()


@pytest.mark.parametrize("i", [3, 40, 100])
def test_tau_row_reciprocity_with_block_column(i):
    # tau^{j0} from the first block COLUMN of M^{-1} (an independent solve,
    # [M^{-1}]_{j0} t_0) equals (tau^{0j})^T: t and g0 are symmetric, so tau
    # is complex symmetric.  A t_j placed on the wrong side or a transposed
    # block fails this.
    w = _tiny([i])
    rows, info = oracle.tau_row_workload(w)
    M, spec = _M(w, 0)
    kk = w.kk
    X = np.linalg.solve(M, np.eye(M.shape[0], kk))  # first block column of M^-1
    t0 = _t_blocks(w, 0, spec[:1])
    col = X * t0[None, :]  # tau^{j0} stacked over j
    n_liz = M.shape[0] // kk
    for j in range(n_liz):
        tj0 = col[j * kk:(j + 1) * kk, :]
        t0j = rows[0][:, j * kk:(j + 1) * kk]
        assert np.abs(tj0 - t0j.T).max() <= 1e-12 * np.abs(rows[0]).max()


def test_tau_row_lmax0_dimer_closed_form():
    # two s-wave scatterers: M = [[1, -tA g], [-tB g, 1]], g = -exp(i k R)/R,
    # tau^{00} = tA / (1 - tA tB g^2), tau^{01} = tA g tB / (1 - tA tB g^2)
    E = 0.25 + 0.1j
    delta = np.array([[[0.3 + 0.02j]], [[-0.7 + 0.05j]]])
    R = np.array([[0, 0, 0], [2.0, -3.0, 1.5]])
    rows, info = oracle.tau_row_batch(0, [0, 2], R, [0, 1], [E], [0], delta)
    tA = oracle.tmat(0, E, delta[0, 0])[0]
    tB = oracle.tmat(0, E, delta[1, 0])[0]
    r = np.linalg.norm(R[1])
    g = -np.exp(1j * np.sqrt(E) * r) / r
    den = 1 - tA * tB * g * g
    np.testing.assert_allclose(rows[0][0], [tA / den, tA * g * tB / den], rtol=1e-14)


def test_tau_row_one_atom_and_zero_t():
    w = inputs.config1()
    e = np.array([0, 9], np.int32)
    rows, info = oracle.tau_row_batch(3, [0, 1, 2], np.zeros((2, 3)), [0, 1], w.energies, e, w.delta)
    lv = _lvec(16)
    for q, s in enumerate([0, 1]):
        t = oracle.tmat(3, w.energies[e[q]], w.delta[s, e[q]])[lv]
        np.testing.assert_allclose(rows[q], np.diag(t), rtol=0, atol=1e-15 * np.abs(t).max())
    w0 = _tiny([0, 1])
    w0.delta = np.zeros_like(w0.delta)
    rows0, info0 = oracle.tau_row_workload(w0)
    assert np.all(info0 == 0) and all(np.all(r == 0) for r in rows0)


# ------------------------------------------------------------ ln det M
def _wrap(x):
    return np.angle(np.exp(1j * x))


@pytest.mark.parametrize("lmax", [0, 1, 3])
def test_logdet_matches_numpy_slogdet(lmax):
    w = _tiny(np.arange(0, 128, 11))
    if lmax != 3:
        w = w.with_lmax(lmax)
    ld, info = oracle.logdet_workload(w)
    assert np.all(info == 0)
    for q in range(w.n_inst):
        M, _ = _M(w, q)
        sign, lab = np.linalg.slogdet(M)
        assert abs(ld[q].real - lab) <= 1e-12 * max(1.0, abs(lab))
        assert abs(_wrap(ld[q].imag - np.angle(sign))) <= 1e-12
        assert -np.pi < ld[q].imag <= np.pi


def test_logdet_one_atom_zero_t_and_dimer():
    w = inputs.config1()
    ld, info = oracle.logdet_batch(3, [0, 1], np.zeros((1, 3)), [1], w.energies, [4], w.delta)
    assert info[0] == 0 and ld[0] == 0  # M = I
    w0 = _tiny([0, 5])
    w0.delta = np.zeros_like(w0.delta)
    ld0, _ = oracle.logdet_workload(w0)
    assert np.all(ld0 == 0)  # t = 0: M = I
    # lmax = 0 dimer: det M = 1 - tA tB g^2
    E = 0.25 + 0.1j
    delta = np.array([[[0.3 + 0.02j]], [[-0.7 + 0.05j]]])
    R = np.array([[0, 0, 0], [2.0, -3.0, 1.5]])
    ldd, _ = oracle.logdet_batch(0, [0, 2], R, [0, 1], [E], [0], delta)
    tA = oracle.tmat(0, E, delta[0, 0])[0]
    tB = oracle.tmat(0, E, delta[1, 0])[0]
    r = np.linalg.norm(R[1])
    g = -np.exp(1j * np.sqrt(E) * r) / r
    ref = np.log(1 - tA * tB * g * g)
    assert abs(ldd[0] - ref) <= 1e-14


def _M_at(w, i, E):
    liz_off, pos, spec = oracle.liz_batch(w)
    a, b = liz_off[i], liz_off[i + 1]
    d = np.stack([inputs.square_well_delta(np.array([E]), w.lmax, v)[0] for v in inputs.V0_SPECIES])
    M, st = oracle.build_m(w.lmax, pos[a:b], spec[a:b], E, d)
    assert st == 0
    return M, pos[a:b], spec[a:b], d


@pytest.mark.parametrize("E", [-0.3 + 0.2j, 0.15 + 0.55j, 0.6 + 0.1j])
def test_logdet_derivative_is_trace_of_inverse_times_derivative(E):
    # d/dE ln det M = tr(M^{-1} dM/dE): central differences of the oracle's
    # ln det against the trace formula on the oracle's matrices
    w = _tiny([17])
    h = 1e-5
    liz_off, pos, spec = oracle.liz_batch(w)

    def ld_at(Ez):
        M, p, s, d = _M_at(w, 0, Ez)
        v, info = oracle.logdet_batch(w.lmax, [0, p.shape[0]], p, s, [Ez], [0], d[:, None, :])
        assert info[0] == 0
        return v[0]

    lp, lm = ld_at(E + h), ld_at(E - h)
    dld = (lp.real - lm.real + 1j * _wrap(lp.imag - lm.imag)) / (2 * h)
    M0, *_ = _M_at(w, 0, E)
    dM = (_M_at(w, 0, E + h)[0] - _M_at(w, 0, E - h)[0]) / (2 * h)
    tr = np.trace(np.linalg.solve(M0, dM))
    assert abs(dld - tr) <= 1e-6 * abs(tr)


def test_lloyd_unwrapped_phase_equals_integrated_trace():
    # Along the contour, the unwrapped phase change of det M between
    # neighbouring nodes equals Im of the integral of tr(M^{-1} dM/dE) along
    # the arc between them (fine Gauss-Legendre quadrature of the trace),
    # so lloyd_ms_idos is Lloyd's -(1/pi) Im [ln det M(E_k) - ln det M(E_0)].
    w = _tiny(np.arange(32, 48))  # one site, all 16 energies
    ld, info = oracle.logdet_workload(w)
    assert np.all(info == 0)
    order = np.argsort(w.energies[w.e_idx].real)
    n_ms = oracle.lloyd_ms_idos(ld[order])
    E = w.energies[w.e_idx][order]
    th = np.angle(E - 0.1)
    xg, wg = np.polynomial.legendre.leggauss(12)
    h = 1e-6
    acc = 0.0
    for k in range(3):  # the first three segments (checks the unwrapping where the phase moves most)
        a, b = th[k], th[k + 1]
        tt = (a + b) / 2 + (b - a) / 2 * xg
        s = 0.0
        for t_, wt in zip(tt, wg):
            Ez = 0.1 + 0.6 * np.exp(1j * t_)
            dE = 1j * 0.6 * np.exp(1j * t_) * (b - a) / 2
            M0, *_ = _M_at(w, 0, Ez)
            dM = (_M_at(w, 0, Ez + h)[0] - _M_at(w, 0, Ez - h)[0]) / (2 * h)
            s += wt * np.trace(np.linalg.solve(M0, dM)) * dE
        acc += s.imag
        assert abs(-acc / np.pi - n_ms[k + 1]) <= 1e-6, (k, -acc / np.pi, n_ms[k + 1])


# ------------------------------------------------------ contour quadrature
def test_contour_weights_integrate_polynomials():
    # the arc integral of E^n is (b^{n+1} - a^{n+1})/(n+1) whatever the path;
    # in the angle the integrand is a trigonometric polynomial, which the
    # Gauss-Legendre rule integrates with an error that falls exponentially
    # with the number of nodes (2.4e-12 at 16 nodes for n = 7)
    for ne, tol in ((16, 1e-11), (32, 1e-14)):
        e = inputs.contour_energies(ne)
        wq = inputs.contour_weights(ne)
        a, b = inputs.contour_ends()
        for n in range(0, 8):
            got = oracle.contour_integral(e ** n, wq)
            ref = (b ** (n + 1) - a ** (n + 1)) / (n + 1)
            assert abs(got - ref) <= tol * max(1.0, abs(ref)), (ne, n)
        assert abs(a.imag - 0.01) < 1e-15 and abs(b.imag - 0.01) < 1e-15


def test_contour_integral_of_a_pole_outside():
    # f = 1/(E - p) with p below the contour: log((b - p)/(a - p))
    e = inputs.contour_energies(32)
    wq = inputs.contour_weights(32)
    a, b = inputs.contour_ends()
    for p in (-0.8 + 0.0j, 0.1 - 0.05j, 1.0 - 0.2j):
        got = oracle.contour_integral(1.0 / (e - p), wq)
        assert abs(got - np.log((b - p) / (a - p))) <= 1e-10


def test_contour_integral_blocks():
    # the quadrature applies entrywise to matrix-valued f
    e = inputs.contour_energies(32)
    wq = inputs.contour_weights(32)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    vals = np.stack([A * z ** 2 for z in e])
    a, b = inputs.contour_ends()
    np.testing.assert_allclose(oracle.contour_integral(vals, wq), A * (b ** 3 - a ** 3) / 3, rtol=1e-13)
