"""Workload recipes: fcc NiAu-shaped alloys, energies and square-well phase shifts.

Units are Rydberg atomic units (lengths in bohr, energies in Ry).  The paper
benchmarks NiAu and CoCrFeMnNi alloys whose potentials are not available here
(Sec. 4.1); these seeded fcc stand-ins take the shapes it names (fcc lattice,
lmax = 3 or 4, a LIZ of 135 atoms, Sec. 4.1) and a square-well muffin-tin in
place of the self-consistent potentials.

Species codes: 0 = Ni (well depth 1.0 Ry), 1 = Au (well depth 1.4 Ry).
"""

from __future__ import annotations

import dataclasses

import numpy as np
from scipy.special import spherical_jn, spherical_yn

A_LAT = 7.0                 # fcc lattice constant, bohr
R_MT = 0.35 * A_LAT         # muffin-tin radius, bohr
V0_SPECIES = (1.0, 1.4)     # square-well depths (Ry) of Ni and Au
# exchange splitting of the wells in the spin-canted recipe (Ry): the spin
# parallel to a site's moment sees the well deepened by half of it, the other
# spin the well made shallower by half of it (Ni magnetic, Au weakly polarised)
SPLIT_SPECIES = (0.10, 0.02)

# Semicircle contour: centre 0.1 Ry, radius 0.6 Ry, from -0.5 to 0.7 Ry, with
# Gauss-Legendre nodes in the angle restricted to [theta0, pi - theta0] so that
# every node keeps Im E >= 0.01 Ry.
_E_CENTRE = 0.1
_E_RADIUS = 0.6
_IM_MIN = 0.01


def fcc_supercell(n: int, a: float = A_LAT):
    """n x n x n conventional fcc cells; site id = 4*(i*n*n + j*n + k) + b.

    Returns (positions [4 n^3, 3] in bohr, box [3] in bohr).
    """
    basis = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
    pos = np.empty((4 * n ** 3, 3))
    s = 0
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for b in range(4):
                    pos[s] = (np.array([i, j, k], float) + basis[b]) * a
                    s += 1
    return pos, np.full(3, n * a)


def contour_energies(n_e: int) -> np.ndarray:
    """Complex energies on the semicircle, ascending in Re E (Ry)."""
    x, _ = np.polynomial.legendre.leggauss(n_e)
    th0 = np.arcsin(_IM_MIN / _E_RADIUS)
    th = th0 + (np.pi - 2.0 * th0) * (1.0 - x) / 2.0
    e = _E_CENTRE + _E_RADIUS * np.exp(1j * th)
    return e[np.argsort(e.real)]


def contour_weights(n_e: int) -> np.ndarray:
    """Complex quadrature weights of the same contour, in the order of
    contour_energies: sum_k w_k f(E_k) approximates the integral of f along
    the arc from its left end E(pi - theta0) to its right end E(theta0)
    through the upper half plane (Gauss-Legendre weights times dE/dx)."""
    x, wx = np.polynomial.legendre.leggauss(n_e)
    th0 = np.arcsin(_IM_MIN / _E_RADIUS)
    th = th0 + (np.pi - 2.0 * th0) * (1.0 - x) / 2.0
    e = _E_CENTRE + _E_RADIUS * np.exp(1j * th)
    w = wx * (1j * _E_RADIUS * np.exp(1j * th)) * (-(np.pi - 2.0 * th0) / 2.0)
    return w[np.argsort(e.real)]


def contour_ends() -> tuple:
    """The contour's end points (left, right), Im E = 0.01 Ry each."""
    th0 = np.arcsin(_IM_MIN / _E_RADIUS)
    return (_E_CENTRE + _E_RADIUS * np.exp(1j * (np.pi - th0)), _E_CENTRE + _E_RADIUS * np.exp(1j * th0))


def square_well_delta(energies, lmax: int, v0: float, r_mt: float = R_MT) -> np.ndarray:
    """Complex phase shifts delta_l(E) of a square well V = -v0 for r < r_mt.

    Continuity of the logarithmic derivative at r_mt between j_l(q r) inside
    (q = sqrt(E + v0)) and cos(d) j_l(k r) - sin(d) y_l(k r) outside
    (k = sqrt(E), principal branch) gives tan(d) = num / den.
    Returns an array [len(energies), lmax + 1] of complex128.
    """
    e = np.asarray(energies, dtype=complex)
    kap = np.sqrt(e)
    q = np.sqrt(e + v0)
    x = kap * r_mt
    y = q * r_mt
    out = np.empty(e.shape + (lmax + 1,), dtype=complex)
    for l in range(lmax + 1):
        jx = spherical_jn(l, x)
        jpx = spherical_jn(l, x, derivative=True)
        yx = spherical_yn(l, x)
        ypx = spherical_yn(l, x, derivative=True)
        jy = spherical_jn(l, y)
        jpy = spherical_jn(l, y, derivative=True)
        num = kap * jpx * jy - q * jx * jpy
        den = kap * ypx * jy - q * yx * jpy
        out[..., l] = np.arctan(num / den)
    return out


def phase_shift_table(energies, lmax: int, depths=V0_SPECIES) -> np.ndarray:
    """delta[species][energy][l] for every species' square well."""
    return np.stack([square_well_delta(energies, lmax, v0) for v0 in depths])


def spin_phase_shift_tables(energies, lmax: int, depths=V0_SPECIES, splits=SPLIT_SPECIES):
    """(delta_up, delta_dn), each [species][energy][l]: the phase shifts of the
    spin parallel (well depth v0 + split/2) and antiparallel (v0 - split/2) to
    a site's moment."""
    up = np.stack([square_well_delta(energies, lmax, v0 + 0.5 * d) for v0, d in zip(depths, splits)])
    dn = np.stack([square_well_delta(energies, lmax, v0 - 0.5 * d) for v0, d in zip(depths, splits)])
    return up, dn


@dataclasses.dataclass
class Workload:
    """Everything the path takes for a batch of (site, energy) instances.

    atom_pos/atom_species describe the periodic supercell (box lengths in
    `box`); instance i is centred on atom `centre[i]` with LIZ cutoff radius
    `rc[i]` (bohr) at energy `energies[e_idx[i]]`.  `delta` holds the phase
    shifts [n_species][n_energy][lmax + 1].  Spin-canted workloads also carry
    a unit moment direction per atom (`atom_moment` [n_atoms, 3]) and the
    phase shifts of the spin antiparallel to the moment (`delta_dn`, layout of
    `delta`, which then holds the parallel spin).
    """

    name: str
    lmax: int
    box: np.ndarray
    atom_pos: np.ndarray
    atom_species: np.ndarray
    energies: np.ndarray
    delta: np.ndarray
    centre: np.ndarray
    rc: np.ndarray
    e_idx: np.ndarray
    atom_moment: np.ndarray | None = None
    delta_dn: np.ndarray | None = None

    @property
    def n_inst(self) -> int:
        return int(self.centre.shape[0])

    @property
    def kk(self) -> int:
        return (self.lmax + 1) ** 2

    @property
    def spin(self) -> bool:
        return self.atom_moment is not None

    def with_lmax(self, lmax: int) -> "Workload":
        name = f"{self.name.rsplit('-lmax', 1)[0]}-lmax{lmax}"
        if self.spin:
            up, dn = spin_phase_shift_tables(self.energies, lmax)
            return dataclasses.replace(self, lmax=lmax, delta=up, delta_dn=dn, name=name)
        return dataclasses.replace(self, lmax=lmax, delta=phase_shift_table(self.energies, lmax), name=name)


def _children(seed: int):
    return np.random.SeedSequence(seed).spawn(5)


def config1(seed: int = 0) -> Workload:
    """Tiny case: 2x2x2 cells (32 atoms), Bernoulli(0.5) species, centres are
    sites 0..7, cutoff 0.75a (13-atom LIZ), 16 energies, lmax = 3: 128 instances."""
    rng = np.random.default_rng(_children(seed)[0])
    pos, box = fcc_supercell(2)
    species = (rng.random(pos.shape[0]) < 0.5).astype(np.int32)
    e = contour_energies(16)
    sites = np.repeat(np.arange(8), e.size)
    eidx = np.tile(np.arange(e.size), 8)
    return Workload("fcc-NiAu-13atomLIZ-lmax3", 3, box, pos, species, e,
                    phase_shift_table(e, 3), sites.astype(np.int32),
                    np.full(sites.size, 0.75 * A_LAT), eidx.astype(np.int32))


def config2(seed: int = 0) -> Workload:
    """Real shape: 4x4x4 cells (256 atoms), exactly 128 Ni + 128 Au, every site a
    centre, cutoff 1.9a (135-atom LIZ, N = 2160 at lmax = 3), 32 energies:
    8192 instances, site-major."""
    rng = np.random.default_rng(_children(seed)[1])
    pos, box = fcc_supercell(4)
    species = rng.permutation(np.repeat(np.array([0, 1], np.int32), pos.shape[0] // 2))
    e = contour_energies(32)
    sites = np.repeat(np.arange(pos.shape[0]), e.size)
    eidx = np.tile(np.arange(e.size), pos.shape[0])
    return Workload("fcc-NiAu-135atomLIZ-lmax3", 3, box, pos, species.astype(np.int32), e,
                    phase_shift_table(e, 3), sites.astype(np.int32),
                    np.full(sites.size, 1.9 * A_LAT), eidx.astype(np.int32))


def config3(seed: int = 0, lmax: int = 4) -> Workload:
    """The config-2 systems at another lmax (lmax = 4 gives N = 3375)."""
    return config2(seed).with_lmax(lmax)


def canted_moments(n_atoms: int, seed: int = 0, cone_deg: float = 60.0) -> np.ndarray:
    """Unit moment directions [n_atoms, 3], canted from +z: polar angle
    uniform in [0, cone_deg], azimuth uniform in [0, 2 pi)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(7)[6])
    th = np.deg2rad(rng.uniform(0.0, cone_deg, n_atoms))
    ph = rng.uniform(0.0, 2.0 * np.pi, n_atoms)
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def config_canted(seed: int = 0, lmax: int = 3) -> Workload:
    """Spin-canted case: the config-2 systems (135-atom LIZ) with a canted
    moment on every atom and spin-split square wells; rank 2 kk 135 = 4320
    at lmax = 3, 6750 at lmax = 4 (the CoCrFeMnNi rank of the paper's
    spin-canted benchmark).  8192 instances, site-major."""
    w = config2(seed)
    up, dn = spin_phase_shift_tables(w.energies, lmax)
    return dataclasses.replace(w, name=f"fcc-NiAu-canted-135atomLIZ-lmax{lmax}", lmax=lmax, delta=up, delta_dn=dn,
                               atom_moment=canted_moments(w.atom_pos.shape[0], seed))


def config_large(seed: int = 0, lmax: int = 4) -> Workload:
    """One matrix per instance at the paper's non-canted NiAu rank: 6x6x6 fcc
    cells (864 atoms, box 6a, so that the cutoff stays below half the box),
    exact 50/50 species, cutoff 2.46a (the shell closure of 249 atoms: N =
    25 * 249 = 6225 at lmax = 4), 32 energies; 864 x 32 instances, site-major."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(8)[7])
    pos, box = fcc_supercell(6)
    species = rng.permutation(np.repeat(np.array([0, 1], np.int32), pos.shape[0] // 2))
    e = contour_energies(32)
    sites = np.repeat(np.arange(pos.shape[0]), e.size)
    eidx = np.tile(np.arange(e.size), pos.shape[0])
    return Workload(f"fcc-NiAu-249atomLIZ-lmax{lmax}", lmax, box, pos, species.astype(np.int32), e,
                    phase_shift_table(e, lmax), sites.astype(np.int32), np.full(sites.size, 2.46 * A_LAT),
                    eidx.astype(np.int32))


def config4(seed: int = 0, n_inst: int = 1024) -> Workload:
    """Ragged case: 10x10x10 cells (4000 sites), 3% vacancies, Gaussian noise
    sigma = 0.02a per component, exact 50/50 species over occupied sites,
    `n_inst` (site, energy) pairs drawn without replacement over occupied sites
    x 32 energies, cutoff radius uniform in [1.7a, 2.1a] per instance."""
    rng = np.random.default_rng(_children(seed)[3])
    pos, box = fcc_supercell(10)
    keep = rng.random(pos.shape[0]) >= 0.03
    pos = pos[keep] + rng.normal(0.0, 0.02 * A_LAT, size=(int(keep.sum()), 3))
    n_occ = pos.shape[0]
    species = rng.permutation(np.concatenate([np.zeros(n_occ // 2, np.int32),
                                              np.ones(n_occ - n_occ // 2, np.int32)]))
    e = contour_energies(32)
    pick = rng.choice(n_occ * e.size, size=n_inst, replace=False)
    sites = (pick // e.size).astype(np.int32)
    eidx = (pick % e.size).astype(np.int32)
    rc = rng.uniform(1.7 * A_LAT, 2.1 * A_LAT, size=n_inst)
    return Workload("fcc-NiAu-vac-noise-ragged-lmax3", 3, box, pos, species.astype(np.int32), e,
                    phase_shift_table(e, 3), sites, rc, eidx)


def subset(w: Workload, idx) -> Workload:
    """The same system restricted to the instances `idx`."""
    idx = np.asarray(idx)
    return dataclasses.replace(w, centre=w.centre[idx], rc=w.rc[idx], e_idx=w.e_idx[idx])


# layer widths of the learned form's network (18 features -> 1024 outputs)
MLP_LAYERS = (18, 256, 256, 256, 1024)


def mlp_init(seed: int = 0) -> np.ndarray:
    """Initial parameters of the learned form's network as one flat float64
    vector [W1 b1 W2 b2 W3 b3 W4 b4], W_l of shape [out][in] drawn from
    N(0, 1/in) (scaled by 0.1 for the output layer), biases zero."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[5])
    parts = []
    dims = list(zip(MLP_LAYERS[:-1], MLP_LAYERS[1:]))
    for l, (i, o) in enumerate(dims):
        scale = (0.1 if l + 1 == len(dims) else 1.0) / np.sqrt(i)
        parts.append(rng.standard_normal(o * i) * scale)
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def config_large_canted(seed: int = 0, lmax: int = 4) -> Workload:
    """The large-instance systems (249-atom LIZ) with a canted moment on every
    atom and spin-split square wells: rank 2 kk 249 = 12450 at lmax = 4, the
    paper's spin-canted NiAu rank.  864 x 32 instances, site-major."""
    w = config_large(seed, lmax)
    up, dn = spin_phase_shift_tables(w.energies, lmax)
    return dataclasses.replace(w, name=f"fcc-NiAu-canted-249atomLIZ-lmax{lmax}", delta=up, delta_dn=dn,
                               atom_moment=canted_moments(w.atom_pos.shape[0], seed))
