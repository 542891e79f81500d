/*
 * Plain CPU FP64 oracle for the LSMS tau00 path.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the product library never does.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * What it computes.  The paper obtains the multiple-scattering matrix from
 * the Dyson equation tau = [t^{-1} - g0]^{-1} (Sec. 2.1, eq. Dyson_equation)
 * and, in LSMS, builds that matrix per atom over the atom's local interaction
 * zone (LIZ) and keeps only the central block tau^{00} (Sec. 2.2).  Written
 * with M = 1 - t G (block (i,j) = delta_ij I - t_i G^{ij}), the same block is
 * tau00 = [M^{-1}]_{00} t_0.  The oracle takes the plain definition:
 *   - LIZ: atoms within the cutoff of the centre (minimum image), centre first;
 *   - t_l = -(1/kappa) sin(delta_l) exp(i delta_l), kappa = sqrt(E);
 *   - G^{ij}_{LL'} = -4 pi i kappa sum_L'' i^{l-l'+l''} C^{L''}_{LL'}
 *                     h_{l''}(kappa |R_ij|) Y_{L''}(R_ij/|R_ij|),  R_ij = R_i - R_j,
 *     the expansion of the free propagator -exp(i kappa r)/(4 pi r) between
 *     two sites (g0 of Sec. 2.1) in real spherical harmonics (no Condon-Shortley
 *     phase, L = l*l + l + m) and spherical Bessel functions;
 *   - M assembled, factorised by LU with row partial pivoting (the zgetrf
 *     semantics the paper's GPU path uses, Sec. 3.2), solved for the first
 *     kk unit columns, refined twice with residuals accumulated in 80-bit
 *     long double, tau00 = X_00 diag(t_0).
 *   - The Schur-complement route of Sec. 2.2 (only the first block of the
 *     inverse is needed) is provided separately so that tests can check that
 *     both give the same block.
 *   - The block row tau^{0j} = [M^{-1}]_{0j} t_j of the multiple-scattering
 *     matrix tau = M^{-1} t (eq. Dyson_equation: (t^{-1} - g0)^{-1} =
 *     (1 - t g0)^{-1} t), whose blocks feed the Green's function of
 *     eq. Green_KKR: rows 0..kk-1 of M^{-1} from M^T Z = E_0, refined as above.
 *   - The spin-canted matrix (rank 2 kk n_liz, Sec. 2.1) and its tau00, with
 *     the global-frame t of a canted site written out from the rotation of
 *     its spin-diagonal local t (the reading is stated at that code).
 *   - ln det M from the same LU (the sum of the logarithms of U's diagonal and
 *     i pi per row interchange), the quantity Lloyd's formula turns into the
 *     multiple-scattering part of the integrated density of states behind
 *     eq. Density.
 *
 * Units: Rydberg atomic units (E in Ry, lengths in bohr).  Complex matrices
 * are column-major, interleaved (re, im).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;
typedef long double complex lzc;

#define ORC_PI 3.14159265358979323846264338327950288

/* OpenMP thread count used by orc_tau00_batch. */
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* a1: local interaction zone                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    double d2, dx, dy, dz;
    int idx;
} orc_cand;

static int orc_cand_cmp(const void *pa, const void *pb)
{
    const orc_cand *a = (const orc_cand *)pa, *b = (const orc_cand *)pb;
    if (a->d2 != b->d2) return a->d2 < b->d2 ? -1 : 1;
    if (a->dx != b->dx) return a->dx < b->dx ? -1 : 1;
    if (a->dy != b->dy) return a->dy < b->dy ? -1 : 1;
    if (a->dz != b->dz) return a->dz < b->dz ? -1 : 1;
    return a->idx - b->idx;
}

/* LIZ of atom `centre` (Sec. 2.2): every other atom whose minimum-image
 * vector d = R_j - R_c (each component reduced by box * rint(d / box))
 * satisfies dx*dx + dy*dy + dz*dz <= rc*rc.  Output: the centre first
 * (relative vector 0), then the members by ascending squared distance, ties
 * broken by (dx, dy, dz) lexicographically.  Writes at most max_out rows of
 * rel[.,3] / idx[.] and returns the LIZ size (which may exceed max_out). */
int orc_liz(const double *pos, int n_atoms, const double *box, int centre, double rc,
            int max_out, double *rel, int32_t *idx)
{
    orc_cand *c = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(n_atoms > 0 ? n_atoms : 1));
    int n = 0;
    const double *p0 = pos + 3 * (size_t)centre;
    const double rc2 = rc * rc;
    for (int j = 0; j < n_atoms; ++j) {
        if (j == centre) continue;
        double d[3];
        for (int k = 0; k < 3; ++k) {
            d[k] = pos[3 * (size_t)j + k] - p0[k];
            d[k] -= box[k] * rint(d[k] / box[k]);
        }
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (d2 <= rc2) {
            c[n].d2 = d2; c[n].dx = d[0]; c[n].dy = d[1]; c[n].dz = d[2]; c[n].idx = j;
            ++n;
        }
    }
    qsort(c, (size_t)n, sizeof(orc_cand), orc_cand_cmp);
    if (max_out >= 1) {
        rel[0] = rel[1] = rel[2] = 0.0;
        idx[0] = centre;
    }
    for (int q = 0; q < n && q + 1 < max_out; ++q) {
        rel[3 * (q + 1) + 0] = c[q].dx;
        rel[3 * (q + 1) + 1] = c[q].dy;
        rel[3 * (q + 1) + 2] = c[q].dz;
        idx[q + 1] = c[q].idx;
    }
    free(c);
    return n + 1;
}

/* ------------------------------------------------------------------ */
/* Angular and radial functions                                        */
/* ------------------------------------------------------------------ */

/* Real spherical harmonics Y_L(r/|r|), L = l*l + l + m, l <= lmax:
 *   Y_{l0}  = N_{l0} P_l(cos th)
 *   Y_{lm}  = sqrt2 N_{lm} P_l^m(cos th) cos(m phi)      m > 0
 *   Y_{l-m} = sqrt2 N_{lm} P_l^m(cos th) sin(m phi)      m > 0
 * with N_{lm} = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^m without the
 * Condon-Shortley factor (P_m^m = (2m-1)!! sin^m th >= 0). */
void orc_ylm(int lmax, const double *r, double *Y)
{
    const double x = r[0], y = r[1], z = r[2];
    const double rr = sqrt(x * x + y * y + z * z);
    const double ct = z / rr;
    const double st = sqrt(x * x + y * y) / rr;
    const double phi = atan2(y, x);
    for (int m = 0; m <= lmax; ++m) {
        /* P_m^m, then upward in l */
        double pmm = 1.0;
        for (int k = 1; k <= m; ++k) pmm *= (2.0 * k - 1.0) * st;
        double plm2 = 0.0, plm1 = pmm;
        for (int l = m; l <= lmax; ++l) {
            double p;
            if (l == m) p = pmm;
            else if (l == m + 1) p = ct * (2.0 * m + 1.0) * pmm;
            else p = ((2.0 * l - 1.0) * ct * plm1 - (l + m - 1.0) * plm2) / (double)(l - m);
            if (l > m) { plm2 = plm1; plm1 = p; }
            double ratio = 1.0; /* (l-m)!/(l+m)! */
            for (int k = l - m + 1; k <= l + m; ++k) ratio /= (double)k;
            const double nlm = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * ratio);
            if (m == 0) {
                Y[l * l + l] = nlm * p;
            } else {
                Y[l * l + l + m] = sqrt(2.0) * nlm * p * cos(m * phi);
                Y[l * l + l - m] = sqrt(2.0) * nlm * p * sin(m * phi);
            }
        }
    }
}

/* Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n. */
static void orc_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double t = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            /* p1 = P_n(t), p0 = P_{n-1}(t) */
            double dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        double dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

/* Real Gaunt coefficients C[(L*kk + L')*kk2 + L''] = int Y_L Y_L' Y_L'' dOmega
 * for l, l' <= lmax and l'' <= 2 lmax (kk = (lmax+1)^2, kk2 = (2lmax+1)^2),
 * by a product rule that is exact for the integrand's degree 4 lmax:
 * Gauss-Legendre in cos(theta) and the uniform rule in phi.  Entries that the
 * selection rules make zero (l+l'+l'' odd, l'' outside |l-l'|..l+l', or a
 * vanishing m combination, which the rule returns at rounding level) are set
 * to exactly zero.  Returns the number of nonzero entries. */
int orc_gaunt(int lmax, double *C)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int l2 = 2 * lmax;
    const int kk2 = (l2 + 1) * (l2 + 1);
    const int nth = 2 * lmax + 4, nph = 4 * lmax + 4;
    double *xg = (double *)malloc(sizeof(double) * nth);
    double *wg = (double *)malloc(sizeof(double) * nth);
    double *Y = (double *)malloc(sizeof(double) * kk2);
    orc_gauss_legendre(nth, xg, wg);
    memset(C, 0, sizeof(double) * (size_t)kk * kk * kk2);
    for (int a = 0; a < nth; ++a) {
        for (int b = 0; b < nph; ++b) {
            const double phi = 2.0 * ORC_PI * b / nph;
            const double st = sqrt(1.0 - xg[a] * xg[a]);
            const double r[3] = {st * cos(phi), st * sin(phi), xg[a]};
            orc_ylm(l2, r, Y);
            const double wt = wg[a] * 2.0 * ORC_PI / nph;
            for (int L = 0; L < kk; ++L)
                for (int Lp = 0; Lp < kk; ++Lp) {
                    const double yy = wt * Y[L] * Y[Lp];
                    double *row = C + ((size_t)L * kk + Lp) * kk2;
                    for (int Lpp = 0; Lpp < kk2; ++Lpp) row[Lpp] += yy * Y[Lpp];
                }
        }
    }
    int nnz = 0;
    for (int L = 0; L < kk; ++L) {
        const int l = (int)floor(sqrt((double)L) + 1e-9);
        for (int Lp = 0; Lp < kk; ++Lp) {
            const int lp = (int)floor(sqrt((double)Lp) + 1e-9);
            for (int Lpp = 0; Lpp < kk2; ++Lpp) {
                const int lpp = (int)floor(sqrt((double)Lpp) + 1e-9);
                double *c = C + ((size_t)L * kk + Lp) * kk2 + Lpp;
                const int lo = l > lp ? l - lp : lp - l;
                if (((l + lp + lpp) & 1) || lpp < lo || lpp > l + lp || fabs(*c) < 1e-13) *c = 0.0;
                else ++nnz;
            }
        }
    }
    free(xg); free(wg); free(Y);
    return nnz;
}

static const zc ORC_IPOW[4] = {1.0, I, -1.0, -I}; /* i^n, n mod 4 */

/* Spherical Hankel functions of the first kind h_l(z), l = 0..lmax, from the
 * finite sum h_l(z) = (-i)^{l+1} (e^{iz}/z) sum_{k=0}^{l} i^k (l+k)! / (k! (l-k)!) (2z)^{-k}. */
void orc_hankel(int lmax, const double *zri, double *hri)
{
    const zc z = zri[0] + I * zri[1];
    const zc ez = cexp(I * z) / z;
    for (int l = 0; l <= lmax; ++l) {
        zc s = 0.0;
        zc zk = 1.0;
        for (int k = 0; k <= l; ++k) {
            double coef = 1.0; /* (l+k)! / (k! (l-k)!) */
            for (int q = l - k + 1; q <= l + k; ++q) coef *= (double)q;
            for (int q = 2; q <= k; ++q) coef /= (double)q;
            s += ORC_IPOW[k & 3] * coef * zk;
            zk /= (2.0 * z);
        }
        /* (-i)^{l+1} = i^{3(l+1)} */
        const zc h = ORC_IPOW[(3 * (l + 1)) & 3] * ez * s;
        hri[2 * l] = creal(h);
        hri[2 * l + 1] = cimag(h);
    }
}

/* Single-site t-matrix t_l = -(1/kappa) sin(delta_l) e^{i delta_l}, kappa = sqrt(E). */
void orc_tmat(int lmax, const double *Eri, const double *dri, double *tri)
{
    const zc E = Eri[0] + I * Eri[1];
    const zc kap = csqrt(E);
    for (int l = 0; l <= lmax; ++l) {
        const zc d = dri[2 * l] + I * dri[2 * l + 1];
        const zc t = -csin(d) * cexp(I * d) / kap;
        tri[2 * l] = creal(t);
        tri[2 * l + 1] = cimag(t);
    }
}

static int orc_lof(int L) { return (int)floor(sqrt((double)L) + 1e-9); }

/* Structure constants G^{ij} (kk x kk, column-major, G[L + kk L']) for the
 * separation R = R_i - R_j and kappa = sqrt(E); `gaunt` from orc_gaunt(lmax). */
static void orc_gij(int lmax, zc kap, const double *R, const double *gaunt, zc *G)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int l2 = 2 * lmax;
    const int kk2 = (l2 + 1) * (l2 + 1);
    double Y[(2 * 8 + 1) * (2 * 8 + 1) * 4];
    double hri[2 * (2 * 16 + 2)];
    double *Yp = Y;
    double *Ybig = NULL;
    if (kk2 > (int)(sizeof(Y) / sizeof(Y[0]))) { Ybig = (double *)malloc(sizeof(double) * kk2); Yp = Ybig; }
    double *hbig = NULL, *hp = hri;
    if (2 * (l2 + 1) > (int)(sizeof(hri) / sizeof(hri[0]))) { hbig = (double *)malloc(sizeof(double) * 2 * (l2 + 1)); hp = hbig; }
    const double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    orc_ylm(l2, R, Yp);
    const zc z = kap * r;
    const double zri[2] = {creal(z), cimag(z)};
    orc_hankel(l2, zri, hp);
    const zc pref = -4.0 * ORC_PI * I * kap;
    for (int Lp = 0; Lp < kk; ++Lp) {
        const int lp = orc_lof(Lp);
        for (int L = 0; L < kk; ++L) {
            const int l = orc_lof(L);
            const double *c = gaunt + ((size_t)L * kk + Lp) * kk2;
            zc s = 0.0;
            for (int Lpp = 0; Lpp < kk2; ++Lpp) {
                if (c[Lpp] == 0.0) continue;
                const int lpp = orc_lof(Lpp);
                const int e = ((l - lp + lpp) % 4 + 4) % 4;
                const zc h = hp[2 * lpp] + I * hp[2 * lpp + 1];
                s += ORC_IPOW[e] * c[Lpp] * h * Yp[Lpp];
            }
            G[L + (size_t)kk * Lp] = pref * s;
        }
    }
    free(Ybig);
    free(hbig);
}

/* Exported for the structure-constant pins: G (kk x kk, interleaved complex). */
void orc_structure_constants(int lmax, const double *kri, const double *R, const double *gaunt,
                             double *Gri)
{
    const zc kap = kri[0] + I * kri[1];
    orc_gij(lmax, kap, R, gaunt, (zc *)Gri);
}

/* ------------------------------------------------------------------ */
/* a2 + a3: KKR matrix over one LIZ                                    */
/* ------------------------------------------------------------------ */

/* M = 1 - t G over the LIZ (n_liz sites, rel[n_liz][3] relative positions,
 * spec[n_liz] species), for energy E and phase shifts dl[s*(lmax+1) + l]
 * (the species' delta_l at this energy).  M is N x N column-major,
 * N = kk * n_liz, row kk*i + L, column kk*j + L':
 *   M_ii = I,  M_ij = -diag(t_{s(i), l(L)}) G^{ij}.
 * Returns 0, or -2 when two LIZ sites coincide (|R_ij| < 1e-8 bohr). */
static int orc_build_m_z(int lmax, int n_liz, const double *rel, const int32_t *spec, zc E,
                         const zc *dl, int n_species, const double *gaunt, zc *M)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const size_t N = (size_t)kk * n_liz;
    const zc kap = csqrt(E);
    zc *t = (zc *)malloc(sizeof(zc) * (size_t)n_species * (lmax + 1));
    for (int s = 0; s < n_species; ++s)
        for (int l = 0; l <= lmax; ++l) {
            const zc d = dl[s * (lmax + 1) + l];
            t[s * (lmax + 1) + l] = -csin(d) * cexp(I * d) / kap;
        }
    zc *G = (zc *)malloc(sizeof(zc) * kk * kk);
    memset(M, 0, sizeof(zc) * N * N);
    int rc = 0;
    for (int j = 0; j < n_liz; ++j) {
        for (int i = 0; i < n_liz; ++i) {
            if (i == j) {
                for (int L = 0; L < kk; ++L) M[(kk * i + L) + N * (kk * j + L)] = 1.0;
                continue;
            }
            double R[3];
            for (int k = 0; k < 3; ++k) R[k] = rel[3 * i + k] - rel[3 * j + k];
            if (sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]) < 1e-8) { rc = -2; continue; }
            orc_gij(lmax, kap, R, gaunt, G);
            for (int Lp = 0; Lp < kk; ++Lp)
                for (int L = 0; L < kk; ++L) {
                    const zc ti = t[spec[i] * (lmax + 1) + orc_lof(L)];
                    M[(kk * i + L) + N * (kk * j + Lp)] = -ti * G[L + kk * Lp];
                }
        }
    }
    free(G);
    free(t);
    return rc;
}

int orc_build_m(int lmax, int n_liz, const double *rel, const int32_t *spec, const double *Eri,
                const double *dri, int n_species, const double *gaunt, double *Mri)
{
    const zc E = Eri[0] + I * Eri[1];
    return orc_build_m_z(lmax, n_liz, rel, spec, E, (const zc *)dri, n_species, gaunt, (zc *)Mri);
}

/* ------------------------------------------------------------------ */
/* a4 + a5: LU with partial pivoting, solve, tau00                     */
/* ------------------------------------------------------------------ */

static double orc_cabs1(zc a) { return fabs(creal(a)) + fabs(cimag(a)); }

/* Doolittle LU with row partial pivoting of the n x n column-major A in
 * place: the pivot of column k is the row in k..n-1 maximising |Re| + |Im|,
 * the lowest such row on ties.  ipiv[k] = pivot row (0-based).  Returns 0 or
 * k + 1 for the first column whose pivot is exactly zero (the factorisation
 * continues, as zgetrf does). */
int orc_lu_factor(int n, double *Ari, int32_t *ipiv)
{
    zc *A = (zc *)Ari;
    const size_t ld = (size_t)n;
    int info = 0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = orc_cabs1(A[k + ld * k]);
        for (int i = k + 1; i < n; ++i) {
            const double v = orc_cabs1(A[i + ld * k]);
            if (v > best) { best = v; p = i; }
        }
        ipiv[k] = p;
        if (best == 0.0) {
            if (!info) info = k + 1;
            continue;
        }
        if (p != k)
            for (int j = 0; j < n; ++j) {
                const zc tmp = A[k + ld * j];
                A[k + ld * j] = A[p + ld * j];
                A[p + ld * j] = tmp;
            }
        const zc inv = 1.0 / A[k + ld * k];
        for (int i = k + 1; i < n; ++i) A[i + ld * k] *= inv;
        for (int j = k + 1; j < n; ++j) {
            const zc u = A[k + ld * j];
            if (u == 0.0) continue;
            zc *cj = A + ld * j;
            const zc *ck = A + ld * k;
            for (int i = k + 1; i < n; ++i) cj[i] -= ck[i] * u;
        }
    }
    return info;
}

/* Solve A X = B for nrhs columns of B (n x nrhs, column-major) in place,
 * from orc_lu_factor's output. */
void orc_lu_solve(int n, const double *LUri, const int32_t *ipiv, int nrhs, double *Bri)
{
    const zc *A = (const zc *)LUri;
    zc *B = (zc *)Bri;
    const size_t ld = (size_t)n;
    for (int r = 0; r < nrhs; ++r) {
        zc *b = B + ld * r;
        for (int k = 0; k < n; ++k)
            if (ipiv[k] != k) { const zc tmp = b[k]; b[k] = b[ipiv[k]]; b[ipiv[k]] = tmp; }
        for (int k = 0; k < n; ++k) {
            const zc bk = b[k];
            if (bk == 0.0) continue;
            for (int i = k + 1; i < n; ++i) b[i] -= A[i + ld * k] * bk;
        }
        for (int k = n - 1; k >= 0; --k) {
            b[k] /= A[k + ld * k];
            const zc bk = b[k];
            if (bk == 0.0) continue;
            for (int i = 0; i < k; ++i) b[i] -= A[i + ld * k] * bk;
        }
    }
}

/* R = B - A X with every product and sum carried in 80-bit long double. */
static void orc_residual_ld(int n, int nrhs, const zc *A, const zc *X, const zc *B, zc *R)
{
    const size_t ld = (size_t)n;
    lzc *acc = (lzc *)malloc(sizeof(lzc) * ld);
    for (int r = 0; r < nrhs; ++r) {
        for (int i = 0; i < n; ++i) acc[i] = (lzc)B[i + ld * r];
        for (int k = 0; k < n; ++k) {
            const lzc xk = (lzc)X[k + ld * r];
            const zc *ak = A + ld * k;
            for (int i = 0; i < n; ++i) acc[i] -= (lzc)ak[i] * xk;
        }
        for (int i = 0; i < n; ++i) R[i + ld * r] = (zc)acc[i];
    }
    free(acc);
}

static int orc_finite(const zc *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(creal(a[i])) || !isfinite(cimag(a[i]))) return 0;
    return 1;
}

/* tau00 of one instance by the full-matrix route.  tau is kk x kk
 * column-major.  Returns 0, k > 0 (zero pivot), -1 (non-finite input or
 * output) or -2 (coincident sites); tau is NaN on any nonzero return. */
static int orc_tau00_one(int lmax, int n_liz, const double *rel, const int32_t *spec, zc E,
                         const zc *dl, int n_species, const double *gaunt, int refine, zc *tau)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int n = kk * n_liz;
    const size_t nn = (size_t)n * n;
    int info = 0;
    for (int q = 0; q < kk * kk; ++q) tau[q] = NAN + I * NAN;
    if (!isfinite(creal(E)) || !isfinite(cimag(E)) || !orc_finite(dl, (size_t)n_species * (lmax + 1)))
        return -1;
    zc *M = (zc *)malloc(sizeof(zc) * nn);
    zc *LU = (zc *)malloc(sizeof(zc) * nn);
    zc *X = (zc *)calloc((size_t)n * kk, sizeof(zc));
    zc *E0 = (zc *)calloc((size_t)n * kk, sizeof(zc));
    zc *R = (zc *)malloc(sizeof(zc) * (size_t)n * kk);
    int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * n);
    info = orc_build_m_z(lmax, n_liz, rel, spec, E, dl, n_species, gaunt, M);
    if (info == 0 && !orc_finite(M, nn)) info = -1;
    if (info == 0) {
        memcpy(LU, M, sizeof(zc) * nn);
        info = orc_lu_factor(n, (double *)LU, ipiv);
    }
    if (info == 0) {
        for (int c = 0; c < kk; ++c) E0[c + (size_t)n * c] = 1.0;
        memcpy(X, E0, sizeof(zc) * (size_t)n * kk);
        orc_lu_solve(n, (const double *)LU, ipiv, kk, (double *)X);
        for (int it = 0; it < refine; ++it) {
            orc_residual_ld(n, kk, M, X, E0, R);
            orc_lu_solve(n, (const double *)LU, ipiv, kk, (double *)R);
            for (size_t q = 0; q < (size_t)n * kk; ++q) X[q] += R[q];
        }
        const zc kap = csqrt(E);
        for (int Lp = 0; Lp < kk; ++Lp) {
            const zc d = dl[spec[0] * (lmax + 1) + orc_lof(Lp)];
            const zc t0 = -csin(d) * cexp(I * d) / kap;
            for (int L = 0; L < kk; ++L) tau[L + kk * Lp] = X[L + (size_t)n * Lp] * t0;
        }
        if (!orc_finite(tau, (size_t)kk * kk)) info = -1;
    }
    if (info != 0)
        for (int q = 0; q < kk * kk; ++q) tau[q] = NAN + I * NAN;
    free(M); free(LU); free(X); free(E0); free(R); free(ipiv);
    return info;
}

/* Batched tau00 over ragged LIZs, mirroring the library's problem layout:
 * instance i owns LIZ rows liz_off[i]..liz_off[i+1]-1 of pos[.,3] (relative
 * to its centre, row 0 = centre) and species[.]; its energy is
 * energy[e_idx[i]] and its phase shifts delta[(s*n_energy + e)*(lmax+1) + l].
 * tau00 is [n_inst][kk*kk]; info[i] as orc_tau00_one.  OpenMP over instances. */
void orc_tau00_batch(int lmax, int n_inst, const int64_t *liz_off, const double *pos,
                     const int32_t *species, const double *energy, const int32_t *e_idx,
                     const double *delta, int n_species, int n_energy, int refine,
                     double *tau00, int32_t *info)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int kk2 = (2 * lmax + 1) * (2 * lmax + 1);
    double *gaunt = (double *)malloc(sizeof(double) * (size_t)kk * kk * kk2);
    orc_gaunt(lmax, gaunt);
    const zc *Ez = (const zc *)energy;
    const zc *dz = (const zc *)delta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_inst; ++i) {
        const int e = e_idx[i];
        const int n_liz = (int)(liz_off[i + 1] - liz_off[i]);
        zc *dl = (zc *)malloc(sizeof(zc) * (size_t)n_species * (lmax + 1));
        for (int s = 0; s < n_species; ++s)
            for (int l = 0; l <= lmax; ++l)
                dl[s * (lmax + 1) + l] = dz[((size_t)s * n_energy + e) * (lmax + 1) + l];
        info[i] = orc_tau00_one(lmax, n_liz, pos + 3 * liz_off[i], species + liz_off[i], Ez[e], dl,
                                n_species, gaunt, refine, (zc *)tau00 + (size_t)i * kk * kk);
        free(dl);
    }
    free(gaunt);
}

/* The Schur-complement route (Sec. 2.2: only the first block of the inverse
 * is needed): with D = M_rr (all sites but the centre), factorised with
 * partial pivoting inside D,  S = M_00 - M_0r D^{-1} M_r0  and
 * [M^{-1}]_00 = S^{-1};  tau00 = S^{-1} diag(t_0).  Used to check that both
 * routes give the same block.  No refinement. */
int orc_tau00_schur(int lmax, int n_liz, const double *rel, const int32_t *spec, const double *Eri,
                    const double *dri, int n_species, const double *gaunt, double *tauri)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int n = kk * n_liz, nd = n - kk;
    const zc E = Eri[0] + I * Eri[1];
    const zc *dl = (const zc *)dri;
    zc *tau = (zc *)tauri;
    zc *M = (zc *)malloc(sizeof(zc) * (size_t)n * n);
    int info = orc_build_m_z(lmax, n_liz, rel, spec, E, dl, n_species, gaunt, M);
    zc *S = (zc *)malloc(sizeof(zc) * kk * kk);
    for (int c = 0; c < kk; ++c)
        for (int r = 0; r < kk; ++r) S[r + kk * c] = M[r + (size_t)n * c];
    if (info == 0 && nd > 0) {
        zc *D = (zc *)malloc(sizeof(zc) * (size_t)nd * nd);
        zc *Y = (zc *)malloc(sizeof(zc) * (size_t)nd * kk);
        int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * nd);
        for (int c = 0; c < nd; ++c)
            for (int r = 0; r < nd; ++r) D[r + (size_t)nd * c] = M[(kk + r) + (size_t)n * (kk + c)];
        for (int c = 0; c < kk; ++c)
            for (int r = 0; r < nd; ++r) Y[r + (size_t)nd * c] = M[(kk + r) + (size_t)n * c];
        info = orc_lu_factor(nd, (double *)D, ipiv);
        if (info == 0) {
            orc_lu_solve(nd, (const double *)D, ipiv, kk, (double *)Y);
            for (int c = 0; c < kk; ++c)
                for (int r = 0; r < kk; ++r) {
                    zc s = 0.0;
                    for (int k = 0; k < nd; ++k) s += M[r + (size_t)n * (kk + k)] * Y[k + (size_t)nd * c];
                    S[r + kk * c] -= s;
                }
        }
        free(D); free(Y); free(ipiv);
    }
    if (info == 0) {
        int32_t piv[64];
        zc *Z = (zc *)calloc((size_t)kk * kk, sizeof(zc));
        for (int c = 0; c < kk; ++c) Z[c + kk * c] = 1.0;
        info = orc_lu_factor(kk, (double *)S, piv);
        if (info == 0) orc_lu_solve(kk, (const double *)S, piv, kk, (double *)Z);
        const zc kap = csqrt(E);
        for (int Lp = 0; Lp < kk; ++Lp) {
            const zc d = dl[spec[0] * (lmax + 1) + orc_lof(Lp)];
            const zc t0 = -csin(d) * cexp(I * d) / kap;
            for (int L = 0; L < kk; ++L) tau[L + kk * Lp] = Z[L + kk * Lp] * t0;
        }
        free(Z);
    }
    free(S);
    free(M);
    return info;
}

/* ------------------------------------------------------------------ */
/* Block row of tau and ln det M                                       */
/* ------------------------------------------------------------------ */

/* tau^{0j} for every LIZ site j of one instance: out is kk x n column-major,
 * out[L + kk*(j*kk + L')] = [M^{-1}]_{0j}(L, L') t_{s(j), l(L')}.  The rows
 * 0..kk-1 of M^{-1} are Z^T with M^T Z = E_0 (E_0 the first kk unit columns),
 * solved by the LU of M^T and refined twice with 80-bit residuals.  Returns
 * as orc_tau00_one; out is NaN on a nonzero return. */
static int orc_tau_row_one(int lmax, int n_liz, const double *rel, const int32_t *spec, zc E,
                           const zc *dl, int n_species, const double *gaunt, int refine, zc *out)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int n = kk * n_liz;
    const size_t nn = (size_t)n * n;
    int info = 0;
    for (size_t q = 0; q < (size_t)kk * n; ++q) out[q] = NAN + I * NAN;
    if (!isfinite(creal(E)) || !isfinite(cimag(E)) || !orc_finite(dl, (size_t)n_species * (lmax + 1)))
        return -1;
    zc *M = (zc *)malloc(sizeof(zc) * nn);
    zc *MT = (zc *)malloc(sizeof(zc) * nn);
    zc *LU = (zc *)malloc(sizeof(zc) * nn);
    zc *Z = (zc *)calloc((size_t)n * kk, sizeof(zc));
    zc *E0 = (zc *)calloc((size_t)n * kk, sizeof(zc));
    zc *R = (zc *)malloc(sizeof(zc) * (size_t)n * kk);
    int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * n);
    info = orc_build_m_z(lmax, n_liz, rel, spec, E, dl, n_species, gaunt, M);
    if (info == 0 && !orc_finite(M, nn)) info = -1;
    if (info == 0) {
        for (int c = 0; c < n; ++c)
            for (int r = 0; r < n; ++r) MT[r + (size_t)n * c] = M[c + (size_t)n * r];
        memcpy(LU, MT, sizeof(zc) * nn);
        info = orc_lu_factor(n, (double *)LU, ipiv);
    }
    if (info == 0) {
        for (int c = 0; c < kk; ++c) E0[c + (size_t)n * c] = 1.0;
        memcpy(Z, E0, sizeof(zc) * (size_t)n * kk);
        orc_lu_solve(n, (const double *)LU, ipiv, kk, (double *)Z);
        for (int it = 0; it < refine; ++it) {
            orc_residual_ld(n, kk, MT, Z, E0, R);
            orc_lu_solve(n, (const double *)LU, ipiv, kk, (double *)R);
            for (size_t q = 0; q < (size_t)n * kk; ++q) Z[q] += R[q];
        }
        const zc kap = csqrt(E);
        for (int j = 0; j < n_liz; ++j)
            for (int Lp = 0; Lp < kk; ++Lp) {
                const int col = j * kk + Lp;
                const zc d = dl[spec[j] * (lmax + 1) + orc_lof(Lp)];
                const zc tj = -csin(d) * cexp(I * d) / kap;
                /* [M^{-1}]_{0, col}(L) = Z(col, L) */
                for (int L = 0; L < kk; ++L) out[L + (size_t)kk * col] = Z[col + (size_t)n * L] * tj;
            }
        if (!orc_finite(out, (size_t)kk * n)) info = -1;
    }
    if (info != 0)
        for (size_t q = 0; q < (size_t)kk * n; ++q) out[q] = NAN + I * NAN;
    free(M); free(MT); free(LU); free(Z); free(E0); free(R); free(ipiv);
    return info;
}

/* ln det M of one instance from the LU of M with row partial pivoting:
 * sum_k log U_kk plus i pi for every row interchange, the imaginary part
 * reduced to (-pi, pi] (the principal logarithm of det M).  Returns as
 * orc_tau00_one (a zero pivot gives k > 0 and ld = NaN). */
static int orc_logdet_one(int lmax, int n_liz, const double *rel, const int32_t *spec, zc E,
                          const zc *dl, int n_species, const double *gaunt, zc *ld)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int n = kk * n_liz;
    const size_t nn = (size_t)n * n;
    *ld = NAN + I * NAN;
    if (!isfinite(creal(E)) || !isfinite(cimag(E)) || !orc_finite(dl, (size_t)n_species * (lmax + 1)))
        return -1;
    zc *M = (zc *)malloc(sizeof(zc) * nn);
    int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * n);
    int info = orc_build_m_z(lmax, n_liz, rel, spec, E, dl, n_species, gaunt, M);
    if (info == 0 && !orc_finite(M, nn)) info = -1;
    if (info == 0) info = orc_lu_factor(n, (double *)M, ipiv);
    if (info == 0) {
        double re = 0.0, ph = 0.0;
        int swaps = 0;
        for (int k = 0; k < n; ++k) {
            const zc u = M[k + (size_t)n * k];
            re += log(cabs(u));
            ph += carg(u);
            swaps += ipiv[k] != k;
        }
        if (swaps & 1) ph += ORC_PI;
        ph = remainder(ph, 2.0 * ORC_PI);           /* [-pi, pi] */
        if (ph <= -ORC_PI) ph += 2.0 * ORC_PI;      /* (-pi, pi] */
        *ld = re + I * ph;
        if (!isfinite(re)) info = -1;
    }
    free(M); free(ipiv);
    return info;
}

static zc *orc_instance_delta(int lmax, const zc *dz, int n_species, int n_energy, int e)
{
    zc *dl = (zc *)malloc(sizeof(zc) * (size_t)n_species * (lmax + 1));
    for (int s = 0; s < n_species; ++s)
        for (int l = 0; l <= lmax; ++l) dl[s * (lmax + 1) + l] = dz[((size_t)s * n_energy + e) * (lmax + 1) + l];
    return dl;
}

/* Batched block rows: instance i's kk x N_i block row at out + 2*row_off[i]
 * doubles (complex offsets), problem layout as orc_tau00_batch. */
void orc_tau_row_batch(int lmax, int n_inst, const int64_t *liz_off, const double *pos, const int32_t *species,
                       const double *energy, const int32_t *e_idx, const double *delta, int n_species, int n_energy,
                       int refine, const int64_t *row_off, double *out, int32_t *info)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int kk2 = (2 * lmax + 1) * (2 * lmax + 1);
    double *gaunt = (double *)malloc(sizeof(double) * (size_t)kk * kk * kk2);
    orc_gaunt(lmax, gaunt);
    const zc *Ez = (const zc *)energy;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_inst; ++i) {
        zc *dl = orc_instance_delta(lmax, (const zc *)delta, n_species, n_energy, e_idx[i]);
        const int n_liz = (int)(liz_off[i + 1] - liz_off[i]);
        info[i] = orc_tau_row_one(lmax, n_liz, pos + 3 * liz_off[i], species + liz_off[i], Ez[e_idx[i]], dl,
                                  n_species, gaunt, refine, (zc *)out + row_off[i]);
        free(dl);
    }
    free(gaunt);
}

/* Batched ln det M: ld[i] complex, problem layout as orc_tau00_batch. */
void orc_logdet_batch(int lmax, int n_inst, const int64_t *liz_off, const double *pos, const int32_t *species,
                      const double *energy, const int32_t *e_idx, const double *delta, int n_species, int n_energy,
                      double *ld, int32_t *info)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int kk2 = (2 * lmax + 1) * (2 * lmax + 1);
    double *gaunt = (double *)malloc(sizeof(double) * (size_t)kk * kk * kk2);
    orc_gaunt(lmax, gaunt);
    const zc *Ez = (const zc *)energy;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_inst; ++i) {
        zc *dl = orc_instance_delta(lmax, (const zc *)delta, n_species, n_energy, e_idx[i]);
        const int n_liz = (int)(liz_off[i + 1] - liz_off[i]);
        info[i] = orc_logdet_one(lmax, n_liz, pos + 3 * liz_off[i], species + liz_off[i], Ez[e_idx[i]], dl,
                                 n_species, gaunt, (zc *)ld + i);
        free(dl);
    }
    free(gaunt);
}

/* ------------------------------------------------------------------ */
/* Spin-canted KKR matrix and tau00                                    */
/* ------------------------------------------------------------------ */
/* With spin canting (non-collinear moments) every matrix carries a spin
 * index and the rank doubles to 2 kk n_liz (paper Sec. 2.1 and 2.2).  The
 * paper does not spell out how the spin enters; the reading taken here is
 * the usual one for non-collinear multiple scattering: site i has a unit
 * moment direction e_i and, in its own frame (spin axis along e_i), the
 * spin-diagonal t-matrix diag(t_up, t_dn), t_up from the phase shifts of the
 * spin parallel to the moment.  Rotated to the global frame by the spin-1/2
 * rotation U that takes z to e_i,
 *     t_i(L) = U diag(t_up,l, t_dn,l) U^+ = tbar_l 1 + dt_l (e_i . sigma),
 * tbar = (t_up + t_dn)/2, dt = (t_up - t_dn)/2, sigma the Pauli matrices.
 * The free propagator does not act on spin (G (x) 1).  Row/column index of
 * (site j, spin s, L): 2 kk j + kk s + L, s = 0 the spin along global +z.
 *     M_ii = 1,   M_ij[(s,L),(s',L')] = -t_i(L)_{s s'} G^{ij}_{L L'}
 *     tau00[(s,L),(s',L')] = sum_s'' [M^{-1}]_{00}[(s,L),(s'',L')] t_0(L')_{s'' s'}
 */

/* t of one channel in the global frame: t2[2 s + s'] = t(L)_{s s'}. */
static void orc_spin_t(zc tu, zc td, const double *e, zc *t2)
{
    const zc tb = 0.5 * (tu + td), dt = 0.5 * (tu - td);
    t2[0] = tb + dt * e[2];
    t2[1] = dt * (e[0] - I * e[1]);
    t2[2] = dt * (e[0] + I * e[1]);
    t2[3] = tb - dt * e[2];
}

/* Spin-canted M over one LIZ (2 kk n_liz square, column-major); mom[n_liz][3]
 * unit moment directions, dlu / dld the up / down phase shifts
 * [s*(lmax+1) + l] at this energy.  Returns as orc_build_m_z. */
static int orc_build_m_spin_z(int lmax, int n_liz, const double *rel, const int32_t *spec, const double *mom,
                              zc E, const zc *dlu, const zc *dld, int n_species, const double *gaunt, zc *M)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int nl = lmax + 1;
    const size_t N = (size_t)2 * kk * n_liz;
    const zc kap = csqrt(E);
    zc *tu = (zc *)malloc(sizeof(zc) * (size_t)n_species * nl);
    zc *td = (zc *)malloc(sizeof(zc) * (size_t)n_species * nl);
    for (int q = 0; q < n_species * nl; ++q) {
        tu[q] = -csin(dlu[q]) * cexp(I * dlu[q]) / kap;
        td[q] = -csin(dld[q]) * cexp(I * dld[q]) / kap;
    }
    zc *G = (zc *)malloc(sizeof(zc) * kk * kk);
    memset(M, 0, sizeof(zc) * N * N);
    int rc = 0;
    for (int j = 0; j < n_liz; ++j) {
        for (int i = 0; i < n_liz; ++i) {
            if (i == j) {
                for (int a = 0; a < 2 * kk; ++a) M[(2 * kk * i + a) + N * (2 * kk * j + a)] = 1.0;
                continue;
            }
            double R[3];
            for (int k = 0; k < 3; ++k) R[k] = rel[3 * i + k] - rel[3 * j + k];
            if (sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]) < 1e-8) { rc = -2; continue; }
            orc_gij(lmax, kap, R, gaunt, G);
            for (int L = 0; L < kk; ++L) {
                zc t2[4];
                const int q = spec[i] * nl + orc_lof(L);
                orc_spin_t(tu[q], td[q], mom + 3 * i, t2);
                for (int s = 0; s < 2; ++s)
                    for (int sp = 0; sp < 2; ++sp)
                        for (int Lp = 0; Lp < kk; ++Lp)
                            M[(2 * kk * i + kk * s + L) + N * (2 * kk * j + kk * sp + Lp)] =
                                -t2[2 * s + sp] * G[L + kk * Lp];
            }
        }
    }
    free(G); free(tu); free(td);
    return rc;
}

int orc_build_m_spin(int lmax, int n_liz, const double *rel, const int32_t *spec, const double *mom,
                     const double *Eri, const double *dlu, const double *dld, int n_species, const double *gaunt,
                     double *Mri)
{
    const zc E = Eri[0] + I * Eri[1];
    return orc_build_m_spin_z(lmax, n_liz, rel, spec, mom, E, (const zc *)dlu, (const zc *)dld, n_species, gaunt,
                              (zc *)Mri);
}

/* Spin-canted tau00 of one instance (2kk x 2kk column-major); LU with row
 * partial pivoting on the whole M, the first 2 kk unit columns solved and
 * refined twice with 80-bit residuals, as orc_tau00_one. */
static int orc_tau00_spin_one(int lmax, int n_liz, const double *rel, const int32_t *spec, const double *mom,
                              zc E, const zc *dlu, const zc *dld, int n_species, const double *gaunt, int refine,
                              zc *tau)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int kc = 2 * kk;
    const int nl = lmax + 1;
    const int n = kc * n_liz;
    const size_t nn = (size_t)n * n;
    int info = 0;
    for (int q = 0; q < kc * kc; ++q) tau[q] = NAN + I * NAN;
    if (!isfinite(creal(E)) || !isfinite(cimag(E)) || !orc_finite(dlu, (size_t)n_species * nl) ||
        !orc_finite(dld, (size_t)n_species * nl))
        return -1;
    zc *M = (zc *)malloc(sizeof(zc) * nn);
    zc *LU = (zc *)malloc(sizeof(zc) * nn);
    zc *X = (zc *)calloc((size_t)n * kc, sizeof(zc));
    zc *E0 = (zc *)calloc((size_t)n * kc, sizeof(zc));
    zc *R = (zc *)malloc(sizeof(zc) * (size_t)n * kc);
    int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * n);
    info = orc_build_m_spin_z(lmax, n_liz, rel, spec, mom, E, dlu, dld, n_species, gaunt, M);
    if (info == 0 && !orc_finite(M, nn)) info = -1;
    if (info == 0) {
        memcpy(LU, M, sizeof(zc) * nn);
        info = orc_lu_factor(n, (double *)LU, ipiv);
    }
    if (info == 0) {
        for (int c = 0; c < kc; ++c) E0[c + (size_t)n * c] = 1.0;
        memcpy(X, E0, sizeof(zc) * (size_t)n * kc);
        orc_lu_solve(n, (const double *)LU, ipiv, kc, (double *)X);
        for (int it = 0; it < refine; ++it) {
            orc_residual_ld(n, kc, M, X, E0, R);
            orc_lu_solve(n, (const double *)LU, ipiv, kc, (double *)R);
            for (size_t q = 0; q < (size_t)n * kc; ++q) X[q] += R[q];
        }
        const zc kap = csqrt(E);
        for (int Lp = 0; Lp < kk; ++Lp) {
            const int q = spec[0] * nl + orc_lof(Lp);
            const zc tu = -csin(dlu[q]) * cexp(I * dlu[q]) / kap;
            const zc td = -csin(dld[q]) * cexp(I * dld[q]) / kap;
            zc t2[4];
            orc_spin_t(tu, td, mom, t2);
            for (int sp = 0; sp < 2; ++sp)
                for (int a = 0; a < kc; ++a) {
                    zc v = 0.0;
                    for (int s2 = 0; s2 < 2; ++s2) v += X[a + (size_t)n * (kk * s2 + Lp)] * t2[2 * s2 + sp];
                    tau[a + (size_t)kc * (kk * sp + Lp)] = v;
                }
        }
        if (!orc_finite(tau, (size_t)kc * kc)) info = -1;
    }
    if (info != 0)
        for (int q = 0; q < kc * kc; ++q) tau[q] = NAN + I * NAN;
    free(M); free(LU); free(X); free(E0); free(R); free(ipiv);
    return info;
}

/* Batched spin-canted tau00: problem layout as orc_tau00_batch plus moment
 * [liz rows][3] (unit directions, per LIZ row like pos) and the down-spin
 * phase shifts delta_dn (same layout as delta, which holds the up spin).
 * tau00 is [n_inst][(2kk)^2] column-major per instance. */
void orc_tau00_spin_batch(int lmax, int n_inst, const int64_t *liz_off, const double *pos, const int32_t *species,
                          const double *moment, const double *energy, const int32_t *e_idx, const double *delta,
                          const double *delta_dn, int n_species, int n_energy, int refine, double *tau00,
                          int32_t *info)
{
    const int kk = (lmax + 1) * (lmax + 1);
    const int kk2 = (2 * lmax + 1) * (2 * lmax + 1);
    double *gaunt = (double *)malloc(sizeof(double) * (size_t)kk * kk * kk2);
    orc_gaunt(lmax, gaunt);
    const zc *Ez = (const zc *)energy;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_inst; ++i) {
        zc *du = orc_instance_delta(lmax, (const zc *)delta, n_species, n_energy, e_idx[i]);
        zc *dd = orc_instance_delta(lmax, (const zc *)delta_dn, n_species, n_energy, e_idx[i]);
        const int n_liz = (int)(liz_off[i + 1] - liz_off[i]);
        info[i] = orc_tau00_spin_one(lmax, n_liz, pos + 3 * liz_off[i], species + liz_off[i],
                                     moment + 3 * liz_off[i], Ez[e_idx[i]], du, dd, n_species, gaunt, refine,
                                     (zc *)tau00 + (size_t)i * 4 * kk * kk);
        free(du);
        free(dd);
    }
    free(gaunt);
}
