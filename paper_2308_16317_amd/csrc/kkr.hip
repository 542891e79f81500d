// KKR matrix assembly M = 1 - t G over each LIZ (paper Sec. 2.1: the KKR
// matrix t^{-1} - g0 built from the single-site scattering matrices t and the
// free-particle propagator g0 between two different sites; Sec. 2.2: over the
// atoms of the LIZ).  Here the equivalent form M = 1 - t G is assembled:
//   M_ii = I,   M_ij = -diag(t_{s(i), l(L)}) G^{ij}   (i != j)
// with the structure constants
//   G^{ij}_{LL'} = -4 pi i kappa sum_L'' i^{l-l'+l''} C^{L''}_{LL'} h_l''(kappa R) Y_L''(R^),
// R = R_i - R_j, kappa = sqrt(E) (principal branch), real spherical
// harmonics without the Condon-Shortley factor (L = l*l + l + m), h the
// spherical Hankel function of the first kind (upward recurrence), and
// t_l = -(1/kappa) sin(delta_l) exp(i delta_l) from the phase shifts.
//
// The real Gaunt coefficients C are built on the host from the Wigner 3j
// closed form (Racah's sum) and the unitary map between real and complex
// harmonics, and stored as a sparse list per (L, L') with the factor
// i^{l-l'+l''} (always +-1 because l+l'+l'' is even) folded in.
//
// M is stored column-major with leading dimension N = kk * n_liz: element
// (row kk*i + L, column kk*j + L') at M[(kk*j + L') * N + kk*i + L].
#include <cmath>
#include <complex>
#include <vector>

#include "lsms_common.h"

using namespace lsms;

// ------------------------------------------------------------------ host
namespace {

long double fact(int n) {
  long double r = 1.0L;
  for (int k = 2; k <= n; ++k) r *= k;
  return r;
}

// Wigner 3j symbol (j1 j2 j3; m1 m2 m3) for integer arguments, Racah formula.
long double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0) return 0.0L;
  if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0L;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0L;
  const long double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
  const long double pre = std::sqrt(tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) *
                                    fact(j3 + m3) * fact(j3 - m3));
  long double s = 0.0L;
  for (int k = 0; k <= j1 + j2 + j3; ++k) {
    const int a1 = j3 - j2 + k + m1, a2 = j3 - j1 + k - m2, a3 = j1 + j2 - j3 - k, a4 = j1 - k - m1,
              a5 = j2 - k + m2;
    if (a1 < 0 || a2 < 0 || a3 < 0 || a4 < 0 || a5 < 0) continue;
    const long double term = 1.0L / (fact(k) * fact(a1) * fact(a2) * fact(a3) * fact(a4) * fact(a5));
    s += (k & 1) ? -term : term;
  }
  const int ph = j1 - j2 - m3;
  return ((ph % 2 + 2) % 2 ? -1.0L : 1.0L) * pre * s;
}

// int Y_l1^m1 Y_l2^m2 Y_l3^m3 dOmega for complex harmonics (Condon-Shortley phase)
long double complex_gaunt(int l1, int l2, int l3, int m1, int m2, int m3) {
  const long double pi = 3.14159265358979323846264338327950288L;
  const long double w0 = wigner3j(l1, l2, l3, 0, 0, 0);
  if (w0 == 0.0L) return 0.0L;
  return std::sqrt((2.0L * l1 + 1) * (2.0L * l2 + 1) * (2.0L * l3 + 1) / (4.0L * pi)) * w0 *
         wigner3j(l1, l2, l3, m1, m2, m3);
}

// Real harmonic Y^R_{l,m} = sum over mu in {m, -m} of U(m, mu) Y_l^mu.
typedef std::complex<long double> cld;
void real_from_complex(int m, int mu[2], cld u[2], int& n) {
  const long double s2 = 1.0L / std::sqrt(2.0L);
  if (m == 0) {
    n = 1;
    mu[0] = 0;
    u[0] = 1.0L;
  } else if (m > 0) {
    n = 2;
    mu[0] = m;
    u[0] = ((m & 1) ? -s2 : s2);
    mu[1] = -m;
    u[1] = s2;
  } else {
    const int a = -m;
    n = 2;
    const cld inv_i(0.0L, -1.0L);  // 1/i
    mu[0] = a;
    u[0] = ((a & 1) ? -s2 : s2) * inv_i;
    mu[1] = -a;
    u[1] = -s2 * inv_i;
  }
}

}  // namespace

// Builds the sparse real Gaunt list for lmax: row_ptr[kk*kk+1] over pairs
// p = L + kk*L', with (L'', coef * i^{l-l'+l''}) entries.
void lsms_gaunt_host(int lmax, std::vector<int32_t>& row_ptr, std::vector<int16_t>& lpp_out,
                     std::vector<double>& coef_out) {
  const int kk = (lmax + 1) * (lmax + 1);
  const int l2 = 2 * lmax;
  const int kk2 = (l2 + 1) * (l2 + 1);
  row_ptr.assign(kk * kk + 1, 0);
  lpp_out.clear();
  coef_out.clear();
  for (int Lp = 0; Lp < kk; ++Lp) {
    const int lp = l_of(Lp), mp = Lp - lp * lp - lp;
    for (int L = 0; L < kk; ++L) {
      const int l = l_of(L), m = L - l * l - l;
      for (int Lpp = 0; Lpp < kk2; ++Lpp) {
        const int lpp = l_of(Lpp), mpp = Lpp - lpp * lpp - lpp;
        if ((l + lp + lpp) & 1) continue;
        if (lpp < std::abs(l - lp) || lpp > l + lp) continue;
        int mu1[2], mu2[2], mu3[2], n1, n2, n3;
        cld u1[2], u2[2], u3[2];
        real_from_complex(m, mu1, u1, n1);
        real_from_complex(mp, mu2, u2, n2);
        real_from_complex(mpp, mu3, u3, n3);
        cld s = 0.0L;
        for (int a = 0; a < n1; ++a)
          for (int b = 0; b < n2; ++b)
            for (int c = 0; c < n3; ++c) {
              const long double g = complex_gaunt(l, lp, lpp, mu1[a], mu2[b], mu3[c]);
              if (g != 0.0L) s += u1[a] * u2[b] * u3[c] * g;
            }
        const double v = (double)s.real();
        if (std::fabs(v) < 1e-14) continue;  // vanishes by the m selection rules
        const int e = ((l - lp + lpp) % 4 + 4) % 4;  // 0 or 2
        lpp_out.push_back((int16_t)Lpp);
        coef_out.push_back(e == 2 ? -v : v);
      }
      row_ptr[L + kk * Lp + 1] = (int32_t)lpp_out.size();
    }
  }
}

// ---------------------------------------------------------------- device
namespace {

constexpr int kBuildThreads = 256;
constexpr int kPairs = 4;            // row blocks processed per round (one per wave)
constexpr int kMaxL2 = 8;            // 2 * lmax for lmax <= 4
constexpr int kMaxKK2 = (kMaxL2 + 1) * (kMaxL2 + 1);
constexpr int kMaxSpecies = 8;
constexpr int kMaxLm = 5;

// Real spherical harmonics up to l2 for direction r (unnormalised vector),
// computed by lane m of a wave for m = 0..l2, written to Y[L''].
__device__ void ylm_column(int m, int l2, double x, double y, double z, double* Y) {
  const double rho2 = x * x + y * y;
  const double r = sqrt(rho2 + z * z);
  const double rho = sqrt(rho2);
  const double ct = z / r, st = rho / r;
  // cos(m phi) + i sin(m phi) as (x + i y)^m / rho^m
  double cm = 1.0, sm = 0.0;
  if (rho > 0.0) {
    const double cp = x / rho, sp = y / rho;
    for (int k = 0; k < m; ++k) {
      const double c2 = cm * cp - sm * sp;
      sm = sm * cp + cm * sp;
      cm = c2;
    }
  } else if (m > 0) {
    cm = 0.0;
  }
  double pmm = 1.0;
  for (int k = 1; k <= m; ++k) pmm *= (2.0 * k - 1.0) * st;
  double p_lm2 = 0.0, p_lm1 = 0.0;
  for (int l = m; l <= l2; ++l) {
    double p;
    if (l == m) p = pmm;
    else if (l == m + 1) p = ct * (2.0 * m + 1.0) * p_lm1;
    else p = ((2.0 * l - 1.0) * ct * p_lm1 - (l + m - 1.0) * p_lm2) / (double)(l - m);
    p_lm2 = p_lm1;
    p_lm1 = p;
    double ratio = 1.0;  // (l-m)!/(l+m)!
    for (int k = l - m + 1; k <= l + m; ++k) ratio /= (double)k;
    const double nlm = sqrt((2.0 * l + 1.0) * ratio * 0.07957747154594767);  // 1/(4 pi)
    if (m == 0) {
      Y[l * l + l] = nlm * p;
    } else {
      const double s = 1.4142135623730951 * nlm * p;
      Y[l * l + l + m] = s * cm;
      Y[l * l + l - m] = s * sm;
    }
  }
}

__global__ __launch_bounds__(kBuildThreads) void build_kkr_kernel(lsms_prob_dev p, lsms_gaunt_dev g, int i0,
                                                                 int n, double* __restrict__ Mbase,
                                                                 const int64_t* __restrict__ m_off, int64_t slot,
                                                                 int32_t* __restrict__ info) {
  __shared__ double Ysh[kPairs][kMaxKK2];
  __shared__ zd hsh[kPairs][kMaxL2 + 1];
  __shared__ zd tsh[kMaxSpecies][kMaxLm];
  __shared__ int bad;

  const int inst = i0 + blockIdx.y;
  const int j = blockIdx.x;
  const int64_t a = p.liz_off[inst];
  const int nliz = (int)(p.liz_off[inst + 1] - a);
  if (j >= nliz) return;
  {
    const int ee = p.e_idx[inst];
    if (nliz > p.max_liz || ee < 0 || ee >= p.n_energy) {
      if (j == 0 && threadIdx.x == 0) info[inst] = -3;
      return;
    }
  }
  const int kk = p.kk, lmax = p.lmax, l2 = 2 * lmax;
  const int64_t N = (int64_t)kk * nliz;
  zd* M = reinterpret_cast<zd*>(Mbase) + (m_off ? m_off[inst] : (int64_t)(inst - i0) * slot);
  const int e = p.e_idx[inst];
  const zd E = reinterpret_cast<const zd*>(p.energy)[e];
  const zd kap = zsqrt(E);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  if (tid < p.n_species * (lmax + 1)) {
    const int s = tid / (lmax + 1), l = tid % (lmax + 1);
    const zd d = reinterpret_cast<const zd*>(p.delta)[((int64_t)s * p.n_energy + e) * (lmax + 1) + l];
    tsh[s][l] = tmat_from_delta(d, kap);
  }
  if (tid == 0) bad = 0;
  __shared__ int bad_species;
  if (tid == 0) bad_species = 0;
  const double* rel = p.pos + 3 * a;
  const int32_t* spec = p.species + a;
  const double rjx = rel[3 * j], rjy = rel[3 * j + 1], rjz = rel[3 * j + 2];
  // -4 pi i kappa
  const zd pref = zmake(4.0 * M_PI * kap.y, -4.0 * M_PI * kap.x);
  const int kk2pairs = kk * kk;
  __syncthreads();

  for (int ib = 0; ib < nliz; ib += kPairs) {
    // phase 1: wave w prepares Y and h for row block ib + w
    const int iw = ib + wave;
    if (iw < nliz && iw != j) {
      const double Rx = rel[3 * iw] - rjx, Ry = rel[3 * iw + 1] - rjy, Rz = rel[3 * iw + 2] - rjz;
      const double R = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
      if (R < 1e-8) {
        if (lane == 0) bad = 1;
      } else {
        if (lane <= l2) ylm_column(lane, l2, Rx, Ry, Rz, Ysh[wave]);
        if (lane == 0) {
          const zd z = zmake(kap.x * R, kap.y * R);
          const zd iz = zinv(z);
          const zd eiz = zexpi(z);
          zd h0 = zmul(zmake(0.0, -1.0), zmul(eiz, iz));        // -i e^{iz}/z
          zd h1 = zmul(h0, zmake(iz.x, iz.y - 1.0));            // h0 (1/z - i)
          hsh[wave][0] = h0;
          if (l2 >= 1) hsh[wave][1] = h1;
          for (int l = 1; l < l2; ++l) {
            const zd h2 = zsub(zscale(zmul(iz, h1), 2.0 * l + 1.0), h0);
            hsh[wave][l + 1] = h2;
            h0 = h1;
            h1 = h2;
          }
        }
      }
    }
    __syncthreads();
    // phase 2: all threads write the kk x kk blocks of the prepared rows
    const int nb = min(kPairs, nliz - ib);
    for (int q = tid; q < nb * kk2pairs; q += kBuildThreads) {
      const int slotw = q / kk2pairs, pidx = q % kk2pairs;
      const int iw2 = ib + slotw;
      const int L = pidx % kk, Lp = pidx / kk;
      zd val;
      if (iw2 == j) {
        val = zmake(L == Lp ? 1.0 : 0.0, 0.0);
      } else {
        double sr = 0.0, si = 0.0;
        const int e0 = g.row_ptr[pidx], e1 = g.row_ptr[pidx + 1];
        for (int k = e0; k < e1; ++k) {
          const int Lpp = g.lpp[k];
          const double cy = g.coef[k] * Ysh[slotw][Lpp];
          const zd h = hsh[slotw][l_of(Lpp)];
          sr += cy * h.x;
          si += cy * h.y;
        }
        const zd G = zmul(pref, zmake(sr, si));
        const int sp = spec[iw2];
        const bool sp_ok = sp >= 0 && sp < p.n_species;
        if (!sp_ok) bad_species = 1;
        const zd t = tsh[sp_ok ? sp : 0][l_of(L)];
        const zd tg = zmul(t, G);
        val = zmake(-tg.x, -tg.y);
      }
      M[(int64_t)(kk * j + Lp) * N + (int64_t)kk * iw2 + L] = val;
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0 && bad_species) info[inst] = -3;
  else if (tid == 0 && bad) info[inst] = -2;
}

}  // namespace

hipError_t lsms_launch_build(const lsms_prob_dev& p, const lsms_gaunt_dev& g, int32_t i0, int32_t n, double* M,
                             const int64_t* m_off, int64_t slot, int32_t* info, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(p.max_liz, n);
  hipLaunchKernelGGL(build_kkr_kernel, grid, dim3(kBuildThreads), 0, s, p, g, i0, n, M, m_off, slot, info);
  return hipGetLastError();
}
