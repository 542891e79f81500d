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

#include "kkr_device.h"
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

// One workgroup per (block column j, instance).
__global__ __launch_bounds__(kBuildThreads) void build_kkr_kernel(lsms_prob_dev p, lsms_gaunt_dev g, int i0,
                                                                 int n, double* __restrict__ Mbase,
                                                                 const int64_t* __restrict__ m_off, int64_t slot,
                                                                 int32_t* __restrict__ info) {
  __shared__ BuildSmem sb;
  const int inst = i0 + blockIdx.y;
  const int j = blockIdx.x;
  const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
  if (j >= nliz) return;
  const int ee = p.e_idx[inst];
  if (nliz > p.max_liz || ee < 0 || ee >= p.n_energy) {
    if (j == 0 && threadIdx.x == 0) info[inst] = -3;
    return;
  }
  zd* M = reinterpret_cast<zd*>(Mbase) + (m_off ? m_off[inst] : (int64_t)(inst - i0) * slot);
  build_setup<kBuildThreads>(p, g, inst, sb);
  build_column_body<kBuildThreads>(p, inst, j, M, sb);
  if (threadIdx.x == 0 && sb.bad_species) info[inst] = -3;
  else if (threadIdx.x == 0 && sb.bad) info[inst] = -2;
}

}  // namespace

hipError_t lsms_launch_build(const lsms_prob_dev& p, const lsms_gaunt_dev& g, int32_t i0, int32_t n, double* M,
                             const int64_t* m_off, int64_t slot, int32_t* info, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(p.max_liz, n);
  hipLaunchKernelGGL(build_kkr_kernel, grid, dim3(kBuildThreads), 0, s, p, g, i0, n, M, m_off, slot, info);
  return hipGetLastError();
}
