// Device routines of the KKR matrix assembly (M = 1 - t G over a LIZ), shared
// by the stand-alone build kernel and the fused persistent kernel.
//
//   M_ii = I,   M_ij = -diag(t_{s(i), l(L)}) G^{ij}   (i != j)
//   G^{ij}_{LL'} = -4 pi i kappa sum_L'' i^{l-l'+l''} C^{L''}_{LL'} h_l''(kappa R) Y_L''(R^),
// R = R_i - R_j, kappa = sqrt(E) (principal branch), real spherical
// harmonics without the Condon-Shortley factor, h the spherical Hankel
// function of the first kind, t_l = -(1/kappa) sin(delta_l) exp(i delta_l)
// (paper Sec. 2.1: t and the propagator g0 between two different sites;
// Sec. 2.2: over the LIZ).  M is column-major, ld N = kk * n_liz.
#pragma once

#include "lsms_common.h"

namespace lsms {

constexpr int kBuildChunk = 64;  // LIZ row blocks prepared per phase (one per lane)
constexpr int kBMaxL2 = 8;       // 2 * lmax for lmax <= 4
constexpr int kBMaxKK2 = (kBMaxL2 + 1) * (kBMaxL2 + 1);
constexpr int kBMaxKK = 25;
constexpr int kBMaxNnz = 2304;   // >= nonzeros of the lmax = 4 Gaunt table (2229)
constexpr int kBMaxSpecies = 8;
constexpr int kBMaxLm = 5;

struct BuildSmem {
  zd F[kBuildChunk][kBMaxKK2];     // h_l''(kappa R) Y_L''(R^) of each row block of the chunk
  zd h[kBuildChunk][kBMaxL2 + 1];
  double nlm[kBMaxL2 + 1][kBMaxL2 + 1];  // sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
  double rcp[kBMaxL2 + 2];               // 1/k
  zd t[kBMaxSpecies][kBMaxLm];
  zd tdn[kBMaxSpecies][kBMaxLm];  // spin canting: the spin antiparallel to the moment
  double mom[kBuildChunk][3];      // spin canting: moment of each row block of the chunk
  double coef[kBMaxNnz];
  int32_t rp[kBMaxKK * kBMaxKK + 1];
  int16_t lpp[kBMaxNnz];
  int spec[kBuildChunk];
  int bad, bad_species;
};

// F_L'' = h_l'' Y_L''(r) for the l'' = m .. l2 of one order m >= 0 (both
// signs of m), of a nonzero vector r, given the Hankel values h_l'':
// cos(m phi) + i sin(m phi) as ((x + i y)/rho)^m, P_m^m = (2m-1)!!
// sin^m(theta) and upward recurrence in l; normalisation constants and
// reciprocals from LDS (no divisions in the recurrence).
__device__ inline void ylm_order(int l2, int m, double x, double y, double z, const BuildSmem& sb,
                                 const zd* __restrict__ h, zd* __restrict__ F) {
  const double rho2 = x * x + y * y;
  const double r = sqrt(rho2 + z * z);
  const double rho = sqrt(rho2);
  const double ir = 1.0 / r;
  const double ct = z * ir, st = rho * ir;
  const double irho = rho > 0.0 ? 1.0 / rho : 0.0;
  const double cp = rho > 0.0 ? x * irho : 1.0, sp = rho > 0.0 ? y * irho : 0.0;
  double cm = 1.0, sm = 0.0, pmm = 1.0;
  for (int k = 1; k <= m; ++k) {
    const double c2 = cm * cp - sm * sp;
    sm = sm * cp + cm * sp;
    cm = c2;
    pmm *= (2.0 * k - 1.0) * st;
  }
  double p_lm2 = 0.0, p_lm1 = 0.0;
  for (int l = m; l <= l2; ++l) {
    double pl;
    if (l == m) pl = pmm;
    else if (l == m + 1) pl = ct * (2.0 * m + 1.0) * p_lm1;
    else pl = ((2.0 * l - 1.0) * ct * p_lm1 - (l + m - 1.0) * p_lm2) * sb.rcp[l - m];
    p_lm2 = p_lm1;
    p_lm1 = pl;
    const double nlm = sb.nlm[l][m];
    const zd hl = h[l];
    if (m == 0) {
      F[l * l + l] = zscale(hl, nlm * pl);
    } else {
      const double sc = 1.4142135623730951 * nlm * pl;
      F[l * l + l + m] = zscale(hl, sc * cm);
      F[l * l + l - m] = zscale(hl, sc * sm);
    }
  }
}

// Spherical Hankel functions h_l(z), l <= l2, by upward recurrence from
// h_0 = -i e^{iz}/z and h_1 = h_0 (1/z - i).
__device__ inline void hankel_all(int l2, zd z, zd* __restrict__ h) {
  const zd iz = zinv(z);
  const zd eiz = zexpi(z);
  zd h0 = zmul(zmake(0.0, -1.0), zmul(eiz, iz));
  zd h1 = zmul(h0, zmake(iz.x, iz.y - 1.0));
  h[0] = h0;
  if (l2 >= 1) h[1] = h1;
  for (int l = 1; l < l2; ++l) {
    const zd h2 = zsub(zscale(zmul(iz, h1), 2.0 * l + 1.0), h0);
    h[l + 1] = h2;
    h0 = h1;
    h1 = h2;
  }
}

// Stage the Gaunt list and the instance's t-matrices in LDS.  Ends with a
// barrier.
template <int kNT>
__device__ void build_setup(const lsms_prob_dev& p, const lsms_gaunt_dev& g, int inst, BuildSmem& sb) {
  const int tid = threadIdx.x;
  const int lmax = p.lmax, kkp = p.kk * p.kk;
  const int e = p.e_idx[inst];
  const zd kap = zsqrt(reinterpret_cast<const zd*>(p.energy)[e]);
  if (tid < p.n_species * (lmax + 1)) {
    const int s = tid / (lmax + 1), l = tid % (lmax + 1);
    const zd d = reinterpret_cast<const zd*>(p.delta)[((int64_t)s * p.n_energy + e) * (lmax + 1) + l];
    sb.t[s][l] = tmat_from_delta(d, kap);
    if (p.nspin == 2) {
      const zd dd = reinterpret_cast<const zd*>(p.delta_dn)[((int64_t)s * p.n_energy + e) * (lmax + 1) + l];
      sb.tdn[s][l] = tmat_from_delta(dd, kap);
    }
  }
  for (int q = tid; q <= kkp; q += kNT) sb.rp[q] = g.row_ptr[q];
  for (int q = tid; q < g.nnz; q += kNT) {
    const int lpp = g.lpp[q];
    sb.lpp[q] = (int16_t)lpp;
    sb.coef[q] = g.coef[q];
  }
  if (tid <= kBMaxL2 + 1) sb.rcp[tid] = tid > 0 ? 1.0 / (double)tid : 0.0;
  if (tid < (kBMaxL2 + 1) * (kBMaxL2 + 1)) {
    const int l = tid / (kBMaxL2 + 1), m = tid % (kBMaxL2 + 1);
    double ratio = 1.0;  // (l-m)!/(l+m)!
    for (int k = l - m + 1; k <= l + m; ++k) ratio /= (double)k;
    sb.nlm[l][m] = m <= l ? sqrt((2.0 * l + 1.0) * ratio * 0.07957747154594767) : 0.0;  // 1/(4 pi)
  }
  if (tid == 0) {
    sb.bad = 0;
    sb.bad_species = 0;
  }
  __syncthreads();
}

// Spin canting: the 2 kk columns of site j.  Entry (s, L; s', L') of row
// block i is -t_i(L)_{s s'} G^{ij}_{LL'} (t_i the global-frame t of site i,
// spin_t), at row kc i + kk s + L and column kc j + kk s' + L'; the diagonal
// block is the identity.  Sums as build_column_body; a thread takes one L
// and two row blocks.
template <int kNT>
__device__ __forceinline__ void build_spin_phase_b(const lsms_prob_dev& p, int j, int ib, int nb, int64_t N,
                                                   zd pref, zd* __restrict__ M, const BuildSmem& sb) {
  const int tid = threadIdx.x;
  const int kk = p.kk, kc = p.kc;
  const int npair = (nb + 1) >> 1;
  for (int t = tid; t < npair * kk; t += kNT) {
    const int ip = t / kk;
    const int L = t - ip * kk;
    const int i0 = 2 * ip, i1 = min(2 * ip + 1, nb - 1);
    const bool two = 2 * ip + 1 < nb;
    const int iw0 = ib + i0, iw1 = ib + i1;
    const int l = l_of(L);
    zd ta[4], tb[4];
    spin_t(sb.t[sb.spec[i0]][l], sb.tdn[sb.spec[i0]][l], sb.mom[i0][0], sb.mom[i0][1], sb.mom[i0][2], ta);
    spin_t(sb.t[sb.spec[i1]][l], sb.tdn[sb.spec[i1]][l], sb.mom[i1][0], sb.mom[i1][1], sb.mom[i1][2], tb);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ta[q] = zmul(ta[q], pref);
      tb[q] = zmul(tb[q], pref);
    }
    const int64_t r0 = (int64_t)kc * iw0 + L, r1 = (int64_t)kc * iw1 + L;
    for (int Lp = 0; Lp < kk; ++Lp) {
      double sr0 = 0.0, si0 = 0.0, sr1 = 0.0, si1 = 0.0;
      const int pidx = L + kk * Lp;
      const int e0 = sb.rp[pidx], e1 = sb.rp[pidx + 1];
      for (int k = e0; k < e1; ++k) {
        const double c = sb.coef[k];
        const int lp = sb.lpp[k];
        const zd f0 = sb.F[i0][lp], f1 = sb.F[i1][lp];
        sr0 += c * f0.x;
        si0 += c * f0.y;
        sr1 += c * f1.x;
        si1 += c * f1.y;
      }
      const zd g0 = zmake(sr0, si0), g1 = zmake(sr1, si1);
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
          const int64_t col = (int64_t)kc * j + kk * sp + Lp;
          const zd one = zmake((s == sp && L == Lp) ? 1.0 : 0.0, 0.0);
          const zd v0 = iw0 == j ? one : zmul(zmake(-ta[2 * s + sp].x, -ta[2 * s + sp].y), g0);
          M[col * N + r0 + kk * s] = v0;
          if (two) {
            const zd v1 = iw1 == j ? one : zmul(zmake(-tb[2 * s + sp].x, -tb[2 * s + sp].y), g1);
            M[col * N + r1 + kk * s] = v1;
          }
        }
    }
  }
}

// Block column j of M, in chunks of kBuildChunk LIZ row blocks.  Phase A:
// for each row block i of the chunk the Hankel functions h_l''(kappa R_ij),
// then 2 lmax + 1 tasks, one per order m = 0 .. 2 lmax, forming
// F_L'' = h_l'' Y_L''(R_ij) of that order; task (m, i) is thread 64 m + i,
// so that a wave runs one order.  Phase B: each thread owns one L and two
// row blocks (which share the Gaunt lists) and sweeps the kk columns L'
// (sum over the list of (L, L') of coefficient x F), entry (L, L') of row
// block i at index L + kk (i + nb L'), so consecutive threads write
// consecutive rows.
template <int kNT>
__device__ __forceinline__ void build_column_body(const lsms_prob_dev& p, int inst, int j, zd* __restrict__ M,
                                                  BuildSmem& sb, zf* __restrict__ M32 = nullptr) {
  const int tid = threadIdx.x;
  const int64_t a = p.liz_off[inst];
  const int nliz = (int)(p.liz_off[inst + 1] - a);
  const int kk = p.kk, l2 = 2 * p.lmax;
  const int64_t N = (int64_t)p.kc * nliz;
  const zd kap = zsqrt(reinterpret_cast<const zd*>(p.energy)[p.e_idx[inst]]);
  const double* rel = p.pos + 3 * a;
  const int32_t* spec = p.species + a;
  const double rjx = rel[3 * j], rjy = rel[3 * j + 1], rjz = rel[3 * j + 2];
  const zd pref = zmake(4.0 * M_PI * kap.y, -4.0 * M_PI * kap.x);  // -4 pi i kappa
  for (int ib = 0; ib < nliz; ib += kBuildChunk) {
    const int nb = min(kBuildChunk, nliz - ib);
    // phase A1: per row block its species (and moment) and the Hankel
    // functions; A2: per (order m, row block) the F_L'' of that order
    for (int il = tid; il < kBuildChunk; il += kNT) {
      const int iw = ib + il;
      if (il >= nb) continue;
      const int sp = spec[iw];
      if (sp < 0 || sp >= p.n_species) sb.bad_species = 1;
      sb.spec[il] = (sp >= 0 && sp < p.n_species) ? sp : 0;
      if (p.nspin == 2) {
        const double* e = p.moment + 3 * (a + iw);
        sb.mom[il][0] = e[0];
        sb.mom[il][1] = e[1];
        sb.mom[il][2] = e[2];
      }
      if (iw != j) {
        const double Rx = rel[3 * iw] - rjx, Ry = rel[3 * iw + 1] - rjy, Rz = rel[3 * iw + 2] - rjz;
        const double R2 = Rx * Rx + Ry * Ry + Rz * Rz;
        if (R2 < 1e-16) {
          sb.bad = 1;
        } else {
          const double R = sqrt(R2);
          hankel_all(l2, zmake(kap.x * R, kap.y * R), sb.h[il]);
        }
      }
    }
    __syncthreads();
    for (int t = tid; t < (l2 + 1) * kBuildChunk; t += kNT) {
      const int m = t >> 6, il = t & 63;  // one order per wave
      const int iw = ib + il;
      if (il >= nb || iw == j) continue;
      const double Rx = rel[3 * iw] - rjx, Ry = rel[3 * iw + 1] - rjy, Rz = rel[3 * iw + 2] - rjz;
      if (Rx * Rx + Ry * Ry + Rz * Rz >= 1e-16) ylm_order(l2, m, Rx, Ry, Rz, sb, sb.h[il], sb.F[il]);
    }
    __syncthreads();
    if (p.nspin == 2) {
      build_spin_phase_b<kNT>(p, j, ib, nb, N, pref, M, sb);
      __syncthreads();
      continue;
    }
    // a thread takes one L and two row blocks 2 ip, 2 ip + 1 of the chunk,
    // which share the Gaunt list of every (L, L')
    const int npair = (nb + 1) >> 1;
    for (int t = tid; t < npair * kk; t += kNT) {
      const int ip = t / kk;
      const int L = t - ip * kk;
      const int i0 = 2 * ip, i1 = min(2 * ip + 1, nb - 1);
      const bool two = 2 * ip + 1 < nb;
      const int iw0 = ib + i0, iw1 = ib + i1;
      const int64_t o0 = (int64_t)(kk * j) * N + (int64_t)kk * iw0 + L;
      const int64_t o1 = (int64_t)(kk * j) * N + (int64_t)kk * iw1 + L;
      const zd tp0 = zmul(sb.t[sb.spec[i0]][l_of(L)], pref);
      const zd tp1 = zmul(sb.t[sb.spec[i1]][l_of(L)], pref);
      for (int Lp = 0; Lp < kk; ++Lp) {
        double sr0 = 0.0, si0 = 0.0, sr1 = 0.0, si1 = 0.0;
        const int pidx = L + kk * Lp;
        const int e0 = sb.rp[pidx], e1 = sb.rp[pidx + 1];
        for (int k = e0; k < e1; ++k) {
          const double c = sb.coef[k];
          const int lp = sb.lpp[k];
          const zd f0 = sb.F[i0][lp], f1 = sb.F[i1][lp];
          sr0 += c * f0.x;
          si0 += c * f0.y;
          sr1 += c * f1.x;
          si1 += c * f1.y;
        }
        zd v0, v1;
        if (iw0 == j) {
          v0 = zmake(L == Lp ? 1.0 : 0.0, 0.0);
        } else {
          const zd tg = zmul(tp0, zmake(sr0, si0));
          v0 = zmake(-tg.x, -tg.y);
        }
        if (iw1 == j) {
          v1 = zmake(L == Lp ? 1.0 : 0.0, 0.0);
        } else {
          const zd tg = zmul(tp1, zmake(sr1, si1));
          v1 = zmake(-tg.x, -tg.y);
        }
        M[o0 + (int64_t)Lp * N] = v0;
        if (M32) M32[o0 + (int64_t)Lp * N] = zmake((float)v0.x, (float)v0.y);
        if (two) {
          M[o1 + (int64_t)Lp * N] = v1;
          if (M32) M32[o1 + (int64_t)Lp * N] = zmake((float)v1.x, (float)v1.y);
        }
      }
    }
    __syncthreads();
  }
}

// Out-of-line form for kernels that also eliminate (separate register
// allocation for the build and the factorisation); M32, if given, receives an
// FP32 copy of the column at the same positions.
template <int kNT>
__device__ __noinline__ void build_column(const lsms_prob_dev& p, int inst, int j, zd* __restrict__ M,
                                          BuildSmem& sb, zf* __restrict__ M32 = nullptr) {
  build_column_body<kNT>(p, inst, j, M, sb, M32);
}

}  // namespace lsms
