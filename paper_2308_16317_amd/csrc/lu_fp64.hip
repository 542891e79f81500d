// FP64 block LU / Schur-complement elimination and tau00 (paper Sec. 2.2:
// only the first block of the inverse of the KKR matrix is needed, obtained
// by block LU; Sec. 3.2: the paper's GPU path factorises with row partial
// pivoting and solves).
//
// For each instance, tau00 = [M^{-1}]_{00} diag(t_0).  With D the KKR matrix
// restricted to the non-central sites, [M^{-1}]_{00} = S^{-1},
// S = M_00 - M_0r D^{-1} M_r0.  The kernel reads the column-major M buffer as
// the row-major storage of A = M^T, eliminates every non-central column of A
// by right-looking blocked LU with row partial pivoting restricted to the
// non-central rows (i.e. column pivoting of M), and is left with
// S_A = S^T in the central block.  Then [M^{-1}]_{00} = (S_A^{-1})^T.  The
// block is unique whenever M and D are invertible, so the pivot order only
// changes rounding.  Reading M transposed makes every row swap a contiguous
// move and every operand load of the trailing update row-contiguous.
//
// Internal index v runs over the non-central rows first and the central
// block last: physical row/column phys(v) = v + kk for v < Nd = N - kk, and
// v - Nd for the central block.
//
// One workgroup (8 waves, two per SIMD) per instance.  Per panel of w <= 128
// columns (two 64-column diagonal blocks when w > 64):
//   1. recursive panel factorisation: leaves of kWL columns are factorised
//      with the leaf held in registers (each thread owns rows lc + t + 512 q),
//      pivot search by DPP within each wave and an 8-entry LDS reduction
//      across the waves; after each leaf the completed block of the
//      recursion updates its sibling block (triangular solve and product on
//      MFMA);
//   2. the panel's row interchanges applied to the trailing columns;
//   3. the inverses of the unit lower diagonal blocks of L11 (LDS, global);
//   4. per strip of trailing columns (64 in FP64, 128 in FP32): U12 = L11^-1
//      A12 (MFMA) into LDS, then A22 -= L21 U12 (complex GEMM on MFMA; a
//      complex product is three real MFMAs in FP64, the three-multiplication
//      form, and four on real/imaginary accumulators in FP32).
// Finally S_A is inverted by Gauss-Jordan with partial pivoting.
#include "kkr_device.h"
#include "lsms_common.h"
#include "lu_device.h"

using namespace lsms;

namespace {

constexpr int kThreads = kLuThreads;
typedef LuSmem<double> LuSmemD;

// ----------------------------------------------------------------------
// Optional outputs of the FP64 path: the central block row of tau and
// ln det M.
//
// With the pivots confined to the non-central rows, the elimination gives
// P A_int = L U with the central rows never interchanged, so that
// Y = A_int^{-1} E_c (E_c the unit vectors of the central rows) solves
// U Y = E_c: the central rows are Y_c = S_A^{-1} and the others
// Y_r = -U_rr^{-1} U_rc S_A^{-1}, one backward solve with U (L and the
// interchanges act only on the zero non-central rows of E_c).  As A = M^T,
// Y^T is the central block row of M^{-1}, and the block row of tau through
// the central site is tau^{0j}(L, L') = Y[kk j + L'][L] t_{s(j), l(L')}
// (paper Sec. 2.1: the blocks of the Dyson-equation inverse, which enter the
// Green's function of eq. Green_KKR).
//
// ln det M = ln det A = sum over the elimination pivots of ln U_vv, plus the
// logarithms of the Gauss-Jordan pivots of S_A, plus i pi per row
// interchange; the imaginary part is reduced to (-pi, pi] (the principal
// logarithm).  ln det M is the multiple-scattering term of Lloyd's formula
// for the integrated density of states, the energy integral of eq. Density.
// ----------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;

// The Gauss-Jordan workspace [S_A | 1] (kc x 2 kc, row stride 2 kMaxKC) at
// the start of sh.X, whose 128 KB with sh.U hold it for kc up to 50.
typedef zd GjRow[2 * kMaxKC];
static_assert(sizeof(GjRow) * kMaxKC <= sizeof(LuSmemD::X) + sizeof(LuSmemD::U), "Gauss-Jordan workspace");
__device__ __forceinline__ GjRow* gj_view(LuSmemD& sh) { return reinterpret_cast<GjRow*>(&sh.X[0][0]); }

struct RowOut {
  zd* z;          // N x kp workspace, internal rows (needed for row)
  int32_t* ipiv;  // N workspace (needed for logdet)
  zd* row;        // block row of tau, kk x N column-major (ld kk), or null
  zd* logdet;     // ln det M (one complex), or null
  int kp;         // 16 (kk <= 16) or 32
};

// Sums of a, b and c over the workgroup, returned to every thread in a fixed
// order (the same result on every run).
__device__ __forceinline__ void block_sum(double& a, double& b, int& c, LuSmemD& sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
    c += __shfl_xor(c, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh.red[0][wave] = a;
    sh.red[1][wave] = b;
    sh.redi[wave] = c;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  c = 0;
#pragma unroll
  for (int q = 0; q < kLuWaves; ++q) {
    a += sh.red[0][q];
    b += sh.red[1][q];
    c += sh.redi[q];
  }
  __syncthreads();
}

// Y_r := -U_rr^{-1} (U_rc Y_c) for the non-central rows, with Y_c already in
// the central rows of z (N x kp, internal rows, columns >= kk zero), by
// 64-row blocks from the bottom: part = U(c .. c+w, c+w .. N) z(c+w .. N) on
// MFMA (four 16-row tiles per 16 columns, the reduction split between wave
// groups when kp = 16), then z(c .. c+w) = -X part with X the inverse of the
// diagonal block of U.
__device__ __noinline__ void back_solve_rows(const Mat<zd>& Ain, zd* zin, int kp, LuSmemD& sh) {
  const Mat<zd> A = Ain;  // by value: fields stay in registers
  typedef Prec<double>::V4 V4;
  LSMS_GLOBAL zd* z = glb(zin);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int N = (int)A.N, Nd = A.Nd, nct = kp / 16;
  const int nblk = (Nd + kNB - 1) / kNB;
  for (int pi = nblk - 1; pi >= 0; --pi) {
    const int c = pi * kNB, w = min(kNB, Nd - c);
    invert_upper<double>(A, c, w, sh);  // sh.X; ends with a barrier
    const int ntile = 4 * nct, nsplit = kLuWaves / ntile;
    const int tile = wave % ntile, split = wave / ntile;
    const int rt = tile & 3, ct = tile >> 2;
    const int k0 = c + w, klen = N - k0;
    const int kchunk = ((klen + nsplit - 1) / nsplit + 15) & ~15;
    const int ka = k0 + split * kchunk, kz = min(N, ka + kchunk);
    V4 ar = V4{0.0, 0.0, 0.0, 0.0}, ai = V4{0.0, 0.0, 0.0, 0.0};
    const int row = c + 16 * rt + li;
    const bool rok = 16 * rt + li < w;
    const LSMS_GLOBAL zd* urow = A.base + A.phys(rok ? row : c) * A.N;
    // chunks of 16 (lane (li, lq) takes k = kb + 4 lq + j at step j), loaded
    // one chunk ahead from clamped in-range addresses; entries past the
    // range are zeroed before they enter the product
    zd an[4], yn[4];
    auto ld = [&](int kb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = min(kb + 4 * lq + j, N - 1);
        an[j] = urow[A.phys(k)];
        yn[j] = z[(int64_t)k * kp + 16 * ct + li];
      }
    };
    if (ka < kz) ld(ka);
    for (int kb = ka; kb < kz; kb += 16) {
      zd a[4], y[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a[j] = an[j];
        y[j] = yn[j];
      }
      if (kb + 16 < kz) ld(kb + 16);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = rok && kb + 4 * lq + j < kz;
        const double axr = ok ? a[j].x : 0.0, axi = ok ? a[j].y : 0.0;
        ar = Prec<double>::mfma(axr, y[j].x, ar);
        ar = Prec<double>::mfma(-axi, y[j].y, ar);
        ai = Prec<double>::mfma(axr, y[j].y, ai);
        ai = Prec<double>::mfma(axi, y[j].x, ai);
      }
    }
    // partial sums of split q in columns [32 q, 32 q + kp) of sh.U
#pragma unroll
    for (int r = 0; r < 4; ++r)
      sh.U[16 * rt + Prec<double>::drow(r, lq)][32 * split + 16 * ct + li] = zmake(ar[r], ai[r]);
    __syncthreads();
    for (int q = tid; q < kNB * kp; q += kThreads) {
      const int i = q / kp, j = q % kp;
      zd v = zmake(0.0, 0.0);
      if (i < w) {
        const zd p0 = sh.U[i][j];
        const zd p1 = nsplit > 1 ? sh.U[i][32 + j] : zmake(0.0, 0.0);
        v = zmake(-(p0.x + p1.x), -(p0.y + p1.y));
      }
      sh.U[i][j] = v;
    }
    __syncthreads();
    // z(c .. c+w) = X * sh.U (rows >= w of sh.U and columns >= w of X are zero)
    const int rt2 = wave & 3, ct2 = wave >> 2;
    if (ct2 < nct) {
      V4 br = V4{0.0, 0.0, 0.0, 0.0}, bi = V4{0.0, 0.0, 0.0, 0.0};
      for (int kb = 0; kb < w; kb += 4) {
        const int k = kb + lq;
        const zd x = sh.X[16 * rt2 + li][k];
        const zd y = sh.U[k][16 * ct2 + li];
        br = Prec<double>::mfma(x.x, y.x, br);
        br = Prec<double>::mfma(-x.y, y.y, br);
        bi = Prec<double>::mfma(x.x, y.y, bi);
        bi = Prec<double>::mfma(x.y, y.x, bi);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * rt2 + Prec<double>::drow(r, lq);
        if (i < w) z[(int64_t)(c + i) * kp + 16 * ct2 + li] = zmake(br[r], bi[r]);
      }
    }
    __syncthreads();
  }
}

// The block row of tau of one instance from S_A^{-1} (Gauss-Jordan result in
// the right half of G) and the factored A; NaN when info0 != 0.  Sets sh.bad
// on a non-finite entry.  Ends after a barrier.
__device__ __noinline__ void row_output(const lsms_prob_dev& p, int inst, const Mat<zd>& Ain, const RowOut& ro,
                                        int info0, LuSmemD& sh) {
  const Mat<zd> A = Ain;
  const int tid = threadIdx.x, kk = A.kk, N = (int)A.N, Nd = A.Nd, kp = ro.kp;
  LSMS_GLOBAL zd* z = glb(ro.z);
  LSMS_GLOBAL zd* out = glb(ro.row);
  if (info0 != 0) {
    for (int q = tid; q < kk * N; q += kThreads) out[q] = zmake((double)NAN, (double)NAN);
    __syncthreads();
    return;
  }
  const GjRow* G = gj_view(sh);
  for (int q = tid; q < kk * kp; q += kThreads) {
    const int r = q / kp, L = q % kp;
    z[(int64_t)(Nd + r) * kp + L] = L < kk ? G[r][kk + L] : zmake(0.0, 0.0);
  }
  __syncthreads();
  if (Nd > 0) back_solve_rows(A, ro.z, kp, sh);
  // t of every (species, l) at this energy, in sh.X
  zd* tt = &sh.X[0][0];
  const int e = p.e_idx[inst], nl = p.lmax + 1;
  const zd kap = zsqrt(reinterpret_cast<const zd*>(p.energy)[e]);
  const zd* dz = reinterpret_cast<const zd*>(p.delta);
  for (int q = tid; q < p.n_species * nl; q += kThreads)
    tt[q] = tmat_from_delta(dz[((int64_t)(q / nl) * p.n_energy + e) * nl + q % nl], kap);
  __syncthreads();
  const int32_t* spec = p.species + p.liz_off[inst];
  bool bad = false;
  for (int q = tid; q < kk * N; q += kThreads) {
    const int col = q / kk, L = q - col * kk;  // col = kk j + L' (physical)
    const int j = col / kk, Lp = col - j * kk;
    const int v = col >= kk ? col - kk : Nd + col;  // internal row of Y
    const int sj = min(max(spec[j], 0), p.n_species - 1);
    const zd val = zmul(z[(int64_t)v * kp + L], tt[sj * nl + l_of(Lp)]);
    bad |= !zfinite(val);
    out[q] = val;
  }
  if (bad) sh.bad = 1;
  __syncthreads();
}

// The end of one instance after its elimination (sh.info holds the first
// zero-pivot step or 0): Gauss-Jordan inverse of the Schur block S_A,
// tau00, and with ro the block row and ln det M (ld_*: the sums over the U
// diagonal).  All threads call it; it ends after a barrier.
__device__ __noinline__ void finish_instance(const lsms_prob_dev& p, int inst, const Mat<zd>& A, const RowOut& ro,
                                             double ld_re, double ld_im, int ld_sw, double* __restrict__ tau00,
                                             int32_t* __restrict__ info, LuSmemD& sh) {
  const int tid = threadIdx.x;
  const int kk = p.kk, kc = p.kc;
  const int N = (int)A.N, Nd = A.Nd;
  zd* tout = reinterpret_cast<zd*>(tau00) + (int64_t)inst * kc * kc;
  const bool want_row = ro.row != nullptr, want_ld = ro.logdet != nullptr;
  // Gauss-Jordan inverse of S_A (kc x kc, physical rows/cols 0..kc-1)
  GjRow* G = gj_view(sh);
  for (int q = tid; q < kc * 2 * kc; q += kThreads) {
    const int r = q / (2 * kc), col = q % (2 * kc);
    G[r][col] = col < kc ? A.base[(int64_t)r * N + col] : zmake(col - kc == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < kc; ++k) {
    if (tid == 0) {
      int pr = k;
      double best = zcabs1(G[k][k]);
      for (int r = k + 1; r < kc; ++r) {
        const double v = zcabs1(G[r][k]);
        if (v > best) {
          best = v;
          pr = r;
        }
      }
      if (best == 0.0 && sh.info == 0) sh.info = Nd + k + 1;
      sh.gj_piv = pr;
    }
    __syncthreads();
    const int pr = sh.gj_piv;
    if (pr != k && tid < 2 * kc) {
      const zd t = G[k][tid];
      G[k][tid] = G[pr][tid];
      G[pr][tid] = t;
    }
    __syncthreads();
    if (tid == 0) {
      const zd g = G[k][k];
      sh.pinv = zinv(g);
      if (want_ld) {
        ld_re += log(hypot(g.x, g.y));
        ld_im += atan2(g.y, g.x);
        ld_sw += pr != k;
      }
    }
    __syncthreads();
    if (tid < 2 * kc) G[k][tid] = zmul(G[k][tid], sh.pinv);
    if (tid < kc) sh.tz[tid] = G[tid][k];  // elimination factors (row k unused)
    __syncthreads();
    for (int q = tid; q < kc * 2 * kc; q += kThreads) {
      const int r = q / (2 * kc), col = q % (2 * kc);
      if (r != k) G[r][col] = zfms(G[r][col], sh.tz[r], G[k][col]);
    }
    __syncthreads();
  }
  // [M^{-1}]_{00}(a, b) = S_A^{-1}(b, a) = G[b][kc + a].  tau00 = [M^{-1}]_{00} t0:
  // without spin tau00(L, L') = G[L'][kk + L] t0_{l(L')}; with spin (a = kk s + L,
  // b' = kk s' + L') tau00(a, b') = sum_s'' G[kk s'' + L'][kc + a] t0(L')_{s'' s'}.
  const int e = p.e_idx[inst];
  const zd kap = zsqrt(reinterpret_cast<const zd*>(p.energy)[e]);
  const int64_t r0 = p.liz_off[inst];
  const int s0 = min(max(p.species[r0], 0), p.n_species - 1);
  const int64_t doff = ((int64_t)s0 * p.n_energy + e) * (p.lmax + 1);
  const zd* dl = reinterpret_cast<const zd*>(p.delta) + doff;
  const int info0 = sh.info;
  for (int q = tid; q < kc * kc; q += kThreads) {
    const int a = q % kc, bp = q / kc;
    zd v;
    if (p.nspin == 2) {
      const int sp = bp / kk, Lp = bp - sp * kk;
      const zd* dd = reinterpret_cast<const zd*>(p.delta_dn) + doff;
      const double* m0 = p.moment + 3 * r0;
      zd t2[4];
      spin_t(tmat_from_delta(dl[l_of(Lp)], kap), tmat_from_delta(dd[l_of(Lp)], kap), m0[0], m0[1], m0[2], t2);
      v = zadd(zmul(G[Lp][kc + a], t2[sp]), zmul(G[kk + Lp][kc + a], t2[2 + sp]));
    } else {
      v = zmul(G[bp][kk + a], tmat_from_delta(dl[l_of(bp)], kap));
    }
    if (info0 != 0) v = zmake((double)NAN, (double)NAN);
    if (!zfinite(v)) sh.bad = 1;
    tout[q] = v;
  }
  __syncthreads();
  if (want_row) row_output(p, inst, A, ro, info0, sh);
  if (want_ld && tid == 0) {
    // every thread holds the sums over the U diagonal; thread 0 also those
    // of the Gauss-Jordan pivots
    double im = ld_im + ((ld_sw & 1) ? kPi : 0.0);
    im = remainder(im, 2.0 * kPi);
    if (im <= -kPi) im += 2.0 * kPi;
    zd v = zmake(ld_re, im);
    if (info0 != 0) v = zmake((double)NAN, (double)NAN);
    else if (!zfinite(v)) sh.bad = 1;
    *ro.logdet = v;
  }
  __syncthreads();
  if (tid == 0) info[inst] = info0 != 0 ? info0 : (sh.bad ? -1 : 0);
  __syncthreads();
}

// Eliminates one instance whose matrix is at `base` and writes its tau00 and
// info (and, with ro, its block row of tau and ln det M).  All threads of the
// workgroup call it; it ends after a barrier.
template <int kR, int kWL>
__device__ void lu_instance(const lsms_prob_dev& p, int inst, zd* base, zd* xg, double* __restrict__ tau00,
                            int32_t* __restrict__ info, int nb, LuSmemD& sh, const RowOut ro = RowOut{}) {
  const int tid = threadIdx.x;
  const int kc = p.kc;  // kk, or 2 kk with spin canting
  const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
  const int N = kc * nliz, Nd = N - kc;
  Mat<zd> A;
  A.base = glb(base);
  A.N = N;
  A.Nd = Nd;
  A.kk = kc;
  if (tid == 0) {
    sh.info = 0;
    sh.bad = 0;
  }
  __syncthreads();
  const bool want_ld = ro.logdet != nullptr;
  eliminate<double, kR, kWL>(A, 0, Nd, Nd, nb, ro.row != nullptr, want_ld ? ro.ipiv : nullptr, xg, sh);
  double ld_re = 0.0, ld_im = 0.0;
  int ld_sw = 0;
  if (want_ld) {
    for (int v = tid; v < Nd; v += kThreads) {
      const zd u = *A.ptr(v, v);
      ld_re += log(hypot(u.x, u.y));
      ld_im += atan2(u.y, u.x);
      ld_sw += ro.ipiv[v] != v;
    }
    block_sum(ld_re, ld_im, ld_sw, sh);
  }

  finish_instance(p, inst, A, ro, ld_re, ld_im, ld_sw, tau00, info, sh);
}

// True when the instance cannot be processed (empty LIZ, LIZ above max_liz,
// energy index out of range, matrix too large for the leaf registers).
template <int kR>
__device__ __forceinline__ bool instance_invalid(const lsms_prob_dev& p, int inst) {
  const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
  const int e = p.e_idx[inst];
  return nliz < 1 || nliz > p.max_liz || e < 0 || e >= p.n_energy || p.kc * nliz > kThreads * kR;
}

__device__ __forceinline__ void fill_nan(const lsms_prob_dev& p, int inst, double* tau00) {
  zd* tout = reinterpret_cast<zd*>(tau00) + (int64_t)inst * p.kc * p.kc;
  for (int q = threadIdx.x; q < p.kc * p.kc; q += kThreads) tout[q] = zmake((double)NAN, (double)NAN);
}

template <int kR, int kWL>
__global__ __launch_bounds__(kThreads) void lu_schur_fp64_kernel(lsms_prob_dev p, int i0, double* __restrict__ Mb,
                                                                const int64_t* __restrict__ m_off, int64_t slot,
                                                                double* __restrict__ xgb, int64_t xstride,
                                                                double* __restrict__ tau00,
                                                                int32_t* __restrict__ info, int keep_info,
                                                                int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmemD& sh = *reinterpret_cast<LuSmemD*>(smem_raw);
  const int inst = i0 + blockIdx.x;
  const bool invalid = instance_invalid<kR>(p, inst);
  if ((keep_info && info[inst] != 0) || invalid) {
    fill_nan(p, inst, tau00);
    if (invalid && threadIdx.x == 0) info[inst] = -3;
    return;
  }
  zd* base = reinterpret_cast<zd*>(Mb) + (m_off ? m_off[inst] : (int64_t)(inst - i0) * slot);
  zd* xg = xgb ? reinterpret_cast<zd*>(xgb) + (int64_t)(inst - i0) * xstride : nullptr;
  lu_instance<kR, kWL>(p, inst, base, xg, tau00, info, nb, sh);
}

// Per-instance workspace of the block-row kernel: [xg | z | ipiv], each
// 256-byte aligned, for matrices up to nmax.
__host__ __device__ inline int row_kp(int kk) { return kk <= 16 ? 16 : 32; }
__host__ __device__ inline int64_t row_z_off() { return kLsmsXgBytes; }
__host__ __device__ inline int64_t row_ipiv_off(int64_t nmax, int kk) {
  return row_z_off() + ((nmax * row_kp(kk) * 16 + 255) & ~(int64_t)255);
}
__host__ __device__ inline int64_t row_slot_bytes(int64_t nmax, int kk) {
  return row_ipiv_off(nmax, kk) + ((nmax * 4 + 255) & ~(int64_t)255);
}

// One workgroup per instance i0 + blockIdx.x: tau00 and, where requested,
// the block row of tau (at row + 2 row_off[i] doubles) and ln det M (at
// logdet + 2 i).  Caller-built M at m_off[i]; the instance's workspace at
// work + (i - i0) wslot bytes.
template <int kR, int kWL>
__global__ __launch_bounds__(kThreads) void tau_row_fp64_kernel(
    lsms_prob_dev p, int i0, double* __restrict__ Mb, const int64_t* __restrict__ m_off,
    unsigned char* __restrict__ work, int64_t wslot, const int64_t* __restrict__ row_off,
    double* __restrict__ row, double* __restrict__ logdet, double* __restrict__ tau00,
    int32_t* __restrict__ info, int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmemD& sh = *reinterpret_cast<LuSmemD*>(smem_raw);
  const int inst = i0 + blockIdx.x;
  if (instance_invalid<kR>(p, inst)) {
    fill_nan(p, inst, tau00);
    if (threadIdx.x == 0) {
      info[inst] = -3;
      if (logdet) reinterpret_cast<zd*>(logdet)[inst] = zmake((double)NAN, (double)NAN);
    }
    return;
  }
  unsigned char* ws = work + (int64_t)(inst - i0) * wslot;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  RowOut ro;
  ro.z = reinterpret_cast<zd*>(ws + row_z_off());
  ro.ipiv = reinterpret_cast<int32_t*>(ws + row_ipiv_off(nmax, p.kk));
  ro.row = row ? reinterpret_cast<zd*>(row) + row_off[inst] : nullptr;
  ro.logdet = logdet ? reinterpret_cast<zd*>(logdet) + inst : nullptr;
  ro.kp = row_kp(p.kk);
  zd* base = reinterpret_cast<zd*>(Mb) + m_off[inst];
  lu_instance<kR, kWL>(p, inst, base, reinterpret_cast<zd*>(ws), tau00, info, nb, sh, ro);
}

// Next instance index from the device counter, the same for every thread of
// the workgroup (a wave-uniform scalar).  Must be reached by all threads, each
// coming from a barrier.
__device__ __forceinline__ int pop_instance(int32_t* counter, int* next) {
  if (threadIdx.x == 0) *next = atomicAdd(counter, 1);
  __syncthreads();
  const int k = __builtin_amdgcn_readfirstlane(*next);
  __syncthreads();
  return k;
}

// Persistent fused kernel: every resident workgroup repeatedly takes the
// next instance from the device counter (instances in the given order,
// largest first), builds its M in the workgroup's own slot of the workspace,
// eliminates it and writes tau00.  A workgroup leaves when the counter has
// passed n, so every workgroup exits after at most n + 1 increments.
//
// The loop-control values are wave-uniform scalars and every iteration ends
// with a barrier right before the next pop.  Without that barrier the compiler
// merged the thread-0 store at the end of an iteration with the thread-0
// increment at the top, so that lanes other than thread 0 looped back to the
// counter read without the increment ever running.
template <int kR, int kWL>
__global__ __launch_bounds__(kThreads) void tau00_persistent_kernel(lsms_prob_dev p, lsms_gaunt_dev g,
                                                                   const int32_t* __restrict__ order, int n,
                                                                   int32_t* __restrict__ counter,
                                                                   double* __restrict__ work, int64_t slot,
                                                                   int64_t xoff, double* __restrict__ tau00,
                                                                   int32_t* __restrict__ info, int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmemD& sh = *reinterpret_cast<LuSmemD*>(smem_raw);
  BuildSmem& sb = *reinterpret_cast<BuildSmem*>(smem_raw);  // used before sh, never at the same time
  __shared__ int next;
  zd* M = reinterpret_cast<zd*>(work) + (int64_t)blockIdx.x * slot;
  zd* xg = xoff ? M + xoff : nullptr;
  __syncthreads();
  int k = pop_instance(counter, &next);
  while (k < n) {
    const int inst = __builtin_amdgcn_readfirstlane(order ? order[k] : k);
    int status = __builtin_amdgcn_readfirstlane(instance_invalid<kR>(p, inst) ? -3 : 0);
    if (status == 0) {
      const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
      build_setup<kThreads>(p, g, inst, sb);
      for (int j = 0; j < nliz; ++j) build_column<kThreads>(p, inst, j, M, sb);
      status = __builtin_amdgcn_readfirstlane(sb.bad_species ? -3 : (sb.bad ? -2 : 0));
      __syncthreads();
    }
    if (status == 0) {
      lu_instance<kR, kWL>(p, inst, M, xg, tau00, info, nb, sh);
    } else {
      fill_nan(p, inst, tau00);
      if (threadIdx.x == 0) info[inst] = status;
    }
    __syncthreads();
    k = pop_instance(counter, &next);
  }
}

// ======================================================================
// Precision form: FP32 factorisation, FP64 iterative refinement.
//
// Y = A_int^{-1} E_c (E_c: the unit vectors of the central rows) holds
// [M^{-1}]_{00}^T in its central rows.  A copy of A in complex FP32 is
// factorised completely (non-central columns with pivots among the
// non-central rows, then the central block with pivots among the central
// rows), keeping L, U and the pivots.  Then Y_0 = A32^{-1} E_c and, until the
// correction of the central rows is below tol relative to them,
//   R = E_c - A Y   (FP64, the FP64 matrix is never modified)
//   D = A32^{-1} R  (FP32 forward/backward solves on MFMA)
//   Y = Y + D       (FP64)
// (mixed-precision iterative refinement with the residual in the working
// precision).  An instance that does not converge in max_refine steps, or
// whose FP32 factorisation meets an exactly zero pivot, is recomputed by the
// FP64 Schur path on its unmodified FP64 matrix and flagged in info (bit 8).
// ======================================================================

// Fallback flag of the precision form: bit 20, above every elimination step
// (N < 2^20), ORed onto the fallback's own non-negative info.
constexpr int kInfoIrFallback = 1 << 20;

struct MixedBufs {
  LSMS_GLOBAL zf* A32;        // N x N FP32 factors, same physical layout as M
  LSMS_GLOBAL zf* z;          // N x kp FP32 right-hand sides / corrections, internal rows
  LSMS_GLOBAL zd* Y;          // N x kp FP64 solution, internal rows
  LSMS_GLOBAL int32_t* ipiv;  // N pivot rows
  LSMS_GLOBAL zd* xg;         // two 64 x 64 blocks (FP64, or FP32 in the first half) for wide panels
  LSMS_GLOBAL zf* lcache;     // inverses of the 64-column diagonal blocks of L (factorisation order)
  LSMS_GLOBAL zf* ucache;     // inverses of the 64-row diagonal blocks of U (filled by the first solve)
  int kp;                // 16 or 32: kk rounded up to a multiple of 16
};

// Number of cached diagonal blocks of L in the panels of [0, c) (panels of
// nb columns over [0, Nd); a panel wider than 64 has two).
__device__ inline int lower_blocks_before(int c, int Nd, int nb) {
  int n = 0;
  for (int q = 0; q < c && q < Nd; q += nb) n += (min(nb, Nd - q) + kNB - 1) / kNB;
  return n;
}

// sh.X := the 64 x 64 block at src.
__device__ inline void load_x(const zf* __restrict__ src, LuSmem<float>& sh) {
  for (int q = threadIdx.x; q < kNB * kNB; q += kLuThreads) sh.X[q / kNB][q % kNB] = src[q];
  __syncthreads();
}

struct MixedSmem {
  LuSmem<float> f;
  zf part[2 * kNB * 16];  // split-K partial sums of the backward solve: [split][row][kp]
  double red[2][kLuWaves];
  int flag;
};
static_assert(sizeof(MixedSmem) <= 160 * 1024 && sizeof(LuSmem<double>) <= 160 * 1024 &&
                  sizeof(BuildSmem) <= 160 * 1024,
              "a workgroup's LDS on gfx950 is 160 KB");

// z[v][j] (v in [r0, r0 + s), j < kp) = X * z[r0 .. r0 + s) with X = sh.X (s x s):
// up to eight 16x16 tiles, one per wave; the result also goes to sh.U.
__device__ void tri_apply(const MixedBufs& b, int r0, int s, LuSmem<float>& sh) {
  typedef Prec<float>::V4 V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int nct = b.kp / 16;
  const int rt = wave & 3, ct = wave >> 2;
  V4 ar = V4{0.f, 0.f, 0.f, 0.f}, ai = V4{0.f, 0.f, 0.f, 0.f};
  const bool act = ct < nct;
  if (act) {
    // the lane's z entries for the whole block, loaded together (rows
    // clamped to the block; X is zero in the columns k >= s)
    zf y[kNB / 4];
#pragma unroll
    for (int m = 0; m < kNB / 4; ++m) y[m] = b.z[(int64_t)(r0 + min(4 * m + lq, s - 1)) * b.kp + 16 * ct + li];
#pragma unroll
    for (int m = 0; m < kNB / 4; ++m) {
      if (4 * m >= s) break;
      const int k = 4 * m + lq;
      const zf x = sh.X[16 * rt + li][k];
      const float xr = (k < s) ? x.x : 0.f, xi = (k < s) ? x.y : 0.f;
      ar = Prec<float>::mfma(xr, y[m].x, ar);
      ar = Prec<float>::mfma(-xi, y[m].y, ar);
      ai = Prec<float>::mfma(xr, y[m].y, ai);
      ai = Prec<float>::mfma(xi, y[m].x, ai);
    }
  }
  __syncthreads();  // every wave has read z[r0 ..] and sh.X
  if (act) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rt + Prec<float>::drow(r, lq);
      const zf v = zmake(ar[r], ai[r]);
      sh.U[i][16 * ct + li] = v;
      if (i < s) b.z[(int64_t)(r0 + i) * b.kp + 16 * ct + li] = v;
    }
  }
  __syncthreads();
}

// z[v] -= sum_{k < s} A(v, r0 + k) sh.U[k] for v in [v0, N), s <= 64: 16-row
// blocks per wave, accumulators starting from the loaded block of z; lane
// (li, lq) supplies k = 16 c + 4 lq + j at MFMA step j of chunk c.  All
// operands of the next row block (its whole reduction and its z entries) are
// loaded while the current block is multiplied, so that a wave keeps a whole
// block of loads in flight.  Loads are unconditional from clamped in-range
// addresses (rows >= N are never stored; L entries of columns >= s meet the
// zero rows s.. of sh.U), and a finished block is stored after the next
// block's loads are issued (loads and stores share one completion counter).
template <int NCT>
__device__ void rhs_update_rows(const Mat<zf>& A, const MixedBufs& b, int r0, int s, int v0,
                                const LuSmem<float>& sh) {
  typedef Prec<float>::V4 V4;
  constexpr int KC = kNB / 16;  // chunks of 16 in a reduction of at most kNB
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int N = (int)A.N;
  const int64_t pr0 = A.phys(r0);
  int rb = v0 + 16 * wave;
  if (rb < N) {
    zf cn[NCT][4], an[KC][4], pv[NCT][4];
    int pb = -1;
    auto load_c = [&](int q) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = min(q + Prec<float>::drow(r, lq), N - 1);
#pragma unroll
        for (int t = 0; t < NCT; ++t) cn[t][r] = b.z[(int64_t)v * b.kp + 16 * t + li];
      }
    };
    auto load_a = [&](int q) {
      const int va = q + li;
      const auto arow = A.base + A.phys(va < N ? va : v0) * A.N + pr0;
#pragma unroll
      for (int c = 0; c < KC; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) an[c][j] = arow[min(16 * c + 4 * lq + j, s - 1)];
    };
    auto store_pv = [&](int q) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = q + Prec<float>::drow(r, lq);
        if (v >= N) continue;
#pragma unroll
        for (int t = 0; t < NCT; ++t) b.z[(int64_t)v * b.kp + 16 * t + li] = pv[t][r];
      }
    };
    load_c(rb);
    load_a(rb);
    for (; rb < N; rb += 16 * kLuWaves) {
      const int rn = rb + 16 * kLuWaves;
      V4 ar[NCT], ai[NCT];
#pragma unroll
      for (int t = 0; t < NCT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          ar[t][r] = cn[t][r].x;
          ai[t][r] = cn[t][r].y;
        }
      zf a[KC][4];
#pragma unroll
      for (int c = 0; c < KC; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) a[c][j] = an[c][j];
      if (rn < N) {
        load_c(rn);
        load_a(rn);
      }
      if (pb >= 0) store_pv(pb);
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        if (16 * c >= s) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = 16 * c + 4 * lq + j;
          const float nx = -a[c][j].x, ny = -a[c][j].y;
#pragma unroll
          for (int t = 0; t < NCT; ++t) {
            const zf u = sh.U[k][16 * t + li];
            ar[t] = Prec<float>::mfma(nx, u.x, ar[t]);
            ar[t] = Prec<float>::mfma(a[c][j].y, u.y, ar[t]);
            ai[t] = Prec<float>::mfma(nx, u.y, ai[t]);
            ai[t] = Prec<float>::mfma(ny, u.x, ai[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NCT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) pv[t][r] = zmake(ar[t][r], ai[t][r]);
      pb = rb;
    }
    if (pb >= 0) store_pv(pb);
  }
  __syncthreads();
}

__device__ void rhs_update(const Mat<zf>& A, const MixedBufs& b, int r0, int s, int v0, const LuSmem<float>& sh) {
  if (b.kp > 16) rhs_update_rows<2>(A, b, r0, s, v0, sh);
  else rhs_update_rows<1>(A, b, r0, s, v0, sh);
}

// z := A32^{-1} z with the panel structure of the factorisation: forward with
// the unit lower factor (each panel's interchanges applied just before its
// columns are used, since earlier columns of L keep their own row order; a
// panel wider than 64 is then taken in 64-column blocks, its own L being in
// the panel's final row order), then backward with the upper factor in
// 64-row blocks.
__device__ void solve_f32(const Mat<zf>& A, const MixedBufs& b, int nb, bool have_uinv, MixedSmem& ms) {
  typedef Prec<float>::V4 V4;
  LuSmem<float>& sh = ms.f;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int N = (int)A.N, Nd = A.Nd, nct = b.kp / 16;
  if (!b.xg) nb = min(nb, kNB);
  // panels: [0, Nd) in steps of nb, then [Nd, N)
  const int npan = (Nd + nb - 1) / nb + 1;
  for (int pi = 0; pi < npan; ++pi) {
    const int c = pi + 1 < npan ? pi * nb : Nd;
    const int w = pi + 1 < npan ? min(nb, Nd - c) : N - Nd;
    if (w <= 0) continue;
    if (tid < b.kp) {
      for (int jj = 0; jj < w; ++jj) {
        const int pr = b.ipiv[c + jj];
        if (pr != c + jj) {
          zf* a0 = b.z + (int64_t)(c + jj) * b.kp + tid;
          zf* a1 = b.z + (int64_t)pr * b.kp + tid;
          const zf x = *a0, y = *a1;
          *a0 = y;
          *a1 = x;
        }
      }
    }
    __syncthreads();
    int blk = pi + 1 < npan ? lower_blocks_before(c, Nd, nb) : lower_blocks_before(Nd, Nd, nb);
    for (int c2 = c; c2 < c + w; c2 += kNB, ++blk) {
      const int w2 = min(kNB, c + w - c2);
      load_x(b.lcache + (int64_t)blk * kNB * kNB, sh);
      tri_apply(b, c2, w2, sh);
      if (c2 + w2 < N) rhs_update(A, b, c2, w2, c2 + w2, sh);
    }
  }
  const int nblk = (Nd + kNB - 1) / kNB + 1;
  for (int pi = nblk - 1; pi >= 0; --pi) {
    const int c = pi + 1 < nblk ? pi * kNB : Nd;
    const int w = pi + 1 < nblk ? min(kNB, Nd - c) : N - Nd;
    if (w <= 0) continue;
    // part = U(c .. c+w, c+w .. N) z(c+w .. N), split over k between wave halves
    const int ntile = 4 * nct, nsplit = kLuWaves / ntile;
    const int tile = wave % ntile, split = wave / ntile;
    const int rt = tile & 3, ct = tile >> 2;
    const int k0 = c + w, klen = N - k0;
    const int kchunk = ((klen + nsplit - 1) / nsplit + 15) & ~15;
    const int ka = k0 + split * kchunk, kz = min(N, ka + kchunk);
    V4 ar = V4{0.f, 0.f, 0.f, 0.f}, ai = V4{0.f, 0.f, 0.f, 0.f};
    const int row = c + 16 * rt + li;
    const bool rok = 16 * rt + li < w;
    const auto urow = A.base + A.phys(rok ? row : c) * A.N;
    // chunks of 16 (lane (li, lq) takes k = kb + 4 lq + j at step j), loaded
    // one chunk ahead from clamped addresses; entries past the range are
    // zeroed before they enter the product
    zf an[4], yn[4];
    auto ld = [&](int kb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = min(kb + 4 * lq + j, N - 1);
        an[j] = urow[A.phys(k)];
        yn[j] = b.z[(int64_t)k * b.kp + 16 * ct + li];
      }
    };
    if (ka < kz) ld(ka);
    for (int kb = ka; kb < kz; kb += 16) {
      zf a[4], y[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a[j] = an[j];
        y[j] = yn[j];
      }
      if (kb + 16 < kz) ld(kb + 16);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = rok && kb + 4 * lq + j < kz;
        const float axr = ok ? a[j].x : 0.f, axi = ok ? a[j].y : 0.f;
        ar = Prec<float>::mfma(axr, y[j].x, ar);
        ar = Prec<float>::mfma(-axi, y[j].y, ar);
        ai = Prec<float>::mfma(axr, y[j].y, ai);
        ai = Prec<float>::mfma(axi, y[j].x, ai);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      ms.part[(split * kNB + 16 * rt + Prec<float>::drow(r, lq)) * b.kp + 16 * ct + li] = zmake(ar[r], ai[r]);
    if (have_uinv) {
      __syncthreads();
      load_x(b.ucache + (int64_t)pi * kNB * kNB, sh);
    } else {
      invert_upper<float>(A, c, w, sh);  // starts and ends with a barrier
      save_x<float>(sh, b.ucache + (int64_t)pi * kNB * kNB);
    }
    for (int q = tid; q < kNB * 32; q += kLuThreads) {
      const int i = q / 32, j = q % 32;
      zf v = zmake(0.f, 0.f);
      if (i < w && j < b.kp) {
        const zf zc = b.z[(int64_t)(c + i) * b.kp + j];
        zf acc = ms.part[i * b.kp + j];
        if (nsplit > 1) {
          const zf p1 = ms.part[(kNB + i) * b.kp + j];
          acc = zmake(acc.x + p1.x, acc.y + p1.y);
        }
        v = zmake(zc.x - acc.x, zc.y - acc.y);
      }
      if (j < kSWp<float>) sh.U[i][j] = v;
    }
    __syncthreads();
    // z(c .. c+w) = X_u * sh.U
    V4 br = V4{0.f, 0.f, 0.f, 0.f}, bi = V4{0.f, 0.f, 0.f, 0.f};
    const int rt2 = wave & 3, ct2 = wave >> 2;
    const bool act = ct2 < nct;
    if (act) {
      for (int kb = 0; kb < w; kb += 4) {
        const int k = kb + lq;
        const zf x = sh.X[16 * rt2 + li][k];
        const zf y = sh.U[k][16 * ct2 + li];
        const float xr = (k < w) ? x.x : 0.f, xi = (k < w) ? x.y : 0.f;
        br = Prec<float>::mfma(xr, y.x, br);
        br = Prec<float>::mfma(-xi, y.y, br);
        bi = Prec<float>::mfma(xr, y.y, bi);
        bi = Prec<float>::mfma(xi, y.x, bi);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * rt2 + Prec<float>::drow(r, lq);
        if (i < w) b.z[(int64_t)(c + i) * b.kp + 16 * ct2 + li] = zmake(br[r], bi[r]);
      }
    }
    __syncthreads();
  }
}

// z = E_c - A64 Y in FP32 (rows of the FP64 matrix times the FP64 solution),
// one 16-row block per wave at a time.  The reduction over k runs in chunks
// of 16 (lane (li, lq) supplies k = kc + 4 lq + j at MFMA step j, four
// consecutive entries of its matrix row) with the next chunk's operands
// loaded while the current one is multiplied.
template <int NCT>
__device__ void residual_rows(const Mat<zd>& A, const MixedBufs& b) {
  typedef Prec<double>::V4 V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int N = (int)A.N, Nd = A.Nd, kk = A.kk;
  for (int rb = 16 * wave; rb < N; rb += 16 * kLuWaves) {
    V4 ar[NCT], ai[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      ar[t] = V4{0.0, 0.0, 0.0, 0.0};
      ai[t] = V4{0.0, 0.0, 0.0, 0.0};
    }
    const int va = rb + li;
    const bool rok = va < N;
    const auto arow = A.base + A.phys(rok ? va : 0) * A.N;
    // A(va, k) for k < Nd is at arow[kk + k], for k >= Nd at arow[k - Nd];
    // clamped in-range loads, entries of k >= N zeroed before the product
    zd an[4], yn[NCT][4];
    auto load = [&](int kc) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = min(kc + 4 * lq + j, N - 1);
        an[j] = arow[A.phys(k)];
#pragma unroll
        for (int t = 0; t < NCT; ++t) yn[t][j] = b.Y[(int64_t)k * b.kp + 16 * t + li];
      }
    };
    load(0);
    for (int kc = 0; kc < N; kc += 16) {
      zd a[4], y[NCT][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = kc + 4 * lq + j < N;
        a[j] = ok ? an[j] : zmake(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < NCT; ++t) y[t][j] = yn[t][j];
      }
      if (kc + 16 < N) load(kc + 16);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
          ar[t] = Prec<double>::mfma(a[j].x, y[t][j].x, ar[t]);
          ar[t] = Prec<double>::mfma(-a[j].y, y[t][j].y, ar[t]);
          ai[t] = Prec<double>::mfma(a[j].x, y[t][j].y, ai[t]);
          ai[t] = Prec<double>::mfma(a[j].y, y[t][j].x, ai[t]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = rb + Prec<double>::drow(r, lq);
        const int j = 16 * t + li;
        if (v < N) {
          const double e = (j < kk && v == Nd + j) ? 1.0 : 0.0;
          b.z[(int64_t)v * b.kp + j] = zmake((float)(e - ar[t][r]), (float)(-ai[t][r]));
        }
      }
    }
  }
  __syncthreads();
}

__device__ void residual(const Mat<zd>& A, const MixedBufs& b) {
  if (b.kp > 16) residual_rows<2>(A, b);
  else residual_rows<1>(A, b);
}

// Precision-form tau00 of one instance.  A64 is the FP64 matrix (left
// unmodified unless the FP64 fallback runs).  Ends after a barrier.
template <int kR, int kWL>
__device__ __noinline__ void mixed_instance(const lsms_prob_dev& p, int inst, zd* A64, const MixedBufs& bin,
                                            double* tau00, int32_t* info, int nb, double tol, int max_refine,
                                            bool have_a32, unsigned char* smem) {
  // By value: the pointers and kp stay in registers.  Read through the
  // reference, every use would reload them with a generic load (a store
  // through z might alias the struct), and each such load waits for every
  // outstanding memory access.
  const MixedBufs b = bin;
  MixedSmem& ms = *reinterpret_cast<MixedSmem*>(smem);
  LuSmem<float>& sh = ms.f;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kk = p.kk;
  const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
  const int N = kk * nliz, Nd = N - kk;
  Mat<zd> A;
  A.base = glb(A64);
  A.N = N;
  A.Nd = Nd;
  A.kk = kk;
  Mat<zf> F;
  F.base = glb(b.A32);
  F.N = N;
  F.Nd = Nd;
  F.kk = kk;
  if (!have_a32) {
    for (int64_t q = tid; q < (int64_t)N * N; q += kLuThreads) {
      const zd x = A64[q];
      b.A32[q] = zmake((float)x.x, (float)x.y);
    }
  }
  if (tid == 0) sh.info = 0;
  __syncthreads();
  eliminate<float, kR, kWL>(F, 0, Nd, Nd, nb, true, b.ipiv, reinterpret_cast<zf*>(b.xg), sh, b.lcache);
  eliminate<float, kR, kWL>(F, Nd, N, N, nb, true, b.ipiv, reinterpret_cast<zf*>(b.xg), sh);
  // the central block's unit lower inverse (it has no trailing columns)
  invert_unit_lower<float>(F, Nd, N - Nd, sh);
  save_x<float>(sh, b.lcache + (int64_t)lower_blocks_before(Nd, Nd, nb) * kNB * kNB);
  bool ok = __builtin_amdgcn_readfirstlane(sh.info) == 0;
  if (ok) {
    for (int q = tid; q < N * b.kp; q += kLuThreads) {
      const int v = q / b.kp, j = q % b.kp;
      b.z[q] = zmake((j < kk && v == Nd + j) ? 1.f : 0.f, 0.f);
    }
    __syncthreads();
    solve_f32(F, b, nb, false, ms);
    for (int q = tid; q < N * b.kp; q += kLuThreads) {
      const zf x = b.z[q];
      b.Y[q] = zmake((double)x.x, (double)x.y);
    }
    __syncthreads();
    bool conv = false;
    double dprev = 0.0;
    for (int it = 0; it < max_refine && !conv; ++it) {
      residual(A, b);
      solve_f32(F, b, nb, true, ms);
      double dn = 0.0, yn = 0.0;
      for (int q = tid; q < N * b.kp; q += kLuThreads) {
        const int v = q / b.kp, j = q % b.kp;
        const zf d = b.z[q];
        zd y = b.Y[q];
        y = zmake(y.x + (double)d.x, y.y + (double)d.y);
        b.Y[q] = y;
        if (v >= Nd && j < kk) {
          dn += (double)d.x * d.x + (double)d.y * d.y;
          yn += y.x * y.x + y.y * y.y;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        dn += __shfl_xor(dn, off);
        yn += __shfl_xor(yn, off);
      }
      if (lane == 0) {
        ms.red[0][wave] = dn;
        ms.red[1][wave] = yn;
      }
      __syncthreads();
      dn = 0.0;
      yn = 0.0;
#pragma unroll
      for (int q = 0; q < kLuWaves; ++q) {
        dn += ms.red[0][q];
        yn += ms.red[1][q];
      }
      // converged when the correction is below tol, or when the contraction
      // seen over the last two steps (at most 1/2) predicts that the next
      // correction is: |d_k|^2 / |d_{k-1}| <= tol |Y|.  The first FP32 solve
      // is the step from a zero start (its correction is Y itself, |Y| taken
      // after this step), so one refinement step can already show it; that
      // first estimate of the contraction is asked for a margin of 4
      // (predicted correction at most tol / 4).
      const double dp = it > 0 ? dprev : yn;
      const double margin = it > 0 ? 1.0 : 1.0 / 16.0;
      const bool small = dn <= tol * tol * yn;
      const bool predicted = dn <= 0.25 * dp && dn * dn <= margin * tol * tol * yn * dp;
      conv = __builtin_amdgcn_readfirstlane((int)(small || predicted)) != 0;
      dprev = dn;
      __syncthreads();
    }
    ok = conv;
  }
  if (ok) {
    const int e = p.e_idx[inst];
    const zd kap = zsqrt(reinterpret_cast<const zd*>(p.energy)[e]);
    const int s0 = min(max(p.species[p.liz_off[inst]], 0), p.n_species - 1);
    const zd* dl = reinterpret_cast<const zd*>(p.delta) + ((int64_t)s0 * p.n_energy + e) * (p.lmax + 1);
    zd* tout = reinterpret_cast<zd*>(tau00) + (int64_t)inst * kk * kk;
    if (tid == 0) ms.flag = 0;
    __syncthreads();
    for (int q = tid; q < kk * kk; q += kLuThreads) {
      const int L = q % kk, Lp = q / kk;
      // [M^{-1}]_00(L, L') = Y(Nd + L', L)
      const zd v = zmul(b.Y[(int64_t)(Nd + Lp) * b.kp + L], tmat_from_delta(dl[l_of(Lp)], kap));
      if (!zfinite(v)) ms.flag = 1;
      tout[q] = v;
    }
    __syncthreads();
    if (tid == 0) info[inst] = ms.flag ? -1 : 0;
    __syncthreads();
  } else {
    lu_instance<kR, kWL>(p, inst, A64, b.xg, tau00, info, nb, *reinterpret_cast<LuSmemD*>(smem));
    if (tid == 0 && info[inst] >= 0) info[inst] |= kInfoIrFallback;
    __syncthreads();
  }
}

// LDS of the precision-form kernels: the FP32 elimination, the FP64 fallback
// and (persistent form) the build use the same bytes one after the other.
size_t mixed_smem_bytes() {
  size_t b = sizeof(MixedSmem) > sizeof(LuSmemD) ? sizeof(MixedSmem) : sizeof(LuSmemD);
  return b > sizeof(BuildSmem) ? b : sizeof(BuildSmem);
}

// Per-instance buffers of the precision form laid out as
// [FP32 matrix | z | Y | pivots | X blocks], each 256-byte aligned, for
// matrices up to nmax.
constexpr int64_t kXgBytes = 2 * kNB * kNB * 16;
// inverse-block caches: L blocks follow the panels (at most one per 16
// columns for panel widths >= 16), U blocks the 64-row blocks
__host__ __device__ inline int64_t mixed_lcache_bytes(int64_t nmax) { return (nmax / 16 + 2) * kNB * kNB * 8; }
__host__ __device__ inline int64_t mixed_ucache_bytes(int64_t nmax) {
  return ((nmax + kNB - 1) / kNB + 1) * kNB * kNB * 8;
}
__host__ __device__ inline int64_t mixed_extra_bytes(int64_t nmax, int kp) {
  const int64_t a = ((nmax * nmax * 8) + 255) & ~(int64_t)255;
  const int64_t z = ((nmax * kp * 8) + 255) & ~(int64_t)255;
  const int64_t y = ((nmax * kp * 16) + 255) & ~(int64_t)255;
  const int64_t pv = ((nmax * 4) + 255) & ~(int64_t)255;
  return a + z + y + pv + kXgBytes + mixed_lcache_bytes(nmax) + mixed_ucache_bytes(nmax);
}

__device__ inline MixedBufs mixed_bufs(unsigned char* base, int64_t nmax, int kp) {
  MixedBufs b;
  const int64_t a = ((nmax * nmax * 8) + 255) & ~(int64_t)255;
  const int64_t z = ((nmax * kp * 8) + 255) & ~(int64_t)255;
  const int64_t y = ((nmax * kp * 16) + 255) & ~(int64_t)255;
  const int64_t pv = ((nmax * 4) + 255) & ~(int64_t)255;
  b.A32 = glb(reinterpret_cast<zf*>(base));
  b.z = glb(reinterpret_cast<zf*>(base + a));
  b.Y = glb(reinterpret_cast<zd*>(base + a + z));
  b.ipiv = glb(reinterpret_cast<int32_t*>(base + a + z + y));
  b.xg = glb(reinterpret_cast<zd*>(base + a + z + y + pv));
  b.lcache = glb(reinterpret_cast<zf*>(base + a + z + y + pv + kXgBytes));
  b.ucache = glb(reinterpret_cast<zf*>(base + a + z + y + pv + kXgBytes + mixed_lcache_bytes(nmax)));
  b.kp = kp;
  return b;
}

// Chunked form: one workgroup per instance of the pass; M_i (FP64) at
// M + (i - i0) * slot, its precision-form buffers at extra + (i - i0) * xslot.
template <int kR, int kWL>
__global__ __launch_bounds__(kThreads) void tau00_mixed_kernel(lsms_prob_dev p, int i0, double* __restrict__ Mb,
                                                              int64_t slot, unsigned char* __restrict__ extra,
                                                              int64_t xslot, double* __restrict__ tau00,
                                                              int32_t* __restrict__ info, int nb, double tol,
                                                              int max_refine) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int inst = i0 + blockIdx.x;
  const bool invalid = instance_invalid<kR>(p, inst);
  if (info[inst] != 0 || invalid) {
    fill_nan(p, inst, tau00);
    if (invalid && threadIdx.x == 0) info[inst] = -3;
    return;
  }
  const int kp = p.kk > 16 ? 32 : 16;
  const MixedBufs b = mixed_bufs(extra + (int64_t)blockIdx.x * xslot, (int64_t)p.kc * p.max_liz, kp);
  mixed_instance<kR, kWL>(p, inst, reinterpret_cast<zd*>(Mb) + (int64_t)blockIdx.x * slot, b, tau00, info, nb,
                          tol, max_refine, false, smem_raw);
}

// Persistent form, as tau00_persistent_kernel with the precision form per
// instance; slot bytes per workgroup: FP64 matrix then the extra buffers.
template <int kR, int kWL>
__global__ __launch_bounds__(kThreads) void tau00_mixed_persistent_kernel(
    lsms_prob_dev p, lsms_gaunt_dev g, const int32_t* __restrict__ order, int n, int32_t* __restrict__ counter,
    unsigned char* __restrict__ work, int64_t slot_bytes, int64_t m_bytes, double* __restrict__ tau00,
    int32_t* __restrict__ info, int nb, double tol, int max_refine) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  BuildSmem& sb = *reinterpret_cast<BuildSmem*>(smem_raw);
  __shared__ int next;
  unsigned char* base = work + (int64_t)blockIdx.x * slot_bytes;
  zd* M = reinterpret_cast<zd*>(base);
  const int kp = p.kk > 16 ? 32 : 16;
  const MixedBufs b = mixed_bufs(base + m_bytes, (int64_t)p.kc * p.max_liz, kp);
  __syncthreads();
  int k = pop_instance(counter, &next);
  while (k < n) {
    const int inst = __builtin_amdgcn_readfirstlane(order ? order[k] : k);
    int status = __builtin_amdgcn_readfirstlane(instance_invalid<kR>(p, inst) ? -3 : 0);
    if (status == 0) {
      const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
      build_setup<kThreads>(p, g, inst, sb);
      for (int j = 0; j < nliz; ++j) build_column<kThreads>(p, inst, j, M, sb, b.A32);
      status = __builtin_amdgcn_readfirstlane(sb.bad_species ? -3 : (sb.bad ? -2 : 0));
      __syncthreads();
    }
    if (status == 0) {
      mixed_instance<kR, kWL>(p, inst, M, b, tau00, info, nb, tol, max_refine, true, smem_raw);
    } else {
      fill_nan(p, inst, tau00);
      if (threadIdx.x == 0) info[inst] = status;
    }
    __syncthreads();
    k = pop_instance(counter, &next);
  }
}

// ======================================================================
// Learned form: block GMRES on A Y = E_c (A = M^T, E_c the unit vectors of
// the central rows, as in the precision form), seeded by an approximation D
// of [M^{-1}]_{00}, with the FP64 Schur path as the fallback.
//
// Seed: Y_c = D^T in the central rows, then Y_r = (E_c - A Y)_r, one Jacobi
// step on the other rows (exact when the other sites do not scatter among
// themselves).  Restarted block GMRES(m) with the 16 right-hand sides as one
// block: block Arnoldi with classical Gram-Schmidt applied twice, each new
// block orthonormalised by Cholesky QR applied twice, the least-squares
// problem on the block Hessenberg matrix solved by Householder QR, restarts
// until ||E_c - A Y||_F <= tol ||E_c||_F (all in FP64).  lmax = 3 only
// (kk = 16, one 16-column block).
// ======================================================================

// Fallback flag of the GMRES form: bit 21, ORed like kInfoIrFallback.
constexpr int kInfoLuFallback = 1 << 21;
// Instances sent straight to the FP64 path by the caller's routing: bit 22.
constexpr int kInfoRouted = 1 << 22;
constexpr int kGmMaxM = 8;  // block Arnoldi steps per restart, at most

struct GmresBufs {
  LSMS_GLOBAL zd* Y;  // N x 16 solution (row-major, internal rows)
  LSMS_GLOBAL zd* R;  // N x 16 residual
  LSMS_GLOBAL zd* V;  // (m + 1) blocks of N x 16
  LSMS_GLOBAL zd* H;  // ((m + 1) 16) x (m 16) block Hessenberg, column-major
  LSMS_GLOBAL zd* G;  // ((m + 1) 16) x 16 least-squares right-hand side, column-major
  LSMS_GLOBAL zd* Q;  // Householder vectors of the QR of H, 32 per column (16 m columns)
  LSMS_GLOBAL double* beta;  // their scale factors
  int m;
};

struct GmresSmem {
  zd h[(kGmMaxM + 1) * 16][16];  // Gram-Schmidt coefficients of one block column
  zd l[16][16];                  // Cholesky factor, then its inverse
  zd r[16][16];                  // triangular factor of a block QR
  zd t[16][16];                  // scratch
  zd hv[48];                     // Householder vector
  zd part[kLuWaves][16][16];     // per-wave partial sums of a block inner product
  double red[kLuWaves];
  double beta;
  int flag;
};

__device__ __forceinline__ zd zconj(zd a) { return zmake(a.x, -a.y); }

// out = A X (resid = false) or E_c - A X (resid = true); X, out N x 16
// row-major.  FP64 MFMA, one 16-row block per wave at a time, the reduction
// in chunks of 16 loaded one chunk ahead.
__device__ void gm_amul(const Mat<zd>& A, const zd* __restrict__ X, zd* __restrict__ out, bool resid) {
  typedef Prec<double>::V4 V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int N = (int)A.N, Nd = A.Nd;
  for (int rb = 16 * wave; rb < N; rb += 16 * kLuWaves) {
    V4 ar = V4{0.0, 0.0, 0.0, 0.0}, ai = V4{0.0, 0.0, 0.0, 0.0};
    const int va = rb + li;
    const bool rok = va < N;
    const auto arow = A.base + A.phys(rok ? va : 0) * A.N;
    zd an[4], xn[4];
    auto load = [&](int kc) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kc + 4 * lq + j;
        zd av = zmake(0.0, 0.0), xv = zmake(0.0, 0.0);
        if (k < N) {
          if (rok) av = arow[A.phys(k)];
          xv = X[(int64_t)k * 16 + li];
        }
        an[j] = av;
        xn[j] = xv;
      }
    };
    load(0);
    for (int kc = 0; kc < N; kc += 16) {
      zd a[4], x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a[j] = an[j];
        x[j] = xn[j];
      }
      if (kc + 16 < N) load(kc + 16);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        ar = Prec<double>::mfma(a[j].x, x[j].x, ar);
        ar = Prec<double>::mfma(-a[j].y, x[j].y, ar);
        ai = Prec<double>::mfma(a[j].x, x[j].y, ai);
        ai = Prec<double>::mfma(a[j].y, x[j].x, ai);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = rb + Prec<double>::drow(r, lq);
      if (v < N) {
        zd o = zmake(ar[r], ai[r]);
        if (resid) o = zmake(((v == Nd + li) ? 1.0 : 0.0) - o.x, -o.y);
        out[(int64_t)v * 16 + li] = o;
      }
    }
  }
  __syncthreads();
}

// gs.h[16 i + a][b] = sum_v conj(V_i[v][a]) W[v][b], i < nb, on FP64 MFMA:
// for each block i the waves take interleaved chunks of 4 rows (lane (li, lq)
// supplies conj(V_i[v0 + lq][li]) and W[v0 + lq][li], so that a chunk is one
// MFMA step of a 16 x 16 tile), two chunks loaded ahead, and the eight
// partial tiles are summed through LDS in a fixed order.
__device__ void gm_gram(const zd* __restrict__ V, int nb, int N, const zd* __restrict__ W, GmresSmem& gs) {
  typedef Prec<double>::V4 V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  for (int i = 0; i < nb; ++i) {
    const zd* vi = V + (int64_t)i * N * 16;
    V4 ar = V4{0.0, 0.0, 0.0, 0.0}, ai = V4{0.0, 0.0, 0.0, 0.0};
    auto ld = [&](int v0, zd& x, zd& y) {
      const int v = v0 + lq;
      x = v < N ? vi[(int64_t)v * 16 + li] : zmake(0.0, 0.0);
      y = v < N ? W[(int64_t)v * 16 + li] : zmake(0.0, 0.0);
    };
    constexpr int kStep = 4 * kLuWaves;
    zd x0, y0, x1, y1;
    ld(4 * wave, x0, y0);
    ld(4 * wave + kStep, x1, y1);
    for (int v0 = 4 * wave; v0 < N; v0 += kStep) {
      const zd x = x0, y = y0;
      x0 = x1;
      y0 = y1;
      ld(v0 + 2 * kStep, x1, y1);
      ar = Prec<double>::mfma(x.x, y.x, ar);
      ar = Prec<double>::mfma(x.y, y.y, ar);
      ai = Prec<double>::mfma(x.x, y.y, ai);
      ai = Prec<double>::mfma(-x.y, y.x, ai);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) gs.part[wave][Prec<double>::drow(r, lq)][li] = zmake(ar[r], ai[r]);
    __syncthreads();
    if (tid < 256) {
      const int a = tid >> 4, b = tid & 15;
      zd acc = gs.part[0][a][b];
#pragma unroll
      for (int w = 1; w < kLuWaves; ++w) acc = zadd(acc, gs.part[w][a][b]);
      gs.h[16 * i + a][b] = acc;
    }
    __syncthreads();
  }
}

// W[v][b] -= sum_{i < nb, a} V_i[v][a] gs.h[16 i + a][b] on FP64 MFMA: one
// 16-row block per wave at a time, the 16 nb columns of V in chunks of 4
// (lane (li, lq) supplies V_i[rb + li][a0 + lq] and gs.h[16 i + a0 + lq][li]).
__device__ void gm_subtract(const zd* __restrict__ V, int nb, int N, zd* __restrict__ W, const GmresSmem& gs) {
  typedef Prec<double>::V4 V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  for (int rb = 16 * wave; rb < N; rb += 16 * kLuWaves) {
    V4 ar = V4{0.0, 0.0, 0.0, 0.0}, ai = V4{0.0, 0.0, 0.0, 0.0};
    const int va = min(rb + li, N - 1);
    for (int i = 0; i < nb; ++i) {
      const zd* vr = V + ((int64_t)i * N + va) * 16;
      zd x[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) x[c] = vr[4 * c + lq];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const zd hh = gs.h[16 * i + 4 * c + lq][li];
        ar = Prec<double>::mfma(x[c].x, hh.x, ar);
        ar = Prec<double>::mfma(-x[c].y, hh.y, ar);
        ai = Prec<double>::mfma(x[c].x, hh.y, ai);
        ai = Prec<double>::mfma(x[c].y, hh.x, ai);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = rb + Prec<double>::drow(r, lq);
      if (v < N) {
        zd* o = W + (int64_t)v * 16 + li;
        *o = zmake(o->x - ar[r], o->y - ai[r]);
      }
    }
  }
  __syncthreads();
}

// W (N x 16) := Q with W = Q R, R upper triangular into gs.r (Cholesky QR
// applied twice: G = W^H W = L L^H, Q = W L^{-H}, R = L^H).  Returns false
// when the block is numerically rank deficient (a non-positive pivot).
__device__ bool gm_cholqr(zd* __restrict__ W, int N, GmresSmem& gs) {
  const int tid = threadIdx.x;
  for (int pass = 0; pass < 2; ++pass) {
    gm_gram(W, 1, N, W, gs);
    if (tid == 0) {
      int bad = 0;
      for (int j = 0; j < 16 && !bad; ++j) {
        double d = gs.h[j][j].x;
        for (int k = 0; k < j; ++k) d -= gs.l[j][k].x * gs.l[j][k].x + gs.l[j][k].y * gs.l[j][k].y;
        if (!(d > 1e-280)) {
          bad = 1;
          break;
        }
        const double ljj = sqrt(d);
        gs.l[j][j] = zmake(ljj, 0.0);
        for (int i = j + 1; i < 16; ++i) {
          zd acc = gs.h[i][j];
          for (int k = 0; k < j; ++k) acc = zfms(acc, gs.l[i][k], zconj(gs.l[j][k]));
          gs.l[i][j] = zscale(acc, 1.0 / ljj);
        }
        for (int i = 0; i < j; ++i) gs.l[i][j] = zmake(0.0, 0.0);
      }
      if (!bad) {
        // R := L^H R (R = I before the first pass)
        for (int i = 0; i < 16; ++i)
          for (int j = 0; j < 16; ++j) gs.t[i][j] = pass == 0 ? zmake(i == j ? 1.0 : 0.0, 0.0) : gs.r[i][j];
        for (int i = 0; i < 16; ++i)
          for (int j = 0; j < 16; ++j) {
            zd acc = zmake(0.0, 0.0);
            for (int k = i; k <= j; ++k) acc = zadd(acc, zmul(zconj(gs.l[k][i]), gs.t[k][j]));
            gs.r[i][j] = j >= i ? acc : zmake(0.0, 0.0);
          }
        // L := L^{-1} (forward substitution, column by column, via gs.t)
        for (int j = 0; j < 16; ++j) {
          for (int i = 0; i < 16; ++i) gs.t[i][j] = zmake(0.0, 0.0);
          gs.t[j][j] = zinv(gs.l[j][j]);
          for (int i = j + 1; i < 16; ++i) {
            zd acc = zmake(0.0, 0.0);
            for (int k = j; k < i; ++k) acc = zadd(acc, zmul(gs.l[i][k], gs.t[k][j]));
            gs.t[i][j] = zmul(zmake(-acc.x, -acc.y), zinv(gs.l[i][i]));
          }
        }
        for (int i = 0; i < 16; ++i)
          for (int j = 0; j < 16; ++j) gs.l[i][j] = gs.t[i][j];
      }
      gs.flag = bad;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(gs.flag)) return false;
    // W := W L^{-H}: W[v][b] = sum_{a <= b} W[v][a] conj(Linv[b][a])
    for (int v = tid; v < N; v += kLuThreads) {
      zd w[16];
#pragma unroll
      for (int a = 0; a < 16; ++a) w[a] = W[(int64_t)v * 16 + a];
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        zd acc = zmake(0.0, 0.0);
#pragma unroll
        for (int a = 0; a <= b; ++a) acc = zadd(acc, zmul(w[a], zconj(gs.l[b][a])));
        W[(int64_t)v * 16 + b] = acc;
      }
    }
    __syncthreads();
  }
  return true;
}

// Incremental Householder QR of the block Hessenberg H for the least-squares
// problem min || G - H y ||: block column j (16 columns, nonzero in rows
// < 16 (j + 2)) first receives the reflections of the earlier columns, then
// its own (one per column, at most 32 rows, vectors kept in b.Q), which are
// also applied to G.  Returns the Frobenius norm of rows 16 (j + 1) ..
// 16 (j + 2) of Q^H G, the residual norm of the least-squares solution over
// the first 16 (j + 1) columns.
__device__ double gm_qr_block(const GmresBufs& b, int ldh, int j, GmresSmem& gs) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // earlier reflections on the new columns (one thread per column, in order)
  if (tid < 16) {
    zd* col = b.H + (int64_t)(16 * j + tid) * ldh;
    for (int c = 0; c < 16 * j; ++c) {
      const int len = min(16 * (j + 2), 16 * (c / 16 + 2)) - c;
      const zd* v = b.Q + (int64_t)c * 32;
      zd acc = zmake(0.0, 0.0);
      for (int r = 0; r < len; ++r) acc = zadd(acc, zmul(zconj(v[r]), col[c + r]));
      acc = zscale(acc, b.beta[c]);
      for (int r = 0; r < len; ++r) col[c + r] = zfms(col[c + r], v[r], acc);
    }
  }
  __syncthreads();
  for (int c = 16 * j; c < 16 * (j + 1); ++c) {
    const int len = 16 * (j + 2) - c;
    if (tid == 0) {
      const zd* x = b.H + (int64_t)c * ldh + c;
      double nrm2 = 0.0;
      for (int r = 0; r < len; ++r) {
        gs.hv[r] = x[r];
        nrm2 += x[r].x * x[r].x + x[r].y * x[r].y;
      }
      const double nrm = sqrt(nrm2);
      const zd x0 = gs.hv[0];
      const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
      const zd ph = ax0 > 0.0 ? zscale(x0, 1.0 / ax0) : zmake(1.0, 0.0);
      // v = x + e^{i arg x0} ||x|| e_1, beta = 2 / (v^H v)
      gs.hv[0] = zadd(x0, zscale(ph, nrm));
      double vn = 0.0;
      for (int r = 0; r < len; ++r) vn += gs.hv[r].x * gs.hv[r].x + gs.hv[r].y * gs.hv[r].y;
      gs.beta = vn > 0.0 ? 2.0 / vn : 0.0;
      for (int r = 0; r < 32; ++r) b.Q[(int64_t)c * 32 + r] = r < len ? gs.hv[r] : zmake(0.0, 0.0);
      b.beta[c] = gs.beta;
    }
    __syncthreads();
    // apply to the block's columns c .. 16 (j + 1) - 1 and to the 16 columns of G
    const int ncol = 16 * (j + 1) - c;
    for (int q = tid; q < ncol + 16; q += kLuThreads) {
      zd* col = q < ncol ? b.H + (int64_t)(c + q) * ldh : b.G + (int64_t)(q - ncol) * ldh;
      zd acc = zmake(0.0, 0.0);
      for (int r = 0; r < len; ++r) acc = zadd(acc, zmul(zconj(gs.hv[r]), col[c + r]));
      acc = zscale(acc, gs.beta);
      for (int r = 0; r < len; ++r) col[c + r] = zfms(col[c + r], gs.hv[r], acc);
    }
    __syncthreads();
  }
  // residual norm: rows 16 (j + 1) .. 16 (j + 2) of G
  double sq = 0.0;
  for (int q = tid; q < 256; q += kLuThreads) {
    const zd g = b.G[(int64_t)(q & 15) * ldh + 16 * (j + 1) + (q >> 4)];
    sq += g.x * g.x + g.y * g.y;
  }
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
  if (lane == 0) gs.red[wave] = sq;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < kLuWaves; ++q) t += gs.red[q];
  __syncthreads();
  return sqrt(t);
}

// y = R^{-1} (Q^H G)[0 .. nc) for the triangular R left in H; y overwrites
// the first nc rows of G.  Returns false on a zero diagonal.
__device__ bool gm_backsolve(const GmresBufs& b, int ldh, int nc, GmresSmem& gs) {
  const int tid = threadIdx.x;
  if (tid == 0) gs.flag = 0;
  __syncthreads();
  if (tid < 16) {
    zd* g = b.G + (int64_t)tid * ldh;
    for (int c = nc - 1; c >= 0; --c) {
      zd acc = g[c];
      for (int k = c + 1; k < nc; ++k) acc = zfms(acc, b.H[(int64_t)k * ldh + c], g[k]);
      const zd d = b.H[(int64_t)c * ldh + c];
      if (d.x == 0.0 && d.y == 0.0) gs.flag = 1;
      g[c] = zdiv(acc, d);
    }
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(gs.flag) == 0;
}

// Frobenius norm of an N x 16 block (all threads get it).
__device__ double gm_norm(const zd* __restrict__ X, int N, GmresSmem& gs) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double s = 0.0;
  for (int q = tid; q < N * 16; q += kLuThreads) s += X[q].x * X[q].x + X[q].y * X[q].y;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) gs.red[wave] = s;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < kLuWaves; ++q) t += gs.red[q];
  __syncthreads();
  return sqrt(t);
}

// Block GMRES for one instance; returns true when converged (Y holds the
// solution) and the number of block Arnoldi steps taken in *steps.
// Block-diagonal right preconditioner over the LIZ sites: the block of site
// j approximates the site's diagonal block of A^{-1} = (M^{-1})^T; blk
// holds kk x kk column-major approximations D_j of [M^{-1}]_{jj} (for
// instance blocks of the network, [M^{-1}]_{00} of the instance centred on
// that site), row[j] the block of site j (< 0: identity).  blk null: none.
struct GmresPc {
  const zd* blk;
  const int32_t* row;  // this instance's LIZ rows
  int nliz;
};

// T = P^{-1} X (N x 16 row-major, internal rows): site j's rows (internal
// kk (j - 1) .. for j >= 1, the central rows Nd .. for j = 0) times D_j^T,
// T[r][c] = sum_a D_j[a][r] X[a][c].  Ends after a barrier.
__device__ void gm_precond(const GmresPc& pc, int Nd, const zd* __restrict__ X, zd* __restrict__ T) {
  for (int q = threadIdx.x; q < pc.nliz * 256; q += kLuThreads) {
    const int j = q >> 8, r = (q >> 4) & 15, c = q & 15;
    const int64_t base = j ? 16 * (int64_t)(j - 1) : (int64_t)Nd;
    const int pr = pc.row[j];
    zd acc;
    if (pr < 0) {
      acc = X[(base + r) * 16 + c];
    } else {
      const zd* D = pc.blk + (int64_t)pr * 256 + 16 * r;  // column r of D_j
      acc = zmake(0.0, 0.0);
#pragma unroll 4
      for (int a = 0; a < 16; ++a) acc = zfms(acc, zmake(-D[a].x, -D[a].y), X[(base + a) * 16 + c]);
    }
    T[(base + r) * 16 + c] = acc;
  }
  __syncthreads();
}

__device__ __noinline__ bool gmres_solve(const Mat<zd>& A, const GmresBufs& b, const double* seed, double tol,
                                         int max_cycles, unsigned char* smem, int* steps,
                                         const GmresPc pc = GmresPc{}) {
  GmresSmem& gs = *reinterpret_cast<GmresSmem*>(smem);
  const int tid = threadIdx.x;
  const int N = (int)A.N, Nd = A.Nd, m = b.m;
  const int ldh = 16 * (m + 1);
  // initial guess: the seed in the central rows, then one Jacobi step
  for (int q = tid; q < N * 16; q += kLuThreads) {
    const int v = q >> 4, c = q & 15;
    zd y = zmake(0.0, 0.0);
    if (seed && v >= Nd) y = reinterpret_cast<const zd*>(seed)[c + 16 * (v - Nd)];
    b.Y[q] = y;
  }
  __syncthreads();
  if (seed) {
    gm_amul(A, b.Y, b.R, true);
    for (int q = tid; q < Nd * 16; q += kLuThreads) b.Y[q] = zadd(b.Y[q], b.R[q]);
    __syncthreads();
  }
  const double enorm = 4.0;  // ||E_c||_F with 16 unit columns
  int it = 0;
  bool conv = false;
  for (int cycle = 0;; ++cycle) {
    gm_amul(A, b.Y, b.R, true);
    const double rn = gm_norm(b.R, N, gs);
    if (!(rn == rn)) break;
    if (rn <= tol * enorm) {
      conv = true;
      break;
    }
    if (cycle == max_cycles) break;
    // V_0 R_0 = R
    for (int q = tid; q < N * 16; q += kLuThreads) b.V[q] = b.R[q];
    __syncthreads();
    if (!gm_cholqr(b.V, N, gs)) break;
    for (int q = tid; q < ldh * 16; q += kLuThreads) {
      const int r = q % ldh, c = q / ldh;
      b.G[q] = r < 16 ? gs.r[r][c] : zmake(0.0, 0.0);
    }
    for (int q = tid; q < ldh * 16 * m; q += kLuThreads) b.H[q] = zmake(0.0, 0.0);
    __syncthreads();
    int jdone = 0;
    for (int j = 0; j < m; ++j) {
      zd* Vj = b.V + (int64_t)j * N * 16;
      zd* W = b.V + (int64_t)(j + 1) * N * 16;
      if (pc.blk) {  // W = A P^{-1} V_j, P^{-1} V_j in R (free during the cycle)
        gm_precond(pc, Nd, Vj, b.R);
        gm_amul(A, b.R, W, false);
      } else {
        gm_amul(A, Vj, W, false);
      }
      for (int pass = 0; pass < 2; ++pass) {
        gm_gram(b.V, j + 1, N, W, gs);
        for (int q = tid; q < (j + 1) * 256; q += kLuThreads) {
          const int r = q >> 4, c = q & 15;
          zd* hq = b.H + (int64_t)(16 * j + c) * ldh + r;
          *hq = zadd(*hq, gs.h[r][c]);
        }
        gm_subtract(b.V, j + 1, N, W, gs);
      }
      ++it;
      // a rank-deficient new block means the Krylov space is exhausted: its
      // part of H stays zero and the least-squares solution is exact
      const bool ok = gm_cholqr(W, N, gs);
      if (ok) {
        for (int q = tid; q < 256; q += kLuThreads) {
          const int r = q >> 4, c = q & 15;
          b.H[(int64_t)(16 * j + c) * ldh + 16 * (j + 1) + r] = gs.r[r][c];
        }
        __syncthreads();
      }
      const double est = gm_qr_block(b, ldh, j, gs);
      jdone = j + 1;
      if (!ok || est <= tol * enorm) break;
    }
    if (!gm_backsolve(b, ldh, 16 * jdone, gs)) break;
    // Y += P^{-1} [V_0 .. V_{jdone-1}] y (P^{-1} = 1 without preconditioner)
    for (int q = tid; q < N * 16; q += kLuThreads) {
      const int v = q >> 4, c = q & 15;
      zd acc = pc.blk ? zmake(0.0, 0.0) : b.Y[q];
      for (int i = 0; i < jdone; ++i) {
        const zd* vr = b.V + ((int64_t)i * N + v) * 16;
        const zd* g = b.G + (int64_t)c * ldh + 16 * i;
        for (int a = 0; a < 16; ++a) acc = zfms(acc, zmake(-vr[a].x, -vr[a].y), g[a]);
      }
      if (pc.blk) b.R[q] = acc;
      else b.Y[q] = acc;
    }
    __syncthreads();
    if (pc.blk) {
      gm_precond(pc, Nd, b.R, b.V);  // V_0 is free once y is applied
      for (int q = tid; q < N * 16; q += kLuThreads) b.Y[q] = zadd(b.Y[q], b.V[q]);
      __syncthreads();
    }
  }
  *steps = it;
  return conv;
}

int64_t gmres_extra_bytes(int64_t nmax, int m) {
  const int64_t blk = ((nmax * 16 * 16) + 255) & ~(int64_t)255;
  const int64_t h = (((int64_t)16 * (m + 1) * 16 * m * 16) + 255) & ~(int64_t)255;
  const int64_t g = (((int64_t)16 * (m + 1) * 16 * 16) + 255) & ~(int64_t)255;
  const int64_t q = (((int64_t)16 * m * 32 * 16) + 255) & ~(int64_t)255;
  const int64_t bt = (((int64_t)16 * m * 8) + 255) & ~(int64_t)255;
  return kXgBytes + blk * (2 + m + 1) + h + g + q + bt;
}

__device__ inline GmresBufs gmres_bufs(unsigned char* base, int64_t nmax, int m) {
  const int64_t blk = ((nmax * 16 * 16) + 255) & ~(int64_t)255;
  const int64_t h = (((int64_t)16 * (m + 1) * 16 * m * 16) + 255) & ~(int64_t)255;
  GmresBufs b;
  unsigned char* q = base + kXgBytes;
  b.Y = glb(reinterpret_cast<zd*>(q));
  b.R = glb(reinterpret_cast<zd*>(q + blk));
  b.V = glb(reinterpret_cast<zd*>(q + 2 * blk));
  b.H = glb(reinterpret_cast<zd*>(q + (3 + m) * blk));
  const int64_t g = (((int64_t)16 * (m + 1) * 16 * 16) + 255) & ~(int64_t)255;
  const int64_t qv = (((int64_t)16 * m * 32 * 16) + 255) & ~(int64_t)255;
  b.G = glb(reinterpret_cast<zd*>(q + (3 + m) * blk + h));
  b.Q = glb(reinterpret_cast<zd*>(q + (3 + m) * blk + h + g));
  b.beta = glb(reinterpret_cast<double*>(q + (3 + m) * blk + h + g + qv));
  b.m = m;
  return b;
}

size_t gmres_smem_bytes() {
  size_t b = sizeof(GmresSmem) > sizeof(LuSmemD) ? sizeof(GmresSmem) : sizeof(LuSmemD);
  return b > sizeof(BuildSmem) ? b : sizeof(BuildSmem);
}

// Persistent learned-form kernel: build each instance's M in the workgroup's
// slot ([M | X blocks | GMRES buffers]), run block GMRES from the seed
// (seed[i]: kk x kk complex column-major approximation of [M^{-1}]_{00}, or
// none), write tau00 = Y_c^T diag(t0); on failure the FP64 Schur path on the
// untouched M (info 512).  steps[i]: block Arnoldi steps taken.
template <int kR, int kWL>
__global__ __launch_bounds__(kThreads) void tau00_gmres_persistent_kernel(
    lsms_prob_dev p, lsms_gaunt_dev g, const int32_t* __restrict__ order, int n, int32_t* __restrict__ counter,
    unsigned char* __restrict__ work, int64_t slot_bytes, int64_t m_bytes, const double* __restrict__ seed,
    const double* __restrict__ pc_blk, const int32_t* __restrict__ pc_row, const int8_t* __restrict__ route,
    double* __restrict__ tau00, int32_t* __restrict__ info, int32_t* __restrict__ steps, int nb, double tol,
    int max_cycles, int m) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  BuildSmem& sb = *reinterpret_cast<BuildSmem*>(smem_raw);
  GmresSmem& gs = *reinterpret_cast<GmresSmem*>(smem_raw);
  __shared__ int next;
  unsigned char* base = work + (int64_t)blockIdx.x * slot_bytes;
  zd* M = reinterpret_cast<zd*>(base);
  zd* xg = reinterpret_cast<zd*>(base + m_bytes);
  const GmresBufs bufs = gmres_bufs(base + m_bytes, (int64_t)p.kc * p.max_liz, m);
  __syncthreads();
  int k = pop_instance(counter, &next);
  while (k < n) {
    const int inst = __builtin_amdgcn_readfirstlane(order ? order[k] : k);
    int status = __builtin_amdgcn_readfirstlane(instance_invalid<kR>(p, inst) ? -3 : 0);
    if (status == 0) {
      const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
      build_setup<kThreads>(p, g, inst, sb);
      for (int j = 0; j < nliz; ++j) build_column<kThreads>(p, inst, j, M, sb);
      status = __builtin_amdgcn_readfirstlane(sb.bad_species ? -3 : (sb.bad ? -2 : 0));
      __syncthreads();
    }
    if (status == 0) {
      const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
      Mat<zd> A;
      A.base = glb(M);
      A.N = (int64_t)p.kk * nliz;
      A.Nd = (int)A.N - p.kk;
      A.kk = p.kk;
      int nsteps = 0;
      GmresPc pc;
      pc.blk = reinterpret_cast<const zd*>(pc_blk);
      pc.row = pc_row ? pc_row + p.liz_off[inst] : nullptr;
      pc.nliz = nliz;
      if (!pc_row) pc.blk = nullptr;
      const bool direct = route && __builtin_amdgcn_readfirstlane((int)route[inst]) != 0;
      const bool conv = !direct && gmres_solve(A, bufs, seed ? seed + (int64_t)inst * 2 * 256 : nullptr, tol,
                                               max_cycles, smem_raw, &nsteps, pc);
      if (threadIdx.x == 0) steps[inst] = nsteps;
      if (__builtin_amdgcn_readfirstlane((int)conv)) {
        const int e = p.e_idx[inst];
        const zd kap = zsqrt(reinterpret_cast<const zd*>(p.energy)[e]);
        const int s0 = min(max(p.species[p.liz_off[inst]], 0), p.n_species - 1);
        const zd* dl = reinterpret_cast<const zd*>(p.delta) + ((int64_t)s0 * p.n_energy + e) * (p.lmax + 1);
        zd* tout = reinterpret_cast<zd*>(tau00) + (int64_t)inst * 256;
        if (threadIdx.x == 0) gs.flag = 0;
        __syncthreads();
        for (int q = threadIdx.x; q < 256; q += kThreads) {
          const int L = q % 16, Lp = q / 16;
          const zd v = zmul(bufs.Y[(int64_t)(A.Nd + Lp) * 16 + L], tmat_from_delta(dl[l_of(Lp)], kap));
          if (!zfinite(v)) gs.flag = 1;
          tout[q] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) info[inst] = gs.flag ? -1 : 0;
        __syncthreads();
      } else {
        lu_instance<kR, kWL>(p, inst, M, xg, tau00, info, nb, *reinterpret_cast<LuSmemD*>(smem_raw));
        if (threadIdx.x == 0 && info[inst] >= 0) info[inst] |= direct ? kInfoRouted : kInfoLuFallback;
        __syncthreads();
      }
    } else {
      fill_nan(p, inst, tau00);
      if (threadIdx.x == 0) {
        info[inst] = status;
        steps[inst] = 0;
      }
    }
    __syncthreads();
    k = pop_instance(counter, &next);
  }
}

// ======================================================================
// One instance across the whole GPU (paper Sec. 5: offloading the whole KKR
// inverse, whose ranks, 6225 to 12450 in Sec. 4.1, are too large for one
// compute unit to factorise quickly).  The same elimination as lu_instance
// (A = M^T, pivots among the non-central rows, the central block last, then
// Gauss-Jordan on the Schur block), split over many workgroups: per panel
// of 64 columns
//   big_panel_coop_kernel: ceil(rows / 128) workgroups factorise the panel
//     together, each holding 128 of its rows in LDS, with one grid barrier
//     per column for the pivot choice; it writes the pivots and the inverse
//     of the unit lower diagonal block;
//   big_u12_kernel: one workgroup per 64-column strip of the trailing
//     columns applies the panel's interchanges to the strip and forms
//     U12 = L11^{-1} A12 (stored in A);
//   big_gemm_kernel: one workgroup per (strip, block of rows) updates
//     A22 -= L21 U12 on MFMA.
// The host issues the launches on two streams with one panel of
// look-ahead: the next strip's update and the next panel run on the
// caller's stream while the rest of the trailing update runs on the second,
// started once the next strip's update is done.
// ======================================================================
constexpr int kBigRows = 512;    // trailing-update rows per workgroup (up to 4x while >= 1024 workgroups)
constexpr int kAheadRows = 128;  // rows per workgroup in the next panel's strip

struct BigView {
  Mat<zd> A;
  int N, Nd;
};

__device__ __forceinline__ BigView big_view(const lsms_prob_dev& p, double* Mb) {
  BigView v;
  v.N = p.kc * p.max_liz;
  v.Nd = v.N - p.kc;
  v.A.base = glb(reinterpret_cast<zd*>(Mb));
  v.A.N = v.N;
  v.A.Nd = v.Nd;
  v.A.kk = p.kc;
  return v;
}

// state[0] := 0, or -3 when the instance is not one of max_liz sites with a
// valid energy index (its rank would differ from the planned N); state[1]
// (a barrier wait gave up) := 0; the panels' arrival counters := 0; the
// pivots := the identity (a panel that gave up leaves them so).
__global__ void big_init_kernel(lsms_prob_dev p, int32_t* state, int32_t* counters, int np, int32_t* ipiv, int N) {
  for (int q = threadIdx.x; q < np; q += blockDim.x) counters[q] = 0;
  for (int q = threadIdx.x; q < N; q += blockDim.x) ipiv[q] = q;  // no interchange until a panel writes one
  if (threadIdx.x != 0) return;
  const int64_t nliz = p.liz_off[1] - p.liz_off[0];
  const int e = p.e_idx[0];
  state[0] = (nliz != p.max_liz || e < 0 || e >= p.n_energy) ? -3 : 0;
  state[1] = 0;
}

// Cooperative panel factorisation: P workgroups, workgroup b owning the panel
// rows [c + 128 b, c + 128 b + 128) (all panel columns) in LDS.  Per column:
// each workgroup finds its best pivot candidate (|Re| + |Im| among its rows
// in [c + j, plim), lowest row on ties) and publishes it with the
// candidate's row and, if it owns row c + j, that row; one grid barrier;
// every workgroup takes the same winner, swaps the two rows where it owns
// them and eliminates the column in its own rows.  The barrier counts
// arrivals on this panel's own counter (zeroed by big_init_kernel); a wait
// gives up after `spin` polls, setting state[1], and every workgroup then
// leaves (a later panel kernel leaves at once when state[1] is set).  After
// the last column the rows are written back and workgroup 0, which owns the
// diagonal block, inverts its unit lower part into xg.
constexpr int kCoopRows = 128;  // panel rows per workgroup
constexpr int kCoopMaxP = 128;  // workgroups of a panel (N <= 16384)

struct CoopSmem {
  zd blk[kCoopRows][kNB + 1];  // this workgroup's rows of the panel (row stride padded: rows start on different LDS banks)
  zd prow[kNB];            // the pivot row
  int stop;
  double winv;
};

struct CoopBufs {
  int32_t* counter;  // this panel's arrival counter
  double* candv;     // [2][kCoopMaxP]
  int32_t* candi;    // [2][kCoopMaxP]
  zd* candrow;       // [2][kCoopMaxP][kNB]
  zd* rowj;          // [2][kNB]
};

// Exchange between the workgroups of one panel: relaxed device-scope atomic
// loads and stores, which reach the level where all XCDs meet without a
// write-back or invalidation of this XCD's whole L2 (a device-scope fence
// costs both, twice per column).
__device__ __forceinline__ void st_dev(double* a, double x) {
  __hip_atomic_store(a, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int32_t* a, int32_t x) {
  __hip_atomic_store(a, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(double* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_dev(int32_t* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(zd* a, zd x) {
  st_dev(reinterpret_cast<double*>(a), x.x);
  st_dev(reinterpret_cast<double*>(a) + 1, x.y);
}
__device__ __forceinline__ zd ld_dev(zd* a) {
  return zmake(ld_dev(reinterpret_cast<double*>(a)), ld_dev(reinterpret_cast<double*>(a) + 1));
}

// Arrival of this workgroup at barrier `target` (all threads call it) and the
// wait for every workgroup; false (uniform) when the wait gave up.  Every
// thread's exchange stores are acknowledged (all memory counters drained)
// before thread 0 adds the arrival; then every thread runs `work` (bounded,
// no barrier inside) while the other workgroups arrive, and thread 0 waits.
template <typename F>
__device__ bool coop_barrier(int32_t* counter, int target, int64_t spin, int* stop, F&& work) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  work();
  if (threadIdx.x == 0) {
    int ok = 1;
    int64_t it = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++it >= spin) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *stop = !ok;
  }
  __syncthreads();
  return !__builtin_amdgcn_readfirstlane(*stop);
}

__global__ __launch_bounds__(kThreads) void big_panel_coop_kernel(lsms_prob_dev p, double* Mb, int c, int w,
                                                                  int32_t* __restrict__ ipiv,
                                                                  double* __restrict__ xg,
                                                                  int32_t* __restrict__ state, CoopBufs cb,
                                                                  int64_t spin) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  CoopSmem& cs = *reinterpret_cast<CoopSmem*>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) cs.stop = state[1];  // an earlier wait gave up: leave at once
  __syncthreads();
  if (__builtin_amdgcn_readfirstlane(cs.stop) != 0) return;
  const BigView v = big_view(p, Mb);
  const int N = v.N, plim = v.Nd;
  const int P = (int)gridDim.x, b = (int)blockIdx.x;
  const int row0 = c + kCoopRows * b;
  const int nr = max(0, min(kCoopRows, N - row0));
  for (int q = tid; q < kCoopRows * kNB; q += kThreads) {
    const int r = q / kNB, j = q % kNB;
    cs.blk[r][j] = (r < nr && j < w) ? *v.A.ptr(row0 + r, c + j) : zmake(0.0, 0.0);
  }
  __syncthreads();
  // Column j's elimination updates column j + 1 at once and the columns
  // > j + 1 during the next column's barrier (after this workgroup's arrival,
  // while the others arrive), so the rows published
  // for column j + 1 lack that update in the columns > j + 1: their readers
  // apply it (multiplier in the row's column j, column j's pivot row still
  // in cs.prow).  pend: such an update is outstanding.
  bool pend = false;
  for (int j = 0; j < w; ++j) {
    const int cj = c + j, buf = j & 1;
    // wave 0 finds this workgroup's candidate (lane q takes rows q and q + 64:
    // |Re| + |Im| among the rows in [cj, plim), lowest row on ties) and
    // publishes it: lane 0 the value and row index, lanes < w the candidate's
    // row and, in the owner of row cj, that row
    if (wave == 0) {
      double bb = -1.0;
      int ii = cj;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = lane + 64 * h, g = row0 + r;
        if (r < nr && g >= cj && g < plim) {
          const double x = zcabs1(cs.blk[r][j]);
          if (better(x, g, bb, ii)) {
            bb = x;
            ii = g;
          }
        }
      }
      wave_argmax(bb, ii);
      bb = __shfl(bb, 0);
      ii = __shfl(ii, 0);
      if (lane == 0) {
        st_dev(cb.candv + buf * kCoopMaxP + b, bb);
        st_dev(cb.candi + buf * kCoopMaxP + b, ii);
      }
      const int wr = min(max(ii - row0, 0), kCoopRows - 1);  // local row of the candidate (its values; any if none)
      if (lane < w) {
        st_dev(cb.candrow + ((int64_t)buf * kCoopMaxP + b) * kNB + lane, cs.blk[wr][lane]);
        if (cj >= row0 && cj < row0 + nr) st_dev(cb.rowj + buf * kNB + lane, cs.blk[cj - row0][lane]);
      }
    }
    // the barrier; once this workgroup has arrived, its threads apply column
    // j - 1's update to the columns > j of the rows below its pivot (four
    // threads per row, each every fourth column)
    const bool pj = pend;
    const bool ok = coop_barrier(cb.counter, P * (j + 1), spin, &cs.stop, [&]() {
      if (!pj) return;
      const int r = tid >> 2, part = tid & 3;
      if (r < nr && row0 + r >= cj) {
        const zd l = cs.blk[r][j - 1];
        for (int g = (j + 1) >> 4; g < ((w + 15) >> 4); ++g) {
          zd a[4], u[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int jj = 16 * g + 4 * m + part;
            a[m] = cs.blk[r][jj];
            u[m] = cs.prow[jj];
          }
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int jj = 16 * g + 4 * m + part;
            if (jj > j && jj < w) cs.blk[r][jj] = zfms(a[m], l, u[m]);
          }
        }
      }
    });
    if (!ok) {
      if (tid == 0) state[1] = 1;
      return;
    }
    // the winner, the same in every workgroup: wave 0 reads the P candidates
    // (lane q those of workgroups q and q + 64) and row cj at once, reduces
    // the candidates, takes lane 0's result, reads the winning row from its
    // owner (workgroup 0 owns row cj), brings both rows up to date and swaps
    // them where it owns them
    if (wave == 0) {
      zd rj = zmake(0.0, 0.0);
      if (lane < w) rj = ld_dev(cb.rowj + buf * kNB + lane);
      double bb = -1.0;
      int ii = 0x7fffffff;
      if (lane < P) {
        bb = ld_dev(cb.candv + buf * kCoopMaxP + lane);
        ii = ld_dev(cb.candi + buf * kCoopMaxP + lane);
      }
      if (lane + 64 < P) {
        const double ob = ld_dev(cb.candv + buf * kCoopMaxP + lane + 64);
        const int oi = ld_dev(cb.candi + buf * kCoopMaxP + lane + 64);
        if (better(ob, oi, bb, ii)) {
          bb = ob;
          ii = oi;
        }
      }
      wave_argmax(bb, ii);
      bb = __shfl(bb, 0);
      ii = __shfl(ii, 0);
      const bool zero = !(bb > 0.0);
      const int pr = zero ? cj : ii;
      if (lane == 0) {
        cs.winv = zero ? 0.0 : bb;
        if (zero && bb == 0.0 && b == 0 && state[0] == 0) state[0] = cj + 1;
        if (b == 0) ipiv[cj] = pr;
      }
      const int wb = min(max((pr - c) / kCoopRows, 0), P - 1);
      zd pv = zmake(0.0, 0.0);
      if (lane < w) pv = ld_dev(cb.candrow + ((int64_t)buf * kCoopMaxP + wb) * kNB + lane);
      if (pj) {
        // column j - 1's update of the columns > j, as the other rows had it
        const zd mp = zmake(__shfl(pv.x, j - 1), __shfl(pv.y, j - 1));
        const zd mr = zmake(__shfl(rj.x, j - 1), __shfl(rj.y, j - 1));
        if (lane > j && lane < w) {
          const zd pu = cs.prow[lane];
          pv = zfms(pv, mp, pu);
          rj = zfms(rj, mr, pu);
        }
      }
      if (lane < w) {
        cs.prow[lane] = pv;
        if (pr != cj) {
          if (pr >= row0 && pr < row0 + nr) cs.blk[pr - row0][lane] = rj;
          if (cj >= row0 && cj < row0 + nr) cs.blk[cj - row0][lane] = pv;
        }
      }
    }
    __syncthreads();
    // rows below the pivot: l = a_rj / pivot, a_rj := l, a_r(j+1) -= l prow(j+1)
    // (one thread per row); the columns > j + 1 follow in the next barrier
    pend = cs.winv > 0.0;
    if (pend) {
      const zd inv = zinv(cs.prow[j]);
      if (tid < nr && row0 + tid > cj) {
        const zd l = zmul(cs.blk[tid][j], inv);
        cs.blk[tid][j] = l;
        if (j + 1 < w) cs.blk[tid][j + 1] = zfms(cs.blk[tid][j + 1], l, cs.prow[j + 1]);
      }
    }
    __syncthreads();
  }
  for (int q = tid; q < nr * kNB; q += kThreads) {
    const int r = q / kNB, j = q % kNB;
    if (j < w) *v.A.ptr(row0 + r, c + j) = cs.blk[r][j];
  }
  __syncthreads();
  // the diagonal block (rows c .. c+w-1) is workgroup 0's own
  if (b == 0 && c + w < N) {
    LuSmemD& sh = *reinterpret_cast<LuSmemD*>(smem_raw);
    invert_unit_lower<double>(v.A, c, w, sh);
    save_x<double>(sh, reinterpret_cast<zd*>(xg));
  }
}

// Strips [s_begin + 64 b, ...) of the trailing columns, b = blockIdx.x.
__global__ __launch_bounds__(kThreads) void big_u12_kernel(lsms_prob_dev p, double* Mb, int c, int w,
                                                           const int32_t* __restrict__ ipiv,
                                                           const double* __restrict__ xg, int s_begin,
                                                           int s_end) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmemD& sh = *reinterpret_cast<LuSmemD*>(smem_raw);
  const BigView v = big_view(p, Mb);
  const int s0 = s_begin + kNB * blockIdx.x, sw = min(kNB, s_end - s0);
  if (threadIdx.x < w) {
    // a pivot row below the column and inside the matrix (anything else,
    // which only a panel that gave up could leave, means no interchange)
    const int r = c + threadIdx.x, pv = ipiv[r];
    sh.ipiv[threadIdx.x] = (pv >= r && pv < v.N) ? pv : r;
  }
  const zd* x = reinterpret_cast<const zd*>(xg);
  for (int q = threadIdx.x; q < kNB * kNB; q += kThreads) sh.X[q / kNB][q % kNB] = x[q];
  __syncthreads();
  apply_swaps<double>(v.A, c, w, s0, s0 + sw, sh);
  __syncthreads();
  trsm_strip<double>(v.A, c, w, s0, sw, true, sh);
}

// A22 -= L21 U12 for the strip s_begin + 64 blockIdx.x and the rows
// [c + w + rows blockIdx.y, + rows) (U12 read back from A into LDS).
// Panels wider than 32 columns take the MFMA row-block update with row
// bounds; narrower ones (only a ragged last panel) one workgroup per strip
// over all rows (launched with one row block).
__global__ __launch_bounds__(kThreads) void big_gemm_kernel(lsms_prob_dev p, double* Mb, int c, int w,
                                                            int s_begin, int s_end, int rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmemD& sh = *reinterpret_cast<LuSmemD*>(smem_raw);
  const BigView v = big_view(p, Mb);
  const int s0 = s_begin + kNB * blockIdx.x, sw = min(kNB, s_end - s0);
  const int vlo = c + w + rows * blockIdx.y, vhi = min(v.N, vlo + rows);
  if (vlo >= v.N) return;
  for (int q = threadIdx.x; q < kNB * kNB; q += kThreads) {
    const int k = q / kNB, j = q % kNB;
    sh.U[k][j] = (k < w && j < sw) ? *v.A.ptr(c + k, s0 + j) : zmake(0.0, 0.0);
  }
  __syncthreads();
  if (w <= 32) {
    update_strip<double>(v.A, c, w, s0, sw, sh.U);
  } else if (sw > 48) {
    update_rows<double, 4>(v.A, c, w, s0, sw, sh.U, vlo, vhi);
  } else if (sw > 32) {
    update_rows<double, 3>(v.A, c, w, s0, sw, sh.U, vlo, vhi);
  } else if (sw > 16) {
    update_rows<double, 2>(v.A, c, w, s0, sw, sh.U, vlo, vhi);
  } else {
    update_rows<double, 1>(v.A, c, w, s0, sw, sh.U, vlo, vhi);
  }
}

// Gauss-Jordan on the Schur block and tau00 (instance 0).
__global__ __launch_bounds__(kThreads) void big_finish_kernel(lsms_prob_dev p, double* Mb,
                                                              double* __restrict__ tau00,
                                                              int32_t* __restrict__ info,
                                                              const int32_t* __restrict__ state) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmemD& sh = *reinterpret_cast<LuSmemD*>(smem_raw);
  const int st = state[1] ? -4 : state[0];
  if (st < 0) {
    fill_nan(p, 0, tau00);
    if (threadIdx.x == 0) info[0] = st;
    return;
  }
  const BigView v = big_view(p, Mb);
  if (threadIdx.x == 0) {
    sh.info = st;
    sh.bad = 0;
  }
  __syncthreads();
  finish_instance(p, 0, v.A, RowOut{}, 0.0, 0.0, 0, tau00, info, sh);
}

template <int kR, int kWL>
hipError_t launch(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, const int64_t* m_off, int64_t slot,
                  double* xgb, int64_t xstride, double* tau00, int32_t* info, int keep_info, int32_t nb,
                  hipStream_t s) {
  const size_t smem = sizeof(LuSmemD);
  hipLaunchKernelGGL((lu_schur_fp64_kernel<kR, kWL>), dim3(n), dim3(kThreads), smem, s, p, i0, M, m_off, slot,
                     xgb, xstride, tau00, info, keep_info, nb);
  return hipGetLastError();
}

template <int kR, int kWL>
hipError_t launch_persistent(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order, int32_t n,
                             int32_t* counter, double* work, int64_t slot, int64_t xoff, int grid, double* tau00,
                             int32_t* info, int32_t nb, hipStream_t s) {
  const size_t smem = sizeof(LuSmemD) > sizeof(BuildSmem) ? sizeof(LuSmemD) : sizeof(BuildSmem);
  hipLaunchKernelGGL((tau00_persistent_kernel<kR, kWL>), dim3(grid), dim3(kThreads), smem, s, p, g, order, n,
                     counter, work, slot, xoff, tau00, info, nb);
  return hipGetLastError();
}

template <int kR, int kWL>
hipError_t launch_mixed(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, int64_t slot,
                        unsigned char* extra, int64_t xslot, double* tau00, int32_t* info, int32_t nb, double tol,
                        int32_t max_refine, hipStream_t s) {
  hipLaunchKernelGGL((tau00_mixed_kernel<kR, kWL>), dim3(n), dim3(kThreads), mixed_smem_bytes(), s, p, i0, M, slot,
                     extra, xslot, tau00, info, nb, tol, max_refine);
  return hipGetLastError();
}

template <int kR, int kWL>
hipError_t launch_mixed_persistent(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order,
                                   int32_t* counter, unsigned char* work, int64_t slot_bytes, int64_t m_bytes,
                                   int grid, double* tau00, int32_t* info, int32_t nb, double tol,
                                   int32_t max_refine, hipStream_t s) {
  hipLaunchKernelGGL((tau00_mixed_persistent_kernel<kR, kWL>), dim3(grid), dim3(kThreads), mixed_smem_bytes(), s,
                     p, g, order, p.n_inst, counter, work, slot_bytes, m_bytes, tau00, info, nb, tol, max_refine);
  return hipGetLastError();
}

template <int kR, int kWL>
hipError_t launch_gmres(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order, int32_t* counter,
                        unsigned char* work, int64_t slot_bytes, int64_t m_bytes, int grid, const double* seed,
                        const double* pc_blk, const int32_t* pc_row, const int8_t* route, double* tau00,
                        int32_t* info, int32_t* steps, int32_t nb, double tol, int max_cycles, int m,
                        hipStream_t s) {
  hipLaunchKernelGGL((tau00_gmres_persistent_kernel<kR, kWL>), dim3(grid), dim3(kThreads), gmres_smem_bytes(), s, p,
                     g, order, p.n_inst, counter, work, slot_bytes, m_bytes, seed, pc_blk, pc_row, route, tau00,
                     info, steps, nb, tol, max_cycles, m);
  return hipGetLastError();
}

// Instances ordered by LIZ size, largest first (counting sort, one workgroup).
__global__ __launch_bounds__(1024) void lpt_order_kernel(const int64_t* __restrict__ liz_off, int n, int max_liz,
                                                         int32_t* __restrict__ order) {
  __shared__ int start[1026];
  for (int b = threadIdx.x; b < 1026; b += 1024) start[b] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 1024) {
    const int key = min(max((int)(liz_off[i + 1] - liz_off[i]), 0), max_liz);
    atomicAdd(&start[key], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int b = max_liz; b >= 0; --b) {
      const int c = start[b];
      start[b] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 1024) {
    const int key = min(max((int)(liz_off[i + 1] - liz_off[i]), 0), max_liz);
    order[atomicAdd(&start[key], 1)] = i;
  }
}

}  // namespace

// Leaf rows per thread kR bounds N <= 512 kR: kR = 5 covers N <= 2560 (leaves
// 8 columns wide), kR = 8 covers N <= 4096 (4 wide) and, for the FP64 path
// only, kR = 16 covers N <= 8192 (2 wide: the spin-canted ranks 4320 and 6750).
hipError_t lsms_launch_lu_fp64(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, const int64_t* m_off,
                               int64_t slot, double* xgb, int64_t xstride, double* tau00, int32_t* info,
                               int keep_info, int32_t nb, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  if (nmax <= kThreads * 5)
    return launch<5, 8>(p, i0, n, M, m_off, slot, xgb, xstride, tau00, info, keep_info, nb, s);
  if (nmax <= kThreads * 8)
    return launch<8, 4>(p, i0, n, M, m_off, slot, xgb, xstride, tau00, info, keep_info, nb, s);
  return launch<16, 2>(p, i0, n, M, m_off, slot, xgb, xstride, tau00, info, keep_info, nb, s);
}

int64_t lsms_row_slot_bytes(const lsms_prob_dev& p) { return row_slot_bytes((int64_t)p.kc * p.max_liz, p.kk); }

hipError_t lsms_launch_tau_row(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, const int64_t* m_off,
                               unsigned char* work, const int64_t* row_off, double* row, double* logdet,
                               double* tau00, int32_t* info, int32_t nb, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  const int64_t wslot = row_slot_bytes(nmax, p.kk);
  const size_t smem = sizeof(LuSmemD);
  if (nmax <= kThreads * 5)
    hipLaunchKernelGGL((tau_row_fp64_kernel<5, 8>), dim3(n), dim3(kThreads), smem, s, p, i0, M, m_off, work, wslot,
                       row_off, row, logdet, tau00, info, nb);
  else
    hipLaunchKernelGGL((tau_row_fp64_kernel<8, 4>), dim3(n), dim3(kThreads), smem, s, p, i0, M, m_off, work, wslot,
                       row_off, row, logdet, tau00, info, nb);
  return hipGetLastError();
}

hipError_t lsms_launch_lpt_order(const lsms_prob_dev& p, int32_t* order, hipStream_t s) {
  if (p.n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(lpt_order_kernel, dim3(1), dim3(1024), 0, s, p.liz_off, p.n_inst,
                     p.max_liz < 1024 ? p.max_liz : 1024, order);
  return hipGetLastError();
}

// Resident workgroups of the persistent kernel on `device` (one per CU when
// its LDS use allows one).
hipError_t lsms_persistent_grid(const lsms_prob_dev& p, int device, int* grid) {
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  const size_t smem = sizeof(LuSmemD) > sizeof(BuildSmem) ? sizeof(LuSmemD) : sizeof(BuildSmem);
  int per_cu = 0;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  if (nmax <= kThreads * 5)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_persistent_kernel<5, 8>, kThreads, smem);
  else if (nmax <= kThreads * 8)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_persistent_kernel<8, 4>, kThreads, smem);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_persistent_kernel<16, 2>, kThreads, smem);
  if (e != hipSuccess) return e;
  *grid = cus * (per_cu > 0 ? per_cu : 1);
  return hipSuccess;
}

hipError_t lsms_launch_persistent(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order,
                                  int32_t* counter, double* work, int64_t slot, int64_t xoff, int grid,
                                  double* tau00, int32_t* info, int32_t nb, hipStream_t s) {
  if (p.n_inst <= 0) return hipSuccess;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  if (nmax <= kThreads * 5)
    return launch_persistent<5, 8>(p, g, order, p.n_inst, counter, work, slot, xoff, grid, tau00, info, nb, s);
  if (nmax <= kThreads * 8)
    return launch_persistent<8, 4>(p, g, order, p.n_inst, counter, work, slot, xoff, grid, tau00, info, nb, s);
  return launch_persistent<16, 2>(p, g, order, p.n_inst, counter, work, slot, xoff, grid, tau00, info, nb, s);
}

// Dynamic LDS limits of every elimination kernel; called once per device
// (at handle creation) so that no attribute call happens inside a capture.
hipError_t lsms_prepare_kernels() {
  const int gsm = (int)gmres_smem_bytes();
  {
    const hipFuncAttribute at = hipFuncAttributeMaxDynamicSharedMemorySize;
    hipError_t eg;
    if ((eg = hipFuncSetAttribute((const void*)tau00_gmres_persistent_kernel<5, 8>, at, gsm)) != hipSuccess) return eg;
    if ((eg = hipFuncSetAttribute((const void*)tau00_gmres_persistent_kernel<8, 4>, at, gsm)) != hipSuccess) return eg;
  }
  const int a = (int)sizeof(LuSmemD);
  const int b = (int)(sizeof(LuSmemD) > sizeof(BuildSmem) ? sizeof(LuSmemD) : sizeof(BuildSmem));
  const int m = (int)mixed_smem_bytes();
  const hipFuncAttribute attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)tau00_mixed_kernel<5, 8>, attr, m)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)tau00_mixed_kernel<8, 4>, attr, m)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)tau00_mixed_persistent_kernel<5, 8>, attr, m)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)tau00_mixed_persistent_kernel<8, 4>, attr, m)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)lu_schur_fp64_kernel<5, 8>, attr, a)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)lu_schur_fp64_kernel<8, 4>, attr, a)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)tau_row_fp64_kernel<5, 8>, attr, a)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)tau_row_fp64_kernel<8, 4>, attr, a)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)lu_schur_fp64_kernel<16, 2>, attr, a)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)tau00_persistent_kernel<5, 8>, attr, b)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)tau00_persistent_kernel<16, 2>, attr, b)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)tau00_persistent_kernel<8, 4>, attr, b);
}

int64_t lsms_mixed_extra_bytes(const lsms_prob_dev& p) {
  return mixed_extra_bytes((int64_t)p.kc * p.max_liz, p.kk > 16 ? 32 : 16);
}

hipError_t lsms_launch_mixed(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, int64_t slot,
                             unsigned char* extra, int64_t xslot, double* tau00, int32_t* info, int32_t nb, double tol,
                             int32_t max_refine, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  if (nmax <= kThreads * 5)
    return launch_mixed<5, 8>(p, i0, n, M, slot, extra, xslot, tau00, info, nb, tol, max_refine, s);
  return launch_mixed<8, 4>(p, i0, n, M, slot, extra, xslot, tau00, info, nb, tol, max_refine, s);
}

hipError_t lsms_mixed_persistent_grid(const lsms_prob_dev& p, int device, int* grid) {
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  if (nmax <= kThreads * 5)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_mixed_persistent_kernel<5, 8>, kThreads,
                                                     mixed_smem_bytes());
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_mixed_persistent_kernel<8, 4>, kThreads,
                                                     mixed_smem_bytes());
  if (e != hipSuccess) return e;
  *grid = cus * (per_cu > 0 ? per_cu : 1);
  return hipSuccess;
}

hipError_t lsms_launch_mixed_persistent(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order,
                                        int32_t* counter, unsigned char* work, int64_t slot_bytes, int64_t m_bytes,
                                        int grid, double* tau00, int32_t* info, int32_t nb, double tol,
                                        int32_t max_refine, hipStream_t s) {
  if (p.n_inst <= 0) return hipSuccess;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  if (nmax <= kThreads * 5)
    return launch_mixed_persistent<5, 8>(p, g, order, counter, work, slot_bytes, m_bytes, grid, tau00, info, nb, tol,
                                         max_refine, s);
  return launch_mixed_persistent<8, 4>(p, g, order, counter, work, slot_bytes, m_bytes, grid, tau00, info, nb, tol,
                                       max_refine, s);
}

int64_t lsms_gmres_extra_bytes(const lsms_prob_dev& p, int m) { return gmres_extra_bytes((int64_t)p.kc * p.max_liz, m); }

int lsms_gmres_max_restart() { return kGmMaxM; }

hipError_t lsms_gmres_grid(const lsms_prob_dev& p, int device, int* grid) {
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  if (nmax <= kThreads * 5)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_gmres_persistent_kernel<5, 8>, kThreads,
                                                     gmres_smem_bytes());
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_gmres_persistent_kernel<8, 4>, kThreads,
                                                     gmres_smem_bytes());
  if (e != hipSuccess) return e;
  *grid = cus * (per_cu > 0 ? per_cu : 1);
  return hipSuccess;
}

hipError_t lsms_launch_gmres(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order, int32_t* counter,
                             unsigned char* work, int64_t slot_bytes, int64_t m_bytes, int grid, const double* seed,
                             const double* pc_blk, const int32_t* pc_row, const int8_t* route, double* tau00,
                             int32_t* info, int32_t* steps, int32_t nb, double tol, int max_cycles, int m,
                             hipStream_t s) {
  if (p.n_inst <= 0) return hipSuccess;
  const int64_t nmax = (int64_t)p.kc * p.max_liz;
  if (nmax <= kThreads * 5)
    return launch_gmres<5, 8>(p, g, order, counter, work, slot_bytes, m_bytes, grid, seed, pc_blk, pc_row, route,
                              tau00, info, steps, nb, tol, max_cycles, m, s);
  return launch_gmres<8, 4>(p, g, order, counter, work, slot_bytes, m_bytes, grid, seed, pc_blk, pc_row, route,
                            tau00, info, steps, nb, tol, max_cycles, m, s);
}

namespace {
// row[r] = index of the block of LIZ row r: inst_of[atom[r] * n_energy + e]
// for the energy index e of the instance owning the row (-1 when absent).
// One workgroup per instance.
__global__ __launch_bounds__(256) void site_blocks_kernel(lsms_prob_dev p, const int32_t* __restrict__ liz_atom,
                                                          int32_t n_atoms, const int32_t* __restrict__ inst_of,
                                                          int32_t* __restrict__ row) {
  const int i = blockIdx.x;
  const int64_t a = p.liz_off[i], b = p.liz_off[i + 1];
  const int e = p.e_idx[i];
  for (int64_t r = a + threadIdx.x; r < b; r += 256) {
    const int at = liz_atom[r];
    row[r] = (at >= 0 && at < n_atoms && e >= 0 && e < p.n_energy) ? inst_of[(int64_t)at * p.n_energy + e] : -1;
  }
}

// inst_of[q] = -1 for q < n, then inst_of[centre[i] * n_energy + e_idx[i]] = i.
__global__ __launch_bounds__(256) void inst_of_clear_kernel(int32_t* __restrict__ inst_of, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) inst_of[q] = -1;
}
__global__ __launch_bounds__(256) void inst_of_fill_kernel(lsms_prob_dev p, const int32_t* __restrict__ centre,
                                                           int32_t n_atoms, int32_t* __restrict__ inst_of) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= p.n_inst) return;
  const int c = centre[i], e = p.e_idx[i];
  if (c >= 0 && c < n_atoms && e >= 0 && e < p.n_energy) inst_of[(int64_t)c * p.n_energy + e] = i;
}
}  // namespace

hipError_t lsms_launch_site_blocks(const lsms_prob_dev& p, const int32_t* liz_atom, const int32_t* centre,
                                   int32_t n_atoms, int32_t* row, int32_t* inst_of, hipStream_t s) {
  if (p.n_inst <= 0) return hipSuccess;
  const int64_t n = (int64_t)n_atoms * p.n_energy;
  const unsigned gb = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(inst_of_clear_kernel, dim3(gb), dim3(256), 0, s, inst_of, n);
  hipLaunchKernelGGL(inst_of_fill_kernel, dim3((p.n_inst + 255) / 256), dim3(256), 0, s, p, centre, n_atoms, inst_of);
  hipLaunchKernelGGL(site_blocks_kernel, dim3(p.n_inst), dim3(256), 0, s, p, liz_atom, n_atoms, inst_of, row);
  return hipGetLastError();
}

// One instance across the whole GPU: workspace layout [state | ipiv | two
// 64 x 64 blocks | panel counters | pivot candidates, their rows, row j],
// each part 256-byte aligned; see lsms_big_work_bytes.
namespace {
struct BigLayout {
  int64_t ipiv, xg, counters, candv, candi, candrow, rowj, total;
};
BigLayout big_layout(const lsms_prob_dev& p) {
  const int64_t N = (int64_t)p.kc * p.max_liz;
  const int64_t np = (N - p.kc + kNB - 1) / kNB;
  auto al = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
  BigLayout L;
  L.ipiv = 256;
  L.xg = L.ipiv + al(N * 4);
  L.counters = L.xg + 2 * kNB * kNB * 16;
  L.candv = L.counters + al(np * 4);
  L.candi = L.candv + al(2 * kCoopMaxP * 8);
  L.candrow = L.candi + al(2 * kCoopMaxP * 4);
  L.rowj = L.candrow + al(2 * (int64_t)kCoopMaxP * kNB * 16);
  L.total = L.rowj + al(2 * kNB * 16);
  return L;
}
size_t coop_smem() { return sizeof(CoopSmem) > sizeof(LuSmemD) ? sizeof(CoopSmem) : sizeof(LuSmemD); }
}  // namespace

int64_t lsms_big_work_bytes(const lsms_prob_dev& p) { return big_layout(p).total; }

int lsms_big_events(const lsms_prob_dev& p) {
  const int Nd = p.kc * p.max_liz - p.kc;
  return 2 * ((Nd + kNB - 1) / kNB);
}

hipError_t lsms_launch_big(const lsms_prob_dev& p, double* M, unsigned char* work, double* tau00, int32_t* info,
                           int32_t nb, int64_t spin, hipStream_t s0, hipStream_t s1, hipEvent_t* ev) {
  (void)nb;  // panels are 64 wide
  const int N = p.kc * p.max_liz, Nd = N - p.kc;
  if ((N + kCoopRows - 1) / kCoopRows > kCoopMaxP) return hipErrorInvalidValue;  // more panel rows than workgroups
  const int np = (Nd + kNB - 1) / kNB;
  const BigLayout L = big_layout(p);
  int32_t* state = reinterpret_cast<int32_t*>(work);
  int32_t* ipiv = reinterpret_cast<int32_t*>(work + L.ipiv);
  double* xg = reinterpret_cast<double*>(work + L.xg);
  int32_t* counters = reinterpret_cast<int32_t*>(work + L.counters);
  const size_t smem = sizeof(LuSmemD);
  auto xgk = [&](int k) { return xg + (size_t)(k & 1) * kNB * kNB * 2; };
  auto panel = [&](int k, hipStream_t s) {
    const int c = kNB * k, w = min(kNB, Nd - c);
    CoopBufs cb;
    cb.counter = counters + k;
    cb.candv = reinterpret_cast<double*>(work + L.candv);
    cb.candi = reinterpret_cast<int32_t*>(work + L.candi);
    cb.candrow = reinterpret_cast<zd*>(work + L.candrow);
    cb.rowj = reinterpret_cast<zd*>(work + L.rowj);
    const unsigned P = (unsigned)((N - c + kCoopRows - 1) / kCoopRows);
    hipLaunchKernelGGL(big_panel_coop_kernel, dim3(P), dim3(kThreads), coop_smem(), s, p, M, c, w, ipiv, xgk(k),
                       state, cb, spin);
  };
  // the update by panel k of the columns [a, b).  The next panel's strip
  // (`ahead`, on the path to the next panel) spreads its rows over many small
  // workgroups; the rest gives each workgroup up to 2048 rows (fewer U12
  // loads and pipeline starts) while keeping at least 1024 workgroups.
  auto update = [&](int k, int a, int b, hipStream_t s, bool ahead) {
    if (a >= b) return;
    const int c = kNB * k, w = min(kNB, Nd - c);
    const unsigned ns = (unsigned)((b - a + kNB - 1) / kNB);
    hipLaunchKernelGGL(big_u12_kernel, dim3(ns), dim3(kThreads), smem, s, p, M, c, w, ipiv, xgk(k), a, b);
    const int below = N - (c + w);
    int rows = ahead ? kAheadRows : kBigRows;
    while (!ahead && rows < 4 * kBigRows && (int64_t)ns * ((below + 2 * rows - 1) / (2 * rows)) >= 1024) rows *= 2;
    const unsigned nr = w <= 32 ? 1u : (unsigned)((below + rows - 1) / rows);
    if (below > 0)
      hipLaunchKernelGGL(big_gemm_kernel, dim3(ns, nr), dim3(kThreads), smem, s, p, M, c, w, a, b, rows);
  };
  hipLaunchKernelGGL(big_init_kernel, dim3(1), dim3(256), 0, s0, p, state, counters, np, ipiv, N);
  panel(0, s0);
  for (int k = 0; k < np; ++k) {
    const int next = kNB * (k + 1);  // first column of panel k + 1 (Nd after the last)
    const int rest = k + 1 < np ? min(next + kNB, Nd) : Nd;
    // the next panel's columns first, alone on the device (on the path to
    // the next panel); the rest of the update then starts beside that panel
    if (k + 1 < np) update(k, next, rest, s0, true);
    hipError_t e = hipEventRecord(ev[2 * k], s0);
    if (e != hipSuccess) return e;
    if (k + 1 < np) panel(k + 1, s0);
    if ((e = hipStreamWaitEvent(s1, ev[2 * k], 0)) != hipSuccess) return e;
    update(k, rest, N, s1, false);  // every other trailing column, beside the next panel
    if ((e = hipEventRecord(ev[2 * k + 1], s1)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s0, ev[2 * k + 1], 0)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(big_finish_kernel, dim3(1), dim3(kThreads), smem, s0, p, M, tau00, info, state);
  return hipGetLastError();
}

// Workgroups of the cooperative panel kernel that `device` can hold at once
// (resident per compute unit, with its LDS and registers, times the compute
// units): a panel's grid must not exceed it, so that every workgroup of a
// grid barrier can be resident together.
int lsms_big_panel_groups(const lsms_prob_dev& p) {
  return (p.kc * p.max_liz + kCoopRows - 1) / kCoopRows;
}

hipError_t lsms_big_resident(int device, int* n) {
  int per_cu = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)big_panel_coop_kernel, kThreads,
                                                             coop_smem());
  if (e != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess) return e;
  *n = per_cu * cus;
  return hipSuccess;
}

hipError_t lsms_prepare_big_kernels() {
  const int a = (int)sizeof(LuSmemD);
  const hipFuncAttribute attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)big_panel_coop_kernel, attr, (int)coop_smem())) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)big_u12_kernel, attr, a)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)big_gemm_kernel, attr, a)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)big_finish_kernel, attr, a);
}
