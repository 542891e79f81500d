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
// One workgroup (8 waves, two per SIMD) per instance.  Per panel of w <= 64
// columns:
//   1. recursive panel factorisation: leaves of kWL columns are factorised
//      with the leaf held in registers (each thread owns rows lc + t + 512 q),
//      pivot search by wave shuffles and an 8-entry LDS reduction, row
//      exchange through LDS; after each leaf the completed block of the
//      recursion updates its sibling block (triangular solve and product on
//      MFMA);
//   2. the panel's row interchanges applied to the trailing columns;
//   3. X = L11^{-1} (unit lower, w x w) into LDS;
//   4. per strip of 64 trailing columns: U12 = X A12 (MFMA) into LDS, then
//      A22 -= L21 U12 (complex GEMM on v_mfma_f64_16x16x4f64; a complex
//      product is four real MFMAs on separate real/imaginary accumulators).
// Finally S_A is inverted by Gauss-Jordan with partial pivoting.
#include "kkr_device.h"
#include "lsms_common.h"

using namespace lsms;

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kNB = 64;   // maximum panel width
constexpr int kSW = 64;   // trailing-update strip width (columns)
constexpr int kMaxKK = 25;
constexpr int kMaxWL = 8;

struct LuSmem {
  zd X[kNB][kNB];    // inverse of a unit lower triangular block
  zd U[kNB][kSW];    // U12 strip; L staging; Gauss-Jordan workspace at the end
  zd rowP[kMaxWL];   // pivot row of a leaf step
  zd rowJ[kMaxWL];
  zd tz[kMaxKK];
  zd pinv;
  double redv[kWaves];
  int redi[kWaves];
  int ipiv[kNB];
  int info;
  int bad;
  int gj_piv;
};

struct Mat {
  zd* base;
  int64_t N;
  int Nd, kk;
  __device__ __forceinline__ int64_t phys(int v) const { return v < Nd ? (int64_t)v + kk : (int64_t)(v - Nd); }
  __device__ __forceinline__ zd* ptr(int r, int c) const { return base + phys(r) * N + phys(c); }
};

// v_mfma_f64_16x16x4f64, D = A B + C with A 16x4, B 4x16: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; register r of lane l holds
// D[4 r + l / 16][l % 16].
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bool better(double ob, int oi, double b, int i) {
  return ob > b || (ob == b && oi < i);
}

// ------------------------------------------------------------ leaf
// Factorises the leaf columns [lc, lc + kWL) of the panel [c, c + w), rows
// [lc, N), with the leaf in registers.  Interchanges are applied at once to
// the other panel columns in memory.
// Kept out of line (with invert_unit_lower and apply_swaps) so that the
// register allocator treats the panel phase and the trailing update apart.
template <int kR, int kWL>
__device__ __noinline__ void leaf_factor(const Mat& A, int c, int w, int lc, LuSmem& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = (int)A.N, Nd = A.Nd;
  const int wl = min(kWL, c + w - lc);
  zd a[kR][kWL];
#pragma unroll
  for (int q = 0; q < kR; ++q) {
    const int v = lc + tid + kThreads * q;
    if (v < N) {
      const zd* row = A.ptr(v, lc);
#pragma unroll
      for (int k = 0; k < kWL; ++k) a[q][k] = (k < wl) ? row[k] : zmake(0.0, 0.0);
    } else {
#pragma unroll
      for (int k = 0; k < kWL; ++k) a[q][k] = zmake(0.0, 0.0);
    }
  }
  for (int jj = 0; jj < wl; ++jj) {
    const int j = lc + jj;
    double best = -1.0;
    int bi = j;
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      const int v = lc + tid + kThreads * q;
      if (v >= j && v < Nd) {
        double x = 0.0;
#pragma unroll
        for (int k = 0; k < kWL; ++k)
          if (k == jj) x = zcabs1(a[q][k]);
        if (x > best || (x == best && v < bi)) {
          best = x;
          bi = v;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (better(ob, oi, best, bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      sh.redv[wave] = best;
      sh.redi[wave] = bi;
    }
    __syncthreads();
    best = sh.redv[0];
    bi = sh.redi[0];
#pragma unroll
    for (int q = 1; q < kWaves; ++q)
      if (better(sh.redv[q], sh.redi[q], best, bi)) {
        best = sh.redv[q];
        bi = sh.redi[q];
      }
    const bool zero = !(best > 0.0);
    if (zero) bi = j;
    // owners of rows j and bi publish them
    const int oj = j - lc, ob = bi - lc;
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      if (oj == tid + kThreads * q) {
#pragma unroll
        for (int k = 0; k < kWL; ++k) sh.rowJ[k] = a[q][k];
      }
      if (ob == tid + kThreads * q) {
#pragma unroll
        for (int k = 0; k < kWL; ++k) sh.rowP[k] = a[q][k];
      }
    }
    // interchange the rows in the panel columns outside the leaf
    if (bi != j && tid < w) {
      const int col = c + tid;
      if (col < lc || col >= lc + wl) {
        zd* pj = A.ptr(j, col);
        zd* pb = A.ptr(bi, col);
        const zd x = *pj, y = *pb;
        *pj = y;
        *pb = x;
      }
    }
    if (tid == 0) {
      sh.ipiv[j - c] = bi;
      if (zero && best == 0.0 && sh.info == 0) sh.info = j + 1;
    }
    __syncthreads();
    if (bi != j) {
#pragma unroll
      for (int q = 0; q < kR; ++q) {
        if (oj == tid + kThreads * q) {
#pragma unroll
          for (int k = 0; k < kWL; ++k) a[q][k] = sh.rowP[k];
        }
        if (ob == tid + kThreads * q) {
#pragma unroll
          for (int k = 0; k < kWL; ++k) a[q][k] = sh.rowJ[k];
        }
      }
    }
    if (!zero) {
      zd piv = zmake(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < kWL; ++k)
        if (k == jj) piv = sh.rowP[k];
      const zd inv = zinv(piv);
#pragma unroll
      for (int q = 0; q < kR; ++q) {
        const int v = lc + tid + kThreads * q;
        if (v > j && v < N) {
          zd l = zmake(0.0, 0.0);
#pragma unroll
          for (int k = 0; k < kWL; ++k)
            if (k == jj) l = zmul(a[q][k], inv);
#pragma unroll
          for (int k = 0; k < kWL; ++k) {
            if (k == jj) a[q][k] = l;
            else if (k > jj) a[q][k] = zfms(a[q][k], l, sh.rowP[k]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kR; ++q) {
    const int v = lc + tid + kThreads * q;
    if (v < N) {
      zd* row = A.ptr(v, lc);
#pragma unroll
      for (int k = 0; k < kWL; ++k)
        if (k < wl) row[k] = a[q][k];
    }
  }
  __syncthreads();
}

// X = inverse of the unit lower triangular s x s block of A at (r0, r0),
// staged first in sh.U; zero outside [0, s)^2.  Eight lanes per column: lane
// p of a column accumulates the terms k = p (mod 8) of each row's dot product.
__device__ __noinline__ void invert_unit_lower(const Mat& A, int r0, int s, LuSmem& sh) {
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += kThreads) {
    const int i = q / kNB, k = q % kNB;
    sh.U[i][k] = (i < s && k < i) ? *A.ptr(r0 + i, r0 + k) : zmake(0.0, 0.0);
  }
  __syncthreads();
  const int j = tid >> 3, p = tid & 7;  // column j (0..63), part p
  zd xr[kNB / 8];
#pragma unroll
  for (int m = 0; m < kNB / 8; ++m) xr[m] = zmake(0.0, 0.0);
  if (j < s) {
#pragma unroll
    for (int m = 0; m < kNB / 8; ++m)
      if (p + 8 * m == j) xr[m] = zmake(1.0, 0.0);
    for (int i = j + 1; i < s; ++i) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int m = 0; m < kNB / 8; ++m) {
        const int k = p + 8 * m;
        if (k >= j && k < i) {
          const zd l = sh.U[i][k];
          sr += l.x * xr[m].x - l.y * xr[m].y;
          si += l.x * xr[m].y + l.y * xr[m].x;
        }
      }
      sr += __shfl_xor(sr, 1);
      si += __shfl_xor(si, 1);
      sr += __shfl_xor(sr, 2);
      si += __shfl_xor(si, 2);
      sr += __shfl_xor(sr, 4);
      si += __shfl_xor(si, 4);
#pragma unroll
      for (int m = 0; m < kNB / 8; ++m)
        if (p + 8 * m == i) xr[m] = zmake(-sr, -si);
    }
  }
#pragma unroll
  for (int m = 0; m < kNB / 8; ++m) sh.X[p + 8 * m][j] = xr[m];
  __syncthreads();
}

// U = X * A(r0 .. r0+s-1, s0 .. s0+sw-1) into sh.U rows 0..63 (rows >= s are
// zero).  Sixteen 16x16 output tiles, two per wave.
__device__ void trsm_strip(const Mat& A, int r0, int s, int s0, int sw, LuSmem& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rt = wave & 3;            // row tile
  const int ct0 = 2 * (wave >> 2);    // first of two column tiles
  d4 ar[2], ai[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    ar[t] = d4{0.0, 0.0, 0.0, 0.0};
    ai[t] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const int row = 16 * rt + li;
  const int kend = min(s, 16 * rt + 16);  // X is lower triangular
  for (int kb = 0; kb < kend; kb += 4) {
    const int k = kb + lk;
    const zd x = sh.X[row][k];
    const double xr = (k < s) ? x.x : 0.0;
    const double xi = (k < s) ? x.y : 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int col = 16 * (ct0 + t) + li;
      zd b = zmake(0.0, 0.0);
      if (k < s && col < sw) b = *A.ptr(r0 + k, s0 + col);
      ar[t] = mfma(xr, b.x, ar[t]);
      ar[t] = mfma(-xi, b.y, ar[t]);
      ai[t] = mfma(xr, b.y, ai[t]);
      ai[t] = mfma(xi, b.x, ai[t]);
    }
  }
  __syncthreads();  // earlier readers of sh.U are done
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.U[16 * rt + 4 * r + lk][16 * (ct0 + t) + li] = zmake(ar[t][r], ai[t][r]);
  __syncthreads();
}

// A(v, s0 + j) -= sum_{k < s} A(v, r0 + k) U[k][j] for v in [r0 + s, N),
// j < sw.  Each wave owns blocks of 16 rows x 64 columns (four MFMA tiles);
// MFMA step kb uses k = kb + lane/16.
__device__ void update_strip(const Mat& A, int r0, int s, int s0, int sw, const LuSmem& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int N = (int)A.N;
  const int rstart = r0 + s;
  const int ncs = (sw + 15) >> 4;
  for (int rb = rstart + 16 * wave; rb < N; rb += 16 * kWaves) {
    d4 accr[4], acci[4];
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) {
      accr[cs] = d4{0.0, 0.0, 0.0, 0.0};
      acci[cs] = d4{0.0, 0.0, 0.0, 0.0};
    }
    const int va = rb + li;
    const bool rok = va < N;
    const zd* arow = A.base + A.phys(rok ? va : rstart) * A.N + A.phys(r0);
#pragma unroll 4
    for (int kb = 0; kb < s; kb += 4) {
      const int k = kb + lq;
      const zd a = (rok && k < s) ? arow[k] : zmake(0.0, 0.0);
      zd b[4];
#pragma unroll
      for (int cs = 0; cs < 4; ++cs) b[cs] = sh.U[k & (kNB - 1)][16 * cs + li];
#pragma unroll
      for (int cs = 0; cs < 4; ++cs) {
        if (cs < ncs) {
          accr[cs] = mfma(a.x, b[cs].x, accr[cs]);
          accr[cs] = mfma(-a.y, b[cs].y, accr[cs]);
          acci[cs] = mfma(a.x, b[cs].y, acci[cs]);
          acci[cs] = mfma(a.y, b[cs].x, acci[cs]);
        }
      }
    }
    // C -= acc ; register r of lane (li, lq) holds row 4*r + lq, column li of each tile
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = rb + 4 * r + lq;
      if (v >= N) continue;
      zd* crow = A.base + A.phys(v) * A.N;
#pragma unroll
      for (int cs = 0; cs < 4; ++cs) {
        const int col = 16 * cs + li;
        if (col < sw) {
          zd* p = crow + A.phys(s0 + col);
          const zd cv = *p;
          *p = zmake(cv.x - accr[cs][r], cv.y - acci[cs][r]);
        }
      }
    }
  }
}

// Row interchanges of the panel applied to the columns [c0, N).  Each thread
// owns whole columns, so the interchanges are applied in order per thread.
__device__ __noinline__ void apply_swaps(const Mat& A, int c, int w, int c0, const LuSmem& sh) {
  const int N = (int)A.N;
  for (int jj = 0; jj < w; ++jj) {
    const int p = sh.ipiv[jj], r = c + jj;
    if (p == r) continue;
    zd* rr = A.base + A.phys(r) * A.N;
    zd* rp = A.base + A.phys(p) * A.N;
    for (int u = c0 + threadIdx.x; u < N; u += kThreads) {
      const int64_t pu = A.phys(u);
      const zd x = rr[pu], y = rp[pu];
      rr[pu] = y;
      rp[pu] = x;
    }
  }
}

template <int kR, int kWL>
__device__ void panel_factor(const Mat& A, int c, int w, LuSmem& sh) {
  const int nleaf = (w + kWL - 1) / kWL;
  for (int i = 0; i < nleaf; ++i) {
    const int lc = c + kWL * i;
    leaf_factor<kR, kWL>(A, c, w, lc, sh);
    // the completed block of the recursion updates its sibling block
    const int s = kWL << __builtin_ctz(i + 1);
    const int start = lc + kWL - s;
    const int t0 = lc + kWL;
    const int tw = min(s, c + w - t0);
    if (tw > 0) {
      invert_unit_lower(A, start, s, sh);
      trsm_strip(A, start, s, t0, tw, sh);
      update_strip(A, start, s, t0, tw, sh);
      __syncthreads();
    }
  }
}

// Eliminates one instance whose matrix is at `base` and writes its tau00 and
// info.  All threads of the workgroup call it; it ends after a barrier.
template <int kR, int kWL>
__device__ void lu_instance(const lsms_prob_dev& p, int inst, zd* base, double* __restrict__ tau00,
                            int32_t* __restrict__ info, int nb, LuSmem& sh) {
  const int tid = threadIdx.x;
  const int kk = p.kk;
  const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
  const int N = kk * nliz, Nd = N - kk;
  zd* tout = reinterpret_cast<zd*>(tau00) + (int64_t)inst * kk * kk;
  Mat A;
  A.base = base;
  A.N = N;
  A.Nd = Nd;
  A.kk = kk;
  if (tid == 0) {
    sh.info = 0;
    sh.bad = 0;
  }
  __syncthreads();

  for (int c = 0; c < Nd; c += nb) {
    const int w = min(nb, Nd - c);
    panel_factor<kR, kWL>(A, c, w, sh);
    apply_swaps(A, c, w, c + w, sh);
    __syncthreads();
    invert_unit_lower(A, c, w, sh);
    for (int s0 = c + w; s0 < N; s0 += kSW) {
      const int sw = min(kSW, N - s0);
      trsm_strip(A, c, w, s0, sw, sh);
      update_strip(A, c, w, s0, sw, sh);
    }
    __syncthreads();
  }

  // Gauss-Jordan inverse of S_A (kk x kk, physical rows/cols 0..kk-1) in sh.U
  zd(*G)[2 * kMaxKK] = reinterpret_cast<zd(*)[2 * kMaxKK]>(&sh.U[0][0]);
  for (int q = tid; q < kk * 2 * kk; q += kThreads) {
    const int r = q / (2 * kk), col = q % (2 * kk);
    G[r][col] = col < kk ? A.base[(int64_t)r * N + col] : zmake(col - kk == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < kk; ++k) {
    if (tid == 0) {
      int pr = k;
      double best = zcabs1(G[k][k]);
      for (int r = k + 1; r < kk; ++r) {
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
    if (pr != k && tid < 2 * kk) {
      const zd t = G[k][tid];
      G[k][tid] = G[pr][tid];
      G[pr][tid] = t;
    }
    __syncthreads();
    if (tid == 0) sh.pinv = zinv(G[k][k]);
    __syncthreads();
    if (tid < 2 * kk) G[k][tid] = zmul(G[k][tid], sh.pinv);
    if (tid < kk) sh.tz[tid] = G[tid][k];  // elimination factors (row k unused)
    __syncthreads();
    for (int q = tid; q < kk * 2 * kk; q += kThreads) {
      const int r = q / (2 * kk), col = q % (2 * kk);
      if (r != k) G[r][col] = zfms(G[r][col], sh.tz[r], G[k][col]);
    }
    __syncthreads();
  }
  // tau00(L, L') = [M^{-1}]_{00}(L, L') t0_{l(L')} = S_A^{-1}(L', L) t0_{l(L')}
  const int e = p.e_idx[inst];
  const zd kap = zsqrt(reinterpret_cast<const zd*>(p.energy)[e]);
  const int s0 = min(max(p.species[p.liz_off[inst]], 0), p.n_species - 1);
  const zd* dl = reinterpret_cast<const zd*>(p.delta) + ((int64_t)s0 * p.n_energy + e) * (p.lmax + 1);
  const int info0 = sh.info;
  for (int q = tid; q < kk * kk; q += kThreads) {
    const int L = q % kk, Lp = q / kk;
    zd v = zmul(G[Lp][kk + L], tmat_from_delta(dl[l_of(Lp)], kap));
    if (info0 != 0) v = zmake(NAN, NAN);
    if (!zfinite(v)) sh.bad = 1;
    tout[q] = v;
  }
  __syncthreads();
  if (tid == 0) info[inst] = info0 != 0 ? info0 : (sh.bad ? -1 : 0);
  __syncthreads();
}

// True when the instance cannot be processed (empty LIZ, LIZ above max_liz,
// energy index out of range, matrix too large for the leaf registers).
template <int kR>
__device__ __forceinline__ bool instance_invalid(const lsms_prob_dev& p, int inst) {
  const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
  const int e = p.e_idx[inst];
  return nliz < 1 || nliz > p.max_liz || e < 0 || e >= p.n_energy || p.kk * nliz > kThreads * kR;
}

__device__ __forceinline__ void fill_nan(const lsms_prob_dev& p, int inst, double* tau00) {
  zd* tout = reinterpret_cast<zd*>(tau00) + (int64_t)inst * p.kk * p.kk;
  for (int q = threadIdx.x; q < p.kk * p.kk; q += kThreads) tout[q] = zmake(NAN, NAN);
}

template <int kR, int kWL>
__global__ __launch_bounds__(kThreads) void lu_schur_fp64_kernel(lsms_prob_dev p, int i0, double* __restrict__ Mb,
                                                                const int64_t* __restrict__ m_off, int64_t slot,
                                                                double* __restrict__ tau00,
                                                                int32_t* __restrict__ info, int keep_info,
                                                                int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmem& sh = *reinterpret_cast<LuSmem*>(smem_raw);
  const int inst = i0 + blockIdx.x;
  const bool invalid = instance_invalid<kR>(p, inst);
  if ((keep_info && info[inst] != 0) || invalid) {
    fill_nan(p, inst, tau00);
    if (invalid && threadIdx.x == 0) info[inst] = -3;
    return;
  }
  zd* base = reinterpret_cast<zd*>(Mb) + (m_off ? m_off[inst] : (int64_t)(inst - i0) * slot);
  lu_instance<kR, kWL>(p, inst, base, tau00, info, nb, sh);
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
                                                                   double* __restrict__ tau00,
                                                                   int32_t* __restrict__ info, int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmem& sh = *reinterpret_cast<LuSmem*>(smem_raw);
  BuildSmem& sb = *reinterpret_cast<BuildSmem*>(smem_raw);  // used before sh, never at the same time
  __shared__ int next;
  zd* M = reinterpret_cast<zd*>(work) + (int64_t)blockIdx.x * slot;
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
      lu_instance<kR, kWL>(p, inst, M, tau00, info, nb, sh);
    } else {
      fill_nan(p, inst, tau00);
      if (threadIdx.x == 0) info[inst] = status;
    }
    __syncthreads();
    k = pop_instance(counter, &next);
  }
}

template <int kR, int kWL>
hipError_t launch(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, const int64_t* m_off, int64_t slot,
                  double* tau00, int32_t* info, int keep_info, int32_t nb, hipStream_t s) {
  const size_t smem = sizeof(LuSmem);
  hipLaunchKernelGGL((lu_schur_fp64_kernel<kR, kWL>), dim3(n), dim3(kThreads), smem, s, p, i0, M, m_off, slot,
                     tau00, info, keep_info, nb);
  return hipGetLastError();
}

template <int kR, int kWL>
hipError_t launch_persistent(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order, int32_t n,
                             int32_t* counter, double* work, int64_t slot, int grid, double* tau00, int32_t* info,
                             int32_t nb, hipStream_t s) {
  const size_t smem = sizeof(LuSmem) > sizeof(BuildSmem) ? sizeof(LuSmem) : sizeof(BuildSmem);
  hipLaunchKernelGGL((tau00_persistent_kernel<kR, kWL>), dim3(grid), dim3(kThreads), smem, s, p, g, order, n,
                     counter, work, slot, tau00, info, nb);
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

// Leaf rows per thread kR bounds N <= 512 kR: kR = 5 covers N <= 2560 and
// kR = 8 covers N <= 4096; leaves are 4 columns wide.
hipError_t lsms_launch_lu_fp64(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, const int64_t* m_off,
                               int64_t slot, double* tau00, int32_t* info, int keep_info, int32_t nb,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nmax = (int64_t)p.kk * p.max_liz;
  if (nmax <= kThreads * 5) return launch<5, 4>(p, i0, n, M, m_off, slot, tau00, info, keep_info, nb, s);
  return launch<8, 4>(p, i0, n, M, m_off, slot, tau00, info, keep_info, nb, s);
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
  const size_t smem = sizeof(LuSmem) > sizeof(BuildSmem) ? sizeof(LuSmem) : sizeof(BuildSmem);
  int per_cu = 0;
  const int64_t nmax = (int64_t)p.kk * p.max_liz;
  if (nmax <= kThreads * 5)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_persistent_kernel<5, 4>, kThreads, smem);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tau00_persistent_kernel<8, 4>, kThreads, smem);
  if (e != hipSuccess) return e;
  *grid = cus * (per_cu > 0 ? per_cu : 1);
  return hipSuccess;
}

hipError_t lsms_launch_persistent(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order,
                                  int32_t* counter, double* work, int64_t slot, int grid, double* tau00,
                                  int32_t* info, int32_t nb, hipStream_t s) {
  if (p.n_inst <= 0) return hipSuccess;
  const int64_t nmax = (int64_t)p.kk * p.max_liz;
  if (nmax <= kThreads * 5)
    return launch_persistent<5, 4>(p, g, order, p.n_inst, counter, work, slot, grid, tau00, info, nb, s);
  return launch_persistent<8, 4>(p, g, order, p.n_inst, counter, work, slot, grid, tau00, info, nb, s);
}

// Dynamic LDS limits of every elimination kernel; called once per device
// (at handle creation) so that no attribute call happens inside a capture.
hipError_t lsms_prepare_kernels() {
  const int a = (int)sizeof(LuSmem);
  const int b = (int)(sizeof(LuSmem) > sizeof(BuildSmem) ? sizeof(LuSmem) : sizeof(BuildSmem));
  const hipFuncAttribute attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)lu_schur_fp64_kernel<5, 4>, attr, a)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)lu_schur_fp64_kernel<8, 4>, attr, a)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)tau00_persistent_kernel<5, 4>, attr, b)) != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)tau00_persistent_kernel<8, 4>, attr, b);
}
