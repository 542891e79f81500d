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
// One workgroup (4 waves) per instance.  Per panel of w <= 64 columns:
//   1. panel factorisation, column by column (pivot search by wave shuffles
//      and an LDS reduction, pivot row staged in LDS, rank-1 update);
//   2. the panel's row interchanges applied to the trailing columns;
//   3. X = L11^{-1} (unit lower, w x w) into LDS;
//   4. per strip of 64 trailing columns: U12 = X A12 (MFMA) into LDS, then
//      A22 -= L21 U12 (complex GEMM on v_mfma_f64_16x16x4f64; complex
//      products as four real MFMAs on separate real/imaginary accumulators).
// Finally S_A is inverted by Gauss-Jordan with partial pivoting.
#include "lsms_common.h"

using namespace lsms;

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kNB = 64;   // maximum panel width
constexpr int kSW = 64;   // trailing-update strip width (columns)
constexpr int kMaxKK = 25;

struct LuSmem {
  zd X[kNB][kNB];    // L11^{-1}
  zd U[kNB][kSW];    // U12 strip; L11 staging; Gauss-Jordan workspace at the end
  zd prow[kNB];
  zd tz[kMaxKK];
  double redv[kThreads / 64];
  int redi[kThreads / 64];
  int ipiv[kNB];
  int info;
  int bad;
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

// ------------------------------------------------------------ panel
__device__ void panel_factor(const Mat& A, int c, int w, LuSmem& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = (int)A.N, Nd = A.Nd;
  for (int jj = 0; jj < w; ++jj) {
    const int j = c + jj;
    // pivot search over the non-central rows j..Nd-1 of column j
    double best = -1.0;
    int bi = j;
    for (int v = j + tid; v < Nd; v += kThreads) {
      const double a = zcabs1(*A.ptr(v, j));
      if (a > best) {
        best = a;
        bi = v;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) {
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
    for (int q = 1; q < kThreads / 64; ++q) {
      const double ob = sh.redv[q];
      const int oi = sh.redi[q];
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const bool zero = (best == 0.0);
    if (zero) bi = j;
    // swap rows j and bi inside the panel, stage the pivot row
    if (tid < w) {
      zd* pj = A.ptr(j, c + tid);
      zd vj = *pj;
      if (bi != j) {
        zd* pb = A.ptr(bi, c + tid);
        const zd vb = *pb;
        *pb = vj;
        *pj = vb;
        vj = vb;
      }
      sh.prow[tid] = vj;
    }
    if (tid == 0) {
      sh.ipiv[jj] = bi;
      if (zero && sh.info == 0) sh.info = j + 1;
    }
    __syncthreads();
    if (!zero) {
      const zd inv = zinv(sh.prow[jj]);
      const int k = lane;
      const int g = wave;
      const bool upd = (k > jj) && (k < w);
      const zd pk = upd ? sh.prow[k] : zmake(0.0, 0.0);
      int v = j + 1 + g;
      for (; v + 12 < N; v += 16) {
        zd a[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = *A.ptr(v + 4 * u, j);
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = upd ? *A.ptr(v + 4 * u, c + k) : zmake(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const zd l = zmul(a[u], inv);
          if (k == jj) *A.ptr(v + 4 * u, j) = l;
          else if (upd) *A.ptr(v + 4 * u, c + k) = zfms(x[u], l, pk);
        }
      }
      for (; v < N; v += 4) {
        const zd a = *A.ptr(v, j);
        const zd l = zmul(a, inv);
        if (k == jj) *A.ptr(v, j) = l;
        else if (upd) {
          zd* p = A.ptr(v, c + k);
          *p = zfms(*p, l, pk);
        }
      }
    }
    __syncthreads();
  }
}

// Row interchanges of the panel applied to the columns [c0, N).  Each thread
// owns whole columns, so the interchanges are applied in order per thread.
__device__ void apply_swaps(const Mat& A, int c, int w, int c0, const LuSmem& sh) {
  const int N = (int)A.N;
  for (int jj = 0; jj < w; ++jj) {
    const int p = sh.ipiv[jj], r = c + jj;
    if (p == r) continue;
    zd* rr = A.base + A.phys(r) * A.N;
    zd* rp = A.base + A.phys(p) * A.N;
    for (int u = c0 + threadIdx.x; u < N; u += kThreads) {
      const int64_t pu = A.phys(u);
      const zd a = rr[pu], b = rp[pu];
      rr[pu] = b;
      rp[pu] = a;
    }
  }
}

// X = L11^{-1} (unit lower triangular), from L11 staged in sh.U; zero outside w.
__device__ void invert_l11(int w, LuSmem& sh) {
  const int j = threadIdx.x;
  if (j < kNB) {
    for (int i = 0; i < kNB; ++i) {
      zd x;
      if (j >= w || i >= w || i < j) {
        x = zmake(0.0, 0.0);
      } else if (i == j) {
        x = zmake(1.0, 0.0);
      } else {
        double sr = 0.0, si = 0.0;
        for (int k = j; k < i; ++k) {
          const zd l = sh.U[i][k];
          const zd xk = sh.X[k][j];
          sr += l.x * xk.x - l.y * xk.y;
          si += l.x * xk.y + l.y * xk.x;
        }
        x = zmake(-sr, -si);
      }
      sh.X[i][j] = x;
    }
  }
}

// U12 strip = X * A(c .. c+w-1, s0 .. s0+sw-1) into sh.U (rows >= w are zero).
__device__ void trsm_strip(const Mat& A, int c, int w, int s0, int sw, LuSmem& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  d4 ar[4], ai[4];
#pragma unroll
  for (int cs = 0; cs < 4; ++cs) {
    ar[cs] = d4{0.0, 0.0, 0.0, 0.0};
    ai[cs] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const int row = 16 * wave + li;
  for (int kb = 0; kb < w; kb += 4) {
    const int k = kb + lk;
    const zd x = sh.X[row][k < kNB ? k : 0];
    const double xr = (k < w) ? x.x : 0.0;
    const double xi = (k < w) ? x.y : 0.0;
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) {
      const int col = 16 * cs + li;
      zd b = zmake(0.0, 0.0);
      if (k < w && col < sw) b = *A.ptr(c + k, s0 + col);
      ar[cs] = mfma(xr, b.x, ar[cs]);
      ar[cs] = mfma(-xi, b.y, ar[cs]);
      ai[cs] = mfma(xr, b.y, ai[cs]);
      ai[cs] = mfma(xi, b.x, ai[cs]);
    }
  }
  __syncthreads();  // the previous strip's update has finished reading sh.U
#pragma unroll
  for (int cs = 0; cs < 4; ++cs)
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.U[16 * wave + 4 * r + lk][16 * cs + li] = zmake(ar[cs][r], ai[cs][r]);
  __syncthreads();
}

// A(v, s0 + j) -= sum_k A(v, c + k) U[k][j] for v in [c + w, N), j < sw.
// Wave rows: blocks of 32 rows (two 16-row MFMA tiles) x 64 columns (four
// tiles).  The k dimension is taken in groups of 16: lane (i, q) loads the
// four consecutive elements A(v_i, c + kb + 4q .. 4q+3) and MFMA step s uses
// k = kb + 4q + s, with the matching B fragment U[kb + 4q + s][j].
__device__ void update_strip(const Mat& A, int c, int w, int s0, int sw, const LuSmem& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int N = (int)A.N;
  const int r0 = c + w;
  for (int rb = r0 + 32 * wave; rb < N; rb += 32 * (kThreads / 64)) {
    d4 accr[2][4], acci[2][4];
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int cs = 0; cs < 4; ++cs) {
        accr[rs][cs] = d4{0.0, 0.0, 0.0, 0.0};
        acci[rs][cs] = d4{0.0, 0.0, 0.0, 0.0};
      }
    const zd* arow[2];
    bool rok[2];
#pragma unroll
    for (int rs = 0; rs < 2; ++rs) {
      const int v = rb + 16 * rs + li;
      rok[rs] = v < N;
      arow[rs] = A.base + A.phys(rok[rs] ? v : r0) * A.N + A.phys(c);
    }
    for (int kb = 0; kb < w; kb += 16) {
      zd a[2][4];
#pragma unroll
      for (int rs = 0; rs < 2; ++rs)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = kb + 4 * lq + s;
          a[rs][s] = (rok[rs] && k < w) ? arow[rs][k] : zmake(0.0, 0.0);
        }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kb + 4 * lq + s;
        zd b[4];
#pragma unroll
        for (int cs = 0; cs < 4; ++cs) b[cs] = sh.U[k][16 * cs + li];
#pragma unroll
        for (int rs = 0; rs < 2; ++rs) {
          const double xr = a[rs][s].x, xi = a[rs][s].y;
#pragma unroll
          for (int cs = 0; cs < 4; ++cs) {
            accr[rs][cs] = mfma(xr, b[cs].x, accr[rs][cs]);
            accr[rs][cs] = mfma(-xi, b[cs].y, accr[rs][cs]);
            acci[rs][cs] = mfma(xr, b[cs].y, acci[rs][cs]);
            acci[rs][cs] = mfma(xi, b[cs].x, acci[rs][cs]);
          }
        }
      }
    }
    // C -= acc ; register r of lane (li, lq) holds row 4*r + lq, column li of each 16 x 16 tile
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = rb + 16 * rs + 4 * r + lq;
        if (v >= N) continue;
        zd* crow = A.base + A.phys(v) * A.N;
#pragma unroll
        for (int cs = 0; cs < 4; ++cs) {
          const int col = 16 * cs + li;
          if (col < sw) {
            zd* p = crow + A.phys(s0 + col);
            const zd cv = *p;
            *p = zmake(cv.x - accr[rs][cs][r], cv.y - acci[rs][cs][r]);
          }
        }
      }
  }
}

__global__ __launch_bounds__(kThreads) void lu_schur_fp64_kernel(lsms_prob_dev p, int i0, double* __restrict__ Mb,
                                                                const int64_t* __restrict__ m_off, int64_t slot,
                                                                double* __restrict__ tau00,
                                                                int32_t* __restrict__ info, int keep_info,
                                                                int nb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LuSmem& sh = *reinterpret_cast<LuSmem*>(smem_raw);
  const int inst = i0 + blockIdx.x;
  const int tid = threadIdx.x;
  const int kk = p.kk;
  const int nliz = (int)(p.liz_off[inst + 1] - p.liz_off[inst]);
  const int N = kk * nliz, Nd = N - kk;
  zd* tout = reinterpret_cast<zd*>(tau00) + (int64_t)inst * kk * kk;
  const int e_chk = p.e_idx[inst];
  const bool invalid = nliz < 1 || nliz > p.max_liz || e_chk < 0 || e_chk >= p.n_energy;
  if ((keep_info && info[inst] != 0) || invalid) {
    for (int q = tid; q < kk * kk; q += kThreads) tout[q] = zmake(NAN, NAN);
    if (invalid && tid == 0) info[inst] = -3;
    return;
  }
  Mat A;
  A.base = reinterpret_cast<zd*>(Mb) + (m_off ? m_off[inst] : (int64_t)(inst - i0) * slot);
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
    panel_factor(A, c, w, sh);
    apply_swaps(A, c, w, c + w, sh);
    // stage L11 (strict lower part is used)
    for (int q = tid; q < kNB * kNB; q += kThreads) {
      const int i = q / kNB, k = q % kNB;
      sh.U[i][k] = (i < w && k < i) ? *A.ptr(c + i, c + k) : zmake(0.0, 0.0);
    }
    __syncthreads();
    invert_l11(w, sh);
    __syncthreads();
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
      sh.redi[0] = pr;
    }
    __syncthreads();
    const int pr = sh.redi[0];
    if (pr != k && tid < 2 * kk) {
      const zd t = G[k][tid];
      G[k][tid] = G[pr][tid];
      G[pr][tid] = t;
    }
    __syncthreads();
    if (tid == 0) sh.prow[0] = zinv(G[k][k]);
    __syncthreads();
    if (tid < 2 * kk) G[k][tid] = zmul(G[k][tid], sh.prow[0]);
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
}

}  // namespace

hipError_t lsms_launch_lu_fp64(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, const int64_t* m_off,
                               int64_t slot, double* tau00, int32_t* info, int keep_info, int32_t nb,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t smem = sizeof(LuSmem);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)lu_schur_fp64_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(lu_schur_fp64_kernel, dim3(n), dim3(kThreads), smem, s, p, i0, M, m_off, slot, tau00, info,
                     keep_info, nb);
  return hipGetLastError();
}
