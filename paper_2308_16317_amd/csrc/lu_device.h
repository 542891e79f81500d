// Building blocks of the blocked complex LU used by the tau00 kernels, generic
// over the real type R (double for the plain path, float for the
// factorisation of the precision form).  All of them are called by every
// thread of a 512-thread workgroup that owns one matrix.
//
// Matrix view.  The column-major M buffer is read as the row-major storage of
// A = M^T; the internal index v runs over the non-central rows first and the
// central block last: physical row/column phys(v) = v + kk for v < Nd = N - kk
// and v - Nd for the central block.  Row interchanges of A are contiguous
// moves and every operand of the trailing update is read in row segments.
//
// Pivoting is row partial pivoting restricted to rows below a limit `plim`
// (Nd while the non-central columns are eliminated; N for the central block
// of a full factorisation), the pivot being the row that maximises
// |Re| + |Im|, the lowest such row on ties.
#pragma once

#include "lsms_common.h"

namespace lsms {

constexpr int kLuThreads = 512;
constexpr int kLuWaves = kLuThreads / 64;
constexpr int kNB = 64;         // triangular blocks and LDS tiles
constexpr int kSW = 64;         // trailing-update strip width in FP64 (columns)
constexpr int kPanelMax = 128;  // maximum panel width (two triangular blocks)

// Strip width of the trailing update: 64 columns in FP64; 128 in FP32, whose
// 128-row U12 strip of 128 columns takes the LDS of FP64's 64, and whose
// update, bound by HBM traffic, then re-reads L21 half as often.
template <typename R>
constexpr int kSWp = sizeof(R) == 4 ? 128 : kSW;
constexpr int kMaxKK = 25;
constexpr int kMaxKC = 2 * kMaxKK;  // rows per LIZ site with spin canting
constexpr int kMaxWL = 8;

template <typename R>
struct Prec;

// v_mfma_f64_16x16x4f64, D = A B + C with A 16x4, B 4x16: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; register r of lane l holds
// D[4 r + l / 16][l % 16] (measured on gfx950).
template <>
struct Prec<double> {
  typedef double2 C;
  typedef double V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 mfma(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int r, int lq) { return 4 * r + lq; }
};

// v_mfma_f32_16x16x4f32: same operand layout; register r of lane l holds
// D[4 (l / 16) + r][l % 16] (measured on gfx950).
template <>
struct Prec<float> {
  typedef float2 C;
  typedef float V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 mfma(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int r, int lq) { return 4 * lq + r; }
};

template <typename R>
struct LuSmem {
  typedef typename Prec<R>::C C;
  C X[kNB][kSWp<R>];  // inverse of a triangular block (columns < 64)
  C U[kNB][kSWp<R>];  // U12 strip; block staging; Gauss-Jordan workspace at the end
                    // (X and U together: the 128-row U12 strip of a wide panel)
  C cand[2][kLuWaves][kMaxWL];  // each wave's pivot candidate row (two buffers)
  R candv[2][kLuWaves];         // its magnitude |Re| + |Im|
  int candi[2][kLuWaves];       // its row
  zd tz[kMaxKC];
  zd pinv;
  int ipiv[kPanelMax];
  int lrow[2 * kMaxWL];  // rows touched by a leaf's interchanges
  int lsrc[2 * kMaxWL];  // lrow[q] receives the old content of lrow[lsrc[q]]
  int lcnt;
  int info;
  int bad;
  int gj_piv;
  double red[2][kLuWaves];  // per-wave partial sums of a workgroup reduction
  int redi[kLuWaves];
};

// Pointers into the matrix reach the kernels as generic pointers; the hot
// loops cast them to the global address space so that they compile to
// global (not flat) memory instructions, whose completion is tracked apart
// from LDS accesses (a flat load also counts as an LDS access, so every LDS
// wait would also wait for the loads issued ahead).
// The qualifiers exist only in the device pass; the host pass sees plain
// pointers.
#ifdef __HIP_DEVICE_COMPILE__
#define LSMS_GLOBAL __attribute__((address_space(1)))
#define LSMS_LDS __attribute__((address_space(3)))
#else
#define LSMS_GLOBAL
#define LSMS_LDS
#endif

template <typename T>
__device__ __forceinline__ LSMS_GLOBAL T* glb(T* p) {
  return (LSMS_GLOBAL T*)p;
}

// Non-temporal access to entries of the trailing block, which an update
// reads and writes once, so that they do not displace the L21 panel that
// every strip re-reads.
template <typename C>
__device__ __forceinline__ C ntload(const LSMS_GLOBAL C* p) {
  C v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  return v;
}
template <typename C>
__device__ __forceinline__ void ntstore(LSMS_GLOBAL C* p, C v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

template <typename C>
struct Mat {
  LSMS_GLOBAL C* base;  // global memory (see glb above)
  int64_t N;
  int Nd, kk;
  __device__ __forceinline__ int64_t phys(int v) const { return v < Nd ? (int64_t)v + kk : (int64_t)(v - Nd); }
  __device__ __forceinline__ LSMS_GLOBAL C* ptr(int r, int c) const {
    return base + phys(r) * N + phys(c);
  }
};

// The 128 x kSWp view of sh.X and sh.U (contiguous), holding the U12 strip
// of a panel wider than kNB.
template <typename R>
__device__ __forceinline__ typename Prec<R>::C (*ustrip2(LuSmem<R>& sh))[kSWp<R>] {
  static_assert(sizeof(sh.X) == kNB * kSWp<R> * sizeof(typename Prec<R>::C), "X rows must match U rows");
  return reinterpret_cast<typename Prec<R>::C(*)[kSWp<R>]>(&sh.X[0][0]);
}

template <typename R>
__device__ __forceinline__ bool better(R ob, int oi, R b, int i) {
  return ob > b || (ob == b && oi < i);
}

// Lane exchanges inside rows of 16 lanes by DPP (a VALU operand modifier, no
// LDS round trip).  Each control pairs every lane with one other lane:
// quad_perm [1,0,3,2] with lane ^ 1, quad_perm [2,3,0,1] with lane ^ 2,
// row_half_mirror with 7 - i inside each group of 8, row_mirror with 15 - i
// inside each row of 16.  Applied in this order to a reduction, each pairs a
// lane with one from the half not yet combined with it.
enum : int { kDppX1 = 0xB1, kDppX2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };

template <int kCtrl>
__device__ __forceinline__ int dpp_int(int x) {
  return __builtin_amdgcn_update_dpp(x, x, kCtrl, 0xF, 0xF, false);
}
template <int kCtrl>
__device__ __forceinline__ double dpp_val(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)dpp_int<kCtrl>((int)(unsigned)u);
  const unsigned hi = (unsigned)dpp_int<kCtrl>((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int kCtrl>
__device__ __forceinline__ float dpp_val(float x) {
  return __int_as_float(dpp_int<kCtrl>(__float_as_int(x)));
}

template <int kCtrl, typename R>
__device__ __forceinline__ void argmax_dpp(R& best, int& bi) {
  const R ob = dpp_val<kCtrl>(best);
  const int oi = dpp_int<kCtrl>(bi);
  if (better(ob, oi, best, bi)) {
    best = ob;
    bi = oi;
  }
}

// Sum over each aligned group of 8 lanes, by DPP (xor 1, xor 2, then the
// mirror inside the group of 8), the same value in all 8 lanes (the two
// operands of every addition are the same pair in both lanes).  The 8 lanes
// of a group must be active together.
template <typename R>
__device__ __forceinline__ R sum8(R x) {
  x += dpp_val<kDppX1>(x);
  x += dpp_val<kDppX2>(x);
  x += dpp_val<kDppHalfMirror>(x);
  return x;
}

// (best, bi) of every lane becomes the wave's maximum of best, ties to the
// smallest bi; all lanes must be active.
template <typename R>
__device__ __forceinline__ void wave_argmax(R& best, int& bi) {
  argmax_dpp<kDppX1>(best, bi);
  argmax_dpp<kDppX2>(best, bi);
  argmax_dpp<kDppHalfMirror>(best, bi);
  argmax_dpp<kDppMirror>(best, bi);
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
    const R ob = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (better(ob, oi, best, bi)) {
      best = ob;
      bi = oi;
    }
  }
}

// Factorises the leaf columns [lc, lc + kWL) of the panel [c, c + w), rows
// [lc, N), with the leaf in registers (thread t owns rows lc + t + 512 q).
// Interchanges are applied at once to the other panel columns in memory.
// Kept out of line (with the triangle inverses and apply_swaps) so that the
// register allocator treats the panel phase and the trailing update apart.
template <typename R, int kR, int kWL>
__device__ __noinline__ void leaf_factor(const Mat<typename Prec<R>::C>& Ain, int c, int w, int lc, int plim,
                                         LuSmem<R>& sh) {
  const Mat<typename Prec<R>::C> A = Ain;  // by value: fields stay in registers
  typedef typename Prec<R>::C C;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = (int)A.N;
  const int wl = min(kWL, c + w - lc);
  C a[kR][kWL];
#pragma unroll
  for (int q = 0; q < kR; ++q) {
    const int v = lc + tid + kLuThreads * q;
    if (v < N) {
      const auto row = A.ptr(v, lc);
#pragma unroll
      for (int k = 0; k < kWL; ++k) a[q][k] = (k < wl) ? row[k] : zmake(R(0), R(0));
    } else {
#pragma unroll
      for (int k = 0; k < kWL; ++k) a[q][k] = zmake(R(0), R(0));
    }
  }
  // Rows are not moved in registers: pos[q] is the current position of the
  // row held in a[q].  An interchange of positions j and bi only relabels the
  // two rows; each row is stored at its final position at the end.  The loop
  // is unrolled over the leaf's columns so that every register index is a
  // compile-time constant (a run-time column index turns each access into a
  // chain of selects).
  int pos[kR];
#pragma unroll
  for (int q = 0; q < kR; ++q) pos[q] = lc + tid + kLuThreads * q;
#pragma unroll
  for (int jj = 0; jj < kWL; ++jj) {
    if (jj >= wl) break;
    const int j = lc + jj;
    R best = R(-1);
    int bi = j;
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      if (pos[q] >= j && pos[q] < plim) {
        const R x = zcabs1(a[q][jj]);
        if (x > best || (x == best && pos[q] < bi)) {
          best = x;
          bi = pos[q];
        }
      }
    }
    // each wave publishes its candidate and the candidate's row (the lane
    // holding it writes the row); one barrier, then every thread picks the
    // winner.  Two buffers: a wave writes buffer jj & 1 only after the barrier
    // of step jj - 1, which every thread passes after its reads of step jj - 2.
    wave_argmax(best, bi);
    const int buf = jj & 1;
    if (lane == 0) {
      sh.candv[buf][wave] = best;
      sh.candi[buf][wave] = bi;
    }
#pragma unroll
    for (int q = 0; q < kR; ++q) {
      if (pos[q] == bi) {
#pragma unroll
        for (int k = 0; k < kWL; ++k) sh.cand[buf][wave][k] = a[q][k];
      }
    }
    __syncthreads();
    best = sh.candv[buf][0];
    bi = sh.candi[buf][0];
    int wv = 0;
#pragma unroll
    for (int q = 1; q < kLuWaves; ++q)
      if (better(sh.candv[buf][q], sh.candi[buf][q], best, bi)) {
        best = sh.candv[buf][q];
        bi = sh.candi[buf][q];
        wv = q;
      }
    const bool zero = !(best > R(0));
    if (zero) bi = j;
    if (tid == 0) {
      sh.ipiv[j - c] = bi;
      if (zero && best == R(0) && sh.info == 0) sh.info = j + 1;
    }
#pragma unroll
    for (int q = 0; q < kR; ++q) pos[q] = pos[q] == bi ? j : (pos[q] == j ? bi : pos[q]);
    if (!zero) {
      const C inv = zinv(sh.cand[buf][wv][jj]);
      C pr[kWL];
#pragma unroll
      for (int k = jj + 1; k < kWL; ++k) pr[k] = sh.cand[buf][wv][k];
#pragma unroll
      for (int q = 0; q < kR; ++q) {
        // rows that do not take part get a zero multiplier: a - 0 p == a
        const bool act = pos[q] > j && pos[q] < N;
        const C l0 = zmul(a[q][jj], inv);
        const C l = act ? l0 : zmake(R(0), R(0));
        if (act) a[q][jj] = l0;
#pragma unroll
        for (int k = jj + 1; k < kWL; ++k) a[q][k] = zfms(a[q][k], l, pr[k]);
      }
    }
  }
  // The leaf's interchanges, composed into one permutation of at most 2 wl
  // rows, applied to the other columns of the panel: every touched row is
  // loaded first, then stored in its final place.
  if (tid == 0) {
    int n = 0;
    for (int jj = 0; jj < wl; ++jj) {
      const int r0 = lc + jj, r1 = sh.ipiv[lc + jj - c];
      if (r0 == r1) continue;
      int i0 = -1, i1 = -1;
      for (int q = 0; q < n; ++q) {
        if (sh.lrow[q] == r0) i0 = q;
        if (sh.lrow[q] == r1) i1 = q;
      }
      if (i0 < 0) {
        sh.lrow[n] = r0;
        sh.lsrc[n] = n;
        i0 = n++;
      }
      if (i1 < 0) {
        sh.lrow[n] = r1;
        sh.lsrc[n] = n;
        i1 = n++;
      }
      const int t = sh.lsrc[i0];
      sh.lsrc[i0] = sh.lsrc[i1];
      sh.lsrc[i1] = t;
    }
    sh.lcnt = n;
  }
#pragma unroll
  for (int q = 0; q < kR; ++q) {
    if (pos[q] < N) {
      const auto row = A.ptr(pos[q], lc);
#pragma unroll
      for (int k = 0; k < kWL; ++k)
        if (k < wl) row[k] = a[q][k];
    }
  }
  __syncthreads();
  const int n = sh.lcnt;
  if (n > 0 && tid < w && (c + tid < lc || c + tid >= lc + wl)) {
    const int col = c + tid;
    C v[2 * kWL];
#pragma unroll
    for (int q = 0; q < 2 * kWL; ++q)
      if (q < n) v[q] = *A.ptr(sh.lrow[q], col);
#pragma unroll
    for (int q = 0; q < 2 * kWL; ++q) {
      if (q < n) {
        const int sidx = sh.lsrc[q];
        C x = v[0];
#pragma unroll
        for (int r = 1; r < 2 * kWL; ++r)
          if (sidx == r) x = v[r];
        *A.ptr(sh.lrow[q], col) = x;
      }
    }
  }
  __syncthreads();
}

// X = inverse of the unit lower triangular s x s block of A at (r0, r0),
// staged first in sh.U; zero outside [0, s)^2.  Eight lanes per column: lane
// p of a column accumulates the terms k = p (mod 8) of each row's dot product.
template <typename R>
__device__ __noinline__ void invert_unit_lower(const Mat<typename Prec<R>::C>& Ain, int r0, int s, LuSmem<R>& sh) {
  const Mat<typename Prec<R>::C> A = Ain;  // by value: fields stay in registers
  typedef typename Prec<R>::C C;
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += kLuThreads) {
    const int i = q / kNB, k = q % kNB;
    sh.U[i][k] = (i < s && k < i) ? *A.ptr(r0 + i, r0 + k) : zmake(R(0), R(0));
  }
  __syncthreads();
  const int j = tid >> 3, p = tid & 7;  // column j (0..63), part p
  C xr[kNB / 8];
#pragma unroll
  for (int m = 0; m < kNB / 8; ++m) xr[m] = zmake(R(0), R(0));
  if (j < s) {
#pragma unroll
    for (int m = 0; m < kNB / 8; ++m)
      if (p + 8 * m == j) xr[m] = zmake(R(1), R(0));
    for (int i = j + 1; i < s; ++i) {
      R sr = R(0), si = R(0);
#pragma unroll
      for (int m = 0; m < kNB / 8; ++m) {
        const int k = p + 8 * m;
        if (k >= j && k < i) {
          const C l = sh.U[i][k];
          sr += l.x * xr[m].x - l.y * xr[m].y;
          si += l.x * xr[m].y + l.y * xr[m].x;
        }
      }
      sr = sum8(sr);
      si = sum8(si);
#pragma unroll
      for (int m = 0; m < kNB / 8; ++m)
        if (p + 8 * m == i) xr[m] = zmake(-sr, -si);
    }
  }
#pragma unroll
  for (int m = 0; m < kNB / 8; ++m) sh.X[p + 8 * m][j] = xr[m];
  __syncthreads();
}

// X = inverse of the upper triangular s x s block of A at (r0, r0) (non-unit
// diagonal), staged first in sh.U; zero outside [0, s)^2.  Column j of X
// solves U x = e_j from the bottom: x_j = 1/U_jj, x_i = -(sum_{k=i+1..j}
// U_ik x_k) / U_ii for i < j; eight lanes per column as in invert_unit_lower.
template <typename R>
__device__ __noinline__ void invert_upper(const Mat<typename Prec<R>::C>& Ain, int r0, int s, LuSmem<R>& sh) {
  const Mat<typename Prec<R>::C> A = Ain;  // by value: fields stay in registers
  typedef typename Prec<R>::C C;
  const int tid = threadIdx.x;
  for (int q = tid; q < kNB * kNB; q += kLuThreads) {
    const int i = q / kNB, k = q % kNB;
    sh.U[i][k] = (i < s && k < s && k >= i) ? *A.ptr(r0 + i, r0 + k) : zmake(R(0), R(0));
  }
  __syncthreads();
  const int j = tid >> 3, p = tid & 7;
  C xr[kNB / 8];
#pragma unroll
  for (int m = 0; m < kNB / 8; ++m) xr[m] = zmake(R(0), R(0));
  if (j < s) {
    const C dj = zinv(sh.U[j][j]);
#pragma unroll
    for (int m = 0; m < kNB / 8; ++m)
      if (p + 8 * m == j) xr[m] = dj;
    for (int i = j - 1; i >= 0; --i) {
      R sr = R(0), si = R(0);
#pragma unroll
      for (int m = 0; m < kNB / 8; ++m) {
        const int k = p + 8 * m;
        if (k > i && k <= j) {
          const C u = sh.U[i][k];
          sr += u.x * xr[m].x - u.y * xr[m].y;
          si += u.x * xr[m].y + u.y * xr[m].x;
        }
      }
      sr = sum8(sr);
      si = sum8(si);
      const C xi = zmul(zmake(-sr, -si), zinv(sh.U[i][i]));
#pragma unroll
      for (int m = 0; m < kNB / 8; ++m)
        if (p + 8 * m == i) xr[m] = xi;
    }
  }
#pragma unroll
  for (int m = 0; m < kNB / 8; ++m) sh.X[p + 8 * m][j] = xr[m];
  __syncthreads();
}

// U12 of a panel of w in (64, 128] columns for the strip [s0, s0 + sw):
//   U_a = X_a A(c .. c+63, strip),
//   U_b = X_b (A(c+64 .. c+w-1, strip) - L(c+64 .. c+w-1, c .. c+63) U_a),
// X_a and X_b being the inverses of the two unit lower diagonal blocks
// (64 x 64 each, row-major at xg and xg + 64*64, zero outside their blocks).
// The result goes to the 128-row view of sh.X and sh.U (rows >= w zero) and,
// if `store`, to A.  4 x kSWp/16 output tiles per 64-row half, kSWp/32 per
// wave.
template <typename R>
__device__ __noinline__ void trsm2_strip(const Mat<typename Prec<R>::C>& Ain, int c, int w, int s0, int sw,
                                         bool store, const typename Prec<R>::C* __restrict__ xg, LuSmem<R>& sh) {
  const Mat<typename Prec<R>::C> A = Ain;  // by value: fields stay in registers
  typedef typename Prec<R>::C C;
  typedef typename Prec<R>::V4 V4;
  constexpr int NT = kSWp<R> / 32;  // column tiles per wave
  C(*U2)[kSWp<R>] = ustrip2(sh);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // waves w and w + 4 share a SIMD: they take row tiles r and 3 - r, so
  // every SIMD carries the same share of the triangular work
  const int rt = wave < 4 ? wave : 7 - wave, ct0 = NT * (wave >> 2);
  const int row = 16 * rt + li;
  const int wb = w - kNB;  // rows of the second block
  int64_t bcol[NT];
  bool cok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = 16 * (ct0 + t) + li;
    cok[t] = col < sw;
    bcol[t] = A.phys(s0 + min(col, sw - 1));
  }
  // FP64: products by the three-multiplication form (ar, ai, a3 the sums of
  // Re x Re b, Im x Im b, (Re x + Im x)(Re b + Im b) until the product is
  // complete), as in update_rows
  constexpr bool k3M = sizeof(R) == 8;
  V4 ar[NT], ai[NT], a3[k3M ? NT : 1];
  // U_a = X_a B, B[k][col] = A(c + k, s0 + col)
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    ar[t] = V4{R(0), R(0), R(0), R(0)};
    ai[t] = V4{R(0), R(0), R(0), R(0)};
    if constexpr (k3M) a3[t] = V4{R(0), R(0), R(0), R(0)};
  }
  {
    const int kend = 16 * rt + 16;
    C bn[NT][4], xn[4];
    trsm_load_chunk(A, c, kNB, 0, lk, bcol, cok, bn);
#pragma unroll
    for (int j = 0; j < 4; ++j) xn[j] = xg[row * kNB + 4 * lk + j];
    for (int kc = 0; kc < kend; kc += 16) {
      C b[NT][4], x[4];
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) b[t][j] = bn[t][j];
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = xn[j];
      if (kc + 16 < kend) {
        trsm_load_chunk(A, c, kNB, kc + 16, lk, bcol, cok, bn);
#pragma unroll
        for (int j = 0; j < 4; ++j) xn[j] = xg[row * kNB + kc + 16 + 4 * lk + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if constexpr (k3M) {
            ar[t] = Prec<R>::mfma(x[j].x, b[t][j].x, ar[t]);
            ai[t] = Prec<R>::mfma(x[j].y, b[t][j].y, ai[t]);
            a3[t] = Prec<R>::mfma(x[j].x + x[j].y, b[t][j].x + b[t][j].y, a3[t]);
          } else {
            ar[t] = Prec<R>::mfma(x[j].x, b[t][j].x, ar[t]);
            ar[t] = Prec<R>::mfma(-x[j].y, b[t][j].y, ar[t]);
            ai[t] = Prec<R>::mfma(x[j].x, b[t][j].y, ai[t]);
            ai[t] = Prec<R>::mfma(x[j].y, b[t][j].x, ai[t]);
          }
        }
    }
  }
  if constexpr (k3M) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const V4 re = ar[t] - ai[t], im = a3[t] - ar[t] - ai[t];
      ar[t] = re;
      ai[t] = im;
    }
  }
  __syncthreads();  // earlier readers of the strip are done
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rt + Prec<R>::drow(r, lk), col = 16 * (ct0 + t) + li;
      const C u = zmake(ar[t][r], ai[t][r]);
      U2[i][col] = u;
      if (store && col < sw) *A.ptr(c + i, s0 + col) = u;
    }
  __syncthreads();
  // T = A(c + 64 + i, strip) - L(c + 64 + i, c .. c+63) U_a, rows i < wb
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rt + Prec<R>::drow(r, lk);
      // rows >= wb clamped (their T rows meet zero columns of X_b and zero rows of it)
      const C v = A.base[A.phys(c + kNB + min(i, wb - 1)) * A.N + bcol[t]];
      if constexpr (k3M) {  // sums (Re, 0, Re + Im) of the starting value
        ar[t][r] = v.x;
        ai[t][r] = R(0);
        a3[t][r] = v.x + v.y;
      } else {
        ar[t][r] = v.x;
        ai[t][r] = v.y;
      }
    }
  {
    const auto lrow = A.base + A.phys(c + kNB + min(row, wb - 1)) * A.N + A.phys(c) + 4 * lk;
    C ln[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) ln[j] = lrow[j];
    for (int kc = 0; kc < kNB; kc += 16) {
      C l[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) l[j] = ln[j];
      if (kc + 16 < kNB) {
#pragma unroll
        for (int j = 0; j < 4; ++j) ln[j] = lrow[kc + 16 + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kc + 4 * lk + j;
        const R nx = -l[j].x, ny = -l[j].y;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const C u = U2[k][16 * (ct0 + t) + li];
          if constexpr (k3M) {
            ar[t] = Prec<R>::mfma(nx, u.x, ar[t]);
            ai[t] = Prec<R>::mfma(ny, u.y, ai[t]);
            a3[t] = Prec<R>::mfma(nx + ny, u.x + u.y, a3[t]);
          } else {
            ar[t] = Prec<R>::mfma(nx, u.x, ar[t]);
            ar[t] = Prec<R>::mfma(l[j].y, u.y, ar[t]);
            ai[t] = Prec<R>::mfma(nx, u.y, ai[t]);
            ai[t] = Prec<R>::mfma(ny, u.x, ai[t]);
          }
        }
      }
    }
  }
  if constexpr (k3M) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const V4 re = ar[t] - ai[t], im = a3[t] - ar[t] - ai[t];
      ar[t] = re;
      ai[t] = im;
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rt + Prec<R>::drow(r, lk), col = 16 * (ct0 + t) + li;
      U2[kNB + i][col] = zmake(ar[t][r], ai[t][r]);
    }
  __syncthreads();
  // U_b = X_b T
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    ar[t] = V4{R(0), R(0), R(0), R(0)};
    ai[t] = V4{R(0), R(0), R(0), R(0)};
    if constexpr (k3M) a3[t] = V4{R(0), R(0), R(0), R(0)};
  }
  {
    const int kend = min(wb, 16 * rt + 16);
    const C* xb = xg + kNB * kNB;
    C xn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) xn[j] = xb[row * kNB + 4 * lk + j];
    for (int kc = 0; kc < kend; kc += 16) {
      C xc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) xc[j] = xn[j];
      if (kc + 16 < kend) {
#pragma unroll
        for (int j = 0; j < 4; ++j) xn[j] = xb[row * kNB + kc + 16 + 4 * lk + j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kc + 4 * lk + j;
        const C x = xc[j];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const C b = U2[kNB + k][16 * (ct0 + t) + li];
          if constexpr (k3M) {
            ar[t] = Prec<R>::mfma(x.x, b.x, ar[t]);
            ai[t] = Prec<R>::mfma(x.y, b.y, ai[t]);
            a3[t] = Prec<R>::mfma(x.x + x.y, b.x + b.y, a3[t]);
          } else {
            ar[t] = Prec<R>::mfma(x.x, b.x, ar[t]);
            ar[t] = Prec<R>::mfma(-x.y, b.y, ar[t]);
            ai[t] = Prec<R>::mfma(x.x, b.y, ai[t]);
            ai[t] = Prec<R>::mfma(x.y, b.x, ai[t]);
          }
        }
      }
    }
  }
  if constexpr (k3M) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const V4 re = ar[t] - ai[t], im = a3[t] - ar[t] - ai[t];
      ar[t] = re;
      ai[t] = im;
    }
  }
  __syncthreads();  // T fully read
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rt + Prec<R>::drow(r, lk), col = 16 * (ct0 + t) + li;
      const C u = zmake(ar[t][r], ai[t][r]);
      U2[kNB + i][col] = u;
      if (store && i < wb && col < sw) *A.ptr(c + kNB + i, s0 + col) = u;
    }
  __syncthreads();
}

// Copies sh.X (after invert_unit_lower) to the 64 x 64 row-major block at dst.
template <typename R>
__device__ __forceinline__ void save_x(const LuSmem<R>& sh, typename Prec<R>::C* __restrict__ dst) {
  for (int q = threadIdx.x; q < kNB * kNB; q += kLuThreads) dst[q] = sh.X[q / kNB][q % kNB];
  __syncthreads();
}

// Loads the B operands of one 16-deep chunk of trsm_strip: lane (li, lk)
// takes rows k = kc + 4 lk + j (j < 4) of its two columns, the row clamped to
// s - 1 and the column to the strip (in-range, straight-line loads).
template <typename C, int NT>
__device__ __forceinline__ void trsm_load_chunk(const Mat<C>& A, int r0, int s, int kc, int lk,
                                                const int64_t (&bcol)[NT], const bool (&cok)[NT], C (&dst)[NT][4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    // rows k >= s clamped to s - 1: X is zero in those columns
    const auto rowp = glb(A.base + A.phys(r0 + min(kc + 4 * lk + j, s - 1)) * A.N);
#pragma unroll
    for (int t = 0; t < NT; ++t) dst[t][j] = rowp[bcol[t]];  // columns >= sw are never stored
  }
}

// U = X * A(r0 .. r0+s-1, s0 .. s0+sw-1) into sh.U rows 0..63 (rows >= s are
// zero), and, if `store`, also into those rows of A.  4 x kSWp/16 output
// tiles of 16x16, kSWp/32 per wave.  The reduction runs in chunks of 16 (lane (li, lk)
// supplies k = kc + 4 lk + j at MFMA step j), the next chunk being loaded
// while the current one is multiplied; X is lower triangular, so row tile rt
// stops at k = 16 rt + 16.
template <typename R>
__device__ __noinline__ void trsm_strip(const Mat<typename Prec<R>::C>& Ain, int r0, int s, int s0, int sw,
                                        bool store, LuSmem<R>& sh) {
  const Mat<typename Prec<R>::C> A = Ain;  // by value: fields stay in registers
  typedef typename Prec<R>::C C;
  typedef typename Prec<R>::V4 V4;
  constexpr int NT = kSWp<R> / 32;  // column tiles per wave
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rt = wave < 4 ? wave : 7 - wave;  // row tile (r and 3 - r per SIMD, as in trsm2_strip)
  const int ct0 = NT * (wave >> 2);           // first of NT column tiles
  // FP64: products by the three-multiplication form, as in trsm2_strip
  constexpr bool k3M = sizeof(R) == 8;
  V4 ar[NT], ai[NT], a3[k3M ? NT : 1];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    ar[t] = V4{R(0), R(0), R(0), R(0)};
    ai[t] = V4{R(0), R(0), R(0), R(0)};
    if constexpr (k3M) a3[t] = V4{R(0), R(0), R(0), R(0)};
  }
  int64_t bcol[NT];
  bool cok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = 16 * (ct0 + t) + li;
    cok[t] = col < sw;
    bcol[t] = A.phys(s0 + min(col, sw - 1));
  }
  const int row = 16 * rt + li;
  const int kend = min(s, 16 * rt + 16);
  C bn[NT][4];
  if (kend > 0) trsm_load_chunk(A, r0, s, 0, lk, bcol, cok, bn);
  for (int kc = 0; kc < kend; kc += 16) {
    C b[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) b[t][j] = bn[t][j];
    if (kc + 16 < kend) trsm_load_chunk(A, r0, s, kc + 16, lk, bcol, cok, bn);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = kc + 4 * lk + j;
      const C x = sh.X[row][k & (kNB - 1)];
      const R xr = (k < s) ? x.x : R(0);
      const R xi = (k < s) ? x.y : R(0);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if constexpr (k3M) {
          ar[t] = Prec<R>::mfma(xr, b[t][j].x, ar[t]);
          ai[t] = Prec<R>::mfma(xi, b[t][j].y, ai[t]);
          a3[t] = Prec<R>::mfma(xr + xi, b[t][j].x + b[t][j].y, a3[t]);
        } else {
          ar[t] = Prec<R>::mfma(xr, b[t][j].x, ar[t]);
          ar[t] = Prec<R>::mfma(-xi, b[t][j].y, ar[t]);
          ai[t] = Prec<R>::mfma(xr, b[t][j].y, ai[t]);
          ai[t] = Prec<R>::mfma(xi, b[t][j].x, ai[t]);
        }
      }
    }
  }
  if constexpr (k3M) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const V4 re = ar[t] - ai[t], im = a3[t] - ar[t] - ai[t];
      ar[t] = re;
      ai[t] = im;
    }
  }
  __syncthreads();  // earlier readers of sh.U are done
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rt + Prec<R>::drow(r, lk), col = 16 * (ct0 + t) + li;
      const C u = zmake(ar[t][r], ai[t][r]);
      sh.U[i][col] = u;
      if (store && i < s && col < sw) *A.ptr(r0 + i, s0 + col) = u;
    }
  __syncthreads();
}

// Reduction depth of one chunk of the trailing update: 16 in FP64; 32 in
// FP32, whose MFMA takes half the cycles, so that a chunk of MFMA work still
// covers the latency of the next chunk's loads.
template <typename R>
constexpr int kUpdChunk = sizeof(R) == 4 ? 32 : 16;

// A(v, s0 + j) -= sum_{k < s} A(v, r0 + k) U[k][j] for v in [r0 + s, N),
// j < sw <= 16 NCS, s > kUpdChunk.  Each wave owns blocks of 16 rows x 16 NCS
// columns (NCS MFMA tiles).  The reduction runs in chunks of KC = kUpdChunk:
// in a chunk starting at kc, lane (li, lq) supplies k = kc + (KC/4) lq + j at
// MFMA step j, so that it reads KC/4 consecutive entries of its row.  Loads run one chunk
// ahead: the next chunk of the row block or, during its last chunk, the
// block's own entries of A (added to the product at the end) and the next
// row block's first chunk.  A finished block stays in registers and is
// stored after the first MFMA step of the next block: loads and stores share
// one completion counter, so a store issued just before a wait for loads
// would be waited for too; issued there it completes behind three steps of
// MFMA work.  The first and last chunks are peeled so that the block of A
// and the pending results occupy registers only there.  The LDS operand rows
// U[k] are zero for k >= s.
template <typename R, int NCS>
__device__ __forceinline__ void update_rows(const Mat<typename Prec<R>::C>& A, int r0, int s, int s0, int sw,
                                            const typename Prec<R>::C (*Ub)[kSWp<R>], int vlo = 0,
                                            int vhi = 0x7fffffff) {
  typedef typename Prec<R>::C C;
  typedef typename Prec<R>::V4 V4;
  constexpr int KJ = kUpdChunk<R> / 4;  // MFMA steps per chunk
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  // rows [max(r0 + s, vlo), min(N, vhi)) (all rows below the block by default)
  const int N = min((int)A.N, vhi);
  const int rstart = max(r0 + s, vlo);
  int64_t ccol[NCS];
  bool cok[NCS];
#pragma unroll
  for (int cs = 0; cs < NCS; ++cs) {
    cok[cs] = 16 * cs + li < sw;
    ccol[cs] = A.phys(s0 + min(16 * cs + li, sw - 1));
  }
  int rb = rstart + 16 * wave;
  if (rb >= N) return;
  // Loads are unconditional, from clamped in-range addresses, so that they
  // stay in straight-line code with exact wait counts: entries of rows >= N
  // or columns >= sw are never stored, and an L entry of a column >= s
  // (clamped to s - 1, a finite matrix entry) meets a zero row of Ub.
  C cv[NCS][4], an[KJ], pv[NCS][4];
  // block q of A: rows q + drow(r, lq)
  auto load_c = [&](int q) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = q + Prec<R>::drow(r, lq);
      const auto crow = glb(A.base + A.phys(v < N ? v : rstart) * A.N);
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs) cv[cs][r] = ntload(&crow[ccol[cs]]);
    }
  };
  auto store_pv = [&](int q) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = q + Prec<R>::drow(r, lq);
      if (v >= N) continue;
      const auto crow = glb(A.base + A.phys(v) * A.N);
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs)
        if (cok[cs]) ntstore(&crow[ccol[cs]], pv[cs][r]);
    }
  };
  // chunk kc of the L operand of row block q: row q + li, k = kc + KJ lq + j
  const int64_t pc0 = A.phys(r0);
  auto load_a = [&](int q, int kc) {
    const int va = q + li;
    const auto arow = glb(A.base + A.phys(va < N ? va : rstart) * A.N + pc0);
#pragma unroll
    for (int j = 0; j < KJ; ++j) an[j] = arow[min(kc + KJ * lq + j, s - 1)];
  };
  const LSMS_LDS C(*U)[kSWp<R>] = (const LSMS_LDS C(*)[kSWp<R>])Ub;
  // FP64: complex products by the three-multiplication form: with P1 = Re a
  // Re b, P2 = Im a Im b, P3 = (Re a + Im a)(Re b + Im b), a b = (P1 - P2) +
  // i (P3 - P1 - P2), three MFMAs per operand pair instead of four (acc1..3
  // hold the sums of P1, P2, P3).  FP32 keeps four (acc1, acc2 the real and
  // imaginary parts of -a b): its three-accumulator form does not fit the
  // registers of the 128-column strips.
  constexpr bool k3M = sizeof(R) == 8;
  V4 acc1[NCS], acc2[NCS], acc3[k3M ? NCS : 1];
  auto step = [&](int kc, int j, const C& aj) {
    const int k = (kc + KJ * lq + j) & (kPanelMax - 1);
    if constexpr (k3M) {
      const R as = aj.x + aj.y;
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs) {
        const C b = U[k][16 * cs + li];
        acc1[cs] = Prec<R>::mfma(aj.x, b.x, acc1[cs]);
        acc2[cs] = Prec<R>::mfma(aj.y, b.y, acc2[cs]);
        acc3[cs] = Prec<R>::mfma(as, b.x + b.y, acc3[cs]);
      }
    } else {
      const R nx = -aj.x, ny = -aj.y;
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs) {
        const C b = U[k][16 * cs + li];
        acc1[cs] = Prec<R>::mfma(nx, b.x, acc1[cs]);
        acc1[cs] = Prec<R>::mfma(aj.y, b.y, acc1[cs]);
        acc2[cs] = Prec<R>::mfma(nx, b.y, acc2[cs]);
        acc2[cs] = Prec<R>::mfma(ny, b.x, acc2[cs]);
      }
    }
  };
  const int klast = kUpdChunk<R> * ((s - 1) / kUpdChunk<R>);  // first k of the last chunk (> 0)
  int pb = -1;
  load_a(rb, 0);
  for (; rb < N; rb += 16 * kLuWaves) {
    const int rn = rb + 16 * kLuWaves;
#pragma unroll
    for (int cs = 0; cs < NCS; ++cs) {
      acc1[cs] = V4{R(0), R(0), R(0), R(0)};
      acc2[cs] = V4{R(0), R(0), R(0), R(0)};
      if constexpr (k3M) acc3[cs] = V4{R(0), R(0), R(0), R(0)};
    }
    {
      C a[KJ];
#pragma unroll
      for (int j = 0; j < KJ; ++j) a[j] = an[j];
      step(0, 0, a[0]);
      __builtin_amdgcn_sched_barrier(0);
      if (pb >= 0) store_pv(pb);
      load_a(rb, kUpdChunk<R>);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 1; j < KJ; ++j) step(0, j, a[j]);
    }
    for (int kc = kUpdChunk<R>; kc < klast; kc += kUpdChunk<R>) {
      C a[KJ];
#pragma unroll
      for (int j = 0; j < KJ; ++j) a[j] = an[j];
      load_a(rb, kc + kUpdChunk<R>);
#pragma unroll
      for (int j = 0; j < KJ; ++j) step(kc, j, a[j]);
    }
    {
      C a[KJ];
#pragma unroll
      for (int j = 0; j < KJ; ++j) a[j] = an[j];
      load_c(rb);
      if (rn < N) load_a(rn, 0);
#pragma unroll
      for (int j = 0; j < KJ; ++j) step(klast, j, a[j]);
    }
#pragma unroll
    for (int cs = 0; cs < NCS; ++cs)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (k3M)
          pv[cs][r] = zmake(cv[cs][r].x - (acc1[cs][r] - acc2[cs][r]),
                            cv[cs][r].y - (acc3[cs][r] - acc1[cs][r] - acc2[cs][r]));
        else
          pv[cs][r] = zmake(cv[cs][r].x + acc1[cs][r], cv[cs][r].y + acc2[cs][r]);
      }
    pb = rb;
  }
  store_pv(pb);
}

// As update_rows for short reductions, s <= 4 KA <= 32 (the sibling updates
// of the recursive panel), sw <= 16 NCS: each wave takes RB row blocks at a time
// (row blocks rb + 16 kLuWaves i, i < RB), with all their operands for the
// whole reduction loaded together, one group ahead; lane (li, lq) supplies
// k = lq + 4 j at step j, so that a reduction of s takes ceil(s / 4) MFMA
// steps.  A finished group's results are stored after the next group's loads
// have been issued, so that they complete behind a group of MFMA work.
template <typename R, int NCS, int RB, int KA>
__device__ __forceinline__ void update_rows_multi(const Mat<typename Prec<R>::C>& A, int r0, int s, int s0,
                                                  int sw, const typename Prec<R>::C (*Ub)[kSWp<R>]) {
  typedef typename Prec<R>::C C;
  typedef typename Prec<R>::V4 V4;
  static_assert(KA == 4 || KA == 8, "L entries per lane and row block: s <= 4 KA");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int N = (int)A.N;
  const int rstart = r0 + s;
  const int64_t pc0 = A.phys(r0);
  constexpr int kStep = 16 * kLuWaves;
  const int nj = (s + 3) >> 2;  // MFMA steps
  int64_t ccol[NCS];
  bool cok[NCS];
#pragma unroll
  for (int cs = 0; cs < NCS; ++cs) {
    cok[cs] = 16 * cs + li < sw;
    ccol[cs] = A.phys(s0 + min(16 * cs + li, sw - 1));
  }
  int rb = rstart + 16 * wave;
  if (rb >= N) return;
  // operands of the group starting at row block q: clamped in-range loads
  // (rows >= N and columns >= sw are never stored; L entries of columns
  // >= s, clamped to s - 1, meet zero rows of Ub)
  C cn[RB][NCS][4], an[RB][KA];
  auto load_group = [&](int q) {
#pragma unroll
    for (int b = 0; b < RB; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = q + b * kStep + Prec<R>::drow(r, lq);
        const auto crow = glb(A.base + A.phys(v < N ? v : rstart) * A.N);
#pragma unroll
        for (int cs = 0; cs < NCS; ++cs) cn[b][cs][r] = crow[ccol[cs]];
      }
      const int va = q + b * kStep + li;
      const auto arow = glb(A.base + A.phys(va < N ? va : rstart) * A.N + pc0);
#pragma unroll
      for (int j = 0; j < KA; ++j)
        if (j < nj) an[b][j] = arow[min(lq + 4 * j, s - 1)];
    }
  };
  C pv[RB][NCS][4];
  int pb = -1;
  auto store_group = [&](int q) {
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = q + b * kStep + Prec<R>::drow(r, lq);
        if (v >= N) continue;
        const auto crow = glb(A.base + A.phys(v) * A.N);
#pragma unroll
        for (int cs = 0; cs < NCS; ++cs)
          if (cok[cs]) crow[ccol[cs]] = pv[b][cs][r];
      }
  };
  load_group(rb);
  // FP64: products by the three-multiplication form (accr, acci, acc3 the
  // sums of Re a Re u, Im a Im u, (Re a + Im a)(Re u + Im u) of the negated
  // L entries, started from (Re c, 0, Re c + Im c) of the block's own
  // entries), as in update_rows
  constexpr bool k3M = sizeof(R) == 8;
  for (; rb < N; rb += RB * kStep) {
    V4 accr[RB][NCS], acci[RB][NCS], acc3[k3M ? RB : 1][k3M ? NCS : 1];
    C a[RB][KA];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if constexpr (k3M) {
            accr[b][cs][r] = cn[b][cs][r].x;
            acci[b][cs][r] = R(0);
            acc3[b][cs][r] = cn[b][cs][r].x + cn[b][cs][r].y;
          } else {
            accr[b][cs][r] = cn[b][cs][r].x;
            acci[b][cs][r] = cn[b][cs][r].y;
          }
        }
#pragma unroll
      for (int j = 0; j < KA; ++j) a[b][j] = an[b][j];
    }
    const int rn = rb + RB * kStep;
    if (rn < N) load_group(rn);
    if (pb >= 0) store_group(pb);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < KA; ++j) {
      if (j >= nj) break;
      const int k = lq + 4 * j;
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs) {
        const C u = ((const LSMS_LDS C(*)[kSWp<R>])Ub)[k][16 * cs + li];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const R nx = -a[b][j].x, ny = -a[b][j].y;
          if constexpr (k3M) {
            accr[b][cs] = Prec<R>::mfma(nx, u.x, accr[b][cs]);
            acci[b][cs] = Prec<R>::mfma(ny, u.y, acci[b][cs]);
            acc3[b][cs] = Prec<R>::mfma(nx + ny, u.x + u.y, acc3[b][cs]);
          } else {
            accr[b][cs] = Prec<R>::mfma(nx, u.x, accr[b][cs]);
            accr[b][cs] = Prec<R>::mfma(a[b][j].y, u.y, accr[b][cs]);
            acci[b][cs] = Prec<R>::mfma(nx, u.y, acci[b][cs]);
            acci[b][cs] = Prec<R>::mfma(ny, u.x, acci[b][cs]);
          }
        }
      }
    }
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if constexpr (k3M)
            pv[b][cs][r] = zmake(accr[b][cs][r] - acci[b][cs][r], acc3[b][cs][r] - accr[b][cs][r] - acci[b][cs][r]);
          else
            pv[b][cs][r] = zmake(accr[b][cs][r], acci[b][cs][r]);
        }
    pb = rb;
  }
  store_group(pb);
}

// A(v, s0 + j) -= sum_{k < s} A(v, r0 + k) Ub[k][j] for v in [r0 + s, N),
// j < sw <= kSWp, s <= 128 (Ub in LDS, rows k >= s zero).
template <typename R>
__device__ __noinline__ void update_strip(const Mat<typename Prec<R>::C>& Ain, int r0, int s, int s0, int sw,
                                          const typename Prec<R>::C (*Ub)[kSWp<R>]) {
  const Mat<typename Prec<R>::C> A = Ain;  // by value: fields stay in registers
  typedef const typename Prec<R>::C(*Rows)[kSWp<R>];
  if (s <= 16) {  // short reductions: operands of whole row blocks at once
    if (sw > 32) {  // strips of at most 32 columns
      for (int o = 0; o < sw; o += 32)
        update_rows_multi<R, 2, 1, 4>(A, r0, s, s0 + o, min(32, sw - o), reinterpret_cast<Rows>(&Ub[0][o]));
    } else if (sw > 16) {
      update_rows_multi<R, 2, 1, 4>(A, r0, s, s0, sw, Ub);
    } else {
      update_rows_multi<R, 1, 2, 4>(A, r0, s, s0, sw, Ub);
    }
  } else if (s <= 32) {
    if (sw > 32) {
      for (int o = 0; o < sw; o += 32)
        update_rows_multi<R, 2, 1, 8>(A, r0, s, s0 + o, min(32, sw - o), reinterpret_cast<Rows>(&Ub[0][o]));
    } else if (sw > 16) {
      update_rows_multi<R, 2, 1, 8>(A, r0, s, s0, sw, Ub);
    } else {
      update_rows_multi<R, 1, 1, 8>(A, r0, s, s0, sw, Ub);
    }
  } else if (kSWp<R> > 96 && sw > 112) {
    update_rows<R, (kSWp<R> > 96 ? 8 : 4)>(A, r0, s, s0, sw, Ub);
  } else if (kSWp<R> > 96 && sw > 96) {
    update_rows<R, (kSWp<R> > 96 ? 7 : 4)>(A, r0, s, s0, sw, Ub);
  } else if (kSWp<R> > 64 && sw > 80) {
    update_rows<R, (kSWp<R> > 64 ? 6 : 4)>(A, r0, s, s0, sw, Ub);
  } else if (kSWp<R> > 64 && sw > 64) {
    update_rows<R, (kSWp<R> > 64 ? 5 : 4)>(A, r0, s, s0, sw, Ub);
  } else if (sw > 48) {
    update_rows<R, 4>(A, r0, s, s0, sw, Ub);
  } else if (sw > 32) {
    update_rows<R, 3>(A, r0, s, s0, sw, Ub);
  } else if (sw > 16) {
    update_rows<R, 2>(A, r0, s, s0, sw, Ub);
  } else {
    update_rows<R, 1>(A, r0, s, s0, sw, Ub);
  }
}

// Row interchanges of the panel [c, c + w) applied to the columns [c0, c1).
// Each thread owns whole columns, so the interchanges are applied in order
// per thread.
template <typename R>
__device__ __noinline__ void apply_swaps(const Mat<typename Prec<R>::C>& Ain, int c, int w, int c0, int c1,
                                         const LuSmem<R>& sh) {
  const Mat<typename Prec<R>::C> A = Ain;  // by value: fields stay in registers
  typedef typename Prec<R>::C C;
  for (int jj = 0; jj < w; ++jj) {
    const int p = sh.ipiv[jj], r = c + jj;
    if (p == r) continue;
    const auto rr = A.base + A.phys(r) * A.N;
    const auto rp = A.base + A.phys(p) * A.N;
    for (int u = c0 + threadIdx.x; u < c1; u += kLuThreads) {
      const int64_t pu = A.phys(u);
      const C x = rr[pu], y = rp[pu];
      rr[pu] = y;
      rp[pu] = x;
    }
  }
}

// Recursive panel factorisation of columns [c, c + w): leaves of kWL columns
// in registers; after each leaf the completed block of the recursion updates
// its sibling block (triangular solve and product on MFMA).  With store_u the
// upper-triangular part of the panel is kept in A.
template <typename R, int kR, int kWL>
__device__ void panel_factor(const Mat<typename Prec<R>::C>& A, int c, int w, int plim, bool store_u,
                             LuSmem<R>& sh) {
  const int nleaf = (w + kWL - 1) / kWL;
  for (int i = 0; i < nleaf; ++i) {
    const int lc = c + kWL * i;
    leaf_factor<R, kR, kWL>(A, c, w, lc, plim, sh);
    const int s = kWL << __builtin_ctz(i + 1);
    const int start = lc + kWL - s;
    const int t0 = lc + kWL;
    const int tw = min(s, c + w - t0);
    if (tw > 0) {
      invert_unit_lower<R>(A, start, s, sh);
      trsm_strip<R>(A, start, s, t0, tw, store_u, sh);
      update_strip<R>(A, start, s, t0, tw, sh.U);
      __syncthreads();
    }
  }
}

// Blocked right-looking elimination of the columns [c_begin, ncols) of the
// N x N matrix: panels of nb <= 128 columns with pivot rows below plim,
// interchanges applied to every column right of the panel (the columns left
// of a panel keep the row order of their own elimination step), the U part
// written back when store_u, and the panel pivots stored at ipiv_out[column]
// (if non-null).  A panel wider than 64 needs xg, room for two 64 x 64
// blocks (the inverses of its diagonal blocks); without xg panels are at most
// 64 wide.  With xcache, the inverse of every (at most 64-column) diagonal
// block of L, in panel order, is kept at xcache + 64*64*q for block q
// (panels that have trailing columns only).  Ends after a barrier.
template <typename R, int kR, int kWL>
__device__ void eliminate(const Mat<typename Prec<R>::C>& A, int c_begin, int ncols, int plim, int nb,
                          bool store_u, int32_t* ipiv_out, typename Prec<R>::C* xg, LuSmem<R>& sh,
                          typename Prec<R>::C* xcache = nullptr) {
  const int N = (int)A.N;
  if (!xg && !xcache) nb = min(nb, kNB);
  int blk = 0;
  for (int c = c_begin; c < ncols; c += nb) {
    const int w = min(nb, ncols - c);
    panel_factor<R, kR, kWL>(A, c, w, plim, store_u, sh);
    apply_swaps<R>(A, c, w, c + w, N, sh);
    if (ipiv_out && threadIdx.x < w) ipiv_out[c + threadIdx.x] = sh.ipiv[threadIdx.x];
    __syncthreads();
    if (c + w < N) {
      if (w <= kNB) {
        invert_unit_lower<R>(A, c, w, sh);
        if (xcache) save_x<R>(sh, xcache + (int64_t)blk * kNB * kNB);
        blk += 1;
        for (int s0 = c + w; s0 < N; s0 += kSWp<R>) {
          const int sw = min(kSWp<R>, N - s0);
          trsm_strip<R>(A, c, w, s0, sw, store_u, sh);
          update_strip<R>(A, c, w, s0, sw, sh.U);
        }
      } else {
        typename Prec<R>::C* xp = xcache ? xcache + (int64_t)blk * kNB * kNB : xg;
        blk += 2;
        invert_unit_lower<R>(A, c, kNB, sh);
        save_x<R>(sh, xp);
        invert_unit_lower<R>(A, c + kNB, w - kNB, sh);
        save_x<R>(sh, xp + kNB * kNB);
        for (int s0 = c + w; s0 < N; s0 += kSWp<R>) {
          const int sw = min(kSWp<R>, N - s0);
          trsm2_strip<R>(A, c, w, s0, sw, store_u, xp, sh);
          update_strip<R>(A, c, w, s0, sw, ustrip2(sh));
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace lsms
