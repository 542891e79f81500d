// Local interaction zone extraction (paper Sec. 2.2: the KKR matrix of each
// atom is built over the atoms of its LIZ, the cluster centred on it).
//
// For instance i with centre atom c = centre[i] and cutoff rc[i], the LIZ is
// the centre followed by every other atom whose minimum-image vector
// d = R_j - R_c (each component reduced by box * rint(d / box)) satisfies
// dx*dx + dy*dy + dz*dz <= rc*rc, ordered by ascending squared distance with
// ties broken by (dx, dy, dz) lexicographically.  Distances are formed with
// FP contraction off so that membership and order depend only on IEEE-rounded
// products and sums.
//
// Three launches: count per instance, exclusive scan into offsets, fill.  A
// LIZ larger than max_liz keeps its max_liz nearest sites (the same order).
#include "lsms_common.h"

using namespace lsms;

namespace {

constexpr int kLizThreads = 256;
constexpr int kLizCap = 1024;  // candidates held in LDS per instance

struct Cand {
  double d2, dx, dy, dz;
  int idx;
};

__device__ __forceinline__ bool cand_less(const Cand& a, const Cand& b) {
  if (a.d2 != b.d2) return a.d2 < b.d2;
  if (a.dx != b.dx) return a.dx < b.dx;
  if (a.dy != b.dy) return a.dy < b.dy;
  if (a.dz != b.dz) return a.dz < b.dz;
  return a.idx < b.idx;
}

__device__ __forceinline__ void min_image(const double* __restrict__ pos, int j, const double* p0, double bx,
                                          double by, double bz, double d[3], double& d2) {
#pragma clang fp contract(off)
  d[0] = pos[3 * (size_t)j + 0] - p0[0];
  d[1] = pos[3 * (size_t)j + 1] - p0[1];
  d[2] = pos[3 * (size_t)j + 2] - p0[2];
  d[0] -= bx * rint(d[0] / bx);
  d[1] -= by * rint(d[1] / by);
  d[2] -= bz * rint(d[2] / bz);
  const double a = d[0] * d[0];
  const double b = d[1] * d[1];
  const double c = d[2] * d[2];
  d2 = (a + b) + c;
}

__global__ __launch_bounds__(kLizThreads) void liz_count_kernel(const double* __restrict__ pos, int n_atoms,
                                                                double bx, double by, double bz,
                                                                const int32_t* __restrict__ centre,
                                                                const double* __restrict__ rc,
                                                                int32_t* __restrict__ liz_n) {
  __shared__ int cnt;
  const int i = blockIdx.x;
  const int c = centre[i];
  if (c < 0 || c >= n_atoms) {  // invalid centre: empty LIZ
    if (threadIdx.x == 0) liz_n[i] = 0;
    return;
  }
  const double r = rc[i];
  const double rc2 = r * r;
  const double p0[3] = {pos[3 * (size_t)c], pos[3 * (size_t)c + 1], pos[3 * (size_t)c + 2]};
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int local = 0;
  for (int j = threadIdx.x; j < n_atoms; j += kLizThreads) {
    if (j == c) continue;
    double d[3], d2;
    min_image(pos, j, p0, bx, by, bz, d, d2);
    local += (d2 <= rc2);
  }
  atomicAdd(&cnt, local);
  __syncthreads();
  if (threadIdx.x == 0) liz_n[i] = cnt + 1;
}

// Exclusive scan of min(liz_n, max_liz) into liz_off[0..n], one workgroup.
__global__ __launch_bounds__(1024) void liz_scan_kernel(const int32_t* __restrict__ liz_n, int n, int max_liz,
                                                        int64_t* __restrict__ liz_off) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int a = t * per, b = min(n, a + per);
  int64_t s = 0;
  for (int k = a; k < b; ++k) s += min(liz_n[k], max_liz);
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;  // exclusive prefix of this chunk
  for (int k = a; k < b; ++k) {
    liz_off[k] = run;
    run += min(liz_n[k], max_liz);
  }
  if (t == 1023) liz_off[n] = part[1023];
}

__global__ __launch_bounds__(kLizThreads) void liz_fill_kernel(
    const double* __restrict__ pos, const int32_t* __restrict__ atom_species, int n_atoms, double bx, double by,
    double bz, const int32_t* __restrict__ centre, const double* __restrict__ rc, int max_liz,
    const int64_t* __restrict__ liz_off, double* __restrict__ liz_pos, int32_t* __restrict__ liz_species,
    int32_t* __restrict__ liz_atom) {
  __shared__ Cand cand[kLizCap];
  __shared__ int ncand;
  const int i = blockIdx.x;
  const int c = centre[i];
  if (c < 0 || c >= n_atoms) return;
  const double r = rc[i];
  const double rc2 = r * r;
  const double p0[3] = {pos[3 * (size_t)c], pos[3 * (size_t)c + 1], pos[3 * (size_t)c + 2]};
  const int64_t base = liz_off[i];
  const int cap = (int)(liz_off[i + 1] - base);  // rows reserved for this instance
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < n_atoms; j += kLizThreads) {
    if (j == c) continue;
    double d[3], d2;
    min_image(pos, j, p0, bx, by, bz, d, d2);
    if (d2 <= rc2) {
      const int slot = atomicAdd(&ncand, 1);
      if (slot < kLizCap) cand[slot] = Cand{d2, d[0], d[1], d[2], j};
    }
  }
  __syncthreads();
  const int n = min(ncand, kLizCap);
  if (threadIdx.x == 0 && cap > 0) {
    liz_pos[3 * base + 0] = 0.0;
    liz_pos[3 * base + 1] = 0.0;
    liz_pos[3 * base + 2] = 0.0;
    liz_species[base] = atom_species[c];
    if (liz_atom) liz_atom[base] = c;
  }
  if (ncand > kLizCap) {
    // More candidates than LDS holds: each candidate's rank is counted
    // against every atom within the cutoff, read again from global memory,
    // so that the rows kept are the nearest ones, in order, whatever the
    // order in which the candidates were found.
    for (int j = threadIdx.x; j < n_atoms; j += kLizThreads) {
      if (j == c) continue;
      double d[3], d2;
      min_image(pos, j, p0, bx, by, bz, d, d2);
      if (!(d2 <= rc2)) continue;
      const Cand me{d2, d[0], d[1], d[2], j};
      int rank = 0;
      for (int o = 0; o < n_atoms; ++o) {
        if (o == c) continue;
        double e[3], e2;
        min_image(pos, o, p0, bx, by, bz, e, e2);
        rank += (e2 <= rc2) && cand_less(Cand{e2, e[0], e[1], e[2], o}, me);
      }
      const int row = 1 + rank;
      if (row < cap) {
        liz_pos[3 * (base + row) + 0] = me.dx;
        liz_pos[3 * (base + row) + 1] = me.dy;
        liz_pos[3 * (base + row) + 2] = me.dz;
        liz_species[base + row] = atom_species[me.idx];
        if (liz_atom) liz_atom[base + row] = me.idx;
      }
    }
    return;
  }
  for (int q = threadIdx.x; q < n; q += kLizThreads) {
    const Cand me = cand[q];
    int rank = 0;
    for (int o = 0; o < n; ++o) rank += cand_less(cand[o], me);
    const int row = 1 + rank;
    if (row < cap) {
      liz_pos[3 * (base + row) + 0] = me.dx;
      liz_pos[3 * (base + row) + 1] = me.dy;
      liz_pos[3 * (base + row) + 2] = me.dz;
      liz_species[base + row] = atom_species[me.idx];
      if (liz_atom) liz_atom[base + row] = me.idx;
    }
  }
}

}  // namespace

namespace {

// out[r] = src[idx[r]] (three doubles per row); NaN for an index outside
// [0, n_src).
__global__ __launch_bounds__(256) void gather3_kernel(int64_t n, const int32_t* __restrict__ idx,
                                                      const double* __restrict__ src, int32_t n_src,
                                                      double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const int32_t a = idx[r];
  const bool ok = a >= 0 && a < n_src;
#pragma unroll
  for (int k = 0; k < 3; ++k) out[3 * r + k] = ok ? src[3 * (int64_t)a + k] : (double)NAN;
}

}  // namespace

hipError_t lsms_launch_gather3(int64_t n, const int32_t* idx, const double* src, int32_t n_src, double* out,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather3_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx, src, n_src, out);
  return hipGetLastError();
}

hipError_t lsms_launch_liz(const double* atom_pos, const int32_t* atom_species, int32_t n_atoms, double bx,
                           double by, double bz, const int32_t* centre, const double* rc, int32_t n_inst,
                           int32_t max_liz, int32_t* liz_n, int64_t* liz_off, double* liz_pos,
                           int32_t* liz_species, int32_t* liz_atom, hipStream_t s) {
  if (n_inst == 0) {
    hipLaunchKernelGGL(liz_scan_kernel, dim3(1), dim3(1024), 0, s, liz_n, 0, max_liz, liz_off);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(liz_count_kernel, dim3(n_inst), dim3(kLizThreads), 0, s, atom_pos, n_atoms, bx, by, bz,
                     centre, rc, liz_n);
  hipLaunchKernelGGL(liz_scan_kernel, dim3(1), dim3(1024), 0, s, liz_n, n_inst, max_liz, liz_off);
  hipLaunchKernelGGL(liz_fill_kernel, dim3(n_inst), dim3(kLizThreads), 0, s, atom_pos, atom_species, n_atoms, bx,
                     by, bz, centre, rc, max_liz, liz_off, liz_pos, liz_species, liz_atom);
  return hipGetLastError();
}
