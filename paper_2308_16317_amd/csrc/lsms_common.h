// Device-side helpers shared by the HIP kernels of liblsms_tau (complex FP64
// arithmetic, index maps) and the internal launch interface between the C-ABI
// layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsms {

typedef double2 zd;  // complex FP64, (re, im)

__device__ __forceinline__ zd zmake(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ zd zadd(zd a, zd b) { return zmake(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ zd zsub(zd a, zd b) { return zmake(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ zd zmul(zd a, zd b) { return zmake(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ zd zscale(zd a, double s) { return zmake(a.x * s, a.y * s); }
// a - b*c
__device__ __forceinline__ zd zfms(zd a, zd b, zd c) {
  return zmake(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
__device__ __forceinline__ double zcabs1(zd a) { return fabs(a.x) + fabs(a.y); }
// 1 / a, scaled to avoid overflow in |a|^2
__device__ __forceinline__ zd zinv(zd a) {
  const double s = fmax(fabs(a.x), fabs(a.y));
  const double ar = a.x / s, ai = a.y / s;
  const double d = s * (ar * ar + ai * ai);
  return zmake(ar / d, -ai / d);
}
__device__ __forceinline__ zd zdiv(zd a, zd b) { return zmul(a, zinv(b)); }
// principal square root
__device__ __forceinline__ zd zsqrt(zd z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return zmake(0.0, 0.0);
  if (z.x >= 0.0) {
    const double s = sqrt(0.5 * (r + z.x));
    return zmake(s, z.y / (2.0 * s));
  }
  const double s = sqrt(0.5 * (r - z.x));
  return zmake(fabs(z.y) / (2.0 * s), copysign(s, z.y));
}
// exp(i z)
__device__ __forceinline__ zd zexpi(zd z) {
  double s, c;
  sincos(z.x, &s, &c);
  const double e = exp(-z.y);
  return zmake(e * c, e * s);
}
// single-site t-matrix element t = -(1/kappa) sin(d) e^{i d}
__device__ __forceinline__ zd tmat_from_delta(zd d, zd kap) {
  double sa, ca;
  sincos(d.x, &sa, &ca);
  const double sd = sa * cosh(d.y), cd = ca * sinh(d.y);  // sin(a + ib)
  const zd s = zmake(sd, cd);
  const zd e = zexpi(d);
  const zd se = zmul(s, e);
  const zd q = zdiv(se, kap);
  return zmake(-q.x, -q.y);
}
__device__ __forceinline__ bool zfinite(zd a) { return isfinite(a.x) && isfinite(a.y); }

// Complex FP32 counterparts (same names, float2 arguments), used by the
// FP32 factorisation of the precision form.
typedef float2 zf;
__device__ __forceinline__ zf zmake(float r, float i) { return make_float2(r, i); }
__device__ __forceinline__ zf zmul(zf a, zf b) { return zmake(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ zf zfms(zf a, zf b, zf c) {
  return zmake(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
__device__ __forceinline__ float zcabs1(zf a) { return fabsf(a.x) + fabsf(a.y); }
__device__ __forceinline__ zf zinv(zf a) {
  const float s = fmaxf(fabsf(a.x), fabsf(a.y));
  const float ar = a.x / s, ai = a.y / s;
  const float d = s * (ar * ar + ai * ai);
  return zmake(ar / d, -ai / d);
}

__host__ __device__ __forceinline__ int l_of(int L) {
  int l = 0;
  while ((l + 1) * (l + 1) <= L) ++l;
  return l;
}

}  // namespace lsms

// ---------------------------------------------------------------------------
// Internal launch interface (host functions defined in the kernel TUs).
// ---------------------------------------------------------------------------
struct lsms_gaunt_dev {
  const int32_t* row_ptr;  // [kk*kk + 1], pair index p = L + kk*L'
  const int16_t* lpp;      // L'' of each nonzero
  const double* coef;      // C^{L''}_{LL'} * i^{l-l'+l''} (always real: l-l'+l'' is even)
  int32_t lmax;
  int32_t nnz;
};

struct lsms_prob_dev {
  int32_t lmax, kk, n_inst, n_species, n_energy, max_liz;
  const int64_t* liz_off;
  const double* pos;
  const int32_t* species;
  const double* energy;  // complex
  const int32_t* e_idx;
  const double* delta;   // complex [n_species][n_energy][lmax+1]
  // Spin canting: nspin = 2 doubles every site block (kc = 2 kk rows and
  // columns per LIZ site, index kk s + L within a site); delta then holds the
  // phase shifts of the spin parallel to a site's moment and delta_dn those
  // of the antiparallel spin.  nspin = 1: kc = kk, moment and delta_dn null.
  int32_t nspin, kc;
  const double* moment;    // [liz rows][3] unit moment directions
  const double* delta_dn;  // complex, layout of delta
};

// Global-frame t of one channel of a site with moment e (spin-diagonal
// diag(tu, td) in the site's own frame, rotated by the spin-1/2 rotation
// that takes z to e): t = tbar 1 + dt (e . sigma), tbar = (tu + td)/2,
// dt = (tu - td)/2; t2[2 s + s'] = t_{s s'}.
namespace lsms {
__device__ __forceinline__ void spin_t(zd tu, zd td, double ex, double ey, double ez, zd* t2) {
  const zd tb = zmake(0.5 * (tu.x + td.x), 0.5 * (tu.y + td.y));
  const zd dt = zmake(0.5 * (tu.x - td.x), 0.5 * (tu.y - td.y));
  t2[0] = zmake(tb.x + dt.x * ez, tb.y + dt.y * ez);
  t2[1] = zmul(dt, zmake(ex, -ey));
  t2[2] = zmul(dt, zmake(ex, ey));
  t2[3] = zmake(tb.x - dt.x * ez, tb.y - dt.y * ez);
}
}  // namespace lsms

hipError_t lsms_launch_liz(const double* atom_pos, const int32_t* atom_species, int32_t n_atoms,
                           double bx, double by, double bz, const int32_t* centre, const double* rc,
                           int32_t n_inst, int32_t max_liz, int32_t* liz_n, int64_t* liz_off,
                           double* liz_pos, int32_t* liz_species, int32_t* liz_atom, hipStream_t s);

// Build M for instances [i0, i0 + n) of the problem.  M_i is written at
// M + 2 * moff(i) doubles, where moff(i) = m_off[i] if m_off is non-null and
// (i - i0) * slot otherwise.  info[i] = 0 or -2 (coincident sites).
hipError_t lsms_launch_build(const lsms_prob_dev& p, const lsms_gaunt_dev& g, int32_t i0, int32_t n,
                             double* M, const int64_t* m_off, int64_t slot, int32_t* info,
                             hipStream_t s);

// FP64 LU / Schur elimination and tau00 for instances [i0, i0 + n); M
// addressing as lsms_launch_build.  xgb (or null): per-instance room for two
// 64 x 64 complex blocks at xgb + (i - i0) * xstride complex elements, needed
// for panels wider than 64 (without it panels are at most 64 wide).  If
// keep_info, instances whose info is already nonzero are skipped (tau00
// filled with NaN).
constexpr int64_t kLsmsXgBytes = 2 * 64 * 64 * 16;
hipError_t lsms_launch_lu_fp64(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M,
                               const int64_t* m_off, int64_t slot, double* xgb, int64_t xstride,
                               double* tau00, int32_t* info, int keep_info, int32_t nb, hipStream_t s);

// Persistent fused path: instance order (largest LIZ first), resident grid
// size, and the fused build + elimination launch.  `counter` must be zero at
// launch; slot is the per-workgroup slot in complex elements, the matrix
// first and (xoff > 0) the two 64 x 64 blocks xoff elements in.
// Block row of tau and ln det M (FP64 path on caller-built M, one workgroup
// per instance i0 .. i0+n-1, workspace of lsms_row_slot_bytes per instance
// at work + (i - i0) * slot); row / logdet may be null.
int64_t lsms_row_slot_bytes(const lsms_prob_dev& p);
hipError_t lsms_launch_tau_row(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, const int64_t* m_off,
                               unsigned char* work, const int64_t* row_off, double* row, double* logdet,
                               double* tau00, int32_t* info, int32_t nb, hipStream_t s);
hipError_t lsms_launch_lpt_order(const lsms_prob_dev& p, int32_t* order, hipStream_t s);

// One instance (n_inst = 1, exactly max_liz sites) across the whole GPU:
// workspace bytes, events needed (2 per panel), the launch sequence on the
// streams s0 (the caller's) and s1, and the kernels' LDS attributes.
int64_t lsms_big_work_bytes(const lsms_prob_dev& p);
int lsms_big_events(const lsms_prob_dev& p);
// spin: polls of a grid-barrier wait before it gives up (info -4).
hipError_t lsms_launch_big(const lsms_prob_dev& p, double* M, unsigned char* work, double* tau00, int32_t* info,
                           int32_t nb, int64_t spin, hipStream_t s0, hipStream_t s1, hipEvent_t* ev);
hipError_t lsms_prepare_big_kernels();
// Workgroups of the cooperative panel kernel the device holds at once, and
// the workgroups of the first (largest) panel grid of a problem.
hipError_t lsms_big_resident(int device, int* n);
int lsms_big_panel_groups(const lsms_prob_dev& p);

// out[r][0..2] = src[idx[r]][0..2] (liz.hip): per-row moments of the LIZs.
hipError_t lsms_launch_gather3(int64_t n, const int32_t* idx, const double* src, int32_t n_src, double* out,
                               hipStream_t s);

// Contour quadrature and Lloyd's integrated density of states (contour.hip).
hipError_t lsms_launch_contour_sum(int32_t n_sites, int32_t n_energy, int32_t m, const double* w, const double* v,
                                   double* out, hipStream_t s);
hipError_t lsms_launch_lloyd_idos(int32_t n_sites, int32_t n_energy, const double* logdet, double* idos,
                                  hipStream_t s);
hipError_t lsms_persistent_grid(const lsms_prob_dev& p, int device, int* grid);
hipError_t lsms_launch_persistent(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order,
                                  int32_t* counter, double* work, int64_t slot, int64_t xoff, int grid,
                                  double* tau00, int32_t* info, int32_t nb, hipStream_t s);
hipError_t lsms_prepare_kernels();

// Precision form (FP32 factorisation + FP64 refinement).  extra bytes per
// instance beyond its FP64 matrix; chunked launch (M at (i-i0)*slot complex
// elements, extra buffers at extra + (i-i0)*xslot bytes; instances whose info
// is already nonzero are skipped) and persistent launch (slot_bytes per
// workgroup, FP64 matrix first, its extra buffers m_bytes in).
int64_t lsms_mixed_extra_bytes(const lsms_prob_dev& p);
hipError_t lsms_launch_mixed(const lsms_prob_dev& p, int32_t i0, int32_t n, double* M, int64_t slot,
                             unsigned char* extra, int64_t xslot, double* tau00, int32_t* info, int32_t nb,
                             double tol, int32_t max_refine, hipStream_t s);
hipError_t lsms_mixed_persistent_grid(const lsms_prob_dev& p, int device, int* grid);
hipError_t lsms_launch_mixed_persistent(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order,
                                        int32_t* counter, unsigned char* work, int64_t slot_bytes, int64_t m_bytes,
                                        int grid, double* tau00, int32_t* info, int32_t nb, double tol,
                                        int32_t max_refine, hipStream_t s);

// Learned form, solver: persistent build + block GMRES from a seed (or none)
// + FP64 Schur fallback, lmax = 3.  Slot: [M (m_bytes) | X blocks | Y | R |
// V (m + 1 blocks) | H | G].
int64_t lsms_gmres_extra_bytes(const lsms_prob_dev& p, int m);
int lsms_gmres_max_restart();
hipError_t lsms_gmres_grid(const lsms_prob_dev& p, int device, int* grid);
hipError_t lsms_launch_gmres(const lsms_prob_dev& p, const lsms_gaunt_dev& g, const int32_t* order, int32_t* counter,
                             unsigned char* work, int64_t slot_bytes, int64_t m_bytes, int grid, const double* seed,
                             const double* pc_blk, const int32_t* pc_row, const int8_t* route, double* tau00,
                             int32_t* info, int32_t* steps, int32_t nb, double tol, int max_cycles, int m,
                             hipStream_t s);
// Block index of each LIZ row for the GMRES preconditioner: the instance of
// the batch centred on the row's atom at the row's instance's energy (-1 if
// none); inst_of: n_atoms * n_energy ints of scratch.
hipError_t lsms_launch_site_blocks(const lsms_prob_dev& p, const int32_t* liz_atom, const int32_t* centre,
                                   int32_t n_atoms, int32_t* row, int32_t* inst_of, hipStream_t s);

// Learned form, network (mlp.hip).
int64_t lsms_mlp_param_count();
int64_t lsms_mlp_act_floats();
hipError_t lsms_launch_mlp_features(const lsms_prob_dev& p, double a, float* feat, hipStream_t s);
hipError_t lsms_launch_mlp_forward(const float* params, const uint16_t* wb, const float* feat, int n, float* out,
                                   float* act, hipStream_t s);
hipError_t lsms_launch_mlp_backward(const uint16_t* wb, const float* feat, const float* act, const float* dout,
                                    int n, float* grad, float* work, hipStream_t s);
hipError_t lsms_launch_mlp_mse(const float* out, const float* target, int64_t total, float* dout, float* loss,
                               hipStream_t s);
hipError_t lsms_launch_mlp_adamw(int64_t n, float* w, uint16_t* wb, float* m, float* v, const float* g, float lr,
                                 float b1, float b2, float eps, float wd, int step, hipStream_t s);
hipError_t lsms_launch_mlp_to_bf16(int64_t n, const float* w, uint16_t* wb, hipStream_t s);
hipError_t lsms_launch_mlp_seed(int n, int kk, const float* out, const float* scale, const float* shift, double* seed,
                                hipStream_t s);
hipError_t lsms_launch_mlp_targets(const lsms_prob_dev& p, const double* tau00, const float* scale,
                                   const float* shift, float* target, hipStream_t s);
hipError_t lsms_launch_mlp_norm_stats(int n, const float* target, float* scale, float* shift, hipStream_t s);
