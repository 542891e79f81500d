// Energy integration along the contour (paper Sec. 2.1, eq. Density: the
// density of states and the charge are energy integrals of the Green's
// function, taken by quadrature on a complex contour; Lloyd's formula gives
// the integrated density of states from ln det M).
//
// Both kernels are small reductions over the energy axis of a batch laid out
// [site][energy] (instance s * n_energy + k), the energies in contour order.
#include "lsms_common.h"

using namespace lsms;

namespace {

constexpr int kThreads = 256;

// out[s][c] = sum_k w[k] v[s][k][c], the sum taken in ascending k.  One
// thread per output entry; consecutive threads read consecutive c.
__global__ __launch_bounds__(kThreads) void contour_sum_kernel(int n_sites, int n_energy, int m,
                                                               const zd* __restrict__ w, const zd* __restrict__ v,
                                                               zd* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= (int64_t)n_sites * m) return;
  const int64_t s = q / m, c = q - s * m;
  zd acc = zmake(0.0, 0.0);
  for (int k = 0; k < n_energy; ++k) acc = zadd(acc, zmul(w[k], v[(s * n_energy + k) * m + c]));
  out[q] = acc;
}

// Lloyd's formula along the contour nodes of one site: the multiple-
// scattering integrated density of states relative to the first node,
// N_k - N_0 = -(phi_k - phi_0) / pi, with phi the phase of det M followed
// continuously node by node (each step taken as the difference of the
// principal phases reduced to [-pi, pi], i.e. the phase is assumed to move
// by less than pi between neighbouring nodes).  One thread per site.
__global__ __launch_bounds__(kThreads) void lloyd_idos_kernel(int n_sites, int n_energy,
                                                              const zd* __restrict__ logdet,
                                                              double* __restrict__ idos) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= n_sites) return;
  constexpr double kTwoPi = 6.28318530717958647692;
  constexpr double kPi = 3.14159265358979323846;
  const zd* ld = logdet + (int64_t)s * n_energy;
  double* out = idos + (int64_t)s * n_energy;
  double phi = 0.0, prev = ld[0].y;
  out[0] = 0.0;
  for (int k = 1; k < n_energy; ++k) {
    const double cur = ld[k].y;
    phi += remainder(cur - prev, kTwoPi);
    prev = cur;
    out[k] = -phi / kPi;
  }
}

}  // namespace

hipError_t lsms_launch_contour_sum(int32_t n_sites, int32_t n_energy, int32_t m, const double* w, const double* v,
                                   double* out, hipStream_t s) {
  const int64_t total = (int64_t)n_sites * m;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(contour_sum_kernel, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     n_sites, n_energy, m, reinterpret_cast<const zd*>(w), reinterpret_cast<const zd*>(v),
                     reinterpret_cast<zd*>(out));
  return hipGetLastError();
}

hipError_t lsms_launch_lloyd_idos(int32_t n_sites, int32_t n_energy, const double* logdet, double* idos,
                                  hipStream_t s) {
  if (n_sites <= 0) return hipSuccess;
  hipLaunchKernelGGL(lloyd_idos_kernel, dim3((n_sites + kThreads - 1) / kThreads), dim3(kThreads), 0, s, n_sites,
                     n_energy, reinterpret_cast<const zd*>(logdet), idos);
  return hipGetLastError();
}
