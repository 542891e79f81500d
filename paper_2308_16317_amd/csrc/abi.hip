// C ABI of liblsms_tau (declared in include/lsms_tau.h): argument
// validation on the host, the handle's Gaunt tables, and the launches.
#include <cstring>
#include <vector>

#include "../../include/lsms_tau.h"
#include "lsms_common.h"

void lsms_gaunt_host(int lmax, std::vector<int32_t>& row_ptr, std::vector<int16_t>& lpp,
                     std::vector<double>& coef);

namespace {

constexpr int kMaxLmax = 4;
constexpr int kMaxSpeciesAbi = 8;

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

int check_problem(const lsms_problem* p) {
  if (!p) return -2;
  if (p->lmax < 0 || p->lmax > kMaxLmax) return -2;
  if (p->n_inst < 0 || p->n_species < 1 || p->n_species > kMaxSpeciesAbi || p->n_energy < 1) return -2;
  if (p->max_liz < 1) return -2;
  if (p->n_inst > 0 && (!p->liz_off || !p->pos || !p->species || !p->energy || !p->e_idx || !p->delta))
    return -2;
  return 0;
}

lsms_prob_dev to_dev(const lsms_problem* p) {
  lsms_prob_dev d;
  d.lmax = p->lmax;
  d.kk = (p->lmax + 1) * (p->lmax + 1);
  d.n_inst = p->n_inst;
  d.n_species = p->n_species;
  d.n_energy = p->n_energy;
  d.max_liz = p->max_liz;
  d.liz_off = p->liz_off;
  d.pos = p->pos;
  d.species = p->species;
  d.energy = p->energy;
  d.e_idx = p->e_idx;
  d.delta = p->delta;
  return d;
}

int check_opts(const lsms_opts* o, int32_t* nb) {
  *nb = 64;
  if (!o) return 0;
  if (o->precision != LSMS_PREC_FP64) return -1;
  if (o->nb != 0) {
    if (o->nb < 16 || o->nb > 64 || (o->nb % 16) != 0) return -1;
    *nb = o->nb;
  }
  if (o->chunk < 0) return -1;
  return 0;
}

}  // namespace

struct lsms_handle_s {
  int device;
  lsms_gaunt_dev g[kMaxLmax + 1];
  void* mem[kMaxLmax + 1];
};

#define HIP_TRY(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return LSMS_EHIP; \
  } while (0)

extern "C" int lsms_create(lsms_handle_t* out, int device) {
  if (!out) return -1;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return -2;
  HIP_TRY(hipSetDevice(device));
  lsms_handle_s* h = new lsms_handle_s();
  h->device = device;
  for (int lmax = 0; lmax <= kMaxLmax; ++lmax) {
    std::vector<int32_t> rp;
    std::vector<int16_t> lpp;
    std::vector<double> coef;
    lsms_gaunt_host(lmax, rp, lpp, coef);
    const size_t b_rp = rp.size() * sizeof(int32_t), b_c = coef.size() * sizeof(double),
                 b_l = lpp.size() * sizeof(int16_t);
    char* mem = nullptr;
    if (hipMalloc((void**)&mem, b_rp + b_c + b_l + 64) != hipSuccess) {
      for (int q = 0; q < lmax; ++q) (void)hipFree(h->mem[q]);
      delete h;
      return LSMS_EHIP;
    }
    // coef first (8-byte aligned), then row_ptr, then lpp
    (void)hipMemcpy(mem, coef.data(), b_c, hipMemcpyHostToDevice);
    (void)hipMemcpy(mem + b_c, rp.data(), b_rp, hipMemcpyHostToDevice);
    (void)hipMemcpy(mem + b_c + b_rp, lpp.data(), b_l, hipMemcpyHostToDevice);
    h->mem[lmax] = mem;
    h->g[lmax].coef = reinterpret_cast<const double*>(mem);
    h->g[lmax].row_ptr = reinterpret_cast<const int32_t*>(mem + b_c);
    h->g[lmax].lpp = reinterpret_cast<const int16_t*>(mem + b_c + b_rp);
    h->g[lmax].lmax = lmax;
    h->g[lmax].nnz = (int32_t)coef.size();
  }
  if (hipDeviceSynchronize() != hipSuccess) return LSMS_EHIP;
  *out = h;
  return 0;
}

extern "C" int lsms_destroy(lsms_handle_t h) {
  if (!h) return -1;
  (void)hipSetDevice(h->device);
  for (int q = 0; q <= kMaxLmax; ++q) (void)hipFree(h->mem[q]);
  delete h;
  return 0;
}

extern "C" int lsms_build_liz(lsms_handle_t h, const double* atom_pos, const int32_t* atom_species,
                              int32_t n_atoms, const double* box, const int32_t* centre, const double* rc,
                              int32_t n_inst, int32_t max_liz, int32_t* liz_n, int64_t* liz_off, double* liz_pos,
                              int32_t* liz_species, int32_t* liz_atom, void* stream) {
  if (!h) return -1;
  if (n_atoms < 1 || !atom_pos) return -2;
  if (!atom_species) return -3;
  if (!box || !(box[0] > 0.0) || !(box[1] > 0.0) || !(box[2] > 0.0)) return -5;
  if (n_inst < 0) return -8;
  if (n_inst > 0 && !centre) return -6;
  if (n_inst > 0 && !rc) return -7;
  if (max_liz < 1 || max_liz > 1024) return -9;
  if (n_inst > 0 && !liz_n) return -10;
  if (!liz_off) return -11;
  if (n_inst > 0 && !liz_pos) return -12;
  if (n_inst > 0 && !liz_species) return -13;
  (void)hipSetDevice(h->device);
  hipError_t e = lsms_launch_liz(atom_pos, atom_species, n_atoms, box[0], box[1], box[2], centre, rc, n_inst,
                                 max_liz, liz_n, liz_off, liz_pos, liz_species, liz_atom, (hipStream_t)stream);
  return e == hipSuccess ? 0 : LSMS_EHIP;
}

extern "C" int build_kkr(lsms_handle_t h, const lsms_problem* p, double* M, const int64_t* m_off, int32_t* info,
                         void* stream) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (p->n_inst == 0) return 0;
  if (!M) return -3;
  if (!m_off) return -4;
  if (!info) return -5;
  (void)hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  const lsms_prob_dev d = to_dev(p);
  if (fill_i32(info, 0, p->n_inst, s) != hipSuccess) return LSMS_EHIP;
  if (lsms_launch_build(d, h->g[p->lmax], 0, p->n_inst, M, m_off, 0, info, s) != hipSuccess) return LSMS_EHIP;
  return 0;
}

extern "C" int tau00_batched(lsms_handle_t h, const lsms_problem* p, double* M, const int64_t* m_off,
                             const lsms_opts* opts, double* tau00, int32_t* info, void* work, size_t work_bytes,
                             void* stream) {
  (void)work;
  (void)work_bytes;
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  int32_t nb;
  if (check_opts(opts, &nb)) return -5;
  if (p->n_inst == 0) return 0;
  if (!M) return -3;
  if (!m_off) return -4;
  if (!tau00) return -6;
  if (!info) return -7;
  (void)hipSetDevice(h->device);
  const lsms_prob_dev d = to_dev(p);
  if (lsms_launch_lu_fp64(d, 0, p->n_inst, M, m_off, 0, tau00, info, 0, nb, (hipStream_t)stream) != hipSuccess)
    return LSMS_EHIP;
  return 0;
}

static size_t slot_elems(const lsms_problem* p) {
  const size_t kk = (size_t)(p->lmax + 1) * (p->lmax + 1);
  const size_t n = kk * (size_t)p->max_liz;
  return n * n;
}

extern "C" int lsms_workspace_size(lsms_handle_t h, const lsms_problem* p, const lsms_opts* opts, int32_t chunk,
                                   size_t* bytes) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  int32_t nb;
  if (check_opts(opts, &nb)) return -3;
  if (chunk < 1) return -4;
  if (!bytes) return -5;
  *bytes = (size_t)chunk * slot_elems(p) * 16;
  return 0;
}

extern "C" int tau00_solve(lsms_handle_t h, const lsms_problem* p, const lsms_opts* opts, double* tau00,
                           int32_t* info, void* work, size_t work_bytes, void* stream) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  int32_t nb;
  if (check_opts(opts, &nb)) return -3;
  if (p->n_inst == 0) return 0;
  if (!tau00) return -4;
  if (!info) return -5;
  const size_t slot_b = slot_elems(p) * 16;
  if (!work || work_bytes < slot_b) return -7;
  int64_t chunk = (int64_t)(work_bytes / slot_b);
  if (opts && opts->chunk > 0 && opts->chunk < chunk) chunk = opts->chunk;
  (void)hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  const lsms_prob_dev d = to_dev(p);
  if (fill_i32(info, 0, p->n_inst, s) != hipSuccess) return LSMS_EHIP;
  for (int64_t i0 = 0; i0 < p->n_inst; i0 += chunk) {
    const int32_t n = (int32_t)(p->n_inst - i0 < chunk ? p->n_inst - i0 : chunk);
    if (lsms_launch_build(d, h->g[p->lmax], (int32_t)i0, n, (double*)work, nullptr, (int64_t)slot_elems(p), info,
                          s) != hipSuccess)
      return LSMS_EHIP;
    if (lsms_launch_lu_fp64(d, (int32_t)i0, n, (double*)work, nullptr, (int64_t)slot_elems(p), tau00, info, 1, nb,
                            s) != hipSuccess)
      return LSMS_EHIP;
  }
  return 0;
}
