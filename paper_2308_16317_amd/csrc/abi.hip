// C ABI of liblsms_tau (declared in include/lsms_tau.h): argument
// validation on the host, the handle (Gaunt tables, tuned panel widths,
// captured graphs), and the launches.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/lsms_tau.h"
#include "lsms_common.h"

void lsms_gaunt_host(int lmax, std::vector<int32_t>& row_ptr, std::vector<int16_t>& lpp,
                     std::vector<double>& coef);

namespace {

constexpr int kMaxLmax = 4;
constexpr int kMaxSpeciesAbi = 8;
constexpr int kBuckets = 33;     // tuned panel width per 128-wide bucket of N <= 4096 and precision
constexpr int kPrecisions = 2;   // LSMS_PREC_FP64, LSMS_PREC_FP32_IR
constexpr int kGraphCache = 8;

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

// Largest matrix of the FP64 elimination (leaf registers, kR = 16) and of the
// precision form, the learned form and the block-row solve (kR = 8).
constexpr int64_t kMaxN = 8192;        // batched FP64 kernels (register leaves)
constexpr int64_t kMaxNSmall = 4096;   // precision form, GMRES, block row
constexpr int64_t kMaxNLarge = 16384;  // the build and tau00_large

int64_t n_max(const lsms_problem* p, int nspin = 1) {
  return (int64_t)nspin * (p->lmax + 1) * (p->lmax + 1) * p->max_liz;
}

int check_problem(const lsms_problem* p, int nspin = 1, int64_t nmax = kMaxN) {
  if (!p) return -2;
  if (p->lmax < 0 || p->lmax > kMaxLmax) return -2;
  if (p->n_inst < 0 || p->n_species < 1 || p->n_species > kMaxSpeciesAbi || p->n_energy < 1) return -2;
  if (p->max_liz < 1 || p->max_liz > 1024) return -2;
  if (n_max(p, nspin) > nmax) return -2;
  if (p->n_inst > 0 && (!p->liz_off || !p->pos || !p->species || !p->energy || !p->e_idx || !p->delta))
    return -2;
  return 0;
}

// check_problem for the entry points whose kernels hold at most 4096 rows.
int check_problem_small(const lsms_problem* p) {
  const int r = check_problem(p);
  if (r) return r;
  return n_max(p) > kMaxNSmall ? -2 : 0;
}

lsms_prob_dev to_dev(const lsms_problem* p, const lsms_spin* sp = nullptr) {
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
  d.nspin = sp ? 2 : 1;
  d.kc = d.nspin * d.kk;
  d.moment = sp ? sp->moment : nullptr;
  d.delta_dn = sp ? sp->delta_dn : nullptr;
  return d;
}

int check_opts(const lsms_opts* o) {
  if (!o) return 0;
  if (o->precision != LSMS_PREC_FP64 && o->precision != LSMS_PREC_FP32_IR) return -1;
  if (o->max_refine < 0 || o->max_refine > 100 || o->reserved != 0) return -1;
  if (!(o->tol == 0.0 || (o->tol >= 1e-15 && o->tol <= 1e-3))) return -1;
  if (o->nb != 0 && (o->nb < 16 || o->nb > 128 || (o->nb % 16) != 0)) return -1;
  if (o->chunk < 0) return -1;
  if (o->flags & ~(LSMS_PERSISTENT | LSMS_GRAPH)) return -1;
  return 0;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t slot_elems(const lsms_problem* p, const lsms_spin* sp = nullptr) {
  const size_t n = (size_t)n_max(p, sp ? 2 : 1);
  return n * n;
}

bool mixed(const lsms_opts* o) { return o && o->precision == LSMS_PREC_FP32_IR; }

// Bytes of one instance slot: the FP64 matrix (256-byte aligned), then the
// two 64 x 64 blocks of wide panels (FP64 form) or the buffers of the
// precision form (which include those blocks).
size_t m_bytes(const lsms_problem* p, const lsms_spin* sp = nullptr) { return align256(slot_elems(p, sp) * 16); }

size_t slot_bytes(const lsms_problem* p, const lsms_opts* o, const lsms_spin* sp = nullptr) {
  return m_bytes(p, sp) + (mixed(o) ? (size_t)lsms_mixed_extra_bytes(to_dev(p)) : (size_t)kLsmsXgBytes);
}

double ir_tol(const lsms_opts* o) { return o->tol > 0.0 ? o->tol : 1e-12; }
int32_t ir_steps(const lsms_opts* o) { return o->max_refine > 0 ? o->max_refine : 10; }

int bucket_of(int64_t n) { return (int)((n + 127) / 128 < kBuckets ? (n + 127) / 128 : kBuckets - 1); }

struct GraphEntry {
  bool used;
  lsms_problem prob;
  lsms_opts opts;
  int32_t nb;  // panel width resolved at capture (opts->nb or the tuned value)
  double* tau00;
  int32_t* info;
  void* work;
  size_t work_bytes;
  hipGraphExec_t exec;
  uint64_t stamp;
};

// Scratch of tau00_batched_noalloc: room for the inverses of the two 64 x 64
// diagonal blocks of a wide panel for kNoAllocSlots instances (one pass of
// the batch).  Host code never passes the array's name to a kernel: it uses
// the device address taken once per device by scratch_setup.
constexpr int kNoAllocSlots = 256;
constexpr size_t kScratchBytes = (size_t)kNoAllocSlots * kLsmsXgBytes;  // 32 MiB
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on `device` (which must be current),
// taken on the first call for that device.  Returns 0 or LSMS_EHIP.
int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return LSMS_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return 0;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LSMS_EHIP;
  g_scratch_ptr[device] = ptr;
  return 0;
}

}  // namespace

struct lsms_handle_s {
  int device;
  void* scratch;  // this device's address of the scratch array
  lsms_gaunt_dev g[kMaxLmax + 1];
  void* mem[kMaxLmax + 1];
  int32_t tuned_nb[kPrecisions][kBuckets];
  GraphEntry graphs[kGraphCache];
  uint64_t clock;
  // tau00_large: the second stream of its look-ahead and its events (made on
  // the first call)
  hipStream_t aux = nullptr;
  std::vector<hipEvent_t> big_ev;
  int64_t big_spin = 0;  // polls of a grid-barrier wait, 0 = default
  int big_resident = 0;  // panel workgroups the device holds at once
};

#define HIP_TRY(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return LSMS_EHIP; \
  } while (0)

namespace {

int prec_index(const lsms_opts* o) { return mixed(o) ? 1 : 0; }

int32_t panel_width(const lsms_handle_s* h, const lsms_problem* p, const lsms_opts* o,
                    const lsms_spin* sp = nullptr) {
  if (o && o->nb) return o->nb;
  const int32_t t = h->tuned_nb[prec_index(o)][bucket_of(n_max(p, sp ? 2 : 1))];
  return t ? t : 128;
}

struct PersistLayout {
  int grid;
  size_t order_off, slots_off, slot_stride, total;  // bytes
};

int persist_layout(const lsms_handle_s* h, const lsms_problem* p, const lsms_opts* o, PersistLayout* L,
                   const lsms_spin* sp = nullptr) {
  const lsms_prob_dev d = to_dev(p, sp);
  const hipError_t e = mixed(o) ? lsms_mixed_persistent_grid(d, h->device, &L->grid)
                                : lsms_persistent_grid(d, h->device, &L->grid);
  if (e != hipSuccess) return LSMS_EHIP;
  // no more resident workgroups (and slots) than instances
  if (L->grid > p->n_inst) L->grid = p->n_inst > 0 ? p->n_inst : 1;
  L->order_off = 256;
  L->slots_off = align256(256 + 4 * (size_t)p->n_inst);
  L->slot_stride = slot_bytes(p, o, sp);
  L->total = L->slots_off + (size_t)L->grid * L->slot_stride;
  return 0;
}

// Enqueue the launches of one tau00_solve call (no graph handling); sp: spin
// canting (FP64 only), or null.
int enqueue_solve(lsms_handle_s* h, const lsms_problem* p, const lsms_opts* o, double* tau00, int32_t* info,
                  void* work, size_t work_bytes, hipStream_t s, const lsms_spin* sp = nullptr) {
  const lsms_prob_dev d = to_dev(p, sp);
  const int32_t nb = panel_width(h, p, o, sp);
  if (o && (o->flags & LSMS_PERSISTENT)) {
    PersistLayout L;
    if (persist_layout(h, p, o, &L, sp)) return LSMS_EHIP;
    if (work_bytes < L.total) return -7;
    char* w = (char*)work;
    int32_t* counter = (int32_t*)w;
    int32_t* order = (int32_t*)(w + L.order_off);
    if (fill_i32(counter, 0, 1, s) != hipSuccess) return LSMS_EHIP;
    if (lsms_launch_lpt_order(d, order, s) != hipSuccess) return LSMS_EHIP;
    const hipError_t e =
        mixed(o) ? lsms_launch_mixed_persistent(d, h->g[p->lmax], order, counter, (unsigned char*)(w + L.slots_off),
                                                (int64_t)L.slot_stride, (int64_t)m_bytes(p), L.grid, tau00, info, nb,
                                                ir_tol(o), ir_steps(o), s)
                 : lsms_launch_persistent(d, h->g[p->lmax], order, counter, (double*)(w + L.slots_off),
                                          (int64_t)(L.slot_stride / 16), (int64_t)(m_bytes(p, sp) / 16), L.grid,
                                          tau00, info, nb, s);
    return e == hipSuccess ? 0 : LSMS_EHIP;
  }
  // chunked: M slots first, then the per-instance extra buffers
  const size_t mb = m_bytes(p, sp), slot_b = slot_bytes(p, o, sp);
  if (work_bytes < slot_b) return -7;
  int64_t chunk = (int64_t)(work_bytes / slot_b);
  if (o && o->chunk > 0 && o->chunk < chunk) chunk = o->chunk;
  unsigned char* extra = (unsigned char*)work + (size_t)chunk * mb;
  const int64_t xslot = (int64_t)(slot_b - mb);
  if (fill_i32(info, 0, p->n_inst, s) != hipSuccess) return LSMS_EHIP;
  for (int64_t i0 = 0; i0 < p->n_inst; i0 += chunk) {
    const int32_t n = (int32_t)(p->n_inst - i0 < chunk ? p->n_inst - i0 : chunk);
    if (lsms_launch_build(d, h->g[p->lmax], (int32_t)i0, n, (double*)work, nullptr, (int64_t)(mb / 16), info, s) !=
        hipSuccess)
      return LSMS_EHIP;
    const hipError_t e =
        mixed(o) ? lsms_launch_mixed(d, (int32_t)i0, n, (double*)work, (int64_t)(mb / 16), extra, xslot, tau00, info,
                                     nb, ir_tol(o), ir_steps(o), s)
                 : lsms_launch_lu_fp64(d, (int32_t)i0, n, (double*)work, nullptr, (int64_t)(mb / 16), (double*)extra,
                                       xslot / 16, tau00, info, 1, nb, s);
    if (e != hipSuccess) return LSMS_EHIP;
  }
  return 0;
}

bool same_args(const GraphEntry& e, const lsms_problem* p, const lsms_opts* o, int32_t nb, double* tau00,
               int32_t* info, void* work, size_t work_bytes) {
  return e.used && std::memcmp(&e.prob, p, sizeof(lsms_problem)) == 0 &&
         std::memcmp(&e.opts, o, sizeof(lsms_opts)) == 0 && e.nb == nb && e.tau00 == tau00 && e.info == info &&
         e.work == work && e.work_bytes == work_bytes;
}

}  // namespace

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
  if (lsms_prepare_kernels() != hipSuccess || lsms_prepare_big_kernels() != hipSuccess ||
      scratch_setup(device) != 0 || hipDeviceSynchronize() != hipSuccess) {
    for (int q = 0; q <= kMaxLmax; ++q) (void)hipFree(h->mem[q]);
    delete h;
    return LSMS_EHIP;
  }
  h->scratch = g_scratch_ptr[device];
  if (lsms_big_resident(device, &h->big_resident) != hipSuccess) h->big_resident = 0;
  *out = h;
  return 0;
}

extern "C" int lsms_destroy(lsms_handle_t h) {
  if (!h) return -1;
  (void)hipSetDevice(h->device);
  for (int q = 0; q < kGraphCache; ++q)
    if (h->graphs[q].used) (void)hipGraphExecDestroy(h->graphs[q].exec);
  for (int q = 0; q <= kMaxLmax; ++q) (void)hipFree(h->mem[q]);
  for (hipEvent_t e : h->big_ev) (void)hipEventDestroy(e);
  if (h->aux) (void)hipStreamDestroy(h->aux);
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
  int r = check_problem(p, 1, kMaxNLarge);
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
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (check_opts(opts) || mixed(opts)) return -5;
  if (p->n_inst == 0) return 0;
  if (!M) return -3;
  if (!m_off) return -4;
  if (!tau00) return -6;
  if (!info) return -7;
  if (work && work_bytes < (size_t)p->n_inst * kLsmsXgBytes) return -9;
  (void)hipSetDevice(h->device);
  const lsms_prob_dev d = to_dev(p);
  if (lsms_launch_lu_fp64(d, 0, p->n_inst, M, m_off, 0, (double*)work, work ? kLsmsXgBytes / 16 : 0, tau00, info,
                          0, panel_width(h, p, opts), (hipStream_t)stream) != hipSuccess)
    return LSMS_EHIP;
  return 0;
}

extern "C" int lsms_row_workspace_size(lsms_handle_t h, const lsms_problem* p, size_t* bytes) {
  if (!h) return -1;
  int r = check_problem_small(p);
  if (r) return r;
  if (!bytes) return -3;
  *bytes = (size_t)p->n_inst * (size_t)lsms_row_slot_bytes(to_dev(p));
  return 0;
}

extern "C" int tau_row_batched(lsms_handle_t h, const lsms_problem* p, double* M, const int64_t* m_off,
                               const lsms_opts* opts, const int64_t* row_off, double* tau_row, double* logdet,
                               double* tau00, int32_t* info, void* work, size_t work_bytes, void* stream) {
  if (!h) return -1;
  int r = check_problem_small(p);
  if (r) return r;
  if (check_opts(opts) || mixed(opts)) return -5;
  if (p->n_inst == 0) return 0;
  if (!M) return -3;
  if (!m_off) return -4;
  if (tau_row && !row_off) return -6;
  if (!tau00) return -9;
  if (!info) return -10;
  if (!work) return -11;
  if (work_bytes < (size_t)p->n_inst * (size_t)lsms_row_slot_bytes(to_dev(p))) return -12;
  (void)hipSetDevice(h->device);
  const lsms_prob_dev d = to_dev(p);
  if (lsms_launch_tau_row(d, 0, p->n_inst, M, m_off, (unsigned char*)work, row_off, tau_row, logdet, tau00, info,
                          panel_width(h, p, opts), (hipStream_t)stream) != hipSuccess)
    return LSMS_EHIP;
  return 0;
}

extern "C" int lsms_contour_sum(lsms_handle_t h, int32_t n_sites, int32_t n_energy, int32_t m,
                                const double* weights, const double* values, double* out, void* stream) {
  if (!h) return -1;
  if (n_sites < 0) return -2;
  if (n_energy < 1) return -3;
  if (m < 0) return -4;
  if ((int64_t)n_sites * m == 0) return 0;
  if (!weights) return -5;
  if (!values) return -6;
  if (!out) return -7;
  (void)hipSetDevice(h->device);
  return lsms_launch_contour_sum(n_sites, n_energy, m, weights, values, out, (hipStream_t)stream) == hipSuccess
             ? 0
             : LSMS_EHIP;
}

extern "C" int lsms_lloyd_idos(lsms_handle_t h, int32_t n_sites, int32_t n_energy, const double* logdet,
                               double* idos, void* stream) {
  if (!h) return -1;
  if (n_sites < 0) return -2;
  if (n_energy < 1) return -3;
  if (n_sites == 0) return 0;
  if (!logdet) return -4;
  if (!idos) return -5;
  (void)hipSetDevice(h->device);
  return lsms_launch_lloyd_idos(n_sites, n_energy, logdet, idos, (hipStream_t)stream) == hipSuccess ? 0 : LSMS_EHIP;
}

// ---------------------------------------------------------- spin canting
int check_spin(const lsms_problem* p, const lsms_spin* sp) {
  if (!sp) return -3;
  if (p->n_inst > 0 && (!sp->moment || !sp->delta_dn)) return -3;
  return 0;
}

extern "C" int lsms_liz_moments(lsms_handle_t h, int64_t n_rows, const int32_t* liz_atom,
                                const double* atom_moment, int32_t n_atoms, double* liz_moment, void* stream) {
  if (!h) return -1;
  if (n_rows < 0) return -2;
  if (n_rows == 0) return 0;
  if (!liz_atom) return -3;
  if (!atom_moment) return -4;
  if (n_atoms < 1) return -5;
  if (!liz_moment) return -6;
  (void)hipSetDevice(h->device);
  return lsms_launch_gather3(n_rows, liz_atom, atom_moment, n_atoms, liz_moment, (hipStream_t)stream) == hipSuccess
             ? 0
             : LSMS_EHIP;
}

extern "C" int build_kkr_spin(lsms_handle_t h, const lsms_problem* p, const lsms_spin* spin, double* M,
                              const int64_t* m_off, int32_t* info, void* stream) {
  if (!h) return -1;
  int r = check_problem(p, 2, kMaxNLarge);
  if (r) return r;
  if ((r = check_spin(p, spin))) return r;
  if (p->n_inst == 0) return 0;
  if (!M) return -4;
  if (!m_off) return -5;
  if (!info) return -6;
  (void)hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  const lsms_prob_dev d = to_dev(p, spin);
  if (fill_i32(info, 0, p->n_inst, s) != hipSuccess) return LSMS_EHIP;
  if (lsms_launch_build(d, h->g[p->lmax], 0, p->n_inst, M, m_off, 0, info, s) != hipSuccess) return LSMS_EHIP;
  return 0;
}

extern "C" int tau00_spin_batched(lsms_handle_t h, const lsms_problem* p, const lsms_spin* spin, double* M,
                                  const int64_t* m_off, const lsms_opts* opts, double* tau00, int32_t* info,
                                  void* work, size_t work_bytes, void* stream) {
  if (!h) return -1;
  int r = check_problem(p, 2);
  if (r) return r;
  if ((r = check_spin(p, spin))) return r;
  if (check_opts(opts) || mixed(opts)) return -6;
  if (p->n_inst == 0) return 0;
  if (!M) return -4;
  if (!m_off) return -5;
  if (!tau00) return -7;
  if (!info) return -8;
  if (work && work_bytes < (size_t)p->n_inst * kLsmsXgBytes) return -10;
  (void)hipSetDevice(h->device);
  const lsms_prob_dev d = to_dev(p, spin);
  if (lsms_launch_lu_fp64(d, 0, p->n_inst, M, m_off, 0, (double*)work, work ? kLsmsXgBytes / 16 : 0, tau00, info,
                          0, panel_width(h, p, opts, spin), (hipStream_t)stream) != hipSuccess)
    return LSMS_EHIP;
  return 0;
}

extern "C" int lsms_spin_workspace_size(lsms_handle_t h, const lsms_problem* p, const lsms_spin* spin,
                                        const lsms_opts* opts, int32_t chunk, size_t* bytes) {
  if (!h) return -1;
  int r = check_problem(p, 2);
  if (r) return r;
  if ((r = check_spin(p, spin))) return r;
  if (check_opts(opts) || mixed(opts) || (opts && (opts->flags & LSMS_GRAPH))) return -4;
  if (!bytes) return -6;
  if (opts && (opts->flags & LSMS_PERSISTENT)) {
    (void)hipSetDevice(h->device);
    PersistLayout L;
    if (persist_layout(h, p, opts, &L, spin)) return LSMS_EHIP;
    *bytes = L.total;
    return 0;
  }
  if (chunk < 1) return -5;
  *bytes = (size_t)chunk * slot_bytes(p, opts, spin);
  return 0;
}

extern "C" int tau00_spin_solve(lsms_handle_t h, const lsms_problem* p, const lsms_spin* spin,
                                const lsms_opts* opts, double* tau00, int32_t* info, void* work, size_t work_bytes,
                                void* stream) {
  if (!h) return -1;
  int r = check_problem(p, 2);
  if (r) return r;
  if ((r = check_spin(p, spin))) return r;
  if (check_opts(opts) || mixed(opts) || (opts && (opts->flags & LSMS_GRAPH))) return -4;
  if (p->n_inst == 0) return 0;
  if (!tau00) return -5;
  if (!info) return -6;
  if (!work) return -7;
  (void)hipSetDevice(h->device);
  const int er = enqueue_solve(h, p, opts, tau00, info, work, work_bytes, (hipStream_t)stream, spin);
  return er == -7 ? -8 : er;
}

// ------------------------------------------------ one instance, whole GPU
constexpr int64_t kBigSpinDefault = int64_t(1) << 22;  // polls (each with a short sleep): seconds
int check_large(const lsms_problem* p, const lsms_spin* spin, const lsms_opts* opts) {
  int r = check_problem(p, spin ? 2 : 1, kMaxNLarge);
  if (r) return r;
  if (p->n_inst != 1) return -2;
  if (spin && (r = check_spin(p, spin))) return r;
  if (check_opts(opts) || mixed(opts) || (opts && opts->nb != 0 && opts->nb != 64) || (opts && opts->flags))
    return -5;
  return 0;
}

extern "C" int lsms_large_workspace_size(lsms_handle_t h, const lsms_problem* p, const lsms_spin* spin,
                                         size_t* bytes) {
  if (!h) return -1;
  const int r = check_large(p, spin, nullptr);
  if (r) return r;
  if (!bytes) return -4;
  *bytes = (size_t)lsms_big_work_bytes(to_dev(p, spin));
  return 0;
}

extern "C" int tau00_large(lsms_handle_t h, const lsms_problem* p, const lsms_spin* spin, double* M,
                           const lsms_opts* opts, double* tau00, int32_t* info, void* work, size_t work_bytes,
                           void* stream) {
  if (!h) return -1;
  const int r = check_large(p, spin, opts);
  if (r) return r;
  if (!M) return -4;
  if (!tau00) return -6;
  if (!info) return -7;
  if (!work) return -8;
  const lsms_prob_dev d = to_dev(p, spin);
  if (work_bytes < (size_t)lsms_big_work_bytes(d)) return -9;
  // every workgroup of the first (largest) panel grid must be resident at
  // once for its grid barriers
  if (lsms_big_panel_groups(d) > h->big_resident) return -10;
  (void)hipSetDevice(h->device);
  if (!h->aux && hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess) {
    h->aux = nullptr;
    return LSMS_EHIP;
  }
  const size_t nev = (size_t)lsms_big_events(d);
  while (h->big_ev.size() < nev) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return LSMS_EHIP;
    h->big_ev.push_back(e);
  }
  const int64_t polls = h->big_spin > 0 ? h->big_spin : kBigSpinDefault;
  return lsms_launch_big(d, M, (unsigned char*)work, tau00, info, 64, polls, (hipStream_t)stream, h->aux,
                         h->big_ev.data()) == hipSuccess
             ? 0
             : LSMS_EHIP;
}

extern "C" int lsms_large_set_spin_limit(lsms_handle_t h, int64_t polls) {
  if (!h) return -1;
  if (polls < 0) return -2;
  h->big_spin = polls;
  return 0;
}

// The allocation-free variant of tau00_batched: the same kernels, the
// wide-panel blocks in the handle device's scratch array, the batch in
// passes of kNoAllocSlots instances (stream-ordered, so each pass reuses the
// array).  Enqueues kernel launches only.
extern "C" int tau00_batched_noalloc(lsms_handle_t h, const lsms_problem* p, double* M, const int64_t* m_off,
                                     const lsms_opts* opts, double* tau00, int32_t* info, void* stream) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (check_opts(opts) || mixed(opts)) return -5;
  if (p->n_inst == 0) return 0;
  if (!M) return -3;
  if (!m_off) return -4;
  if (!tau00) return -6;
  if (!info) return -7;
  if (!h->scratch) return LSMS_EHIP;
  (void)hipSetDevice(h->device);
  const lsms_prob_dev d = to_dev(p);
  const int32_t nb = panel_width(h, p, opts);
  for (int32_t i0 = 0; i0 < p->n_inst; i0 += kNoAllocSlots) {
    const int32_t n = p->n_inst - i0 < kNoAllocSlots ? p->n_inst - i0 : kNoAllocSlots;
    // the kernel addresses the scratch of instance i at (i - i0) * stride
    if (lsms_launch_lu_fp64(d, i0, n, M, m_off, 0, (double*)h->scratch, kLsmsXgBytes / 16, tau00, info, 0, nb,
                            (hipStream_t)stream) != hipSuccess)
      return LSMS_EHIP;
  }
  return 0;
}

extern "C" int lsms_workspace_size(lsms_handle_t h, const lsms_problem* p, const lsms_opts* opts, int32_t chunk,
                                   size_t* bytes) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (check_opts(opts)) return -3;
  if (mixed(opts) && n_max(p) > kMaxNSmall) return -2;
  if (!bytes) return -5;
  if (opts && (opts->flags & LSMS_PERSISTENT)) {
    (void)hipSetDevice(h->device);
    PersistLayout L;
    if (persist_layout(h, p, opts, &L)) return LSMS_EHIP;
    *bytes = L.total;
    return 0;
  }
  if (chunk < 1) return -4;
  *bytes = (size_t)chunk * slot_bytes(p, opts);
  return 0;
}

extern "C" int tau00_solve(lsms_handle_t h, const lsms_problem* p, const lsms_opts* opts, double* tau00,
                           int32_t* info, void* work, size_t work_bytes, void* stream) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (check_opts(opts)) return -3;
  if (mixed(opts) && n_max(p) > kMaxNSmall) return -2;
  if (p->n_inst == 0) return 0;
  if (!tau00) return -4;
  if (!info) return -5;
  if (!work) return -6;
  (void)hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  const bool graph = opts && (opts->flags & LSMS_GRAPH) && s != nullptr;
  if (!graph) return enqueue_solve(h, p, opts, tau00, info, work, work_bytes, s);

  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return LSMS_EHIP;
  if (cs != hipStreamCaptureStatusNone) return enqueue_solve(h, p, opts, tau00, info, work, work_bytes, s);
  // the key holds the resolved panel width: a graph captured before the
  // tuned width changed is not replayed after
  const int32_t nb = panel_width(h, p, opts);
  GraphEntry* hit = nullptr;
  for (int q = 0; q < kGraphCache; ++q)
    if (same_args(h->graphs[q], p, opts, nb, tau00, info, work, work_bytes)) hit = &h->graphs[q];
  if (!hit) {
    // check the arguments outside the capture (errors must not leave a capture open)
    if (opts->flags & LSMS_PERSISTENT) {
      PersistLayout L;
      if (persist_layout(h, p, opts, &L)) return LSMS_EHIP;
      if (work_bytes < L.total) return -7;
    } else if (work_bytes < slot_bytes(p, opts)) {
      return -7;
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return LSMS_EHIP;
    const int er = enqueue_solve(h, p, opts, tau00, info, work, work_bytes, s);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &g);
    if (er != 0 || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return er != 0 ? er : LSMS_EHIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return LSMS_EHIP;
    GraphEntry* slot = &h->graphs[0];
    for (int q = 0; q < kGraphCache; ++q) {
      if (!h->graphs[q].used) {
        slot = &h->graphs[q];
        break;
      }
      if (h->graphs[q].stamp < slot->stamp) slot = &h->graphs[q];
    }
    if (slot->used) (void)hipGraphExecDestroy(slot->exec);
    slot->used = true;
    slot->prob = *p;
    slot->opts = *opts;
    slot->nb = nb;
    slot->tau00 = tau00;
    slot->info = info;
    slot->work = work;
    slot->work_bytes = work_bytes;
    slot->exec = exec;
    hit = slot;
  }
  hit->stamp = ++h->clock;
  return hipGraphLaunch(hit->exec, s) == hipSuccess ? 0 : LSMS_EHIP;
}

extern "C" int lsms_set_tuned_nb(lsms_handle_t h, int32_t n, int32_t precision, int32_t nb) {
  if (!h) return -1;
  if (n < 1 || n > 4096) return -2;
  if (precision != LSMS_PREC_FP64 && precision != LSMS_PREC_FP32_IR) return -3;
  if (nb < 16 || nb > 128 || nb % 16) return -4;
  h->tuned_nb[precision][bucket_of(n)] = nb;
  return 0;
}

extern "C" int lsms_get_tuned_nb(lsms_handle_t h, int32_t n, int32_t precision, int32_t* nb) {
  if (!h) return -1;
  if (n < 1 || n > 4096) return -2;
  if (precision != LSMS_PREC_FP64 && precision != LSMS_PREC_FP32_IR) return -3;
  if (!nb) return -4;
  *nb = h->tuned_nb[precision][bucket_of(n)];
  return 0;
}

extern "C" int lsms_autotune(lsms_handle_t h, const lsms_problem* p, const lsms_opts* opts, double* tau00,
                             int32_t* info, void* work, size_t work_bytes, void* stream, int32_t* best_nb,
                             double* ms_out) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (check_opts(opts)) return -3;
  if (mixed(opts) && n_max(p) > kMaxNSmall) return -2;
  if (!best_nb) return -9;
  (void)hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  lsms_opts o = opts ? *opts : lsms_opts{LSMS_PREC_FP64, 0, 0, 0, 0, 0, 0.0};
  o.flags &= ~LSMS_GRAPH;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int32_t cand[4] = {32, 64, 96, 128};
  constexpr int kSamples = 3;
  int32_t best = 128;
  float best_ms = 0.0f;
  for (int c = 0; c < 4; ++c) {
    o.nb = cand[c];
    int er = tau00_solve(h, p, &o, tau00, info, work, work_bytes, stream);  // warm-up
    if (er) return er;
    float t[kSamples];
    for (int k = 0; k < kSamples; ++k) {
      HIP_TRY(hipEventRecord(e0, s));
      er = tau00_solve(h, p, &o, tau00, info, work, work_bytes, stream);
      if (er) return er;
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(&t[k], e0, e1));
    }
    std::sort(t, t + kSamples);
    const float ms = t[kSamples / 2];  // median of the samples
    if (ms_out) ms_out[c] = ms;
    if (c == 0 || ms < best_ms) {
      best_ms = ms;
      best = cand[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->tuned_nb[prec_index(&o)][bucket_of((int64_t)(p->lmax + 1) * (p->lmax + 1) * p->max_liz)] = best;
  *best_nb = best;
  return 0;
}

// Tuning cache file: a JSON array with one object per line,
//   {"n_max": 2176, "precision": 0, "nb": 128}
// (n_max the upper end of the 128-wide bucket of N).  lsms_autotune_load reads
// the lines of that form (as lsms_autotune_save writes them) and ignores
// every other line.
extern "C" int lsms_autotune_save(lsms_handle_t h, const char* path) {
  if (!h) return -1;
  if (!path) return -2;
  FILE* f = std::fopen(path, "w");
  if (!f) return -2;
  std::fprintf(f, "[\n");
  bool first = true;
  for (int pr = 0; pr < kPrecisions; ++pr)
    for (int b = 0; b < kBuckets; ++b)
      if (h->tuned_nb[pr][b]) {
        std::fprintf(f, "%s{\"n_max\": %d, \"precision\": %d, \"nb\": %d}", first ? "" : ",\n",
                     b == 0 ? 1 : 128 * b, pr, h->tuned_nb[pr][b]);
        first = false;
      }
  std::fprintf(f, "%s]\n", first ? "" : "\n");
  return std::fclose(f) == 0 ? 0 : -2;
}

extern "C" int lsms_autotune_load(lsms_handle_t h, const char* path, int32_t* n_loaded) {
  if (!h) return -1;
  if (!path) return -2;
  FILE* f = std::fopen(path, "r");
  if (!f) return -2;
  char line[256];
  int n = 0;
  while (std::fgets(line, sizeof line, f)) {
    int nmax = 0, pr = -1, nb = 0;
    const char* q = std::strchr(line, '{');
    if (!q || std::sscanf(q, "{\"n_max\": %d, \"precision\": %d, \"nb\": %d}", &nmax, &pr, &nb) != 3) continue;
    if (nmax < 1 || nmax > 4096 || (pr != 0 && pr != 1) || nb < 16 || nb > 128 || nb % 16) continue;
    h->tuned_nb[pr][bucket_of(nmax)] = nb;
    ++n;
  }
  std::fclose(f);
  if (n_loaded) *n_loaded = n;
  return 0;
}

// ---------------------------------------------------------------- learned form

namespace {

struct GmresLayout {
  int grid;
  size_t order_off, slots_off, slot_stride, total;
};

int gmres_layout(const lsms_handle_s* h, const lsms_problem* p, int restart, GmresLayout* L) {
  const lsms_prob_dev d = to_dev(p);
  if (lsms_gmres_grid(d, h->device, &L->grid) != hipSuccess) return LSMS_EHIP;
  if (L->grid > p->n_inst) L->grid = p->n_inst > 0 ? p->n_inst : 1;
  L->order_off = 256;
  L->slots_off = align256(256 + 4 * (size_t)p->n_inst);
  L->slot_stride = m_bytes(p) + (size_t)lsms_gmres_extra_bytes(d, restart);
  L->total = L->slots_off + (size_t)L->grid * L->slot_stride;
  return 0;
}

}  // namespace

extern "C" int lsms_gmres_workspace_size(lsms_handle_t h, const lsms_problem* p, int32_t restart, size_t* bytes) {
  if (!h) return -1;
  int r = check_problem_small(p);
  if (r) return r;
  if (p->lmax != 3) return -2;
  if (restart < 1 || restart > lsms_gmres_max_restart()) return -3;
  if (!bytes) return -4;
  (void)hipSetDevice(h->device);
  GmresLayout L;
  if (gmres_layout(h, p, restart, &L)) return LSMS_EHIP;
  *bytes = L.total;
  return 0;
}

extern "C" int tau00_gmres_pc(lsms_handle_t h, const lsms_problem* p, const double* seed, const double* precond,
                              const int32_t* precond_row, const int8_t* route, int32_t restart, int32_t max_cycles,
                              double tol, double* tau00, int32_t* info, int32_t* steps, void* work,
                              size_t work_bytes, void* stream);

extern "C" int tau00_gmres(lsms_handle_t h, const lsms_problem* p, const double* seed, int32_t restart,
                           int32_t max_cycles, double tol, double* tau00, int32_t* info, int32_t* steps, void* work,
                           size_t work_bytes, void* stream) {
  const int r = tau00_gmres_pc(h, p, seed, nullptr, nullptr, nullptr, restart, max_cycles, tol, tau00, info, steps,
                               work, work_bytes, stream);
  return (r <= -7 && r >= -14) ? r + 3 : r;  // argument numbers of this signature
}

extern "C" int lsms_site_blocks(lsms_handle_t h, const lsms_problem* p, const int32_t* liz_atom,
                                const int32_t* centre, int32_t n_atoms, int32_t* precond_row, int32_t* work,
                                void* stream) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (p->n_inst == 0) return 0;
  if (!liz_atom) return -3;
  if (!centre) return -4;
  if (n_atoms < 1) return -5;
  if (!precond_row) return -6;
  if (!work) return -7;
  (void)hipSetDevice(h->device);
  return lsms_launch_site_blocks(to_dev(p), liz_atom, centre, n_atoms, precond_row, work, (hipStream_t)stream) ==
                 hipSuccess
             ? 0
             : LSMS_EHIP;
}

extern "C" int tau00_gmres_pc(lsms_handle_t h, const lsms_problem* p, const double* seed, const double* precond,
                              const int32_t* precond_row, const int8_t* route, int32_t restart, int32_t max_cycles,
                              double tol, double* tau00, int32_t* info, int32_t* steps, void* work,
                              size_t work_bytes, void* stream) {
  if (!h) return -1;
  int r = check_problem_small(p);
  if (r) return r;
  if (p->lmax != 3) return -2;
  if (restart < 1 || restart > lsms_gmres_max_restart()) return -7;
  if (precond && !precond_row) return -5;
  if (max_cycles < 0 || max_cycles > 1000) return -8;
  if (!(tol > 0.0 && tol < 1.0)) return -9;
  if (p->n_inst == 0) return 0;
  if (!tau00) return -10;
  if (!info) return -11;
  if (!steps) return -12;
  if (!work) return -13;
  (void)hipSetDevice(h->device);
  hipStream_t s = (hipStream_t)stream;
  GmresLayout L;
  if (gmres_layout(h, p, restart, &L)) return LSMS_EHIP;
  if (work_bytes < L.total) return -14;
  const lsms_prob_dev d = to_dev(p);
  char* w = (char*)work;
  int32_t* counter = (int32_t*)w;
  int32_t* order = (int32_t*)(w + L.order_off);
  if (fill_i32(counter, 0, 1, s) != hipSuccess) return LSMS_EHIP;
  if (lsms_launch_lpt_order(d, order, s) != hipSuccess) return LSMS_EHIP;
  if (lsms_launch_gmres(d, h->g[p->lmax], order, counter, (unsigned char*)(w + L.slots_off), (int64_t)L.slot_stride,
                        (int64_t)m_bytes(p), L.grid, seed, precond_row ? precond : nullptr, precond_row, route,
                        tau00, info, steps, panel_width(h, p, nullptr), tol,
                        max_cycles, restart, s) != hipSuccess)
    return LSMS_EHIP;
  return 0;
}

extern "C" int lsms_mlp_features(lsms_handle_t h, const lsms_problem* p, double a_lat, float* feat, void* stream) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (!(a_lat > 0.0)) return -3;
  if (p->n_inst == 0) return 0;
  if (!feat) return -4;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_features(to_dev(p), a_lat, feat, (hipStream_t)stream) == hipSuccess ? 0 : LSMS_EHIP;
}

extern "C" int lsms_mlp_cast(lsms_handle_t h, const float* params, uint16_t* w_bf16, void* stream) {
  if (!h) return -1;
  if (!params) return -2;
  if (!w_bf16) return -3;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_to_bf16(lsms_mlp_param_count(), params, w_bf16, (hipStream_t)stream) == hipSuccess
             ? 0
             : LSMS_EHIP;
}

extern "C" int lsms_mlp_forward(lsms_handle_t h, const float* params, const uint16_t* w_bf16, const float* feat,
                                int32_t n, float* out, float* act, void* stream) {
  if (!h) return -1;
  if (!params) return -2;
  if (!w_bf16) return -3;
  if (n < 0) return -5;
  if (n == 0) return 0;
  if (!feat) return -4;
  if (!act) return -7;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_forward(params, w_bf16, feat, n, out, act, (hipStream_t)stream) == hipSuccess ? 0
                                                                                                      : LSMS_EHIP;
}

extern "C" int lsms_mlp_backward(lsms_handle_t h, const uint16_t* w_bf16, const float* feat, const float* act,
                                 const float* dout, int32_t n, float* grad, float* work, void* stream) {
  if (!h) return -1;
  if (!w_bf16) return -2;
  if (!feat) return -3;
  if (!act) return -4;
  if (!dout) return -5;
  if (n < 1) return -6;
  if (!grad) return -7;
  if (!work) return -8;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_backward(w_bf16, feat, act, dout, n, grad, work, (hipStream_t)stream) == hipSuccess
             ? 0
             : LSMS_EHIP;
}

extern "C" int lsms_mlp_mse(lsms_handle_t h, const float* out, const float* target, int64_t count, float* dout,
                            float* loss, void* stream) {
  if (!h) return -1;
  if (!out) return -2;
  if (!target) return -3;
  if (count < 0) return -4;
  if (!dout) return -5;
  if (!loss) return -6;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_mse(out, target, count, dout, loss, (hipStream_t)stream) == hipSuccess ? 0 : LSMS_EHIP;
}

extern "C" int lsms_mlp_adamw(lsms_handle_t h, float* params, uint16_t* w_bf16, float* m, float* v,
                              const float* grad, float lr, float beta1, float beta2, float eps, float weight_decay,
                              int32_t step, void* stream) {
  if (!h) return -1;
  if (!params) return -2;
  if (!w_bf16) return -3;
  if (!m) return -4;
  if (!v) return -5;
  if (!grad) return -6;
  if (!(lr >= 0.f)) return -7;
  if (!(beta1 >= 0.f && beta1 < 1.f)) return -8;
  if (!(beta2 >= 0.f && beta2 < 1.f)) return -9;
  if (!(eps > 0.f)) return -10;
  if (!(weight_decay >= 0.f)) return -11;
  if (step < 1) return -12;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_adamw(lsms_mlp_param_count(), params, w_bf16, m, v, grad, lr, beta1, beta2, eps,
                               weight_decay, step, (hipStream_t)stream) == hipSuccess
             ? 0
             : LSMS_EHIP;
}

extern "C" int lsms_mlp_seed(lsms_handle_t h, const float* out, const float* scale, const float* shift, int32_t n,
                             double* seed, void* stream) {
  if (!h) return -1;
  if (!out) return -2;
  if (!scale) return -3;
  if (!shift) return -4;
  if (n < 0) return -5;
  if (n == 0) return 0;
  if (!seed) return -6;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_seed(n, 16, out, scale, shift, seed, (hipStream_t)stream) == hipSuccess ? 0 : LSMS_EHIP;
}

extern "C" int lsms_mlp_targets(lsms_handle_t h, const lsms_problem* p, const double* tau00, const float* scale,
                                const float* shift, float* target, void* stream) {
  if (!h) return -1;
  int r = check_problem(p);
  if (r) return r;
  if (p->lmax != 3) return -2;
  if (p->n_inst == 0) return 0;
  if (!tau00) return -3;
  if ((scale == nullptr) != (shift == nullptr)) return -4;
  if (!target) return -6;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_targets(to_dev(p), tau00, scale, shift, target, (hipStream_t)stream) == hipSuccess
             ? 0
             : LSMS_EHIP;
}

extern "C" int lsms_mlp_norm_stats(lsms_handle_t h, const float* target, int32_t n, float* scale, float* shift,
                                   void* stream) {
  if (!h) return -1;
  if (!target) return -2;
  if (n < 1) return -3;
  if (!scale) return -4;
  if (!shift) return -5;
  (void)hipSetDevice(h->device);
  return lsms_launch_mlp_norm_stats(n, target, scale, shift, (hipStream_t)stream) == hipSuccess ? 0 : LSMS_EHIP;
}
