// Learned form: per-instance features, the seed network (18 -> 256 -> 256 ->
// 256 -> 1024, SiLU after the hidden layers) with bf16 weights and FP32
// accumulation, its backward, the MSE loss and AdamW.  The network maps an
// instance's local environment and energy to normalised approximations of
// tau00 and of [M^{-1}]_{00}; the latter seeds the GMRES solve.
//
// Forward products: Z = bf16(H) bf16(W)^T + b on the bf16 matrix cores
// (v_mfma_f32_16x16x16_bf16: every product of two bf16 values is exact, the
// sums in FP32), the activations rounded to bf16 (round to nearest even) as
// they are loaded.  Backward products use FP32 operands on
// v_mfma_f32_16x16x4f32 (the rounding is taken as the identity).
#include <cstdint>

#include "lsms_common.h"

using namespace lsms;

namespace {

constexpr int kLayers = 4;
constexpr int kDims[kLayers + 1] = {18, 256, 256, 256, 1024};
constexpr int kActPerSample = 6 * 256 + 1024;  // Z1 H1 Z2 H2 Z3 H3 and the output

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename T, bool kRound>
__device__ __forceinline__ float load_op(const T* p, int64_t i) {
  float v;
  if constexpr (sizeof(T) == 2) {
    v = bf16_to_f32(reinterpret_cast<const uint16_t*>(p)[i]);
  } else {
    v = p[i];
  }
  if constexpr (kRound) v = bf16_round(v);
  return v;
}

// C[i][j] (ldc) = sum_k A(i, k) B(k, j) (+ bias[j]) (+ C[i][j] if accumulate),
// A(i, k) = A[i sai + k sak], B(k, j) = B[k sbk + j sbj].  A 64x64 tile per
// 256-thread workgroup, 32x32 (2x2 MFMA tiles) per wave.
template <typename TA, bool kRA, typename TB, bool kRB>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const TA* __restrict__ A, int64_t sai,
                                                   int64_t sak, const TB* __restrict__ B, int64_t sbk, int64_t sbj,
                                                   float* __restrict__ C, int64_t ldc,
                                                   const float* __restrict__ bias, int accumulate) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int i0 = blockIdx.y * 64 + 32 * (wave >> 1), j0 = blockIdx.x * 64 + 32 * (wave & 1);
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int kb = 0; kb < K; kb += 4) {
    const int k = kb + lq;
    float av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = i0 + 16 * a + li;
      av[a] = (i < M && k < K) ? load_op<TA, kRA>(A, (int64_t)i * sai + (int64_t)k * sak) : 0.f;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + 16 * b + li;
      bv[b] = (j < N && k < K) ? load_op<TB, kRB>(B, (int64_t)k * sbk + (int64_t)j * sbj) : 0.f;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
  // register r of lane l holds D[4 (l / 16) + r][l % 16]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * a + 4 * lq + r, j = j0 + 16 * b + li;
        if (i < M && j < N) {
          float v = acc[a][b][r];
          if (bias) v += bias[j];
          float* c = C + (int64_t)i * ldc + j;
          if (accumulate) v += *c;
          *c = v;
        }
      }
}

typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// C[i][j] (ldc) = sum_k bf16(A[i lda + k]) Wb[j ldw + k] + bias[j]: both
// operands run along k, so lane (li, lq) of a 16 x 16 x 16 step supplies k =
// kb + 4 lq .. + 3 of row i (A) and of column j (W).  A 64x64 tile per
// 256-thread workgroup, 32x32 (2x2 MFMA tiles) per wave; K ragged (zeros).
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const float* __restrict__ A, int64_t lda,
                                                        const uint16_t* __restrict__ Wb, int64_t ldw,
                                                        float* __restrict__ C, int64_t ldc,
                                                        const float* __restrict__ bias) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int i0 = blockIdx.y * 64 + 32 * (wave >> 1), j0 = blockIdx.x * 64 + 32 * (wave & 1);
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int kb = 0; kb < K; kb += 16) {
    const int k0 = kb + 4 * lq;
    v4s av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = i0 + 16 * a + li;
#pragma unroll
      for (int t = 0; t < 4; ++t) av[a][t] = (i < M && k0 + t < K) ? bf16_bits(A[(int64_t)i * lda + k0 + t]) : 0;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + 16 * b + li;
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[b][t] = (j < N && k0 + t < K) ? (short)Wb[(int64_t)j * ldw + k0 + t] : 0;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
  // register r of lane l holds D[4 (l / 16) + r][l % 16]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * a + 4 * lq + r, j = j0 + 16 * b + li;
        if (i < M && j < N) C[(int64_t)i * ldc + j] = acc[a][b][r] + (bias ? bias[j] : 0.f);
      }
}

template <typename TA, bool kRA, typename TB, bool kRB>
hipError_t gemm(int M, int N, int K, const TA* A, int64_t sai, int64_t sak, const TB* B, int64_t sbk, int64_t sbj,
                float* C, int64_t ldc, const float* bias, int accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((gemm_kernel<TA, kRA, TB, kRB>), grid, dim3(256), 0, s, M, N, K, A, sai, sak, B, sbk, sbj, C,
                     ldc, bias, accumulate);
  return hipGetLastError();
}

// H = silu(Z) for a [n][256] block inside the activation rows (stride ld).
__global__ void silu_kernel(int n, const float* __restrict__ Z, float* __restrict__ H, int64_t ld) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * 256) return;
  const int64_t r = q / 256, c = q % 256;
  const float z = Z[r * ld + c];
  H[r * ld + c] = z / (1.f + __expf(-z));
}

// G = dH * silu'(Z) in place (dH in G, [n][256] contiguous).
__global__ void dsilu_kernel(int n, const float* __restrict__ Z, int64_t ldz, float* __restrict__ G) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * 256) return;
  const int64_t r = q / 256, c = q % 256;
  const float z = Z[r * ldz + c];
  const float sg = 1.f / (1.f + __expf(-z));
  G[q] *= sg * (1.f + z * (1.f - sg));
}

// db[j] = sum_i G[i][j] (G [n][m] with row stride ld), one thread per column.
__global__ void colsum_kernel(int n, int m, const float* __restrict__ G, int64_t ld, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  float s = 0.f;
  for (int i = 0; i < n; ++i) s += G[(int64_t)i * ld + j];
  db[j] = s;
}

// Features of each instance: centre one-hot, per-shell Ni/Au fractions of the
// first seven fcc shells (nearest ideal radius a sqrt(k/2); sites nearest to
// the eighth shell are dropped), Re E, Im E.
__global__ void features_kernel(lsms_prob_dev p, double a, float* __restrict__ feat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n_inst) return;
  float* f = feat + (int64_t)i * 18;
  const int64_t s = p.liz_off[i], e = p.liz_off[i + 1];
  int cnt[7][2];
#pragma unroll
  for (int k = 0; k < 7; ++k) cnt[k][0] = cnt[k][1] = 0;
  double radius[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) radius[k] = a * sqrt((k + 1) * 0.5);
  for (int64_t j = s + 1; j < e; ++j) {
    const double x = p.pos[3 * j], y = p.pos[3 * j + 1], z = p.pos[3 * j + 2];
    const double r = sqrt(x * x + y * y + z * z);
    int best = 0;
    double bd = fabs(radius[0] - r);
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      const double d = fabs(radius[k] - r);
      if (d < bd) {
        bd = d;
        best = k;
      }
    }
    const int sp = p.species[j];
    if (best < 7 && sp >= 0 && sp < 2) cnt[best][sp] += 1;
  }
  const int sc = e > s ? p.species[s] : -1;
  f[0] = sc == 0 ? 1.f : 0.f;
  f[1] = sc == 1 ? 1.f : 0.f;
  const double size[7] = {12.0, 6.0, 24.0, 12.0, 24.0, 8.0, 48.0};
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    f[2 + 2 * k] = (float)(cnt[k][0] / size[k]);
    f[3 + 2 * k] = (float)(cnt[k][1] / size[k]);
  }
  const int ei = p.e_idx[i];
  const bool eok = ei >= 0 && ei < p.n_energy;
  f[16] = eok ? (float)p.energy[2 * ei] : 0.f;
  f[17] = eok ? (float)p.energy[2 * ei + 1] : 0.f;
}

// dout = 2 (out - target) / (n m); loss += sum (out - target)^2 / (n m).
__global__ void mse_kernel(int64_t total, const float* __restrict__ out, const float* __restrict__ target,
                           float* __restrict__ dout, float* __restrict__ loss) {
  __shared__ float part[256];
  float s = 0.f;
  const float inv = 1.f / (float)total;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const float d = out[q] - target[q];
    dout[q] = 2.f * d * inv;
    s += d * d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, part[0] * inv);
}

__global__ void fill_f32_kernel(float* p, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// AdamW on the FP32 master parameters; the bf16 copy is refreshed.
__global__ void adamw_kernel(int64_t n, float* __restrict__ w, uint16_t* __restrict__ wb, float* __restrict__ m,
                             float* __restrict__ v, const float* __restrict__ g, float lr, float b1, float b2,
                             float eps, float wd, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[i]);
    w[i] = wi;
    wb[i] = (uint16_t)(__float_as_uint(bf16_round(wi)) >> 16);
  }
}

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ w, uint16_t* __restrict__ wb) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    wb[i] = (uint16_t)(__float_as_uint(bf16_round(w[i])) >> 16);
}

// seed[i][L + kk L'] (complex FP64) = out[i][512 + 2 (L + kk L') + {0,1}] * scale + shift
// (de-normalised [M^{-1}]_{00} part of the network output; kk <= 16).
__global__ void seed_kernel(int n, int kk, const float* __restrict__ out, const float* __restrict__ scale,
                            const float* __restrict__ shift, double* __restrict__ seed) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * kk * kk * 2) return;
  const int64_t i = q / (kk * kk * 2), r = q % (kk * kk * 2);
  const int o = 512 + (int)r;
  seed[i * kk * kk * 2 + r] = (double)(out[i * 1024 + o] * scale[o] + shift[o]);
}

// Raw training targets of each instance: [tau00 (512 floats) | D (512)],
// D(L, L') = tau00(L, L') / t0_{l(L')} = [M^{-1}]_{00}(L, L') (zero where t0
// vanishes); kk = 16.  If scale is given, normalised: (x - shift) / scale.
__global__ void targets_kernel(lsms_prob_dev p, const double* __restrict__ tau00, const float* __restrict__ scale,
                               const float* __restrict__ shift, float* __restrict__ target) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)p.n_inst * 256) return;
  const int64_t i = q / 256;
  const int e = (int)(q % 256), Lp = e / 16;
  const zd t = reinterpret_cast<const zd*>(tau00)[q];
  const int ei = min(max(p.e_idx[i], 0), p.n_energy - 1);
  const int s0 = min(max(p.species[p.liz_off[i]], 0), p.n_species - 1);
  const zd kap = zsqrt(reinterpret_cast<const zd*>(p.energy)[ei]);
  const zd t0 = tmat_from_delta(reinterpret_cast<const zd*>(p.delta)[((int64_t)s0 * p.n_energy + ei) * (p.lmax + 1) +
                                                                      l_of(Lp)],
                                kap);
  const bool tz = t0.x == 0.0 && t0.y == 0.0;
  const zd d = tz ? zmake(0.0, 0.0) : zdiv(t, t0);
  float v[4] = {(float)t.x, (float)t.y, (float)d.x, (float)d.y};
  const int o[4] = {2 * e, 2 * e + 1, 512 + 2 * e, 512 + 2 * e + 1};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float x = v[c];
    if (scale) x = (x - shift[o[c]]) / scale[o[c]];
    target[i * 1024 + o[c]] = x;
  }
}

// Column statistics of targets [n][1024]: shift = mean, scale = standard
// deviation (1 where it vanishes); one thread per column, two passes.
__global__ void norm_stats_kernel(int n, const float* __restrict__ target, float* __restrict__ scale,
                                  float* __restrict__ shift) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 1024) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += target[(int64_t)i * 1024 + j];
  const double mean = n > 0 ? s / n : 0.0;
  double v = 0.0;
  for (int i = 0; i < n; ++i) {
    const double d = target[(int64_t)i * 1024 + j] - mean;
    v += d * d;
  }
  const double sd = n > 1 ? sqrt(v / n) : 0.0;
  shift[j] = (float)mean;
  scale[j] = sd > 0.0 ? (float)sd : 1.f;
}

int64_t param_offset(int l) {
  int64_t off = 0;
  for (int q = 0; q < l; ++q) off += (int64_t)kDims[q + 1] * kDims[q] + kDims[q + 1];
  return off;
}

int blocks_for(int64_t n) { return (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096); }

}  // namespace

int64_t lsms_mlp_param_count() { return param_offset(kLayers); }
int64_t lsms_mlp_act_floats() { return kActPerSample; }

hipError_t lsms_launch_mlp_features(const lsms_prob_dev& p, double a, float* feat, hipStream_t s) {
  if (p.n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3((p.n_inst + 127) / 128), dim3(128), 0, s, p, a, feat);
  return hipGetLastError();
}

// act rows per sample: Z1 H1 Z2 H2 Z3 H3 (256 each) then the output (1024).
hipError_t lsms_launch_mlp_forward(const float* params, const uint16_t* wb, const float* feat, int n, float* out,
                                   float* act, hipStream_t s) {
  hipError_t e;
  const int64_t ld = kActPerSample;
  const float* hin = feat;
  int64_t ldin = 18;
  for (int l = 0; l < kLayers; ++l) {
    const int in = kDims[l], o = kDims[l + 1];
    const int64_t off = param_offset(l);
    const uint16_t* W = wb + off;
    const float* b = params + off + (int64_t)o * in;
    float* Z = (l + 1 < kLayers) ? act + 512 * l : act + 6 * 256;
    // Z[i][j] = sum_k bf16(hin[i][k]) bf16(W[j][k]) + b[j]
    if (n > 0) {
      hipLaunchKernelGGL(gemm_bf16_kernel, dim3((o + 63) / 64, (n + 63) / 64), dim3(256), 0, s, n, o, in, hin, ldin,
                         W, (int64_t)in, Z, ld, b);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (l + 1 < kLayers) {
      float* H = Z + 256;
      hipLaunchKernelGGL(silu_kernel, dim3(blocks_for((int64_t)n * 256)), dim3(256), 0, s, n, Z, H, ld);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hin = H;
      ldin = ld;
    }
  }
  // the output rows into `out` [n][1024]
  if (out) {
    if ((e = hipMemcpy2DAsync(out, 1024 * sizeof(float), act + 6 * 256, ld * sizeof(float), 1024 * sizeof(float),
                              n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// grad (flat, as the parameters) of sum(dout * out); work: [n][1024 + 256] floats.
hipError_t lsms_launch_mlp_backward(const uint16_t* wb, const float* feat, const float* act, const float* dout,
                                    int n, float* grad, float* work, hipStream_t s) {
  hipError_t e;
  const int64_t ld = kActPerSample;
  float* gA = work;                       // [n][1024] current layer's output gradient
  float* gB = work + (int64_t)n * 1024;   // [n][256]
  if ((e = hipMemcpyAsync(gA, dout, (size_t)n * 1024 * sizeof(float), hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return e;
  int ldg = 1024;
  float* g = gA;
  for (int l = kLayers - 1; l >= 0; --l) {
    const int in = kDims[l], o = kDims[l + 1];
    const int64_t off = param_offset(l);
    if (l + 1 < kLayers) {
      // g holds dH_l [n][256]; times silu'(Z_l)
      hipLaunchKernelGGL(dsilu_kernel, dim3(blocks_for((int64_t)n * 256)), dim3(256), 0, s, n, act + 512 * l, ld, g);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // layer input (bf16-rounded in the forward) and its row stride
    const float* hin = l == 0 ? feat : act + 512 * (l - 1) + 256;
    const int64_t ldin = l == 0 ? 18 : ld;
    // dW[j][k] = sum_i g[i][j] bf16(hin[i][k])
    if ((e = gemm<float, false, float, true>(o, in, n, g, 1, ldg, hin, ldin, 1, grad + off, in, nullptr, 0, s)) !=
        hipSuccess)
      return e;
    hipLaunchKernelGGL(colsum_kernel, dim3((o + 255) / 256), dim3(256), 0, s, n, o, g, (int64_t)ldg,
                       grad + off + (int64_t)o * in);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (l > 0) {
      // dH_{l-1}[i][k] = sum_j g[i][j] bf16(W[j][k])
      float* gn = (g == gA) ? gB : gA;
      if ((e = gemm<float, false, uint16_t, false>(n, in, o, g, ldg, 1, wb + off, in, 1, gn, 256, nullptr, 0, s)) !=
          hipSuccess)
        return e;
      g = gn;
      ldg = 256;
    }
  }
  return hipSuccess;
}

hipError_t lsms_launch_mlp_mse(const float* out, const float* target, int64_t total, float* dout, float* loss,
                               hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(1), dim3(64), 0, s, loss, 0.f, (int64_t)1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || total <= 0) return e;
  hipLaunchKernelGGL(mse_kernel, dim3(blocks_for(total) < 1024 ? blocks_for(total) : 1024), dim3(256), 0, s, total,
                     out, target, dout, loss);
  return hipGetLastError();
}

hipError_t lsms_launch_mlp_adamw(int64_t n, float* w, uint16_t* wb, float* m, float* v, const float* g, float lr,
                                 float b1, float b2, float eps, float wd, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adamw_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, w, wb, m, v, g, lr, b1, b2, eps, wd, c1,
                     c2);
  return hipGetLastError();
}

hipError_t lsms_launch_mlp_to_bf16(int64_t n, const float* w, uint16_t* wb, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, w, wb);
  return hipGetLastError();
}

hipError_t lsms_launch_mlp_seed(int n, int kk, const float* out, const float* scale, const float* shift, double* seed,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t total = (int64_t)n * kk * kk * 2;
  hipLaunchKernelGGL(seed_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, kk, out, scale, shift,
                     seed);
  return hipGetLastError();
}

hipError_t lsms_launch_mlp_targets(const lsms_prob_dev& p, const double* tau00, const float* scale,
                                   const float* shift, float* target, hipStream_t s) {
  if (p.n_inst <= 0) return hipSuccess;
  const int64_t total = (int64_t)p.n_inst * 256;
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, p, tau00, scale, shift,
                     target);
  return hipGetLastError();
}

hipError_t lsms_launch_mlp_norm_stats(int n, const float* target, float* scale, float* shift, hipStream_t s) {
  hipLaunchKernelGGL(norm_stats_kernel, dim3(4), dim3(256), 0, s, n, target, scale, shift);
  return hipGetLastError();
}
