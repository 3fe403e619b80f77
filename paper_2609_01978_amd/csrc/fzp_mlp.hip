// Learned surrogate: a three-layer perceptron from crease parameters and the
// wavelength to the log-intensity of the focal-plane ROI, trained on the
// propagation's own outputs.  The paper motivates full 2-D simulation by
// membrane deformations (introduction) but gives no learned model; this is
// the network the library provides for that use, with the CZT as its arbiter.
//
//   z1 = W1 x + b1, h1 = silu(z1);  z2 = W2 h1 + b2, h2 = silu(z2);
//   y = W3 h2 + b3;  loss = sum (y - t)^2 / (B n_out)
//
// Weights are kept in float32 (master copy, Adam moments) and used by the
// matrix cores as BF16 copies; activations and gradients enter the products as
// BF16, every product accumulates in float32, biases, activation derivatives,
// the loss and the optimizer run in float32.  Parameters form one flat vector
// W1 [H][n_in], b1 [H], W2 [H][H], b2 [H], W3 [n_out][H], b3 [n_out].
//
// One generic MFMA kernel serves every product: C = A B over a 64 x 64 output
// tile per work-group (4 waves, one 32 x 32 block each, K in steps of 32
// through LDS), where A is read either k-contiguous (A[m][k]) or m-contiguous
// (A[k][m]) and B either k-contiguous (B[n][k]) or n-contiguous (B[k][n]); long
// K is split over work-groups into float32 partial planes that the epilogue
// kernels add in a fixed order (no atomics, so training is reproducible).

#include <cmath>
#include <cstdint>
#include <new>
#include <string>

#include "fzp_internal.h"

namespace fzp {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }

constexpr int kGT = 64;    // output tile side
constexpr int kGK = 32;    // K per LDS stage
constexpr int kGLd = 40;   // LDS row stride in BF16 (32 + 8 padding, 80 bytes)

// Stage rows [r0, r0+64) x k [k0, k0+32) of an operand into LDS s[r][k].
// KC: element (r, k) is at p[r * ld + k] (k contiguous), else at p[k * ld + r].
template <bool KC>
__device__ __forceinline__ void stage_operand(uint16_t *s, const uint16_t *p, int64_t ld, int R, int K, int r0,
                                              int k0, int tid, bool vec) {
  if (KC) {
    const int r = tid >> 2, kc = (tid & 3) * 8;
    const int gr = r0 + r, gk = k0 + kc;
    uint16_t *d = s + r * kGLd + kc;
    if (vec && gr < R && gk + 8 <= K) {
      *(u32x4 *)d = *(const u32x4 *)(p + (int64_t)gr * ld + gk);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) d[e] = (gr < R && gk + e < K) ? p[(int64_t)gr * ld + gk + e] : (uint16_t)0;
    }
  } else {
    const int k = tid >> 3, rc = (tid & 7) * 8;
    const int gk = k0 + k, gr = r0 + rc;
    uint16_t v[8];
    if (vec && gk < K && gr + 8 <= R) {
      const u32x4 w = *(const u32x4 *)(p + (int64_t)gk * ld + gr);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[2 * e] = (uint16_t)(w[e] & 0xffffu);
        v[2 * e + 1] = (uint16_t)(w[e] >> 16);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (gk < K && gr + e < R) ? p[(int64_t)gk * ld + gr + e] : (uint16_t)0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) s[(rc + e) * kGLd + k] = v[e];
  }
}

// part[s][m][n] = sum over k in split s of A(m, k) B(k, n).
template <bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm_bf16(const uint16_t *__restrict__ A, int64_t lda,
                                                   const uint16_t *__restrict__ B, int64_t ldb, float *__restrict__ part,
                                                   int M, int N, int K, int kchunk) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[kGT * kGLd];
  __shared__ __attribute__((aligned(16))) uint16_t sB[kGT * kGLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = blockIdx.x * kGT, m0 = blockIdx.y * kGT;
  const int ks = blockIdx.z * kchunk;
  const int ke = ks + kchunk < K ? ks + kchunk : K;
  const bool va = (lda % 8 == 0) && (((uintptr_t)A & 15) == 0);
  const bool vb = (ldb % 8 == 0) && (((uintptr_t)B & 15) == 0);
  const int wm = wave >> 1, wn = wave & 1;
  const int l32 = lane & 31, lhi = lane >> 5;
  f32x16 acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
  for (int k0 = ks; k0 < ke; k0 += kGK) {
    // operands beyond ke are zero-filled by the K bound (ke acts as K here)
    stage_operand<AK>(sA, A, lda, M, ke, m0, k0, tid, va);
    stage_operand<BK>(sB, B, ldb, N, ke, n0, k0, tid, vb);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const bf16x8 a = *(const bf16x8 *)(sA + (wm * 32 + l32) * kGLd + s * 16 + 8 * lhi);
      const bf16x8 b = *(const bf16x8 *)(sB + (wn * 32 + l32) * kGLd + s * 16 + 8 * lhi);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  float *C = part + (int64_t)blockIdx.z * M * N;
  const int n = n0 + wn * 32 + l32;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm * 32 + 8 * (v >> 2) + 4 * lhi + (v & 3);
    if (m < M && n < N) C[(int64_t)m * N + n] = acc[v];
  }
}

// Hidden layer epilogue: z = sum_s part + b; zf = z; h = bf16(silu(z)).
__global__ void k_epi_hidden(const float *__restrict__ part, int S, int64_t MN, int N, const float *__restrict__ bias,
                             float *__restrict__ zf, uint16_t *__restrict__ h) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < MN; i += (int64_t)gridDim.x * blockDim.x) {
    float z = part[i];
    for (int s = 1; s < S; ++s) z += part[s * MN + i];
    z += bias[i % N];
    zf[i] = z;
    h[i] = f2bf(z * sigm(z));
  }
}

// Output epilogue: y = sum_s part + b.
__global__ void k_epi_out(const float *__restrict__ part, int S, int64_t MN, int N, const float *__restrict__ bias,
                          float *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < MN; i += (int64_t)gridDim.x * blockDim.x) {
    float z = part[i];
    for (int s = 1; s < S; ++s) z += part[s * MN + i];
    y[i] = z + (bias ? bias[i % N] : 0.0f);
  }
}

// Loss gradient: dy = 2 (y - t) / (B n_out) (float32 and BF16), and per-block
// partial sums of (y - t)^2 for the loss.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t, int64_t n,
                                             float scale, float *__restrict__ dy, uint16_t *__restrict__ dy16,
                                             float *__restrict__ lpart) {
  __shared__ float red[256];
  float acc = 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    acc += d * d;
    const float g = 2.0f * d * scale;
    dy[i] = g;
    dy16[i] = f2bf(g);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const float *__restrict__ lpart, int nb, float scale,
                                                    float *__restrict__ loss) {
  __shared__ float red[256];
  float acc = 0.0f;
  for (int i = threadIdx.x; i < nb; i += 256) acc += lpart[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] * scale;
}

// Activation backward: dz = (sum_s part) silu'(z) (float32 and BF16).
__global__ void k_epi_dact(const float *__restrict__ part, int S, int64_t MN, const float *__restrict__ z,
                           float *__restrict__ dz, uint16_t *__restrict__ dz16) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < MN; i += (int64_t)gridDim.x * blockDim.x) {
    float g = part[i];
    for (int s = 1; s < S; ++s) g += part[s * MN + i];
    const float zz = z[i];
    const float sg = sigm(zz);
    const float d = g * (sg * (1.0f + zz * (1.0f - sg)));
    dz[i] = d;
    dz16[i] = f2bf(d);
  }
}

// Column sums over rows: out[j] = sum_b a[b][j] (bias gradients), fixed order.
__global__ void k_colsum(const float *__restrict__ a, int rows, int cols, float *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.0f;
  for (int b = 0; b < rows; ++b) s += a[(int64_t)b * cols + j];
  out[j] = s;
}

__global__ void k_to_bf16(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

__global__ void k_fill_f32(float *__restrict__ x, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// Adam (Kingma & Ba, Algorithm 1): bc1 = 1/(1 - beta1^t), bc2 = 1/(1 - beta2^t).
__global__ void k_adam(float *__restrict__ w, uint16_t *__restrict__ w16, float *__restrict__ m,
                       float *__restrict__ v, const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
    w[i] = wi;
    w16[i] = f2bf(wi);
  }
}

// ln(|U|^2 / i0 + floor) and its inverse U = sqrt(max(i0 (e^y - floor), 0)) + 0i.
__global__ void k_log_intensity(const double2 *__restrict__ roi, int64_t n, double inv_i0, double fl,
                                float *__restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 u = roi[i];
    out[i] = (float)log((u.x * u.x + u.y * u.y) * inv_i0 + fl);
  }
}

__global__ void k_field_from_log(const float *__restrict__ y, int64_t n, double i0, double fl,
                                 double2 *__restrict__ roi) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double I = i0 * (exp((double)y[i]) - fl);
    roi[i] = make_double2(I > 0.0 ? sqrt(I) : 0.0, 0.0);
  }
}

unsigned ew_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

}  // namespace fzp

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

namespace {
fzp_status_t mfail(fzp_status_t s, const std::string &m) {
  fzp::set_last_error(m);
  return s;
}
fzp_status_t mhip(const char *what, hipError_t e) {
  return mfail(FZP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t kGTtile = 64;  // output tile side of k_gemm_bf16
}  // namespace

struct fzp_mlp_s {
  int32_t n_in, H, n_out, bmax;
  int64_t P;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3;  // element offsets inside the flat vector
  // workspace byte offsets
  size_t w32, w16, m, v, g, x16, z1, h1, z2, h2, dy, dy16, dz2, dz2_16, dz1, dz1_16, part, lpart, loss;
  size_t part_elems, bytes;
  int64_t step = 0;
};

namespace {

// Split K into chunks (multiples of 32) so that a product with few output
// tiles still has about 256 work-groups; returns the number of splits.
int splits_for(int M, int N, int K, int &kchunk) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int S = 1;
  while (tiles * S < 256 && K / (S * 2) >= 256) S *= 2;
  kchunk = ((K + S - 1) / S + 31) / 32 * 32;
  S = (K + kchunk - 1) / kchunk;
  return S;
}

template <bool AK, bool BK>
hipError_t gemm(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, float *part, int M, int N, int K,
                int &S, hipStream_t st) {
  int kchunk;
  S = splits_for(M, N, K, kchunk);
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)S);
  hipLaunchKernelGGL((fzp::k_gemm_bf16<AK, BK>), grid, dim3(256), 0, st, A, lda, B, ldb, part, M, N, K, kchunk);
  return hipGetLastError();
}

size_t gemm_part_elems(int M, int N, int K) {
  int kc;
  return (size_t)splits_for(M, N, K, kc) * (size_t)M * (size_t)N;
}

struct Ptrs {
  float *w32, *m, *v, *g, *z1, *z2, *dy, *dz2, *dz1, *part, *lpart, *loss;
  uint16_t *w16, *x16, *h1, *h2, *dy16, *dz2_16, *dz1_16;
};

Ptrs ptrs(const fzp_mlp_s &n, char *ws) {
  Ptrs p;
  p.w32 = (float *)(ws + n.w32);
  p.w16 = (uint16_t *)(ws + n.w16);
  p.m = (float *)(ws + n.m);
  p.v = (float *)(ws + n.v);
  p.g = (float *)(ws + n.g);
  p.x16 = (uint16_t *)(ws + n.x16);
  p.z1 = (float *)(ws + n.z1);
  p.h1 = (uint16_t *)(ws + n.h1);
  p.z2 = (float *)(ws + n.z2);
  p.h2 = (uint16_t *)(ws + n.h2);
  p.dy = (float *)(ws + n.dy);
  p.dy16 = (uint16_t *)(ws + n.dy16);
  p.dz2 = (float *)(ws + n.dz2);
  p.dz2_16 = (uint16_t *)(ws + n.dz2_16);
  p.dz1 = (float *)(ws + n.dz1);
  p.dz1_16 = (uint16_t *)(ws + n.dz1_16);
  p.part = (float *)(ws + n.part);
  p.lpart = (float *)(ws + n.lpart);
  p.loss = (float *)(ws + n.loss);
  return p;
}

// Forward pass of `batch` rows; the output goes to y (float32, [batch][n_out]).
hipError_t run_forward(const fzp_mlp_s &n, const Ptrs &p, const float *x, int batch, float *y, hipStream_t st) {
  using namespace fzp;
  const int B = batch, H = n.H;
  int S;
  hipLaunchKernelGGL(k_to_bf16, dim3(ew_grid((int64_t)B * n.n_in)), dim3(256), 0, st, x, (int64_t)B * n.n_in, p.x16);
  hipError_t e = gemm<true, true>(p.x16, n.n_in, p.w16 + n.oW1, n.n_in, p.part, B, H, n.n_in, S, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_epi_hidden, dim3(ew_grid((int64_t)B * H)), dim3(256), 0, st, p.part, S, (int64_t)B * H, H,
                     p.w32 + n.ob1, p.z1, p.h1);
  e = gemm<true, true>(p.h1, H, p.w16 + n.oW2, H, p.part, B, H, H, S, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_epi_hidden, dim3(ew_grid((int64_t)B * H)), dim3(256), 0, st, p.part, S, (int64_t)B * H, H,
                     p.w32 + n.ob2, p.z2, p.h2);
  e = gemm<true, true>(p.h2, H, p.w16 + n.oW3, H, p.part, B, n.n_out, H, S, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_epi_out, dim3(ew_grid((int64_t)B * n.n_out)), dim3(256), 0, st, p.part, S,
                     (int64_t)B * n.n_out, n.n_out, p.w32 + n.ob3, y);
  return hipGetLastError();
}

// Backward pass after run_forward (y in p.dy's companion buffer); gradients of
// the flat parameters into g, of the inputs into dx (may be NULL).
hipError_t run_backward(const fzp_mlp_s &n, const Ptrs &p, const float *y, const float *t, int batch, float *g,
                        float *dx, hipStream_t st) {
  using namespace fzp;
  const int B = batch, H = n.H, O = n.n_out, I = n.n_in;
  const int64_t BO = (int64_t)B * O;
  const int nb = (int)ew_grid(BO);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, y, t, BO, 1.0f / (float)BO, p.dy, p.dy16, p.lpart);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, p.lpart, nb, 1.0f / (float)BO, p.loss);
  int S;
  // W3: dy^T h2
  hipError_t e = gemm<false, false>(p.dy16, O, p.h2, H, p.part, O, H, B, S, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_epi_out, dim3(ew_grid((int64_t)O * H)), dim3(256), 0, st, p.part, S, (int64_t)O * H, H,
                     (const float *)nullptr, g + n.oW3);
  hipLaunchKernelGGL(k_colsum, dim3((O + 255) / 256), dim3(256), 0, st, p.dy, B, O, g + n.ob3);
  // h2: dy W3
  e = gemm<true, false>(p.dy16, O, p.w16 + n.oW3, H, p.part, B, H, O, S, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_epi_dact, dim3(ew_grid((int64_t)B * H)), dim3(256), 0, st, p.part, S, (int64_t)B * H, p.z2,
                     p.dz2, p.dz2_16);
  // W2: dz2^T h1
  e = gemm<false, false>(p.dz2_16, H, p.h1, H, p.part, H, H, B, S, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_epi_out, dim3(ew_grid((int64_t)H * H)), dim3(256), 0, st, p.part, S, (int64_t)H * H, H,
                     (const float *)nullptr, g + n.oW2);
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, st, p.dz2, B, H, g + n.ob2);
  // h1: dz2 W2
  e = gemm<true, false>(p.dz2_16, H, p.w16 + n.oW2, H, p.part, B, H, H, S, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_epi_dact, dim3(ew_grid((int64_t)B * H)), dim3(256), 0, st, p.part, S, (int64_t)B * H, p.z1,
                     p.dz1, p.dz1_16);
  // W1: dz1^T x
  e = gemm<false, false>(p.dz1_16, H, p.x16, I, p.part, H, I, B, S, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_epi_out, dim3(ew_grid((int64_t)H * I)), dim3(256), 0, st, p.part, S, (int64_t)H * I, I,
                     (const float *)nullptr, g + n.oW1);
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, st, p.dz1, B, H, g + n.ob1);
  if (dx) {
    e = gemm<true, false>(p.dz1_16, H, p.w16 + n.oW1, I, p.part, B, I, H, S, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_epi_out, dim3(ew_grid((int64_t)B * I)), dim3(256), 0, st, p.part, S, (int64_t)B * I, I,
                       (const float *)nullptr, dx);
  }
  return hipGetLastError();
}

}  // namespace

extern "C" fzp_status_t fzp_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch_max,
                                       fzp_mlp_t *out) {
  if (!out) return mfail(FZP_E_INVAL, "fzp_mlp_create: NULL argument");
  *out = nullptr;
  if (n_in < 1 || n_in > 4096 || n_hidden < 1 || n_hidden > 8192 || n_out < 1 || n_out > (1 << 20) || batch_max < 1 ||
      batch_max > 65536)
    return mfail(FZP_E_INVAL, "fzp_mlp_create: sizes out of range");
  auto *n = new (std::nothrow) fzp_mlp_s;
  if (!n) return mfail(FZP_E_NOMEM, "fzp_mlp_create: out of host memory");
  n->n_in = n_in;
  n->H = n_hidden;
  n->n_out = n_out;
  n->bmax = batch_max;
  const int64_t H = n_hidden;
  n->oW1 = 0;
  n->ob1 = n->oW1 + H * n_in;
  n->oW2 = n->ob1 + H;
  n->ob2 = n->oW2 + H * H;
  n->oW3 = n->ob2 + H;
  n->ob3 = n->oW3 + (int64_t)n_out * H;
  n->P = n->ob3 + n_out;
  const int64_t B = batch_max;
  size_t pe = 0;
  auto upd = [&](size_t v) { pe = v > pe ? v : pe; };
  upd(gemm_part_elems((int)B, (int)H, n_in));
  upd(gemm_part_elems((int)B, (int)H, (int)H));
  upd(gemm_part_elems((int)B, n_out, (int)H));
  upd(gemm_part_elems(n_out, (int)H, (int)B));
  upd(gemm_part_elems((int)B, (int)H, n_out));
  upd(gemm_part_elems((int)H, (int)H, (int)B));
  upd(gemm_part_elems((int)H, n_in, (int)B));
  upd(gemm_part_elems((int)B, n_in, (int)H));
  // a smaller batch may split K further: splits S < 512 / tiles whenever S > 1,
  // so S M N < 512 * 64 * 64 in that case
  upd((size_t)512 * kGTtile * kGTtile);
  n->part_elems = pe;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = a256(off + bytes);
    return o;
  };
  const size_t P = (size_t)n->P;
  n->w32 = take(4 * P);
  n->w16 = take(2 * P);
  n->m = take(4 * P);
  n->v = take(4 * P);
  n->g = take(4 * P);
  n->x16 = take(2 * (size_t)B * n_in);
  n->z1 = take(4 * (size_t)B * H);
  n->h1 = take(2 * (size_t)B * H);
  n->z2 = take(4 * (size_t)B * H);
  n->h2 = take(2 * (size_t)B * H);
  n->dy = take(4 * (size_t)B * n_out);
  n->dy16 = take(2 * (size_t)B * n_out);
  n->dz2 = take(4 * (size_t)B * H);
  n->dz2_16 = take(2 * (size_t)B * H);
  n->dz1 = take(4 * (size_t)B * H);
  n->dz1_16 = take(2 * (size_t)B * H);
  n->part = take(4 * pe);
  n->lpart = take(4 * 8192);
  n->loss = take(4);
  n->bytes = off;
  *out = n;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_mlp_info(fzp_mlp_t n, size_t *workspace_bytes, int64_t *n_params) {
  if (!n) return mfail(FZP_E_INVAL, "fzp_mlp_info: NULL model");
  if (workspace_bytes) *workspace_bytes = n->bytes;
  if (n_params) *n_params = n->P;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_mlp_set_params(fzp_mlp_t n, void *ws, const float *params_dev, void *stream) {
  if (!n || !ws || !params_dev) return mfail(FZP_E_INVAL, "fzp_mlp_set_params: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const Ptrs p = ptrs(*n, (char *)ws);
  hipError_t e = hipMemcpyAsync(p.w32, params_dev, 4 * (size_t)n->P, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return mhip("fzp_mlp_set_params: copy", e);
  using namespace fzp;
  hipLaunchKernelGGL(k_to_bf16, dim3(ew_grid(n->P)), dim3(256), 0, st, p.w32, n->P, p.w16);
  hipLaunchKernelGGL(k_fill_f32, dim3(ew_grid(n->P)), dim3(256), 0, st, p.m, n->P, 0.0f);
  hipLaunchKernelGGL(k_fill_f32, dim3(ew_grid(n->P)), dim3(256), 0, st, p.v, n->P, 0.0f);
  e = hipGetLastError();
  if (e != hipSuccess) return mhip("fzp_mlp_set_params: kernels", e);
  n->step = 0;
  return FZP_OK;
}

extern "C" fzp_status_t fzp_mlp_get_params(fzp_mlp_t n, void *ws, float *params_dev, void *stream) {
  if (!n || !ws || !params_dev) return mfail(FZP_E_INVAL, "fzp_mlp_get_params: NULL argument");
  const Ptrs p = ptrs(*n, (char *)ws);
  hipError_t e = hipMemcpyAsync(params_dev, p.w32, 4 * (size_t)n->P, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return mhip("fzp_mlp_get_params: copy", e);
  return FZP_OK;
}

extern "C" fzp_status_t fzp_mlp_forward(fzp_mlp_t n, void *ws, const float *x_dev, int32_t batch, float *y_dev,
                                        void *stream) {
  if (!n || !ws || !x_dev || !y_dev) return mfail(FZP_E_INVAL, "fzp_mlp_forward: NULL argument");
  if (batch < 1 || batch > n->bmax) return mfail(FZP_E_INVAL, "fzp_mlp_forward: batch out of range");
  const hipError_t e = run_forward(*n, ptrs(*n, (char *)ws), x_dev, batch, y_dev, (hipStream_t)stream);
  if (e != hipSuccess) return mhip("fzp_mlp_forward", e);
  return FZP_OK;
}

extern "C" fzp_status_t fzp_mlp_backward(fzp_mlp_t n, void *ws, const float *x_dev, const float *t_dev, int32_t batch,
                                         float *y_dev, float *grads_dev, float *dx_dev, float *loss_dev,
                                         void *stream) {
  if (!n || !ws || !x_dev || !t_dev || !y_dev || !grads_dev)
    return mfail(FZP_E_INVAL, "fzp_mlp_backward: NULL argument");
  if (batch < 1 || batch > n->bmax) return mfail(FZP_E_INVAL, "fzp_mlp_backward: batch out of range");
  hipStream_t st = (hipStream_t)stream;
  const Ptrs p = ptrs(*n, (char *)ws);
  hipError_t e = run_forward(*n, p, x_dev, batch, y_dev, st);
  if (e == hipSuccess) e = run_backward(*n, p, y_dev, t_dev, batch, grads_dev, dx_dev, st);
  if (e == hipSuccess && loss_dev) e = hipMemcpyAsync(loss_dev, p.loss, 4, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return mhip("fzp_mlp_backward", e);
  return FZP_OK;
}

extern "C" fzp_status_t fzp_mlp_train_step(fzp_mlp_t n, void *ws, const float *x_dev, const float *t_dev,
                                           int32_t batch, float *y_dev, float lr, float *loss_dev, void *stream) {
  if (!n || !ws || !x_dev || !t_dev || !y_dev) return mfail(FZP_E_INVAL, "fzp_mlp_train_step: NULL argument");
  if (batch < 1 || batch > n->bmax) return mfail(FZP_E_INVAL, "fzp_mlp_train_step: batch out of range");
  if (!(std::isfinite(lr) && lr >= 0.0f)) return mfail(FZP_E_INVAL, "fzp_mlp_train_step: bad learning rate");
  hipStream_t st = (hipStream_t)stream;
  const Ptrs p = ptrs(*n, (char *)ws);
  hipError_t e = run_forward(*n, p, x_dev, batch, y_dev, st);
  if (e == hipSuccess) e = run_backward(*n, p, y_dev, t_dev, batch, p.g, nullptr, st);
  if (e != hipSuccess) return mhip("fzp_mlp_train_step", e);
  n->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = (float)(1.0 / (1.0 - std::pow(b1, (double)n->step)));
  const float bc2 = (float)(1.0 / (1.0 - std::pow(b2, (double)n->step)));
  hipLaunchKernelGGL(fzp::k_adam, dim3(fzp::ew_grid(n->P)), dim3(256), 0, st, p.w32, p.w16, p.m, p.v, p.g, n->P, lr,
                     (float)b1, (float)b2, 1e-8f, bc1, bc2);
  if (loss_dev) e = hipMemcpyAsync(loss_dev, p.loss, 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return mhip("fzp_mlp_train_step: update", e);
  return FZP_OK;
}

extern "C" fzp_status_t fzp_mlp_adam_update(fzp_mlp_t n, void *ws, const float *grads_dev, float lr, void *stream) {
  if (!n || !ws || !grads_dev) return mfail(FZP_E_INVAL, "fzp_mlp_adam_update: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const Ptrs p = ptrs(*n, (char *)ws);
  n->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = (float)(1.0 / (1.0 - std::pow(b1, (double)n->step)));
  const float bc2 = (float)(1.0 / (1.0 - std::pow(b2, (double)n->step)));
  hipLaunchKernelGGL(fzp::k_adam, dim3(fzp::ew_grid(n->P)), dim3(256), 0, st, p.w32, p.w16, p.m, p.v, grads_dev,
                     n->P, lr, (float)b1, (float)b2, 1e-8f, bc1, bc2);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mhip("fzp_mlp_adam_update", e);
  return FZP_OK;
}

extern "C" void fzp_mlp_destroy(fzp_mlp_t n) { delete n; }

extern "C" fzp_status_t fzp_log_intensity(const double *roi_dev, int64_t n_complex, double i0, double floor_,
                                          float *out_dev, void *stream) {
  if (!roi_dev || !out_dev || n_complex < 0 || !(i0 > 0.0) || !(floor_ > 0.0))
    return mfail(FZP_E_INVAL, "fzp_log_intensity: bad argument");
  if (n_complex == 0) return FZP_OK;
  hipLaunchKernelGGL(fzp::k_log_intensity, dim3(fzp::ew_grid(n_complex)), dim3(256), 0, (hipStream_t)stream,
                     (const double2 *)roi_dev, n_complex, 1.0 / i0, floor_, out_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mhip("fzp_log_intensity", e);
  return FZP_OK;
}

extern "C" fzp_status_t fzp_field_from_log_intensity(const float *y_dev, int64_t n_complex, double i0, double floor_,
                                                     double *roi_dev, void *stream) {
  if (!roi_dev || !y_dev || n_complex < 0 || !(i0 > 0.0) || !(floor_ > 0.0))
    return mfail(FZP_E_INVAL, "fzp_field_from_log_intensity: bad argument");
  if (n_complex == 0) return FZP_OK;
  hipLaunchKernelGGL(fzp::k_field_from_log, dim3(fzp::ew_grid(n_complex)), dim3(256), 0, (hipStream_t)stream, y_dev,
                     n_complex, i0, floor_, (double2 *)roi_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mhip("fzp_field_from_log_intensity", e);
  return FZP_OK;
}
