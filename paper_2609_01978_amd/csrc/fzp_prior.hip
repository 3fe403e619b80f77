// Physics prior of the learned surrogate: the focal-plane intensity of a
// deformed binary zone plate's first diffraction order, treated as a thin
// lens with the plate's pupil.  The Eq. 4 plate is periodic in
// s = r^2 / (lambda0 f0) with period 2; the converging term of that Fourier
// series has amplitude 1/pi, and at its focus (lambda z = lambda0 f0) the
// Fresnel integral of Eq. 2 loses the input chirp and becomes a Fourier
// transform of the pupil times the membrane phase screen exp(2 pi i h / lambda)
// (straight Gaussian ridges, the crease model of the propagation).  The zero
// order and the defocused orders are left out; the network learns the rest.
//
// On an Np x Np pupil grid over [-R, R]^2 (pixel centres
// u_i = (2 i + 1 - Np) D / (2 Np)) and the M x M ROI of a default instance at
// its focus (samples (q - M/2) 16 lambda0 f0 / (D M)):
//
//   g[j][i] = P_ij exp(2 pi i h(u_i, u_j) / lambda),
//   P_ij    = share of the pixel's ss x ss sub-sample centres inside the disc
//             (exact integer test),
//   E[q][i] = exp(-2 pi i t_qi),  t_qi = 4 (2 i + 1 - Np)(2 q - M) / (Np M)
//             (an exact rational, reduced in integers),
//   S = E g E^T,   y = ln(16 |S|^2 / (pi^2 Np^4) + floor)   (I / I0 + floor).
//
// Three kernels: the DFT table (float64 phases, complex float32 values), the
// pupil field (float64 ridge heights and phases, complex float32 values), and
// one batched complex float32 product kernel for the two transforms (the
// second with the log-intensity epilogue).  The transforms are a few MFLOP per
// instance, so they stay on the vector ALUs.

#include <cmath>
#include <cstdint>
#include <string>

#include "fzp_internal.h"

namespace fzp {

namespace {

constexpr int kPT = 256;        // threads per work-group
constexpr int kPTile = 64;      // output tile side of the product kernel
constexpr int kPK = 16;         // K per LDS stage
constexpr int kPPad = 68;       // LDS row length (complex), 32-byte aligned rows
constexpr int kMaxCreases = 64;

// E[q][i] for q < M, i < Np.
__global__ __launch_bounds__(kPT) void k_prior_dft(int Np, int M, float2 *__restrict__ E) {
  const int64_t e = blockIdx.x * (int64_t)kPT + threadIdx.x;
  if (e >= (int64_t)M * Np) return;
  const int q = (int)(e / Np), i = (int)(e % Np);
  const int64_t den = (int64_t)Np * M;
  int64_t num = (4 * (int64_t)(2 * i + 1 - Np) * (int64_t)(2 * q - M)) % den;
  if (num < 0) num += den;
  double s, c;
  sincospi(2.0 * (double)num / (double)den, &s, &c);
  E[e] = make_float2((float)c, (float)-s);
}

// g of instance blockIdx.y; creases [n][nc][4] = (theta, offset, width, height).
__global__ __launch_bounds__(kPT) void k_prior_pupil(const double *__restrict__ creases, int nc,
                                                     const double *__restrict__ lam, double D, int Np, int ss,
                                                     float2 *__restrict__ G) {
  __shared__ double cst[kMaxCreases][5];
  const int b = blockIdx.y;
  if (threadIdx.x < nc) {
    const double *c = creases + ((int64_t)b * nc + threadIdx.x) * 4;
    const double sigma = c[2] / (2.0 * sqrt(2.0 * log(2.0)));
    cst[threadIdx.x][0] = cos(c[0]);
    cst[threadIdx.x][1] = sin(c[0]);
    cst[threadIdx.x][2] = c[1];
    cst[threadIdx.x][3] = 1.0 / (2.0 * sigma * sigma);
    cst[threadIdx.x][4] = c[3];
  }
  __syncthreads();
  const int64_t e = blockIdx.x * (int64_t)kPT + threadIdx.x;
  if (e >= (int64_t)Np * Np) return;
  const int j = (int)(e / Np), i = (int)(e % Np);
  // pupil share: sub-sample centres c = 2 (i ss + s) + 1 - n in units D / (2 n)
  const int64_t n = (int64_t)Np * ss;
  int cnt = 0;
  for (int sy = 0; sy < ss; ++sy) {
    const int64_t cy = 2 * ((int64_t)j * ss + sy) + 1 - n;
    for (int sx = 0; sx < ss; ++sx) {
      const int64_t cx = 2 * ((int64_t)i * ss + sx) + 1 - n;
      cnt += cx * cx + cy * cy <= n * n ? 1 : 0;
    }
  }
  if (cnt == 0) {
    G[(int64_t)b * Np * Np + e] = make_float2(0.0f, 0.0f);
    return;
  }
  const double u = (double)(2 * i + 1 - Np) / (2.0 * Np) * D;
  const double v = (double)(2 * j + 1 - Np) / (2.0 * Np) * D;
  double h = 0.0;
  for (int k = 0; k < nc; ++k) {
    const double d = u * cst[k][0] + v * cst[k][1] - cst[k][2];
    h += cst[k][4] * exp(-d * d * cst[k][3]);
  }
  double turns = h / lam[b];
  turns -= floor(turns);
  double s, c;
  sincospi(2.0 * turns, &s, &c);
  const double a = (double)cnt / (double)(ss * ss);
  G[(int64_t)b * Np * Np + e] = make_float2((float)(a * c), (float)(a * s));
}

// C[b] = A[b] B[b] (complex float32), A(r, k) = A[b as + r ars + k aks],
// B(k, c) = B[b bs + k bks + c bcs], over 64 x 64 output tiles; K a multiple
// of 16.  AK / BK: the operand is contiguous along k (else along r / c), which
// sets the coalescing of the tile loads.  LOG: write ln(scale |C|^2 + floor)
// as float instead of C.
template <bool AK, bool BK, bool LOG>
__global__ __launch_bounds__(kPT) void k_prior_cgemm(const float2 *__restrict__ A, int64_t as, int64_t ars,
                                                     int64_t aks, const float2 *__restrict__ B, int64_t bs,
                                                     int64_t bks, int64_t bcs, int R, int K, int C,
                                                     float2 *__restrict__ out_c, float *__restrict__ out_y,
                                                     float scale, float floor_) {
  __shared__ __attribute__((aligned(32))) float2 sA[kPK][kPPad];
  __shared__ __attribute__((aligned(32))) float2 sB[kPK][kPPad];
  const int b = blockIdx.z;
  const int r0 = blockIdx.y * kPTile, c0 = blockIdx.x * kPTile;
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;
  const float2 *Ab = A + (int64_t)b * as;
  const float2 *Bb = B + (int64_t)b * bs;
  float2 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = make_float2(0.0f, 0.0f);

  for (int k0 = 0; k0 < K; k0 += kPK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + kPT * u;
      const int rr = AK ? e / kPK : e % kPTile, kk = AK ? e % kPK : e / kPTile;
      const int r = r0 + rr;
      sA[kk][rr] = r < R ? Ab[r * ars + (int64_t)(k0 + kk) * aks] : make_float2(0.0f, 0.0f);
      const int cc = BK ? e / kPK : e % kPTile, kb = BK ? e % kPK : e / kPTile;
      const int c = c0 + cc;
      sB[kb][cc] = c < C ? Bb[(int64_t)(k0 + kb) * bks + c * bcs] : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kPK; ++kk) {
      float2 a[4], w[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) a[x] = sA[kk][4 * tr + x];
#pragma unroll
      for (int y = 0; y < 4; ++y) w[y] = sB[kk][4 * tc + y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          acc[x][y].x = fmaf(a[x].x, w[y].x, fmaf(-a[x].y, w[y].y, acc[x][y].x));
          acc[x][y].y = fmaf(a[x].x, w[y].y, fmaf(a[x].y, w[y].x, acc[x][y].y));
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int r = r0 + 4 * tr + x;
    if (r >= R) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int c = c0 + 4 * tc + y;
      if (c >= C) continue;
      const int64_t o = ((int64_t)b * R + r) * C + c;
      if constexpr (LOG) {
        const float p = acc[x][y].x * acc[x][y].x + acc[x][y].y * acc[x][y].y;
        out_y[o] = logf(fmaf(scale, p, floor_));
      } else {
        out_c[o] = acc[x][y];
      }
    }
  }
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

fzp_status_t pfail(fzp_status_t s, const std::string &m) {
  set_last_error(m);
  return s;
}

bool prior_cfg_ok(const fzp_prior_t *c) {
  return c && std::isfinite(c->D) && c->D > 0.0 && c->M >= 1 && c->M <= 4096 && c->Np >= 16 && c->Np <= 1024 &&
         c->Np % 16 == 0 && c->ss >= 1 && c->ss <= 16 && c->n_creases >= 0 && c->n_creases <= kMaxCreases &&
         std::isfinite(c->floor_) && c->floor_ > 0.0;
}

// workspace: E [M][Np], then per instance g [Np][Np] and the row transform [Np][M]
size_t prior_bytes(const fzp_prior_t *c, int32_t n) {
  const size_t e = align256((size_t)c->M * c->Np * sizeof(float2));
  const size_t per = (size_t)c->Np * c->Np + (size_t)c->Np * c->M;
  return e + align256((size_t)n * per * sizeof(float2));
}

}  // namespace

}  // namespace fzp

extern "C" fzp_status_t fzp_pupil_prior_workspace(const fzp_prior_t *cfg, int32_t n_max, size_t *bytes) {
  if (!fzp::prior_cfg_ok(cfg) || n_max < 1 || !bytes)
    return fzp::pfail(FZP_E_INVAL, "fzp_pupil_prior_workspace: bad argument");
  *bytes = fzp::prior_bytes(cfg, n_max);
  return FZP_OK;
}

extern "C" fzp_status_t fzp_pupil_prior(const fzp_prior_t *cfg, const double *creases_dev, const double *lam_dev,
                                        int32_t n, float *y_dev, void *workspace, size_t workspace_bytes,
                                        void *stream) {
  using namespace fzp;
  if (!prior_cfg_ok(cfg) || n < 0) return pfail(FZP_E_INVAL, "fzp_pupil_prior: bad configuration");
  if (n == 0) return FZP_OK;
  if (n > 65535 || !lam_dev || !y_dev || !workspace || (cfg->n_creases > 0 && !creases_dev))
    return pfail(FZP_E_INVAL, "fzp_pupil_prior: NULL pointer or n > 65535");
  if (workspace_bytes < prior_bytes(cfg, n)) return pfail(FZP_E_NOMEM, "fzp_pupil_prior: workspace too small");
  const int Np = cfg->Np, M = cfg->M;
  hipStream_t st = (hipStream_t)stream;
  char *ws = (char *)workspace;
  float2 *E = (float2 *)ws;
  float2 *G = (float2 *)(ws + align256((size_t)M * Np * sizeof(float2)));
  float2 *H = G + (size_t)n * Np * Np;
  const int64_t ne = (int64_t)M * Np;
  hipLaunchKernelGGL(k_prior_dft, dim3((unsigned)((ne + kPT - 1) / kPT)), dim3(kPT), 0, st, Np, M, E);
  hipLaunchKernelGGL(k_prior_pupil, dim3((unsigned)(((int64_t)Np * Np + kPT - 1) / kPT), (unsigned)n), dim3(kPT), 0,
                     st, creases_dev, cfg->n_creases, lam_dev, cfg->D, Np, cfg->ss, G);
  // rows: H[b][j][q] = sum_i g[b][j][i] E[q][i]
  const dim3 g1((unsigned)((M + kPTile - 1) / kPTile), (unsigned)((Np + kPTile - 1) / kPTile), (unsigned)n);
  hipLaunchKernelGGL((k_prior_cgemm<true, true, false>), g1, dim3(kPT), 0, st, G, (int64_t)Np * Np, (int64_t)Np,
                     (int64_t)1, E, (int64_t)0, (int64_t)1, (int64_t)Np, Np, Np, M, H, (float *)nullptr, 0.0f, 0.0f);
  // columns: S[b][p][q] = sum_j E[p][j] H[b][j][q], then ln(16 |S|^2 / (pi^2 Np^4) + floor)
  const double npd = (double)Np;
  const float scale = (float)(16.0 / (M_PI * M_PI * npd * npd * npd * npd));
  const dim3 g2((unsigned)((M + kPTile - 1) / kPTile), (unsigned)((M + kPTile - 1) / kPTile), (unsigned)n);
  hipLaunchKernelGGL((k_prior_cgemm<true, false, true>), g2, dim3(kPT), 0, st, E, (int64_t)0, (int64_t)Np,
                     (int64_t)1, H, (int64_t)Np * M, (int64_t)M, (int64_t)1, M, Np, M, (float2 *)nullptr, y_dev,
                     scale, (float)cfg->floor_);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pfail(FZP_E_DEVICE, std::string("fzp_pupil_prior: ") + hipGetErrorString(e));
  return FZP_OK;
}
