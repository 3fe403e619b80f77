// Non-paraxial variant of the propagation: the semi-analytical chirp-z
// transform (SA-CZT, Sec. 3.6, Fig. 5).  The binary zone plate with the
// sag-corrected radii of Eq. 3 is centred in a zero-padded Np x Np grid
// (Np >= 1.5 N); its 2-D FFT is multiplied by exp(i h(K) z), the remainder of
// the exact transfer function exp(i k_z z), k_z = sqrt(k0^2 - K^2), after the
// fitted quadratic c k_max + d K^2 / k_max (SAFT, Sec. 3.4, Fig. 3), and
// transformed back; the quadratic part is then a Fresnel-type transform with
// Z = 4 pi |d| z / k_max in place of lambda z, which the float64 blocked
// Bluestein passes of fzp_fft.hip evaluate onto the ROI (the CZT zoom).
//
// The 2-D FFT of the padded field lives in HBM (float64 complex, Np^2 x 16 B,
// 29.9 GB at N = 28672).  Each axis of length Np = n1 n2 is transformed in two
// passes of small LDS-resident FFTs (four-step, without transposes): with
// x = i1 + n1 i2 and k = k2 + n2 k1,
//   pass A: for each i1, DFT_n2 over i2, times W_Np^(i1 k2), stored at i1 + n1 k2;
//   pass B: for each k2, DFT_n1 over i1 (contiguous), stored at n1 k2 + k1.
// The spectrum is left in that digit-permuted order: the transfer function is
// evaluated for the permuted index and the inverse passes undo the order.  The
// last forward pass (B along y), the product with the transfer function and
// the first inverse pass (B along y) touch the same n1 elements, so they are
// one kernel: seven passes over the array in all, the first of which
// generates the aperture instead of reading it.

#include "fzp_device.h"
#include "fzp_internal.h"

namespace fzp {

namespace {

constexpr int kSaThreads = 512;
constexpr int kSaSlots = 2048;                  // complex elements per LDS buffer (two buffers)
constexpr int kSaEl = kSaSlots / kSaThreads;    // elements a thread moves to or from HBM

// Small DFTs in registers, natural order: X[k] = sum_n x[n] e^{DIR 2 pi i n k / R}.
template <int DIR>
__device__ __forceinline__ void dft2(double2 &a, double2 &b) {
  const double2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft3(double2 &a, double2 &b, double2 &c) {
  constexpr double h = 0.86602540378443864676;  // sqrt(3)/2
  const double2 s = cadd(b, c), d = csub(b, c);
  const double2 m = make_double2(a.x - 0.5 * s.x, a.y - 0.5 * s.y);
  // i DIR h (b - c)
  const double2 r = make_double2(-DIR * h * d.y, DIR * h * d.x);
  a = cadd(a, s);
  b = cadd(m, r);
  c = csub(m, r);
}

template <int DIR>
__device__ __forceinline__ void dft5(double2 v[5]) {
  constexpr double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;  // cos(2 pi/5), cos(4 pi/5)
  constexpr double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;   // sin(2 pi/5), sin(4 pi/5)
  const double2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  const double2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  const double2 m1 = make_double2(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
  const double2 m2 = make_double2(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
  // DIR i (s1 b1 + s2 b2) and DIR i (s2 b1 - s1 b2)
  const double2 n1 = make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
  const double2 n2 = make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
  const double2 r1 = make_double2(-DIR * n1.y, DIR * n1.x);
  const double2 r2 = make_double2(-DIR * n2.y, DIR * n2.x);
  v[0] = cadd(v[0], cadd(a1, a2));
  v[1] = cadd(m1, r1);
  v[4] = csub(m1, r1);
  v[2] = cadd(m2, r2);
  v[3] = csub(m2, r2);
}

template <int DIR>
__device__ __forceinline__ void dft8(double2 v[8]) {
  // even / odd halves by 4-point DFTs, then the radix-2 combination with W8^k
  double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  constexpr double r = 0.70710678118654752440;
  // W8^1 = (r, DIR r), W8^2 = (0, DIR), W8^3 = (-r, DIR r)
  o1 = cmul(o1, make_double2(r, DIR * r));
  o2 = make_double2(-DIR * o2.y, DIR * o2.x);
  o3 = cmul(o3, make_double2(-r, DIR * r));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

struct Radices {
  int n, nst;
  int r[kSaMaxStages];
  const double2 *tw;  // W_n^k = e^{-2 pi i k / n}, k < n (in LDS)
};

// One radix-R Stockham stage over G transforms of length n held in LDS at
// src[t * ld + s] (slot s fastest), into dst; Ns = product of the earlier
// stages' radices.  R is a compile-time constant, so a butterfly moves exactly
// R values.
template <int DIR, int R>
__device__ __forceinline__ void fft_stage(const double2 *src, double2 *dst, int G, int ld, int n, int Ns,
                                          const double2 *tw) {
  const int nb = n / R;           // butterflies per transform
  const int step = n / (Ns * R);  // W_{Ns R}^m = W_n^(m step)
  for (int b = threadIdx.x; b < G * nb; b += kSaThreads) {
    const int s = b % G, j = b / G;
    const int jm = j % Ns;
    double2 v[8];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(j + r * nb) * ld + s];
    if (jm != 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const double2 w = tw[r * jm * step];
        v[r] = cmul(v[r], DIR < 0 ? w : conj(w));
      }
    }
    if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
    if constexpr (R == 3) dft3<DIR>(v[0], v[1], v[2]);
    if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
    if constexpr (R == 5) dft5<DIR>(v);
    if constexpr (R == 8) dft8<DIR>(v);
    const int base = (j - jm) * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(base + r * Ns) * ld + s] = v[r];
  }
}

// G transforms of length n held in LDS at src[t * ld + s] (slot s fastest):
// mixed-radix Stockham stages (autosort, ping-pong between src and dst).
// Returns the buffer with the result in natural order.  Contains the barriers
// it needs; entered after the data is visible to every thread.
template <int DIR>
__device__ double2 *lds_fft(double2 *src, double2 *dst, int G, int ld, const Radices &f) {
  int Ns = 1;
  const int n = f.n;
  for (int st = 0; st < f.nst; ++st) {
    const int R = f.r[st];
    switch (R) {
      case 2: fft_stage<DIR, 2>(src, dst, G, ld, n, Ns, f.tw); break;
      case 3: fft_stage<DIR, 3>(src, dst, G, ld, n, Ns, f.tw); break;
      case 4: fft_stage<DIR, 4>(src, dst, G, ld, n, Ns, f.tw); break;
      case 5: fft_stage<DIR, 5>(src, dst, G, ld, n, Ns, f.tw); break;
      default: fft_stage<DIR, 8>(src, dst, G, ld, n, Ns, f.tw); break;
    }
    __syncthreads();
    double2 *t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  return src;
}

// Eq. 3 zone index floor(c2 q / (sqrt(1 + q) + 1)), q = K c1, in the same
// float64 operations, in the same order and without contraction, as the
// reference definition, so both sides decide every sample alike.
__device__ __forceinline__ int64_t zone_eq3(double K, double c1, double c2) {
#pragma clang fp contract(off)
  const double q = K * c1;
  const double n = c2 * (q / (sqrt(1.0 + q) + 1.0));
  return (int64_t)floor(n);
}

// Aperture transmission at padded position (y, x): zero outside the N x N
// aperture and the disc, else the open/closed zone times the crease phase.
__device__ __forceinline__ double2 sa_aperture(const SaDev &a, int64_t y, int64_t x) {
  const int64_t j = y - a.off, i = x - a.off;
  if (j < 0 || j >= a.N || i < 0 || i >= a.N) return make_double2(0.0, 0.0);
  const double cj = (double)(2 * j - a.N + 1), ci = (double)(2 * i - a.N + 1);
  const double K = ci * ci + cj * cj;  // exact integer
  if (K > a.kmax_disc) return make_double2(0.0, 0.0);
  const int64_t zone = a.radii_eq3 ? zone_eq3(K, a.c1, a.c2) : (int64_t)(K * a.kappa);
  if (((zone & 1) ^ a.centre_open) == 0) return make_double2(0.0, 0.0);
  if (a.n_creases == 0) return make_double2(1.0, 0.0);
  const double xs = 0.5 * ci * a.dx, ys = 0.5 * cj * a.dx;
  double turns = 0.0;
  for (int k = 0; k < a.n_creases; ++k) {
    const CreaseDev &c = a.cr[k];
    const double d = xs * c.c + ys * c.s - c.rho;
    turns += c.h_over_lambda * exp(-c.inv2s2 * d * d);
  }
  return cexp_turns(turns);
}

// The padded field is streamed: each pass reads and writes every element once,
// so its loads and stores bypass cache allocation (non-temporal), leaving the
// caches to the twiddle tables.
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 field_load(const double2 *p) {
  const dvec2 v = __builtin_nontemporal_load((const dvec2 *)p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void field_store(double2 *p, double2 v) {
  dvec2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, (dvec2 *)p);
}

// Signed frequency index of k in [0, Np) (numpy's fftfreq order).
__device__ __forceinline__ double signed_freq(int64_t k, int64_t Np) {
  return (double)(k < (Np + 1) / 2 ? k : k - Np);
}

// exp(i h(K) z) / Np^2 with h = k_z - c k_max - d K^2 / k_max, zero for
// evanescent K; in turns, with rho^2 = K^2 / (2 pi)^2 and c k_max = k0:
//   h z / (2 pi) = -z rho^2 (1 / (sqrt(1/lambda^2 - rho^2) + 1/lambda) + d lambda / k_fit).
__device__ __forceinline__ double2 sa_transfer(const SaDev &a, int64_t kx, int64_t ky) {
  const double fx = signed_freq(kx, a.Np), fy = signed_freq(ky, a.Np);
  const double rho2 = (fx * fx + fy * fy) * a.inv_L2;
  if (rho2 > a.inv_lam2) return make_double2(0.0, 0.0);
  const double turns = -a.z * rho2 * (1.0 / (sqrt(a.inv_lam2 - rho2) + a.inv_lam) + a.coef);
  return cscale(cexp_turns(turns), a.norm);
}

enum SaPass : int {
  kXAgen = 0,   // X pass A, forward, aperture generated
  kXB = 1,      // X pass B (forward or inverse)
  kYA = 2,      // Y pass A (forward: twiddle after; inverse: twiddle before)
  kYBfilt = 3,  // Y pass B forward, transfer function, Y pass B inverse
  kXAinv = 4,   // X pass A, inverse (twiddle before)
};

// One pass.  Work-group tiles:
//   A passes (strided, transform length n2): G consecutive unit-stride
//     positions (i1 or x) x all n2 elements;
//   X pass B (contiguous, length n1): G consecutive groups of n1 elements;
//   Y pass B (strided, length n1): G consecutive x x all n1 rows.
template <int PASS, int DIR>
__global__ __launch_bounds__(kSaThreads, 2) void k_sa_pass(SaDev a, double2 *__restrict__ U, int G, int64_t n_tiles) {
  extern __shared__ __attribute__((aligned(16))) double2 sa_lds[];
  const int64_t Np = a.Np;
  const int n1 = a.n1, n2 = a.n2;
  const bool alen2 = PASS == kXAgen || PASS == kYA || PASS == kXAinv;
  const int n = alen2 ? n2 : n1;
  const int ld = G + 1;
  double2 *bufA = sa_lds, *bufB = sa_lds + (size_t)n * ld;
  const int64_t wg = blockIdx.x;
  // element (slot s, index t) -> array position
  int64_t base = 0, o = 0, u0 = 0, g0 = 0;
  int64_t nslot = G;
  if (PASS == kXAgen || PASS == kXAinv) {
    // row o, i1 = u0 + s, position o Np + i1 + n1 t
    const int64_t tiles = (n1 + G - 1) / G;
    o = wg / tiles;
    u0 = (wg % tiles) * G;
    nslot = n1 - u0 < G ? n1 - u0 : G;
    base = o * Np + u0;
  } else if (PASS == kXB) {
    // group g = g0 + s (g = y n2 + k2), position g n1 + t
    g0 = wg * G;
    const int64_t groups = Np * n2;
    nslot = groups - g0 < G ? groups - g0 : G;
    base = g0 * n1;
  } else {
    // Y passes: o = j1 (pass A) or k2 (pass B), x = u0 + s
    const int64_t tiles = (Np + G - 1) / G;
    o = wg / tiles;
    u0 = (wg % tiles) * G;
    nslot = Np - u0 < G ? Np - u0 : G;
    base = (PASS == kYA ? o : (int64_t)n1 * o) * Np + u0;
  }
  const int64_t tstride = PASS == kXAgen || PASS == kXAinv ? (int64_t)n1
                          : PASS == kXB                   ? 1
                          : PASS == kYA                   ? (int64_t)n1 * Np
                                                          : Np;
  const int total = G * n;
  // element k of this thread: e = tid + k kSaThreads -> (slot s, index t)
  auto slot_of = [&](int e, int &sl, int &t) {
    if (PASS == kXB) {
      sl = e / n;
      t = e % n;
    } else {
      sl = e % G;
      t = e / G;
    }
  };
  // ---- load (or generate) with the twiddle of inverse A passes; every load
  // of the thread is issued before the first is used
  if (PASS == kXAgen && (o < a.off || o >= a.off + a.N)) {
    // a row outside the aperture: its transform is zero
#pragma unroll
    for (int k = 0; k < kSaEl; ++k) {
      int sl, t;
      const int e = threadIdx.x + k * kSaThreads;
      slot_of(e, sl, t);
      if (e < total && sl < nslot) field_store(U + base + sl + t * tstride, make_double2(0.0, 0.0));
    }
    return;
  }
  double2 *twl = bufB + (size_t)n * ld;  // W_n^k of this pass's length
  {
    const double2 *twg = alen2 ? a.tw2 : a.tw1;
    for (int k = threadIdx.x; k < n; k += kSaThreads) twl[k] = twg[k];
  }
  {
    double2 v[kSaEl], w[kSaEl];
#pragma unroll
    for (int k = 0; k < kSaEl; ++k) {
      int sl, t;
      const int e = threadIdx.x + k * kSaThreads;
      slot_of(e, sl, t);
      v[k] = make_double2(0.0, 0.0);
      w[k] = make_double2(1.0, 0.0);
      if (e < total && sl < nslot) {
        if (PASS == kXAgen) {
          v[k] = sa_aperture(a, o, u0 + sl + (int64_t)n1 * t);
        } else {
          v[k] = field_load(U + base + (PASS == kXB ? (int64_t)sl * n : (int64_t)sl) + t * tstride);
          // W_Np^((u0 + s) t), (u0 + s) t < n1 n2 = Np: evaluated here exactly
          // as the table entry would be (each element needs a different one,
          // so a table read is a scattered cache-line fetch per element)
          if (PASS == kXAinv) w[k] = cexp_turns(-(double)((u0 + sl) * (int64_t)t) / (double)Np);
          if (PASS == kYA && DIR > 0) w[k] = a.twNp[o * t];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kSaEl; ++k) {
      int sl, t;
      const int e = threadIdx.x + k * kSaThreads;
      slot_of(e, sl, t);
      if (e < total) bufA[t * ld + sl] = (PASS == kXAinv || (PASS == kYA && DIR > 0)) ? cmul(v[k], conj(w[k])) : v[k];
    }
  }
  __syncthreads();
  Radices f{n, alen2 ? a.nst2 : a.nst1, {}, twl};
  for (int k = 0; k < kSaMaxStages; ++k) f.r[k] = alen2 ? a.rad2[k] : a.rad1[k];
  double2 *res = lds_fft<DIR>(bufA, bufB, G, ld, f);
  if (PASS == kYBfilt) {
    // res[t = k1][s]: ky = k2 + n2 k1 (k2 = o); x = u0 + s holds kx = x / n1 + n2 (x % n1)
#pragma unroll
    for (int k = 0; k < kSaEl; ++k) {
      const int e = threadIdx.x + k * kSaThreads;
      const int sl = e % G, t = e / G;
      if (e < total && sl < nslot) {
        const int64_t x = u0 + sl;
        const int64_t kx = x / n1 + (int64_t)n2 * (x % n1);
        const int64_t ky = o + (int64_t)n2 * t;
        res[t * ld + sl] = cmul(res[t * ld + sl], sa_transfer(a, kx, ky));
      }
    }
    __syncthreads();
    double2 *other = res == bufA ? bufB : bufA;
    res = lds_fft<+1>(res, other, G, ld, f);
  }
  // ---- store, with the twiddle of forward A passes
  {
    double2 w[kSaEl];
#pragma unroll
    for (int k = 0; k < kSaEl; ++k) {
      int sl, t;
      const int e = threadIdx.x + k * kSaThreads;
      slot_of(e, sl, t);
      w[k] = make_double2(1.0, 0.0);
      if (e < total && sl < nslot) {
        if (PASS == kXAgen) w[k] = cexp_turns(-(double)((u0 + sl) * (int64_t)t) / (double)Np);
        if (PASS == kYA && DIR < 0) w[k] = a.twNp[o * t];
      }
    }
#pragma unroll
    for (int k = 0; k < kSaEl; ++k) {
      int sl, t;
      const int e = threadIdx.x + k * kSaThreads;
      slot_of(e, sl, t);
      if (e >= total || sl >= nslot) continue;
      double2 v = res[t * ld + sl];
      if (PASS == kXAgen || (PASS == kYA && DIR < 0)) v = cmul(v, w[k]);
      field_store(U + base + (PASS == kXB ? (int64_t)sl * n : (int64_t)sl) + t * tstride, v);
    }
  }
}

// W_Np^m (m < Np), W_n1^k, W_n2^k: e^{-2 pi i m / n} by sincospi of the exact
// fraction m / n.
__global__ __launch_bounds__(256) void k_sa_twiddles(int64_t Np, int n1, int n2, double2 *twNp, double2 *tw1,
                                                     double2 *tw2) {
  const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (m < Np) twNp[m] = cexp_turns(-(double)m / (double)Np);
  if (m < n1) tw1[m] = cexp_turns(-(double)m / (double)n1);
  if (m < n2) tw2[m] = cexp_turns(-(double)m / (double)n2);
}

}  // namespace

int sa_group(int n, bool contiguous) {
  // slots per work-group: two LDS buffers of n (G + 1) complex within
  // 2 x kSaSlots (n <= 1024 keeps G >= 1); strided passes take a power of two
  // up to 16 consecutive positions (128 to 256 contiguous bytes per element row)
  int g = kSaSlots / n - 1;
  if (!contiguous) {
    int p = 1;
    while (2 * p <= g && 2 * p <= 16) p *= 2;
    g = p;
  }
  return g < 1 ? 1 : g;
}

// two ping-pong buffers of n (G + 1) complex and the W_n table
size_t sa_lds_bytes(int n, int G) { return ((size_t)2 * (size_t)n * (size_t)(G + 1) + (size_t)n) * sizeof(double2); }

hipError_t launch_sa_twiddles(const SaDev &a, double2 *twNp, double2 *tw1, double2 *tw2, hipStream_t st) {
  const int64_t blocks = (a.Np + 255) / 256;
  hipLaunchKernelGGL(k_sa_twiddles, dim3((unsigned)blocks), dim3(256), 0, st, a.Np, a.n1, a.n2, twNp, tw1, tw2);
  return hipGetLastError();
}

namespace {
template <int PASS, int DIR>
hipError_t launch_pass(const SaDev &a, double2 *U, hipStream_t st) {
  const bool alen2 = PASS == kXAgen || PASS == kYA || PASS == kXAinv;
  const int n = alen2 ? a.n2 : a.n1;
  const int G = sa_group(n, PASS == kXB);
  int64_t wgs;
  if (PASS == kXAgen || PASS == kXAinv) wgs = a.Np * ((a.n1 + G - 1) / G);
  else if (PASS == kXB) wgs = (a.Np * a.n2 + G - 1) / G;
  else if (PASS == kYA) wgs = (int64_t)a.n1 * ((a.Np + G - 1) / G);
  else wgs = (int64_t)a.n2 * ((a.Np + G - 1) / G);
  // every element of a work-group's G transforms is one of its threads' kSaEl
  if (wgs > 0x7fffffffLL || (int64_t)G * n > (int64_t)kSaEl * kSaThreads) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sa_pass<PASS, DIR>), dim3((unsigned)wgs), dim3(kSaThreads), sa_lds_bytes(n, G), st, a, U, G,
                     wgs);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_sa_field(const SaDev &a, double2 *U, hipStream_t st) {
  hipError_t e = launch_pass<kXAgen, -1>(a, U, st);
  if (e == hipSuccess) e = launch_pass<kXB, -1>(a, U, st);
  if (e == hipSuccess) e = launch_pass<kYA, -1>(a, U, st);
  if (e == hipSuccess) e = launch_pass<kYBfilt, -1>(a, U, st);
  if (e == hipSuccess) e = launch_pass<kYA, +1>(a, U, st);
  if (e == hipSuccess) e = launch_pass<kXB, +1>(a, U, st);
  if (e == hipSuccess) e = launch_pass<kXAinv, +1>(a, U, st);
  return e;
}

hipError_t init_sa_attributes() {
  static bool done = false;
  if (done) return hipSuccess;
  const int bytes = (2 * kSaSlots + 1024) * (int)sizeof(double2);
  hipError_t e = hipSuccess;
#define FZP_ATTR(P, D)                                                                                        \
  if (e == hipSuccess)                                                                                        \
    e = hipFuncSetAttribute((const void *)k_sa_pass<P, D>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  FZP_ATTR(kXAgen, -1)
  FZP_ATTR(kXB, -1)
  FZP_ATTR(kYA, -1)
  FZP_ATTR(kYBfilt, -1)
  FZP_ATTR(kYA, +1)
  FZP_ATTR(kXB, +1)
  FZP_ATTR(kXAinv, +1)
#undef FZP_ATTR
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace fzp
