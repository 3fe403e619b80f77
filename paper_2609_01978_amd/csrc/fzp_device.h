// Device helpers: complex float64 arithmetic, exact phase reduction in turns,
// and the LDS-resident 4096-point float64 FFT used by the Bluestein passes.
#pragma once

#include <hip/hip_runtime.h>

namespace fzp {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// e^{2 pi i t}.  t - rint(t) is exact in float64, so the reduction loses
// nothing; sincospi then works on |2t| <= 1.
__device__ __forceinline__ double2 cexp_turns(double t) {
  const double f = t - rint(t);
  double s, c;
  sincospi(2.0 * f, &s, &c);
  return make_double2(c, s);
}

// Radix-4 butterfly, DIR = -1 forward (W4 = -i), +1 inverse (W4 = +i).
template <int DIR>
__device__ __forceinline__ void dft4(double2 &x0, double2 &x1, double2 &x2, double2 &x3) {
  const double2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), d = csub(x1, x3);
  const double2 t3 = DIR < 0 ? make_double2(d.y, -d.x) : make_double2(-d.y, d.x);
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

// 16-point DFT in registers, natural order in and out: X[k] = sum_n x[n] e^{DIR 2 pi i nk/16}.
// n = n1 + 4 n2, k = k2 + 4 k1: DFT4 over n2, twiddle W16^{n1 k2}, DFT4 over n1.
template <int DIR>
__device__ __forceinline__ void dft16(double2 v[16]) {
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) dft4<DIR>(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]);
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
  constexpr double c2 = 0.70710678118654752440;
  constexpr double sg = DIR < 0 ? -1.0 : 1.0;
  // y[n1][k2] sits at v[n1 + 4 k2]
  v[1 + 4] = cmul(v[1 + 4], make_double2(c1, sg * s1));    // W^1
  v[1 + 8] = cmul(v[1 + 8], make_double2(c2, sg * c2));    // W^2
  v[1 + 12] = cmul(v[1 + 12], make_double2(s1, sg * c1));  // W^3
  v[2 + 4] = cmul(v[2 + 4], make_double2(c2, sg * c2));    // W^2
  v[2 + 8] = make_double2(-sg * v[2 + 8].y, sg * v[2 + 8].x);  // W^4 = DIR i
  v[2 + 12] = cmul(v[2 + 12], make_double2(-c2, sg * c2)); // W^6
  v[3 + 4] = cmul(v[3 + 4], make_double2(s1, sg * c1));    // W^3
  v[3 + 8] = cmul(v[3 + 8], make_double2(-c2, sg * c2));   // W^6
  v[3 + 12] = cmul(v[3 + 12], make_double2(-c1, -sg * s1)); // W^9
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) dft4<DIR>(v[4 * k2], v[4 * k2 + 1], v[4 * k2 + 2], v[4 * k2 + 3]);
  double2 o[16];
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2)
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) o[k2 + 4 * k1] = v[4 * k2 + k1];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = o[k];
}

// Keeps a value opaque to the optimiser, so that work depending on it stays
// where it is written instead of being hoisted out of loops (hoisted twiddle
// powers would pin 120 registers per lane).
__device__ __forceinline__ double2 opaque(double2 w) {
  asm volatile("" : "+v"(w.x), "+v"(w.y));
  return w;
}

// v[r] *= w^r, r = 1..15 (w a unit phasor), by a recurrence.
__device__ __forceinline__ void twiddle16(double2 v[16], double2 w) {
  w = opaque(w);
  double2 wr = w;
#pragma unroll
  for (int r = 1; r < 16; ++r) {
    v[r] = cmul(v[r], wr);
    wr = cmul(wr, w);
  }
}

__device__ __forceinline__ double2 conj(double2 a) { return make_double2(a.x, -a.y); }

// Per-thread twiddle bases of the two twiddled passes (forward direction):
// e^{-2 pi i (j mod 16)/256} and e^{-2 pi i j/4096}.
struct Tw {
  double2 w1, w2;
};
__device__ __forceinline__ Tw fft_twiddles() {
  const int j = threadIdx.x;
  Tw t;
  double s, c;
  sincospi(2.0 * (double)(j & 15) / 256.0, &s, &c);
  t.w1 = make_double2(c, -s);
  sincospi(2.0 * (double)j / 4096.0, &s, &c);
  t.w2 = make_double2(c, -s);
  return t;
}

constexpr int kLdsN = 4096 + 256;  // one pad slot per 16 entries

// In-register/LDS Stockham radix-16 FFT of length 4096 by 256 threads.
// On entry thread j holds x[j + 256 r] in v[r]; on exit X[j + 256 r].
// DIR = -1: X[k] = sum x[n] e^{-2 pi i nk/4096}; DIR = +1: unnormalised inverse.
// s: kLdsN complex entries; entry a lives at a + a/16 (padding against bank
// conflicts), so every access below is a per-thread base plus a constant.
// Contains the barriers it needs.
template <int DIR>
__device__ __forceinline__ void fft4096(double2 v[16], double2 *s, const Tw &tw) {
  const int j = threadIdx.x;
  const int b0 = 17 * j;                               // pad(16 j + r) = 17 j + r
  const int b1 = j + (j >> 4);                         // pad(j + 256 r) = b1 + 272 r
  const int e2 = (j >> 4) * 256 + (j & 15);
  const int b2 = e2 + (e2 >> 4);                       // pad(e2 + 16 r) = b2 + 17 r
  // pass 0 (Ns = 1): no twiddle
  dft16<DIR>(v);
  __syncthreads();  // earlier readers of s are done
#pragma unroll
  for (int r = 0; r < 16; ++r) s[b0 + r] = v[r];
  __syncthreads();
  // pass 1 (Ns = 16)
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = s[b1 + 272 * r];
  twiddle16(v, DIR < 0 ? tw.w1 : conj(tw.w1));
  dft16<DIR>(v);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) s[b2 + 17 * r] = v[r];
  __syncthreads();
  // pass 2 (Ns = 256)
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = s[b1 + 272 * r];
  twiddle16(v, DIR < 0 ? tw.w2 : conj(tw.w2));
  dft16<DIR>(v);
}

}  // namespace fzp
