// mci_device.h -- device-side helpers shared by the libmci kernels: complex arithmetic
// on float2/double2, storage conversions, and the radix-R butterflies of a Stockham
// (self-sorting) mixed-radix FFT.
//
// Stockham pass with radix R at stage size Ns (the product of the radices already
// applied): butterfly j in [0, len/R) reads x[j + r len/R], r < R, multiplies element r
// by W_{Ns R}^{(j mod Ns) r}, takes a length-R DFT and writes element r to
// (j / Ns) Ns R + (j mod Ns) + r Ns.  After the last stage the output is in natural
// order.  W_L = e^{-2 pi i / L} for the forward direction (S = -1), its conjugate for
// the inverse (S = +1); every twiddle is read from one table e^{-2 pi i k / len}.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mci {

// The dispatcher hands workgroup b of a launch to XCD b mod 8.  xcd_block renumbers the
// launch so that each XCD takes one contiguous range of logical blocks (XCD x: logical
// x floor(G/8) + min(x, G mod 8) + b / 8), which keeps neighbouring blocks that read the same
// data on one XCD and its L2.  A bijection on [0, G) for any grid size G.
constexpr int kXcds = 8;

// Word 3 of a buffer resource for untyped (raw) access on this architecture: buffer loads
// then take a byte offset in one VGPR and a uniform one in an SGPR, with no 64-bit address
// arithmetic per access (out-of-range offsets read zero).
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
  const int64_t x = b % kXcds, s = b / kXcds, q = G / kXcds, r = G % kXcds;
  return x * q + (x < r ? x : r) + s;
}

template <typename T> struct cvec;
template <> struct cvec<float> { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using cx = typename cvec<T>::type;

template <typename C> __host__ __device__ __forceinline__ C cmake(decltype(C::x) re, decltype(C::x) im) {
  C c;
  c.x = re;
  c.y = im;
  return c;
}
template <typename C> __host__ __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __host__ __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __host__ __device__ __forceinline__ C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __host__ __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __host__ __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return cmake<C>(a.x * s, a.y * s); }
// multiply by S*i (S = +-1)
template <int S, typename C> __host__ __device__ __forceinline__ C cmul_si(C a) {
  return S > 0 ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}
// twiddle from the forward table, conjugated for the inverse direction
template <int S, typename C> __device__ __forceinline__ C twid(const C* __restrict__ tw, int64_t k) {
  C w = tw[k];
  return S > 0 ? cconj(w) : w;
}

// ---------------------------------------------------------------- storage conversion
template <typename T, typename St> __device__ __forceinline__ T ld_as(const St* p, int64_t i);
template <> __device__ __forceinline__ float ld_as<float, float>(const float* p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ double ld_as<double, double>(const double* p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ld_as<float, __half>(const __half* p, int64_t i) { return __half2float(p[i]); }
template <typename T, typename St> __device__ __forceinline__ void st_as(St* p, int64_t i, T v);
template <> __device__ __forceinline__ void st_as<float, float>(float* p, int64_t i, float v) { p[i] = v; }
template <> __device__ __forceinline__ void st_as<double, double>(double* p, int64_t i, double v) { p[i] = v; }
template <> __device__ __forceinline__ void st_as<float, __half>(__half* p, int64_t i, float v) { p[i] = __float2half(v); }

// ---------------------------------------------------------------- small DFTs
// In-register DFT of R points with sign S.  Radices 2, 4, 8 are written out; odd radices
// take their roots of unity from the transform's twiddle table (root m of order R is
// entry m * len / R).
template <int S, typename C> __device__ __forceinline__ void dft2(C& a, C& b) {
  C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int S, typename C> __device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  C t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = cmul_si<S>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int S, typename C> __device__ __forceinline__ void dft8(C* v) {
  using T = decltype(C::x);
  const T h = (T)0.70710678118654752440084436210485;  // sqrt(1/2)
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<S>(e0, e1, e2, e3);
  dft4<S>(o0, o1, o2, o3);
  // o_k *= e^{S i pi k / 4}
  o1 = cmake<C>(h * (o1.x - (T)S * o1.y), h * (o1.y + (T)S * o1.x));
  o2 = cmul_si<S>(o2);
  o3 = cmake<C>(h * (-o3.x - (T)S * o3.y), h * (-o3.y + (T)S * o3.x));
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 3 points: X1,2 = a - (b + c)/2 +- S i (sqrt 3 / 2)(b - c)
template <int S, typename C> __device__ __forceinline__ void dft3(C& a, C& b, C& c) {
  using T = decltype(C::x);
  const T h = (T)0.86602540378443864676372317075294;  // sqrt(3)/2
  const C s = cadd(b, c);
  const C m = cmake<C>(a.x - (T)0.5 * s.x, a.y - (T)0.5 * s.y);
  const C d = cmul_si<S>(csub(b, c));
  a = cadd(a, s);
  b = cmake<C>(m.x + h * d.x, m.y + h * d.y);
  c = cmake<C>(m.x - h * d.x, m.y - h * d.y);
}

// 12 = 3 x 4 by the prime-factor (Good-Thomas) mapping, no twiddles: input n = (4 n1 + 3 n2)
// mod 12, output k = (4 k1 + 9 k2) mod 12, so that e^{2 pi i n k / 12} = w3^{n1 k1} w4^{n2 k2}.
template <int S, typename C> __device__ __forceinline__ void dft12(C* v) {
  C a[3][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) a[n1][n2] = v[(4 * n1 + 3 * n2) % 12];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft3<S>(a[0][n2], a[1][n2], a[2][n2]);
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) dft4<S>(a[k1][0], a[k1][1], a[k1][2], a[k1][3]);
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[(4 * k1 + 9 * k2) % 12] = a[k1][k2];
}

template <int R, int S, typename C>
__device__ __forceinline__ void dft_odd(C* v, const C* __restrict__ tw, int64_t len) {
  C out[R];
  const int64_t step = len / R;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    C acc = v[0];
#pragma unroll
    for (int q = 1; q < R; ++q) acc = cadd(acc, cmul(v[q], twid<S>(tw, (int64_t)((q * s) % R) * step)));
    out[s] = acc;
  }
#pragma unroll
  for (int s = 0; s < R; ++s) v[s] = out[s];
}

template <int R, int S, typename C>
__device__ __forceinline__ void dft_small(C* v, const C* __restrict__ tw, int64_t len) {
  if constexpr (R == 2) dft2<S>(v[0], v[1]);
  else if constexpr (R == 4) dft4<S>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<S>(v);
  else dft_odd<R, S>(v, tw, len);
}

}  // namespace mci
