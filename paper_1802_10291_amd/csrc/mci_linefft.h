// mci_linefft.h -- register-staged Stockham FFTs of one line by a group of lanes, shared by
// the 2-D line passes and the two-pass (four-step) transforms of the multi-pass path.
//
// A group of G lanes transforms one line of length L: lane l holds elements l + G c, c < E =
// L / G, and each Stockham pass of radix R (R divides E) runs E / R butterflies per lane
// through the group's LDS scratch of padded(L) slots; after the last pass lane l holds
// output elements l + G c.  Lengths: {32, 48, 64, 96, 128, 192, 256, 384, 512}.
#pragma once
#include <hip/hip_runtime.h>

#include "mci_device.h"

namespace mci {
namespace lfft {

__device__ __forceinline__ int pad(int x) { return x + (x >> 4); }
constexpr int padded(int n) { return n + (n >> 4) + 1; }

template <int R, int S>
__device__ __forceinline__ void dft_r(float2* u) {
  if constexpr (R == 2) dft2<S>(u[0], u[1]);
  else if constexpr (R == 4) dft4<S>(u[0], u[1], u[2], u[3]);
  else if constexpr (R == 8) dft8<S>(u);
  else if constexpr (R == 12) dft12<S>(u);
  else {
    static_assert(R == 16, "radix");
    constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, h = 0.70710678118654752440f;
    float2 a[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = u[q]; a[q + 4] = u[q + 4]; a[q + 8] = u[q + 8]; a[q + 12] = u[q + 12];
      dft4<S>(a[q], a[q + 4], a[q + 8], a[q + 12]);
    }
    const float cs[10] = {1.f, c1, h, s1, 0.f, -s1, -h, -c1, -1.f, -c1};
    const float sn[10] = {0.f, s1, h, c1, 1.f, c1, h, s1, 0.f, -s1};
#pragma unroll
    for (int q = 1; q < 4; ++q)
#pragma unroll
      for (int s = 1; s < 4; ++s) {
        const int m = q * s;
        const float2 x = a[q + 4 * s];
        if (m == 4) {   // e^{S i pi / 2} = S i: a swap and a sign, no products
          a[q + 4 * s] = cmul_si<S>(x);
          continue;
        }
        const float wc = cs[m], ws = (float)S * sn[m];
        a[q + 4 * s] = make_float2(x.x * wc - x.y * ws, x.x * ws + x.y * wc);
      }
#pragma unroll
    for (int s = 0; s < 4; ++s) dft4<S>(a[4 * s], a[4 * s + 1], a[4 * s + 2], a[4 * s + 3]);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) u[s + 4 * t] = a[t + 4 * s];
  }
}

template <int... Rs> struct RList {};

// Length-L transform by a group of G lanes (lane l holds elements l + G c, c < E = L / G);
// buffer = this group's LDS scratch of padded(L) slots.  Same Stockham scheme as the 1-D
// kernel; the whole workgroup passes the barriers together.
template <int L, int G, int S, int NS, int R, int... Rest>
__device__ __forceinline__ void gfft_passes(float2* __restrict__ buf, int l, float2 (&v)[L / G],
                                            const float2* __restrict__ tw, RList<R, Rest...>) {
  constexpr int E = L / G;
  constexpr int BPT = E / R;
  static_assert(BPT * R == E, "radix must divide the elements per lane");
  float2 u[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) u[b][r] = v[b + r * BPT];
    if constexpr (NS > 1) {
      const int j = l + G * b;
      const int k1 = (j % NS) * (L / (NS * R));
      float2 w1 = tw[k1];
      if constexpr (S > 0) w1.y = -w1.y;
      float2 w = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        if (r > 1) w = (r % 4 == 0) ? [&] { float2 t = tw[r * k1]; if constexpr (S > 0) t.y = -t.y; return t; }()
                                    : cmul(w, w1);
        u[b][r] = cmul(u[b][r], w);
      }
    }
    dft_r<R, S>(u[b]);
  }
  if constexpr (sizeof...(Rest) == 0) {
#pragma unroll
    for (int b = 0; b < BPT; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + r * BPT] = u[b][r];
  } else {
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = l + G * b;
      const int base = (j / NS) * NS * R + (j % NS);
      // for power-of-two NS and R, base % 16 + (r NS) % 16 < 16, so pad(base + r NS) =
      // pad(base) + r NS + (r NS) / 16 (one address per butterfly); otherwise pad each
      constexpr bool pow2 = (NS & (NS - 1)) == 0 && (R & (R - 1)) == 0;
      const int pb = pad(base);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (pow2) buf[pb + r * NS + (r * NS) / 16] = u[b][r];
        else buf[pad(base + r * NS)] = u[b][r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < E; ++c) v[c] = buf[pad(l + G * c)];
    gfft_passes<L, G, S, NS * R>(buf, l, v, tw, RList<Rest...>{});
  }
}

// Per line length: E elements per lane (G = L / E lanes per line pair) and the radices of
// the Stockham passes, each dividing E.
template <int L> struct LineFFT;
template <> struct LineFFT<32> { static constexpr int E = 8; using type = RList<8, 4>; };
template <> struct LineFFT<48> { static constexpr int E = 12; using type = RList<12, 4>; };
template <> struct LineFFT<64> { static constexpr int E = 8; using type = RList<8, 8>; };
template <> struct LineFFT<96> { static constexpr int E = 12; using type = RList<12, 4, 2>; };
template <> struct LineFFT<128> { static constexpr int E = 8; using type = RList<8, 8, 2>; };
template <> struct LineFFT<192> { static constexpr int E = 12; using type = RList<12, 4, 4>; };
template <> struct LineFFT<256> { static constexpr int E = 16; using type = RList<16, 16>; };
template <> struct LineFFT<384> { static constexpr int E = 12; using type = RList<12, 4, 4, 2>; };
template <> struct LineFFT<512> { static constexpr int E = 8; using type = RList<8, 8, 8>; };

// The one- and two-pass transforms hold one transform per lane group (the 2-D passes hold the
// inputs of several output transforms at once), so they take fewer elements per lane at 256.
template <int L> struct LinesFFT : LineFFT<L> {};
template <> struct LinesFFT<256> { static constexpr int E = 8; using type = RList<8, 8, 4>; };

template <int L, int S, typename F = LineFFT<L>>
__device__ __forceinline__ void gfft(float2* buf, int l, float2 (&v)[F::E], const float2* tw) {
  gfft_passes<L, L / F::E, S, 1>(buf, l, v, tw, typename F::type{});
}

// COLS: lines are the columns of x [B][N][W] (blockIdx.x = block of 32 columns, blockIdx.y =
// image); output [B][SC N][W].  Rows: lines are the rows of x [lines][N], output [lines][SC N].

}  // namespace lfft
}  // namespace mci
