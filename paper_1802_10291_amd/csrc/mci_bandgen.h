// mci_bandgen.h -- the real-mode apply (eq. matrixeqn1 with the output operator and the real
// part) evaluated at one bin of the polyphase-gathered output spectrum, for the inverse line
// transform of the real-mode path, which computes its input in place.
//
// With the channel spectra Z of one signal (the half-length transforms of the sample rows,
// or the full-length ones for odd N), X_m[r] = E[r'] + e^{-2 pi i r / N} O[r'] (r' = r mod H,
// E and O the DFTs of the even and odd samples recovered from Z), the band coefficient
// a(k) = sum_m X_m[k mod N] Tab[op][m][j][i] for k = n1 + i + j N, S(k) = (a(k) + conj a(-k)) / 2,
// and the bin b of the gathered spectrum is Zc[b] = sum over k = b mod P, |k| <= K, of
// S(k) (1 + i w^k), w = e^{2 pi i / n_out}; one complex inverse transform of length P = n_out / 2
// of Zc gives y[2q] + i y[2q + 1].  The inverse transform's first pass evaluates Zc as it
// loads its input, so Zc never goes through memory.
#pragma once
#include <hip/hip_runtime.h>

#include "mci_device.h"

namespace mci {

struct BandGen {
  const float2* Z;       // channel spectra, [signals][M][Lz]
  int64_t Lz;
  const float2* post;    // Bluestein output chirp applied to Z as it is read, or null
  const float2* wN;      // H entries e^{-2 pi i k / N}
  const float2* D;       // [n_ops][M][2K + 1]: the apply, real part and gather weight of X_m at k
  int M, n_ops, N, H, n1, K, P;
  int half_rows;         // Z holds half-length transforms (even N)
  int one;               // P >= 2K + 1: a bin holds at most one band position (k = b or b - P)
};

// X_m[r] of signal Zs for every channel (r in [0, N)): the transform itself for odd N, else
// E[r'] + e^{-2 pi i r / N} O[r'] from the half-length transform (r' = r mod H)
template <int MM>
__device__ __forceinline__ void chan_x(const BandGen& g, const float2* __restrict__ Zs, int r, float2 (&x)[MM]) {
  if (!g.half_rows) {
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      x[m] = make_float2(0.f, 0.f);
      if (m < g.M) {
        x[m] = Zs[m * g.Lz + r];
        if (g.post) x[m] = cmul(x[m], g.post[r]);
      }
    }
    return;
  }
  const int H = g.H;
  const int rh = r < H ? r : r - H;
  const int rr = rh == 0 ? 0 : H - rh;
  const float sg = r < H ? 1.f : -1.f;
  const float2 w = g.wN[rh];
  float2 p1 = make_float2(1.f, 0.f), p2 = p1;
  if (g.post) {
    p1 = g.post[rh];
    p2 = g.post[rr];
  }
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    x[m] = make_float2(0.f, 0.f);
    if (m < g.M) {
      float2 z1 = Zs[m * g.Lz + rh], z2 = Zs[m * g.Lz + rr];
      if (g.post) {
        z1 = cmul(z1, p1);
        z2 = cmul(z2, p2);
      }
      z2 = make_float2(z2.x, -z2.y);
      const float2 e = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y + z2.y));
      const float2 o = make_float2(0.5f * (z1.y - z2.y), -0.5f * (z1.x - z2.x));   // (z1 - z2) / (2i)
      const float2 wo = cmul(w, o);
      x[m] = make_float2(e.x + sg * wo.x, e.y + sg * wo.y);
    }
  }
}

// Zc[b] of transform tr = signal * n_ops + op (0 <= b < P): for the channels' real samples
// X_m[N - r] = conj X_m[r], so S(k) = sum_m X_m[k mod N] (T_k[m] + conj T_-k[m]) / 2 with T_k the
// apply-table column of position k; the plan folds that factor and the gather weight
// 1 + i w^k into D.
__device__ __forceinline__ float2 band_bin(const BandGen& g, int64_t tr, int b) {
  constexpr int MM = 4;   // channels the real-mode path takes (MCI_MAX_CHANNELS)
  const int64_t sig = tr / g.n_ops;
  const int op = (int)(tr - sig * g.n_ops);
  const float2* Zs = g.Z + sig * g.M * g.Lz;
  const int P = g.P, K = g.K, N = g.N;
  const float2* Dop = g.D + (int64_t)op * g.M * (2 * K + 1);
  float2 acc = make_float2(0.f, 0.f);
  if (g.one) {
    // k = b (b <= K) or b - P (b >= P - K); the bins between hold no band position.  |k| <= K
    // <= M N, so k mod N takes a few conditional steps instead of a division.
    const bool hi = b > K;
    if (hi && b < P - K) return acc;
    const int k = hi ? b - P : b;
    int r = k;
    while (r < 0) r += N;
    while (r >= N) r -= N;
    const float2* Dk = Dop + k + K;
    if (!g.half_rows || g.post) {
      float2 x[MM];
      chan_x<MM>(g, Zs, r, x);
#pragma unroll
      for (int m = 0; m < MM; ++m)
        if (m < g.M) acc = cadd(acc, cmul(x[m], Dk[(int64_t)m * (2 * K + 1)]));
      return acc;
    }
    // X_m = E + s w O with E = (z1 + conj z2) / 2, O = (z1 - conj z2) / (2i), s = +-1, is
    // z1 alpha + conj(z2) beta with alpha = (1 - i s w) / 2, beta = (1 + i s w) / 2, so the bin
    // is alpha sum_m z1_m D_m + beta sum_m conj(z2_m) D_m
    const int H = g.H;
    const int rh = r < H ? r : r - H;
    const int rr = rh == 0 ? 0 : H - rh;
    const float sg = r < H ? 0.5f : -0.5f;
    const float2 w = g.wN[rh];
    const float2 al = make_float2(0.5f + sg * w.y, -sg * w.x), be = make_float2(0.5f - sg * w.y, sg * w.x);
    float2 s1 = make_float2(0.f, 0.f), s2 = s1;
#pragma unroll
    for (int m = 0; m < MM; ++m)
      if (m < g.M) {
        const float2 d = Dk[(int64_t)m * (2 * K + 1)];
        const float2 z1 = Zs[m * g.Lz + rh], z2 = Zs[m * g.Lz + rr];
        s1 = make_float2(s1.x + z1.x * d.x - z1.y * d.y, s1.y + z1.x * d.y + z1.y * d.x);
        s2 = make_float2(s2.x + z2.x * d.x + z2.y * d.y, s2.y + z2.x * d.y - z2.y * d.x);   // conj(z2) d
      }
    return cadd(cmul(al, s1), cmul(be, s2));
  }
  for (int k = b - ((b + K) / P) * P; k <= K; k += P) {
    int r = k % N;
    if (r < 0) r += N;
    float2 x[MM];
    chan_x<MM>(g, Zs, r, x);
#pragma unroll
    for (int m = 0; m < MM; ++m)
      if (m < g.M) acc = cadd(acc, cmul(x[m], Dop[(int64_t)m * (2 * K + 1) + k + K]));
  }
  return acc;
}

}  // namespace mci
