// mci_fused.hip -- single-pass fused kernel for batched real-mode 1-D reconstruction.
//
// One 256-thread workgroup handles one signal and
// never leaves LDS between reading the M channel sample rows and writing the output row:
//
//  1. channel DFTs (Lemma 3.1): the real row g_m of length N = 2H is read as H complex
//     pairs z[p] = g[2p] + i g[2p+1]; Z = DFT_H(z) runs as a power-of-two Stockham FFT,
//     through Bluestein's chirp convolution when H is not a power of two (e.g. H = 683);
//     X_m[k] = E[k] + e^{-2 pi i k / N} O[k], k = 0..H, with E, O the DFTs of the even and
//     odd samples recovered from Z.  X_m[N - k] = conj X_m[k] covers the other half.
//  2. apply (eq. matrixeqn1): for residue n = n1 + i, a(n + jN) = sum_m X_m[n mod N]
//     Tab[m][j][i], Tab holding q_mj(n) o(n + jN) / N.  In real mode the output is
//     Re sum_k a(k) e^{ikt} = sum_k S(k) e^{ikt} with S(k) = (a(k) + conj a(-k)) / 2.  The
//     negatives of residue i's band positions all have residue i' = (-2 n1 - i) mod N,
//     so one thread solving the pair {i, i'} owns S(|k|) for all of them: no atomics.
//  3. output grid: with Q polyphase components, y[Q q + r] = sum_k S(k) w^{k r} e^{2 pi i k q / P}
//     (P = n_out / Q, w = e^{2 pi i / n_out}); the components are real, so components
//     r0 = 2c and r1 = 2c + 1 share one complex inverse FFT of length P:
//     Zc[b] = sum_{k = b mod P} S(k) (w^{k r0} + i w^{k r1}),  y[Qq + r0] + i y[Qq + r1] = IDFT(Zc)[q].
//     The last FFT pass leaves element q = tid + 256 c in thread tid, so the Q outputs
//     of q are written by one vector store and a wave writes 64 consecutive q.
//
// Split Bluestein (BLUE = 2): the chirp convolution has H inputs and only H outputs, so its
// outputs are taken in two halves of Ko = ceil(H / 2).  Half h needs the chirp kernel on
// n in [h Ko - H + 1, h Ko + Ko - 1], H + Ko - 1 values, and a circular convolution of that
// length computes it without wrap-around: with w_h[m] = b[h Ko - H + 1 + m],
// y[h Ko + k'] = (u (*) w_h)[k' + H - 1], k' < Ko.  One forward FFT of the chirped input
// serves both halves, so a length-PF transform triple (PF >= H + Ko - 1, e.g. 1024 for
// H = 683) replaces the pair of length >= 2H - 1 (2048) the full form needs.
//
// The FFTs are register-staged Stockham passes: every thread holds E = L / 256 elements,
// input slot c of a pass is element tid + 256 c for every radix, and so is output slot c
// of the last pass -- which lets the Bluestein forward FFT, the pointwise product and the
// inverse FFT run back to back in registers.
#include <algorithm>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <complex>
#include <vector>

#include "mci_device.h"
#include "mci_fused.h"
#include "mci_host_util.h"
#include "mci_jobs.h"

namespace mci {

constexpr int NT = 256;

struct FusedArgs {
  const void* g;
  void* y;
  const int64_t* offs;  // per-signal (input, output) element offsets, or null for a dense batch
  int64_t batch;
  int M, N, H, n1;
  int Nout, K;        // K = max |k| over the band
  int C, Ch, n_items; // residue pairing: i' = (C - i) mod N; canonical items
  int zero_s;         // 1 when some |k| <= K is in neither the band nor its negative
  int n1r;            // n1 mod N, in [0, N)
  int B0;             // (-2 n1 - C) / N: -(n1 + i + jN) = n1 + i' + (B - j) N, B = B0 for i <= C, else B0 - 1
  const float2* twF;  // PF entries e^{-2 pi i k / PF}
  const float2* chirp;  // H entries e^{-i pi k^2 / H} (Bluestein)
  const float2* bhat;   // full Bluestein: PF entries, DFT_PF of the conjugate chirp, / PF;
                        // split Bluestein: 2 PF entries, the two halves' kernel segments (see the kernel)
  const float2* wN;     // H + 1 entries e^{-2 pi i k / N}
  const float2* tab;    // [M][M][N]: q_mj(n1 + i) o(.) / N
  const float2* twI;    // P entries e^{-2 pi i k / P}
  const float2* U;      // [Q/2][2K + 1]: w^{k r0} + i w^{k r1} for k = -K..K, w = e^{2 pi i / Nout}
  const float2* Ub;     // [Q/2][P]: U at the main band position of b (b if b <= K, else b - P), 0 if none
};

// ---------------------------------------------------------------- register-staged FFT
// LDS index with one padding slot per 16 complex values: the stride-R writes of the first
// Stockham passes then spread over all banks.
__device__ __forceinline__ int pad(int x) { return x + (x >> 4); }

constexpr int padded(int n) { return n + (n >> 4) + 1; }
static_assert(NT % 16 == 0, "pad(tid + NT c) = pad(tid) + c (NT + NT / 16) needs NT % 16 == 0");

template <int R, int S>
__device__ __forceinline__ void dft_r(float2* u) {
  if constexpr (R == 2) dft2<S>(u[0], u[1]);
  else if constexpr (R == 3) dft3<S>(u[0], u[1], u[2]);
  else if constexpr (R == 4) dft4<S>(u[0], u[1], u[2], u[3]);
  else if constexpr (R == 8) dft8<S>(u);
  else if constexpr (R == 12) dft12<S>(u);
  else {
    static_assert(R == 16, "radix");
    // 16 = 4 x 4: DFT4 over each stride-4 group, twiddles e^{S 2 pi i q s / 16}, DFT4 across
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
template <int R0, int... Rs> struct RList<R0, Rs...> { static constexpr int first = R0; };

// Base twiddles of a pass, loaded before the exchange that precedes it so that the load
// overlaps the barrier waits (at most 2 butterflies per thread for the radices used here).
struct PassTw {
  float2 w1[3], w4[3];
};
template <int L, int NS, int R>
__device__ __forceinline__ PassTw load_pass_tw(const float2* __restrict__ tw) {
  constexpr int BPT = (L / NT) / R;
  static_assert(BPT <= 3, "prefetch holds three butterflies");
  PassTw p;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = threadIdx.x + NT * b;
    const int k1 = (j % NS) * (L / (NS * R));
    p.w1[b] = tw[k1];
    if constexpr (R >= 8) p.w4[b] = tw[4 * k1];
  }
  return p;
}

// T independent length-L transforms (buffer t at lds + t * padded(L)); one Stockham pass of
// radix R at stage size NS, then the remaining passes.  On entry v[t][c] holds element
// tid + NT c of transform t's pass input; after the last pass it holds element tid + NT c
// of the transform.  SX: the transforms share one buffer and exchange one after the other
// (the butterflies of all T still share their twiddles).  ptw: this pass's base twiddles
// (unused by the first pass, NS = 1).
template <int L, int S, int T, bool SX, int NS, int R, int... Rest>
__device__ __forceinline__ void fft_passes(float2* __restrict__ lds, float2 (&v)[T][L / NT],
                                           const float2* __restrict__ tw, RList<R, Rest...>, const PassTw& ptw) {
  constexpr int E = L / NT;
  constexpr int BPT = E / R;
  constexpr int LP = padded(L);
  static_assert(BPT * R == E, "radix must divide the elements per thread");
  const int tid = threadIdx.x;
  float2 u[T][BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int r = 0; r < R; ++r) u[t][b][r] = v[t][b + r * BPT];
    if constexpr (NS > 1) {
      // powers w^r of the butterfly's base twiddle, formed as they are used; w^1 and w^4 are
      // exact table entries, every other power is at most three roundings away from them
      float2 w1 = ptw.w1[b];
      if constexpr (S > 0) w1.y = -w1.y;
      float2 w4 = w1;
      if constexpr (R >= 8) {
        w4 = ptw.w4[b];
        if constexpr (S > 0) w4.y = -w4.y;
      }
      float2 wl[4];
      wl[1] = w1;
      if constexpr (R >= 3) wl[2] = cmul(w1, w1);
      if constexpr (R >= 4) wl[3] = cmul(wl[2], w1);
#pragma unroll
      for (int r = 1; r < (R < 4 ? R : 4); ++r)
#pragma unroll
        for (int t = 0; t < T; ++t) u[t][b][r] = cmul(u[t][b][r], wl[r]);
      if constexpr (R >= 8) {
        float2 wh = w4;    // w^{4a}
#pragma unroll
        for (int a4 = 1; a4 < R / 4; ++a4) {
          if (a4 > 1) wh = cmul(wh, w4);
#pragma unroll
          for (int t = 0; t < T; ++t) u[t][b][4 * a4] = cmul(u[t][b][4 * a4], wh);
#pragma unroll
          for (int r = 1; r < 4; ++r) {
            const float2 w = cmul(wh, wl[r]);
#pragma unroll
            for (int t = 0; t < T; ++t) u[t][b][4 * a4 + r] = cmul(u[t][b][4 * a4 + r], w);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) dft_r<R, S>(u[t][b]);
  }
  if constexpr (sizeof...(Rest) == 0) {
    static_assert(NS * R == L, "radices must multiply to L");
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int b = 0; b < BPT; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[t][b + r * BPT] = u[t][b][r];
  } else {
    // For power-of-two NS and R, base % 16 + (r NS) % 16 < 16, so
    // pad(base + r NS) = pad(base) + r NS + (r NS) / 16: one address per butterfly, the
    // rest are immediate offsets.  Likewise pad(tid + NT c) = pad(tid) + c (NT + NT / 16).
    const int pt = pad(tid);
    const PassTw ntw = load_pass_tw<L, NS * R, RList<Rest...>::first>(tw);
    if constexpr (SX) {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        __syncthreads();
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
          const int j = tid + NT * b;
          const int pb = pad((j / NS) * NS * R + (j % NS));
#pragma unroll
          for (int r = 0; r < R; ++r) lds[pb + r * NS + (r * NS) / 16] = u[t][b][r];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < E; ++c) v[t][c] = lds[pt + c * (NT + NT / 16)];
      }
    } else {
      __syncthreads();
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const int j = tid + NT * b;
        const int pb = pad((j / NS) * NS * R + (j % NS));
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int r = 0; r < R; ++r) lds[t * LP + pb + r * NS + (r * NS) / 16] = u[t][b][r];
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < E; ++c) v[t][c] = lds[t * LP + pt + c * (NT + NT / 16)];
    }
    fft_passes<L, S, T, SX, NS * R>(lds, v, tw, RList<Rest...>{}, ntw);
  }
}

template <int L> struct Radices;
template <> struct Radices<512> { using type = RList<2, 2, 2, 2, 2, 2, 2, 2, 2>; };   // 2 elements per thread
template <> struct Radices<1024> { using type = RList<4, 4, 4, 4, 4>; };
template <> struct Radices<2048> { using type = RList<8, 8, 8, 4>; };
template <> struct Radices<4096> { using type = RList<16, 16, 16>; };
// 12 elements per thread; the radix-12 (3 x 4 prime-factor) pass comes last, so every exchange
// is between power-of-two passes (the LDS padding's address arithmetic relies on that)
template <> struct Radices<3072> { using type = RList<4, 4, 4, 4, 12>; };
// 6 elements per thread: nine radix-2 passes, then radix 3
template <> struct Radices<1536> { using type = RList<2, 2, 2, 2, 2, 2, 2, 2, 2, 3>; };

template <int L, int S, int T>
__device__ __forceinline__ void fft(float2* lds, float2 (&v)[T][L / NT], const float2* tw) {
  fft_passes<L, S, T, false, 1>(lds, v, tw, typename Radices<L>::type{}, PassTw{});
}
// T transforms through one scratch buffer of padded(L) slots
template <int L, int S, int T>
__device__ __forceinline__ void fft_serial(float2* lds, float2 (&v)[T][L / NT], const float2* tw) {
  fft_passes<L, S, T, true, 1>(lds, v, tw, typename Radices<L>::type{}, PassTw{});
}

// ---------------------------------------------------------------- the fused kernel
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
// acc + a b as four fused multiply-adds
__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 b) {
  return make_float2(__builtin_fmaf(-a.y, b.y, __builtin_fmaf(a.x, b.x, acc.x)),
                     __builtin_fmaf(a.y, b.x, __builtin_fmaf(a.x, b.y, acc.y)));
}

// LDS use of one workgroup, in complex slots (see the layout in the kernel): the forward
// transforms' scratch, then the channel spectra (computed in place) and S, then the output
// transforms' scratch, each phase reusing the space from slot 0.  Every output transform's
// input is gathered from S before the first one runs, so S is dead by then.
__host__ __device__ constexpr int fused_slots(int PF, int P, int TI, int Q, int M, int H, int K) {
  const int fwd = M * padded(PF);
  const int mid = M * (H + 1) + (K + 1);
  const int inv = TI * padded(P);
  (void)Q;
  return fwd > mid ? (fwd > inv ? fwd : inv) : (mid > inv ? mid : inv);
}

// waves per SIMD the kernel is compiled for: 4 where its LDS can allow it (the split
// Bluestein and power-of-two forms at PF <= 1024 with up to 3 channels), else 3
constexpr int fused_waves(int PF, int M) { return PF <= 1024 && M <= 3 ? 4 : 3; }

// Storage access: two consecutive real samples as one complex value, and four consecutive
// outputs as one vector store (FP32, or FP16 with round-to-nearest conversion).  Samples are
// read once and outputs written once, so both use non-temporal (streaming) accesses, which
// leave L2 to the plan tables every workgroup reads.
typedef float f2_nt __attribute__((ext_vector_type(2)));
typedef float f4_nt __attribute__((ext_vector_type(4)));
typedef unsigned u2_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_pair(const float* r, int p) {
  const f2_nt v = __builtin_nontemporal_load((const f2_nt*)r + p);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_pair(const __half* r, int p) {
  const unsigned u = __builtin_nontemporal_load((const unsigned*)r + p);
  __half2 h;
  __builtin_memcpy(&h, &u, sizeof h);
  return __half22float2(h);
}
// odd N: sample p as a complex value with zero imaginary part
__device__ __forceinline__ float2 ld_real(const float* r, int p) {
  return make_float2(__builtin_nontemporal_load(r + p), 0.f);
}
__device__ __forceinline__ float2 ld_real(const __half* r, int p) {
  const unsigned short u = __builtin_nontemporal_load((const unsigned short*)r + p);
  __half h;
  __builtin_memcpy(&h, &u, sizeof h);
  return make_float2(__half2float(h), 0.f);
}
__device__ __forceinline__ void st_pair(float* y, int q, float2 v) { ((float2*)y)[q] = v; }
__device__ __forceinline__ void st_pair(__half* y, int q, float2 v) { ((__half2*)y)[q] = __float22half2_rn(v); }
__device__ __forceinline__ void st_quad(float* y, int q, float2 lo, float2 hi) {
  const f4_nt v = {lo.x, lo.y, hi.x, hi.y};
  __builtin_nontemporal_store(v, (f4_nt*)y + q);
}
__device__ __forceinline__ void st_quad(__half* y, int q, float2 lo, float2 hi) {
  const __half2 h[2] = {__float22half2_rn(lo), __float22half2_rn(hi)};
  u2_nt u;
  __builtin_memcpy(&u, h, sizeof u);
  __builtin_nontemporal_store(u, (u2_nt*)y + q);
}

// TI: how many of the Q/2 output transforms run side by side (1 or Q/2).  TS: storage type
// of the samples and outputs (float or __half); all arithmetic is FP32.
// BLUE_ 3 and 4: the forms 1 and 2 for odd N, whose channel DFT is the length-N transform of
// the real samples themselves (H = N, X = Z): no even/odd recovery
template <int PF, int BLUE_, int P, int Q, int M, int TI, typename TS>
__device__ __forceinline__ void fused_body(const FusedArgs& a, int64_t sig_index) {
  constexpr bool ODD = BLUE_ >= 3;
  constexpr int BLUE = ODD ? BLUE_ - 2 : BLUE_;
  extern __shared__ float2 sm[];
  constexpr int EF = PF / NT, EI = P / NT;
  const int tid = threadIdx.x;
  const int N = a.N, H = a.H, XH = a.H + 1;
  // layout, each phase from slot 0: forward scratch [M][padded(PF)] | half-length channel
  // spectra Zc [M][H+1] (X is formed from them in the apply), then S [K+1] | output scratch
  float2* F = sm;
  float2* Zc = sm;
  float2* Sv = sm + M * XH;
  float2* Z = sm;

  {
    // one signal per workgroup: a persistent loop would keep the loop invariants of every
    // phase live across the whole body and cut the occupancy
    const int64_t sig = sig_index;
    const TS* gs = (const TS*)a.g + (a.offs ? a.offs[2 * sig] : sig * (int64_t)M * N);
    // ---------------- 1. channel DFTs, all M channels side by side
    {
      float2 v[M][EF];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const TS* zin = gs + (int64_t)m * N;
#pragma unroll
        for (int c = 0; c < EF; ++c) {
          const int p = tid + NT * c;
          float2 z = make_float2(0.f, 0.f);
          if (p < H) z = ODD ? ld_real(zin, p) : ld_pair(zin, p);
          v[m][c] = z;
        }
      }
      if constexpr (BLUE) {
#pragma unroll
        for (int c = 0; c < EF; ++c) {
          const int p = tid + NT * c;
          if (p < H) {
            const float2 ch = a.chirp[p];
#pragma unroll
            for (int m = 0; m < M; ++m) v[m][c] = cmul(v[m][c], ch);
          }
        }
      }
      if constexpr (BLUE == 2) {
        // the split form has H + ceil(H / 2) - 1 <= PF, so H <= (2 PF + 2) / 3: the slots from
        // CZ on hold no sample, and the first pass may know it
        constexpr int CZ = ((2 * PF + 2) / 3 + NT - 1) / NT;
#pragma unroll
        for (int c = CZ; c < EF; ++c)
#pragma unroll
          for (int m = 0; m < M; ++m) v[m][c] = make_float2(0.f, 0.f);
      }
      // the split form's kernel spectra, loaded here so that the loads overlap the transform
      float2 bh[BLUE == 2 ? 2 : 1][EF];
      if constexpr (BLUE == 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int c = 0; c < EF; ++c) bh[h][c] = a.bhat[h * PF + tid + NT * c];
      }
      fft<PF, -1, M>(F, v, a.twF);
      if constexpr (BLUE == 2) {
        // two output halves from one forward transform; the first half's outputs wait in
        // registers until the second transform is done with the scratch
        const int Ko = (H + 1) / 2;
        float2 w0[M][EF], w[M][EF];
        float2 ch[2][EF];   // output chirp at k0 and k1 (clamped), loaded before the second transform
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int c = 0; c < EF; ++c)
#pragma unroll
            for (int m = 0; m < M; ++m) w[m][c] = cmul(v[m][c], bh[h][c]);
          if (h == 1) {
#pragma unroll
            for (int c = 0; c < EF; ++c) {
              const int e = tid + NT * c;
              ch[0][c] = a.chirp[min(max(e - (H - 1), 0), H - 1)];
              ch[1][c] = a.chirp[min(max(Ko + e - (H - 1), 0), H - 1)];
            }
          }
          fft<PF, +1, M>(F, w, a.twF);
          if (h == 0) {
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
              for (int c = 0; c < EF; ++c) w0[m][c] = w[m][c];
          }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < EF; ++c) {
          const int e = tid + NT * c;
          if (e >= H - 1) {
            const int k0 = e - (H - 1), k1 = Ko + e - (H - 1);
            if (k0 < Ko) {
#pragma unroll
              for (int m = 0; m < M; ++m) Zc[m * XH + k0] = cmul(w0[m][c], ch[0][c]);
            }
            if (k1 < H) {
#pragma unroll
              for (int m = 0; m < M; ++m) Zc[m * XH + k1] = cmul(w[m][c], ch[1][c]);
            }
          }
        }
      } else if constexpr (BLUE == 1) {
#pragma unroll
        for (int c = 0; c < EF; ++c) {
          const float2 bh = a.bhat[tid + NT * c];
#pragma unroll
          for (int m = 0; m < M; ++m) v[m][c] = cmul(v[m][c], bh);
        }
        fft<PF, +1, M>(F, v, a.twF);
#pragma unroll
        for (int c = 0; c < EF; ++c) {
          const int k = tid + NT * c;
          if (k < H) {
            const float2 ch = a.chirp[k];
#pragma unroll
            for (int m = 0; m < M; ++m) v[m][c] = cmul(v[m][c], ch);
          }
        }
      }
      if constexpr (BLUE != 2) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
          for (int c = 0; c < EF; ++c) {
            const int k = tid + NT * c;
            if (k < H) Zc[m * XH + k] = v[m][c];
          }
      }
    }
    __syncthreads();
    if (a.zero_s)
      for (int k = tid; k <= a.K; k += NT) Sv[k] = make_float2(0.f, 0.f);
    __syncthreads();   // S zeroed before the apply writes it
    // the apply table [M][M][N] as a buffer: every load takes one per-residue VGPR offset
    const __amdgpu_buffer_rsrc_t trs =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.tab, (short)0, M * M * N * 8, kRawBufferWord3);
    // ---------------- 2. apply, residue pairs -> S
    for (int it = tid; it < a.n_items; it += NT) {
      const int i = it <= a.Ch ? it : a.C + 1 + (it - a.Ch - 1);
      const int ip = i <= a.C ? a.C - i : a.C - i + N;
      // X_m at residue r = (n1 + i) mod N, formed here from the half-length spectrum:
      // X[k] = E[k] + w_N^k O[k] for k = min(r, N - r) <= H, conjugated when r > H.  Residue
      // i' has r' = (N - r) mod N, so its value is the conjugate (the channels are real).
      int r = a.n1r + i;                        // (n1 + i) mod N, 0 <= i < N
      if (r >= N) r -= N;
      // d = 2 X_m (the halves of E and O are folded into the final scale of S)
      float2 d[M];
      if constexpr (ODD) {
        // odd N: the spectrum holds every residue
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const float2 x = Zc[m * XH + r];
          d[m] = make_float2(2.f * x.x, 2.f * x.y);
        }
      } else {
        const bool lo = r <= H;
        const int k = lo ? r : N - r;
        const int k1 = k == H ? 0 : k, k2 = k == 0 ? 0 : H - k;
        const float2 wn = a.wN[k];
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const float2 z1 = Zc[m * XH + k1];
          const float2 z2 = conjf2(Zc[m * XH + k2]);
          const float2 e = make_float2(z1.x + z2.x, z1.y + z2.y);
          const float2 o = make_float2(z1.y - z2.y, z2.x - z1.x);   // (z1 - z2) / i
          const float2 x = cadd(e, cmul(wn, o));
          d[m] = lo ? x : conjf2(x);
        }
      }
      // table entries Tab[m][j][.] at residues i and i': one byte offset per residue, the
      // row offsets (m M + j) N are uniform
      const int o0 = i * 8, o1 = ip * 8;
      auto tab = [&](int m, int j, int off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(trs, off, (m * M + j) * N * 8, 0);
        float2 t;
        __builtin_memcpy(&t, &v, sizeof t);
        return t;
      };
      const int B = i <= a.C ? a.B0 : a.B0 - 1;
      if (B == M - 1) {
        // every band position of residue i has its negative at residue i': position j pairs
        // with position M - 1 - j, and S(|k|) = (a(k) + conj a(-k)) / 2 (conjugated for k < 0)
#pragma unroll
        for (int j = 0; j < M; ++j) {
          float2 s0 = cmul(d[0], tab(0, j, o0)), s1 = cmul(conjf2(d[0]), tab(0, M - 1 - j, o1));
#pragma unroll
          for (int m = 1; m < M; ++m) {
            s0 = cmac(s0, d[m], tab(m, j, o0));
            s1 = cmac(s1, conjf2(d[m]), tab(m, M - 1 - j, o1));
          }
          const float2 sv = make_float2(0.25f * (s0.x + s1.x), 0.25f * (s0.y - s1.y));
          const int k = a.n1 + i + j * N;
          if (k >= 0) Sv[k] = sv;
          else Sv[-k] = conjf2(sv);
        }
        continue;
      }
      float2 av[2][M];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int oo = q ? o1 : o0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          float2 acc = cmul(q ? conjf2(d[0]) : d[0], tab(0, j, oo));
#pragma unroll
          for (int m = 1; m < M; ++m) acc = cmac(acc, q ? conjf2(d[m]) : d[m], tab(m, j, oo));
          av[q][j] = acc;
        }
      }
      const bool single = ip == i;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (q == 1 && single) break;
        const int ii = q ? ip : i, io = q ? i : ip;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const int k = a.n1 + ii + j * N;
          const int num = -k - a.n1 - io;        // partner -k = n1 + io + jp N
          float2 pv = make_float2(0.f, 0.f);
          bool has = false;
#pragma unroll
          for (int jp = 0; jp < M; ++jp)
            if (num == jp * N) { has = true; pv = av[q ^ (single ? 0 : 1)][jp]; }
          const float2 val = av[q][j];
          if (k >= 0) Sv[k] = make_float2(0.25f * (val.x + pv.x), 0.25f * (val.y - pv.y));
          else if (!has) Sv[-k] = make_float2(0.25f * val.x, -0.25f * val.y);
        }
      }
    }
    __syncthreads();
    // ---------------- 3. output grid: Q/2 complex inverse FFTs of length P, TI at a time
    TS* ys = (TS*)a.y + (a.offs ? a.offs[2 * sig + 1] : sig * (int64_t)a.Nout);
    float2 keep[(Q / 2 - TI > 0 ? Q / 2 - TI : 1)][EI];   // earlier transforms' outputs
    // every transform's input is gathered from S first: the scratch then reuses S's space.
    // Zc[b] sums S~(k) U(k) over the band positions k = b and k = b - P (K < P), where S~(k) is
    // S(k) for k >= 0 and conj S(-k) for k < 0.  The main position is b when b <= K, else
    // b - P; its multiplier comes from a per-b table that is zero where neither position is
    // in the band.  Both are in the band only on [P - K, K], where the second term is added.
    const __amdgpu_buffer_rsrc_t urs =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.Ub, (short)0, (Q / 2) * P * 8, kRawBufferWord3);
    float2 vin[Q / 2][EI];
    // in groups of GW elements: the second term's branch after each group bounds how many of
    // the table loads the compiler hoists (registers)
    constexpr int GW = EI < 4 ? EI : 4;
#pragma unroll
    for (int c0 = 0; c0 < EI; c0 += GW) {
#pragma unroll
      for (int c = c0; c < c0 + GW; ++c) {
        const int b = tid + NT * c;
        const bool lo = b <= a.K;
        const int kk = min(lo ? b : P - b, a.K);   // clamped where the multiplier is zero
        float2 sv = Sv[kk];
        if (!lo) sv.y = -sv.y;
#pragma unroll
        for (int pc = 0; pc < Q / 2; ++pc) {
          const auto u = __builtin_amdgcn_raw_buffer_load_b64(urs, tid * 8, (pc * P + NT * c) * 8, 0);
          float2 uf;
          __builtin_memcpy(&uf, &u, sizeof uf);
          vin[pc][c] = cmul(sv, uf);
        }
      }
#pragma unroll
      for (int c = c0; c < c0 + GW; ++c) {
        const int b = tid + NT * c;
        if (NT * c + NT - 1 >= P - a.K && NT * c <= a.K) {   // this block meets [P - K, K]
          if (b >= P - a.K && b <= a.K) {
            const float2 s2 = conjf2(Sv[P - b]);
#pragma unroll
            for (int pc = 0; pc < Q / 2; ++pc)
              vin[pc][c] = cadd(vin[pc][c], cmul(s2, a.U[(int64_t)pc * (2 * a.K + 1) + a.K + (b - P)]));
          }
        }
      }
    }
    if constexpr (TI == 1 && Q == 4) {
      // both transforms' butterflies together (one twiddle formation), exchanges in turn
      // through the one scratch buffer
      fft_serial<P, +1, 2>(Z, vin, a.twI);
#pragma unroll
      for (int c = 0; c < EI; ++c) st_quad(ys, tid + NT * c, vin[0][c], vin[1][c]);
      __syncthreads();
      return;
    }
#pragma unroll
    for (int pc0 = 0; pc0 < Q / 2; pc0 += TI) {
      float2 v[TI][EI];
#pragma unroll
      for (int t = 0; t < TI; ++t)
#pragma unroll
        for (int c = 0; c < EI; ++c) v[t][c] = vin[pc0 + t][c];
      fft<P, +1, TI>(Z, v, a.twI);
      if (pc0 + TI < Q / 2) {
#pragma unroll
        for (int t = 0; t < TI; ++t)
#pragma unroll
          for (int c = 0; c < EI; ++c) keep[pc0 + t][c] = v[t][c];
        continue;
      }
      // all Q outputs of element q are in this thread: one vector store per q
#pragma unroll
      for (int c = 0; c < EI; ++c) {
        const int q = tid + NT * c;
        if constexpr (Q == 4) {
          const float2 lo = TI == 2 ? v[0][c] : keep[0][c];
          const float2 hi = TI == 2 ? v[TI - 1][c] : v[0][c];
          st_quad(ys, q, lo, hi);
        } else {
          st_pair(ys, q, v[0][c]);
        }
      }
    }
    __syncthreads();
  }
}

template <int PF, int BLUE, int P, int Q, int M, int TI, typename TS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(fused_waves(PF, M))))
void k_mci1d_fused(FusedArgs a) {
  fused_body<PF, BLUE, P, Q, M, TI, TS>(a, blockIdx.x);
}

// merged form: one persistent launch over the jobs of an uneven batch (one signal per
// virtual workgroup, as above)
template <int PF, int BLUE, int P, int Q, int M, int TI, typename TS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(fused_waves(PF, M))))
void k_mci1d_fused_jobs(const FusedArgs* jobs, const JobGrid* grids, const int64_t* first, int n_jobs, int64_t total,
                        JobBases b) {
  run_jobs(jobs, grids, first, n_jobs, total, [&](const FusedArgs& j, int64_t bx, int, int) {
    FusedArgs a = j;
    a.g = rebase(a.g, b);
    a.y = rebase(a.y, b);
    fused_body<PF, BLUE, P, Q, M, TI, TS>(a, bx);
  });
}

// ---------------------------------------------------------------- host side
struct FusedTables {
  float2 *twF, *chirp, *bhat, *wN, *twI, *wout;
};

template <int PF, int BLUE, int P, int Q, int M, int TI, typename TS>
static hipError_t launch_jobs(const MergedLaunch& m, const JobBases& b, hipStream_t s) {
  return merged_launch<FusedArgs>((const void*)k_mci1d_fused_jobs<PF, BLUE, P, Q, M, TI, TS>, NT, m, b, s);
}
template <int PF, int BLUE, int P, int Q, int M, int TI, typename TS>
static int occupancy_jobs(size_t lds) {
  return occupancy_of((const void*)k_mci1d_fused_jobs<PF, BLUE, P, Q, M, TI, TS>, NT, lds);
}

template <int PF, int BLUE, int P, int Q, int M, int TI, typename TS>
static hipError_t launch_mt(const FusedPlan& fp, const void* g, void* y, int64_t batch, const int64_t* offs,
                            hipStream_t s) {
  FusedArgs a = *(const FusedArgs*)fp.args;
  a.g = g;
  a.y = y;
  a.offs = offs;
  a.batch = batch;
  const size_t lds = (size_t)fp.lds_bytes;
  const int64_t grid = batch;   // one signal per workgroup
  if (job_recorder()) {
    record_job(launch_jobs<PF, BLUE, P, Q, M, TI, TS>, occupancy_jobs<PF, BLUE, P, Q, M, TI, TS>, a, grid, 1, lds);
    return hipSuccess;
  }
  hipLaunchKernelGGL((k_mci1d_fused<PF, BLUE, P, Q, M, TI, TS>), dim3((unsigned)grid), dim3(NT), lds, s, a);
  return hipGetLastError();
}

// Raise the kernels' dynamic LDS limit once, at plan time (not while a launch may be captured).
template <int PF, int BLUE, int P, int Q, int M, typename TS>
static hipError_t prep_m(const int* lds_ti) {
  if (lds_ti[0] > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_mci1d_fused<PF, BLUE, P, Q, M, 1, TS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_ti[0]);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_mci1d_fused_jobs<PF, BLUE, P, Q, M, 1, TS>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_ti[0]);
    if (e != hipSuccess) return e;
  }
  if constexpr (Q < 4) return hipSuccess;   // one output transform: no side-by-side form
  else if (lds_ti[1] > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_mci1d_fused<PF, BLUE, P, Q, M, 2, TS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_ti[1]);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_mci1d_fused_jobs<PF, BLUE, P, Q, M, 2, TS>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds_ti[1]);
  }
  return hipSuccess;
}

template <int PF, int BLUE, int P, int Q>
static hipError_t prep_t(int M, int store, const int* lds_ti) {
  const bool h = store == ST_F16;
  switch (M) {
    case 1: return h ? prep_m<PF, BLUE, P, Q, 1, __half>(lds_ti) : prep_m<PF, BLUE, P, Q, 1, float>(lds_ti);
    case 2: return h ? prep_m<PF, BLUE, P, Q, 2, __half>(lds_ti) : prep_m<PF, BLUE, P, Q, 2, float>(lds_ti);
    case 3: return h ? prep_m<PF, BLUE, P, Q, 3, __half>(lds_ti) : prep_m<PF, BLUE, P, Q, 3, float>(lds_ti);
    default: return h ? prep_m<PF, BLUE, P, Q, 4, __half>(lds_ti) : prep_m<PF, BLUE, P, Q, 4, float>(lds_ti);
  }
}

template <int PF, int BLUE, int P, int Q, int M>
static hipError_t launch_m(const FusedPlan& fp, const void* g, void* y, int64_t batch, const int64_t* offs,
                           hipStream_t s) {
  if constexpr (Q >= 4) {
    if (fp.ti == 2) {
      if (fp.store == ST_F16) return launch_mt<PF, BLUE, P, Q, M, 2, __half>(fp, g, y, batch, offs, s);
      return launch_mt<PF, BLUE, P, Q, M, 2, float>(fp, g, y, batch, offs, s);
    }
  }
  if (fp.store == ST_F16) return launch_mt<PF, BLUE, P, Q, M, 1, __half>(fp, g, y, batch, offs, s);
  return launch_mt<PF, BLUE, P, Q, M, 1, float>(fp, g, y, batch, offs, s);
}

template <int PF, int BLUE, int P, int Q>
static hipError_t launch_t(const FusedPlan& fp, const void* g, void* y, int64_t batch, const int64_t* offs,
                           hipStream_t s) {
  switch (((const FusedArgs*)fp.args)->M) {
    case 1: return launch_m<PF, BLUE, P, Q, 1>(fp, g, y, batch, offs, s);
    case 2: return launch_m<PF, BLUE, P, Q, 2>(fp, g, y, batch, offs, s);
    case 3: return launch_m<PF, BLUE, P, Q, 3>(fp, g, y, batch, offs, s);
    default: return launch_m<PF, BLUE, P, Q, 4>(fp, g, y, batch, offs, s);
  }
}

using LaunchFn = hipError_t (*)(const FusedPlan&, const void*, void*, int64_t, const int64_t*, hipStream_t);

using PrepFn = hipError_t (*)(int, int, const int*);

struct Variant {
  int PF;
  int blue;   // 0: power-of-two H = PF; 1: Bluestein, PF >= 2H - 1; 2: split Bluestein, PF >= H + ceil(H/2) - 1;
              // 3, 4: forms 1 and 2 for odd N (H = N, the real samples as a length-N complex sequence)
  int P, Q;
  LaunchFn fn;
  PrepFn prep;
};

#define MCI_FV(PF, B, P, Q) {PF, B, P, Q, launch_t<PF, B, P, Q>, prep_t<PF, B, P, Q>}
// at equal PF the first listed wins: the full Bluestein form (two transforms) before the
// split form (three)
static const Variant kVariants[] = {
    MCI_FV(2048, 1, 4096, 4), MCI_FV(1024, 1, 4096, 4), MCI_FV(1024, 0, 4096, 4),
    MCI_FV(2048, 0, 4096, 4), MCI_FV(2048, 1, 2048, 4), MCI_FV(1024, 0, 1024, 4),
    MCI_FV(2048, 0, 2048, 4), MCI_FV(1024, 2, 4096, 4),
    // 512-point channel transforms (two elements per thread, radix-2 passes): H = 512 with
    // 8192- and 16384-point outputs, Bluestein for H <= 256 with 4096-point outputs
    MCI_FV(512, 0, 4096, 4), MCI_FV(512, 0, 2048, 4), MCI_FV(512, 1, 1024, 4),
    // 12288-point outputs (P = 3072 = 4^4 x 12)
    MCI_FV(512, 0, 3072, 4), MCI_FV(1024, 1, 3072, 4), MCI_FV(2048, 1, 3072, 4),
    // Bluestein at 512 for H <= 256 (power-of-two H included) with 8192-point outputs, and one
    // output transform (Q = 2: y[2q] + i y[2q + 1]) for 2048- and 6144-point outputs
    MCI_FV(512, 1, 2048, 4), MCI_FV(512, 1, 1024, 2), MCI_FV(512, 1, 3072, 2), MCI_FV(1024, 1, 3072, 2),
    // 1024- and 3072-point outputs as one transform of 512 or 1536 points
    MCI_FV(512, 1, 512, 2), MCI_FV(512, 1, 1536, 2),
    // odd N: Bluestein at 512 for N <= 256 with 2048-point outputs, split Bluestein at 1024 for
    // 512 < N <= 683 with 8192- and 16384-point outputs
    MCI_FV(512, 3, 1024, 2), MCI_FV(512, 3, 2048, 4), MCI_FV(1024, 4, 2048, 4), MCI_FV(1024, 4, 4096, 4),
};
#undef MCI_FV


mci_status fused_select(const mci_plan_desc& d, int prec, int store, const void* tab, FusedPlan& fp) {
  fp.kind = 0;
  if (prec != MCI_F32 || (store != ST_F32 && store != ST_F16) || !d.real_io || d.n_ops != 1 || d.M > MCI_MAX_CHANNELS) return MCI_OK;
  if (std::getenv("MCI_DISABLE_FUSED")) return MCI_OK;
  const int64_t N = d.N, M = d.M, n1 = d.n1, mu = M * N;
  if (N < 4 || N > (1 << 15) || d.n_out > (1 << 20)) return MCI_OK;
  // even N: the channel DFT through the half-length transform of sample pairs; odd N: the
  // length-N transform of the real samples (Bluestein forms 3 and 4 only)
  const bool odd = N % 2 != 0;
  const int64_t H = odd ? N : N / 2;
  const int64_t K = std::max<int64_t>(std::llabs(n1), std::llabs(n1 + mu - 1));
  const Variant* pick = nullptr;
  for (const Variant& v : kVariants) {
    // (a power-of-two H also takes Bluestein where no plain form fits: the smallest PF wins,
    // and the plain form, PF = H, is always smaller than a chirp convolution's)
    if ((v.blue >= 3) != odd) continue;
    const int bl = v.blue >= 3 ? v.blue - 2 : v.blue;
    const bool fwd_ok = bl == 0 ? H == v.PF
                : bl == 1 ? 2 * H - 1 <= v.PF
                          : H + (H + 1) / 2 - 1 <= v.PF;
    if (!fwd_ok || (int64_t)v.P * v.Q != d.n_out) continue;
    if (!pick || v.PF < pick->PF) pick = &v;
  }
  if (!pick || K >= pick->P) return MCI_OK;
  int max_lds = 64 * 1024;
  {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0) max_lds = v;
  }
  // LDS of the two output-transform groupings: one transform at a time (TI = 1), or all Q/2
  // side by side (TI = 2), which needs more LDS and registers but one FFT pass sequence less
  int64_t lds_ti[2];
  for (int t = 0; t < 2; ++t)
    lds_ti[t] = (int64_t)fused_slots(pick->PF, pick->P, t + 1, pick->Q, (int)M, (int)H, (int)K) * (int64_t)sizeof(float2);
  if (lds_ti[0] > max_lds) return MCI_OK;
  const int n_ti = pick->Q >= 4 && lds_ti[1] <= max_lds ? 2 : 1;
  {
    const int lt[2] = {(int)lds_ti[0], n_ti == 2 ? (int)lds_ti[1] : 0};
    if (pick->prep((int)M, store, lt) != hipSuccess) return MCI_OK;   // no fused kernel then
  }
  const int ti = 1;
  const int64_t lds = lds_ti[0];

  // tables (FP64 on the host, stored FP32)
  const int PF = pick->PF, P = pick->P;
  const int Q = pick->Q;
  const int blue = pick->blue >= 3 ? pick->blue - 2 : pick->blue;   // the Bluestein form, odd N or not
  std::vector<std::complex<double>> twF(PF), chirp(H), bhat((size_t)(blue == 2 ? 2 : 1) * PF, 0.0), wN(H + 1),
      twI(P), U((size_t)(Q / 2) * (2 * K + 1)), Ub((size_t)(Q / 2) * P, 0.0);
  for (int k = 0; k < PF; ++k) twF[k] = root_of_unity(k, PF);
  for (int64_t k = 0; k <= H; ++k) wN[k] = root_of_unity(k, N);
  for (int k = 0; k < P; ++k) twI[k] = root_of_unity(k, P);
  // U[pc][k + K] = w^{k r0} + i w^{k r1}, r0 = 2 pc, r1 = 2 pc + 1, w = e^{2 pi i / n_out}
  for (int pc = 0; pc < Q / 2; ++pc)
    for (int64_t k = -K; k <= K; ++k) {
      const std::complex<double> w0 = std::conj(root_of_unity(k * (2 * pc), d.n_out));
      const std::complex<double> w1 = std::conj(root_of_unity(k * (2 * pc + 1), d.n_out));
      U[(size_t)pc * (2 * K + 1) + (k + K)] = w0 + std::complex<double>(0.0, 1.0) * w1;
    }
  // Ub[pc][b] = U at b's main band position: b if b <= K, else b - P if b >= P - K
  for (int pc = 0; pc < Q / 2; ++pc)
    for (int64_t b = 0; b < P; ++b) {
      const int64_t k = b <= K ? b : (b >= P - K ? b - P : INT64_MIN);
      if (k != INT64_MIN) Ub[(size_t)pc * P + b] = U[(size_t)pc * (2 * K + 1) + (k + K)];
    }
  if (blue) {
    for (int64_t k = 0; k < H; ++k) chirp[k] = chirp_value(k, H, -1);
    std::vector<int> rad;
    for (int64_t r = PF; r > 1; r /= 8) rad.push_back(r >= 8 ? 8 : (int)r);
    if (blue == 1) {
      // the kernel b[n] = conj c[|n|], |n| < H, placed circularly
      for (int64_t m = 0; m < H; ++m) {
        bhat[m] = std::conj(chirp[m]);
        if (m) bhat[PF - m] = std::conj(chirp[m]);
      }
      host_fft(bhat, rad, -1);
    } else {
      // half h: w_h[m] = b[h Ko - H + 1 + m], m < H + Ko - 1 (<= PF), zero beyond
      const int64_t Ko = (H + 1) / 2;
      for (int h = 0; h < 2; ++h) {
        std::vector<std::complex<double>> wh(PF, 0.0);
        for (int64_t m = 0; m < H + Ko - 1; ++m) wh[m] = std::conj(chirp_value(h * Ko - H + 1 + m, H, -1));
        host_fft(wh, rad, -1);
        for (int m = 0; m < PF; ++m) bhat[(size_t)h * PF + m] = wh[m];
      }
    }
    for (auto& x : bhat) x /= (double)PF;
  }
  const size_t n_all = twF.size() + chirp.size() + bhat.size() + wN.size() + twI.size() + U.size() + Ub.size();
  std::vector<float2> h(n_all);
  size_t o = 0;
  auto put = [&](const std::vector<std::complex<double>>& v) {
    const size_t at = o;
    for (auto& x : v) h[o++] = make_float2((float)x.real(), (float)x.imag());
    return at;
  };
  const size_t o_twF = put(twF), o_chirp = put(chirp), o_bhat = put(bhat), o_wN = put(wN), o_twI = put(twI),
               o_U = put(U), o_Ub = put(Ub);
  float2* dt = nullptr;
  if (hipMalloc(&dt, n_all * sizeof(float2)) != hipSuccess) return MCI_E_OUT_OF_MEMORY;
  if (hipMemcpy(dt, h.data(), n_all * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dt);
    return MCI_E_DEVICE;
  }
  FusedArgs* a = new FusedArgs();
  a->M = (int)M; a->N = (int)N; a->H = (int)H; a->n1 = (int)n1;
  a->Nout = (int)d.n_out; a->K = (int)K;
  a->C = (int)((((-2 * n1) % N) + N) % N);
  a->Ch = a->C / 2;
  // S(k), 0 <= k <= K, is written by the apply iff k or -k lies in [n1, n1 + mu)
  a->zero_s = (n1 > 0 || n1 + mu - 1 < 0) ? 1 : 0;
  a->n_items = a->Ch + 1 + (int)((a->C + N) / 2 - a->C);
  a->n1r = (int)(((n1 % N) + N) % N);
  a->B0 = (int)((-2 * n1 - a->C) / N);
  a->twF = dt + o_twF; a->chirp = dt + o_chirp; a->bhat = dt + o_bhat; a->wN = dt + o_wN;
  a->tab = (const float2*)tab; a->twI = dt + o_twI; a->U = dt + o_U; a->Ub = dt + o_Ub;
  fp.tables = dt;
  fp.args = a;
  fp.lds_bytes = (int)lds;
  fp.ti = ti;
  fp.n_ti = n_ti;
  fp.lds_ti[0] = (int)lds_ti[0];
  fp.lds_ti[1] = (int)lds_ti[1];
  fp.store = store;
  fp.launch = (void*)pick->fn;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int per_cu = std::max<int>(1, (int)((160 * 1024) / std::max<int64_t>(lds, 1)));
  fp.grid_cap = std::max(1, cus) * std::min(per_cu, 8);
  std::snprintf(fp.name, sizeof fp.name, "k_mci1d_fused: forward %s %d-point, output %d x %d-point, M=%d",
                blue == 2 ? "split-Bluestein" : blue == 1 ? "Bluestein" : "direct", PF, Q / 2, P, (int)M);
  if (odd) std::snprintf(fp.name + std::strlen(fp.name), sizeof fp.name - std::strlen(fp.name), ", odd N");
  fp.kind = 1;
  return MCI_OK;
}

void fused_release(FusedPlan& fp) {
  if (fp.tables) (void)hipFree(fp.tables);
  delete (FusedArgs*)fp.args;
  fp.tables = nullptr;
  fp.args = nullptr;
  fp.kind = 0;
}

void fused_set_ti(FusedPlan& fp, int ti) {
  fp.ti = (ti == 2 && fp.n_ti == 2) ? 2 : 1;
  fp.lds_bytes = fp.lds_ti[fp.ti - 1];
}

hipError_t fused_run(const FusedPlan& fp, const void* g, void* y, int64_t batch, const int64_t* offs,
                     hipStream_t s) {
  return ((LaunchFn)fp.launch)(fp, g, y, batch, offs, s);
}

}  // namespace mci
