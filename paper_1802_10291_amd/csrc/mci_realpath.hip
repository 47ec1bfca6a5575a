// mci_realpath.hip -- real-mode 1-D reconstruction in a few LDS-pass kernels, for lengths no
// single workgroup holds.  The steps are those of the single-pass kernel, each a pass over HBM:
//
//  1. channel DFTs (Lemma 3.1): row m of the real samples, read as H = N/2 complex pairs
//     z[p] = g[2p] + i g[2p+1] (odd N: as N real values), goes through a one- or two-pass
//     transform of length H (N) (through Bluestein's chirp convolution when that length does
//     not factor: the chirp is applied as the first pass loads, the filter spectrum as the
//     second one stores);
//  2. apply (eq. matrixeqn1) and the real part: X_m[r] = E[r'] + e^{-2 pi i r / N} O[r'],
//     r' = r mod H, with E, O the even/odd-sample DFTs recovered from Z (odd N: X_m = Z);
//     a(k) = sum_m
//     X_m[k mod N] Tab[m][j][i] for k = n1 + i + jN; S(k) = (a(k) + conj a(-k)) / 2;
//  3. output: with P = n_out / 2 and w = e^{2 pi i / n_out}, the two polyphase components
//     y[2q] and y[2q + 1] are the real and imaginary parts of
//       z[q] = sum_b Zc[b] e^{2 pi i b q / P},  Zc[b] = sum_{k = b mod P} S(k) (1 + i w^k),
//     so one complex inverse transform of length P yields the whole real output, and its
//     complex result, stored as it is, is the output row.
// A thread of step 2 owns the bins b and P - b, which receive S(k) and S(-k) = conj S(k).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mci_device.h"
#include "mci_fftlines.h"
#include "mci_realpath.h"

namespace mci {

__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

// a(k) of signal Zs for output op `op`; zero outside the band.  32-bit indices (the plan
// keeps M N and P + K below 2^30): k = n1 + j N + i, and k mod N = (n1 mod N + i) mod N.
__device__ __forceinline__ float2 band_coeff(int k, const float2* __restrict__ Zs, int64_t Lz,
                                             const float2* __restrict__ post, const float2* __restrict__ wN,
                                             const float2* __restrict__ tab, int op, int M, int N, int H,
                                             int n1, int n1r, bool half) {
  const int d = k - n1;
  float2 acc = make_float2(0.f, 0.f);
  if (d < 0 || d >= M * N) return acc;
  int j = 0, i = d;
  while (i >= N) {   // at most M - 1 steps
    i -= N;
    ++j;
  }
  int r = n1r + i;
  if (r >= N) r -= N;
  const float2* tb = tab + ((int64_t)(op * M) * M + j) * N + i;   // Tab[op][m][j][i] at tb[m M N]
  if (!half) {   // X_m[r] is the transform itself
    for (int m = 0; m < M; ++m) {
      float2 x = Zs[m * Lz + r];
      if (post) x = cmul(x, post[r]);
      acc = cadd(acc, cmul(x, tb[(int64_t)m * M * N]));
    }
    return acc;
  }
  const int rh = r < H ? r : r - H;
  const int rr = rh == 0 ? 0 : H - rh;
  const float sg = r < H ? 1.f : -1.f;
  const float2 w = wN[rh];
  for (int m = 0; m < M; ++m) {
    float2 z1 = Zs[m * Lz + rh], z2 = Zs[m * Lz + rr];
    if (post) {
      z1 = cmul(z1, post[rh]);
      z2 = cmul(z2, post[rr]);
    }
    z2 = conj2(z2);
    const float2 e = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y + z2.y));
    const float2 o = make_float2(0.5f * (z1.y - z2.y), -0.5f * (z1.x - z2.x));   // (z1 - z2) / (2i)
    const float2 wo = cmul(w, o);
    const float2 x = make_float2(e.x + sg * wo.x, e.y + sg * wo.y);
    acc = cadd(acc, cmul(x, tb[(int64_t)m * M * N]));
  }
  return acc;
}

// One thread per bin pair {b, P - b} (blockIdx.x), looping over a slice of the signals
// (blockIdx.y): the band positions k = b mod P and their residues are the same for every
// signal, so only the signal's own values are loaded per iteration.
__global__ void k_apply_real(const float2* __restrict__ Z, int64_t Lz, const float2* __restrict__ post,
                             const float2* __restrict__ wN, const float2* __restrict__ tab,
                             const float2* __restrict__ Wo, float2* __restrict__ Zc, int M, int n_ops, int N,
                             int H, int n1, int n1r, int K, int P, int64_t batch, int half_rows) {
  const int half = P / 2 + 1;   // bin pairs {b, P - b}, b = 0 .. P/2
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= half) return;
  const bool self = b == 0 || 2 * b == P;
  const int k0 = b - ((b + K) / P) * P;   // the first k = b mod P with k >= -K
  for (int64_t sig = blockIdx.y; sig < batch; sig += gridDim.y) {
    const float2* Zs = Z + sig * M * Lz;
    for (int op = 0; op < n_ops; ++op) {
      float2 acc_b = make_float2(0.f, 0.f), acc_m = make_float2(0.f, 0.f);
      for (int k = k0; k <= K; k += P) {
        const float2 ak = band_coeff(k, Zs, Lz, post, wN, tab, op, M, N, H, n1, n1r, half_rows);
        const float2 amk = conj2(band_coeff(-k, Zs, Lz, post, wN, tab, op, M, N, H, n1, n1r, half_rows));
        const float2 S = make_float2(0.5f * (ak.x + amk.x), 0.5f * (ak.y + amk.y));
        acc_b = cadd(acc_b, cmul(S, Wo[k + K]));
        if (!self) acc_m = cadd(acc_m, cmul(conj2(S), Wo[K - k]));
      }
      const int64_t bo = sig * n_ops + op;
      Zc[bo * P + b] = acc_b;
      if (!self) Zc[bo * P + (P - b)] = acc_m;
    }
  }
}

static size_t al(size_t n) { return (n + 255) & ~(size_t)255; }

size_t real_path_workspace(const RealPath& r, int64_t batch) {
  if (batch <= 0) return 0;
  const size_t nz = (size_t)batch * r.M * r.fwd->lexec * sizeof(float2);
  const size_t nc = (size_t)batch * r.n_ops * r.P * sizeof(float2);
  return 2 * al(nz) + 2 * al(nc) + 256;
}

hipError_t run_real_1d(const RealPath& r, const void* g, void* y, int64_t batch, void* ws, const int64_t* offs,
                       hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const FftSide& f = *r.fwd;
  const FftSide& v = *r.inv;
  const int64_t Lz = f.lexec;
  char* base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  const size_t nz = al((size_t)batch * r.M * Lz * sizeof(float2));
  const size_t nc = al((size_t)batch * r.n_ops * r.P * sizeof(float2));
  float2* Zf = (float2*)base;
  float2* T1 = (float2*)(base + nz);
  float2* Zc = (float2*)(base + 2 * nz);
  float2* T2 = (float2*)(base + 2 * nz + nc);
  // 1. channel DFTs straight from the sample rows (row m of signal b: complex offset
  //    (b M + m) H, or offs[2 b] / 2 + m H)
  LineXform x;
  x.in = (const float2*)g; x.out = Zf; x.tmp = T1; x.count = batch * r.M;
  x.A = f.fa; x.B = f.fb; x.sign = -1;
  x.twA = (const float2*)f.twA; x.twB = (const float2*)f.twB; x.twL = (const float2*)f.tw;
  const int64_t L_in = r.half ? r.H : r.N;   // complex pairs, or real samples, per row
  x.in_offs = offs; x.in_per = r.M; x.in_sig = r.M * L_in; x.in_tr = L_in;
  x.real_in = !r.half;
  x.in_half = r.f16;
  x.len_in = L_in;
  x.out_sig = Lz;
  if (f.blue) {
    x.pre = (const float2*)f.chirp;
    x.post = (const float2*)f.bhat;
  }
  hipError_t e = fft_lines(x, s);
  if (e != hipSuccess) return e;
  if (f.blue) {
    LineXform u;
    u.in = Zf; u.out = Zf; u.tmp = T1; u.count = batch * r.M;
    u.A = f.fa; u.B = f.fb; u.sign = +1;
    u.twA = (const float2*)f.twA; u.twB = (const float2*)f.twB; u.twL = (const float2*)f.tw;
    u.in_sig = u.out_sig = Lz;
    if ((e = fft_lines(u, s)) != hipSuccess) return e;
  }
  // 2. apply, real part, polyphase gather: bins across x, signals across y (each thread
  //    takes every gridDim.y-th signal)
  const int gx = (int)((r.P / 2 + 1 + 255) / 256);
  const int gy = (int)std::max<int64_t>(1, std::min<int64_t>({batch, std::max<int64_t>(1, 65536 / gx), 65535}));
  const int n1r = (int)(((r.n1 % r.N) + r.N) % r.N);
  hipLaunchKernelGGL(k_apply_real, dim3(gx, gy), dim3(256), 0, s, Zf, Lz, f.blue ? (const float2*)f.chirp : nullptr,
                     r.wN, r.tab, r.Wo, Zc, r.M, r.n_ops, (int)r.N, (int)r.H, (int)r.n1, n1r, (int)r.K, (int)r.P,
                     batch, r.half ? 1 : 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 3. one inverse transform of length P per (signal, op), written as the output row
  LineXform o;
  o.in = Zc; o.out = (float2*)y; o.tmp = T2; o.count = batch * r.n_ops;
  o.A = v.fa; o.B = v.fb; o.sign = +1;
  o.twA = (const float2*)v.twA; o.twB = (const float2*)v.twB; o.twL = (const float2*)v.tw;
  o.in_sig = r.P;
  o.out_offs = offs; o.out_per = r.n_ops; o.out_sig = r.n_ops * r.P; o.out_tr = r.P;
  o.out_half = r.f16;
  return fft_lines(o, s);
}

}  // namespace mci
