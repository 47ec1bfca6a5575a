// mci_realpath.hip -- real-mode 1-D reconstruction in a few LDS-pass kernels, for lengths no
// single workgroup holds.  The steps are those of the single-pass kernel, each a pass over HBM:
//
//  1. channel DFTs (Lemma 3.1): row m of the real samples, read as H = N/2 complex pairs
//     z[p] = g[2p] + i g[2p+1] (odd N: as N real values), goes through a one- or two-pass
//     transform of length H (N) (through Bluestein's chirp convolution when that length does
//     not factor: the chirp is applied as the first pass loads, the filter spectrum between the
//     forward transform's last pass and the inverse's first, which share one kernel for two-pass
//     lengths, and the output chirp as the inverse transform's last pass stores);
//  2. apply (eq. matrixeqn1) and the real part: X_m[r] = E[r'] + e^{-2 pi i r / N} O[r'],
//     r' = r mod H, with E, O the even/odd-sample DFTs recovered from Z (odd N: X_m = Z);
//     a(k) = sum_m X_m[k mod N] Tab[m][j][i] for k = n1 + i + jN; S(k) = (a(k) + conj a(-k)) / 2;
//  3. output: with P = n_out / 2 and w = e^{2 pi i / n_out}, the two polyphase components
//     y[2q] and y[2q + 1] are the real and imaginary parts of
//       z[q] = sum_b Zc[b] e^{2 pi i b q / P},  Zc[b] = sum_{k = b mod P} S(k) (1 + i w^k),
//     so one complex inverse transform of length P yields the whole real output, and its
//     complex result, stored as it is, is the output row.
// Steps 2 and 3 share a pass: the inverse transform's first pass computes each input bin
// Zc[b] from the channel spectra as it loads it (mci_bandgen.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mci_bandgen.h"
#include "mci_device.h"
#include "mci_fftlines.h"
#include "mci_jobs.h"
#include "mci_realpath.h"

namespace mci {

static size_t al(size_t n) { return (n + 255) & ~(size_t)255; }

size_t real_path_workspace(const RealPath& r, int64_t batch) {
  if (batch <= 0) return 0;
  const size_t nz = (size_t)batch * r.M * r.fwd->lexec * sizeof(float2);
  const size_t nc = (size_t)batch * r.n_ops * r.P * sizeof(float2);
  // the third region is the output transform's scratch, and the chirp convolution's middle
  // result before it
  return 2 * al(nz) + al(r.fwd->blue ? std::max(nz, nc) : nc) + 256;
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
  float2* T2 = (float2*)(base + 2 * nz);
  (void)nc;
  // 1. channel DFTs straight from the sample rows (row m of signal b: complex offset
  //    (b M + m) H, or offs[2 b] / 2 + m H)
  LineXform x;
  x.in = (const float2*)g; x.out = Zf; x.tmp = T1; x.count = batch * r.M;
  x.A = f.fa; x.B = f.fb; x.sign = -1;
  x.twA = (const float2*)f.twA; x.twB = (const float2*)f.twB; x.twL = (const float2*)f.twL;
  const int64_t L_in = r.half ? r.H : r.N;   // complex pairs, or real samples, per row
  x.in_offs = offs; x.in_per = r.M; x.in_sig = r.M * L_in; x.in_tr = L_in;
  x.real_in = !r.half;
  x.in_half = r.f16;
  x.len_in = L_in;
  x.out_sig = Lz;
  hipError_t e;
  if (f.blue && f.fa > 1) {
    // the chirp convolution in three passes, Zf = chirp * IDFT(DFT(chirp * z) * bhat), its
    // middle result in T2 (free until the output transform)
    x.pre = (const float2*)f.chirp;
    x.post = (const float2*)f.chirp;
    if ((e = fft_chirp_conv(x, (const float2*)f.bhat, T2, s)) != hipSuccess) return e;
  } else {
    if (f.blue) {
      x.pre = (const float2*)f.chirp;
      x.post = (const float2*)f.bhat;
    }
    if ((e = fft_lines(x, s)) != hipSuccess) return e;
    if (f.blue) {
      LineXform u;
      u.in = Zf; u.out = Zf; u.tmp = T1; u.count = batch * r.M;
      u.A = f.fa; u.B = f.fb; u.sign = +1;
      u.twA = (const float2*)f.twA; u.twB = (const float2*)f.twB; u.twL = (const float2*)f.twL;
      u.in_sig = u.out_sig = Lz;
      u.post = (const float2*)f.chirp;   // the output chirp, applied as the last pass stores
      if ((e = fft_lines(u, s)) != hipSuccess) return e;
    }
  }
  // 2-3. one inverse transform of length P per (signal, op), written as the output row; its
  //    first pass computes its input, the gathered spectrum Zc, from the channel spectra as
  //    it loads it (the apply, the real part and the polyphase gather: band_bin)
  const BandGen bg{Zf, Lz, nullptr, r.wN, r.D, r.M, r.n_ops,
                   (int)r.N, (int)r.H, (int)r.n1, (int)r.K, (int)r.P, r.half ? 1 : 0,
                   r.P >= 2 * r.K + 1 ? 1 : 0};
  LineXform o;
  o.in = nullptr; o.out = (float2*)y; o.tmp = T2; o.count = batch * r.n_ops;
  o.A = v.fa; o.B = v.fb; o.sign = +1;
  o.twA = (const float2*)v.twA; o.twB = (const float2*)v.twB; o.twL = (const float2*)v.twL;
  o.in_sig = r.P;
  o.out_offs = offs; o.out_per = r.n_ops; o.out_sig = r.n_ops * r.P; o.out_tr = r.P;
  o.out_half = r.f16;
  o.gen = &bg;
  return fft_lines(o, s);
}

}  // namespace mci
