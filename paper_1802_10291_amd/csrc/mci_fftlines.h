// mci_fftlines.h -- FP32 transforms of the multi-pass path in one or two LDS passes.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mci_bandgen.h"

namespace mci {

// Pass 1 of an A x B transform of length L multiplies element k_b of line a by w_L^m,
// m = a k_b < L.  The factors come from a two-level table: w_L^m = lo[m mod kTwLo] hi[m / kTwLo],
// lo[j] = w_L^j (entries 0 .. kTwLo - 1) and hi[i] = w_L^{kTwLo i} (entries kTwLo + i), both
// exact roundings, so a factor is one rounding further from w_L^m than a direct table entry,
// and the 8 KB low table stays in the L1 cache where a per-element gather from an L-entry
// table missed it on nearly every element.
constexpr int kTwLoBits = 10;
constexpr int64_t kTwLo = (int64_t)1 << kTwLoBits;
inline int64_t fl_twiddle_entries(int64_t L) { return kTwLo + (L + kTwLo - 1) / kTwLo; }

// a line length of the register-staged line FFT: 32, 48, 64, 96, 128, 192, 256, 384, 512
bool line_length_ok(int64_t n);
// L = A B with A, B line lengths (most balanced, the larger A among equals), or A = 1 and B = L for a line length
bool two_pass_factors(int64_t L, int& A, int& B);
// smallest length >= n that two_pass_factors accepts, or -1
int64_t next_two_pass_length(int64_t n);
// raise the dynamic-LDS limit of the kernels of an A x B transform (plan time)
hipError_t prepare_two_pass(int A, int B);
// A general one- or two-pass transform: count transforms of length A B (A = 1: one pass of
// length B).  Transform t reads from in + base_in(t) and writes to out + base_out(t), where
// base = offs ? offs[2 (t / per) + side] / 2 + (t % per) tr : (t / per) sig + (t % per) tr, in
// complex elements (offs: per-instance element offsets of real data, side 0 input / 1 output).
// pre (optional): input position p < len_in is multiplied by pre[p], positions >= len_in
// read as zero (chirp and zero padding); real_in: the input is real values.  post
// (optional): output position k is multiplied
// by post[k].  tmp holds count A B complex (two passes only).
struct LineXform {
  const float2* in = nullptr;
  float2* out = nullptr;
  float2* tmp = nullptr;
  int64_t count = 0;
  int A = 1, B = 0, sign = -1;
  const float2 *twA = nullptr, *twB = nullptr, *twL = nullptr;   // twL: the two-level table above
  const int64_t* in_offs = nullptr;
  int64_t in_per = 1, in_sig = 0, in_tr = 0;
  const int64_t* out_offs = nullptr;
  int64_t out_per = 1, out_sig = 0, out_tr = 0;
  const float2* pre = nullptr;
  int64_t len_in = 0;
  const float2* post = nullptr;
  // input is real (float): position p reads (in[p], 0) for p < len_in, else 0; in_sig, in_tr
  // and the input offsets are then in real elements
  bool real_in = false;
  // FP16 storage of the input (the first pass reads it) or of the output (the last pass
  // writes it); offsets and strides stay in elements of the stored type
  bool in_half = false, out_half = false;
  // optional: the input is not read but computed, position p of transform t being
  // band_bin(*gen, t, p) (the real-mode apply); in, pre and the input layout are then unused
  const BandGen* gen = nullptr;
};
hipError_t fft_lines(const LineXform& x, hipStream_t s);
// Bluestein's chirp convolution, for two-pass lengths (A > 1): the forward transform of x's
// input (x.pre applied as it loads), times filt at each natural position, then the inverse
// transform (x.post applied as it stores) into x.out, in three passes instead of four: the
// forward's second pass, the product and the inverse's first pass (factors B x A, so that it
// takes the same lines) run in one kernel.  x.tmp and mid hold count A B complex each; x.out,
// x.tmp and mid are distinct.  Forward direction (x.sign = -1), FP32 output.
hipError_t fft_chirp_conv(const LineXform& x, const float2* filt, float2* mid, hipStream_t s);

// count transforms of length A B (contiguous, complex) from in to out with sign `sign`;
// tmp (count A B complex) holds the pass-1 result; twA, twB, twL: e^{-2 pi i k / n} tables of
// n = A, B, A B entries (twA unused when A = 1).  in may equal out; tmp must differ from both.
hipError_t fft_two_pass(const float2* in, float2* out, float2* tmp, int64_t count, int A, int B, int sign,
                        const float2* twA, const float2* twB, const float2* twL, hipStream_t s);

}  // namespace mci
