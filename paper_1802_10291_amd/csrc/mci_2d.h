// mci_2d.h -- fused line passes of the separable 2-D upsampling.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <vector>

#include "mci_internal.h"

namespace mci {

struct LinePassArgs {
  const void* x;
  void* y;
  int64_t lines;       // rows mode: number of lines
  int64_t W;           // columns mode: columns per image (lines per image)
  const float2* H;     // [SC][N] polyphase windows
  const float2* tw;    // N entries e^{-2 pi i k / N}
  // Optional per-image placement (device, 2 per image): columns mode reads image b at
  // x + offs[2 b]; rows mode writes line l to image l / lines_per_img at y + offs[2 b + 1].
  const int64_t* offs = nullptr;
  int64_t lines_per_img = 1;
  // Sample rows passed through (the `zr` forms, FP32 only).  Where the columns pass's
  // polyphase window H_0 is the identity (y[s q] = x[q], interpolation consistency), the
  // columns pass computes and writes only the rows s q + r, r >= 1, packed as row
  // (s - 1) q + r - 1 of a (s - 1) h-row image, and the rows pass reads line s q + 0 of
  // image b straight from row q of the input image: x0 + offs[2 b] (or x0 + b h W) + q W.
  const void* x0 = nullptr;
};

bool line_pass_supported(int N, int SC);
std::vector<std::complex<double>> line_windows(const std::vector<std::complex<double>>& tab, int64_t N, int64_t n1,
                                               int SC, int M);
hipError_t run_line_pass(int N, int SC, bool cols, bool zr, int store_in, int store_out, const LinePassArgs& a,
                         int64_t images, hipStream_t s);
// set the dynamic-LDS limit of the pass's kernel where it exceeds 64 KB (once, at plan time)
hipError_t prepare_line_pass(int N, int SC, bool cols, bool zr, int store_in, int store_out);

}  // namespace mci
