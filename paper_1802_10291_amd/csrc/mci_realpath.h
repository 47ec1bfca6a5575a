// mci_realpath.h -- multi-kernel real-mode 1-D path for lengths no single workgroup holds.
#pragma once
#include <hip/hip_runtime.h>

#include "mci_internal.h"

namespace mci {

struct RealPath {
  bool ok = false;
  bool f16 = false;                // FP16 storage of samples and outputs (arithmetic FP32)
  bool half = true;               // true: rows read as N/2 complex pairs (even N); false: the
                                  // full length-N transform of the real row (fwd has length N)
  int M = 0, n_ops = 0;
  int64_t N = 0, H = 0, n1 = 0, n_out = 0, P = 0, K = 0;
  const FftSide* fwd = nullptr;   // length H (or N), sign -1 (Bluestein when it does not factor)
  const FftSide* inv = nullptr;   // length P = n_out / 2, sign +1, one or two passes
  const float2* wN = nullptr;     // H entries e^{-2 pi i k / N} (half only)
  const float2* D = nullptr;      // [n_ops][M][2K + 1] combined apply / real part / gather weights
};

size_t real_path_workspace(const RealPath& r, int64_t batch);
// g: [batch][M][N] (or per-instance offsets), y: [batch][n_ops][n_out], FP32 or (f16) FP16
hipError_t run_real_1d(const RealPath& r, const void* g, void* y, int64_t batch, void* ws, const int64_t* offs,
                       hipStream_t s);

}  // namespace mci
