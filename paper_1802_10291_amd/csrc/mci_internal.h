// mci_internal.h -- host-side structures and kernel launchers shared by the libmci
// translation units (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mci.h"

namespace mci {

// One direction of a DFT of logical length `len` as the library executes it: a Stockham
// FFT of length `lexec` (= len, or the Bluestein length P for lengths with a prime
// factor above 7) with the given radices.
struct FftSide {
  int64_t len = 0;
  int sign = -1;          // -1: e^{-2 pi i k n / len} (forward), +1: inverse
  bool blue = false;
  int64_t lexec = 0;
  std::vector<int> radices;   // radices of lexec run by the kernels (one of the two below)
  std::vector<int> radices8;  // radix-8 passes first, then at most one 4 and one 2, then 3, 5, 7
  std::vector<int> radices4;  // radix-4 passes, at most one 2, then 3, 5, 7
  void* tw = nullptr;         // e^{-2 pi i k / lexec}, lexec entries, plan precision
  // FP32 plans: lexec = fa fb for the one- or two-pass LDS transform (fa = 1: one pass),
  // with line twiddles twA (fa entries) and twB (fb entries); two_pass selects it
  int fa = 0, fb = 0;
  void* twA = nullptr;
  void* twB = nullptr;
  // pass 1's twiddles w^m, m < lexec, as a product of two small tables (see mci_fftlines.h)
  void* twL = nullptr;
  bool two_pass = false;
  void* chirp = nullptr;      // Bluestein: e^{sign i pi k^2 / len} for k < len, zero-padded to lexec entries
  void* bhat = nullptr;       // Bluestein: forward DFT_P of the conjugate chirp, divided by P
};

// Arguments of the FP64 plan kernel.
struct PlanKernelArgs {
  int M, n_ops;
  int64_t N, n1;
  int kinds[MCI_MAX_CHANNELS], orders[MCI_MAX_CHANNELS];
  int ops[MCI_MAX_OPS], op_orders[MCI_MAX_OPS];
  const double2* tables;  // [M][mu] or null
  double2* tab64;         // [n_ops][M][M][N]
  float2* tab32;          // [n_ops][M][M][N]
  double* cond;           // [N]
  int* sing;              // [N]
  int allow_zero;
  // optional real factor per band index n - n1 (mu entries, device), multiplied into every
  // table entry of coefficient n: the deconvolution of off-grid evaluation; null = none
  const double* oscale = nullptr;
  // optional raw inverse entries q_mj(n1 + i) = (H_n^{-1})[m][j] as [N][M][M] (zero for a
  // singular residue): the averaged-error weights need them without the output operator
  double2* qraw = nullptr;
};

// Arguments of the generic (multi-pass) 1-D path.
struct Generic1D {
  int M, n_ops, real_io;
  int64_t N, n1, n_out;
  const void* tab;        // [n_ops][M][M][N] complex, plan precision
  const FftSide* fwd;
  const FftSide* inv;
};

enum StoreKind { ST_F32 = 0, ST_F64 = 1, ST_F16 = 2 };

// Launchers (mci_kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_plan_tables(const PlanKernelArgs& a, hipStream_t s);
size_t generic_1d_workspace(const Generic1D& g, int prec, int64_t batch);
// offs: per-signal (input, output) element offsets (device, 2 per signal) or null (dense)
hipError_t run_generic_1d(const Generic1D& g, int prec, int store, const void* in, void* out, int64_t batch,
                          void* ws, const int64_t* offs, hipStream_t s);
// 2-D helpers: build the M channels {x, centred difference[, second difference]} of every line.
//   rows: x [B][h][w] -> G [B*h][M][w];  cols: x [B][H][W] (column c is a line of length H)
//   -> G [B*W][M][H].  `deriv_scale` = len / (4 pi).
hipError_t launch_fd_channels(int prec, int store_in, const void* x, void* G, int64_t B, int64_t h, int64_t w,
                              int along_cols, const int64_t* offs, int M, hipStream_t s);
// transpose [B][W][H] -> [B][H][W] with storage conversion to the output type
// (offs: image b's input at x + offs[2 b], output at dst + offs[2 b + 1]; null: dense)
hipError_t launch_transpose_out(int prec, int store_out, const void* src, void* dst, int64_t B, int64_t W,
                                int64_t H, const int64_t* offs, hipStream_t s);

}  // namespace mci
