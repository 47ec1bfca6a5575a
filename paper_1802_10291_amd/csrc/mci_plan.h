// mci_plan.h -- the plan object behind mci_plan_t and the internal entry points shared by
// the plan API, the uneven-batch runner and the autotuner.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "mci_fused.h"
#include "mci_internal.h"
#include "mci_realpath.h"

struct mci_plan_s {
  int dims = 1;  // 1: 1-D plan, 2: 2-D plan
  int device = 0;
  mci_plan_desc d{};
  int64_t mu = 0;
  int prec = MCI_F32;
  int store = mci::ST_F32;
  void* tab = nullptr;      // [n_ops][M][M][N] complex in plan precision
  mci::FftSide fwd, inv;
  double max_cond = 0.0;
  int64_t n_sing = 0, first_sing = INT64_MIN;
  mci::FusedPlan fused;     // single-pass kernel choice (fused.kind == 0: none)
  bool use_fused = false;   // the fused kernel is the active variant
  // real-mode multi-kernel path (FP32, real_io, even N and n_out): transforms of length N/2
  // and n_out/2, and its tables
  mci::FftSide rfwd, rinv;
  void* r_wN = nullptr;
  void* r_D = nullptr;      // [n_ops][M][2K + 1] combined apply / real part / gather weights
  mci::RealPath real;
  bool use_real = false;
  int variant = MCI_VARIANT_MULTIPASS_R8;
  std::vector<std::complex<double>> tab_host;   // FP64 apply table [n_ops][M][M][N]
  void* qdev = nullptr;     // FP64 inverse entries q_mj(n1 + i), [N][M][M] complex (averaged error)
  // 2-D fused line passes: windows H[SC][len] and twiddles per axis (cols, rows)
  bool lp = false;          // active
  bool lp_avail = false;    // built
  bool lp_zr = false;       // sample rows passed through (the columns pass's H_0 is the identity)
  void* lp_H[2] = {nullptr, nullptr};
  void* lp_tw[2] = {nullptr, nullptr};
  // 2-D
  mci_plan2d_desc d2{};
  mci_plan_s* rows = nullptr;
  mci_plan_s* cols = nullptr;
};

namespace mci {

mci_status fail(mci_status s, const std::string& msg);
// data buffers are accessed with 8- and 16-byte vector loads and stores: every entry point
// requires 16-byte-aligned data pointers and workspaces
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// bytes of one storage element, and per-instance input / output sizes in elements
int store_bytes(int store);
int64_t instance_in_elems(const mci_plan_s* p);
int64_t instance_out_elems(const mci_plan_s* p);

size_t plan_workspace(const mci_plan_s* p, int64_t batch);
// Queue `batch` instances.  offs (device, 2 per instance): element offsets of each
// instance's input and output, or null for a dense batch.  Arguments are not validated.
mci_status plan_run(const mci_plan_s* p, const void* in, void* out, int64_t batch, void* ws, const int64_t* offs,
                    hipStream_t s);

// Build a 1-D plan.  oscale (mu entries, or null): a real factor per band index n - n1
// multiplied into the apply tables (off-grid evaluation's deconvolution).
mci_status build_plan(const mci_plan_desc* desc, int device, mci_plan_s** out,
                      const std::vector<double>* oscale = nullptr);
// smallest n' >= n whose prime factors are all at most 7
int64_t next_smooth_length(int64_t n);

uint32_t plan_variant_mask(const mci_plan_s* p);
mci_status plan_set_variant(mci_plan_s* p, int v);
// cache key of the plan's shape on the current device
std::string plan_tune_key(const mci_plan_s* p);
// variant recorded for `key` in the cache file, or -1
int tune_cache_lookup(const std::string& path, const std::string& key);

}  // namespace mci
