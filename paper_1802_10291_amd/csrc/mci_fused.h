// mci_fused.h -- single-pass fused 1-D kernels (one workgroup per signal, every step in LDS).
#pragma once
#include <hip/hip_runtime.h>

#include "mci_internal.h"

namespace mci {

struct FusedPlan {
  int kind = 0;            // 0: no fused kernel for this plan
  void* tables = nullptr;  // device tables owned by the fused plan
  void* args = nullptr;    // kernel argument block (host)
  void* launch = nullptr;  // launcher of the chosen instantiation
  int lds_bytes = 0;
  int grid_cap = 0;
  int ti = 1;              // output transforms run side by side (1 or 2)
  int n_ti = 1;            // 2 when both groupings fit the LDS
  int lds_ti[2] = {0, 0};  // LDS bytes for ti = 1, 2
  int store = ST_F32;      // storage of samples and outputs (ST_F32 or ST_F16)
  char name[96] = {0};     // the kernel instance, for mci_plan_kernel_name
};

// Choose a fused kernel for the descriptor (kind stays 0 when none applies).
mci_status fused_select(const mci_plan_desc& d, int prec, int store, const void* tab, FusedPlan& fp);
void fused_release(FusedPlan& fp);
void fused_set_ti(FusedPlan& fp, int ti);
// offs: per-signal (input, output) element offsets into g and y (device, 2 per signal), or
// null for a dense batch (signal b at b M N and b n_out)
hipError_t fused_run(const FusedPlan& fp, const void* g, void* y, int64_t batch, const int64_t* offs,
                     hipStream_t s);

}  // namespace mci
