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
  int ti = 1;              // output transforms run side by side
};

// Choose a fused kernel for the descriptor (kind stays 0 when none applies).
mci_status fused_select(const mci_plan_desc& d, int prec, int store, const void* tab, FusedPlan& fp);
void fused_release(FusedPlan& fp);
hipError_t fused_run(const FusedPlan& fp, const void* g, void* y, int64_t batch, hipStream_t s);

}  // namespace mci
