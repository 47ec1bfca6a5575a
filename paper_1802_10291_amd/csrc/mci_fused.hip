// mci_fused.hip -- single-pass fused 1-D kernels.
#include "mci_fused.h"

namespace mci {

mci_status fused_select(const mci_plan_desc& d, int prec, int store, const void* tab, FusedPlan& fp) {
  (void)d; (void)prec; (void)store; (void)tab;
  fp.kind = 0;
  return MCI_OK;
}

void fused_release(FusedPlan& fp) {
  if (fp.tables) (void)hipFree(fp.tables);
  fp.tables = nullptr;
  fp.kind = 0;
}

hipError_t fused_run(const FusedPlan& fp, const void* g, void* y, int64_t batch, hipStream_t s) {
  (void)fp; (void)g; (void)y; (void)batch; (void)s;
  return hipErrorInvalidValue;
}

}  // namespace mci
