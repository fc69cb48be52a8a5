// Error state, version and defaults of the C ABI.
#include <string>

#include "pmrf_internal.h"

namespace {
thread_local std::string g_last_error;
}

namespace pmrf {
pmrf_status fail(pmrf_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
void clear_error() { g_last_error.clear(); }
}  // namespace pmrf

extern "C" const char *pmrf_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t pmrf_abi_version(void) { return 2; }

extern "C" void pmrf_em_params_default(pmrf_em_params *p) {
  if (!p) return;
  p->L = 2;
  p->beta = 0.5;
  p->max_iters = 20;
  p->conv_window = 3;
  p->conv_tol = 1e-4;
  p->early_exit = 0;
  p->init_from_labels = 0;
  p->sigma_min = 1e-3;
  p->tie_eps = 1e-9;
  p->scatter_rule = PMRF_SCATTER_OWNER;
}
