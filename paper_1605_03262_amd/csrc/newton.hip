// Batched Newton-matrix solves (I - h gamma J) x = b.  Placeholder entry
// points until the solvers land; they report PYJAC_E_UNSUPPORTED.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/pyjac.h"

namespace pyjac {
pyjac_status fail(pyjac_status code, const std::string& msg);
}

extern "C" {

size_t pyjac_newton_workspace_bytes(const pyjac_mech*, int64_t, int32_t) { return 0; }

pyjac_status pyjac_newton_factor_solve(const pyjac_mech*, int64_t, int64_t, const double*, const double*,
                                       double, const double*, double*, int32_t, int32_t, double, int32_t*,
                                       void*, size_t, void*) {
  return pyjac::fail(PYJAC_E_UNSUPPORTED, "Newton solver not built yet");
}

}  // extern "C"
