// Entry points whose device implementation is not built yet: they report
// SGDG_ERR_UNSUPPORTED so a caller never mistakes them for results.
#include "internal.h"

namespace sgdg {
size_t iif2_ws_bytes(const sgdg_plan*, int, int) { return 0; }
sgdg_status reaction_build(sgdg_plan*) { return SGDG_OK; }
void reaction_destroy(sgdg_plan*) {}
}  // namespace sgdg

using namespace sgdg;

extern "C" sgdg_status sgdg_reaction(const sgdg_plan*, int32_t, const double*, double*, void*, size_t, void*) {
  return fail(SGDG_ERR_UNSUPPORTED, "sgdg_reaction: not built");
}
extern "C" sgdg_status iif2_step(const sgdg_plan*, int32_t, double, int32_t, double*, double*, double, int32_t, void*,
                                 size_t, sgdg_stats*, void*) {
  return fail(SGDG_ERR_UNSUPPORTED, "iif2_step: not built");
}
