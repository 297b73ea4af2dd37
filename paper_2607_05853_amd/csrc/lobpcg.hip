// placeholder, replaced below
#include "bse_internal.h"
extern "C" bse_status bse_lowest_excitons(bse_plan*, int32_t, int32_t, double, const void*, double*, void*,
                                          int32_t*, void*) {
  bse::set_error("bse_lowest_excitons: not available");
  return BSE_EINVAL;
}
