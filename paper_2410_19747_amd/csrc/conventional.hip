// Conventional product (Sec. II.A): placeholder until the variational
// driver lands; reports the call as unsupported.
#include "ttm_internal.h"

namespace ttm {
int conventional_query_impl(const ::ttm_tt *, const ::ttm_tt *, int32_t, const ::ttm_options *,
                            size_t *, int64_t *) {
  return TTM_EUNSUPPORTED;
}
int conventional_multiply_impl(const ::ttm_tt *, const ::ttm_tt *, int32_t, double, ::ttm_tt_out *,
                               void *, size_t, void *, const ::ttm_options *, ::ttm_stats *) {
  return TTM_EUNSUPPORTED;
}
}  // namespace ttm
