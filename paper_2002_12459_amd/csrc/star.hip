// Star join-project (Section 3.2); filled in below the two-path pipeline.
#include "pipeline.hpp"

namespace jp {
jp_result *run_star(const Ctx &, int, const int32_t *const *, const int32_t *const *, const int64_t *,
                    const jp_options &) {
    fail(JP_EINTERNAL, "star query not built yet");
}
}  // namespace jp
