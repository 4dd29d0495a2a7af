// Kernel timing hooks (see ls_stats_enable in ls.h).
#pragma once

#include "ls_internal.h"

namespace ls {

bool stats_on();
// Records the start event of `count` back-to-back timed launches of `kind` on
// `stream`; *slot < 0 when they are not timed.
int stats_before(int kind, hipStream_t stream, int64_t *slot, int64_t count = 1);
int stats_after(int kind, hipStream_t stream, int64_t slot);

}  // namespace ls
