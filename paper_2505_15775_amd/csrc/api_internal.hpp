// Host-side helpers shared by the library's entry-point sources.
#pragma once

#include <string>

#include "alm_bm.h"

namespace almbm {

// Records msg as the calling thread's last error (alm_bm_last_error) and
// returns s.
alm_bm_status set_error(alm_bm_status s, const std::string& msg);

// Default grid of the row kernels for n rows: one block per 64 rows, at least
// 8 and at most 4096 blocks, a multiple of 8 (one share per XCD).
int row_blocks(long n);

}  // namespace almbm
