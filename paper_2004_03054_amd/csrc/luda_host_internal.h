// Library-internal helpers shared by the host runtime sources (not part of
// the C-ABI).
#pragma once
#include "luda.h"

namespace luda {

// Move a result's output tables from device memory to host memory (the
// device buffer is released); a no-op for results without files or with
// host outputs already.  Returns LUDA_OK, LUDA_NOMEM or LUDA_DEVICE.
int result_to_host(luda_ctx* c, luda_result* r);

// The same for the n results of one call: results that share one device
// buffer (one batched pass) come back in one copy into one host block.
int results_to_host(luda_ctx* c, luda_result* res, uint32_t n);

}  // namespace luda
