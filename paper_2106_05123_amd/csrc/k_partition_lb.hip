// Partition pass, deterministic look-back form (PDQ_DETERMINISTIC). The
// kernel itself is in partition_kernel.h.
#include "partition_kernel.h"

namespace pdq {

hipError_t launch_partition_lb(const Ctx& c, int parity, uint32_t ntiles, uint32_t src_buf, hipStream_t s) {
  return launch_mode<true>(c, parity, ntiles, src_buf, s);
}

}  // namespace pdq
