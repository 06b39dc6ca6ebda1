// Partition pass, reservation form (the default), and the entry point that
// picks the form. The kernel itself is in partition_kernel.h.
#include "partition_kernel.h"

namespace pdq {

hipError_t launch_partition_lb(const Ctx& c, int parity, uint32_t ntiles, uint32_t src_buf, hipStream_t s);

hipError_t launch_partition(const Ctx& c, int parity, uint32_t ntiles, uint32_t src_buf, hipStream_t s) {
  if (c.lookback) return launch_partition_lb(c, parity, ntiles, src_buf, s);
  return launch_mode<false>(c, parity, ntiles, src_buf, s);
}

}  // namespace pdq
