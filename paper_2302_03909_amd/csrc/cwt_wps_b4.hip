// cwt_wps_b4.hip -- the statistics variants of the two output kernels for up
// to 4 environment bin(s) (Sec. 5), in a translation unit of their own so
// that the variants compile in parallel.
#include "seg_kernels.h"

namespace cwt {

hipError_t launch_out_kernel_wps4(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st) {
    return launch_out_kernel<4>(id, a, blocks, st);
}

}  // namespace cwt
