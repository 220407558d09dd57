// Kernels of the ragged-batch restore in mode MODE_LEARNED (batch_kernel.h), one source file per
// mode so that the modes compile in parallel.
#include "batch_kernel.h"

namespace ht {

void batch_launch_learned(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid, hipStream_t stream) {
    launch_mode<MODE_LEARNED>(a, c, variant, start, cnt, grid, stream);
}

void batch_launch_learned_rc(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid,
                             hipStream_t stream) {
    launch_mode<MODE_LEARNED_RC>(a, c, variant, start, cnt, grid, stream);
}

}  // namespace ht
