// Kernels of the ragged-batch restore in mode MODE_SCAN (batch_kernel.h), one source file per
// mode so that the modes compile in parallel.
#include "batch_kernel.h"

namespace ht {

void batch_launch_scan(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid, hipStream_t stream) {
    launch_mode<MODE_SCAN>(a, c, variant, start, cnt, grid, stream);
}

template <int LOGP, int S, int SL>
static int max_active(int device) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_restore<LOGP, S, SL, MODE_SCAN>, (1 << LOGP) / SL, 0) !=
        hipSuccess)
        nb = 1;
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) cus = prop.multiProcessorCount;
    return nb > 1 ? nb * cus : cus;
}

int batch_full_grid(int cls, int variant, int device) {
    switch (cls) {
        case 0: return max_active<9, 1, 8>(device);
        case 1: return max_active<10, 1, 8>(device);
        case 2: return max_active<11, 1, 8>(device);
        case 3: return variant ? max_active<12, 1, 16>(device) : max_active<12, 1, 8>(device);
        case 4: return variant ? max_active<13, 1, 16>(device) : max_active<13, 1, 8>(device);
        default: return variant ? max_active<13, 2, 16>(device) : max_active<13, 2, 8>(device);
    }
}

}  // namespace ht
