// Apply kernels, grouped work list, FP32 state storage (FP64 sums).
#include "k_apply.h"

hipError_t launch_apply_grouped_f32(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, int cls,
                                   hipStream_t st) {
    return launch_apply_grouped_prec<float>(a, nchunks, nq, cplx, cpl, waves, cls, st);
}
