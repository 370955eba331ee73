// Apply kernels, grouped work list, FP64 state storage.
#include "k_apply.h"

hipError_t launch_apply_grouped_f64(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, int cls,
                                   hipStream_t st) {
    return launch_apply_grouped_prec<double>(a, nchunks, nq, cplx, cpl, waves, cls, st);
}
