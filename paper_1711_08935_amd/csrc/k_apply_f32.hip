// Apply kernels, per-site (layered) work list, FP32 state storage (FP64 sums).
#include "k_apply.h"

hipError_t launch_apply_f32(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, hipStream_t st) {
    return launch_apply_prec<float>(a, nchunks, nq, cplx, cpl, waves, st);
}
