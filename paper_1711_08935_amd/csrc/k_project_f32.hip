// Projection kernels for FP32 state storage (FP64 products and sums).
#include "k_project.h"

hipError_t launch_project_f32(const ProjArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, int cls,
                              hipStream_t st) {
    return launch_project_prec<float>(a, nchunks, nq, cplx, cpl, waves, cls, st);
}
