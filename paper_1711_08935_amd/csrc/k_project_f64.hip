// Projection kernels for FP64 state storage.
#include "k_project.h"

hipError_t launch_project_f64(const ProjArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, int cls,
                              hipStream_t st) {
    return launch_project_prec<double>(a, nchunks, nq, cplx, cpl, waves, cls, st);
}
