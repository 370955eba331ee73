// Apply kernels, per-site (layered) work list, FP64 state storage.
#include "k_apply.h"

hipError_t launch_apply_f64(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, hipStream_t st) {
    return launch_apply_prec<double>(a, nchunks, nq, cplx, cpl, waves, st);
}
