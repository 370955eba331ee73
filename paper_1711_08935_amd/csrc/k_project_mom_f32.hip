// Orbital and position-moment projection, FP32 state storage.
#include "k_project_mom.h"

hipError_t launch_project_mom_f32(const ProjArgs& a, int nitems, int nq, hipStream_t st) {
    return launch_project_mom_prec<float>(a, nitems, nq, st);
}
