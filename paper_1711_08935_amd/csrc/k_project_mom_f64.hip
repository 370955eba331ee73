// Orbital and position-moment projection, FP64 state storage.
#include "k_project_mom.h"

hipError_t launch_project_mom_f64(const ProjArgs& a, int nitems, int nq, hipStream_t st) {
    return launch_project_mom_prec<double>(a, nitems, nq, st);
}
