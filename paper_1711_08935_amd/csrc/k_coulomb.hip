// On-site Coulomb tensor of one site, evaluated on the real-space grid
// (Sec. III: the integrals are computed from the orbitals on the grid;
// App. B gives the (m m'|m'' m''') notation):
//
//   (ab|cd) = dV^2 sum_{p, p'} rho_ab(p) K(p - p') rho_cd(p'),
//   rho_ab = phi_a phi_b,  K(r) = 1/|r| (r != 0),  K(0) = G0,
//
// over the site's unfolded sphere points (free-space, single-centre).  G0 is
// the average of 1/r over one grid cell.  This is the direct O(P^2) double
// sum: a dense FP64 contraction whose kernel matrix is generated on the fly
// from integer point offsets, so it never touches HBM for K.
//
//   k_coul_rho:      rho[p][pair] for the L(L+1)/2 pairs a <= b
//   k_coul_pot:      W[p][pair] = dV sum_p' K(p - p') rho[p'][pair]
//                    (one point p per lane; p' is uniform across the wave,
//                    so its coordinates and densities are scalar loads)
//   k_coul_contract: T[pair1][pair2] = dV sum_p rho[p][pair1] W[p][pair2],
//                    expanded to the full L^4 tensor.

#include "ksmall.h"

namespace {

__global__ void k_coul_rho(const CoulombArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    int t = 0;
    for (int i = 0; i < a.L; ++i)
        for (int j = i; j < a.L; ++j) a.rho[static_cast<int64_t>(p) * a.npair + t++] = a.phi[p * a.L + i] * a.phi[p * a.L + j];
}

template <int NP>
__global__ void __launch_bounds__(256) k_coul_pot(const CoulombArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = p < a.P;
    const int pp = ok ? p : 0;
    const int ix = a.ijk[3 * pp], iy = a.ijk[3 * pp + 1], iz = a.ijk[3 * pp + 2];
    double acc[NP];
#pragma unroll
    for (int t = 0; t < NP; ++t) acc[t] = 0.0;
    for (int q = 0; q < a.P; ++q) {
        const double dx = static_cast<double>(ix - a.ijk[3 * q]) * a.h[0];
        const double dy = static_cast<double>(iy - a.ijk[3 * q + 1]) * a.h[1];
        const double dz = static_cast<double>(iz - a.ijk[3 * q + 2]) * a.h[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double K = (r2 > 0.0) ? 1.0 / sqrt(r2) : a.g0;
        const double* __restrict__ rq = a.rho + static_cast<int64_t>(q) * NP;
#pragma unroll
        for (int t = 0; t < NP; ++t) acc[t] = fma(K, rq[t], acc[t]);
    }
    if (!ok) return;
#pragma unroll
    for (int t = 0; t < NP; ++t) a.W[static_cast<int64_t>(p) * NP + t] = a.dV * acc[t];
}

__global__ void __launch_bounds__(256) k_coul_contract(const CoulombArgs a) {
    // one work-group; thread handles pair-pair entries o = tid, tid + 256, ...
    __shared__ double red[256];
    const int np = a.npair;
    const int L = a.L;
    __shared__ double Tp[28 * 28];
    for (int o = 0; o < np * np; ++o) {
        const int i = o / np, j = o % np;
        double s = 0.0;
        for (int p = threadIdx.x; p < a.P; p += blockDim.x)
            s = fma(a.rho[static_cast<int64_t>(p) * np + i], a.W[static_cast<int64_t>(p) * np + j], s);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) Tp[o] = a.dV * red[0];
        __syncthreads();
    }
    // expand: pair index of (a, b) with a <= b
    for (int o = threadIdx.x; o < L * L * L * L; o += blockDim.x) {
        const int A = o / (L * L * L), B = (o / (L * L)) % L, C = (o / L) % L, D = o % L;
        auto pidx = [L](int x, int y) {
            const int lo = x < y ? x : y, hi = x < y ? y : x;
            return lo * L - lo * (lo - 1) / 2 + (hi - lo);
        };
        a.tensor[o] = Tp[pidx(A, B) * np + pidx(C, D)];
    }
}

}  // namespace

hipError_t launch_coulomb(const CoulombArgs& a, hipStream_t st) {
    const int nb = (a.P + 255) / 256;
    hipLaunchKernelGGL(k_coul_rho, dim3(nb), dim3(256), 0, st, a);
    switch (a.npair) {
    case 1: hipLaunchKernelGGL(k_coul_pot<1>, dim3(nb), dim3(256), 0, st, a); break;
    case 6: hipLaunchKernelGGL(k_coul_pot<6>, dim3(nb), dim3(256), 0, st, a); break;
    case 15: hipLaunchKernelGGL(k_coul_pot<15>, dim3(nb), dim3(256), 0, st, a); break;
    case 28: hipLaunchKernelGGL(k_coul_pot<28>, dim3(nb), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_coul_contract, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}
