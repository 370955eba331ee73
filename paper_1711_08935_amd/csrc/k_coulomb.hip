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
//                    (a few points p per lane; the source points p' are
//                    staged through LDS and read as broadcasts)
//   k_coul_contract: T[pair1][pair2] = dV sum_p rho[p][pair1] W[p][pair2],
//                    one work-group per entry, written to the full L^4
//                    tensor.

#include "ksmall.h"

namespace {

__global__ void k_coul_rho(const CoulombArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    int t = 0;
    for (int i = 0; i < a.L; ++i)
        for (int j = i; j < a.L; ++j) a.rho[static_cast<int64_t>(p) * a.npair + t++] = a.phi[p * a.L + i] * a.phi[p * a.L + j];
}

// One lane per target point p (PT points per lane), source points p' staged
// through LDS in tiles; every lane reads the same p' (LDS broadcast).
template <int NP, int PT>
__global__ void __launch_bounds__(256) k_coul_pot(const CoulombArgs a) {
    constexpr int TILE = 64;
    __shared__ double rs[TILE][NP];
    __shared__ int qs[TILE][3];
    const int tid = threadIdx.x;
    int ix[PT], iy[PT], iz[PT];
    bool ok[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
        const int p = (blockIdx.x * PT + t) * blockDim.x + tid;
        ok[t] = p < a.P;
        const int pp = ok[t] ? p : 0;
        ix[t] = a.ijk[3 * pp];
        iy[t] = a.ijk[3 * pp + 1];
        iz[t] = a.ijk[3 * pp + 2];
    }
    double acc[PT][NP];
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int k = 0; k < NP; ++k) acc[t][k] = 0.0;
    for (int q0 = 0; q0 < a.P; q0 += TILE) {
        const int nq = min(TILE, a.P - q0);
        for (int i = tid; i < nq * NP; i += blockDim.x)
            rs[i / NP][i % NP] = a.rho[static_cast<int64_t>(q0) * NP + i];
        for (int i = tid; i < nq * 3; i += blockDim.x) qs[i / 3][i % 3] = a.ijk[3 * q0 + i];
        __syncthreads();
        for (int j = 0; j < nq; ++j) {
            double K[PT];
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                const double dx = static_cast<double>(ix[t] - qs[j][0]) * a.h[0];
                const double dy = static_cast<double>(iy[t] - qs[j][1]) * a.h[1];
                const double dz = static_cast<double>(iz[t] - qs[j][2]) * a.h[2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                K[t] = (r2 > 0.0) ? 1.0 / sqrt(r2) : a.g0;
            }
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const double r = rs[j][k];
#pragma unroll
                for (int t = 0; t < PT; ++t) acc[t][k] = fma(K[t], r, acc[t][k]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < PT; ++t) {
        if (!ok[t]) continue;
        const int p = (blockIdx.x * PT + t) * blockDim.x + tid;
#pragma unroll
        for (int k = 0; k < NP; ++k) a.W[static_cast<int64_t>(p) * NP + k] = a.dV * acc[t][k];
    }
}

// One work-group per pair-density entry (i, j): Tp = dV sum_p rho[p][i] W[p][j],
// then written to the four (a,b,c,d) orderings that share the pairs.
__global__ void __launch_bounds__(256) k_coul_contract(const CoulombArgs a) {
    __shared__ double red[256];
    const int np = a.npair;
    const int i = blockIdx.x / np, j = blockIdx.x % np;
    double s = 0.0;
    for (int p = threadIdx.x; p < a.P; p += blockDim.x)
        s = fma(a.rho[static_cast<int64_t>(p) * np + i], a.W[static_cast<int64_t>(p) * np + j], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double v = a.dV * red[0];
    const int L = a.L;
    // pair index i -> (A <= B)
    int A = 0, B = 0, C = 0, D = 0;
    for (int x = 0, t = 0; x < L; ++x)
        for (int y = x; y < L; ++y, ++t) {
            if (t == i) { A = x; B = y; }
            if (t == j) { C = x; D = y; }
        }
    auto at = [L](int w, int x, int y, int z) { return ((w * L + x) * L + y) * L + z; };
    a.tensor[at(A, B, C, D)] = v;
    a.tensor[at(B, A, C, D)] = v;
    a.tensor[at(A, B, D, C)] = v;
    a.tensor[at(B, A, D, C)] = v;
}

}  // namespace

hipError_t launch_coulomb(const CoulombArgs& a, hipStream_t st) {
    const int nb = (a.P + 255) / 256;
    hipLaunchKernelGGL(k_coul_rho, dim3(nb), dim3(256), 0, st, a);
    switch (a.npair) {
    case 1: hipLaunchKernelGGL((k_coul_pot<1, 4>), dim3((a.P + 1023) / 1024), dim3(256), 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_coul_pot<6, 4>), dim3((a.P + 1023) / 1024), dim3(256), 0, st, a); break;
    case 15: hipLaunchKernelGGL((k_coul_pot<15, 2>), dim3((a.P + 511) / 512), dim3(256), 0, st, a); break;
    case 28: hipLaunchKernelGGL((k_coul_pot<28, 2>), dim3((a.P + 511) / 512), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_coul_contract, dim3(a.npair * a.npair), dim3(256), 0, st, a);
    return hipGetLastError();
}
