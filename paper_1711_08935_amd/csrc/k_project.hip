// Projection kernel: partial sums of <phi_j,k|psi> over one work-list chunk.
//
// part[q][row][col] = sum_{e in chunk} exp(+i k.T_e) tab[e][f] psi_q[g_e][col]
// for the chunk's functions f (orbitals, or their three gradient components),
// row = chunk.part0 * tabmult + f.  The dV factor and the sum over the chunks
// of a site are applied by the reduction kernel.  Paper: the brackets of
// Eq. occ_matrices with the Bloch phase of Fig. 1 (Sec. II).
//
// Work mapping (gfx950, 64-wide waves): blockIdx.x = chunk, blockIdx.y =
// tile of 64*CPL columns, blockIdx.z = state set.  Each lane owns CPL
// consecutive columns and reads them with one or two 16-byte loads from the
// state row of grid point g_e, so a wave reads 64*CPL contiguous columns per
// sphere entry.  Entry data (g, image, orbital values) is uniform across the
// wave.  The waves of a work-group take interleaved entries and are summed
// through LDS at the end.  Products and sums are FP64 for both storage
// precisions.

#include "kcommon.h"

namespace {

template <typename T, bool CPX, int CPL, int NF>
__device__ __forceinline__ void project_body(const ProjArgs& a, const HubChunk& C) {
    constexpr int NC = CPX ? 2 : 1;
    constexpr int NV = CPL * NC;
    constexpr int U = (NF > 9) ? 2 : 4;
    const int lane = threadIdx.x & (HUB_WAVE - 1);
    const int wave = threadIdx.x / HUB_WAVE;
    const int nw = blockDim.x / HUB_WAVE;
    const int q = blockIdx.z;
    const int col0 = (blockIdx.y * HUB_WAVE + lane) * CPL;
    const bool active = col0 < a.ncol;
    const int k = a.spinor ? q : q / a.nspin;

    const T* __restrict__ psi_q = reinterpret_cast<const T*>(a.psi) + static_cast<int64_t>(q) * a.qstride;
    const int32_t* __restrict__ gi = a.gidx + C.e0;
    const int32_t* __restrict__ im = a.img + C.e0;
    const double* __restrict__ tb = a.tab + C.phi0 * a.tabmult;
    const double* __restrict__ ph = a.phase + static_cast<int64_t>(k) * a.nimg * 2;

    double acc[NF][NV];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[f][v] = 0.0;

    for (int e = wave; e < C.ne; e += nw * U) {
        T row[U][NV];
        int idx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            idx[u] = e + u * nw;
            const int ii = (idx[u] < C.ne) ? idx[u] : e;
            const int64_t g = gi[ii];
            if (active) {
                load_vec<T, NV>(psi_q + (g * a.ld + col0) * NC, row[u]);
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) row[u][v] = T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = idx[u] < C.ne;
            const int ii = ok ? idx[u] : e;
            const double* __restrict__ w = tb + static_cast<int64_t>(ii) * NF;
            double pr = 1.0, pi = 0.0;
            if constexpr (CPX) {
                const int ig = im[ii];
                pr = ph[2 * ig];
                pi = ph[2 * ig + 1];
            }
            if (!ok) { pr = 0.0; pi = 0.0; }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double wf = w[f];
                if constexpr (CPX) {
                    const double wr = wf * pr, wi = wf * pi;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const double vr = static_cast<double>(row[u][2 * c]);
                        const double vi = static_cast<double>(row[u][2 * c + 1]);
                        acc[f][2 * c] = fma(wr, vr, fma(-wi, vi, acc[f][2 * c]));
                        acc[f][2 * c + 1] = fma(wr, vi, fma(wi, vr, acc[f][2 * c + 1]));
                    }
                } else {
                    const double wr = ok ? wf : 0.0;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) acc[f][c] = fma(wr, static_cast<double>(row[u][c]), acc[f][c]);
                }
            }
        }
    }

    // sum the waves of the work-group, one function at a time
    if (nw > 1) {
        __shared__ double red[3][HUB_WAVE][NV];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (wave > 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v) red[wave - 1][lane][v] = acc[f][v];
            }
            __syncthreads();
            if (wave == 0) {
                for (int w = 1; w < nw; ++w)
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[f][v] += red[w - 1][lane][v];
            }
            __syncthreads();
        }
    }
    if (wave != 0 || !active) return;
    double* __restrict__ out = a.part + (static_cast<int64_t>(q) * a.prows + static_cast<int64_t>(C.part0) * a.tabmult) *
                                            a.ncol * NC;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (col0 + c < a.ncol) {
#pragma unroll
                for (int r = 0; r < NC; ++r)
                    out[(static_cast<int64_t>(f) * a.ncol + col0 + c) * NC + r] = acc[f][c * NC + r];
            }
        }
    }
}

template <typename T, bool CPX, int CPL>
__global__ void __launch_bounds__(256) k_project(const ProjArgs a) {
    const HubChunk C = a.chunks[a.chunk_list[blockIdx.x]];
    switch (C.L * a.tabmult) {
    case 1: project_body<T, CPX, CPL, 1>(a, C); break;
    case 3: project_body<T, CPX, CPL, 3>(a, C); break;
    case 5: project_body<T, CPX, CPL, 5>(a, C); break;
    case 7: project_body<T, CPX, CPL, 7>(a, C); break;
    case 9: project_body<T, CPX, CPL, 9>(a, C); break;
    case 15: project_body<T, CPX, CPL, 15>(a, C); break;
    case 21: project_body<T, CPX, CPL, 21>(a, C); break;
    default: break;
    }
}

template <typename T, bool CPX, int CPL>
hipError_t launch_t(const ProjArgs& a, int nchunks, int nq, int waves, hipStream_t st) {
    const int tiles = (a.ncol + HUB_WAVE * CPL - 1) / (HUB_WAVE * CPL);
    dim3 grid(nchunks, tiles, nq);
    hipLaunchKernelGGL((k_project<T, CPX, CPL>), grid, dim3(HUB_WAVE * waves), 0, st, a);
    return hipGetLastError();
}

template <typename T, bool CPX>
hipError_t launch_c(const ProjArgs& a, int nchunks, int nq, int cpl, int waves, hipStream_t st) {
    switch (cpl) {
    case 1: return launch_t<T, CPX, 1>(a, nchunks, nq, waves, st);
    case 2: return launch_t<T, CPX, 2>(a, nchunks, nq, waves, st);
    case 4: return launch_t<T, CPX, 4>(a, nchunks, nq, waves, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_project(const ProjArgs& a, int nchunks, int nq, int prec, int cplx, int cpl, int waves,
                          hipStream_t st) {
    if (nchunks <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    if (prec == HUB_F64) {
        return cplx ? launch_c<double, true>(a, nchunks, nq, cpl, waves, st)
                    : launch_c<double, false>(a, nchunks, nq, cpl, waves, st);
    }
    return cplx ? launch_c<float, true>(a, nchunks, nq, cpl, waves, st)
                : launch_c<float, false>(a, nchunks, nq, cpl, waves, st);
}
