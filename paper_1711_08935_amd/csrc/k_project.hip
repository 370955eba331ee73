// Projection kernel: partial sums of <phi_j,k|psi> over one work-list chunk.
//
// part[q][row][col] = sum_{e in chunk} tab[e][f] psi_q[g_e][col]
// for the chunk's functions f (orbitals, or their three gradient components),
// row = chunk.part0 * tabmult + f.  Every entry of a chunk has the same
// lattice image, so the Bloch phase exp(+i k.T) of Fig. 1, the dV factor
// and the sum over the chunks of a site are applied once per chunk by the
// reduction kernel.  Paper: the brackets of Eq. occ_matrices (Sec. II).
//
// Work mapping (gfx950, 64-wide waves): blockIdx.x = chunk, blockIdx.y =
// column tile.  Each lane owns CPL consecutive columns of one state set and
// reads them with one or two vector loads from the state row of grid point
// g_e.  Two lane layouts:
//  * WIDE: every wave lies inside one state set (q is uniform), so a row
//    address is a scalar base (set, grid point) plus a 32-bit lane offset;
//  * packed: lanes tile the flattened (set, column group) space, so sets
//    narrower than a wave share one (no idle lanes, per-lane addresses).
// Entry data (g, orbital values) is uniform across the wave and comes
// through scalar loads.  The waves of a work-group take interleaved entries
// and are summed through LDS at the end; the unrolled main loop issues U row
// loads back to back, a remainder loop takes the last entries.  Products and
// sums are FP64 for both storage precisions; for complex states the real
// orbital value multiplies the real and imaginary parts (2 FMAs per column).

#include "kcommon.h"

namespace {

template <int NV>
struct ProjLds {
    double red[3][HUB_WAVE][NV];
};

template <typename T, int NV, int NF, bool WIDE>
__device__ __forceinline__ void project_body(const ProjArgs& a, const HubChunk& C, ProjLds<NV>& lds) {
    constexpr int U = (NF > 9) ? 2 : ((NF > 5) ? 4 : 8);
    const int lane = threadIdx.x & (HUB_WAVE - 1);
    // wave index made provably uniform so entry data goes through scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / HUB_WAVE);
    const int nw = blockDim.x / HUB_WAVE;
    const int NC = a.ncplx;
    const int cpl = NV / NC;
    const int cg = (a.ncol + cpl - 1) / cpl;

    int q, col0;
    bool active;
    if constexpr (WIDE) {
        const int tps = (cg + HUB_WAVE - 1) / HUB_WAVE;          // tiles per set
        q = blockIdx.y / tps;
        col0 = ((blockIdx.y - q * tps) * HUB_WAVE + lane) * cpl;
        active = col0 < a.ncol;
    } else {
        const int t = blockIdx.y * HUB_WAVE + lane;
        active = t < a.nq * cg;
        q = active ? t / cg : 0;
        col0 = (t - (t / cg) * cg) * cpl;
    }
    // lanes past the last column or set read column 0 of their set (their
    // sums are discarded), so every load is unconditional
    const int colc = active ? col0 : 0;
    const T* __restrict__ psi_q = reinterpret_cast<const T*>(a.psi) + static_cast<int64_t>(q) * a.qstride;
    const int32_t* __restrict__ gi = a.gidx + C.e0;
    const double* __restrict__ tb = a.tab + C.phi0 * a.tabmult;
    const int lofs = colc * NC;                                      // lane offset inside a row

    double acc[NF][NV];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[f][v] = 0.0;

    // entries of this wave: wave, wave + nw, ...
    const int nj = (C.ne - wave + nw - 1) / nw;
    int j = 0;
    for (; j + U <= nj; j += U) {
        T row[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t g = gi[wave + (j + u) * nw];
            load_row<T, NV>(psi_q + g * a.ld * NC + lofs, row[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double* __restrict__ w = tb + static_cast<int64_t>(wave + (j + u) * nw) * NF;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double wf = w[f];
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[f][v] = fma(wf, static_cast<double>(row[u][v]), acc[f][v]);
            }
        }
    }
    for (; j < nj; ++j) {
        T row[NV];
        const int e = wave + j * nw;
        const int64_t g = gi[e];
        load_row<T, NV>(psi_q + g * a.ld * NC + lofs, row);
        const double* __restrict__ w = tb + static_cast<int64_t>(e) * NF;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double wf = w[f];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[f][v] = fma(wf, static_cast<double>(row[v]), acc[f][v]);
        }
    }

    // sum the waves of the work-group, one function at a time
    if (nw > 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (wave > 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v) lds.red[wave - 1][lane][v] = acc[f][v];
            }
            __syncthreads();
            if (wave == 0) {
                for (int w = 1; w < nw; ++w)
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[f][v] += lds.red[w - 1][lane][v];
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
        for (int v = 0; v < NV; ++v) {
            const int col = col0 + v / NC;
            if (col < a.ncol) out[(static_cast<int64_t>(f) * a.ncol + col0) * NC + v] = acc[f][v];
        }
    }
}

// NV = scalars per lane (columns per lane times 1 or 2); GRAD selects the
// gradient table (three functions per orbital); WIDE the lane layout.
template <typename T, int NV, bool GRAD, bool WIDE>
__global__ void __launch_bounds__(256) k_project(const ProjArgs a) {
    __shared__ ProjLds<NV> lds;
    const HubChunk C = a.chunks[a.chunk_list[blockIdx.x]];
    if constexpr (!GRAD) {
        // per-site chunks carry L in {1,3,5,7}; grouped chunks carry the
        // concatenated orbitals of their covering sites (up to HUB_GF_MAX)
#define HUB_PCASE(n)                                                  \
    case n:                                                           \
        if constexpr (n * NV <= 96) project_body<T, NV, n, WIDE>(a, C, lds); \
        break;
        switch (C.L) {
            HUB_PCASE(1) HUB_PCASE(2) HUB_PCASE(3) HUB_PCASE(4) HUB_PCASE(5) HUB_PCASE(6) HUB_PCASE(7)
            HUB_PCASE(8) HUB_PCASE(9) HUB_PCASE(10) HUB_PCASE(11) HUB_PCASE(12) HUB_PCASE(13)
            HUB_PCASE(14) HUB_PCASE(15) HUB_PCASE(16)
        default: break;
        }
#undef HUB_PCASE
    } else {
        switch (C.L) {
        case 1: project_body<T, NV, 3, WIDE>(a, C, lds); break;
        case 3: project_body<T, NV, 9, WIDE>(a, C, lds); break;
        case 5: project_body<T, NV, 15, WIDE>(a, C, lds); break;
        case 7: project_body<T, NV, 21, WIDE>(a, C, lds); break;
        default: break;
        }
    }
}

template <typename T, int NV, bool GRAD>
hipError_t launch_t(const ProjArgs& a, int nchunks, int nq, int cpl, int waves, hipStream_t st) {
    const int64_t cg = (a.ncol + cpl - 1) / cpl;
    if (a.wide) {
        const int64_t tiles = static_cast<int64_t>(nq) * ((cg + HUB_WAVE - 1) / HUB_WAVE);
        hipLaunchKernelGGL((k_project<T, NV, GRAD, true>), dim3(nchunks, static_cast<unsigned>(tiles), 1),
                           dim3(HUB_WAVE * waves), 0, st, a);
    } else {
        const int64_t tiles = (static_cast<int64_t>(nq) * cg + HUB_WAVE - 1) / HUB_WAVE;
        hipLaunchKernelGGL((k_project<T, NV, GRAD, false>), dim3(nchunks, static_cast<unsigned>(tiles), 1),
                           dim3(HUB_WAVE * waves), 0, st, a);
    }
    return hipGetLastError();
}

template <typename T, bool GRAD>
hipError_t launch_g(const ProjArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, hipStream_t st) {
    const int nv = cpl * (cplx ? 2 : 1);
    switch (nv) {
    case 1: return launch_t<T, 1, GRAD>(a, nchunks, nq, cpl, waves, st);
    case 2: return launch_t<T, 2, GRAD>(a, nchunks, nq, cpl, waves, st);
    case 4: return launch_t<T, 4, GRAD>(a, nchunks, nq, cpl, waves, st);
    case 8:
        if constexpr (!GRAD) return launch_t<T, 8, GRAD>(a, nchunks, nq, cpl, waves, st);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_project(const ProjArgs& a, int nchunks, int nq, int prec, int cplx, int cpl, int waves,
                          hipStream_t st) {
    if (nchunks <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    const bool grad = a.tabmult == 3;
    if (prec == HUB_F64) {
        return grad ? launch_g<double, true>(a, nchunks, nq, cplx, cpl, waves, st)
                    : launch_g<double, false>(a, nchunks, nq, cplx, cpl, waves, st);
    }
    return grad ? launch_g<float, true>(a, nchunks, nq, cplx, cpl, waves, st)
                : launch_g<float, false>(a, nchunks, nq, cplx, cpl, waves, st);
}
