// Projection kernel: partial sums of <phi_j,k|psi> over one work-list chunk.
//
// part[q][row][col] = sum_{e in chunk} tab[e][f] psi_q[g_e][col]
// for the chunk's functions f (orbitals, or their three gradient components),
// row = chunk.part0 * tabmult + f.  Every entry of a chunk has the same
// lattice image (a grouped chunk: the same covering (site, image) functions),
// so the Bloch phase exp(+i k.T) of Fig. 1, the dV factor and the sum over
// the chunks of a site are applied once per chunk row by the reduction
// kernel.  Paper: the brackets of Eq. occ_matrices (Sec. II).
//
// Work mapping (gfx950, 64-wide waves): a 1-D grid of (chunk, column tile)
// work-groups, the tiles of a chunk consecutive on one XCD (hub_slot).  Each
// lane owns CPL consecutive columns of one state set and reads them with one
// or two vector loads from the state row of grid point g_e.  Two lane layouts:
//  * WIDE: every wave lies inside one state set (q is uniform), so a row
//    address is a scalar base (set, grid point) plus a 32-bit lane offset;
//  * packed: lanes tile the flattened (set, column group) space, so sets
//    narrower than a wave share one (no idle lanes, per-lane addresses).
// Entry data (g, orbital values) is uniform across the wave and comes
// through scalar loads.  Each wave of a work-group takes a contiguous range
// of the chunk's entries (so the indexes and orbital values of a batch are
// one contiguous block, read with wide scalar loads); the waves are summed
// through LDS at the end.  The entry loop is software pipelined: rows are
// loaded in batches of U into two register buffers and the loads of the next
// batch are in flight while a batch is contracted.  Products and sums are
// FP64 for both storage precisions; for complex states the real orbital
// value multiplies the real and imaginary parts (2 FMAs per column).
// Velocity gauge (GAUGE, Sec. V): each complex row value is first rotated by
// the entry's grid-point phase exp(i A.r_g); the image part exp(i A.T) of
// the field's phase is in the reduction's Bloch phase exp(i (k+A).T).
//
// This header holds the kernel templates; each storage precision is
// instantiated in a translation unit of its own.

#pragma once

#include "kcommon.h"

namespace {

template <int NV>
struct ProjLds {
    double red[3][HUB_WAVE][NV];
};

template <typename T, int NV, int NF, bool WIDE, bool GAUGE>
__device__ __forceinline__ void project_body(const ProjArgs& a, const HubChunk& C, int tile,
                                             const int32_t* __restrict__ gidx, const double* __restrict__ tab,
                                             const double* __restrict__ pg, double* __restrict__ part,
                                             ProjLds<NV>& lds) {
    constexpr int U = hub_batch_rows(NV, NF);
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
        q = tile / tps;
        col0 = ((tile - q * tps) * HUB_WAVE + lane) * cpl;
        active = col0 < a.ncol;
    } else {
        const int t = tile * HUB_WAVE + lane;
        active = t < a.nq * cg;
        q = active ? t / cg : 0;
        col0 = (t - (t / cg) * cg) * cpl;
    }
    // lanes past the last column or set read column 0 of their set (their
    // sums are discarded), so every load is unconditional
    const int colc = active ? col0 : 0;
    const T* __restrict__ psi_q = reinterpret_cast<const T*>(a.psi) + static_cast<int64_t>(q) * a.qstride;
    // this wave's entries: e0 + [lo, lo + nj) of the chunk
    int lo, nj;
    hub_wave_range(C.ne, nw, wave, lo, nj);
    const int32_t* __restrict__ gi = gidx + C.e0 + lo;
    const double* __restrict__ tb = tab + (C.phi0 * a.tabmult + static_cast<int64_t>(lo) * NF);
    const int lofs = colc * NC;                                      // lane offset inside a row

    double acc[NF][NV];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[f][v] = 0.0;

    // whole batches of U entries (chunk lengths are multiples of
    // HUB_ENTRY_ALIGN, so every wave's share is); padding entries carry zero
    // orbital values
    const int nbt = nj / U;
    // grid-point phases of a batch (velocity gauge; unused otherwise)
    // row offsets as a 32-bit index times a 32-bit stride (one scalar
    // multiply pair on the path from the index read to the row load; the
    // stride is checked at launch), phases at 32-bit byte offsets
    const uint32_t rowstride = static_cast<uint32_t>(a.ld * NC);
    auto load_batch = [&](int b, T (&r)[U][NV], double (&ph)[U][2]) {
        const int32_t* __restrict__ gb = gi + b * U;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t g = static_cast<uint32_t>(gb[u]);
            load_row_stream<T, NV>(psi_q + static_cast<uint64_t>(g) * rowstride + lofs, r[u]);
            if constexpr (GAUGE) {
                const char* __restrict__ pb =
                    reinterpret_cast<const char*>(pg) + g * static_cast<uint32_t>(2 * sizeof(double));
                ph[u][0] = *reinterpret_cast<const double*>(pb);
                ph[u][1] = *reinterpret_cast<const double*>(pb + sizeof(double));
            }
        }
    };
    auto read_tab = [&](int b, double (&w)[U][NF]) {
        const double* __restrict__ wb = tb + static_cast<int64_t>(b) * U * NF;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int f = 0; f < NF; ++f) w[u][f] = wb[u * NF + f];
    };
    auto fma_batch = [&](const double (&w)[U][NF], const T (&r)[U][NV], const double (&ph)[U][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double x[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) x[v] = static_cast<double>(r[u][v]);
            if constexpr (GAUGE) {
#pragma unroll
                for (int v = 0; v + 1 < NV; v += 2) {
                    const double xr = x[v], xi = x[v + 1];
                    x[v] = xr * ph[u][0] - xi * ph[u][1];
                    x[v + 1] = xr * ph[u][1] + xi * ph[u][0];
                }
            }
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[f][v] = fma(w[u][f], x[v], acc[f][v]);
        }
    };
    // Velocity gauge: the grid-point phases of a batch take scalar registers
    // as well, so the orbital values are read in sub-batches of at most 16
    // values, one sub-batch ahead of the one contracted (the same products
    // in the same order; measured 0.213 ms against 0.232 on the NiO-like
    // workload, where reading a whole batch's values at once spilled them).
    // Without a field the whole-batch reads below are as fast.
    constexpr int UT = [] { int t = U; while (t > 1 && t * NF > 16) t /= 2; return t; }();
    constexpr int NS = U / UT;
    auto read_sub = [&](int b, int t, double (&w)[UT][NF]) {
        const double* __restrict__ wb = tb + (static_cast<int64_t>(b) * U + t * UT) * NF;
#pragma unroll
        for (int u = 0; u < UT; ++u)
#pragma unroll
            for (int f = 0; f < NF; ++f) w[u][f] = wb[u * NF + f];
    };
    auto fma_sub = [&](int t, const double (&w)[UT][NF], const T (&r)[U][NV], const double (&ph)[U][2]) {
#pragma unroll
        for (int i = 0; i < UT; ++i) {
            const int u = t * UT + i;
            double x[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) x[v] = static_cast<double>(r[u][v]);
            if constexpr (GAUGE) {
#pragma unroll
                for (int v = 0; v + 1 < NV; v += 2) {
                    const double xr = x[v], xi = x[v + 1];
                    x[v] = xr * ph[u][0] - xi * ph[u][1];
                    x[v + 1] = xr * ph[u][1] + xi * ph[u][0];
                }
            }
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[f][v] = fma(w[i][f], x[v], acc[f][v]);
        }
    };
    auto fma_batch2 = [&](int b, const double (&w0)[UT][NF], const T (&r)[U][NV], const double (&ph)[U][2]) {
        double w[UT][NF];
#pragma unroll
        for (int u = 0; u < UT; ++u)
#pragma unroll
            for (int f = 0; f < NF; ++f) w[u][f] = w0[u][f];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            double wn[UT][NF];
            if (t + 1 < NS) read_sub(b, t + 1, wn);
            fma_sub(t, w, r, ph);
            __builtin_amdgcn_sched_barrier(0);
            if (t + 1 < NS) {
#pragma unroll
                for (int u = 0; u < UT; ++u)
#pragma unroll
                    for (int f = 0; f < NF; ++f) w[u][f] = wn[u][f];
            }
        }
    };
    if (GAUGE && nbt > 0) {
        T ra[U][NV], rb[U][NV];
        double pa[U][2], pb[U][2];
        double w[UT][NF];
        load_batch(0, ra, pa);
        int b = 0;
        for (; b + 2 <= nbt; b += 2) {
            read_sub(b, 0, w);
            load_batch(b + 1, rb, pb);
            __builtin_amdgcn_sched_barrier(0);
            fma_batch2(b, w, ra, pa);
            read_sub(b + 1, 0, w);
            load_batch(b + 2 < nbt ? b + 2 : nbt - 1, ra, pa);
            __builtin_amdgcn_sched_barrier(0);
            fma_batch2(b + 1, w, rb, pb);
        }
        if (b < nbt) {
            read_sub(b, 0, w);
            fma_batch2(b, w, ra, pa);
        }
    }
    // Two-stage pipeline with a branch-free body (a conditional use of a
    // buffer would let the compiler sink its loads next to the use); the
    // batch after the last reloads the last one, whose copy is never used.
    // A batch's orbital values are read before the next batch's indexes, so
    // the two scalar reads overlap, and the scheduling barriers keep the row
    // loads ahead of the contraction.
    if (!GAUGE && nbt > 0) {
        T ra[U][NV], rb[U][NV];
        double pa[U][2], pb[U][2];
        double w[U][NF];
        load_batch(0, ra, pa);
        int b = 0;
        for (; b + 2 <= nbt; b += 2) {
            read_tab(b, w);
            load_batch(b + 1, rb, pb);
            __builtin_amdgcn_sched_barrier(0);
            fma_batch(w, ra, pa);
            read_tab(b + 1, w);
            load_batch(b + 2 < nbt ? b + 2 : nbt - 1, ra, pa);
            __builtin_amdgcn_sched_barrier(0);
            fma_batch(w, rb, pb);
        }
        if (b < nbt) {
            read_tab(b, w);
            fma_batch(w, ra, pa);
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
    double* __restrict__ out = part + (static_cast<int64_t>(q) * a.prows + static_cast<int64_t>(C.part0) * a.tabmult) *
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

// NV = scalars per lane (columns per lane times 1 or 2); MULT the functions
// per orbital of the table (1: orbitals; 2: the orbitals of both spin
// components, spin-dependent spinor orbitals; 3: gradients or position
// moments); WIDE the lane layout; CLS the function-count class of the
// launched chunks (0: per-site chunks).
// The tables and the output are separate restrict-qualified arguments, so
// the compiler can keep the uniform table reads on scalar loads (a store
// through a pointer that may alias them would force per-lane loads).
template <typename T, int NV, int MULT, bool WIDE, int CLS, bool GAUGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(hub_waves_hint(CLS, NV))))
k_project(const ProjArgs a, const int32_t* __restrict__ gidx,
                                                 const double* __restrict__ tab, const double* __restrict__ pg,
                                                 double* __restrict__ part) {
    __shared__ ProjLds<NV> lds;
    const HubSlot slot = hub_slot(a.tiles);
    if (slot.chunk >= a.nchunks) return;
    const HubChunk C = a.chunks[a.chunk_list[slot.chunk]];
    const int tile = slot.tile;
    if constexpr (MULT > 1) {
        switch (C.L) {
        case 1: project_body<T, NV, MULT * 1, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 3: project_body<T, NV, MULT * 3, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 5: project_body<T, NV, MULT * 5, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 7: project_body<T, NV, MULT * 7, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        default: break;
        }
    } else if constexpr (CLS == 0) {
        switch (C.L) {
        case 1: project_body<T, NV, 1, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 3: project_body<T, NV, 3, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 5: project_body<T, NV, 5, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 7: project_body<T, NV, 7, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        default: break;
        }
    } else if constexpr (CLS > HUB_NCLASS) {
        // merged launch: every function count of the grouped list up to the
        // class's bound
        constexpr int NFM = hub_cls_nfmax(CLS);
#define HUB_PCASE(n)                                                                       \
    case n:                                                                                \
        if constexpr (n <= NFM) project_body<T, NV, n, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); \
        break;
        switch (C.L) {
            HUB_PCASE(1) HUB_PCASE(2) HUB_PCASE(3) HUB_PCASE(4) HUB_PCASE(5) HUB_PCASE(6) HUB_PCASE(7)
            HUB_PCASE(8) HUB_PCASE(9) HUB_PCASE(10) HUB_PCASE(11) HUB_PCASE(12) HUB_PCASE(13) HUB_PCASE(14)
            HUB_PCASE(15) HUB_PCASE(16)
        default: break;
        }
#undef HUB_PCASE
    } else {
        // grouped chunks of one class: the concatenated orbitals of the
        // covering sites
        constexpr int B = 4 * (CLS - 1);
        switch (C.L - B) {
        case 1: project_body<T, NV, B + 1, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 2: project_body<T, NV, B + 2, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 3: project_body<T, NV, B + 3, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        case 4: project_body<T, NV, B + 4, WIDE, GAUGE>(a, C, tile, gidx, tab, pg, part, lds); break;
        default: break;
        }
    }
}

// Largest function count of a class (class 0: per-site chunks, L <= 7; the
// per-site tables hold MULT functions per orbital).
constexpr int proj_nf_max(int mult, int cls) {
    return mult > 1 ? 7 * mult : hub_cls_nfmax(cls);
}

template <typename T, int NV, int MULT, int CLS, bool GAUGE>
void launch_k(const ProjArgs& b, dim3 grid, int waves, hipStream_t st) {
    if (b.wide)
        hipLaunchKernelGGL((k_project<T, NV, MULT, true, CLS, GAUGE>), grid, dim3(HUB_WAVE * waves), 0, st, b, b.gidx,
                           b.tab, b.pg, b.part);
    else
        hipLaunchKernelGGL((k_project<T, NV, MULT, false, CLS, GAUGE>), grid, dim3(HUB_WAVE * waves), 0, st, b,
                           b.gidx, b.tab, b.pg, b.part);
}

template <typename T, int NV, int MULT, int CLS>
hipError_t launch_t(const ProjArgs& a, int nchunks, int nq, int cpl, int waves, hipStream_t st) {
    // a lane's FP64 accumulators (functions x scalars) stay within 96 values
    if constexpr (proj_nf_max(MULT, CLS) * NV > (MULT == 3 ? 84 : 96)) {
        return hipErrorInvalidValue;
    } else {
        const int64_t cg = (a.ncol + cpl - 1) / cpl;
        ProjArgs b = a;
        b.nchunks = nchunks;
        b.tiles = static_cast<int>(a.wide ? static_cast<int64_t>(nq) * ((cg + HUB_WAVE - 1) / HUB_WAVE)
                                          : (static_cast<int64_t>(nq) * cg + HUB_WAVE - 1) / HUB_WAVE);
        const dim3 grid(static_cast<unsigned>(hub_slot_grid(nchunks, b.tiles)));
        if (a.pg) {
            // velocity gauge: complex states, per-site or merged chunk lists
            // (not with spin-dependent orbitals)
            if constexpr (NV % 2 == 0 && MULT != 2 && (CLS == 0 || CLS > HUB_NCLASS))
                launch_k<T, NV, MULT, CLS, true>(b, grid, waves, st);
            else
                return hipErrorInvalidValue;
        } else {
            launch_k<T, NV, MULT, CLS, false>(b, grid, waves, st);
        }
        return hipGetLastError();
    }
}

template <typename T, int MULT, int CLS>
hipError_t launch_g(const ProjArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, hipStream_t st) {
    const int nv = cpl * (cplx ? 2 : 1);
    switch (nv) {
    case 1: return launch_t<T, 1, MULT, CLS>(a, nchunks, nq, cpl, waves, st);
    case 2: return launch_t<T, 2, MULT, CLS>(a, nchunks, nq, cpl, waves, st);
    case 4: return launch_t<T, 4, MULT, CLS>(a, nchunks, nq, cpl, waves, st);
    case 8: return launch_t<T, 8, MULT, CLS>(a, nchunks, nq, cpl, waves, st);
    default: return hipErrorInvalidValue;
    }
}

// Launch the projection for storage type T (orbital or gradient table) over
// chunks of function-count class cls (HUB_MERGED8 / HUB_MERGED16: merged
// launches).
template <typename T>
hipError_t launch_project_prec(const ProjArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, int cls,
                               hipStream_t st) {
    if (nchunks <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    if (a.ld < 0 || a.ld * a.ncplx > static_cast<int64_t>(UINT32_MAX)) return hipErrorInvalidValue;
    if (a.tabmult == 3) return cls == 0 ? launch_g<T, 3, 0>(a, nchunks, nq, cplx, cpl, waves, st)
                                        : hipErrorInvalidValue;
    // spin-dependent orbitals: complex spinor states, per-site chunks
    if (a.tabmult == 2) return (cls == 0 && cplx) ? launch_g<T, 2, 0>(a, nchunks, nq, cplx, cpl, waves, st)
                                                  : hipErrorInvalidValue;
    switch (cls) {
    case 0: return launch_g<T, 1, 0>(a, nchunks, nq, cplx, cpl, waves, st);
    case 1: return launch_g<T, 1, 1>(a, nchunks, nq, cplx, cpl, waves, st);
    case 2: return launch_g<T, 1, 2>(a, nchunks, nq, cplx, cpl, waves, st);
    case 3: return launch_g<T, 1, 3>(a, nchunks, nq, cplx, cpl, waves, st);
    case 4: return launch_g<T, 1, 4>(a, nchunks, nq, cplx, cpl, waves, st);
    case HUB_MERGED8: return launch_g<T, 1, HUB_MERGED8>(a, nchunks, nq, cplx, cpl, waves, st);
    case HUB_MERGED16: return launch_g<T, 1, HUB_MERGED16>(a, nchunks, nq, cplx, cpl, waves, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
