// Projection of complex states on the grouped work list's orbitals and on
// their position moments about the site centres, in one pass over the state
// rows: the projections c and the moments rho_{a,i} of the DFT+U current of
// the velocity gauge (Sec. V).
//
// For a grouped chunk every point carries the same covers (site, image), so
// the displacement of a point from the centre of cover k is its displacement
// d0 from the chunk's first cover plus a constant offset D_k.  The kernel
// sums, per function f and column,
//   acc_0 = sum_e phi_f(e) x(e),   acc_i = sum_e phi_f(e) d0_i(e) x(e)
// (x the state value at the entry's point, rotated by the grid-point phase
// under a field) and writes acc_0 and acc_i + D_k(f),i acc_0, the moment
// about the function's own site, into four planes of the workspace; the
// grouped reduction then applies dV and the Bloch phases to all four.
//
// Work mapping: a 1-D grid of one-wave work-groups over (item, column tile)
// (hub_slot); an item is one half of a chunk's functions (functions
// 8h..8h+7), each lane owns one complex column of one state set (64 columns
// per wave).  The host orders the items by their cost (entries times the
// instructions per entry), longest first, so that short items fill the end
// of the launch.  Per entry a wave does 4 x 2 x NFW FP64 FMAs on one row
// value, its conversion and (under a field) its phase rotation: the orbital
// and moment components share the row's load and preparation.

#pragma once

#include "kcommon.h"

namespace {

// Functions per wave: 8 (4 x 8 x 2 FP64 accumulators, three waves per
// SIMD) measured faster than 6 or 4, and than items of at most 5 functions
// (four waves per SIMD, 424 us against 385 on the NiO-like workload): more
// waves per SIMD, but each point's load and preparation repeated by more
// waves; rows per batch: 4 (8 spills scalar registers and leaves two waves
// per SIMD).
constexpr int MOM_NFW = HUB_MOM_NFW;
static_assert(2 * MOM_NFW >= HUB_GF_MAX, "two halves cover a chunk's functions");
constexpr int MOM_U = 4;

template <typename T, int NFW, bool GAUGE>
__device__ __forceinline__ void mom_body(const ProjArgs& a, const HubChunk& C, int ci, int f0, int q, int col,
                                         bool active, const int32_t* __restrict__ gidx,
                                         const double* __restrict__ tab, const double* __restrict__ d0,
                                         const double* __restrict__ fdel, const double* __restrict__ pg,
                                         double* __restrict__ part) {
    constexpr int U = MOM_U;
    const int NF = C.L;
    const int colc = active ? col : 0;
    const T* __restrict__ psi_q = reinterpret_cast<const T*>(a.psi) + static_cast<int64_t>(q) * a.qstride;
    const int32_t* __restrict__ gi = gidx + C.e0;
    const double* __restrict__ tb = tab + C.phi0 + f0;          // entry e: tb[e * NF + f]
    const double* __restrict__ dp = d0 + 3 * static_cast<int64_t>(C.e0);
    const uint32_t rowstride = static_cast<uint32_t>(a.ld * 2);   // elements (checked at launch)

    double acc[4][NFW][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int f = 0; f < NFW; ++f) acc[i][f][0] = acc[i][f][1] = 0.0;

    // per-entry uniform data: the orbital values of the wave's functions and
    // the displacement d0
    struct Ent {
        double w[NFW];
        double d[3];
    };
    // read at 32-bit byte offsets from the chunk's table and displacement
    // rows (a chunk's are far below 4 GiB), advanced entry by entry; the
    // offsets stop at the last entry, so the read after it repeats it
    const uint32_t wstep = static_cast<uint32_t>(NF) * sizeof(double);
    const uint32_t wlast = static_cast<uint32_t>(C.ne - 1) * wstep;
    const uint32_t dlast = static_cast<uint32_t>(C.ne - 1) * (3 * sizeof(double));
    uint32_t wnext = 0, dnext = 0;
    auto read_next = [&](Ent& x) {
        const char* __restrict__ wb = reinterpret_cast<const char*>(tb) + wnext;
        const char* __restrict__ db = reinterpret_cast<const char*>(dp) + dnext;
#pragma unroll
        for (int f = 0; f < NFW; ++f) x.w[f] = *reinterpret_cast<const double*>(wb + f * sizeof(double));
#pragma unroll
        for (int i = 0; i < 3; ++i) x.d[i] = *reinterpret_cast<const double*>(db + i * sizeof(double));
        wnext = min(wnext + wstep, wlast);
        dnext = min(dnext + static_cast<uint32_t>(3 * sizeof(double)), dlast);
    };
    // grid points of batch b (read one batch before their rows are loaded)
    auto read_idx = [&](int b, int (&g)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = gi[b * U + u];
    };
    auto load_batch = [&](const int (&gg)[U], T (&r)[U][2], double (&ph)[U][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = gg[u];
            load_row_stream<T, 2>(psi_q + static_cast<uint64_t>(static_cast<uint32_t>(g)) * rowstride + 2 * colc,
                                  r[u]);
            if constexpr (GAUGE) {
                const char* __restrict__ pb = reinterpret_cast<const char*>(pg) +
                                              static_cast<uint32_t>(g) * static_cast<uint32_t>(2 * sizeof(double));
                ph[u][0] = *reinterpret_cast<const double*>(pb);
                ph[u][1] = *reinterpret_cast<const double*>(pb + sizeof(double));
            }
        }
    };
    auto fma_entry = [&](const Ent& x, const T (&r)[2], const double (&ph)[2]) {
        double v0 = static_cast<double>(r[0]), v1 = static_cast<double>(r[1]);
        if constexpr (GAUGE) {
            const double t0 = v0 * ph[0] - v1 * ph[1];
            v1 = v0 * ph[1] + v1 * ph[0];
            v0 = t0;
        }
        double z[3][2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            z[i][0] = x.d[i] * v0;
            z[i][1] = x.d[i] * v1;
        }
#pragma unroll
        for (int f = 0; f < NFW; ++f) {
            acc[0][f][0] = fma(x.w[f], v0, acc[0][f][0]);
            acc[0][f][1] = fma(x.w[f], v1, acc[0][f][1]);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                acc[i + 1][f][0] = fma(x.w[f], z[i][0], acc[i + 1][f][0]);
                acc[i + 1][f][1] = fma(x.w[f], z[i][1], acc[i + 1][f][1]);
            }
        }
    };
    // Contract a batch entry by entry; the uniform data of the next entry is
    // read while the current one is contracted (the scheduling barriers keep
    // those reads from being hoisted together).  The entry after the last
    // re-reads the last one.
    auto fma_batch = [&](Ent& cur, const T (&r)[U][2], const double (&ph)[U][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            Ent nx;
            read_next(nx);
            fma_entry(cur, r[u], ph[u]);
            __builtin_amdgcn_sched_barrier(0);
            cur = nx;
        }
    };
    // Two row buffers; the grid points of a batch are read one batch ahead
    // of its row loads, and the batches past the last re-read the last one.
    const int nbt = C.ne / U;
    if (nbt > 0) {
        T ra[U][2], rb[U][2];
        double pa[U][2], pb[U][2];
        int ga[U], gb[U];
        Ent cur;
        read_idx(0, ga);
        read_next(cur);
        load_batch(ga, ra, pa);
        read_idx(nbt > 1 ? 1 : 0, gb);
        int b = 0;
        for (; b + 2 <= nbt; b += 2) {
            load_batch(gb, rb, pb);
            read_idx(b + 2 < nbt ? b + 2 : nbt - 1, ga);
            __builtin_amdgcn_sched_barrier(0);
            fma_batch(cur, ra, pa);
            load_batch(ga, ra, pa);
            read_idx(b + 3 < nbt ? b + 3 : nbt - 1, gb);
            __builtin_amdgcn_sched_barrier(0);
            fma_batch(cur, rb, pb);
        }
        if (b < nbt) fma_batch(cur, ra, pa);
    }
    if (!active) return;
    const double* __restrict__ del = fdel + (static_cast<int64_t>(ci) * HUB_GF_MAX + f0) * 3;
#pragma unroll
    for (int f = 0; f < NFW; ++f) {
        const int64_t o = ((static_cast<int64_t>(q) * a.prows + C.part0 + f0 + f) * a.ncol + col) * 2;
        part[o] = acc[0][f][0];
        part[o + 1] = acc[0][f][1];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double D = del[3 * f + i];
            part[(i + 1) * a.pplane + o] = fma(D, acc[0][f][0], acc[i + 1][f][0]);
            part[(i + 1) * a.pplane + o + 1] = fma(D, acc[0][f][1], acc[i + 1][f][1]);
        }
    }
}

template <typename T, bool GAUGE>
__global__ void __launch_bounds__(HUB_WAVE)
k_project_mom(const ProjArgs a, const int32_t* __restrict__ gidx, const double* __restrict__ tab,
              const double* __restrict__ d0, const double* __restrict__ fdel, const double* __restrict__ pg,
              double* __restrict__ part) {
    const HubSlot slot = hub_slot(a.tiles);
    if (slot.chunk >= a.nchunks) return;
    const int item = a.chunk_list[slot.chunk];
    const int ci = item >> 1;
    const HubChunk C = a.chunks[ci];
    const int lane = threadIdx.x;
    const int f0 = (item & 1) * MOM_NFW;
    const int nfw = C.L - f0 < MOM_NFW ? C.L - f0 : MOM_NFW;
    if (nfw <= 0) return;
    const int tps = (a.ncol + HUB_WAVE - 1) / HUB_WAVE;     // column tiles per state set
    const int q = slot.tile / tps;
    const int col = (slot.tile - q * tps) * HUB_WAVE + lane;
    const bool active = col < a.ncol;
#define HUB_MCASE(n) \
    case n: mom_body<T, n, GAUGE>(a, C, ci, f0, q, col, active, gidx, tab, d0, fdel, pg, part); break;
    static_assert(MOM_NFW == 8, "the cases below cover 1..8 functions");
    switch (nfw) {
        HUB_MCASE(1) HUB_MCASE(2) HUB_MCASE(3) HUB_MCASE(4) HUB_MCASE(5) HUB_MCASE(6) HUB_MCASE(7) HUB_MCASE(8)
    default: break;
    }
#undef HUB_MCASE
}

// Launch over nitems work items of grouped chunks (every pass, functions
// <= 16 per chunk) of complex states of storage type T.
template <typename T>
hipError_t launch_project_mom_prec(const ProjArgs& a, int nitems, int nq, hipStream_t st) {
    if (nitems <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    if (a.ncplx != 2 || !a.d0 || !a.fdel || a.ld < 0 || a.ld * 2 > static_cast<int64_t>(UINT32_MAX))
        return hipErrorInvalidValue;
    ProjArgs b = a;
    b.nchunks = nitems;
    b.tiles = static_cast<int>(static_cast<int64_t>(nq) * ((a.ncol + HUB_WAVE - 1) / HUB_WAVE));
    const dim3 grid(static_cast<unsigned>(hub_slot_grid(nitems, b.tiles)));
    if (a.pg)
        hipLaunchKernelGGL((k_project_mom<T, true>), grid, dim3(HUB_WAVE), 0, st, b, b.gidx, b.tab, b.d0, b.fdel,
                           b.pg, b.part);
    else
        hipLaunchKernelGGL((k_project_mom<T, false>), grid, dim3(HUB_WAVE), 0, st, b, b.gidx, b.tab, b.d0, b.fdel,
                           b.pg, b.part);
    return hipGetLastError();
}

}  // namespace
