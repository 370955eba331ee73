// Apply kernel: hpsi_q[g][col] += alpha * scale * (V_U psi)_q[g][col] for the
// entries of one work-list chunk (Eq. pot_V_U).
//
// Per lane and column: B_a = sum_b V_ab c_b with V_ab = Ueff (delta_ab/2 -
// n_ba) of the function's site and spin channel (spinor: B^s_a = sum_{s' b}
// V^{ss'}_ab c^{s'}_b, V^{ss'}_ab = Ueff (delta delta / 2 - n^{s's}_ba)); the
// transpose follows from differentiating E_U (Eq. minimization).  Then for
// every sphere entry e of the chunk:
//   hpsi[g_e][col] += sum_f phi_f(e) exp(-i k.T_f) B_f(col),
// where the image T_f of function f is the same for every entry of a chunk,
// so its phase is folded into B_f once per chunk.
// The host groups entries in layers that never repeat a grid point and
// launches one layer at a time (or, with the grouped work list, puts every
// grid point in one chunk per pass with the covering functions of that pass
// and launches the passes one at a time), so no two lanes in flight update
// the same element: no atomics, deterministic results.
// Sums are FP64; the updated element is rounded once to the storage type.
// Velocity gauge (GAUGE, Sec. V): the entry's update is rotated by the
// conjugate grid-point phase exp(-i A.r_g); the image part of the field's
// phase is in the coefficients' Bloch phase exp(-i (k+A).T).
//
// Work mapping: a 1-D grid of (chunk, column tile) work-groups, the tiles of
// a chunk consecutive on one XCD (hub_slot), with the same two lane layouts
// as the projection (WIDE: one state set per wave; packed:
// narrow sets share a wave).  Every wave of a work-group serves the same
// columns, so the waves split the chunk's functions, compute B_f for their
// lanes and exchange it through LDS; then each wave takes a contiguous range
// of the chunk's entries.  The entry loop is software pipelined like the
// projection's: the rows of the next batch are loaded while the current
// batch is updated and stored.
//
// This header holds the kernel templates; each storage precision and work
// list is instantiated in a translation unit of its own.

#pragma once

#include "kcommon.h"

namespace {

// B of one function (orbital ai of a site, seen through lattice image img)
// for the CPL columns col0.. of state set q:
// B = alpha scale exp(-i k.T_img) sum_b V_{ai b} c_b (spinor: with the spin
// blocks).  Columns past ncol get B = 0, and so do spinor columns of the
// other spin component when the function is the orbital of component sgf
// (spin-dependent orbitals; sgf < 0: both components).
template <bool CPX, bool SPINOR, int CPL>
__device__ __forceinline__ void coefficient(const ApplyArgs& a, int site, int ai, int img, int q, int col0,
                                            double (&Bf)[CPL * (CPX ? 2 : 1)], int sgf = -1) {
    constexpr int NC = CPX ? 2 : 1;
    // q counts the launch's state sets; q0 + q is the context's set (k-point, spin)
    const int ch = SPINOR ? 0 : ((a.q0 + q) % a.nspin);
    const int k = a.spinor ? a.q0 + q : (a.q0 + q) / a.nspin;
    const int o0 = a.site_orb0[site];
    const int L = a.site_L[site];
    const double U = a.ueff[site];
    const double* __restrict__ nb = a.n + static_cast<int64_t>(site) * a.nblk * 98;
    const double* __restrict__ cq = a.c + (static_cast<int64_t>(q) * a.J + o0) * a.ncol * NC;
    double pr = 1.0, pi = 0.0;
    if constexpr (CPX) {
        pr = a.phase[(static_cast<int64_t>(k) * a.nimg + img) * 2];
        pi = -a.phase[(static_cast<int64_t>(k) * a.nimg + img) * 2 + 1];
    }
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
        const int col = col0 + cc;
        const bool ok = col < a.ncol;
        double sc = a.alpha;
        if (a.colscale != nullptr && ok) {
            const int s = SPINOR ? (col >> 1) : col;
            sc *= a.colscale[static_cast<int64_t>(q) * a.nstates + s];
        }
        if (a.occ != nullptr && ok) {
            // w_k f_s of the column's state (gradient of E_U, Eq. minimization)
            const int s = SPINOR ? (col >> 1) : col;
            sc *= a.kw[k] * a.occ[static_cast<int64_t>(a.q0 + q) * a.nstates + s];
        }
        if (!ok || (sgf >= 0 && (col & 1) != sgf)) sc = 0.0;
        const int colc = ok ? col : 0;
        double br = 0.0, bi = 0.0;
        if constexpr (!SPINOR) {
            const double* __restrict__ nm = nb + ch * 98;
#pragma unroll 1
            for (int b = 0; b < L; ++b) {
                // V_ab = U (delta_ab / 2 - n_ba)
                const double vr = U * ((ai == b ? 0.5 : 0.0) - nm[(b * 7 + ai) * 2]);
                const double cr = cq[(static_cast<int64_t>(b) * a.ncol + colc) * NC];
                if constexpr (CPX) {
                    const double vi = -U * nm[(b * 7 + ai) * 2 + 1];
                    const double ci = cq[(static_cast<int64_t>(b) * a.ncol + colc) * NC + 1];
                    br = fma(vr, cr, fma(-vi, ci, br));
                    bi = fma(vr, ci, fma(vi, cr, bi));
                } else {
                    br = fma(vr, cr, br);
                }
            }
        } else {
            // spinor columns 2s + sigma; V^{sigma sigma'}_ab = U (dd/2 - n^{sigma' sigma}_ba)
            const int sg = colc & 1;
            const int base = colc - sg;
#pragma unroll 1
            for (int t = 0; t < 2; ++t) {
                const double* __restrict__ nm = nb + (2 * t + sg) * 98;   // block (sigma' = t, sigma = sg)
#pragma unroll 1
                for (int b = 0; b < L; ++b) {
                    const double vr = U * ((ai == b && t == sg) ? 0.5 : 0.0) - U * nm[(b * 7 + ai) * 2];
                    const double vi = -U * nm[(b * 7 + ai) * 2 + 1];
                    const double cr = cq[(static_cast<int64_t>(b) * a.ncol + base + t) * 2];
                    const double ci = cq[(static_cast<int64_t>(b) * a.ncol + base + t) * 2 + 1];
                    br = fma(vr, cr, fma(-vi, ci, br));
                    bi = fma(vr, ci, fma(vi, cr, bi));
                }
            }
        }
        br *= sc;
        bi *= sc;
        if constexpr (CPX) {
            Bf[2 * cc] = pr * br - pi * bi;
            Bf[2 * cc + 1] = pr * bi + pi * br;
        } else {
            Bf[cc] = br;
        }
    }
}

// Bs: LDS of the work-group, at least L * NV * HUB_WAVE doubles.
// chunk: the chunk's index in the work-group's launch list; tile: column tile.
// L: functions per entry; SPINDEP: per-site chunks of spin-dependent orbitals,
// function sigma * (L/2) + m is orbital m of spin component sigma, whose
// coefficient is nonzero only in that component's columns.
template <typename T, bool CPX, bool SPINOR, int CPL, int L, bool WIDE, bool GROUPED, bool GAUGE,
          bool SPINDEP = false>
__device__ __forceinline__ void apply_body(const ApplyArgs& a, const HubChunk& C, int chunk_slot, int tile,
                                           const int32_t* __restrict__ gidx, const double* __restrict__ tab,
                                           const double* __restrict__ pg, T* __restrict__ hpsi, double* Bs) {
    constexpr int NC = CPX ? 2 : 1;
    constexpr int NV = CPL * NC;
    constexpr int U = hub_batch_rows(NV, L);
    const int lane = threadIdx.x & (HUB_WAVE - 1);
    // wave index made provably uniform so entry data goes through scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / HUB_WAVE);
    const int nw = blockDim.x / HUB_WAVE;
    const int cg = (a.ncol + CPL - 1) / CPL;
    int q, col0;
    bool active;
    if constexpr (WIDE) {
        const int tps = (cg + HUB_WAVE - 1) / HUB_WAVE;          // tiles per set (q uniform)
        q = tile / tps;
        col0 = ((tile - q * tps) * HUB_WAVE + lane) * CPL;
        active = col0 < a.ncol;
    } else {
        const int t = tile * HUB_WAVE + lane;
        active = t < a.nq * cg;
        q = active ? t / cg : 0;
        col0 = active ? (t - q * cg) * CPL : 0;
    }

    // coefficients: the waves split the functions (lanes past the last
    // column compute zeros for column 0 of their set and are then idle)
    for (int f = wave; f < L; f += nw) {
        int site, ai, img;
        int sgf = -1;
        if constexpr (GROUPED) {
            const int chunk = a.chunk_list[chunk_slot];
            int j = a.f_orb[chunk * HUB_GF_MAX + f];
            if (a.spindep) {
                // function of the spin component sgf's orbital j (stored as j + sgf J)
                sgf = j >= a.J ? 1 : 0;
                j -= sgf * a.J;
            }
            img = a.f_img[chunk * HUB_GF_MAX + f];
            site = a.orb_site[j];
            ai = j - a.site_orb0[site];
        } else {
            site = C.site;
            ai = SPINDEP ? f % C.L : f;
            img = C.img;
        }
        double Bf[NV];
        if constexpr (SPINDEP) sgf = f / C.L;
        coefficient<CPX, SPINOR, CPL>(a, site, ai, img, q, active ? col0 : a.ncol, Bf, sgf);
#pragma unroll
        for (int v = 0; v < NV; ++v) Bs[(f * NV + v) * HUB_WAVE + lane] = Bf[v];
    }
    __syncthreads();
    if (!active) return;
    double B[L][NV];
#pragma unroll
    for (int f = 0; f < L; ++f)
#pragma unroll
        for (int v = 0; v < NV; ++v) B[f][v] = Bs[(f * NV + v) * HUB_WAVE + lane];

    T* __restrict__ h_q = hpsi + static_cast<int64_t>(q) * a.qstride;
    // this wave's entries: e0 + [lo, lo + nj) of the chunk
    int lo, nj;
    hub_wave_range(C.ne, nw, wave, lo, nj);
    const int32_t* __restrict__ gi = gidx + C.e0 + lo;
    const double* __restrict__ tb = tab + (C.phi0 * (SPINDEP ? 2 : 1) + static_cast<int64_t>(lo) * L);
    const int lofs = col0 * NC;

    // whole batches of U entries (chunk lengths are multiples of
    // HUB_ENTRY_ALIGN, so every wave's share is); padding entries (from
    // nreal on) read and write the sink row instead of a state row
    const int nbt = nj / U;
    const int nreal = C.nreal - lo;                                  // real entries of this wave
    T* __restrict__ sink = reinterpret_cast<T*>(a.sink) + lofs;
    auto row_ptr = [&](int j, int32_t g) {
        return j < nreal ? h_q + static_cast<int64_t>(g) * a.ld * NC + lofs : sink;
    };
    T* rp[2][U];                                                     // row addresses of the two buffers
    // grid-point phases of a batch (velocity gauge; unused otherwise)
    double ph[2][U][2];
    auto load_batch = [&](int b, T (&r)[U][NV], T* (&p)[U], double (&phb)[U][2]) {
        const int32_t* __restrict__ gb = gi + b * U;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            p[u] = row_ptr(b * U + u, gb[u]);
            load_row<T, NV>(p[u], r[u]);
            if constexpr (GAUGE) {
                phb[u][0] = pg[2 * static_cast<int64_t>(gb[u])];
                phb[u][1] = pg[2 * static_cast<int64_t>(gb[u]) + 1];
            }
        }
    };
    auto read_tab = [&](int b, double (&w)[U][L]) {
        const double* __restrict__ wb = tb + static_cast<int64_t>(b) * U * L;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int ai = 0; ai < L; ++ai) w[u][ai] = wb[u * L + ai];
    };
    auto update_batch = [&](const double (&w)[U][L], const T (&r)[U][NV], T* const (&p)[U],
                            const double (&phb)[U][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double add[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) add[v] = 0.0;
#pragma unroll
            for (int ai = 0; ai < L; ++ai)
#pragma unroll
                for (int v = 0; v < NV; ++v) add[v] = fma(w[u][ai], B[ai][v], add[v]);
            if constexpr (GAUGE) {
#pragma unroll
                for (int v = 0; v + 1 < NV; v += 2) {
                    const double xr = add[v], xi = add[v + 1];
                    add[v] = xr * phb[u][0] + xi * phb[u][1];
                    add[v + 1] = xi * phb[u][0] - xr * phb[u][1];
                }
            }
            T out[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = static_cast<T>(static_cast<double>(r[u][v]) + add[v]);
            store_row<T, NV>(p[u], out);
        }
    };
    // Two-stage pipeline with a branch-free body; the batch after the last
    // reloads the last one (before its stores), and that copy is never used.
    // A batch's orbital values are read before the next batch's indexes, and
    // the scheduling barriers keep the row loads ahead of the updates.
    if (nbt > 0) {
        T ra[U][NV], rb[U][NV];
        double w[U][L];
        load_batch(0, ra, rp[0], ph[0]);
        int b = 0;
        for (; b + 2 <= nbt; b += 2) {
            read_tab(b, w);
            load_batch(b + 1, rb, rp[1], ph[1]);
            __builtin_amdgcn_sched_barrier(0);
            update_batch(w, ra, rp[0], ph[0]);
            read_tab(b + 1, w);
            load_batch(b + 2 < nbt ? b + 2 : nbt - 1, ra, rp[0], ph[0]);
            __builtin_amdgcn_sched_barrier(0);
            update_batch(w, rb, rp[1], ph[1]);
        }
        if (b < nbt) {
            read_tab(b, w);
            update_batch(w, ra, rp[0], ph[0]);
        }
    }
}

// The sphere tables and the output are separate restrict-qualified kernel
// arguments: the stores into hpsi inside the entry loop then cannot alias the
// table reads, and the uniform entry data stays on scalar loads.
template <typename T, bool CPX, bool SPINOR, int CPL, bool WIDE, bool GAUGE, bool SPINDEP = false>
__global__ void __launch_bounds__(256) k_apply(const ApplyArgs a, const int32_t* __restrict__ gidx,
                                               const double* __restrict__ tab, const double* __restrict__ pg,
                                               T* __restrict__ hpsi) {
    constexpr int NV = CPL * (CPX ? 2 : 1);
    constexpr int M = SPINDEP ? 2 : 1;
    __shared__ double Bs[7 * M * NV * HUB_WAVE];
    const HubSlot slot = hub_slot(a.tiles);
    if (slot.chunk >= a.nchunks) return;
    const HubChunk C = a.chunks[a.chunk_list[slot.chunk]];
    switch (C.L) {
#define HUB_PCALL(n) \
    apply_body<T, CPX, SPINOR, CPL, M * n, WIDE, false, GAUGE, SPINDEP>(a, C, slot.chunk, slot.tile, gidx, tab, pg, \
                                                                        hpsi, Bs)
    case 1: HUB_PCALL(1); break;
    case 3: HUB_PCALL(3); break;
    case 5: HUB_PCALL(5); break;
    case 7: HUB_PCALL(7); break;
#undef HUB_PCALL
    default: break;
    }
}

// Grouped chunks: L is the number of concatenated functions of the chunk's
// covering sites, 4(CLS-1) < L <= 4 CLS; every grid point lies in one chunk,
// so the launches of the classes write disjoint points.
// CLS > HUB_NCLASS: merged launch over every function count up to
// hub_cls_nfmax(CLS).
template <typename T, bool CPX, bool SPINOR, int CPL, bool WIDE, int CLS, bool GAUGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(hub_waves_hint(CLS, CPL * (CPX ? 2 : 1)))))
k_apply_grouped(const ApplyArgs a, const int32_t* __restrict__ gidx,
                                                       const double* __restrict__ tab, const double* __restrict__ pg,
                                                       T* __restrict__ hpsi) {
    constexpr int NV = CPL * (CPX ? 2 : 1);
    constexpr int NFMAX = hub_cls_nfmax(CLS);
    __shared__ double Bs[NFMAX * NV * HUB_WAVE];
    const HubSlot slot = hub_slot(a.tiles);
    if (slot.chunk >= a.nchunks) return;
    const HubChunk C = a.chunks[a.chunk_list[slot.chunk]];
#define HUB_ACALL(n) \
    apply_body<T, CPX, SPINOR, CPL, (n), WIDE, true, GAUGE>(a, C, slot.chunk, slot.tile, gidx, tab, pg, hpsi, Bs)
#define HUB_ACASE(n)                      \
    case n:                               \
        if constexpr (n <= NFMAX) HUB_ACALL(n); \
        break;
    if constexpr (CLS > HUB_NCLASS) {
        switch (C.L) {
            HUB_ACASE(1) HUB_ACASE(2) HUB_ACASE(3) HUB_ACASE(4) HUB_ACASE(5) HUB_ACASE(6) HUB_ACASE(7)
            HUB_ACASE(8) HUB_ACASE(9) HUB_ACASE(10) HUB_ACASE(11) HUB_ACASE(12) HUB_ACASE(13) HUB_ACASE(14)
            HUB_ACASE(15) HUB_ACASE(16)
        default: break;
        }
    } else {
        constexpr int B = 4 * (CLS - 1);
        switch (C.L - B) {
        case 1: HUB_ACALL(B + 1); break;
        case 2: HUB_ACALL(B + 2); break;
        case 3: HUB_ACALL(B + 3); break;
        case 4: HUB_ACALL(B + 4); break;
        default: break;
        }
    }
#undef HUB_ACASE
#undef HUB_ACALL
}

// The grouped apply is built in the one-set-per-wave layout only (uniform
// potential matrices; the packed layout never won the autotuner here).
template <typename T, bool CPX, bool SPINOR, int CPL, int CLS>
hipError_t launch_tg(const ApplyArgs& a, int nchunks, int nq, int waves, hipStream_t st) {
    // a lane's FP64 coefficients (functions x scalars) stay within 96 values
    if constexpr (hub_cls_nfmax(CLS) * CPL * (CPX ? 2 : 1) > 96) {
        return hipErrorInvalidValue;
    } else {
        const int64_t cg = (a.ncol + CPL - 1) / CPL;
        ApplyArgs b = a;
        b.nchunks = nchunks;
        b.tiles = static_cast<int>(static_cast<int64_t>(nq) * ((cg + HUB_WAVE - 1) / HUB_WAVE));
        const dim3 grid(static_cast<unsigned>(hub_slot_grid(nchunks, b.tiles)));
        if (a.pg) {
            // velocity gauge: complex states, merged launch only
            if constexpr (CPX && CLS > HUB_NCLASS)
                hipLaunchKernelGGL((k_apply_grouped<T, CPX, SPINOR, CPL, true, CLS, true>), grid,
                                   dim3(HUB_WAVE * waves), 0, st, b, b.gidx, b.tab, b.pg, reinterpret_cast<T*>(b.hpsi));
            else
                return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((k_apply_grouped<T, CPX, SPINOR, CPL, true, CLS, false>), grid, dim3(HUB_WAVE * waves),
                               0, st, b, b.gidx, b.tab, b.pg, reinterpret_cast<T*>(b.hpsi));
        }
        return hipGetLastError();
    }
}

template <typename T, bool CPX, bool SPINOR, int CLS>
hipError_t launch_cg(const ApplyArgs& a, int nchunks, int nq, int cpl, int waves, hipStream_t st) {
    switch (cpl) {
    case 1: return launch_tg<T, CPX, SPINOR, 1, CLS>(a, nchunks, nq, waves, st);
    case 2: return launch_tg<T, CPX, SPINOR, 2, CLS>(a, nchunks, nq, waves, st);
    case 4: return launch_tg<T, CPX, SPINOR, 4, CLS>(a, nchunks, nq, waves, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int CLS>
hipError_t launch_kg(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, hipStream_t st) {
    if (a.spinor) return launch_cg<T, true, true, CLS>(a, nchunks, nq, cpl, waves, st);
    return cplx ? launch_cg<T, true, false, CLS>(a, nchunks, nq, cpl, waves, st)
                : launch_cg<T, false, false, CLS>(a, nchunks, nq, cpl, waves, st);
}

template <typename T, bool CPX, bool SPINOR, int CPL>
hipError_t launch_t(const ApplyArgs& a, int nchunks, int nq, int waves, hipStream_t st) {
    const int64_t cg = (a.ncol + CPL - 1) / CPL;
    ApplyArgs b = a;
    b.nchunks = nchunks;
    b.tiles = static_cast<int>(a.wide ? static_cast<int64_t>(nq) * ((cg + HUB_WAVE - 1) / HUB_WAVE)
                                      : (static_cast<int64_t>(nq) * cg + HUB_WAVE - 1) / HUB_WAVE);
    const dim3 grid(static_cast<unsigned>(hub_slot_grid(nchunks, b.tiles)));
    T* h = reinterpret_cast<T*>(b.hpsi);
    if (a.spindep) {
        // spin-dependent spinor orbitals: 2L coefficients per lane column
        if constexpr (SPINOR && CPL <= 2) {
            if (a.pg) return hipErrorInvalidValue;
            if (a.wide)
                hipLaunchKernelGGL((k_apply<T, CPX, SPINOR, CPL, true, false, true>), grid, dim3(HUB_WAVE * waves), 0,
                                   st, b, b.gidx, b.tab, b.pg, h);
            else
                hipLaunchKernelGGL((k_apply<T, CPX, SPINOR, CPL, false, false, true>), grid, dim3(HUB_WAVE * waves), 0,
                                   st, b, b.gidx, b.tab, b.pg, h);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (a.pg) {
        // velocity gauge: complex states only
        if constexpr (CPX) {
            if (a.wide)
                hipLaunchKernelGGL((k_apply<T, CPX, SPINOR, CPL, true, true>), grid, dim3(HUB_WAVE * waves), 0, st, b,
                                   b.gidx, b.tab, b.pg, h);
            else
                hipLaunchKernelGGL((k_apply<T, CPX, SPINOR, CPL, false, true>), grid, dim3(HUB_WAVE * waves), 0, st, b,
                                   b.gidx, b.tab, b.pg, h);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (a.wide) {
        hipLaunchKernelGGL((k_apply<T, CPX, SPINOR, CPL, true, false>), grid, dim3(HUB_WAVE * waves), 0, st, b, b.gidx,
                           b.tab, b.pg, h);
    } else {
        hipLaunchKernelGGL((k_apply<T, CPX, SPINOR, CPL, false, false>), grid, dim3(HUB_WAVE * waves), 0, st, b,
                           b.gidx, b.tab, b.pg, h);
    }
    return hipGetLastError();
}

template <typename T, bool CPX, bool SPINOR>
hipError_t launch_c(const ApplyArgs& a, int nchunks, int nq, int cpl, int waves, hipStream_t st) {
    switch (cpl) {
    case 1: return launch_t<T, CPX, SPINOR, 1>(a, nchunks, nq, waves, st);
    case 2: return launch_t<T, CPX, SPINOR, 2>(a, nchunks, nq, waves, st);
    case 4: return launch_t<T, CPX, SPINOR, 4>(a, nchunks, nq, waves, st);
    default: return hipErrorInvalidValue;
    }
}

// Per-site (layered) work list, storage type T.
template <typename T>
hipError_t launch_apply_prec(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves,
                             hipStream_t st) {
    if (nchunks <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    if (a.spinor) return launch_c<T, true, true>(a, nchunks, nq, cpl, waves, st);
    return cplx ? launch_c<T, true, false>(a, nchunks, nq, cpl, waves, st)
                : launch_c<T, false, false>(a, nchunks, nq, cpl, waves, st);
}

// Grouped work list, storage type T, chunks of function-count class cls.
template <typename T>
hipError_t launch_apply_grouped_prec(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, int cls,
                                     hipStream_t st) {
    if (nchunks <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    switch (cls) {
    case 1: return launch_kg<T, 1>(a, nchunks, nq, cplx, cpl, waves, st);
    case 2: return launch_kg<T, 2>(a, nchunks, nq, cplx, cpl, waves, st);
    case 3: return launch_kg<T, 3>(a, nchunks, nq, cplx, cpl, waves, st);
    case 4: return launch_kg<T, 4>(a, nchunks, nq, cplx, cpl, waves, st);
    case HUB_MERGED8: return launch_kg<T, HUB_MERGED8>(a, nchunks, nq, cplx, cpl, waves, st);
    case HUB_MERGED16: return launch_kg<T, HUB_MERGED16>(a, nchunks, nq, cplx, cpl, waves, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
