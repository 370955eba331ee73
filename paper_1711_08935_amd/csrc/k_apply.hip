// Apply kernel: hpsi_q[g][col] += alpha * scale * (V_U psi)_q[g][col] for the
// entries of one work-list chunk (Eq. pot_V_U).
//
// Per lane and column: B_a = sum_b V_ab c_b with V_ab = Ueff (delta_ab/2 -
// n_ba) of the chunk's site and spin channel (spinor: B^s_a = sum_{s' b}
// V^{ss'}_ab c^{s'}_b, V^{ss'}_ab = Ueff (delta delta / 2 - n^{s's}_ba)); the
// transpose follows from differentiating E_U (Eq. minimization).  Then for
// every sphere entry e of the chunk:
//   hpsi[g_e][col] += exp(-i k.T_e) sum_a phi_a(e) B_a(col),
// where the phase is the same for every entry of a chunk and is folded into
// B once per chunk.
// The host groups entries in layers that never repeat a grid point, and
// launches one layer at a time, so no two lanes in flight update the same
// element: no atomics, deterministic results.  Sums are FP64; the updated
// element is rounded once to the storage type.
//
// Work mapping: blockIdx.x = chunk, blockIdx.y = column tile, with the same
// two lane layouts as the projection (WIDE: one state set per wave, so the
// set's potential matrix and phase are uniform; packed: narrow sets share a
// wave).  Each wave of the work-group takes interleaved entries (no
// reduction needed; B is recomputed per wave).

#include "kcommon.h"

namespace {

template <bool CPX, bool SPINOR, int CPL, int L>
__device__ __forceinline__ void coefficients(const ApplyArgs& a, const HubChunk& C, int q, int col0,
                                             double (&B)[L][CPL * (CPX ? 2 : 1)]) {
    constexpr int NC = CPX ? 2 : 1;
    const double U = a.ueff[C.site];
    const int ch = SPINOR ? 0 : (q % a.nspin);
    const double* __restrict__ nb = a.n + static_cast<int64_t>(C.site) * a.nblk * 98;
    const double* __restrict__ cq = a.c + (static_cast<int64_t>(q) * a.J + C.orb0) * a.ncol * NC;
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
        const int col = col0 + cc;
        const bool ok = col < a.ncol;
        double sc = a.alpha;
        if (a.colscale != nullptr && ok) {
            const int s = SPINOR ? (col >> 1) : col;
            sc *= a.colscale[static_cast<int64_t>(q) * a.nstates + s];
        }
        if (!ok) sc = 0.0;
        if constexpr (!SPINOR) {
            double cv[L][NC];
#pragma unroll
            for (int b = 0; b < L; ++b)
#pragma unroll
                for (int r = 0; r < NC; ++r) cv[b][r] = ok ? cq[(static_cast<int64_t>(b) * a.ncol + col) * NC + r] : 0.0;
            const double* __restrict__ nm = nb + ch * 98;
#pragma unroll
            for (int ai = 0; ai < L; ++ai) {
                double br = 0.0, bi = 0.0;
#pragma unroll
                for (int b = 0; b < L; ++b) {
                    // V_ab = U (delta_ab / 2 - n_ba)
                    const double vr = U * ((ai == b ? 0.5 : 0.0) - nm[(b * 7 + ai) * 2]);
                    if constexpr (CPX) {
                        const double vi = -U * nm[(b * 7 + ai) * 2 + 1];
                        br = fma(vr, cv[b][0], fma(-vi, cv[b][1], br));
                        bi = fma(vr, cv[b][1], fma(vi, cv[b][0], bi));
                    } else {
                        br = fma(vr, cv[b][0], br);
                    }
                }
                B[ai][cc * NC] = sc * br;
                if constexpr (CPX) B[ai][cc * NC + 1] = sc * bi;
            }
        } else {
            // spinor columns 2s + sigma; V^{sigma sigma'}_ab = U (dd/2 - n^{sigma' sigma}_ba)
            const int sg = col & 1;
            const int base = col - sg;
            double cv[2][L][2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int b = 0; b < L; ++b)
#pragma unroll
                    for (int r = 0; r < 2; ++r)
                        cv[t][b][r] = ok ? cq[(static_cast<int64_t>(b) * a.ncol + base + t) * 2 + r] : 0.0;
#pragma unroll
            for (int ai = 0; ai < L; ++ai) {
                double br = 0.0, bi = 0.0;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const double* __restrict__ nm = nb + (2 * t + sg) * 98;   // block (sigma' = t, sigma = sg)
#pragma unroll
                    for (int b = 0; b < L; ++b) {
                        const double vr = U * ((ai == b && t == sg) ? 0.5 : 0.0) - U * nm[(b * 7 + ai) * 2];
                        const double vi = -U * nm[(b * 7 + ai) * 2 + 1];
                        br = fma(vr, cv[t][b][0], fma(-vi, cv[t][b][1], br));
                        bi = fma(vr, cv[t][b][1], fma(vi, cv[t][b][0], bi));
                    }
                }
                B[ai][cc * 2] = sc * br;
                B[ai][cc * 2 + 1] = sc * bi;
            }
        }
    }
    if constexpr (CPX) {
        // fold the chunk's Bloch phase exp(-i k.T) into the coefficients
        const int k = a.spinor ? q : q / a.nspin;
        const double pr = a.phase[(static_cast<int64_t>(k) * a.nimg + C.img) * 2];
        const double pi = -a.phase[(static_cast<int64_t>(k) * a.nimg + C.img) * 2 + 1];
#pragma unroll
        for (int ai = 0; ai < L; ++ai)
#pragma unroll
            for (int cc = 0; cc < CPL; ++cc) {
                const double br = B[ai][2 * cc], bi = B[ai][2 * cc + 1];
                B[ai][2 * cc] = pr * br - pi * bi;
                B[ai][2 * cc + 1] = pr * bi + pi * br;
            }
    }
}

// Coefficients of a grouped chunk: function f is orbital a of site s(f)
// seen through lattice image img(f); B_f = alpha scale exp(-i k.T_img(f))
// sum_b V^{s(f)}_{a b} c_{s(f), b} (spinor: with the spin blocks).
template <bool CPX, bool SPINOR, int CPL, int NF>
__device__ __forceinline__ void coefficients_grouped(const ApplyArgs& a, int chunk, int q, int col0,
                                                     double (&B)[NF][CPL * (CPX ? 2 : 1)]) {
    constexpr int NC = CPX ? 2 : 1;
    const int ch = SPINOR ? 0 : (q % a.nspin);
    const int k = a.spinor ? q : q / a.nspin;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int j = a.f_orb[chunk * HUB_GF_MAX + f];
        const int img = a.f_img[chunk * HUB_GF_MAX + f];
        const int site = a.orb_site[j];
        const int o0 = a.site_orb0[site];
        const int L = a.site_L[site];
        const int ai = j - o0;
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
            if (!ok) sc = 0.0;
            const int colc = ok ? col : 0;
            double br = 0.0, bi = 0.0;
            if constexpr (!SPINOR) {
                const double* __restrict__ nm = nb + ch * 98;
#pragma unroll 1
                for (int b = 0; b < 7; ++b) {
                    if (b < L) {
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
                }
            } else {
                const int sg = colc & 1;
                const int base = colc - sg;
#pragma unroll 1
                for (int t = 0; t < 2; ++t) {
                    const double* __restrict__ nm = nb + (2 * t + sg) * 98;
#pragma unroll 1
                    for (int b = 0; b < 7; ++b) {
                        if (b < L) {
                            const double vr = U * ((ai == b && t == sg) ? 0.5 : 0.0) - U * nm[(b * 7 + ai) * 2];
                            const double vi = -U * nm[(b * 7 + ai) * 2 + 1];
                            const double cr = cq[(static_cast<int64_t>(b) * a.ncol + base + t) * 2];
                            const double ci = cq[(static_cast<int64_t>(b) * a.ncol + base + t) * 2 + 1];
                            br = fma(vr, cr, fma(-vi, ci, br));
                            bi = fma(vr, ci, fma(vi, cr, bi));
                        }
                    }
                }
            }
            br *= sc;
            bi *= sc;
            if constexpr (CPX) {
                B[f][2 * cc] = pr * br - pi * bi;
                B[f][2 * cc + 1] = pr * bi + pi * br;
            } else {
                B[f][cc] = br;
            }
        }
    }
}

template <typename T, bool CPX, bool SPINOR, int CPL, int L, bool WIDE, bool GROUPED = false>
__device__ __forceinline__ void apply_body(const ApplyArgs& a, const HubChunk& C, const int32_t* __restrict__ gidx,
                                           const double* __restrict__ tab, T* __restrict__ hpsi) {
    constexpr int NC = CPX ? 2 : 1;
    constexpr int NV = CPL * NC;
    constexpr int U = (L > 5) ? 2 : 4;
    const int lane = threadIdx.x & (HUB_WAVE - 1);
    // wave index made provably uniform so entry data goes through scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / HUB_WAVE);
    const int nw = blockDim.x / HUB_WAVE;
    const int cg = (a.ncol + CPL - 1) / CPL;
    int q, col0;
    if constexpr (WIDE) {
        const int tps = (cg + HUB_WAVE - 1) / HUB_WAVE;          // tiles per set (q uniform)
        q = blockIdx.y / tps;
        col0 = ((blockIdx.y - q * tps) * HUB_WAVE + lane) * CPL;
        if (col0 >= a.ncol) return;
    } else {
        const int t = blockIdx.y * HUB_WAVE + lane;
        if (t >= a.nq * cg) return;
        q = t / cg;
        col0 = (t - q * cg) * CPL;
    }

    double B[L][NV];
    if constexpr (GROUPED)
        coefficients_grouped<CPX, SPINOR, CPL, L>(a, a.chunk_list[blockIdx.x], q, col0, B);
    else
        coefficients<CPX, SPINOR, CPL, L>(a, C, q, col0, B);

    T* __restrict__ h_q = hpsi + static_cast<int64_t>(q) * a.qstride;
    const int32_t* __restrict__ gi = gidx + C.e0;
    const double* __restrict__ tb = tab + C.phi0;
    const int lofs = col0 * NC;

    const int nj = (C.ne - wave + nw - 1) / nw;
    int j = 0;
    for (; j + U <= nj; j += U) {
        T row[U][NV];
        int64_t rbase[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rbase[u] = static_cast<int64_t>(gi[wave + (j + u) * nw]) * a.ld * NC;
            load_row<T, NV>(h_q + rbase[u] + lofs, row[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double* __restrict__ w = tb + static_cast<int64_t>(wave + (j + u) * nw) * L;
            double add[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) add[v] = 0.0;
#pragma unroll
            for (int ai = 0; ai < L; ++ai) {
                const double wa = w[ai];
#pragma unroll
                for (int v = 0; v < NV; ++v) add[v] = fma(wa, B[ai][v], add[v]);
            }
            T out[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = static_cast<T>(static_cast<double>(row[u][v]) + add[v]);
            store_row<T, NV>(h_q + rbase[u] + lofs, out);
        }
    }
    for (; j < nj; ++j) {
        const int e = wave + j * nw;
        const int64_t rb = static_cast<int64_t>(gi[e]) * a.ld * NC;
        T row[NV];
        load_row<T, NV>(h_q + rb + lofs, row);
        const double* __restrict__ w = tb + static_cast<int64_t>(e) * L;
        double add[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) add[v] = 0.0;
#pragma unroll
        for (int ai = 0; ai < L; ++ai) {
            const double wa = w[ai];
#pragma unroll
            for (int v = 0; v < NV; ++v) add[v] = fma(wa, B[ai][v], add[v]);
        }
        T out[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v] = static_cast<T>(static_cast<double>(row[v]) + add[v]);
        store_row<T, NV>(h_q + rb + lofs, out);
    }
}

// The sphere tables and the output are separate restrict-qualified kernel
// arguments: the stores into hpsi inside the entry loop then cannot alias the
// table reads, and the uniform entry data stays on scalar loads.
template <typename T, bool CPX, bool SPINOR, int CPL, bool WIDE>
__global__ void __launch_bounds__(256) k_apply(const ApplyArgs a, const int32_t* __restrict__ gidx,
                                               const double* __restrict__ tab, T* __restrict__ hpsi) {
    const HubChunk C = a.chunks[a.chunk_list[blockIdx.x]];
    switch (C.L) {
    case 1: apply_body<T, CPX, SPINOR, CPL, 1, WIDE>(a, C, gidx, tab, hpsi); break;
    case 3: apply_body<T, CPX, SPINOR, CPL, 3, WIDE>(a, C, gidx, tab, hpsi); break;
    case 5: apply_body<T, CPX, SPINOR, CPL, 5, WIDE>(a, C, gidx, tab, hpsi); break;
    case 7: apply_body<T, CPX, SPINOR, CPL, 7, WIDE>(a, C, gidx, tab, hpsi); break;
    default: break;
    }
}

// Grouped chunks: L is the number of concatenated functions of the chunk's
// covering sites; every grid point lies in one chunk, so one launch writes
// every point once.
template <typename T, bool CPX, bool SPINOR, int CPL, bool WIDE>
__global__ void __launch_bounds__(256) k_apply_grouped(const ApplyArgs a, const int32_t* __restrict__ gidx,
                                                       const double* __restrict__ tab, T* __restrict__ hpsi) {
    const HubChunk C = a.chunks[a.chunk_list[blockIdx.x]];
    constexpr int NV = CPL * (CPX ? 2 : 1);
#define HUB_ACASE(n)                                                                              \
    case n:                                                                                       \
        if constexpr (n * NV <= 96) apply_body<T, CPX, SPINOR, CPL, n, WIDE, true>(a, C, gidx, tab, hpsi); \
        break;
    switch (C.L) {
        HUB_ACASE(1) HUB_ACASE(2) HUB_ACASE(3) HUB_ACASE(4) HUB_ACASE(5) HUB_ACASE(6) HUB_ACASE(7)
        HUB_ACASE(8) HUB_ACASE(9) HUB_ACASE(10) HUB_ACASE(11) HUB_ACASE(12) HUB_ACASE(13)
        HUB_ACASE(14) HUB_ACASE(15) HUB_ACASE(16)
    default: break;
    }
#undef HUB_ACASE
}

// The grouped apply is built in the one-set-per-wave layout only (uniform
// potential matrices; the packed layout never won the autotuner here).
template <typename T, bool CPX, bool SPINOR, int CPL>
hipError_t launch_tg(const ApplyArgs& a, int nchunks, int nq, int waves, hipStream_t st) {
    const int64_t cg = (a.ncol + CPL - 1) / CPL;
    const int64_t tiles = static_cast<int64_t>(nq) * ((cg + HUB_WAVE - 1) / HUB_WAVE);
    hipLaunchKernelGGL((k_apply_grouped<T, CPX, SPINOR, CPL, true>), dim3(nchunks, static_cast<unsigned>(tiles), 1),
                       dim3(HUB_WAVE * waves), 0, st, a, a.gidx, a.tab, reinterpret_cast<T*>(a.hpsi));
    return hipGetLastError();
}

template <typename T, bool CPX, bool SPINOR>
hipError_t launch_cg(const ApplyArgs& a, int nchunks, int nq, int cpl, int waves, hipStream_t st) {
    switch (cpl) {
    case 1: return launch_tg<T, CPX, SPINOR, 1>(a, nchunks, nq, waves, st);
    case 2: return launch_tg<T, CPX, SPINOR, 2>(a, nchunks, nq, waves, st);
    case 4: return launch_tg<T, CPX, SPINOR, 4>(a, nchunks, nq, waves, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool CPX, bool SPINOR, int CPL>
hipError_t launch_t(const ApplyArgs& a, int nchunks, int nq, int waves, hipStream_t st) {
    const int64_t cg = (a.ncol + CPL - 1) / CPL;
    if (a.wide) {
        const int64_t tiles = static_cast<int64_t>(nq) * ((cg + HUB_WAVE - 1) / HUB_WAVE);
        hipLaunchKernelGGL((k_apply<T, CPX, SPINOR, CPL, true>), dim3(nchunks, static_cast<unsigned>(tiles), 1),
                           dim3(HUB_WAVE * waves), 0, st, a, a.gidx, a.tab, reinterpret_cast<T*>(a.hpsi));
    } else {
        const int64_t tiles = (static_cast<int64_t>(nq) * cg + HUB_WAVE - 1) / HUB_WAVE;
        hipLaunchKernelGGL((k_apply<T, CPX, SPINOR, CPL, false>), dim3(nchunks, static_cast<unsigned>(tiles), 1),
                           dim3(HUB_WAVE * waves), 0, st, a, a.gidx, a.tab, reinterpret_cast<T*>(a.hpsi));
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

}  // namespace

hipError_t launch_apply(const ApplyArgs& a, int nchunks, int nq, int prec, int cplx, int cpl, int waves,
                        hipStream_t st) {
    if (nchunks <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    if (prec == HUB_F64) {
        if (a.spinor) return launch_c<double, true, true>(a, nchunks, nq, cpl, waves, st);
        return cplx ? launch_c<double, true, false>(a, nchunks, nq, cpl, waves, st)
                    : launch_c<double, false, false>(a, nchunks, nq, cpl, waves, st);
    }
    if (a.spinor) return launch_c<float, true, true>(a, nchunks, nq, cpl, waves, st);
    return cplx ? launch_c<float, true, false>(a, nchunks, nq, cpl, waves, st)
                : launch_c<float, false, false>(a, nchunks, nq, cpl, waves, st);
}

hipError_t launch_apply_grouped(const ApplyArgs& a, int nchunks, int nq, int prec, int cplx, int cpl, int waves,
                                hipStream_t st) {
    if (nchunks <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    if (prec == HUB_F64) {
        if (a.spinor) return launch_cg<double, true, true>(a, nchunks, nq, cpl, waves, st);
        return cplx ? launch_cg<double, true, false>(a, nchunks, nq, cpl, waves, st)
                    : launch_cg<double, false, false>(a, nchunks, nq, cpl, waves, st);
    }
    if (a.spinor) return launch_cg<float, true, true>(a, nchunks, nq, cpl, waves, st);
    return cplx ? launch_cg<float, true, false>(a, nchunks, nq, cpl, waves, st)
                : launch_cg<float, false, false>(a, nchunks, nq, cpl, waves, st);
}
