// Small FP64 kernels of the Hubbard step: chunk reduction of the projections,
// renormalized occupations N-bar, occupation matrices n and P-bar, ACBN0
// U-bar/J-bar, Dudarev energy and Hubbard forces.  All reductions run in a
// fixed order (no atomics), so results are bitwise reproducible.

#include <algorithm>

#include "ksmall.h"

namespace {

constexpr int NB = 256;   // threads of the per-site kernels
constexpr int TILE = 64;  // (k-point, state) pairs staged per LDS tile in k_occ_part

// ---------------------------------------------------------------- reduction
// out[q][r][col] = dV * sum over the chunks of the row's site of
// exp(+i k.T_chunk) part[q][chunk.part0 * mult + (r - orb0 * mult)][col]
// (the Bloch phase of Fig. 1, shared by all entries of a chunk).
__global__ void __launch_bounds__(256) k_reduce(const ReduceArgs a) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const int q = blockIdx.z;
    if (col >= a.ncol) return;
    const int site = a.orb_site[r / a.mult];
    const int local = r - a.site_orb0[site] * a.mult;
    const int NC = a.ncplx;
    const int k = a.spinor ? a.q0 + q : (a.q0 + q) / a.nspin;
    const double* ph = a.phase + static_cast<int64_t>(k) * a.nimg * 2;
    double s0 = 0.0, s1 = 0.0;
    // gradient or moment tables of spin-dependent orbitals: one launch per
    // spin component, each writing the columns of its component
    if (a.colpar >= 0 && (col & 1) != a.colpar) return;
    // spin-dependent orbitals: column 2s + sigma of orbital m is the partial
    // row sigma L + m of the chunk (the orbital of its spin component)
    const int srow = a.spindep ? (col & 1) * a.site_L[site] + local : local;
    for (int t = a.site_chunk_ptr[site]; t < a.site_chunk_ptr[site + 1]; ++t) {
        const HubChunk& C = a.chunks[a.site_chunk_ids[t]];
        const int64_t row = static_cast<int64_t>(q) * a.prows + static_cast<int64_t>(C.part0) * a.pmult + srow;
        const double* p = a.part + (row * a.ncol + col) * NC;
        if (NC == 2) {
            const double pr = ph[2 * C.img], pi = ph[2 * C.img + 1];
            s0 += pr * p[0] - pi * p[1];
            s1 += pr * p[1] + pi * p[0];
        } else {
            s0 += p[0];
        }
    }
    double* o = a.out + ((static_cast<int64_t>(q) * a.nrows + r) * a.ncol + col) * NC;
    o[0] = a.dV * s0;
    if (NC == 2) o[1] = a.dV * s1;
}

// Grouped work list: out[q][j][col] = dV sum over the workspace rows that
// belong to orbital j of exp(+i k.T_row) part[q][row][col].  A work-group
// serves 64 columns of one (j, q); each of its RW waves takes a contiguous
// range of the orbital's rows and walks it in batches of 8: the batch's row
// indexes and images are uniform (scalar loads), its 8 row values are in
// flight together (one 8- or 16-byte load per lane each), then added in row
// order.  The waves' sums are combined in wave order through LDS.  RW
// follows the rows per orbital.
template <int RW, int NC>
__global__ void __launch_bounds__(RW * 64) k_reduce_grouped(const ReduceGroupedArgs a) {
    constexpr int NBATCH = 8;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = blockIdx.x * 64 + lane;
    const int j = blockIdx.y;
    const int ncomp = a.ncomp > 1 ? a.ncomp : 1;
    const int comp = blockIdx.z % ncomp;
    const int q = blockIdx.z / ncomp;
    const bool active = col < a.ncol;
    const int k = a.spinor ? a.q0 + q : (a.q0 + q) / a.nspin;
    const double* __restrict__ ph = a.phase + static_cast<int64_t>(k) * a.nimg * 2;
    // spin-dependent orbitals: spinor column 2s + sigma reads the rows of the
    // orbital of its spin component
    const int64_t shift = (a.spin_shift && (col & 1)) ? a.spin_shift[j] : 0;
    const double* __restrict__ base = a.part + comp * a.pplane +
                                      (static_cast<int64_t>(q) * a.prows + shift) * a.ncol * NC +
                                      static_cast<int64_t>(active ? col : 0) * NC;
    const int t0 = a.red_ptr[j], t1 = a.red_ptr[j + 1];
    int lo, len;
    hub_wave_range(t1 - t0, RW, wave, lo, len);
    const int32_t* __restrict__ rows = a.red_row + t0 + lo;
    const int32_t* __restrict__ imgs = a.red_img + t0 + lo;
    double s0 = 0.0, s1 = 0.0;
    for (int b = 0; b < len; b += NBATCH) {
        const int nb = len - b < NBATCH ? len - b : NBATCH;
        double v[NBATCH][NC];
        double pr[NBATCH], pi[NBATCH];
#pragma unroll
        for (int u = 0; u < NBATCH; ++u) {
            // rows past the wave's range re-read its last row; their values
            // are replaced by zeros below (branch-free, so that every load of
            // the batch is issued before the first add)
            const int t = b + (u < nb ? u : nb - 1);
            const double* p = base + static_cast<int64_t>(rows[t]) * a.ncol * NC;
            if constexpr (NC == 2) {
                const hub_d2 x = *reinterpret_cast<const hub_d2*>(p);
                v[u][0] = x[0];
                v[u][1] = x[1];
                const int im = imgs[t];
                pr[u] = ph[2 * im];
                pi[u] = ph[2 * im + 1];
            } else {
                v[u][0] = p[0];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NBATCH; ++u) {
            const bool use = u < nb;
            if constexpr (NC == 2) {
                const double x0 = use ? v[u][0] : 0.0, x1 = use ? v[u][1] : 0.0;
                s0 += pr[u] * x0 - pi[u] * x1;
                s1 += pr[u] * x1 + pi[u] * x0;
            } else {
                s0 += use ? v[u][0] : 0.0;
            }
        }
    }
    __shared__ double red[RW][64][2];
    red[wave][lane][0] = s0;
    red[wave][lane][1] = s1;
    __syncthreads();
    if (wave != 0 || !active) return;
    double r0 = 0.0, r1 = 0.0;
    for (int w = 0; w < RW; ++w) {
        r0 += red[w][lane][0];
        r1 += red[w][lane][1];
    }
    double* o = comp == 0 ? a.out + ((static_cast<int64_t>(q) * a.J + j) * a.ncol + col) * NC
                          : a.mout + ((static_cast<int64_t>(q) * a.J * 3 + 3 * j + comp - 1) * a.ncol + col) * NC;
    o[0] = a.dV * r0;
    if (NC == 2) o[1] = a.dV * r1;
}

// ---------------------------------------------------------------- N-bar
// nbar[q][T][s] = sum_{j in species T} sum_{columns of s} |c[q][j][col]|^2
// (Eq. notation_Nbar).  The species' orbitals are split into NBPART
// interleaved parts, each summed in order; the parts are combined as
// (p0 + p1) + (p2 + p3).  k_nbar and the fused occupation kernel of the step
// use exactly this order, so both give the same N-bar to the last bit.
constexpr int NBPART = 4;

// part ``part`` of N-bar for state s of set q: the species' orbitals
// ids[t], t = t0 + part, t0 + part + NBPART, ... < t1, added in that order.
// The orbitals are taken in batches of 8 whose values are all loaded before
// the first add (orbitals past t1 re-read the batch's first one and add 0),
// so a long species list costs a few load latencies, not one per orbital.
template <int NC, int CPS>
__device__ __forceinline__ double nbar_part_t(const double* __restrict__ c, const int32_t* __restrict__ ids, int t0,
                                              int t1, int part, int64_t qbase, int s, int ncol) {
    constexpr int NB8 = 8;
    const double* cq = c + qbase + static_cast<int64_t>(s) * CPS * NC;
    double acc = 0.0;
    for (int t = t0 + part; t < t1; t += NB8 * NBPART) {
        double r[NB8][CPS * NC];
#pragma unroll
        for (int u = 0; u < NB8; ++u) {
            const int tt = t + u * NBPART < t1 ? t + u * NBPART : t;
            const double* p = cq + static_cast<int64_t>(ids[tt]) * ncol * NC;
#pragma unroll
            for (int x = 0; x < CPS * NC; ++x) r[u][x] = p[x];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NB8; ++u) {
            double v = 0.0;
#pragma unroll
            for (int x = 0; x < CPS * NC; ++x) v = fma(r[u][x], r[u][x], v);
            acc += t + u * NBPART < t1 ? v : 0.0;
        }
    }
    return acc;
}

__device__ __forceinline__ double nbar_part(const double* __restrict__ c, const int32_t* __restrict__ ids, int t0,
                                            int t1, int part, int64_t qbase, int s, int ncol, int NC, int cps) {
    if (NC == 2)
        return cps == 2 ? nbar_part_t<2, 2>(c, ids, t0, t1, part, qbase, s, ncol)
                        : nbar_part_t<2, 1>(c, ids, t0, t1, part, qbase, s, ncol);
    return nbar_part_t<1, 1>(c, ids, t0, t1, part, qbase, s, ncol);
}

// A work-group serves 64 states of one (T, q): wave w sums part w.
__global__ void __launch_bounds__(NBPART * 64) k_nbar(const NbarArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int s = blockIdx.x * 64 + lane;
    const int T = blockIdx.y;
    const int q = blockIdx.z;
    const bool active = s < a.nstates;
    const int NC = a.ncplx;
    __shared__ double red[NBPART][64];
    red[wave][lane] = nbar_part(a.c, a.species_orb_ids, a.species_orb_ptr[T], a.species_orb_ptr[T + 1], wave,
                                static_cast<int64_t>(q) * a.J * a.ncol * NC, active ? s : 0, a.ncol, NC,
                                a.spinor ? 2 : 1);
    __syncthreads();
    if (wave != 0 || !active) return;
    const double r = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    a.nbar[(static_cast<int64_t>(q) * a.nspecies + T) * a.nstates + s] = r;
}

// ---------------------------------------------------------------- occupations
// n_ab = sum_k w_k sum_s f_s conj(c_a) c_b (Eq. occ_matrices) for every
// block (spin channel, or spinor block sigma sigma') and P-bar_ab, the same
// with the extra weight N-bar_s of the site's species (Eq. notation_Pbar).
// Pass 1: work-group (site, channel, split) sums the (k-point, state) pairs
// of its split: the states are staged through LDS, the (a, b) pairs of the
// combined matrix are spread over the threads with several state slices
// each, and the slices are summed in a fixed order into the workspace.
// Pass 2 sums the splits in order and writes n and P-bar.
__global__ void __launch_bounds__(NB) k_occ_part(const OccArgs a) {
    const int site = blockIdx.x;
    const int ch = blockIdx.y;
    const int split = blockIdx.z;
    const int L = a.site_L[site];
    const int orb0 = a.site_orb0[site];
    const int T = a.site_species[site];
    const int NC = a.ncplx;
    const int nsig = a.spinor ? 2 : 1;               // spin components staged per state
    const int ncp = a.spinor ? 2 * L : L;            // rows of the combined matrix
    const int npairs = ncp * ncp;
    const int nslice = NB / npairs;
    const int tid = threadIdx.x;
    const int pair = tid % npairs;
    const int slice = tid / npairs;
    const bool worker = slice < nslice;
    const int ra = pair / ncp, rb = pair % ncp;      // combined index: sigma * L + m

    __shared__ double cs[2][7][TILE][2];
    __shared__ double wt[TILE], wtn[TILE];
    __shared__ double red[NB][4];

    // this split's (k, state) pairs, flattened as k * nstates + s
    const int np = a.nk * a.nstates;
    const int per = (np + a.nsplit - 1) / a.nsplit;
    const int p0 = split * per;
    const int p1 = min(np, p0 + per);
    double nr = 0.0, ni = 0.0, pr = 0.0, pi = 0.0;
    for (int t0 = p0; t0 < p1; t0 += TILE) {
        const int pp = t0 + tid;
        if (tid >= TILE) {
        } else if (pp < p1) {
            const int k = pp / a.nstates, s = pp - k * a.nstates;
            const int q = a.spinor ? k : k * a.nspin + ch;
            const double wk = a.kweights[k];
            const double f = a.f[static_cast<int64_t>(q) * a.nstates + s];
            const double nb =
                (a.nbar != nullptr) ? a.nbar[(static_cast<int64_t>(q) * a.nspecies + T) * a.nstates + s] : 0.0;
            wt[tid] = wk * f;
            wtn[tid] = wk * f * nb;
            for (int x = 0; x < nsig; ++x)
                for (int m = 0; m < L; ++m) {
                    const double* p = a.c + ((static_cast<int64_t>(q) * a.J + orb0 + m) * a.ncol + s * nsig + x) * NC;
                    cs[x][m][tid][0] = p[0];
                    cs[x][m][tid][1] = (NC == 2) ? p[1] : 0.0;
                }
        } else {
            wt[tid] = 0.0;
            wtn[tid] = 0.0;
            for (int x = 0; x < nsig; ++x)
                for (int m = 0; m < L; ++m) cs[x][m][tid][0] = cs[x][m][tid][1] = 0.0;
        }
        __syncthreads();
        if (worker) {
            const int xa = ra / L, ma = ra % L, xb = rb / L, mb = rb % L;
            const int nt = min(TILE, p1 - t0);
            for (int t = slice; t < nt; t += nslice) {
                // conj(c_a) c_b
                const double ar = cs[xa][ma][t][0], ai = cs[xa][ma][t][1];
                const double br = cs[xb][mb][t][0], bi = cs[xb][mb][t][1];
                const double re = ar * br + ai * bi;
                const double im = ar * bi - ai * br;
                nr = fma(wt[t], re, nr);
                ni = fma(wt[t], im, ni);
                pr = fma(wtn[t], re, pr);
                pi = fma(wtn[t], im, pi);
            }
        }
        __syncthreads();
    }
    red[tid][0] = nr;
    red[tid][1] = ni;
    red[tid][2] = pr;
    red[tid][3] = pi;
    __syncthreads();
    const int nchan = gridDim.y;
    double* w = a.ws + ((static_cast<int64_t>(site) * nchan + ch) * a.nsplit + split) * (HUB_OCC_PAIRS * 4);
    for (int o = tid; o < npairs; o += NB) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int z = 0; z < nslice; ++z)
            for (int r = 0; r < 4; ++r) v[r] += red[z * npairs + o][r];
        for (int r = 0; r < 4; ++r) w[o * 4 + r] = v[r];
    }
}

// Sums the splits of one site and NCH channels (ch0, ch0 + 1, ...) in
// order: out = n and P-bar entries (blocks of the channel, zeros outside the
// L x L corner), one thread per (entry, value) so that every split's load is
// in flight, the loads of all NCH channels issued before the adds (each
// channel's sum in split order, as with one channel at a time).
template <int NCH>
__device__ void occ_final_sums(const OccArgs& a, int site, int ch0, int nchan, double* n, double* pbar,
                               double (*Nf)[7][7][2], double (*P)[7][7][2]) {
    const int L = a.site_L[site];
    const int ncp = a.spinor ? 2 * L : L;
    const int64_t chstride = static_cast<int64_t>(a.nsplit) * (HUB_OCC_PAIRS * 4);
    const double* w = a.ws + (static_cast<int64_t>(site) * nchan + ch0) * chstride;
    const int nblk_here = a.spinor ? 4 : 1;
    for (int o = threadIdx.x; o < nblk_here * 49 * 4; o += NB) {
        const int r = o & 3, eb = o >> 2;
        const int blk = eb / 49, e = eb % 49, i = e / 7, j = e % 7;
        double v[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) v[c] = 0.0;
        if (i < L && j < L) {
            const int x = a.spinor ? blk / 2 : 0, y = a.spinor ? blk % 2 : 0;
            const int p = (x * L + i) * ncp + (y * L + j);
            const double* wp = w + static_cast<int64_t>(p) * 4 + r;
            // splits in batches of 8, every load of a batch issued before
            // the adds, which run in split order (splits past the end add 0)
            for (int z0 = 0; z0 < a.nsplit; z0 += 8) {
                double t[NCH][8];
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int z = z0 + u < a.nsplit ? z0 + u : z0;
                        t[c][u] = wp[c * chstride + static_cast<int64_t>(z) * HUB_OCC_PAIRS * 4];
                    }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[c] += z0 + u < a.nsplit ? t[c][u] : 0.0;
            }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int oblk = a.spinor ? blk : ch0 + c;
            const int64_t base = ((static_cast<int64_t>(site) * a.nblk + oblk) * 49 + e) * 2;
            if (r < 2) {
                n[base + r] = v[c];
                if (Nf) Nf[oblk][i][j][r] = v[c];
            } else {
                if (pbar) pbar[base + r - 2] = v[c];
                if (P) P[oblk][i][j][r - 2] = v[c];
            }
        }
    }
}

__global__ void __launch_bounds__(NB) k_occ_final(const OccArgs a) {
    occ_final_sums<1>(a, blockIdx.x, blockIdx.y, gridDim.y, a.n, a.pbar, nullptr, nullptr);
}

// ---------------------------------------------------------------- ACBN0
// U-bar and J-bar of one site (Eqs. ACBN0_U, ACBN0_J; App. B), with the
// numerators read as P_mm' P_m''m''' (mm'|m''m''') and P_mm' P_m''m'''
// (mm'''|m''m'), denominators from the bare diagonal occupations.
// The site's P-bar and n blocks ([blk][7][7] complex) are in LDS.
struct AcbLds {
    double P[4][7][7][2];
    double Nf[4][7][7][2];
    double Ts[2401];
    double redU[NB], redJ[NB];
};

// tensor_in_lds: the caller has already put the site's tensor in sm.Ts.
__device__ void acbn0_site(const Acbn0Args& a, int site, AcbLds& sm, bool tensor_in_lds = false) {
    const int L = a.site_L[site];
    const int tid = threadIdx.x;
    const double fixed = a.ueff_fixed[site];
    __syncthreads();                          // P and Nf written by the caller
    if (!isnan(fixed)) {
        if (tid == 0) {
            a.U[site] = fixed;
            a.J[site] = 0.0;
            a.Ueff[site] = fixed;
            if (a.status) {
                // flag occupations that are not finite (NaN or Inf in the states)
                bool finite = true;
                for (int b = 0; b < a.nblk; ++b)
                    for (int e = 0; e < L * L; ++e)
                        finite = finite && isfinite(sm.Nf[b][e / L][e % L][0]) && isfinite(sm.Nf[b][e / L][e % L][1]);
                a.status[site] = finite ? 0 : HUB_ENONFINITE;
            }
        }
        return;
    }
    auto& P = sm.P;
    auto& Ts = sm.Ts;
    auto& redU = sm.redU;
    auto& redJ = sm.redJ;
    const int nb = a.nblk;
    const int L2 = L * L, L4 = L2 * L2;
    if (!tensor_in_lds) {
        const double* Tg = a.tensor + static_cast<int64_t>(site) * 2401;
        for (int o = tid; o < L4; o += NB) Ts[o] = Tg[o];
        __syncthreads();
    }

    // channel layout: unpolarized -> both channels are block 0
    const int c0 = 0;
    const int c1 = (nb == 2) ? 1 : (nb == 4 ? 3 : 0);
    double su = 0.0, sj = 0.0;
    // o = ((A L + B) L + C) L + D; quotients by L2 and L through a float
    // reciprocal: (o + 0.5) / L2 stays at least 0.5 / 49 from an integer, far
    // above the reciprocal's rounding for o < 2401
    const float rL = 1.0f / static_cast<float>(L), rL2 = 1.0f / static_cast<float>(L2);
    for (int o = tid; o < L4; o += NB) {
        const int ab = static_cast<int>((static_cast<float>(o) + 0.5f) * rL2), cd = o - ab * L2;
        const int A = static_cast<int>((static_cast<float>(ab) + 0.5f) * rL), B = ab - A * L;
        const int Cc = static_cast<int>((static_cast<float>(cd) + 0.5f) * rL), D = cd - Cc * L;
        const double t_abcd = Ts[o];
        const double t_adcb = Ts[((A * L + D) * L + Cc) * L + B];
        // numerator U: sum_{alpha beta} P^a_ab P^b_cd (ab|cd) = Re(Ps_ab Ps_cd) (ab|cd)
        const double sr_ab = P[c0][A][B][0] + P[c1][A][B][0], si_ab = P[c0][A][B][1] + P[c1][A][B][1];
        const double sr_cd = P[c0][Cc][D][0] + P[c1][Cc][D][0], si_cd = P[c0][Cc][D][1] + P[c1][Cc][D][1];
        su = fma(sr_ab * sr_cd - si_ab * si_cd, t_abcd, su);
        if (nb == 4) {
            // sum_{s s'} Re(P^{ss'}_ab P^{s's}_cd) (ad|cb)
            double v = 0.0;
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 2; ++y) {
                    const int b1 = 2 * x + y, b2 = 2 * y + x;
                    v += P[b1][A][B][0] * P[b2][Cc][D][0] - P[b1][A][B][1] * P[b2][Cc][D][1];
                }
            sj = fma(v, t_adcb, sj);
        } else {
            double v = P[c0][A][B][0] * P[c0][Cc][D][0] - P[c0][A][B][1] * P[c0][Cc][D][1];
            v += P[c1][A][B][0] * P[c1][Cc][D][0] - P[c1][A][B][1] * P[c1][Cc][D][1];
            sj = fma(v, t_adcb, sj);
        }
    }
    // sum over the lanes of each wave (butterfly), then the waves in order
    for (int m = 32; m >= 1; m >>= 1) {
        su += __shfl_xor(su, m, 64);
        sj += __shfl_xor(sj, m, 64);
    }
    if ((tid & 63) == 0) {
        redU[tid >> 6] = su;
        redJ[tid >> 6] = sj;
    }
    __syncthreads();
    if (tid != 0) return;
    for (int w = 1; w < NB / 64; ++w) {
        redU[0] += redU[w];
        redJ[0] += redJ[w];
    }
    double dU = 0.0, dJ = 0.0;
    if (nb != 4) {
        // collinear: N^alpha_m = n^alpha_mm (real part)
        double N[2][7];
        for (int m = 0; m < L; ++m) {
            N[0][m] = sm.Nf[c0][m][m][0];
            N[1][m] = sm.Nf[c1][m][m][0];
        }
        for (int al = 0; al < 2; ++al)
            for (int m = 0; m < L; ++m)
                for (int mp = 0; mp < L; ++mp)
                    if (m != mp) dJ += N[al][m] * N[al][mp];
        dU = dJ;
        for (int al = 0; al < 2; ++al)
            for (int m = 0; m < L; ++m)
                for (int mp = 0; mp < L; ++mp) dU += N[al][m] * N[1 - al][mp];
    } else {
        // spinor (App. B): complex diagonal blocks N^{xy}_m = n^{xy}_mm
        auto re_mul = [&](int b1, int m1, int b2, int m2) {
            return sm.Nf[b1][m1][m1][0] * sm.Nf[b2][m2][m2][0] - sm.Nf[b1][m1][m1][1] * sm.Nf[b2][m2][m2][1];
        };
        for (int s = 0; s < 2; ++s) {
            const int ss = 3 * s, oo = 3 * (1 - s), so = 2 * s + (1 - s), os = 2 * (1 - s) + s;
            for (int m = 0; m < L; ++m)
                for (int mp = 0; mp < L; ++mp) {
                    dU += re_mul(ss, m, oo, mp);
                    if (m != mp) {
                        dU += re_mul(ss, m, ss, mp);
                        dJ += re_mul(ss, m, ss, mp) + re_mul(so, m, os, mp);
                    }
                }
            for (int m = 0; m < L; ++m) dU -= re_mul(so, m, os, m);
        }
    }
    int st = 0;
    double U = 0.0, J = 0.0;
    if (fabs(dU) < 1e-12) st = HUB_WDEGENERATE; else U = redU[0] / dU;
    if (fabs(dJ) < 1e-12) st = HUB_WDEGENERATE; else J = redJ[0] / dJ;
    if (!isfinite(redU[0]) || !isfinite(redJ[0]) || !isfinite(dU) || !isfinite(dJ)) {
        // occupations that are not finite: report it and keep U, J NaN
        st = HUB_ENONFINITE;
        U = J = __builtin_nan("");
    }
    a.U[site] = U;
    a.J[site] = J;
    a.Ueff[site] = U - J;
    if (a.status) a.status[site] = st;
}

__global__ void __launch_bounds__(NB) k_acbn0(const Acbn0Args a) {
    const int site = blockIdx.x;
    __shared__ AcbLds sm;
    for (int o = threadIdx.x; o < a.nblk * 49; o += NB) {
        const int b = o / 49, e = o % 49;
        const int64_t base = ((static_cast<int64_t>(site) * a.nblk + b) * 49 + e) * 2;
        sm.P[b][e / 7][e % 7][0] = a.pbar[base];
        sm.P[b][e / 7][e % 7][1] = a.pbar[base + 1];
        sm.Nf[b][e / 7][e % 7][0] = a.n[base];
        sm.Nf[b][e / 7][e % 7][1] = a.n[base + 1];
    }
    acbn0_site(a, site, sm);
}

// ---------------------------------------------------------------- fused step
// N-bar, n, P-bar and U-bar/J-bar of the batched step in two launches.
// k_step_occ_part: work-group (site, channel, split) stages the c of its
// (k-point, state) pairs tile by tile, forms N-bar of each pair from the
// species' projections (nbar_part: the order of k_nbar; the first site of a
// species writes it out) and sums its split of n and P-bar as k_occ_part
// does.  k_step_occ_final: one work-group per site sums every split of every
// channel in order (as k_occ_final), writes n and P-bar and runs the site's
// ACBN0 step from LDS (acbn0_site).  The kernel boundary orders the two; a
// completion count inside one launch was measured slower, since every
// work-group's device-scope release then writes back its L2.
struct OccLds {
    double cs[2][7][TILE][2];
    double wt[TILE], wtn[TILE];
    double red[NB][4];
    double nbp[NBPART][TILE];
};

__global__ void __launch_bounds__(NB) k_step_occ_part(const OccArgs a) {
    const int site = blockIdx.x;
    const int ch = blockIdx.y;
    const int split = blockIdx.z;
    const int nchan = gridDim.y;
    const int L = a.site_L[site];
    const int orb0 = a.site_orb0[site];
    const int T = a.site_species[site];
    const int NC = a.ncplx;
    const int nsig = a.spinor ? 2 : 1;
    const int ncp = a.spinor ? 2 * L : L;
    const int npairs = ncp * ncp;
    const int nslice = NB / npairs;
    const int tid = threadIdx.x;
    const int pair = tid % npairs;
    const int slice = tid / npairs;
    const bool worker = slice < nslice;
    const int ra = pair / ncp, rb = pair % ncp;

    __shared__ struct {
        OccLds o;
    } sm;

    // the first site of each species writes that species' N-bar
    bool writer = a.nbar_out != nullptr;
    for (int s2 = 0; s2 < site && writer; ++s2) writer = a.site_species[s2] != T;
    const int sp0 = a.species_orb_ptr[T], sp1 = a.species_orb_ptr[T + 1];

    const int np = a.nk * a.nstates;
    const int per = (np + a.nsplit - 1) / a.nsplit;
    const int p0 = split * per;
    const int p1 = min(np, p0 + per);
    double nr = 0.0, ni = 0.0, pr = 0.0, pi = 0.0;
    for (int t0 = p0; t0 < p1; t0 += TILE) {
        const int pp = t0 + tid;
        if (tid < TILE) {
            if (pp < p1) {
                const int k = pp / a.nstates, s = pp - k * a.nstates;
                const int q = a.spinor ? k : k * a.nspin + ch;
                sm.o.wt[tid] = a.kweights[k] * a.f[static_cast<int64_t>(q) * a.nstates + s];
                for (int x = 0; x < nsig; ++x)
                    for (int m = 0; m < L; ++m) {
                        const double* p =
                            a.c + ((static_cast<int64_t>(q) * a.J + orb0 + m) * a.ncol + s * nsig + x) * NC;
                        sm.o.cs[x][m][tid][0] = p[0];
                        sm.o.cs[x][m][tid][1] = (NC == 2) ? p[1] : 0.0;
                    }
            } else {
                sm.o.wt[tid] = 0.0;
                for (int x = 0; x < nsig; ++x)
                    for (int m = 0; m < L; ++m) sm.o.cs[x][m][tid][0] = sm.o.cs[x][m][tid][1] = 0.0;
            }
        }
        {
            // N-bar of the tile's pairs: part tid / TILE (one wave each) of pair tid % TILE
            static_assert(TILE == 64 && NB == NBPART * TILE, "one N-bar part per wave");
            const int pl = tid % TILE, part = __builtin_amdgcn_readfirstlane(tid / TILE);
            const int pq = t0 + pl;
            double v = 0.0;
            if (pq < p1) {
                const int k = pq / a.nstates, s = pq - k * a.nstates;
                const int q = a.spinor ? k : k * a.nspin + ch;
                v = nbar_part(a.c, a.species_orb_ids, sp0, sp1, part, static_cast<int64_t>(q) * a.J * a.ncol * NC, s,
                              a.ncol, NC, nsig);
            }
            sm.o.nbp[part][pl] = v;
        }
        __syncthreads();
        if (tid < TILE) {
            const double nb = (sm.o.nbp[0][tid] + sm.o.nbp[1][tid]) + (sm.o.nbp[2][tid] + sm.o.nbp[3][tid]);
            sm.o.wtn[tid] = sm.o.wt[tid] * nb;
            if (a.nbar_out != nullptr && pp < p1) {
                const int k = pp / a.nstates, s = pp - k * a.nstates;
                const int q = a.spinor ? k : k * a.nspin + ch;
                double* out = a.nbar_out + static_cast<int64_t>(q) * a.nspecies * a.nstates + s;
                if (writer) out[static_cast<int64_t>(T) * a.nstates] = nb;
                // species ids without a site: N-bar 0 (written by site 0)
                if (site == 0)
                    for (int T2 = 0; T2 < a.nspecies; ++T2)
                        if (a.species_orb_ptr[T2] == a.species_orb_ptr[T2 + 1])
                            out[static_cast<int64_t>(T2) * a.nstates] = 0.0;
            }
        }
        __syncthreads();
        if (worker) {
            const int xa = ra / L, ma = ra % L, xb = rb / L, mb = rb % L;
            const int nt = min(TILE, p1 - t0);
            for (int t = slice; t < nt; t += nslice) {
                const double ar = sm.o.cs[xa][ma][t][0], ai = sm.o.cs[xa][ma][t][1];
                const double br = sm.o.cs[xb][mb][t][0], bi = sm.o.cs[xb][mb][t][1];
                const double re = ar * br + ai * bi;
                const double im = ar * bi - ai * br;
                nr = fma(sm.o.wt[t], re, nr);
                ni = fma(sm.o.wt[t], im, ni);
                pr = fma(sm.o.wtn[t], re, pr);
                pi = fma(sm.o.wtn[t], im, pi);
            }
        }
        __syncthreads();
    }
    sm.o.red[tid][0] = nr;
    sm.o.red[tid][1] = ni;
    sm.o.red[tid][2] = pr;
    sm.o.red[tid][3] = pi;
    __syncthreads();
    {
        double* w = a.ws + ((static_cast<int64_t>(site) * nchan + ch) * a.nsplit + split) * (HUB_OCC_PAIRS * 4);
        for (int o = tid; o < npairs; o += NB) {
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int z = 0; z < nslice; ++z)
                for (int r = 0; r < 4; ++r) v[r] += sm.o.red[z * npairs + o][r];
            for (int r = 0; r < 4; ++r) w[o * 4 + r] = v[r];
        }
    }
}

__global__ void __launch_bounds__(NB) k_step_occ_final(const OccArgs a, const Acbn0Args u) {
    const int site = blockIdx.x;
    const int nchan = a.spinor ? 1 : a.nspin;
    __shared__ AcbLds sm;
    // the site's tensor first: its loads overlap the sums below
    const bool tens = isnan(u.ueff_fixed[site]);
    if (tens) {
        const int L = a.site_L[site];
        const double* Tg = u.tensor + static_cast<int64_t>(site) * 2401;
#pragma unroll 4
        for (int o = threadIdx.x; o < L * L * L * L; o += NB) sm.Ts[o] = Tg[o];
    }
    if (nchan == 2)
        occ_final_sums<2>(a, site, 0, 2, a.n, a.pbar, sm.Nf, sm.P);
    else
        for (int ch = 0; ch < nchan; ++ch) occ_final_sums<1>(a, site, ch, nchan, a.n, a.pbar, sm.Nf, sm.P);
    __syncthreads();
    acbn0_site(u, site, sm, tens);
}

// ---------------------------------------------------------------- energy
// E_U = Ueff/2 sum_channels Tr[n - n n] (Eq. E_Dudarev); spinor: the 2L x 2L
// matrix of App. A.  Unpolarized contexts count their channel twice.
__global__ void k_energy(const EnergyArgs a) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= a.nsites) return;
    const int L = a.site_L[site];
    const double* nb = a.n + static_cast<int64_t>(site) * a.nblk * 98;
    double val = 0.0;
    if (a.nblk == 4) {
        const int M = 2 * L;
        auto el = [&](int i, int j, int r) {
            const int x = i / L, y = j / L;
            return nb[((2 * x + y) * 49 + (i % L) * 7 + (j % L)) * 2 + r];
        };
        for (int i = 0; i < M; ++i) {
            val += el(i, i, 0);
            for (int j = 0; j < M; ++j) val -= el(i, j, 0) * el(j, i, 0) - el(i, j, 1) * el(j, i, 1);
        }
    } else {
        for (int b = 0; b < a.nblk; ++b) {
            const double* m = nb + b * 98;
            double v = 0.0;
            for (int i = 0; i < L; ++i) {
                v += m[(i * 7 + i) * 2];
                for (int j = 0; j < L; ++j)
                    v -= m[(i * 7 + j) * 2] * m[(j * 7 + i) * 2] - m[(i * 7 + j) * 2 + 1] * m[(j * 7 + i) * 2 + 1];
            }
            val += (a.nblk == 1) ? 2.0 * v : v;
        }
    }
    a.EU[site] = 0.5 * a.Ueff[site] * val;
}

// ---------------------------------------------------------------- FLL terms
// App. A, per site from the diagonal elements d(s,t,a) = n^{st}_aa: the shell
// electron count N, the magnetization m_i = sum_st (sigma_i)_st rho^{st}
// (rho^{st} = sum_a d(s,t,a)), the double counting
// E_DC = U/2 N(N-1) - J/2 N(N/2-1) - J/4 m.m and the Hartree-Fock energy
// written for m-diagonal occupations.  Collinear blocks have no
// spin-off-diagonal part; an unpolarized block stands for both spins.
__global__ void k_fll(const FllArgs a) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= a.nsites) return;
    const int L = a.site_L[site];
    const double* nb = a.n + static_cast<int64_t>(site) * a.nblk * 98;
    // d(s,t,a) as (re, im); zero where the storage has no such block
    auto d = [&](int s, int t, int o, double& re, double& im) {
        int blk = -1;
        if (a.nblk == 4) blk = 2 * s + t;
        else if (s == t) blk = a.nblk == 2 ? s : 0;
        if (blk < 0) { re = im = 0.0; return; }
        re = nb[blk * 98 + (o * 7 + o) * 2];
        im = nb[blk * 98 + (o * 7 + o) * 2 + 1];
    };
    double rr[2][2], ri[2][2];          // rho^{st}
    double sdd[2] = {0.0, 0.0};         // sum_a d(s,s,a)^2
    double xr[2] = {0.0, 0.0}, xi[2] = {0.0, 0.0};   // sum_a d(s,o,a) d(o,s,a)
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) {
            rr[s][t] = ri[s][t] = 0.0;
            for (int o = 0; o < L; ++o) {
                double re, im;
                d(s, t, o, re, im);
                rr[s][t] += re;
                ri[s][t] += im;
            }
        }
    for (int s = 0; s < 2; ++s)
        for (int o = 0; o < L; ++o) {
            double ar, ai, br, bi, cr, ci;
            d(s, s, o, ar, ai);
            sdd[s] += ar * ar - ai * ai;
            d(s, 1 - s, o, br, bi);
            d(1 - s, s, o, cr, ci);
            xr[s] += br * cr - bi * ci;
            xi[s] += br * ci + bi * cr;
        }
    const double U = a.U[site], J = a.J[site];
    const double N = rr[0][0] + rr[1][1];
    const double m[3] = {2.0 * rr[0][1], 2.0 * ri[0][1], rr[0][0] - rr[1][1]};
    const double mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    const double edc = 0.5 * U * N * (N - 1.0) - 0.5 * J * N * (0.5 * N - 1.0) - 0.25 * J * mm;
    double eee = 0.0;
    for (int s = 0; s < 2; ++s) {
        const int o = 1 - s;
        // sum_{a,b} d(s,s,a) d(o,o,b), sum_{a!=b} d(s,o,a) d(o,s,b), sum_{a!=b} d(s,s,a) d(s,s,b)  (real parts)
        const double same = rr[s][s] * rr[o][o] - ri[s][s] * ri[o][o];
        const double flip = (rr[s][o] * rr[o][s] - ri[s][o] * ri[o][s]) - xr[s];
        const double par = (rr[s][s] * rr[s][s] - ri[s][s] * ri[s][s]) - sdd[s];
        eee += 0.5 * U * same - 0.5 * U * xr[s] - 0.5 * J * flip + 0.5 * (U - J) * par;
    }
    double* out = a.out + static_cast<int64_t>(site) * 6;
    out[0] = N;
    out[1] = m[0];
    out[2] = m[1];
    out[3] = m[2];
    out[4] = edc;
    out[5] = eee;
}

// ---------------------------------------------------------------- forces
// F_i = g_s 2 Re sum_q w_k sum_col f_s sum_a conj(d_{a,i}(col)) B_a(col),
// B = V c as in the apply kernel (Sec. IV with U_eff fixed).  One
// work-group of NBF threads per site: the site's potential blocks V are
// formed once in LDS, then each thread takes (state set, column) pairs (one
// each for up to NBF pairs per site), holds the pair's L (two spin
// components: 2L) projections in registers and forms B from them; the
// threads' sums are added within each wave (butterfly) and then over the
// waves in order.
constexpr int NBF = 1024;
__global__ void __launch_bounds__(NBF) k_forces(const ForceArgs a) {
    const int site = blockIdx.x;
    const int L = a.site_L[site];
    const int orb0 = a.site_orb0[site];
    const int NC = a.ncplx;
    const double U = a.ueff[site];
    const int tid = threadIdx.x;
    // V[blk][a][b] = U (delta_ab / 2 on the spin-diagonal blocks - n_blk[b][a])
    __shared__ double V[4][7][7][2];
    const double* nb = a.n + static_cast<int64_t>(site) * a.nblk * 98;
    for (int o = tid; o < a.nblk * 49; o += NBF) {
        const int blk = o / 49, r = o - blk * 49, ai = r / 7, b = r - ai * 7;
        const bool diag = a.spinor ? (blk == 0 || blk == 3) : true;
        V[blk][ai][b][0] = U * ((ai == b && diag) ? 0.5 : 0.0) - U * nb[blk * 98 + (b * 7 + ai) * 2];
        V[blk][ai][b][1] = -U * nb[blk * 98 + (b * 7 + ai) * 2 + 1];
    }
    __syncthreads();
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t total = static_cast<int64_t>(a.nq) * a.ncol;
    for (int64_t o = tid; o < total; o += NBF) {
        const int q = static_cast<int>(o / a.ncol);
        const int col = static_cast<int>(o % a.ncol);
        const int k = a.spinor ? q : q / a.nspin;
        const int ch = a.spinor ? 0 : q % a.nspin;
        const int s = a.spinor ? col / 2 : col;
        const double wf = a.kweights[k] * a.f[static_cast<int64_t>(q) * a.nstates + s];
        if (wf == 0.0) continue;
        const double* cq = a.c + (static_cast<int64_t>(q) * a.J + orb0) * a.ncol * NC;
        // the pair's projections: component t of spinor column 2s + sigma is
        // column 2s + t; collinear columns use t = 0 only
        const int sg = col & 1, base = a.spinor ? col - sg : col;
        const int nt = a.spinor ? 2 : 1;
        double cr[2][7], ci[2][7];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int b = 0; b < 7; ++b) {
                const bool use = t < nt && b < L;
                const double* p = cq + (static_cast<int64_t>(b) * a.ncol + base + t) * NC;
                cr[t][b] = use ? p[0] : 0.0;
                ci[t][b] = (use && NC == 2) ? p[1] : 0.0;
            }
#pragma unroll
        for (int ai = 0; ai < 7; ++ai) {
            if (ai >= L) break;
            double br = 0.0, bi = 0.0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (t >= nt) break;
                const int blk = a.spinor ? 2 * t + sg : ch;
#pragma unroll
                for (int b = 0; b < 7; ++b) {
                    if (b >= L) break;
                    const double vr = V[blk][ai][b][0], vi = V[blk][ai][b][1];
                    br += vr * cr[t][b] - vi * ci[t][b];
                    bi += vr * ci[t][b] + vi * cr[t][b];
                }
            }
            for (int i = 0; i < 3; ++i) {
                const double* dp = a.d + ((static_cast<int64_t>(q) * a.J * 3 + (orb0 + ai) * 3 + i) * a.ncol + col) * NC;
                const double dr = dp[0], di = (NC == 2) ? dp[1] : 0.0;
                acc[i] += wf * (a.imag ? (dr * bi - di * br) : (dr * br + di * bi));   // Re or Im of conj(d) B
            }
        }
    }
    __shared__ double red[NBF / 64][3];
    for (int m = 32; m >= 1; m >>= 1)
        for (int i = 0; i < 3; ++i) acc[i] += __shfl_xor(acc[i], m, 64);
    if ((tid & 63) == 0)
        for (int i = 0; i < 3; ++i) red[tid >> 6][i] = acc[i];
    __syncthreads();
    if (tid == 0) {
        const double gs = (a.nblk == 1) ? 2.0 : 1.0;
        for (int i = 0; i < 3; ++i) {
            double v = 0.0;
            for (int w = 0; w < NBF / 64; ++w) v += red[w][i];
            a.F[site * 3 + i] = a.scale * (gs * 2.0 * v);
        }
    }
}

// ---------------------------------------------------------------- gauge
// Tables of the velocity-gauge phases (Sec. V): the image phases with the
// crystal momentum shifted by A and the phase of every cell grid point.
__global__ void __launch_bounds__(256) k_gauge_tables(const GaugeArgs a) {
    const int64_t G = static_cast<int64_t>(a.ngrid[0]) * a.ngrid[1] * a.ngrid[2];
    const int64_t nph = static_cast<int64_t>(a.nk) * a.nimg;
    const double two_pi = 6.283185307179586;
    for (int64_t o = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; o < G + nph;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double t;
        double* out;
        if (o < G) {
            const int64_t iz = o % a.ngrid[2];
            const int64_t iy = (o / a.ngrid[2]) % a.ngrid[1];
            const int64_t ix = o / (static_cast<int64_t>(a.ngrid[2]) * a.ngrid[1]);
            t = (a.A[0] * (ix * a.h[0]) + a.A[1] * (iy * a.h[1])) + a.A[2] * (iz * a.h[2]);
            out = a.pg + 2 * o;
        } else {
            const int64_t j = o - G;
            const int k = static_cast<int>(j / a.nimg), im = static_cast<int>(j % a.nimg);
            const int32_t* n = a.images + 3 * im;
            const double* kr = a.kred + 3 * k;
            t = 0.0;
            for (int i = 0; i < 3; ++i) t += two_pi * (kr[i] * n[i]) + a.A[i] * (n[i] * a.cell[i]);
            out = a.phase + 2 * j;
        }
        double sv, cv;
        sincos(t, &sv, &cv);
        out[0] = cv;
        out[1] = sv;
    }
}

// ---------------------------------------------------------------- fill
template <typename T>
__global__ void __launch_bounds__(256) k_zero_cols(T* __restrict__ p, int64_t rows, int64_t ld, int ncol) {
    const int64_t total = rows * ncol;
    for (int64_t o = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; o < total;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t r = o / ncol;
        p[r * ld + (o - r * ncol)] = T(0);
    }
}

}  // namespace

hipError_t launch_gauge_tables(const GaugeArgs& a, hipStream_t st) {
    const int64_t total = static_cast<int64_t>(a.ngrid[0]) * a.ngrid[1] * a.ngrid[2] +
                          static_cast<int64_t>(a.nk) * a.nimg;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_gauge_tables, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, int nq, hipStream_t st) {
    if (a.nrows <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    dim3 grid((a.ncol + 255) / 256, a.nrows, nq);
    hipLaunchKernelGGL(k_reduce, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reduce_grouped(const ReduceGroupedArgs& a, int nq, hipStream_t st) {
    if (a.J <= 0 || nq <= 0 || a.ncol <= 0) return hipSuccess;
    if (a.ncomp > 1 && !a.mout) return hipErrorInvalidValue;
    dim3 grid((a.ncol + 63) / 64, a.J, nq * (a.ncomp > 1 ? a.ncomp : 1));
    // many rows per orbital (overlapping spheres, small chunks): 16 waves
    const bool wide = a.rows_per_orbital >= 64;
    if (a.ncplx == 2) {
        if (wide) hipLaunchKernelGGL((k_reduce_grouped<16, 2>), grid, dim3(16 * 64), 0, st, a);
        else hipLaunchKernelGGL((k_reduce_grouped<4, 2>), grid, dim3(4 * 64), 0, st, a);
    } else {
        if (wide) hipLaunchKernelGGL((k_reduce_grouped<16, 1>), grid, dim3(16 * 64), 0, st, a);
        else hipLaunchKernelGGL((k_reduce_grouped<4, 1>), grid, dim3(4 * 64), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_nbar(const NbarArgs& a, int nq, hipStream_t st) {
    if (a.nstates <= 0 || nq <= 0) return hipSuccess;
    dim3 grid((a.nstates + 63) / 64, a.nspecies, nq);
    hipLaunchKernelGGL(k_nbar, grid, dim3(NBPART * 64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_occ(const OccArgs& a, int site0, int nsites, hipStream_t st) {
    OccArgs b = a;
    b.site_L += site0;
    b.site_orb0 += site0;
    b.site_species += site0;
    b.n += static_cast<int64_t>(site0) * a.nblk * 98;
    if (b.pbar) b.pbar += static_cast<int64_t>(site0) * a.nblk * 98;
    const int nchan = a.spinor ? 1 : a.nspin;
    hipLaunchKernelGGL(k_occ_part, dim3(nsites, nchan, a.nsplit), dim3(NB), 0, st, b);
    hipLaunchKernelGGL(k_occ_final, dim3(nsites, nchan), dim3(NB), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_step_occ(const OccArgs& a, const Acbn0Args& u, hipStream_t st) {
    const int nsites = static_cast<int>(a.nsites);
    if (nsites <= 0) return hipSuccess;
    const int nchan = a.spinor ? 1 : a.nspin;
    hipLaunchKernelGGL(k_step_occ_part, dim3(nsites, nchan, a.nsplit), dim3(NB), 0, st, a);
    hipLaunchKernelGGL(k_step_occ_final, dim3(nsites), dim3(NB), 0, st, a, u);
    return hipGetLastError();
}

hipError_t launch_acbn0(const Acbn0Args& a, int site0, int nsites, hipStream_t st) {
    Acbn0Args b = a;
    b.site_L += site0;
    b.ueff_fixed += site0;
    b.n += static_cast<int64_t>(site0) * a.nblk * 98;
    b.pbar += static_cast<int64_t>(site0) * a.nblk * 98;
    b.tensor += static_cast<int64_t>(site0) * 2401;
    b.U += site0;
    b.J += site0;
    b.Ueff += site0;
    if (b.status) b.status += site0;
    hipLaunchKernelGGL(k_acbn0, dim3(nsites), dim3(NB), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_fll(const FllArgs& a, hipStream_t st) {
    if (a.nsites <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fll, dim3((a.nsites + 63) / 64), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_energy(const EnergyArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_energy, dim3((a.nsites + 63) / 64), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_forces(const ForceArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_forces, dim3(a.nsites), dim3(NBF), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_zero_cols(void* p, int elem_bytes, int64_t rows, int64_t ld, int ncol, hipStream_t st) {
    if (rows <= 0 || ncol <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((rows * ncol + 255) / 256, 8192);
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_zero_cols<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                           static_cast<double*>(p), rows, ld, ncol);
    else
        hipLaunchKernelGGL(k_zero_cols<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                           static_cast<float*>(p), rows, ld, ncol);
    return hipGetLastError();
}
