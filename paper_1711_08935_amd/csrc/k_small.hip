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
// serves 64 columns of one (j, q); its RW waves take interleaved rows with
// four independent partial sums each (many loads in flight), and the partial
// sums are combined in a fixed order.  RW follows the rows per orbital.
constexpr int RW = 16;   // waves of the N-bar kernel and of the wide reduction
template <int RW>
__global__ void __launch_bounds__(RW * 64) k_reduce_grouped(const ReduceGroupedArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane;
    const int j = blockIdx.y;
    const int q = blockIdx.z;
    const bool active = col < a.ncol;
    const int NC = a.ncplx;
    const int k = a.spinor ? a.q0 + q : (a.q0 + q) / a.nspin;
    const double* ph = a.phase + static_cast<int64_t>(k) * a.nimg * 2;
    // spin-dependent orbitals: spinor column 2s + sigma reads the rows of the
    // orbital of its spin component
    const int64_t shift = (a.spin_shift && (col & 1)) ? a.spin_shift[j] : 0;
    const double* base = a.part + (static_cast<int64_t>(q) * a.prows + shift) * a.ncol * NC +
                         static_cast<int64_t>(active ? col : 0) * NC;
    double s0[4] = {0.0, 0.0, 0.0, 0.0}, s1[4] = {0.0, 0.0, 0.0, 0.0};
    const int t0 = a.red_ptr[j], t1 = a.red_ptr[j + 1];
    int t = t0 + wave;
    for (; t + 3 * RW < t1; t += 4 * RW) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int tt = t + u * RW;
            const double* p = base + static_cast<int64_t>(a.red_row[tt]) * a.ncol * NC;
            if (NC == 2) {
                const int im = a.red_img[tt];
                const double pr = ph[2 * im], pi = ph[2 * im + 1];
                s0[u] += pr * p[0] - pi * p[1];
                s1[u] += pr * p[1] + pi * p[0];
            } else {
                s0[u] += p[0];
            }
        }
    }
    for (; t < t1; t += RW) {
        const double* p = base + static_cast<int64_t>(a.red_row[t]) * a.ncol * NC;
        if (NC == 2) {
            const int im = a.red_img[t];
            const double pr = ph[2 * im], pi = ph[2 * im + 1];
            s0[0] += pr * p[0] - pi * p[1];
            s1[0] += pr * p[1] + pi * p[0];
        } else {
            s0[0] += p[0];
        }
    }
    __shared__ double red[RW][64][2];
    red[wave][lane][0] = (s0[0] + s0[1]) + (s0[2] + s0[3]);
    red[wave][lane][1] = (s1[0] + s1[1]) + (s1[2] + s1[3]);
    __syncthreads();
    if (wave != 0 || !active) return;
    double r0 = 0.0, r1 = 0.0;
    for (int w = 0; w < RW; ++w) {
        r0 += red[w][lane][0];
        r1 += red[w][lane][1];
    }
    double* o = a.out + ((static_cast<int64_t>(q) * a.J + j) * a.ncol + col) * NC;
    o[0] = a.dV * r0;
    if (NC == 2) o[1] = a.dV * r1;
}

// ---------------------------------------------------------------- N-bar
// nbar[q][T][s] = sum_{j in species T} sum_{columns of s} |c[q][j][col]|^2.
// A work-group serves 64 states of one (T, q); its RW waves take
// interleaved orbitals with four independent sums each, combined in order.
__global__ void __launch_bounds__(RW * 64) k_nbar(const NbarArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int s = blockIdx.x * 64 + lane;
    const int T = blockIdx.y;
    const int q = blockIdx.z;
    const bool active = s < a.nstates;
    const int NC = a.ncplx;
    const int cps = a.spinor ? 2 : 1;
    const double* cq = a.c + static_cast<int64_t>(q) * a.J * a.ncol * NC + static_cast<int64_t>(active ? s : 0) * cps * NC;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int t0 = a.species_orb_ptr[T], t1 = a.species_orb_ptr[T + 1];
    int t = t0 + wave;
    auto term = [&](int tt) {
        const double* p = cq + static_cast<int64_t>(a.species_orb_ids[tt]) * a.ncol * NC;
        double v = 0.0;
        for (int x = 0; x < cps; ++x) {
            v = fma(p[x * NC], p[x * NC], v);
            if (NC == 2) v = fma(p[x * NC + 1], p[x * NC + 1], v);
        }
        return v;
    };
    for (; t + 3 * RW < t1; t += 4 * RW) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += term(t + u * RW);
    }
    for (; t < t1; t += RW) acc[0] += term(t);
    __shared__ double red[RW][64];
    red[wave][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (wave != 0 || !active) return;
    double r = 0.0;
    for (int w = 0; w < RW; ++w) r += red[w][lane];
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

__global__ void __launch_bounds__(NB) k_occ_final(const OccArgs a) {
    const int site = blockIdx.x;
    const int ch = blockIdx.y;
    const int nchan = gridDim.y;
    const int L = a.site_L[site];
    const int ncp = a.spinor ? 2 * L : L;
    const double* w = a.ws + (static_cast<int64_t>(site) * nchan + ch) * a.nsplit * (HUB_OCC_PAIRS * 4);
    // write all blocks of this channel (zeros outside the L x L corner)
    const int nblk_here = a.spinor ? 4 : 1;
    for (int o = threadIdx.x; o < nblk_here * 49; o += NB) {
        const int blk = o / 49, e = o % 49, i = e / 7, j = e % 7;
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (i < L && j < L) {
            const int x = a.spinor ? blk / 2 : 0, y = a.spinor ? blk % 2 : 0;
            const int p = (x * L + i) * ncp + (y * L + j);
            for (int z = 0; z < a.nsplit; ++z)
                for (int r = 0; r < 4; ++r) v[r] += w[(static_cast<int64_t>(z) * HUB_OCC_PAIRS + p) * 4 + r];
        }
        const int oblk = a.spinor ? blk : ch;
        const int64_t base = ((static_cast<int64_t>(site) * a.nblk + oblk) * 49 + e) * 2;
        a.n[base] = v[0];
        a.n[base + 1] = v[1];
        if (a.pbar != nullptr) {
            a.pbar[base] = v[2];
            a.pbar[base + 1] = v[3];
        }
    }
}

// ---------------------------------------------------------------- ACBN0
// U-bar and J-bar of one site (Eqs. ACBN0_U, ACBN0_J; App. B), with the
// numerators read as P_mm' P_m''m''' (mm'|m''m''') and P_mm' P_m''m'''
// (mm'''|m''m'), denominators from the bare diagonal occupations.
__global__ void __launch_bounds__(NB) k_acbn0(const Acbn0Args a) {
    const int site = blockIdx.x;
    const int L = a.site_L[site];
    const int tid = threadIdx.x;
    const double fixed = a.ueff_fixed[site];
    if (!isnan(fixed)) {
        if (tid == 0) {
            a.U[site] = fixed;
            a.J[site] = 0.0;
            a.Ueff[site] = fixed;
            if (a.status) {
                // flag occupations that are not finite (NaN or Inf in the states)
                bool finite = true;
                const double* nb0 = a.n + static_cast<int64_t>(site) * a.nblk * 98;
                for (int b = 0; b < a.nblk; ++b)
                    for (int e = 0; e < L * L; ++e) {
                        const int64_t o = b * 98 + ((e / L) * 7 + e % L) * 2;
                        finite = finite && isfinite(nb0[o]) && isfinite(nb0[o + 1]);
                    }
                a.status[site] = finite ? 0 : HUB_ENONFINITE;
            }
        }
        return;
    }
    __shared__ double P[4][7][7][2];
    __shared__ double Nd[4][7][2];
    __shared__ double Ts[2401];
    __shared__ double redU[NB], redJ[NB];
    const int nb = a.nblk;
    for (int o = tid; o < nb * 49; o += NB) {
        const int b = o / 49, e = o % 49;
        const int64_t base = ((static_cast<int64_t>(site) * nb + b) * 49 + e) * 2;
        P[b][e / 7][e % 7][0] = a.pbar[base];
        P[b][e / 7][e % 7][1] = a.pbar[base + 1];
        if (e / 7 == e % 7) {
            Nd[b][e / 7][0] = a.n[base];
            Nd[b][e / 7][1] = a.n[base + 1];
        }
    }
    const int L2 = L * L, L4 = L2 * L2;
    const double* Tg = a.tensor + static_cast<int64_t>(site) * 2401;
    for (int o = tid; o < L4; o += NB) Ts[o] = Tg[o];
    __syncthreads();

    // channel layout: unpolarized -> both channels are block 0
    const int c0 = 0;
    const int c1 = (nb == 2) ? 1 : (nb == 4 ? 3 : 0);
    double su = 0.0, sj = 0.0;
    for (int o = tid; o < L4; o += NB) {
        const int ab = o / L2, cd = o % L2;
        const int A = ab / L, B = ab % L, Cc = cd / L, D = cd % L;
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
    redU[tid] = su;
    redJ[tid] = sj;
    __syncthreads();
    for (int w = NB / 2; w > 0; w >>= 1) {
        if (tid < w) {
            redU[tid] += redU[tid + w];
            redJ[tid] += redJ[tid + w];
        }
        __syncthreads();
    }
    if (tid != 0) return;
    double dU = 0.0, dJ = 0.0;
    if (nb != 4) {
        // collinear: N^alpha_m = n^alpha_mm (real part)
        double N[2][7];
        for (int m = 0; m < L; ++m) {
            N[0][m] = Nd[c0][m][0];
            N[1][m] = Nd[c1][m][0];
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
            return Nd[b1][m1][0] * Nd[b2][m2][0] - Nd[b1][m1][1] * Nd[b2][m2][1];
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
// B = V c as in the apply kernel (Sec. IV with U_eff fixed).
__global__ void __launch_bounds__(NB) k_forces(const ForceArgs a) {
    const int site = blockIdx.x;
    const int L = a.site_L[site];
    const int orb0 = a.site_orb0[site];
    const int NC = a.ncplx;
    const double U = a.ueff[site];
    const int tid = threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t total = static_cast<int64_t>(a.nq) * a.ncol;
    for (int64_t o = tid; o < total; o += NB) {
        const int q = static_cast<int>(o / a.ncol);
        const int col = static_cast<int>(o % a.ncol);
        const int k = a.spinor ? q : q / a.nspin;
        const int ch = a.spinor ? 0 : q % a.nspin;
        const int s = a.spinor ? col / 2 : col;
        const double wf = a.kweights[k] * a.f[static_cast<int64_t>(q) * a.nstates + s];
        if (wf == 0.0) continue;
        const double* cq = a.c + (static_cast<int64_t>(q) * a.J + orb0) * a.ncol * NC;
        const double* nb = a.n + static_cast<int64_t>(site) * a.nblk * 98;
        for (int ai = 0; ai < L; ++ai) {
            double br = 0.0, bi = 0.0;
            if (!a.spinor) {
                const double* nm = nb + ch * 98;
                for (int b = 0; b < L; ++b) {
                    const double vr = U * ((ai == b ? 0.5 : 0.0) - nm[(b * 7 + ai) * 2]);
                    const double vi = -U * nm[(b * 7 + ai) * 2 + 1];
                    const double cr = cq[(static_cast<int64_t>(b) * a.ncol + col) * NC];
                    const double ci = (NC == 2) ? cq[(static_cast<int64_t>(b) * a.ncol + col) * NC + 1] : 0.0;
                    br += vr * cr - vi * ci;
                    bi += vr * ci + vi * cr;
                }
            } else {
                const int sg = col & 1, base = col - sg;
                for (int t = 0; t < 2; ++t) {
                    const double* nm = nb + (2 * t + sg) * 98;
                    for (int b = 0; b < L; ++b) {
                        const double vr = U * ((ai == b && t == sg) ? 0.5 : 0.0) - U * nm[(b * 7 + ai) * 2];
                        const double vi = -U * nm[(b * 7 + ai) * 2 + 1];
                        const double cr = cq[(static_cast<int64_t>(b) * a.ncol + base + t) * 2];
                        const double ci = cq[(static_cast<int64_t>(b) * a.ncol + base + t) * 2 + 1];
                        br += vr * cr - vi * ci;
                        bi += vr * ci + vi * cr;
                    }
                }
            }
            for (int i = 0; i < 3; ++i) {
                const double* dp = a.d + ((static_cast<int64_t>(q) * a.J * 3 + (orb0 + ai) * 3 + i) * a.ncol + col) * NC;
                const double dr = dp[0], di = (NC == 2) ? dp[1] : 0.0;
                acc[i] += wf * (a.imag ? (dr * bi - di * br) : (dr * br + di * bi));   // Re or Im of conj(d) B
            }
        }
    }
    __shared__ double red[NB][3];
    for (int i = 0; i < 3; ++i) red[tid][i] = acc[i];
    __syncthreads();
    for (int w = NB / 2; w > 0; w >>= 1) {
        if (tid < w)
            for (int i = 0; i < 3; ++i) red[tid][i] += red[tid + w][i];
        __syncthreads();
    }
    if (tid == 0) {
        const double gs = (a.nblk == 1) ? 2.0 : 1.0;
        for (int i = 0; i < 3; ++i) a.F[site * 3 + i] = a.scale * (gs * 2.0 * red[0][i]);
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
    dim3 grid((a.ncol + 63) / 64, a.J, nq);
    // many rows per orbital (overlapping spheres, small chunks): 16 waves
    if (a.rows_per_orbital >= 64)
        hipLaunchKernelGGL(k_reduce_grouped<16>, grid, dim3(16 * 64), 0, st, a);
    else
        hipLaunchKernelGGL(k_reduce_grouped<4>, grid, dim3(4 * 64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_nbar(const NbarArgs& a, int nq, hipStream_t st) {
    if (a.nstates <= 0 || nq <= 0) return hipSuccess;
    dim3 grid((a.nstates + 63) / 64, a.nspecies, nq);
    hipLaunchKernelGGL(k_nbar, grid, dim3(RW * 64), 0, st, a);
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
    hipLaunchKernelGGL(k_forces, dim3(a.nsites), dim3(NB), 0, st, a);
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
