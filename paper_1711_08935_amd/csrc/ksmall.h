// Launch argument blocks of the small FP64 kernels (reduction, N-bar,
// occupations, ACBN0, energy, forces, Coulomb).
#pragma once

#include "kcommon.h"

struct ReduceArgs {
    const double* part; int64_t prows;    // workspace rows per state set
    double* out; int nrows;               // output rows per state set (J * mult)
    int ncol; int ncplx; int mult;
    int pmult;                            // workspace rows per chunk orbital (mult, or 2: spin-dependent)
    int spindep;                          // 1: column 2s + sigma reads the rows of orbital sigma L + m
    int colpar;                           // >= 0: write only the columns of this parity (spin component)
    const HubChunk* chunks;
    const int32_t* site_chunk_ptr; const int32_t* site_chunk_ids;
    const int32_t* orb_site; const int32_t* site_orb0; const int32_t* site_L;
    const double* phase; int nimg;        // exp(+i k.T) per k-point and image
    int nspin; int spinor;                // state set -> k-point
    int q0;                               // context index of the first state set of the launch
    double dV;
};

struct ReduceGroupedArgs {
    const double* part; int64_t prows;
    double* out; int J; int ncol; int ncplx;
    const int32_t* red_ptr; const int32_t* red_row; const int32_t* red_img;
    const double* phase; int nimg; int nspin; int spinor;
    int q0;                   // context index of the first state set of the launch
    double dV;
    int rows_per_orbital;     // average workspace rows per orbital (host)
    const int32_t* spin_shift;  // spin-dependent orbitals: per orbital, the rows from a
                                // spin-up function to its spin-down one (L); else null
    // ncomp = 4: the workspace also holds the position-moment projections
    // (component i + 1 at part + (i + 1) * pplane), reduced into
    // mout[q][3 j + i][col]
    int ncomp;                  // 1 or 4 (0 is taken as 1)
    double* mout;
    int64_t pplane;
};

struct NbarArgs {
    const double* c; double* nbar;
    int J; int ncol; int nstates; int ncplx; int spinor; int nspecies;
    const int32_t* species_orb_ptr; const int32_t* species_orb_ids;
};

// pairs (a, b) of a site's combined occupation matrix (2L x 2L, L <= 7)
#define HUB_OCC_PAIRS 196

struct OccArgs {
    const double* c; const double* f; const double* nbar;
    double* n; double* pbar;
    const double* kweights;
    const int32_t* site_L; const int32_t* site_orb0; const int32_t* site_species;
    int J; int ncol; int nstates; int ncplx; int spinor; int nspin; int nk; int nblk; int nspecies;
    int nsplit;               // (k-point, state) splits of the first pass
    double* ws;               // [site][channel][nsplit][HUB_OCC_PAIRS][4] partial sums
    // batched step kernels (k_step_occ_part / k_step_occ_final) only:
    int nsites;
    const int32_t* species_orb_ptr; const int32_t* species_orb_ids;   // N-bar from c
    double* nbar_out;         // [q][species][nstates] or null
};

// (k-point, state) splits of the occupation sums: about 64 pairs each
inline int hub_occ_splits(int nk, int nstates) {
    const int np = nk * nstates;
    const int s = (np + 63) / 64;
    return s < 1 ? 1 : (s > 64 ? 64 : s);
}

struct Acbn0Args {
    const double* n; const double* pbar; const double* tensor;   // tensor: [site][2401]
    const int32_t* site_L; const double* ueff_fixed;
    double* U; double* J; double* Ueff; int32_t* status;
    int nblk;
};

struct EnergyArgs {
    const double* n; const double* Ueff; double* EU;
    const int32_t* site_L; int nsites; int nblk;
};

// Per site: N, m_x, m_y, m_z, E_DC, E_ee (App. A).
struct FllArgs {
    const double* n; const double* U; const double* J; double* out;
    const int32_t* site_L; int nsites; int nblk;
};

struct ForceArgs {
    const double* c; const double* d; const double* f; const double* n; const double* ueff;
    const double* kweights; double* F;
    const int32_t* site_L; const int32_t* site_orb0;
    int nsites; int J; int ncol; int nstates; int ncplx; int spinor; int nspin; int nq; int nblk;
    int imag;                 // 0: 2 Re sum conj(d) B (forces); 1: 2 Im (current)
    double scale;             // multiplies the result
};

// Velocity-gauge tables for a uniform vector potential A:
// phase[k][img] = exp(i (k + A).T_img), pg[g] = exp(i A.r_g).
struct GaugeArgs {
    double A[3];
    double cell[3];
    double h[3];
    int ngrid[3];
    const int32_t* images; int nimg;     // lattice images (3 ints each)
    const double* kred; int nk;          // reduced k-points (3 each)
    double* phase;                       // [nk][nimg] (re, im)
    double* pg;                          // [G] (re, im)
};

struct CoulombArgs {
    const int32_t* ijk;        // unfolded integer coordinates of the site's points [P][3]
    const double* phi;         // [P][L]
    int P; int L; int npair;
    double* rho;               // scratch [P][npair]
    double* W;                 // scratch [P][npair]
    double* tensor;            // output [L^4]
    double h[3]; double g0; double dV;
};

hipError_t launch_reduce(const ReduceArgs& a, int nq, hipStream_t st);
hipError_t launch_reduce_grouped(const ReduceGroupedArgs& a, int nq, hipStream_t st);
hipError_t launch_nbar(const NbarArgs& a, int nq, hipStream_t st);
hipError_t launch_occ(const OccArgs& a, int site0, int nsites, hipStream_t st);
hipError_t launch_acbn0(const Acbn0Args& a, int site0, int nsites, hipStream_t st);
// N-bar, n, P-bar, U-bar, J-bar, U_eff of every site in two launches (batched step)
hipError_t launch_step_occ(const OccArgs& a, const Acbn0Args& u, hipStream_t st);
hipError_t launch_energy(const EnergyArgs& a, hipStream_t st);
hipError_t launch_forces(const ForceArgs& a, hipStream_t st);
hipError_t launch_fll(const FllArgs& a, hipStream_t st);
hipError_t launch_gauge_tables(const GaugeArgs& a, hipStream_t st);
hipError_t launch_coulomb(const CoulombArgs& a, hipStream_t st);
// p[r * ld + i] = 0 for every row r < rows and scalar i < ncol (elem_bytes 4
// or 8): clears the used columns of a state-layout buffer, padding untouched.
hipError_t launch_zero_cols(void* p, int elem_bytes, int64_t rows, int64_t ld, int ncol, hipStream_t st);
