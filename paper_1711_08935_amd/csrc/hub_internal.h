// Internal declarations shared by the host builder, the C-ABI layer and the
// HIP kernels of the Hubbard library.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <vector>

#include "hub.h"

// One work-list chunk: a run of sphere entries of one site inside one apply
// layer, all with the same lattice image (so one Bloch phase serves the whole
// chunk).  Within a layer no two entries share a grid point, so chunks of the
// same layer can be applied concurrently without atomics.
struct HubChunk {
    int32_t site;
    int32_t layer;
    int32_t e0;      // first entry
    int32_t ne;      // entries, padded to a multiple of HUB_ENTRY_ALIGN
    int32_t L;       // orbitals of the site (2l+1)
    int32_t orb0;    // global index j of the site's first orbital
    int32_t part0;   // first row of this chunk in the projection workspace
    int32_t species;
    int64_t phi0;    // offset of the chunk's orbital values (entries * L)
    int32_t img;     // lattice image shared by every entry of the chunk
    int32_t nreal;   // real entries; entries nreal..ne-1 repeat the last grid
                     // point with zero orbital values
};

// Chunk entry lists are padded to a multiple of this many entries, so that
// every wave's share (1, 2 or 4 waves per work-group) holds whole batches of
// the kernels' entry loops (at most 8 entries).
#define HUB_ENTRY_ALIGN 32

struct SiteDef {
    double R[3];
    int l;
    double zeta;
    double rc;
    int species;
    double ueff_fixed;   // NaN: ACBN0
    double zeta_dn;      // spin-down exponent of spinor orbitals; NaN: zeta
};

// Host copy of one site's sphere, points sorted by (g, image).
struct SiteSphere {
    std::vector<int32_t> g;      // folded grid index
    std::vector<int32_t> img3;   // lattice image (3 per point)
    std::vector<int32_t> ijk;    // unfolded integer coordinates (3 per point)
    std::vector<double> phi;     // [p][m]
    std::vector<double> grad;    // [p][m][3]
    std::vector<double> phi_dn;  // [p][m], spin-down orbitals (spin-dependent contexts)
    std::vector<double> grad_dn; // [p][m][3], their gradients
};

// Largest number of functions (orbitals of all covering sites) a grouped
// chunk may carry; the covers of a point with more are split over passes
// of at most this many functions each.
#define HUB_GF_MAX 16

// Work list grouped by cover signature: every grid point covered by any
// sphere appears in one grouped chunk per pass, together with its
// (site, image) covers in a fixed slot order, so the projection reads each
// state row once per pass and the apply writes it once per pass.  The
// chunk's functions are the concatenated orbitals of its slots; a point with
// more than HUB_GF_MAX functions has its slots split over several passes.
struct GroupTables {
    bool ok = false;
    int nfmax = 0;                           // most functions covering one grid point
    int npass = 1;                           // apply passes (chunk.layer): points with more
                                             // than HUB_GF_MAX functions are split over passes
    std::vector<HubChunk> chunks;            // L = number of functions, e0/ne over points
    std::vector<int32_t> gidx;               // per point
    std::vector<double> tab;                 // per point, L values (slot-major)
    // position moments (velocity-gauge current): per point (in gidx order)
    // the displacement of its unfolded position from the centre of the site
    // of its chunk's first cover, d0[point][3]; per chunk and function the
    // offset from that displacement to the one about the function's own
    // site, fdel[chunk][HUB_GF_MAX][3] (constant over a chunk's points)
    std::vector<double> d0;
    std::vector<double> fdel;
    std::vector<int32_t> f_orb;              // per chunk HUB_GF_MAX: global orbital j of function f
    std::vector<int32_t> f_img;              // per chunk HUB_GF_MAX: lattice image of function f
    std::vector<int32_t> red_ptr;            // CSR orbital j -> workspace rows
    std::vector<int32_t> red_row, red_img;
    int64_t part_rows = 0;
};

struct HostTables {
    int nsites = 0, J = 0, nlayers = 0, nspecies = 0;
    std::vector<int32_t> site_L, site_orb0, site_species;
    std::vector<HubChunk> chunks;            // sorted by (layer, site)
    std::vector<int32_t> gidx, img;          // per entry
    std::vector<double> phi;                 // per entry, L values
    std::vector<double> gphi;                // per entry, 3L values [m][i]
    std::vector<double> mphi;                // per entry, 3L values [m][i]: (r_p - R)_i phi_m
    // Spin-dependent orbitals (some site has a spin-down exponent): per
    // entry 2L values [sigma][m], the orbital of each spin component (sites
    // without one repeat their orbital); the grouped list then carries 2L
    // functions per cover as well.
    bool spindep = false;
    std::vector<double> phi2;
    std::vector<double> gphi_dn, mphi_dn;    // per entry, 3L values [m][i] of the spin-down orbitals
    std::vector<int32_t> images;             // unique lattice images, 3 per image
    std::vector<int32_t> site_chunk_ptr;     // CSR site -> chunk ids
    std::vector<int32_t> site_chunk_ids;
    std::vector<int32_t> layer_chunk_ptr;    // chunks of layer l: [ptr[l], ptr[l+1])
    std::vector<int32_t> layer_site_ptr;     // chunk range of (layer, site): [l*nsites+s]
    std::vector<int32_t> species_orb_ptr;    // CSR species -> orbital j
    std::vector<int32_t> species_orb_ids;
    std::vector<int32_t> orb_site;           // j -> site
    int64_t part_rows = 0;                   // sum of L over chunks
    int64_t nentries = 0;
    std::vector<SiteSphere> spheres;
    GroupTables grouped;
};

// Work list of the state-gradient force form (Sec. IV): <phi|D_i psi>, D_i
// the 4th-order central difference along axis i, equals by summation by
// parts -dV sum over the dilated sphere (every unfolded point within two
// steps of a sphere point along an axis) of exp(i k.T) (D_i phi)(p)
// psi(g(p)), with phi zero outside the sphere.  The table holds D_i phi, so
// the projection machinery of the orbital gradients computes
// d = dV sum exp(i k.T) (D phi) psi = -<phi|D psi> and the force contraction
// is shared.  Chunks are per (site, image) as in one layer of the layered
// list; the projection needs no layers.
struct StencilTables {
    std::vector<HubChunk> chunks;            // site-major, then image, g ascending
    std::vector<int32_t> gidx;               // per entry
    std::vector<double> tab;                 // per entry, 3L values [m][i]
    std::vector<double> tab_dn;              // the same for the spin-down orbitals (spin-dependent contexts)
    std::vector<int32_t> site_chunk_ptr;     // CSR site -> chunk ids
    std::vector<int32_t> site_chunk_ids;
    int64_t part_rows = 0;                   // sum of L over chunks
    int64_t nentries = 0;                    // real (unpadded) entries
};

// Host builder (sphere.cpp).  Returns HUB_OK or a negative status.
int hub_build_host(const double cell[3], const int ngrid[3], const std::vector<SiteDef>& sites,
                   int chunk_entries, HostTables& out);

// Closed-form average of 1/|r| over one grid cell centred at the origin.
double hub_g0_cell_average(const double h[3]);

// Dilated-sphere tables of the state-gradient force form from the spheres of
// ``T`` (sphere.cpp).  Every image it needs is in T.images (hub_build_host
// registers the images of the points two steps past each sphere point).
int hub_build_stencil(const double cell[3], const int ngrid[3], const std::vector<SiteDef>& sites,
                      const HostTables& T, int chunk_entries, StencilTables& out);
