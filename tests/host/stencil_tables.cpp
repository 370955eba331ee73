// Host check of the state-gradient work list built by the library's sphere
// builder (no GPU): reads a system and complex states for one k-point, builds
// the sphere and dilated-sphere tables, checks every index against its
// buffer, and writes d[j][i][s] = dV sum_chunks exp(i k.T) sum_entries
// tab[e][m][i] psi[g_e][s] (the sum the projection kernels evaluate), for
// comparison with the oracle's -<phi|D psi>.
//
// Input (binary, native endianness): cell[3] f64, ngrid[3] i32, nsites i32,
// per site {R[3] f64, l i32, zeta f64, rc f64, species i32, zeta_dn f64
// (NaN: none)}, k_red[3] f64, nstates i32, psi[G][nstates] complex f64.
// Output: d as complex f64, then (if some site has a spin-down exponent) the
// same sum over the spin-down orbitals' table.
// Exit status 0 (ok), 1 (bad input or builder error), 2 (an index out of range).
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "hub_internal.h"

namespace {
template <typename T>
bool get(FILE* f, T* p, size_t n) { return std::fread(p, sizeof(T), n, f) == n; }
}  // namespace

int main(int argc, char** argv) {
    if (argc != 3) return 1;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 1;
    double cell[3], k[3];
    int ngrid[3], ns = 0, S = 0;
    bool ok = get(f, cell, 3) && get(f, ngrid, 3) && get(f, &ns, 1) && ns > 0;
    std::vector<SiteDef> sites(ok ? ns : 0);
    for (auto& s : sites) {
        ok = ok && get(f, s.R, 3) && get(f, &s.l, 1) && get(f, &s.zeta, 1) && get(f, &s.rc, 1) &&
             get(f, &s.species, 1) && get(f, &s.zeta_dn, 1);
        s.ueff_fixed = NAN;
    }
    ok = ok && get(f, k, 3) && get(f, &S, 1) && S > 0;
    const long G = static_cast<long>(ngrid[0]) * ngrid[1] * ngrid[2];
    std::vector<std::complex<double>> psi(ok ? G * S : 0);
    ok = ok && get(f, psi.data(), psi.size());
    std::fclose(f);
    if (!ok) return 1;

    HostTables T;
    if (hub_build_host(cell, ngrid, sites, 256, T) != HUB_OK) return 1;
    StencilTables X;
    if (hub_build_stencil(cell, ngrid, sites, T, 256, X) != HUB_OK) return 1;
    const long nimg = static_cast<long>(T.images.size() / 3);
    long bad = 0, tab_used = 0;
    for (int s = 0; s < ns; ++s)
        for (int t = X.site_chunk_ptr[s]; t < X.site_chunk_ptr[s + 1]; ++t) {
            const HubChunk& C = X.chunks[X.site_chunk_ids[t]];
            bad += C.site != s || C.L != T.site_L[s] || C.orb0 != T.site_orb0[s];
            bad += C.e0 < 0 || C.e0 + static_cast<long>(C.ne) > static_cast<long>(X.gidx.size());
            bad += C.phi0 != tab_used;
            bad += (C.phi0 + static_cast<long>(C.ne) * C.L) * 3 > static_cast<long>(X.tab.size());
            bad += C.img < 0 || C.img >= nimg || C.part0 < 0 || C.part0 + C.L > X.part_rows;
            bad += C.ne % HUB_ENTRY_ALIGN != 0 || C.nreal <= 0 || C.nreal > C.ne;
            tab_used += static_cast<long>(C.ne) * C.L;
        }
    for (int g : X.gidx) bad += g < 0 || g >= G;
    bad += T.spindep ? X.tab_dn.size() != X.tab.size() : !X.tab_dn.empty();
    std::printf("chunks %zu entries %ld sphere_entries %ld images %ld bad %ld\n", X.chunks.size(),
                static_cast<long>(X.nentries), static_cast<long>(T.nentries), nimg, bad);
    if (bad) return 2;

    const double dV = cell[0] / ngrid[0] * cell[1] / ngrid[1] * cell[2] / ngrid[2];
    FILE* o = std::fopen(argv[2], "wb");
    if (!o) return 1;
    bool wrote = true;
    for (const std::vector<double>* tab : {&X.tab, &X.tab_dn}) {
    if (tab->empty()) continue;
    std::vector<std::complex<double>> d(static_cast<size_t>(T.J) * 3 * S);
    for (const HubChunk& C : X.chunks) {
        const int32_t* im = &T.images[3 * C.img];
        const double a = 2.0 * M_PI * (k[0] * im[0] + k[1] * im[1] + k[2] * im[2]);
        const std::complex<double> ph(std::cos(a), std::sin(a));
        for (int e = 0; e < C.ne; ++e) {
            const long g = X.gidx[C.e0 + e];
            for (int fn = 0; fn < 3 * C.L; ++fn) {
                const double w = (*tab)[(C.phi0 + static_cast<long>(e) * C.L) * 3 + fn];
                for (int c = 0; c < S; ++c) d[(static_cast<size_t>(C.orb0) * 3 + fn) * S + c] += dV * ph * w * psi[g * S + c];
            }
        }
    }
    wrote = wrote && std::fwrite(d.data(), sizeof(d[0]), d.size(), o) == d.size();
    }
    std::fclose(o);
    return wrote ? 0 : 1;
}
