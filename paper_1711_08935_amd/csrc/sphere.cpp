// Host-side setup of the Hubbard library: sphere maps, orbital tables and
// the layered work list.  Built with -ffp-contract=off: sphere membership is
// decided by the canonical FP64 expression d_i = j_i * h_i - R_i,
// |d|^2 = (dx*dx + dy*dy) + dz*dz <= rc*rc, which must not be contracted.
//
// Paper: localized orbitals on spherical sub-grids around the atoms, points
// outside the periodic box mapped back onto the grid with a phase (Sec. II
// and Fig. 1); sphere truncation radius (Sec. II, radius discussion).

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <tuple>

#include "hub_internal.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

// Real solid harmonics S_lm(x, y, z) = r^l Y_lm, m = -l..l, standard real
// combinations without the Condon-Shortley sign (p: y, z, x), and their
// gradients, written out as polynomials.
void solid_harmonics(int l, double x, double y, double z, double* S, double* dS) {
    switch (l) {
    case 0: {
        S[0] = 0.5 * std::sqrt(1.0 / kPi);
        dS[0] = dS[1] = dS[2] = 0.0;
        break;
    }
    case 1: {
        const double c = std::sqrt(3.0 / (4.0 * kPi));
        S[0] = c * y; dS[0] = 0; dS[1] = c; dS[2] = 0;
        S[1] = c * z; dS[3] = 0; dS[4] = 0; dS[5] = c;
        S[2] = c * x; dS[6] = c; dS[7] = 0; dS[8] = 0;
        break;
    }
    case 2: {
        const double a = std::sqrt(15.0 / (4.0 * kPi));
        const double b = std::sqrt(5.0 / (16.0 * kPi));
        const double c = std::sqrt(15.0 / (16.0 * kPi));
        S[0] = a * x * y;                        dS[0] = a * y;      dS[1] = a * x;       dS[2] = 0;
        S[1] = a * y * z;                        dS[3] = 0;          dS[4] = a * z;       dS[5] = a * y;
        S[2] = b * (2 * z * z - x * x - y * y);  dS[6] = -2 * b * x; dS[7] = -2 * b * y;  dS[8] = 4 * b * z;
        S[3] = a * x * z;                        dS[9] = a * z;      dS[10] = 0;          dS[11] = a * x;
        S[4] = c * (x * x - y * y);              dS[12] = 2 * c * x; dS[13] = -2 * c * y; dS[14] = 0;
        break;
    }
    case 3: {
        const double A = std::sqrt(35.0 / (32.0 * kPi));
        const double B = std::sqrt(105.0 / (4.0 * kPi));
        const double C = std::sqrt(21.0 / (32.0 * kPi));
        const double D = std::sqrt(7.0 / (16.0 * kPi));
        const double E = std::sqrt(105.0 / (16.0 * kPi));
        const double xx = x * x, yy = y * y, zz = z * z;
        S[0] = A * y * (3 * xx - yy);
        dS[0] = 6 * A * x * y; dS[1] = A * (3 * xx - 3 * yy); dS[2] = 0;
        S[1] = B * x * y * z;
        dS[3] = B * y * z; dS[4] = B * x * z; dS[5] = B * x * y;
        S[2] = C * y * (4 * zz - xx - yy);
        dS[6] = -2 * C * x * y; dS[7] = C * (4 * zz - xx - 3 * yy); dS[8] = 8 * C * y * z;
        S[3] = D * z * (2 * zz - 3 * xx - 3 * yy);
        dS[9] = -6 * D * x * z; dS[10] = -6 * D * y * z; dS[11] = D * (6 * zz - 3 * xx - 3 * yy);
        S[4] = C * x * (4 * zz - xx - yy);
        dS[12] = C * (4 * zz - 3 * xx - yy); dS[13] = -2 * C * x * y; dS[14] = 8 * C * x * z;
        S[5] = E * z * (xx - yy);
        dS[15] = 2 * E * x * z; dS[16] = -2 * E * y * z; dS[17] = E * (xx - yy);
        S[6] = A * x * (xx - 3 * yy);
        dS[18] = A * (3 * xx - 3 * yy); dS[19] = -6 * A * x * y; dS[20] = 0;
        break;
    }
    default:
        break;
    }
}

inline int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

struct Pt {
    int32_t g;
    int32_t img[3];
    int32_t ijk[3];
    double d[3];
};

}  // namespace

double hub_g0_cell_average(const double h[3]) {
    // 8/(hx hy hz) * F(a, b, c), F = integral of 1/r over [0,a]x[0,b]x[0,c]
    // with a = hx/2 etc.: the potential of a uniform cuboid at its corner,
    // F = ab asinh(c/sqrt(a^2+b^2)) + bc asinh(a/sqrt(b^2+c^2))
    //   + ca asinh(b/sqrt(c^2+a^2)) - a^2/2 atan(bc/(a r))
    //   - b^2/2 atan(ca/(b r)) - c^2/2 atan(ab/(c r)),  r = sqrt(a^2+b^2+c^2).
    const double a = 0.5 * h[0], b = 0.5 * h[1], c = 0.5 * h[2];
    const double r = std::sqrt(a * a + b * b + c * c);
    const double F = a * b * std::asinh(c / std::hypot(a, b)) + b * c * std::asinh(a / std::hypot(b, c)) +
                     c * a * std::asinh(b / std::hypot(c, a)) - 0.5 * a * a * std::atan(b * c / (a * r)) -
                     0.5 * b * b * std::atan(c * a / (b * r)) - 0.5 * c * c * std::atan(a * b / (c * r));
    return 8.0 * F / (h[0] * h[1] * h[2]);
}

int hub_build_host(const double cell[3], const int ngrid[3], const std::vector<SiteDef>& sites,
                   int chunk_entries, HostTables& T) {
    T = HostTables();
    const int ns = static_cast<int>(sites.size());
    if (ns == 0) return HUB_EINVAL;
    double h[3];
    for (int i = 0; i < 3; ++i) h[i] = cell[i] / static_cast<double>(ngrid[i]);
    const double dV = h[0] * h[1] * h[2];
    const int64_t G = static_cast<int64_t>(ngrid[0]) * ngrid[1] * ngrid[2];
    if (G > INT32_MAX) return HUB_EINVAL;

    T.nsites = ns;
    T.site_L.resize(ns);
    T.site_orb0.resize(ns);
    T.site_species.resize(ns);
    T.spheres.resize(ns);
    int J = 0, nspec = 0;
    for (int s = 0; s < ns; ++s) {
        T.site_L[s] = 2 * sites[s].l + 1;
        T.site_orb0[s] = J;
        T.site_species[s] = sites[s].species;
        J += T.site_L[s];
        nspec = std::max(nspec, sites[s].species + 1);
    }
    T.J = J;
    T.nspecies = nspec;
    for (const SiteDef& sd : sites)
        if (std::isfinite(sd.zeta_dn)) T.spindep = true;

    std::map<std::tuple<int, int, int>, int> image_id;
    std::vector<std::vector<Pt>> pts(ns);

    // ---- spheres: enumerate unfolded integer coordinates around R
    for (int s = 0; s < ns; ++s) {
        const SiteDef& S = sites[s];
        const double rc2 = S.rc * S.rc;
        int64_t lo[3], hi[3];
        for (int i = 0; i < 3; ++i) {
            lo[i] = static_cast<int64_t>(std::floor((S.R[i] - S.rc) / h[i])) - 1;
            hi[i] = static_cast<int64_t>(std::ceil((S.R[i] + S.rc) / h[i])) + 1;
        }
        std::vector<Pt>& P = pts[s];
        for (int64_t jx = lo[0]; jx <= hi[0]; ++jx) {
            const double dx = static_cast<double>(jx) * h[0] - S.R[0];
            for (int64_t jy = lo[1]; jy <= hi[1]; ++jy) {
                const double dy = static_cast<double>(jy) * h[1] - S.R[1];
                const double dxy = dx * dx + dy * dy;
                for (int64_t jz = lo[2]; jz <= hi[2]; ++jz) {
                    const double dz = static_cast<double>(jz) * h[2] - S.R[2];
                    const double d2 = dxy + dz * dz;
                    if (!(d2 <= rc2)) continue;
                    Pt p;
                    const int64_t j[3] = {jx, jy, jz};
                    int64_t f[3];
                    for (int i = 0; i < 3; ++i) {
                        const int64_t n = floor_div(j[i], ngrid[i]);
                        f[i] = j[i] - n * ngrid[i];
                        p.img[i] = static_cast<int32_t>(n);
                        p.ijk[i] = static_cast<int32_t>(j[i]);
                    }
                    p.g = static_cast<int32_t>((f[0] * ngrid[1] + f[1]) * ngrid[2] + f[2]);
                    p.d[0] = dx; p.d[1] = dy; p.d[2] = dz;
                    P.push_back(p);
                }
            }
        }
        if (P.empty()) return HUB_EINVAL;   // a sphere with no grid point has no orbital
        std::sort(P.begin(), P.end(), [](const Pt& a, const Pt& b) {
            return std::tie(a.g, a.img[0], a.img[1], a.img[2]) < std::tie(b.g, b.img[0], b.img[1], b.img[2]);
        });
        // orbital values and grid normalization dV sum phi^2 = 1 per m
        const int L = T.site_L[s];
        SiteSphere& sp = T.spheres[s];
        const size_t np = P.size();
        sp.g.resize(np);
        sp.img3.resize(3 * np);
        sp.ijk.resize(3 * np);
        sp.phi.resize(np * L);
        sp.grad.resize(np * L * 3);
        std::vector<double> norm2(L, 0.0);
        double Sv[7], dSv[21];
        for (size_t p = 0; p < np; ++p) {
            const Pt& q = P[p];
            sp.g[p] = q.g;
            for (int i = 0; i < 3; ++i) {
                sp.img3[3 * p + i] = q.img[i];
                sp.ijk[3 * p + i] = q.ijk[i];
            }
            const double r = std::sqrt((q.d[0] * q.d[0] + q.d[1] * q.d[1]) + q.d[2] * q.d[2]);
            const double rad = std::exp(-S.zeta * r);
            solid_harmonics(S.l, q.d[0], q.d[1], q.d[2], Sv, dSv);
            for (int m = 0; m < L; ++m) {
                const double chi = rad * Sv[m];
                sp.phi[p * L + m] = chi;
                norm2[m] += chi * chi;
                for (int i = 0; i < 3; ++i) {
                    const double radial = (r > 0.0) ? S.zeta * (q.d[i] / r) * Sv[m] : 0.0;
                    sp.grad[(p * L + m) * 3 + i] = rad * (dSv[3 * m + i] - radial);
                }
            }
        }
        for (int m = 0; m < L; ++m) {
            const double nm = 1.0 / std::sqrt(dV * norm2[m]);
            for (size_t p = 0; p < np; ++p) {
                sp.phi[p * L + m] *= nm;
                for (int i = 0; i < 3; ++i) sp.grad[(p * L + m) * 3 + i] *= nm;
            }
        }
        // spin-down orbitals: the same points and harmonics with the site's
        // spin-down exponent, normalized on the grid on their own
        if (T.spindep) {
            const double zd = std::isfinite(S.zeta_dn) ? S.zeta_dn : S.zeta;
            sp.phi_dn.resize(np * L);
            sp.grad_dn.resize(np * L * 3);
            std::vector<double> nd(L, 0.0);
            for (size_t p = 0; p < np; ++p) {
                const Pt& q = P[p];
                const double r = std::sqrt((q.d[0] * q.d[0] + q.d[1] * q.d[1]) + q.d[2] * q.d[2]);
                const double rad = std::exp(-zd * r);
                solid_harmonics(S.l, q.d[0], q.d[1], q.d[2], Sv, dSv);
                for (int m = 0; m < L; ++m) {
                    const double chi = rad * Sv[m];
                    sp.phi_dn[p * L + m] = chi;
                    nd[m] += chi * chi;
                    for (int i = 0; i < 3; ++i) {
                        const double radial = (r > 0.0) ? zd * (q.d[i] / r) * Sv[m] : 0.0;
                        sp.grad_dn[(p * L + m) * 3 + i] = rad * (dSv[3 * m + i] - radial);
                    }
                }
            }
            for (int m = 0; m < L; ++m) {
                const double nm = 1.0 / std::sqrt(dV * nd[m]);
                for (size_t p = 0; p < np; ++p) {
                    sp.phi_dn[p * L + m] *= nm;
                    for (int i = 0; i < 3; ++i) sp.grad_dn[(p * L + m) * 3 + i] *= nm;
                }
            }
        }
        for (size_t p = 0; p < np; ++p) {
            auto key = std::make_tuple(P[p].img[0], P[p].img[1], P[p].img[2]);
            if (!image_id.count(key)) {
                const int id = static_cast<int>(image_id.size());
                image_id[key] = id;
            }
        }
    }
    // images of the dilated spheres of the state-gradient force form: a point
    // up to two steps past a sphere point along one axis; only points within
    // two steps of a cell face can change image
    for (int s = 0; s < ns; ++s)
        for (const Pt& q : pts[s])
            for (int i = 0; i < 3; ++i) {
                const int64_t f = static_cast<int64_t>(q.ijk[i]) - static_cast<int64_t>(q.img[i]) * ngrid[i];
                if (f >= 2 && f < ngrid[i] - 2) continue;
                for (int o = -2; o <= 2; ++o) {
                    if (o == 0) continue;
                    int32_t im[3] = {q.img[0], q.img[1], q.img[2]};
                    im[i] = static_cast<int32_t>(floor_div(static_cast<int64_t>(q.ijk[i]) + o, ngrid[i]));
                    auto key = std::make_tuple(im[0], im[1], im[2]);
                    if (!image_id.count(key)) {
                        const int id = static_cast<int>(image_id.size());
                        image_id[key] = id;
                    }
                }
            }
    T.images.resize(3 * image_id.size());
    for (const auto& kv : image_id) {
        T.images[3 * kv.second + 0] = std::get<0>(kv.first);
        T.images[3 * kv.second + 1] = std::get<1>(kv.first);
        T.images[3 * kv.second + 2] = std::get<2>(kv.first);
    }

    // ---- layers: the k-th entry (in site order) that lands on grid point g
    // goes to layer k, so a layer never holds the same g twice.
    std::vector<uint16_t> cover(static_cast<size_t>(G), 0);
    std::vector<std::vector<int>> layer_of(ns);
    int nlayers = 0;
    for (int s = 0; s < ns; ++s) {
        const size_t np = pts[s].size();
        layer_of[s].resize(np);
        for (size_t p = 0; p < np; ++p) {
            const int32_t g = pts[s][p].g;
            if (cover[g] == 65535) return HUB_EINVAL;
            const int lay = cover[g]++;
            layer_of[s][p] = lay;
            nlayers = std::max(nlayers, lay + 1);
        }
    }
    T.nlayers = nlayers;

    // ---- entries ordered by (layer, site, g); chunks of <= chunk_entries
    const int chunk = std::max(1, chunk_entries);
    T.layer_chunk_ptr.assign(nlayers + 1, 0);
    T.layer_site_ptr.assign(static_cast<size_t>(nlayers) * ns + 1, 0);
    int64_t e = 0, phi0 = 0, nreal = 0;
    int part_rows = 0;
    for (int lay = 0; lay < nlayers; ++lay) {
        T.layer_chunk_ptr[lay] = static_cast<int32_t>(T.chunks.size());
        for (int s = 0; s < ns; ++s) {
            T.layer_site_ptr[static_cast<size_t>(lay) * ns + s] = static_cast<int32_t>(T.chunks.size());
            const int L = T.site_L[s];
            const SiteSphere& sp = T.spheres[s];
            // entries of this (layer, site), grouped by lattice image, g ascending
            std::vector<size_t> mine;
            for (size_t p = 0; p < pts[s].size(); ++p)
                if (layer_of[s][p] == lay) mine.push_back(p);
            auto img_of = [&](size_t p) {
                return image_id[std::make_tuple(pts[s][p].img[0], pts[s][p].img[1], pts[s][p].img[2])];
            };
            std::stable_sort(mine.begin(), mine.end(), [&](size_t a, size_t b) { return img_of(a) < img_of(b); });
            for (size_t b = 0; b < mine.size();) {
                const int im = img_of(mine[b]);
                size_t nb = 0;
                while (b + nb < mine.size() && nb < static_cast<size_t>(chunk) && img_of(mine[b + nb]) == im) ++nb;
                const size_t np = (nb + HUB_ENTRY_ALIGN - 1) / HUB_ENTRY_ALIGN * HUB_ENTRY_ALIGN;
                HubChunk C;
                C.img = im;
                C.nreal = static_cast<int32_t>(nb);
                C.site = s;
                C.layer = lay;
                C.e0 = static_cast<int32_t>(e);
                C.ne = static_cast<int32_t>(np);
                C.L = L;
                C.orb0 = T.site_orb0[s];
                C.part0 = part_rows;
                C.species = sites[s].species;
                C.phi0 = phi0;
                for (size_t t = 0; t < nb; ++t) {
                    const size_t p = mine[b + t];
                    T.gidx.push_back(sp.g[p]);
                    const Pt& q = pts[s][p];
                    T.img.push_back(image_id[std::make_tuple(q.img[0], q.img[1], q.img[2])]);
                    for (int m = 0; m < L; ++m) T.phi.push_back(sp.phi[p * L + m]);
                    if (T.spindep) {
                        for (int m = 0; m < L; ++m) T.phi2.push_back(sp.phi[p * L + m]);
                        for (int m = 0; m < L; ++m) T.phi2.push_back(sp.phi_dn[p * L + m]);
                        for (int m = 0; m < L; ++m)
                            for (int i = 0; i < 3; ++i) {
                                T.gphi_dn.push_back(sp.grad_dn[(p * L + m) * 3 + i]);
                                const double di = static_cast<double>(sp.ijk[3 * p + i]) * h[i] - sites[s].R[i];
                                T.mphi_dn.push_back(di * sp.phi_dn[p * L + m]);
                            }
                    }
                    for (int m = 0; m < L; ++m)
                        for (int i = 0; i < 3; ++i) T.gphi.push_back(sp.grad[(p * L + m) * 3 + i]);
                    // position moments about the site centre (velocity-gauge current)
                    for (int m = 0; m < L; ++m)
                        for (int i = 0; i < 3; ++i) {
                            const double di = static_cast<double>(sp.ijk[3 * p + i]) * h[i] - sites[s].R[i];
                            T.mphi.push_back(di * sp.phi[p * L + m]);
                        }
                }
                // padding entries: the last grid point again, zero values
                for (size_t t = nb; t < np; ++t) {
                    T.gidx.push_back(T.gidx.back());
                    T.img.push_back(T.img.back());
                    T.phi.insert(T.phi.end(), L, 0.0);
                    if (T.spindep) {
                        T.phi2.insert(T.phi2.end(), 2 * L, 0.0);
                        T.gphi_dn.insert(T.gphi_dn.end(), 3 * L, 0.0);
                        T.mphi_dn.insert(T.mphi_dn.end(), 3 * L, 0.0);
                    }
                    T.gphi.insert(T.gphi.end(), 3 * L, 0.0);
                    T.mphi.insert(T.mphi.end(), 3 * L, 0.0);
                }
                e += static_cast<int64_t>(np);
                nreal += static_cast<int64_t>(nb);
                phi0 += static_cast<int64_t>(np) * L;
                part_rows += L;
                T.chunks.push_back(C);
                b += nb;
            }
        }
    }
    T.layer_chunk_ptr[nlayers] = static_cast<int32_t>(T.chunks.size());
    T.layer_site_ptr[static_cast<size_t>(nlayers) * ns] = static_cast<int32_t>(T.chunks.size());
    T.part_rows = part_rows;
    T.nentries = nreal;
    if (e > INT32_MAX) return HUB_EINVAL;

    // ---- grouped work list (cover signatures).  With spin-dependent
    // orbitals every cover contributes 2L functions, the orbitals of the
    // spin-up then of the spin-down component (function sigma L + m; its
    // orbital index is stored as j + sigma J)
    {
        const int smul = T.spindep ? 2 : 1;
        GroupTables& GT = T.grouped;
        struct Cover {
            int32_t g, site, img;
            uint32_t p;
        };
        std::vector<Cover> cov;
        cov.reserve(static_cast<size_t>(nreal));
        for (int s = 0; s < ns; ++s)
            for (size_t p = 0; p < pts[s].size(); ++p) {
                const Pt& q = pts[s][p];
                cov.push_back({q.g, s, image_id[std::make_tuple(q.img[0], q.img[1], q.img[2])],
                               static_cast<uint32_t>(p)});
            }
        std::sort(cov.begin(), cov.end(), [](const Cover& a, const Cover& b) {
            return std::tie(a.g, a.site, a.img) < std::tie(b.g, b.site, b.img);
        });
        // (pass, signature) -> points (each point: index in cov of the first
        // cover of that pass).  A point with more than HUB_GF_MAX functions
        // has its covers split into consecutive slot ranges of at most
        // HUB_GF_MAX functions, one per pass; the apply launches the passes
        // one after the other, so a point is updated by one chunk at a time.
        // Points are grouped by the covers of each pass (not by their whole
        // cover list), which keeps the chunks long when large spheres give
        // nearly every point a cover list of its own.
        using Sig = std::vector<std::pair<int, int>>;
        std::map<std::pair<int, Sig>, std::vector<size_t>> groups;
        std::vector<std::pair<int, Sig>> order;
        bool ok = true;
        int nfmax = 0, npass = 1;
        for (size_t i = 0; i < cov.size();) {
            size_t k = i;
            int nf = 0, acc = 0, pass = 0;
            size_t first = i;
            Sig sig;
            auto close = [&]() {
                auto key = std::make_pair(pass, sig);
                auto it = groups.find(key);
                if (it == groups.end()) {
                    order.push_back(key);
                    groups[key].push_back(first);
                } else {
                    it->second.push_back(first);
                }
            };
            while (k < cov.size() && cov[k].g == cov[i].g) {
                const int Ls = smul * T.site_L[cov[k].site];
                if (acc + Ls > HUB_GF_MAX) {
                    close();
                    ++pass;
                    sig.clear();
                    acc = 0;
                    first = k;
                }
                sig.push_back({cov[k].site, cov[k].img});
                acc += Ls;
                nf += Ls;
                ++k;
            }
            close();
            nfmax = std::max(nfmax, nf);
            npass = std::max(npass, pass + 1);
            i = k;
        }
        GT.nfmax = nfmax;
        GT.ok = ok;
        if (ok) {
            int64_t rows = 0, tab0 = 0;
            for (const auto& key : order) {
                const std::vector<size_t>& firsts = groups[key];
                const int pass = key.first;
                const Sig& sig = key.second;
                int nf = 0;
                for (const auto& sl : sig) nf += smul * T.site_L[sl.first];
                // more than 8 functions: the kernels take half as many entries
                // per batch, so half-length chunks keep the per-wave chains
                // (and the launches' latency) comparable
                const int chunk = std::max(1, nf > 8 ? std::max(64, chunk_entries / 2) : chunk_entries);
                for (size_t b = 0; b < firsts.size(); b += chunk) {
                    const size_t nb = std::min(firsts.size() - b, static_cast<size_t>(chunk));
                    const size_t np = (nb + HUB_ENTRY_ALIGN - 1) / HUB_ENTRY_ALIGN * HUB_ENTRY_ALIGN;
                    HubChunk C;
                    C.site = sig[0].first;
                    C.layer = pass;
                    C.e0 = static_cast<int32_t>(GT.gidx.size());
                    C.ne = static_cast<int32_t>(np);
                    C.nreal = static_cast<int32_t>(nb);
                    C.L = nf;
                    C.orb0 = -1;
                    C.part0 = static_cast<int32_t>(rows);
                    C.species = -1;
                    C.phi0 = tab0;
                    C.img = sig[0].second;
                    // position moments (velocity-gauge current): the displacement
                    // d0 of each point from the centre of its first cover's site
                    // (unfolded, image-shifted coordinates), and per function the
                    // constant offset from that cover's displacement to its own
                    auto disp = [&](const Cover& cv, int i) {
                        return static_cast<double>(T.spheres[cv.site].ijk[3 * cv.p + i]) * h[i] -
                               sites[cv.site].R[i];
                    };
                    {
                        const size_t i0 = firsts[b];
                        double del[HUB_GF_MAX][3] = {};
                        int f = 0;
                        for (size_t sl = 0; sl < sig.size(); ++sl)
                            for (int m = 0; m < smul * T.site_L[sig[sl].first]; ++m, ++f)
                                for (int i = 0; i < 3; ++i) del[f][i] = disp(cov[i0 + sl], i) - disp(cov[i0], i);
                        for (int ff = 0; ff < HUB_GF_MAX; ++ff)
                            for (int i = 0; i < 3; ++i) GT.fdel.push_back(del[ff][i]);
                    }
                    for (size_t t = 0; t < nb; ++t) {
                        const size_t i0 = firsts[b + t];
                        GT.gidx.push_back(cov[i0].g);
                        for (int i = 0; i < 3; ++i) GT.d0.push_back(disp(cov[i0], i));
                        for (size_t sl = 0; sl < sig.size(); ++sl) {
                            const Cover& cv = cov[i0 + sl];
                            const int L = T.site_L[cv.site];
                            const double* src = &T.spheres[cv.site].phi[static_cast<size_t>(cv.p) * L];
                            for (int m = 0; m < L; ++m) GT.tab.push_back(src[m]);
                            if (T.spindep) {
                                const double* dn = &T.spheres[cv.site].phi_dn[static_cast<size_t>(cv.p) * L];
                                for (int m = 0; m < L; ++m) GT.tab.push_back(dn[m]);
                            }
                        }
                    }
                    for (size_t t = nb; t < np; ++t) {
                        GT.gidx.push_back(GT.gidx.back());
                        GT.tab.insert(GT.tab.end(), nf, 0.0);
                        GT.d0.insert(GT.d0.end(), 3, 0.0);
                    }
                    for (int f = 0; f < HUB_GF_MAX; ++f) {
                        GT.f_orb.push_back(-1);
                        GT.f_img.push_back(0);
                    }
                    int f = 0;
                    for (const auto& sl : sig)
                        for (int sg = 0; sg < smul; ++sg)
                            for (int m = 0; m < T.site_L[sl.first]; ++m, ++f) {
                                GT.f_orb[GT.chunks.size() * HUB_GF_MAX + f] = T.site_orb0[sl.first] + m + sg * J;
                                GT.f_img[GT.chunks.size() * HUB_GF_MAX + f] = sl.second;
                            }
                    tab0 += static_cast<int64_t>(np) * nf;
                    rows += nf;
                    GT.chunks.push_back(C);
                }
            }
            GT.npass = npass;
            GT.part_rows = rows;
            if (rows > INT32_MAX) GT.ok = false;
            // CSR orbital j -> (workspace row, image); with spin-dependent
            // orbitals the rows of the spin-up functions (the spin-down
            // function of the same orbital and cover is L rows further)
            std::vector<std::vector<std::pair<int32_t, int32_t>>> red(J);
            for (size_t c = 0; c < GT.chunks.size(); ++c)
                for (int f = 0; f < GT.chunks[c].L; ++f) {
                    const int j = GT.f_orb[c * HUB_GF_MAX + f];
                    if (j >= J) continue;
                    red[j].push_back({GT.chunks[c].part0 + f, GT.f_img[c * HUB_GF_MAX + f]});
                }
            GT.red_ptr.assign(J + 1, 0);
            for (int j = 0; j < J; ++j) {
                GT.red_ptr[j + 1] = GT.red_ptr[j] + static_cast<int32_t>(red[j].size());
                for (const auto& it : red[j]) {
                    GT.red_row.push_back(it.first);
                    GT.red_img.push_back(it.second);
                }
            }
        }
    }

    // ---- CSR maps
    T.site_chunk_ptr.assign(ns + 1, 0);
    for (const HubChunk& C : T.chunks) T.site_chunk_ptr[C.site + 1]++;
    for (int s = 0; s < ns; ++s) T.site_chunk_ptr[s + 1] += T.site_chunk_ptr[s];
    T.site_chunk_ids.resize(T.chunks.size());
    {
        std::vector<int32_t> fill(T.site_chunk_ptr.begin(), T.site_chunk_ptr.end() - 1);
        for (size_t c = 0; c < T.chunks.size(); ++c) T.site_chunk_ids[fill[T.chunks[c].site]++] = static_cast<int32_t>(c);
    }
    T.species_orb_ptr.assign(nspec + 1, 0);
    for (int s = 0; s < ns; ++s) T.species_orb_ptr[sites[s].species + 1] += T.site_L[s];
    for (int t = 0; t < nspec; ++t) T.species_orb_ptr[t + 1] += T.species_orb_ptr[t];
    T.species_orb_ids.resize(J);
    T.orb_site.resize(J);
    {
        std::vector<int32_t> fill(T.species_orb_ptr.begin(), T.species_orb_ptr.end() - 1);
        for (int s = 0; s < ns; ++s)
            for (int m = 0; m < T.site_L[s]; ++m) {
                T.species_orb_ids[fill[sites[s].species]++] = T.site_orb0[s] + m;
                T.orb_site[T.site_orb0[s] + m] = s;
            }
    }
    return HUB_OK;
}

int hub_build_stencil(const double cell[3], const int ngrid[3], const std::vector<SiteDef>& sites,
                      const HostTables& T, int chunk_entries, StencilTables& S) {
    S = StencilTables();
    const int ns = T.nsites;
    if (ns <= 0 || static_cast<int>(sites.size()) != ns || static_cast<int>(T.spheres.size()) != ns) return HUB_EINVAL;
    double h[3];
    for (int i = 0; i < 3; ++i) h[i] = cell[i] / static_cast<double>(ngrid[i]);
    // first derivative, 4th order: weights of the values at offsets -2..2 (times 1/h)
    constexpr int kOff[4] = {-2, -1, 1, 2};
    constexpr double kW[4] = {1.0 / 12.0, -2.0 / 3.0, 2.0 / 3.0, -1.0 / 12.0};
    std::map<std::tuple<int, int, int>, int> image_id;
    for (size_t t = 0; t < T.images.size() / 3; ++t)
        image_id[std::make_tuple(T.images[3 * t], T.images[3 * t + 1], T.images[3 * t + 2])] = static_cast<int>(t);
    const int chunk = std::max(1, chunk_entries);
    S.site_chunk_ptr.assign(ns + 1, 0);
    int64_t e = 0, nreal = 0, part_rows = 0, phi0 = 0;
    for (int s = 0; s < ns; ++s) {
        S.site_chunk_ptr[s] = static_cast<int32_t>(S.chunks.size());
        const SiteSphere& sp = T.spheres[s];
        const int L = T.site_L[s];
        const size_t np = sp.g.size();
        if (np == 0) return HUB_EINVAL;
        // box of unfolded coordinates: the sphere's bounds widened by 2
        int64_t lo[3], hi[3], nb[3];
        for (int i = 0; i < 3; ++i) {
            lo[i] = hi[i] = sp.ijk[i];
            for (size_t p = 0; p < np; ++p) {
                lo[i] = std::min<int64_t>(lo[i], sp.ijk[3 * p + i]);
                hi[i] = std::max<int64_t>(hi[i], sp.ijk[3 * p + i]);
            }
            lo[i] -= 2;
            hi[i] += 2;
            nb[i] = hi[i] - lo[i] + 1;
        }
        const size_t box = static_cast<size_t>(nb[0] * nb[1] * nb[2]);
        auto cell_of = [&](int64_t x, int64_t y, int64_t z) {
            return static_cast<size_t>(((x - lo[0]) * nb[1] + (y - lo[1])) * nb[2] + (z - lo[2]));
        };
        std::vector<int32_t> at(box, -1);     // sphere point at a box cell
        std::vector<char> dil(box, 0);        // cell of the dilated sphere
        for (size_t p = 0; p < np; ++p) {
            const int64_t j[3] = {sp.ijk[3 * p], sp.ijk[3 * p + 1], sp.ijk[3 * p + 2]};
            at[cell_of(j[0], j[1], j[2])] = static_cast<int32_t>(p);
            for (int i = 0; i < 3; ++i)
                for (int o = 0; o < 4; ++o) {
                    int64_t n[3] = {j[0], j[1], j[2]};
                    n[i] += kOff[o];
                    dil[cell_of(n[0], n[1], n[2])] = 1;
                }
        }
        struct DPt {
            int32_t g, img;
            int64_t x, y, z;
        };
        std::vector<DPt> pts;
        for (int64_t x = lo[0]; x <= hi[0]; ++x)
            for (int64_t y = lo[1]; y <= hi[1]; ++y)
                for (int64_t z = lo[2]; z <= hi[2]; ++z) {
                    if (!dil[cell_of(x, y, z)]) continue;
                    const int64_t j[3] = {x, y, z};
                    int64_t f[3];
                    int im[3];
                    for (int i = 0; i < 3; ++i) {
                        const int64_t n = floor_div(j[i], ngrid[i]);
                        f[i] = j[i] - n * ngrid[i];
                        im[i] = static_cast<int>(n);
                    }
                    auto it = image_id.find(std::make_tuple(im[0], im[1], im[2]));
                    if (it == image_id.end()) return HUB_EINVAL;
                    pts.push_back({static_cast<int32_t>((f[0] * ngrid[1] + f[1]) * ngrid[2] + f[2]), it->second, x, y,
                                   z});
                }
        std::sort(pts.begin(), pts.end(),
                  [](const DPt& a, const DPt& b) { return std::tie(a.img, a.g) < std::tie(b.img, b.g); });
        // (D_i phi_m)(n) = sum_o w_o phi_m(n + o e_i) / h_i, phi zero off the sphere
        auto table_row = [&](const DPt& q, const std::vector<double>& phi, std::vector<double>& tab) {
            const int64_t j[3] = {q.x, q.y, q.z};
            for (int m = 0; m < L; ++m)
                for (int i = 0; i < 3; ++i) {
                    double acc = 0.0;
                    for (int o = 0; o < 4; ++o) {
                        int64_t n[3] = {j[0], j[1], j[2]};
                        n[i] += kOff[o];
                        if (n[i] < lo[i] || n[i] > hi[i]) continue;
                        const int32_t p = at[cell_of(n[0], n[1], n[2])];
                        if (p >= 0) acc += kW[o] * phi[static_cast<size_t>(p) * L + m];
                    }
                    tab.push_back(acc / h[i]);
                }
        };
        for (size_t b = 0; b < pts.size();) {
            const int im = pts[b].img;
            size_t n = 0;
            while (b + n < pts.size() && n < static_cast<size_t>(chunk) && pts[b + n].img == im) ++n;
            const size_t npad = (n + HUB_ENTRY_ALIGN - 1) / HUB_ENTRY_ALIGN * HUB_ENTRY_ALIGN;
            HubChunk C;
            C.site = s;
            C.layer = 0;
            C.e0 = static_cast<int32_t>(e);
            C.ne = static_cast<int32_t>(npad);
            C.L = L;
            C.orb0 = T.site_orb0[s];
            C.part0 = static_cast<int32_t>(part_rows);
            C.species = sites[s].species;
            C.phi0 = phi0;
            C.img = im;
            C.nreal = static_cast<int32_t>(n);
            for (size_t t = 0; t < n; ++t) {
                S.gidx.push_back(pts[b + t].g);
                table_row(pts[b + t], sp.phi, S.tab);
                if (T.spindep) table_row(pts[b + t], sp.phi_dn, S.tab_dn);
            }
            for (size_t t = n; t < npad; ++t) {
                S.gidx.push_back(S.gidx.back());
                S.tab.insert(S.tab.end(), 3 * L, 0.0);
                if (T.spindep) S.tab_dn.insert(S.tab_dn.end(), 3 * L, 0.0);
            }
            S.site_chunk_ids.push_back(static_cast<int32_t>(S.chunks.size()));
            S.chunks.push_back(C);
            e += static_cast<int64_t>(npad);
            nreal += static_cast<int64_t>(n);
            phi0 += static_cast<int64_t>(npad) * L;
            part_rows += L;
            b += n;
            if (e > INT32_MAX || part_rows > INT32_MAX) return HUB_EINVAL;
        }
    }
    S.site_chunk_ptr[ns] = static_cast<int32_t>(S.chunks.size());
    S.part_rows = part_rows;
    S.nentries = nreal;
    return HUB_OK;
}

int hub_sphere_radius(int method, int l, double zeta, const double cell[3], double threshold, double* rc) {
    if (!rc) return HUB_EINVAL;
    if (method == HUB_RADIUS_CELL) {
        if (!cell) return HUB_EINVAL;
        double m = cell[0];
        for (int i = 0; i < 3; ++i) {
            if (!(cell[i] > 0.0) || !std::isfinite(cell[i])) return HUB_EINVAL;
            m = std::min(m, cell[i]);
        }
        *rc = m;
        return HUB_OK;
    }
    if (method != HUB_RADIUS_THRESHOLD) return HUB_EINVAL;
    if (l < 0 || l > 3 || !(zeta > 0.0) || !std::isfinite(zeta) || !(threshold > 0.0) || !std::isfinite(threshold))
        return HUB_EINVAL;
    // log R(r) - log threshold; decreasing for r > l / zeta
    double fact = 1.0;
    for (int i = 2; i <= 2 * l + 2; ++i) fact *= i;
    const double logN = 0.5 * ((2 * l + 3) * std::log(2.0 * zeta) - std::log(fact));
    const double logt = std::log(threshold);
    auto g = [&](double r) { return logN + (l > 0 ? l * std::log(r) : 0.0) - zeta * r - logt; };
    double lo = l > 0 ? l / zeta : 0.0;
    if (!(g(lo) > 0.0)) return HUB_EINVAL;
    double hi = lo + 1.0 / zeta;
    for (int it = 0; g(hi) > 0.0; ++it) {
        if (it > 200) return HUB_EINVAL;
        hi = lo + 2.0 * (hi - lo);
    }
    // bisection down to adjacent doubles: g(lo) > 0 >= g(hi)
    for (int it = 0; it < 2000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (g(mid) > 0.0)
            lo = mid;
        else
            hi = mid;
    }
    *rc = hi;
    return HUB_OK;
}
