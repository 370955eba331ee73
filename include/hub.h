/*
 * hub.h -- C ABI of the MI355X (gfx950) DFT+U / ACBN0 Hubbard kernel.
 *
 * Method: Tancogne-Dejean, Oliveira & Rubio, "Self-consistent DFT+U method
 * for real-space time-dependent density functional theory calculations"
 * (arXiv 1711.08935).  Section/equation labels below are the paper's.
 *
 * Conventions (all calls):
 *  - Hartree atomic units.  Orthorhombic cell of lengths cell[3] (bohr) with
 *    ngrid[3] points per axis; h_i = cell_i / ngrid_i; grid point
 *    g = (ix * Ny + iy) * Nz + iz sits at r_g = (ix hx, iy hy, iz hz);
 *    dV = hx hy hz.  G = Nx Ny Nz.
 *  - k-points in reduced units: k_i = 2 pi k_red_i / cell_i.  States are
 *    full Bloch functions on the cell grid, psi(r + T) = exp(i k.T) psi(r).
 *  - "Device pointer": memory the caller allocated on the GPU of the context
 *    (e.g. a torch tensor); "host pointer": ordinary CPU memory.  Every
 *    device-side call is asynchronous on the context stream (hub_set_stream);
 *    results are valid once that stream has reached the call.  The caller
 *    owns every pointer it passes; the context owns only its own tables and
 *    workspaces, released by hub_destroy.
 *  - Errors: the return value is HUB_OK (0), a negative error code, or a
 *    positive warning.  Arguments are validated before any launch; on an
 *    error nothing is launched and no output is touched.  No call aborts the
 *    process and no C++ exception crosses the ABI.  Asynchronous device
 *    faults surface as HUB_EDEVICE from a later call.
 *  - One context per stream; a context is not thread-safe.
 *  - Allocation-failure testing: with HUB_FAIL_ALLOC=N (N >= 1) in the
 *    environment when hub_create runs, that context's N-th device
 *    allocation attempt fails once, as if the GPU were out of memory; the
 *    call returns HUB_ENOMEM, frees what it had allocated, and may be
 *    repeated.
 *
 * State layouts (T = double for HUB_F64, float for HUB_F32; complex states
 * store (re, im) pairs of T):
 *  - unpolarized / collinear: psi[q][g][0..ld), q = ik * nspin + ispin
 *    (nspin = 1 unpolarized, 2 collinear), state s in column s;
 *  - spinor: psi[k][g][0..ld), state s, component sigma in column 2s+sigma.
 *  ncol = nstates (collinear) or 2 * nstates (spinor); ld >= ncol counts
 *  columns (complex elements for complex states) per grid point.
 *
 * Result layouts (always FP64):
 *  - c[q][j][ncol]: projections <phi_j,k|psi>; j runs over all orbitals of
 *    all sites in site order (orbital offset of each site: hub_site_info),
 *    m = -l..l inside a site; complex contexts interleave (re, im).
 *  - n, pbar: [site][nblk][HUB_LMAX][HUB_LMAX] complex (re, im) pairs;
 *    nblk = 1 (unpolarized: one stored channel that stands for two identical
 *    spin channels), 2 (collinear: sigma), 4 (spinor: block 2*sigma+sigma').
 *    Only the leading L x L corner of each block is used.
 *  - nbar[q][species][nstates] (spinor: [k][species][nstates]).
 *  - f: occupations per stored state set, [q][nstates] (spinor [k][nstates]).
 *  - U, J, Ueff, EU: [site]; status: [site] int32; F: [site][3].
 */
#ifndef HUB_H
#define HUB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HUB_LMAX 7           /* 2l+1 for the largest shell, l = 3 (f)       */
#define HUB_MAX_SPECIES 16

/* status codes */
#define HUB_OK 0
#define HUB_EINVAL (-1)      /* bad argument (NULL, size, mode, order)      */
#define HUB_ENOMEM (-2)      /* host or device allocation failed            */
#define HUB_EDEVICE (-3)     /* HIP runtime error (incl. an earlier fault)  */
#define HUB_ESTATE (-4)      /* call not valid in the context's state       */
#define HUB_ENONFINITE (-5)  /* per-site device status: occupations, U or J
                                not finite (NaN or Inf in the states)      */
#define HUB_ESCRATCH (-6)    /* hub_step_noalloc: the step's workspace does
                                not fit HUB_SCRATCH_BYTES                   */
#define HUB_WDEGENERATE 1    /* per-site status: a U/J denominator < 1e-12  */

/* spin modes */
#define HUB_UNPOLARIZED 1
#define HUB_COLLINEAR 2
#define HUB_SPINOR 4

/* storage precision of states (results are always FP64) */
#define HUB_F64 0
#define HUB_F32 1            /* FP32 states, FP64 orbital table, FP64 sums  */

/* hub_step modes */
#define HUB_STEP_BATCHED 0   /* one launch per stage over the work list     */
#define HUB_STEP_GRAPH 1     /* the batched launches captured as a hipGraph */
#define HUB_STEP_PERSITE 2   /* one launch per site and stage, no graph     */

typedef struct hub_ctx hub_ctx;

/* Create a context (host only; touches no GPU).
 * spin_mode: HUB_UNPOLARIZED | HUB_COLLINEAR | HUB_SPINOR (spinor needs
 * is_complex = 1).  precision: HUB_F64 | HUB_F32.  *out receives the handle.
 * Errors: HUB_EINVAL (NULL, ngrid < 1, cell <= 0, bad mode), HUB_ENOMEM. */
int hub_create(hub_ctx** out, const double cell[3], const int ngrid[3],
               int spin_mode, int is_complex, int precision);

/* k-point set (host arrays): k_red[nk][3] reduced coordinates, weights[nk]
 * (the w_k of Eq. occ_matrices).  Default: Gamma only, weight 1.  Real
 * contexts (is_complex = 0) accept only k = 0.  Before hub_finalize*. */
int hub_set_kpoints(hub_ctx* ctx, int nk, const double* k_red, const double* weights);

/* Add one Hubbard shell (Sec. II): centre R[3] (bohr, any position; it is
 * folded by periodicity), angular momentum l in 0..3, Slater exponent zeta of
 * the radial part r^l exp(-zeta r), sphere radius rc (sphere points satisfy
 * |r - R|^2 <= rc^2, inclusive), species id in [0, HUB_MAX_SPECIES) that
 * groups the shells summed in N-bar (Eq. notation_Nbar: atoms of the same
 * type).  *site_id (may be NULL) receives the site index.  Before
 * hub_finalize*. */
int hub_add_site(hub_ctx* ctx, const double R[3], int l, double zeta, double rc,
                 int species, int* site_id);

/* Sphere radius selection (Sec. II, the radius discussion; host only, needs
 * no context or GPU).  Of the paper's three methods, the pseudopotential's
 * non-local cutoff is the caller's own rc; the other two:
 *   HUB_RADIUS_CELL       rc = the shortest cell edge, min(cell[0..2])
 *                         (l, zeta, threshold ignored);
 *   HUB_RADIUS_THRESHOLD  rc = the radius beyond which the normalized
 *                         radial part R(r) = N r^l exp(-zeta r),
 *                         N^2 = (2 zeta)^(2l+3) / (2l+2)!, stays below
 *                         threshold (bohr^-3/2): the root of R(r) = threshold
 *                         on r >= l / zeta, to rounding (cell ignored).
 * *rc (bohr) is written on success.  Errors: HUB_EINVAL (NULL rc, unknown
 * method, l outside 0..3, zeta or threshold not positive and finite, a cell
 * edge not positive, or a threshold at or above the peak of R). */
#define HUB_RADIUS_CELL 1
#define HUB_RADIUS_THRESHOLD 2
int hub_sphere_radius(int method, int l, double zeta, const double cell[3], double threshold, double* rc);

/* Spin-dependent orbitals (App. A: the localized basis may be spinors):
 * give site a Slater exponent zeta_dn for the orbitals of the spin-down
 * component (same l, sphere and points; each component normalized on the
 * grid on its own), so that spin component sigma of the states is projected
 * on, and V_U psi built from, phi^sigma:
 * n^{st}_ab = sum w f conj(<phi^s_a|psi^s>) <phi^t_b|psi^t>.  Spinor
 * contexts only, before hub_finalize*.  Both work lists then carry the two
 * spin components' orbitals (2L functions per cover).  Such sites take a
 * fixed U_eff (hub_set_fixed_ueff; hub_coulomb skips them and rejects them
 * by index).  hub_forces, hub_forces_state_gradient and hub_current use
 * each component's orbital gradients, differences and position moments.
 * Under a vector potential the grouped work list serves the projections and
 * the apply (the per-site list then returns HUB_ESTATE).  Errors: HUB_EINVAL (bad site, zeta_dn not positive and
 * finite, not a spinor context), HUB_ESTATE (after finalize). */
int hub_set_site_spin_orbital(hub_ctx* ctx, int site, double zeta_dn);

/* Fix the effective U of one site (the empirical DFT+U scheme, Sec. II);
 * pass NaN to return the site to ACBN0 (the default).  Any time. */
int hub_set_fixed_ueff(hub_ctx* ctx, int site, double ueff);

/* Entries per work-list chunk (default 512; 64..65536).  Before
 * hub_finalize*. */
int hub_set_chunk(hub_ctx* ctx, int chunk_entries);

/* Kernel shape for the projection (which = 0) and the application
 * (which = 1): columns handled per lane (1, 2 or 4; 0 = automatic), waves
 * per work-group (1, 2 or 4), and the lane layout (1: every wave inside one
 * state set; 0: narrow state sets packed across the lanes of a wave;
 * -1: automatic).  Every shape computes the same result.  Any time after
 * creation. */
int hub_set_tuning(hub_ctx* ctx, int which, int cols_per_lane, int waves, int layout);

/* Work list of the batched launches (hub_project, hub_apply, and hub_step
 * in the batched and graph modes): grouped_list = 1 (default) groups every
 * grid point covered by any sphere with all its (site, lattice image) covers,
 * so each state row is read once by the projection and written once by the
 * apply; 0 uses one chunk per site and image, with overlapping sites applied
 * in successive atomic-free layers.  A grid point covered by more than 16
 * orbitals in total has its covers split over several passes of the
 * grouped list (at most 16 functions each; the apply launches the passes in
 * turn, hub_query 14).  Both give the same results up to summation order.
 * Any time. */
int hub_set_worklist(hub_ctx* ctx, int grouped_list);

/* Launch policy of the grouped work list, whose chunks fall in four classes
 * by function count (1-4, 5-8, 9-12, 13-16):
 *   HUB_CLASSES_MERGED      (default) one launch over every chunk, with a
 *                           kernel that covers every function count
 *                           (registers sized for the largest); chunks with
 *                           the longest entry loops are dispatched first;
 *   HUB_CLASSES_SEQUENTIAL  one launch per class, one after another, each
 *                           kernel's registers sized for its class;
 *   HUB_CLASSES_CONCURRENT  one launch per class on side streams forked from
 *                           and joined back to the context's stream
 *                           (parallel branches of a captured graph).
 * Results are identical.  With more than one pass the launches are merged
 * whatever the policy.  Any time; a captured step graph is rebuilt on the
 * next graph-mode hub_step. */
#define HUB_CLASSES_MERGED 0
#define HUB_CLASSES_SEQUENTIAL 1
#define HUB_CLASSES_CONCURRENT 2
int hub_set_class_launch(hub_ctx* ctx, int policy);

/* Build the sphere maps, orbital tables (grid-normalized, dV sum phi^2 = 1,
 * Sec. II), image/phase tables and the work list on the host.  Needs no GPU.
 * Errors: HUB_EINVAL (no sites, or a sphere that holds no grid point),
 * HUB_ENOMEM. */
int hub_finalize_host(hub_ctx* ctx);

/* hub_finalize_host (if not done) plus upload to the current HIP device;
 * stream (hipStream_t, may be NULL for the null stream) becomes the context
 * stream.  Errors: HUB_EDEVICE, HUB_ENOMEM. */
int hub_finalize(hub_ctx* ctx, void* stream);

/* Change the context stream (hipStream_t). */
int hub_set_stream(hub_ctx* ctx, void* stream);

/* Integer properties after hub_finalize_host: what = 0 sites, 1 orbitals J,
 * 2 state sets (nq; spinor: nk), 3 apply layers, 4 sphere entries, 5 chunks,
 * 6 species, 7 k-points, 8 nblk of n/pbar, 9 bytes of device tables,
 * 10 projection workspace rows (sum of L over chunks), 11 grouped chunks
 * (0 when the grouped work list was not built), 12 largest number of
 * orbitals covering one grid point, 13 dilated-sphere entries of the
 * state-gradient forces (0 before the first hub_forces_state_gradient),
 * 14 passes of the grouped apply (points covered by more than 16 orbitals
 * have their covers split over passes; 0 without a grouped work list),
 * 15 device allocations (hipMalloc) the context has made so far, 16 step
 * graphs captured so far (HUB_STEP_GRAPH keeps the last two argument sets'
 * graphs; a third set replaces the one used least recently). */
int hub_query(const hub_ctx* ctx, int what, int64_t* value);

/* Per-site data after hub_finalize_host: L = 2l+1, offset of its first
 * orbital in j, number of sphere points, species.  Any pointer may be NULL. */
int hub_site_info(const hub_ctx* ctx, int site, int* L, int* orb_offset,
                  int64_t* npoints, int* species);

/* Host copy of one site's sphere (Fig. 1): for every unfolded point p, in
 * order of (g, image): folded grid index g[p], lattice image image3[3p..3p+2]
 * (T_p = image * cell, r_p = r_g + T_p), orbital values phi[p*L + m] and, if
 * grad is not NULL, grad[(p*L + m)*3 + i] = d phi_m / d r_i.  Arrays sized by
 * hub_site_info's npoints.  Any output may be NULL. */
int hub_site_points(const hub_ctx* ctx, int site, int32_t* g, int32_t* image3,
                    double* phi, double* grad);

/* Projections (Eq. occ_matrices brackets; Fig. 1 phase):
 * c[q][j][col] = dV sum_p exp(+i k.T_p) phi_j(r_p) psi_q[g(p)][col] for every
 * state set q, orbital j and column col < ncol.  psi: device, layout above;
 * c: device, [nq][J][ncol].  nstates >= 1, ld >= ncol. */
int hub_project(hub_ctx* ctx, const void* psi, int64_t ld, int nstates, double* c);

/* hub_project for the state sets set0 .. set0 + nsets - 1 only (a caller
 * that holds one k-point, or one k-point and spin, at a time): psi holds
 * those sets (set stride G * ld elements) and c receives [nsets][J][ncol];
 * each set keeps its own k-point phase.  The occupations still need the
 * projections of every set (hub_occupations).  Errors: HUB_EINVAL (set range
 * outside 0 .. number of sets, as hub_project), HUB_ESTATE. */
int hub_project_sets(hub_ctx* ctx, const void* psi, int64_t ld, int nstates, int set0, int nsets,
                     double* c);

/* Occupations (Eq. occ_matrices), renormalized occupations N-bar
 * (Eq. notation_Nbar) and P-bar (Eq. notation_Pbar); spinors: App. A and B.
 * c: device [nq][J][ncol] from hub_project; f: device occupations.  Outputs
 * (device): n, pbar (may be NULL), nbar (may be NULL unless pbar is given:
 * then a NULL nbar uses an internal buffer). */
int hub_occupations(hub_ctx* ctx, const double* c, int nstates, const double* f,
                    double* n, double* pbar, double* nbar);

/* On-site Coulomb tensor (m m'|m'' m''') of one site (Sec. III, evaluated on
 * the grid; App. B notation): dV^2 sum_{p,p'} phi_a phi_b(p) K(p - p')
 * phi_c phi_d(p') over the site's unfolded sphere points, K = 1/|r| and
 * K(0) = the average of 1/r over one grid cell.  Cached in the context for
 * hub_acbn0_uj.  site = -1 computes every site.  tensor (device, may be NULL)
 * receives L^4 doubles [a][b][c][d] for a single site. */
int hub_coulomb(hub_ctx* ctx, int site, double* tensor);

/* Setup cache: the Coulomb tensors are the one costly part of the setup
 * (an O(P^2) sum per site) and depend only on the site's sphere (grid, cell,
 * centre, l, zeta, rc).  hub_get_coulomb copies the context's tensor of one
 * site (L^4 doubles [a][b][c][d], device) out; HUB_ESTATE if it has not been
 * computed or set.  hub_set_coulomb installs one (device, same layout), e.g.
 * from an earlier context with the same sphere, in place of hub_coulomb; the
 * caller vouches that it belongs to this site.  Both are asynchronous on the
 * context stream.  Errors: HUB_EINVAL (null tensor, bad site; set: a site
 * with spin-dependent orbitals), HUB_ESTATE (before hub_finalize). */
int hub_get_coulomb(hub_ctx* ctx, int site, double* tensor);
int hub_set_coulomb(hub_ctx* ctx, int site, const double* tensor);

/* ACBN0 U-bar, J-bar (Eqs. ACBN0_U, ACBN0_J; spinors App. B) and
 * U_eff = U-bar - J-bar per site, from n and pbar (device).  Sites with a
 * fixed U_eff (hub_set_fixed_ueff) report U = Ueff = fixed, J = 0.  Needs the
 * Coulomb tensors (hub_coulomb(ctx, -1, NULL)) or returns HUB_ESTATE.
 * status (device int32, may be NULL): 0, HUB_WDEGENERATE where a
 * denominator is below 1e-12 (that U or J is then 0), or HUB_ENONFINITE
 * where the site's occupations (or its U, J) are not finite (U, J, Ueff are
 * then NaN; a fixed U_eff is kept). */
int hub_acbn0_uj(hub_ctx* ctx, const double* n, const double* pbar,
                 double* U, double* J, double* Ueff, int* status);

/* Hubbard potential (Eq. pot_V_U), accumulated:
 * hpsi_q[g][col] += alpha * scale_q[s] * (V_U psi)_q[g][col], with
 * V_ab = Ueff (delta_ab / 2 - n_ba) per site and spin channel (spinor:
 * V^{ss'}_ab = Ueff (delta delta / 2 - n^{s's}_ba)), evaluated from the
 * projections c.  Ueff, n, c: device.  colscale: device [nsets][nstates] or
 * NULL (all ones).  hpsi: device, same layout as psi with leading dimension
 * ld; only sphere grid points are written. */
int hub_apply(hub_ctx* ctx, const double* Ueff, const double* n, const double* c,
              int nstates, const double* colscale, double alpha, void* hpsi, int64_t ld);

/* hub_apply for the state sets set0 .. set0 + nsets - 1 only: c, hpsi and
 * colscale ([nsets][nstates] or NULL) hold those sets; Ueff and n are the
 * context's (from every set).  Errors as hub_project_sets. */
int hub_apply_sets(hub_ctx* ctx, const double* Ueff, const double* n, const double* c, int nstates,
                   const double* colscale, double alpha, void* hpsi, int64_t ld, int set0, int nsets);

/* Dudarev energy per site (Eq. E_Dudarev; App. A for spinors):
 * EU[I] = Ueff/2 sum_sigma Tr[n - n n] (unpolarized counts the channel
 * twice).  Ueff, n, EU: device. */
int hub_energy(hub_ctx* ctx, const double* Ueff, const double* n, double* EU);

/* Energy bookkeeping of App. A per site, from the occupations n (layout of
 * hub_occupations) and the site's U and J (e.g. U-bar and J-bar of
 * hub_acbn0_uj): out[6 * I + 0..5] = N, m_x, m_y, m_z, E_DC, E_ee with
 *   N = sum_s sum_a n^{ss}_aa (unpolarized contexts count both spins),
 *   m_i = sum_st (sigma_i)_st rho^{st}, rho^{st} = sum_a n^{st}_aa (the
 *   magnetization of the shell: m_x = 2 Re rho^{ud}, m_y = 2 Im rho^{ud},
 *   m_z = rho^{uu} - rho^{dd}; collinear: (0, 0, N_up - N_dn)),
 *   E_DC = U/2 N(N-1) - J/2 N(N/2-1) - J/4 m.m (fully localized limit),
 *   E_ee = the noncollinear Hartree-Fock energy of App. A written for
 *   occupations diagonal in m, evaluated on the diagonal elements n^{st}_aa.
 * For m-diagonal occupations E_ee - E_DC equals hub_energy's E_U at
 * U_eff = U - J.  U, J, n, out: device. */
int hub_energy_fll(hub_ctx* ctx, const double* U, const double* J, const double* n, double* out);

/* Hubbard forces (Sec. IV) with frozen sphere membership and normalization:
 * F[I][i] = g_s * 2 Re sum_q w_k sum_s f_s sum_ab V_ab conj(d_{a,i}) c_b,
 * d = dV sum_p exp(i k.T_p) (d phi_a / d r_i)(r_p) psi[g(p)], g_s = 2 for
 * unpolarized contexts, else 1.  psi, c, f, Ueff, n, F: device. */
int hub_forces(hub_ctx* ctx, const void* psi, int64_t ld, int nstates, const double* c,
               const double* f, const double* Ueff, const double* n, double* F);

/* Hubbard forces through the derivatives of the states (Sec. IV, the form
 * the paper uses to reduce the egg-box effect): as hub_forces with
 * d_{a,i} = -<phi_a|D_i psi>, D_i the 4th-order central difference
 * (weights 1/12, -2/3, 0, 2/3, -1/12 over offsets -2..2, divided by h_i)
 * applied to the Bloch extension of psi (a neighbour past the cell face
 * along axis i is psi at the folded point times exp(i k_i a_i)).  Evaluated
 * by summation by parts as d = dV sum_p exp(i k.T_p) (D_i phi_a)(p) psi[g(p)]
 * over the dilated sphere (unfolded points within two steps of a sphere
 * point along an axis, phi zero off the sphere).  The first call builds and
 * uploads that work list (hipMalloc; not inside graph capture).  With a
 * vector potential on, the phases are those of hub_forces.  Arguments and
 * layout as hub_forces.  psi, c, f, Ueff, n, F: device. */
int hub_forces_state_gradient(hub_ctx* ctx, const void* psi, int64_t ld, int nstates, const double* c,
                              const double* f, const double* Ueff, const double* n, double* F);

/* Gradients of the total Hubbard energy E = sum_I E_U[I] (Eq. E_Dudarev; App. A
 * for spinors) with U_eff held fixed, as the ACBN0 potential prescribes (the
 * paper does not differentiate U-bar, J-bar; Sec. III), multiplied by scale
 * (e.g. the incoming gradient of a reverse-mode pass):
 *  - grad_psi (device, state layout with leading dimension ldg, may be NULL):
 *    overwritten with scale * 2 dE/dpsi*, the convention of PyTorch for
 *    complex inputs (real states: scale * dE/dpsi), i.e. by Eq. minimization
 *      grad_psi_q[g][col] = scale * 2 g_s dV w_k f_s (V_U psi)_q[g][col],
 *    g_s = 2 for unpolarized contexts (their channel stands for two spins),
 *    else 1; every used column of every grid point is written (zero off the
 *    spheres), padding columns past ncol are not touched;
 *  - grad_R (device [site][3], may be NULL): scale * dE/dR_I = -scale * F_I,
 *    F the forces of hub_forces (Sec. IV, through <grad phi|psi>, sphere
 *    membership and normalization frozen); needs psi (ld, nstates as in
 *    hub_forces).
 * c, n: from hub_project / hub_occupations on the same states; f: device
 * occupations [sets][nstates]; Ueff: device [site].  At least one output.
 * Errors: HUB_EINVAL (NULL inputs, no output, sizes, scale not finite),
 * HUB_ESTATE. */
int hub_energy_gradient(hub_ctx* ctx, const void* psi, int64_t ld, int nstates, const double* c,
                        const double* f, const double* Ueff, const double* n, double scale, void* grad_psi,
                        int64_t ldg, double* grad_R);

/* Velocity gauge (Sec. V): with a uniform vector potential A (host array of
 * 3, bohr^-1; NULL switches the field off), the projections and the apply
 * of every later call and graph replay use V^A = exp(-i A.r) V_U exp(i A.r):
 * the phase of sphere point p is exp(i (k+A).T_p) exp(i A.r_g), r_g the
 * cell grid point and T_p its lattice image (r_p = r_g + T_p, the unfolded
 * point).  Complex contexts of at most 2^28 - 1 grid points only (the
 * phase table is addressed with 32-bit byte offsets; HUB_EINVAL
 * otherwise).  The device tables
 * are updated on the context's stream, so a captured step graph stays valid
 * while the field is on; switching it on or off rebuilds the graph at the
 * next graph-mode hub_step.  With a field the grouped work list is launched
 * merged, and hub_forces uses the same phases. */
int hub_set_vector_potential(hub_ctx* ctx, const double* A);

/* DFT+U current correction of the velocity gauge (Sec. V, read with the
 * factor i of the velocity operator i[H, r] restored), per site and
 * Cartesian component: J[I][i] = g_s * 2 Im sum_q w_k sum_s f_s sum_a
 * conj(rho_{a,i}) sum_b V_ab c_b = sum w f <psi| i[V^A, r] |psi> restricted
 * to site I, with the position moments about the site centre
 * rho_{a,i} = dV sum_p exp(i k.T_p) exp(i A.r_p) (r_p - R_I)_i phi_a(p)
 * psi[g(p)] and c from hub_project under the same field; g_s = 2 for
 * unpolarized contexts, else 1.  psi, c, f, Ueff, n, J: device. */
int hub_current(hub_ctx* ctx, const void* psi, int64_t ld, int nstates, const double* c,
                const double* f, const double* Ueff, const double* n, double* J);

/* One whole Hubbard step: project -> occupations
 * (n, N-bar, P-bar) -> U-bar, J-bar, U_eff (or fixed U) -> hpsi += alpha V_U psi.
 * All pointers are device pointers owned by the caller; see the layouts
 * above.  mode: HUB_STEP_BATCHED, HUB_STEP_GRAPH (captured once per distinct
 * argument set and replayed; the graphs of the last two argument sets are
 * kept, counting hub_step_current's output pointer as an argument) or
 * HUB_STEP_PERSITE (one launch per site and stage).  Needs the Coulomb
 * tensors unless every site has a fixed U. */
typedef struct hub_step_io {
    const void* psi; int64_t ld; int nstates;
    const double* f;
    void* hpsi; int64_t ldh; double alpha;
    double* c; double* n; double* pbar; double* nbar;
    double* U; double* J; double* Ueff; int32_t* status;
} hub_step_io;
int hub_step(hub_ctx* ctx, const hub_step_io* io, int mode);

/* hub_step plus the DFT+U current correction of the velocity gauge (Sec. V)
 * of the step's input states and potential: J[site][3] (device, caller
 * owned, overwritten) is what hub_current(psi, io->c, io->f, io->Ueff,
 * io->n, J) returns after the step, formed before the apply (so hpsi may
 * alias psi).  For complex states on the grouped work list (modes
 * HUB_STEP_BATCHED and HUB_STEP_GRAPH; spin-dependent orbitals included)
 * one launch takes the projections c and the position-moment projections
 * rho_{a,i} in the same pass over the states; it sums each column's entries
 * in one sequence, so c and everything that follows from it (n, U, J,
 * U_eff, hpsi) agree with hub_step's to rounding, and J with hub_current's.
 * Elsewhere (HUB_STEP_PERSITE, the per-site work list, real states) it runs
 * hub_step's stages, bit for bit, and hub_current's own projection.  The first fused call uploads the moment
 * tables (three displacements per grouped point).  Errors: those of
 * hub_step; HUB_EINVAL for a null J. */
int hub_step_current(hub_ctx* ctx, const hub_step_io* io, double* J, int mode);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * batched hub_step (HUB_STEP_BATCHED, the same kernels and summation order,
 * hence the same results) with every workspace it needs (projection partial
 * sums, occupation partial sums, N-bar when io->nbar is NULL, the apply's
 * padding row) carved out of one static device array of HUB_SCRATCH_BYTES
 * per GPU, which the library holds until the process ends.  The call makes
 * no hipMalloc or hipFree and creates no event or graph; stage timing
 * (hub_profile) does not record it.  The scratch array is shared by every
 * context and call on one GPU and keeps the last call's contents (every
 * value a step reads from it is written earlier in the same step):
 * overlapping calls on one GPU, e.g. from two streams, race and must be
 * serialized by the caller.  Needs hub_finalize (which takes the array's
 * device address) and the Coulomb tensors unless every U_eff is fixed.
 * Errors: those of hub_step, and HUB_ESCRATCH when the step's workspace
 * exceeds HUB_SCRATCH_BYTES (nothing is launched). */
#define HUB_SCRATCH_BYTES (128u << 20)
int hub_step_noalloc(hub_ctx* ctx, const hub_step_io* io);

/* Per-stage device timing with HIP events recorded around the launches of
 * each stage on the context stream (eager launches only; a captured step
 * graph is not split).  Stages: HUB_STAGE_* below.  hub_profile(ctx, 1)
 * starts recording, 0 stops.  hub_profile_read synchronizes the context
 * stream, returns the accumulated milliseconds ms[HUB_NSTAGES] and launch
 * counts counts[HUB_NSTAGES] (host arrays, either may be NULL) and resets
 * them. */
#define HUB_NSTAGES 8
#define HUB_STAGE_PROJECT 0
#define HUB_STAGE_REDUCE 1
#define HUB_STAGE_NBAR 2
#define HUB_STAGE_OCC 3
#define HUB_STAGE_ACBN0 4
#define HUB_STAGE_APPLY 5
#define HUB_STAGE_GRADPROJ 6
#define HUB_STAGE_FORCES 7
int hub_profile(hub_ctx* ctx, int enable);
int hub_profile_read(hub_ctx* ctx, double* ms, int64_t* counts);

/* Release the context and everything it owns (waits for its stream). */
int hub_destroy(hub_ctx* ctx);

/* Static message for a status code. */
const char* hub_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* HUB_H */
