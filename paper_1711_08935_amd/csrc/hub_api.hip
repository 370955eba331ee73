// C ABI of the Hubbard library (declared in include/hub.h): context
// management, upload of the host tables, kernel-shape selection and the
// sequencing of the launches for each entry point, including the per-step
// hipGraph.  Every compute step runs in the HIP kernels of this directory.

#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "ksmall.h"

namespace {

constexpr double kTwoPi = 6.28318530717958647692;

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
};

struct GraphKey {
    hub_step_io io{};
    double* jcur = nullptr;                  // current output of hub_step_current, else null
    int ncol = 0;
    bool valid = false;
};

}  // namespace

// Workspace of hub_step_noalloc: a file-scope device array, one copy per
// GPU, alive until the process ends.  Host code never passes its name to a
// kernel or a copy (on the host it is only a stand-in symbol): it uses the
// device address that hipGetSymbolAddress returns for each device, taken
// once per device in hub_finalize with that device current.
static __device__ __align__(256) unsigned char scratch[HUB_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the scratch array on the current device ``dev``.
hipError_t scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
    return hipSuccess;
}

void* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}
}  // namespace

struct hub_ctx {
    double cell[3];
    int ngrid[3];
    int spin_mode, is_complex, precision;
    int nk = 1;
    std::vector<double> kred{0.0, 0.0, 0.0}, kw{1.0};
    std::vector<SiteDef> sites;
    int chunk_entries = 512;
    int tune_cpl[2] = {0, 0};
    int tune_waves[2] = {4, 4};
    int tune_layout[2] = {-1, -1};
    bool built_host = false, built_dev = false;
    HostTables T;
    int device = -1;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    // side streams (default priority) for the concurrent per-class launches
    hipStream_t side[HUB_NCLASS] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[HUB_NCLASS] = {};

    // device tables
    HubChunk* d_chunks = nullptr;
    int32_t *d_all = nullptr, *d_gidx = nullptr, *d_img = nullptr;
    double *d_phi = nullptr, *d_gphi = nullptr, *d_phase = nullptr;
    double* d_phi2 = nullptr;                // [e][sigma][m] spin-dependent orbitals
    double *d_gphi_dn = nullptr, *d_mphi_dn = nullptr;   // their gradient and moment tables
    int32_t *d_site_chunk_ptr = nullptr, *d_site_chunk_ids = nullptr, *d_orb_site = nullptr;
    int32_t *d_site_L = nullptr, *d_site_orb0 = nullptr, *d_site_species = nullptr;
    int32_t *d_species_orb_ptr = nullptr, *d_species_orb_ids = nullptr;
    double *d_kw = nullptr, *d_ueff_fixed = nullptr, *d_tensor = nullptr;
    // grouped (cover-signature) work list
    bool use_grouped = true;
    int class_policy = HUB_CLASSES_MERGED;
    int32_t* d_gall_m = nullptr;             // chunk list of the merged launch, by pass
    int32_t* d_gmom = nullptr;               // work items of the moment projection (k_project_mom.h)
    int nmom = 0;
    std::vector<int> gpass_ptr;              // d_gall_m[gpass_ptr[p], gpass_ptr[p+1]): chunks of pass p
    int gcls_ptr[HUB_NCLASS + 1] = {};       // d_gall[gcls_ptr[k-1], gcls_ptr[k]): chunks of class k
    HubChunk* d_gchunks = nullptr;
    int32_t *d_gall = nullptr, *d_ggidx = nullptr, *d_gf_orb = nullptr, *d_gf_img = nullptr;
    int32_t *d_gred_ptr = nullptr, *d_gred_row = nullptr, *d_gred_img = nullptr;
    int32_t* d_gspin_shift = nullptr;        // spin-dependent orbitals: L per orbital
    double* d_gtab = nullptr;
    double *d_gd0 = nullptr, *d_gfdel = nullptr;   // moment tables of the grouped list, uploaded
                                                   // at the first hub_step_current
    std::vector<char> have_tensor;
    size_t table_bytes = 0;

    // workspaces
    double* d_part = nullptr;
    size_t part_cap = 0;
    double* d_sink = nullptr;                // one state row for the apply's padding entries
    size_t sink_cap = 0;
    double* d_occ_ws = nullptr;              // partial occupation sums
    size_t occ_cap = 0;
    // velocity gauge (uniform vector potential A, Sec. V); off by default
    bool gauge = false;
    double A[3] = {0.0, 0.0, 0.0};
    double* d_pg = nullptr;                  // [G] exp(i A.r_g)
    double* d_mphi = nullptr;                // per-site position-moment table
    int32_t* d_images = nullptr;             // lattice images (3 ints each)
    double* d_kred = nullptr;                // reduced k-points (3 each)
    std::vector<double> phase_host;          // exp(i k.T) without a field
    double* d_grad = nullptr;
    size_t grad_cap = 0;
    // state-gradient force form: dilated-sphere tables, built at first use
    bool stencil_built = false;
    int stencil_nchunks = 0;
    int64_t stencil_part_rows = 0, stencil_entries = 0;
    HubChunk* d_st_chunks = nullptr;
    int32_t *d_st_all = nullptr, *d_st_gidx = nullptr, *d_st_site_ptr = nullptr, *d_st_site_ids = nullptr;
    double* d_st_tab = nullptr;
    double* d_st_tab_dn = nullptr;           // spin-down orbitals (spin-dependent contexts)
    double* d_nbar_ws = nullptr;
    size_t nbar_cap = 0;
    // Workspaces of the call in flight come from the buffers above (grown
    // with hipMalloc on demand) unless ws_fixed points at slices of the
    // static scratch array (hub_step_noalloc), which are used as they are.
    struct FixedWs {
        double* part;
        double* occ;
        double* nbar;
        double* sink;
    };
    const FixedWs* ws_fixed = nullptr;
    int64_t nalloc = 0;                      // device allocations made so far (hub_query 15)
    int64_t alloc_attempts = 0;
    int64_t fail_alloc = 0;                  // HUB_FAIL_ALLOC: the attempt that fails (0: none)

    // per-stage event timing
    bool prof = false;
    bool capturing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double prof_ms[HUB_NSTAGES] = {0};
    int64_t prof_n[HUB_NSTAGES] = {0};

    // captured steps: two, so that a caller that alternates between two
    // argument sets (e.g. hub_step and, every few steps, hub_step_current)
    // replays both without capturing again; the least recently used one is
    // replaced
    struct GraphSlot {
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
        GraphKey key;
        uint64_t used = 0;
    };
    GraphSlot gslot[2];
    uint64_t gclock = 0;
    int64_t ncapture = 0;                    // step graphs captured so far (hub_query 16)

    int nsets() const { return spin_mode == HUB_SPINOR ? nk : nk * (spin_mode == HUB_COLLINEAR ? 2 : 1); }
    int nspin() const { return spin_mode == HUB_COLLINEAR ? 2 : 1; }
    int nblk() const { return spin_mode == HUB_SPINOR ? 4 : (spin_mode == HUB_COLLINEAR ? 2 : 1); }
    int ncplx() const { return is_complex ? 2 : 1; }
    int ncol(int nstates) const { return spin_mode == HUB_SPINOR ? 2 * nstates : nstates; }
    size_t elem() const { return (precision == HUB_F64 ? 8 : 4) * static_cast<size_t>(ncplx()); }
    int64_t G() const { return static_cast<int64_t>(ngrid[0]) * ngrid[1] * ngrid[2]; }
};

namespace {

int map_err(hipError_t e) {
    if (e == hipSuccess) return HUB_OK;
    if (e == hipErrorOutOfMemory) return HUB_ENOMEM;
    return HUB_EDEVICE;
}

#define HUB_TRY(expr)                          \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return map_err(_e); \
    } while (0)

// Every device allocation of a context goes through here (counted).  With
// HUB_FAIL_ALLOC=N in the environment at hub_create, the context's N-th
// allocation attempt fails once, as an out-of-memory would.
template <typename T>
hipError_t dev_malloc(hub_ctx* c, T** p, size_t bytes) {
    if (++c->alloc_attempts == c->fail_alloc) return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
    if (e == hipSuccess) ++c->nalloc;
    return e;
}

template <typename T>
hipError_t upload(hub_ctx* c, T** dst, const std::vector<T>& src, size_t& bytes) {
    const size_t nb = std::max<size_t>(1, src.size()) * sizeof(T);
    hipError_t e = dev_malloc(c, dst, nb);
    if (e != hipSuccess) return e;
    bytes += nb;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

void drop_graph(hub_ctx* c);

// Frees every device table and workspace and leaves the pointers null (so a
// failed hub_finalize can be retried and hub_destroy frees nothing twice).
void release(hub_ctx* c) {
    auto f = [](auto*& p) {
        if (p) (void)hipFree(p);
        p = nullptr;
    };
    f(c->d_chunks); f(c->d_all); f(c->d_gidx); f(c->d_img); f(c->d_phi); f(c->d_gphi); f(c->d_phase);
    f(c->d_site_chunk_ptr); f(c->d_site_chunk_ids); f(c->d_orb_site); f(c->d_site_L); f(c->d_site_orb0);
    f(c->d_site_species); f(c->d_species_orb_ptr); f(c->d_species_orb_ids); f(c->d_kw); f(c->d_ueff_fixed);
    f(c->d_tensor); f(c->d_part); f(c->d_grad); f(c->d_nbar_ws); f(c->d_sink); f(c->d_occ_ws);
    f(c->d_pg); f(c->d_mphi); f(c->d_images); f(c->d_kred);
    c->part_cap = c->grad_cap = c->nbar_cap = c->sink_cap = c->occ_cap = 0;
    f(c->d_phi2); f(c->d_gphi_dn); f(c->d_mphi_dn);
    f(c->d_st_chunks); f(c->d_st_all); f(c->d_st_gidx); f(c->d_st_site_ptr); f(c->d_st_site_ids); f(c->d_st_tab); f(c->d_st_tab_dn);
    f(c->d_gchunks); f(c->d_gall); f(c->d_gall_m); f(c->d_gmom); f(c->d_ggidx); f(c->d_gf_orb); f(c->d_gf_img); f(c->d_gred_ptr);
    f(c->d_gred_row); f(c->d_gred_img); f(c->d_gtab); f(c->d_gspin_shift); f(c->d_gd0); f(c->d_gfdel);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (int k = 0; k < HUB_NCLASS; ++k) {
        if (c->side[k]) (void)hipStreamDestroy(c->side[k]);
        if (c->join_ev[k]) (void)hipEventDestroy(c->join_ev[k]);
        c->side[k] = nullptr;
        c->join_ev[k] = nullptr;
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    c->fork_ev = nullptr;
    c->cap_stream = nullptr;
}

void drop_slot(hub_ctx::GraphSlot& g) {
    if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.gexec = nullptr;
    g.graph = nullptr;
    g.key.valid = false;
}

void drop_graph(hub_ctx* c) {
    for (auto& g : c->gslot) drop_slot(g);
}

// Stage timer: records an event pair around the launches of one stage when
// profiling is on and no graph is being captured.
struct StageTimer {
    hub_ctx* c;
    int stage;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEvent_t get() {
        if (!c->ev_pool.empty()) {
            hipEvent_t e = c->ev_pool.back();
            c->ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    StageTimer(hub_ctx* ctx, int st) : c(ctx), stage(st) {
        if (c->prof && !c->capturing && !c->ws_fixed) {
            e0 = get();
            e1 = get();
            if (e0) (void)hipEventRecord(e0, c->stream);
        }
    }
    ~StageTimer() {
        if (e0 && e1) {
            (void)hipEventRecord(e1, c->stream);
            c->ev_pending.push_back({stage, {e0, e1}});
        } else {
            if (e0) c->ev_pool.push_back(e0);
            if (e1) c->ev_pool.push_back(e1);
        }
    }
};

int ensure(double** buf, size_t* cap, size_t n, hub_ctx* c) {
    if (*cap >= n && *buf) return HUB_OK;
    if (*buf) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
        drop_graph(c);
    }
    hipError_t e = dev_malloc(c, buf, std::max<size_t>(1, n) * sizeof(double));
    if (e != hipSuccess) return map_err(e);
    *cap = n;
    return HUB_OK;
}

// Columns per lane: by default the vector that gives each lane 16 bytes per
// state row (lanes span several state sets when a set is narrow), provided
// every lane's columns stay aligned and inside the row (ld % cpl == 0).  The
// apply (which = 1) stores whole vectors, so its lanes must also end at the
// last used column (ncol % cpl == 0): a caller's padding columns past ncol
// are never written.
int pick_cpl(const hub_ctx* c, const void* ptr, int64_t ld, int which, int ncol) {
    const size_t e = c->elem();
    auto ok = [&](int cpl) {
        const size_t vb = std::min<size_t>(16, cpl * e);
        return (ld % cpl == 0) && (which == 0 || ncol % cpl == 0) &&
               (reinterpret_cast<uintptr_t>(ptr) % vb == 0);
    };
    const int want = c->tune_cpl[which];
    if (want == 1 || ((want == 2 || want == 4) && ok(want))) return want;
    for (int cpl : {4, 2, 1}) {
        if (cpl * e <= 16 && ok(cpl)) return cpl;
    }
    return 1;
}

// Lane layout: one state set per wave when a set fills whole waves (uniform
// set index, scalar row bases), else sets packed across the lanes.
int pick_wide(const hub_ctx* c, int ncol, int cpl, int which) {
    if (c->tune_layout[which] >= 0) return c->tune_layout[which];
    return ncol >= 64 * cpl ? 1 : 0;
}

bool built(const hub_ctx* c) { return c && c->built_dev; }

// Batched launches use the grouped work list when it exists.
bool grouped(const hub_ctx* c) { return c->use_grouped && c->T.grouped.ok; }

// Columns per lane so that a lane's FP64 accumulators (functions x scalars)
// stay within 96 values (nf: the largest function count launched).
int clamp_cpl(const hub_ctx* c, int cpl, int nf) {
    while (cpl > 1 && nf * cpl * c->ncplx() > 96) cpl /= 2;
    return cpl;
}

// Runs launch(k, list, nchunks, stream) over the grouped work list: once
// with a merged class k (HUB_MERGED8 when no point carries more than 8
// functions, else HUB_MERGED16) and the merged chunk list, or once per non-empty
// function-count class k.  Concurrent class launches go to side streams
// forked from the context's stream and joined back to it: the classes write
// disjoint outputs, so their kernels run concurrently (parallel branches of
// a captured graph).
//
// With more than one pass (points with more than HUB_GF_MAX functions), the
// launches are merged: the apply (per_pass) launches the passes one after
// the other, since a point appears once per pass; the projection launches
// every pass at once.
template <typename F>
int run_classes(hub_ctx* c, F&& launch, bool per_pass = false) {
    const int np = c->T.grouped.npass;
    if (np > 1) {
        if (!per_pass) {
            HUB_TRY(launch(HUB_MERGED16, c->d_gall_m, c->gpass_ptr[np], c->stream));
            return HUB_OK;
        }
        for (int p = 0; p < np; ++p)
            HUB_TRY(launch(HUB_MERGED16, c->d_gall_m + c->gpass_ptr[p], c->gpass_ptr[p + 1] - c->gpass_ptr[p],
                           c->stream));
        return HUB_OK;
    }
    // the velocity-gauge kernels are built for the merged launch only
    if (c->class_policy == HUB_CLASSES_MERGED || c->gauge) {
        const int merged = c->T.grouped.nfmax <= 8 ? HUB_MERGED8 : HUB_MERGED16;
        HUB_TRY(launch(merged, c->d_gall_m, c->gcls_ptr[HUB_NCLASS], c->stream));
        return HUB_OK;
    }
    auto one = [&](int k, hipStream_t s) {
        return launch(k, c->d_gall + c->gcls_ptr[k - 1], c->gcls_ptr[k] - c->gcls_ptr[k - 1], s);
    };
    // classes with fewer chunks first: their work-groups get CUs before the
    // largest class fills the chip, so their short grids overlap with it
    int used[HUB_NCLASS], nu = 0;
    for (int k = 1; k <= HUB_NCLASS; ++k)
        if (c->gcls_ptr[k] > c->gcls_ptr[k - 1]) used[nu++] = k;
    std::stable_sort(used, used + nu, [c](int x, int y) {
        return c->gcls_ptr[x] - c->gcls_ptr[x - 1] < c->gcls_ptr[y] - c->gcls_ptr[y - 1];
    });
    if (nu == 1 || c->class_policy == HUB_CLASSES_SEQUENTIAL) {
        for (int i = 0; i < nu; ++i) HUB_TRY(one(used[i], c->stream));
        return HUB_OK;
    }
    HUB_TRY(hipEventRecord(c->fork_ev, c->stream));
    for (int i = 0; i < nu; ++i) {
        HUB_TRY(hipStreamWaitEvent(c->side[i], c->fork_ev, 0));
        HUB_TRY(one(used[i], c->side[i]));
        HUB_TRY(hipEventRecord(c->join_ev[i], c->side[i]));
    }
    for (int i = 0; i < nu; ++i) HUB_TRY(hipStreamWaitEvent(c->stream, c->join_ev[i], 0));
    return HUB_OK;
}

// Orbital table of a projection: values, gradients (forces), position
// moments about the site centre (velocity-gauge current) or the 4th-order
// differences of the orbitals on the dilated spheres (state-gradient forces,
// a work list of its own).
enum { TAB_PHI = 0, TAB_GRAD = 1, TAB_MOMENT = 2, TAB_STENCIL = 3, TAB_GRAD_DN = 4, TAB_MOMENT_DN = 5,
       TAB_STENCIL_DN = 6 };
bool stencil_table(int table) { return table == TAB_STENCIL || table == TAB_STENCIL_DN; }

ProjArgs proj_args(hub_ctx* c, const void* psi, int64_t ld, int ncol, int table) {
    const bool grad = table != TAB_PHI;
    ProjArgs a{};
    a.psi = psi;
    a.ld = ld;
    a.qstride = c->G() * ld * c->ncplx();
    a.ncol = ncol;
    a.ncplx = c->ncplx();
    a.nq = c->nsets();
    a.chunks = c->d_chunks;
    a.chunk_list = c->d_all;
    a.gidx = c->d_gidx;
    a.tab = table == TAB_GRAD ? c->d_gphi : (table == TAB_MOMENT ? c->d_mphi : c->d_phi);
    if (table == TAB_GRAD_DN) a.tab = c->d_gphi_dn;         // spin-down orbitals' tables
    if (table == TAB_MOMENT_DN) a.tab = c->d_mphi_dn;
    a.tabmult = grad ? 3 : 1;
    if (table == TAB_PHI && c->T.spindep) {
        // both spin components' orbitals: 2L functions per entry
        a.tab = c->d_phi2;
        a.tabmult = 2;
    }
    a.prows = c->T.part_rows * a.tabmult;
    if (stencil_table(table)) {
        a.chunks = c->d_st_chunks;
        a.chunk_list = c->d_st_all;
        a.gidx = c->d_st_gidx;
        a.tab = table == TAB_STENCIL ? c->d_st_tab : c->d_st_tab_dn;
        a.prows = c->stencil_part_rows * 3;
    }
    a.pg = c->gauge ? c->d_pg : nullptr;
    return a;
}

ReduceArgs reduce_args(hub_ctx* c, const double* part, double* out, int ncol, int mult) {
    ReduceArgs r{};
    r.part = part;
    r.prows = c->T.part_rows * mult;
    r.out = out;
    r.nrows = c->T.J * mult;
    r.ncol = ncol;
    r.ncplx = c->ncplx();
    r.mult = mult;
    r.pmult = mult;
    r.spindep = 0;
    r.q0 = 0;
    r.colpar = -1;
    r.chunks = c->d_chunks;
    r.site_chunk_ptr = c->d_site_chunk_ptr;
    r.site_chunk_ids = c->d_site_chunk_ids;
    r.orb_site = c->d_orb_site;
    r.site_orb0 = c->d_site_orb0;
    r.site_L = c->d_site_L;
    r.phase = c->d_phase;
    r.nimg = static_cast<int>(c->T.images.size() / 3);
    r.nspin = c->nspin();
    r.spinor = c->spin_mode == HUB_SPINOR;
    r.dV = (c->cell[0] / c->ngrid[0]) * (c->cell[1] / c->ngrid[1]) * (c->cell[2] / c->ngrid[2]);
    return r;
}

// project + reduce into c (per_site: one projection launch per site)
size_t part_need(const hub_ctx* c, int ncol, int mult) {
    int64_t rows = std::max<int64_t>(c->T.part_rows * mult, c->T.grouped.ok ? c->T.grouped.part_rows : 0);
    if (mult == 3) rows = std::max<int64_t>(rows, c->stencil_part_rows * 3);
    return static_cast<size_t>(c->nsets()) * rows * ncol * c->ncplx();
}
// the grouped projection with the three position-moment components as well
size_t part_need_moments(const hub_ctx* c, int ncol) {
    return std::max(part_need(c, ncol, 3),
                    static_cast<size_t>(4) * c->nsets() * c->T.grouped.part_rows * ncol * c->ncplx());
}
// whether hub_step_current takes the moments in the step's own projection
bool fused_moments(const hub_ctx* c) { return grouped(c) && c->is_complex; }

// q0, nq: the state sets projected (psi and out hold those sets only);
// nq < 0: every set of the context.
// colpar >= 0: the reduction writes only the columns of that parity (the
// spin component whose orbitals the table holds).
// mout (grouped list, every set): the projections on the position moments
// about the site centres as well, mout[q][3 j + i][col], from the same
// pass over psi.
int do_project(hub_ctx* c, const void* psi, int64_t ld, int nstates, double* out, bool per_site,
               int table = TAB_PHI, int q0 = 0, int nq = -1, int colpar = -1, double* mout = nullptr) {
    if (nq < 0) nq = c->nsets();
    const bool grad = table != TAB_PHI;
    const bool spindep = !grad && c->T.spindep;
    const int ncol = c->ncol(nstates);
    const int mult = grad ? 3 : 1;
    if (mout && (per_site || grad || !fused_moments(c) || !c->d_gd0 || c->ws_fixed || q0 != 0 ||
                 nq != c->nsets()))
        return HUB_ESTATE;
    double* part = c->ws_fixed ? c->ws_fixed->part : nullptr;
    if (!part) {
        const size_t need = mout ? part_need_moments(c, ncol) : part_need(c, ncol, spindep ? 2 : mult);
        const int st = ensure(&c->d_part, &c->part_cap, need, c);
        if (st) return st;
        part = c->d_part;
    }
    ProjArgs a = proj_args(c, psi, ld, ncol, table);
    a.part = part;
    a.nq = nq;
    if (!per_site && !grad && grouped(c)) {
        const GroupTables& GT = c->T.grouped;
        a.chunks = c->d_gchunks;
        a.gidx = c->d_ggidx;
        a.tab = c->d_gtab;
        a.tabmult = 1;               // grouped chunks count their functions in C.L
        a.prows = GT.part_rows;
        const int64_t pplane = static_cast<int64_t>(nq) * GT.part_rows * ncol * c->ncplx();
        if (mout) {
            // orbitals and position moments in one launch over every chunk
            a.chunk_list = c->d_gmom;
            a.d0 = c->d_gd0;
            a.fdel = c->d_gfdel;
            a.pplane = pplane;
            StageTimer tm(c, HUB_STAGE_PROJECT);
            HUB_TRY(c->precision == HUB_F64 ? launch_project_mom_f64(a, c->nmom, nq, c->stream)
                                            : launch_project_mom_f32(a, c->nmom, nq, c->stream));
        } else {
            StageTimer tm(c, HUB_STAGE_PROJECT);
            // one launch per function-count class
            const int st = run_classes(c, [&](int k, const int32_t* list, int nch, hipStream_t s) {
                ProjArgs b = a;
                b.chunk_list = list;
                const int cpl = clamp_cpl(c, pick_cpl(c, psi, ld, 0, ncol), hub_cls_nfmax(k));
                b.wide = pick_wide(c, ncol, cpl, 0);
                return launch_project(b, nch, nq, c->precision, c->is_complex, cpl, c->tune_waves[0], k, s);
            });
            if (st) return st;
        }
        ReduceGroupedArgs r{};
        r.part = part;
        r.prows = GT.part_rows;
        r.out = out;
        r.J = c->T.J;
        r.ncol = ncol;
        r.ncplx = c->ncplx();
        r.red_ptr = c->d_gred_ptr;
        r.red_row = c->d_gred_row;
        r.red_img = c->d_gred_img;
        r.rows_per_orbital = GT.red_ptr.empty() ? 0 : GT.red_ptr.back() / std::max(1, c->T.J);
        r.spin_shift = c->T.spindep ? c->d_gspin_shift : nullptr;
        r.phase = c->d_phase;
        r.nimg = static_cast<int>(c->T.images.size() / 3);
        r.nspin = c->nspin();
        r.spinor = c->spin_mode == HUB_SPINOR;
        r.q0 = q0;
        r.dV = (c->cell[0] / c->ngrid[0]) * (c->cell[1] / c->ngrid[1]) * (c->cell[2] / c->ngrid[2]);
        if (mout) {
            r.ncomp = 4;
            r.mout = mout;
            r.pplane = pplane;
        }
        StageTimer tm(c, HUB_STAGE_REDUCE);
        HUB_TRY(launch_reduce_grouped(r, nq, c->stream));
        return HUB_OK;
    }
    // per-site chunks of spin-dependent orbitals have no velocity-gauge form
    if (spindep && c->gauge) return HUB_ESTATE;
    int cpl = pick_cpl(c, psi, ld, 0, ncol);
    // gradient tiles hold 3L functions, spin-dependent tiles 2L
    if ((grad || spindep) && cpl * c->ncplx() > 4) cpl = 4 / c->ncplx();
    a.wide = pick_wide(c, ncol, cpl, 0);
    const int waves = c->tune_waves[0];
    {
    StageTimer tm(c, grad ? HUB_STAGE_GRADPROJ : HUB_STAGE_PROJECT);
    if (!per_site) {
        const int nch = stencil_table(table) ? c->stencil_nchunks : static_cast<int>(c->T.chunks.size());
        HUB_TRY(launch_project(a, nch, nq, c->precision, c->is_complex, cpl, waves, 0, c->stream));
    } else {
        for (int s = 0; s < c->T.nsites; ++s) {
            ProjArgs b = a;
            b.chunk_list = c->d_site_chunk_ids + c->T.site_chunk_ptr[s];
            HUB_TRY(launch_project(b, c->T.site_chunk_ptr[s + 1] - c->T.site_chunk_ptr[s], nq, c->precision,
                                   c->is_complex, cpl, waves, 0, c->stream));
        }
    }
    }
    ReduceArgs r = reduce_args(c, part, out, ncol, mult);
    r.q0 = q0;
    r.colpar = colpar;
    if (spindep) {
        // column 2s + sigma takes the rows of its spin component's orbitals
        r.pmult = 2;
        r.spindep = 1;
        r.prows = c->T.part_rows * 2;
    }
    if (stencil_table(table)) {
        r.chunks = c->d_st_chunks;
        r.site_chunk_ptr = c->d_st_site_ptr;
        r.site_chunk_ids = c->d_st_site_ids;
        r.prows = c->stencil_part_rows * 3;
    }
    StageTimer tm(c, HUB_STAGE_REDUCE);
    HUB_TRY(launch_reduce(r, nq, c->stream));
    return HUB_OK;
}

size_t occ_need(const hub_ctx* c, int nstates) {
    const int nchan = c->spin_mode == HUB_SPINOR ? 1 : c->nspin();
    return static_cast<size_t>(c->T.nsites) * nchan * hub_occ_splits(c->nk, nstates) * HUB_OCC_PAIRS * 4;
}

int do_occupations(hub_ctx* c, const double* cc, int nstates, const double* f, double* n, double* pbar, double* nbar,
                   bool per_site) {
    const int ncol = c->ncol(nstates);
    double* ws = c->ws_fixed ? c->ws_fixed->occ : nullptr;
    if (!ws) {
        const int st = ensure(&c->d_occ_ws, &c->occ_cap, occ_need(c, nstates), c);
        if (st) return st;
        ws = c->d_occ_ws;
    }
    if (pbar && !nbar) {
        if (c->ws_fixed) {
            nbar = c->ws_fixed->nbar;
        } else {
            const size_t need = static_cast<size_t>(c->nsets()) * c->T.nspecies * nstates;
            const int st = ensure(&c->d_nbar_ws, &c->nbar_cap, need, c);
            if (st) return st;
            nbar = c->d_nbar_ws;
        }
    }
    if (nbar) {
        NbarArgs b{};
        b.c = cc;
        b.nbar = nbar;
        b.J = c->T.J;
        b.ncol = ncol;
        b.nstates = nstates;
        b.ncplx = c->ncplx();
        b.spinor = c->spin_mode == HUB_SPINOR;
        b.nspecies = c->T.nspecies;
        b.species_orb_ptr = c->d_species_orb_ptr;
        b.species_orb_ids = c->d_species_orb_ids;
        StageTimer tm(c, HUB_STAGE_NBAR);
        HUB_TRY(launch_nbar(b, c->nsets(), c->stream));
    }
    OccArgs o{};
    o.c = cc;
    o.f = f;
    o.nbar = nbar;
    o.n = n;
    o.pbar = pbar;
    o.kweights = c->d_kw;
    o.site_L = c->d_site_L;
    o.site_orb0 = c->d_site_orb0;
    o.site_species = c->d_site_species;
    o.J = c->T.J;
    o.ncol = ncol;
    o.nstates = nstates;
    o.ncplx = c->ncplx();
    o.spinor = c->spin_mode == HUB_SPINOR;
    o.nspin = c->nspin();
    o.nk = c->nk;
    o.nblk = c->nblk();
    o.nspecies = c->T.nspecies;
    o.nsplit = hub_occ_splits(c->nk, nstates);
    o.ws = ws;
    StageTimer tm(c, HUB_STAGE_OCC);
    if (!per_site) {
        HUB_TRY(launch_occ(o, 0, c->T.nsites, c->stream));
    } else {
        for (int s = 0; s < c->T.nsites; ++s) HUB_TRY(launch_occ(o, s, 1, c->stream));
    }
    return HUB_OK;
}

// N-bar, n, P-bar and U-bar, J-bar, U_eff of the batched step in two
// launches (k_step_occ_part, k_step_occ_final): the same sums in the same
// order as do_occupations followed by do_acbn0.
int do_step_occ(hub_ctx* c, const hub_step_io* io) {
    double* ws = c->ws_fixed ? c->ws_fixed->occ : nullptr;
    if (!ws) {
        const int st = ensure(&c->d_occ_ws, &c->occ_cap, occ_need(c, io->nstates), c);
        if (st) return st;
        ws = c->d_occ_ws;
    }
    OccArgs o{};
    o.c = io->c;
    o.f = io->f;
    o.n = io->n;
    o.pbar = io->pbar;
    o.kweights = c->d_kw;
    o.site_L = c->d_site_L;
    o.site_orb0 = c->d_site_orb0;
    o.site_species = c->d_site_species;
    o.J = c->T.J;
    o.ncol = c->ncol(io->nstates);
    o.nstates = io->nstates;
    o.ncplx = c->ncplx();
    o.spinor = c->spin_mode == HUB_SPINOR;
    o.nspin = c->nspin();
    o.nk = c->nk;
    o.nblk = c->nblk();
    o.nspecies = c->T.nspecies;
    o.nsplit = hub_occ_splits(c->nk, io->nstates);
    o.ws = ws;
    o.nsites = c->T.nsites;
    o.species_orb_ptr = c->d_species_orb_ptr;
    o.species_orb_ids = c->d_species_orb_ids;
    o.nbar_out = io->nbar;
    Acbn0Args u{};
    u.n = io->n;
    u.pbar = io->pbar;
    u.tensor = c->d_tensor;
    u.site_L = c->d_site_L;
    u.ueff_fixed = c->d_ueff_fixed;
    u.U = io->U;
    u.J = io->J;
    u.Ueff = io->Ueff;
    u.status = io->status;
    u.nblk = c->nblk();
    StageTimer tm(c, HUB_STAGE_OCC);
    HUB_TRY(launch_step_occ(o, u, c->stream));
    return HUB_OK;
}

bool need_tensors(const hub_ctx* c) {
    for (size_t s = 0; s < c->sites.size(); ++s)
        if (std::isnan(c->sites[s].ueff_fixed) && !c->have_tensor[s]) return true;
    return false;
}

int do_acbn0(hub_ctx* c, const double* n, const double* pbar, double* U, double* J, double* Ueff, int32_t* status,
             bool per_site) {
    Acbn0Args a{};
    a.n = n;
    a.pbar = pbar;
    a.tensor = c->d_tensor;
    a.site_L = c->d_site_L;
    a.ueff_fixed = c->d_ueff_fixed;
    a.U = U;
    a.J = J;
    a.Ueff = Ueff;
    a.status = status;
    a.nblk = c->nblk();
    StageTimer tm(c, HUB_STAGE_ACBN0);
    if (!per_site) {
        HUB_TRY(launch_acbn0(a, 0, c->T.nsites, c->stream));
    } else {
        for (int s = 0; s < c->T.nsites; ++s) HUB_TRY(launch_acbn0(a, s, 1, c->stream));
    }
    return HUB_OK;
}

// q0, nq: the state sets updated (cc, colscale and hpsi hold those sets
// only); nq < 0: every set of the context.
// occ: when not null, each column is also weighted by w_k f_s of its state
// (f: [nsets][nstates] of the context, kw: the k-point weights).
int do_apply(hub_ctx* c, const double* Ueff, const double* n, const double* cc, int nstates, const double* colscale,
             double alpha, void* hpsi, int64_t ld, bool per_site, int q0 = 0, int nq = -1,
             const double* occ = nullptr) {
    if (nq < 0) nq = c->nsets();
    const int ncol = c->ncol(nstates);
    double* sink = c->ws_fixed ? c->ws_fixed->sink : nullptr;
    if (!sink) {
        const int st = ensure(&c->d_sink, &c->sink_cap, static_cast<size_t>(ld) * c->ncplx(), c);
        if (st) return st;
        sink = c->d_sink;
    }
    ApplyArgs a{};
    a.hpsi = hpsi;
    a.sink = sink;
    a.pg = c->gauge ? c->d_pg : nullptr;
    a.ld = ld;
    a.qstride = c->G() * ld * c->ncplx();
    a.ncol = ncol;
    a.nstates = nstates;
    a.nq = nq;
    a.q0 = q0;
    a.nspin = c->nspin();
    a.spinor = c->spin_mode == HUB_SPINOR;
    a.nblk = c->nblk();
    a.chunks = c->d_chunks;
    a.gidx = c->d_gidx;
    a.tab = c->d_phi;
    a.phase = c->d_phase;
    a.nimg = static_cast<int>(c->T.images.size() / 3);
    a.c = cc;
    a.J = c->T.J;
    a.n = n;
    a.ueff = Ueff;
    a.colscale = colscale;
    a.occ = occ;
    a.kw = c->d_kw;
    a.alpha = alpha;
    a.orb_site = c->d_orb_site;
    a.site_orb0 = c->d_site_orb0;
    a.site_L = c->d_site_L;
    a.spindep = c->T.spindep ? 1 : 0;
    if (!per_site && grouped(c)) {
        a.wide = 1;
        a.chunks = c->d_gchunks;
        a.gidx = c->d_ggidx;
        a.tab = c->d_gtab;
        a.f_orb = c->d_gf_orb;
        a.f_img = c->d_gf_img;
        StageTimer tm(c, HUB_STAGE_APPLY);
        // one launch per function-count class; the classes hold disjoint points
        return run_classes(c, [&](int k, const int32_t* list, int nch, hipStream_t s) {
            ApplyArgs b = a;
            b.chunk_list = list;
            const int cpl = clamp_cpl(c, pick_cpl(c, hpsi, ld, 1, ncol), hub_cls_nfmax(k));
            return launch_apply_grouped(b, nch, nq, c->precision, c->is_complex, cpl, c->tune_waves[1], k, s);
        }, true);
    }
    int cpl = pick_cpl(c, hpsi, ld, 1, ncol);
    if (c->T.spindep) {
        if (c->gauge) return HUB_ESTATE;       // no velocity-gauge form of these per-site chunks
        // 2L functions per entry: both spin components' orbitals
        a.tab = c->d_phi2;
        a.spindep = 1;
        if (cpl * c->ncplx() > 4) cpl = 4 / c->ncplx();
    }
    a.wide = pick_wide(c, ncol, cpl, 1);
    const int waves = c->tune_waves[1];
    const int ns = c->T.nsites;
    StageTimer tm(c, HUB_STAGE_APPLY);
    for (int lay = 0; lay < c->T.nlayers; ++lay) {
        if (!per_site) {
            ApplyArgs b = a;
            const int c0 = c->T.layer_chunk_ptr[lay];
            b.chunk_list = c->d_all + c0;
            HUB_TRY(launch_apply(b, c->T.layer_chunk_ptr[lay + 1] - c0, nq, c->precision, c->is_complex, cpl,
                                 waves, c->stream));
        } else {
            for (int s = 0; s < ns; ++s) {
                const int c0 = c->T.layer_site_ptr[static_cast<size_t>(lay) * ns + s];
                const int c1 = c->T.layer_site_ptr[static_cast<size_t>(lay) * ns + s + 1];
                if (c1 <= c0) continue;
                ApplyArgs b = a;
                b.chunk_list = c->d_all + c0;
                HUB_TRY(launch_apply(b, c1 - c0, nq, c->precision, c->is_complex, cpl, waves, c->stream));
            }
        }
    }
    return HUB_OK;
}

int contract_moments(hub_ctx* c, const void* psi, int64_t ld, int nstates, const double* cc, const double* f,
                     const double* Ueff, const double* n, double* out, int table, double fscale = 1.0);
int moment_contraction(hub_ctx* c, const double* cc, const double* f, const double* Ueff, const double* n,
                       const double* d, int nstates, double* out, bool imag, double fscale);

// One step; jcur: also the velocity-gauge current of the step's states and
// potential (hub_current), from the moments that the step's projection
// takes in the same pass over psi where the work list allows, else from a
// projection of its own.  It is formed before the apply, so hpsi may alias
// psi.
int run_step(hub_ctx* c, const hub_step_io* io, bool per_site, double* jcur = nullptr) {
    const bool fused = jcur && !per_site && fused_moments(c);
    int st = do_project(c, io->psi, io->ld, io->nstates, io->c, per_site, TAB_PHI, 0, -1, -1,
                        fused ? c->d_grad : nullptr);
    if (st) return st;
    if (per_site) {
        // the plain path: one launch per site and stage
        st = do_occupations(c, io->c, io->nstates, io->f, io->n, io->pbar, io->nbar, true);
        if (st) return st;
        st = do_acbn0(c, io->n, io->pbar, io->U, io->J, io->Ueff, io->status, true);
    } else {
        st = do_step_occ(c, io);
    }
    if (st) return st;
    if (jcur) {
        st = fused ? moment_contraction(c, io->c, io->f, io->Ueff, io->n, c->d_grad, io->nstates, jcur, true, 1.0)
                   : contract_moments(c, io->psi, io->ld, io->nstates, io->c, io->f, io->Ueff, io->n, jcur,
                                      TAB_MOMENT);
        if (st) return st;
    }
    return do_apply(c, io->Ueff, io->n, io->c, io->nstates, nullptr, io->alpha, io->hpsi, io->ldh, per_site);
}

bool valid_states(const hub_ctx* c, const void* psi, int64_t ld, int nstates) {
    return psi != nullptr && nstates >= 1 && ld >= c->ncol(nstates);
}

// Argument checks of a whole step (hub_step, hub_step_noalloc).
int check_step(const hub_ctx* c, const hub_step_io* io) {
    if (!c || !io) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (!valid_states(c, io->psi, io->ld, io->nstates) || !valid_states(c, io->hpsi, io->ldh, io->nstates))
        return HUB_EINVAL;
    if (!io->f || !io->c || !io->n || !io->pbar || !io->U || !io->J || !io->Ueff || !std::isfinite(io->alpha))
        return HUB_EINVAL;
    if (need_tensors(c)) return HUB_ESTATE;
    return HUB_OK;
}

// doubles, rounded up so that every slice of the scratch array starts on a
// 256-byte boundary
size_t slice256(size_t n) { return (n + 31) / 32 * 32; }

// hub_step and hub_step_current (jcur: the current's output, else null).
int step_impl(hub_ctx* c, const hub_step_io* io, int mode, double* jcur) {
    int st = check_step(c, io);
    if (st) return st;
    if (mode != HUB_STEP_BATCHED && mode != HUB_STEP_GRAPH && mode != HUB_STEP_PERSITE) return HUB_EINVAL;
    // the step needs the projection workspace and the N-bar buffer (with the
    // current: the moment projections and, on first use, the grouped moment
    // tables); size them before any capture so that the graph never sees a
    // reallocation
    const int ncol = c->ncol(io->nstates);
    size_t part = part_need(c, ncol, c->T.spindep ? 2 : 1);
    if (jcur) {
        const bool fused = mode != HUB_STEP_PERSITE && fused_moments(c);
        part = std::max(part, fused ? part_need_moments(c, ncol) : part_need(c, ncol, 3));
        st = ensure(&c->d_grad, &c->grad_cap, static_cast<size_t>(c->nsets()) * c->T.J * 3 * ncol * c->ncplx(), c);
        if (st) return st;
        if (fused) {
            size_t bytes = 0;
            if (!c->d_gfdel) HUB_TRY(upload(c, &c->d_gfdel, c->T.grouped.fdel, bytes));
            if (!c->d_gd0) HUB_TRY(upload(c, &c->d_gd0, c->T.grouped.d0, bytes));
            c->table_bytes += bytes;
        }
    }
    st = ensure(&c->d_part, &c->part_cap, part, c);
    if (st) return st;

    if (!io->nbar) {
        st = ensure(&c->d_nbar_ws, &c->nbar_cap, static_cast<size_t>(c->nsets()) * c->T.nspecies * io->nstates, c);
        if (st) return st;
    }
    st = ensure(&c->d_sink, &c->sink_cap, static_cast<size_t>(io->ldh) * c->ncplx(), c);
    if (st) return st;
    st = ensure(&c->d_occ_ws, &c->occ_cap, occ_need(c, io->nstates), c);
    if (st) return st;
    if (mode != HUB_STEP_GRAPH) return run_step(c, io, mode == HUB_STEP_PERSITE, jcur);

    hub_ctx::GraphSlot* slot = nullptr;
    for (auto& g : c->gslot)
        if (g.key.valid && g.key.ncol == ncol && g.key.jcur == jcur &&
            std::memcmp(&g.key.io, io, sizeof(hub_step_io)) == 0)
            slot = &g;
    if (!slot) {
        slot = &c->gslot[0];
        for (auto& g : c->gslot)
            if (!g.key.valid || g.used < slot->used) slot = &g;
        drop_slot(*slot);
        HUB_TRY(hipStreamSynchronize(c->stream));
        hipStream_t keep = c->stream;
        c->stream = c->cap_stream;
        HUB_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        c->capturing = true;
        st = run_step(c, io, false, jcur);
        c->capturing = false;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        c->stream = keep;
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return map_err(e);
        slot->graph = g;
        e = hipGraphInstantiate(&slot->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_slot(*slot);
            return map_err(e);
        }
        slot->key.io = *io;
        slot->key.ncol = ncol;
        slot->key.jcur = jcur;
        slot->key.valid = true;
        ++c->ncapture;
    }
    slot->used = ++c->gclock;
    HUB_TRY(hipGraphLaunch(slot->gexec, c->stream));
    return HUB_OK;
}


}  // namespace

// =====================================================================  ABI

extern "C" {

const char* hub_strerror(int code) {
    switch (code) {
    case HUB_OK: return "ok";
    case HUB_EINVAL: return "invalid argument";
    case HUB_ENOMEM: return "out of memory";
    case HUB_EDEVICE: return "HIP device error";
    case HUB_ESTATE: return "call not valid in the current context state";
    case HUB_WDEGENERATE: return "degenerate U/J denominator";
    case HUB_ENONFINITE: return "occupations, U or J not finite";
    case HUB_ESCRATCH: return "workspace larger than the static scratch buffer";
    default: return "unknown status";
    }
}

int hub_create(hub_ctx** out, const double cell[3], const int ngrid[3], int spin_mode, int is_complex,
               int precision) {
    if (!out || !cell || !ngrid) return HUB_EINVAL;
    *out = nullptr;
    for (int i = 0; i < 3; ++i)
        if (!(cell[i] > 0.0) || !std::isfinite(cell[i]) || ngrid[i] < 1) return HUB_EINVAL;
    if (spin_mode != HUB_UNPOLARIZED && spin_mode != HUB_COLLINEAR && spin_mode != HUB_SPINOR) return HUB_EINVAL;
    if (is_complex != 0 && is_complex != 1) return HUB_EINVAL;
    if (spin_mode == HUB_SPINOR && !is_complex) return HUB_EINVAL;
    if (precision != HUB_F64 && precision != HUB_F32) return HUB_EINVAL;
    if (static_cast<int64_t>(ngrid[0]) * ngrid[1] * ngrid[2] > INT32_MAX) return HUB_EINVAL;
    hub_ctx* c = new (std::nothrow) hub_ctx();
    if (!c) return HUB_ENOMEM;
    for (int i = 0; i < 3; ++i) {
        c->cell[i] = cell[i];
        c->ngrid[i] = ngrid[i];
    }
    c->spin_mode = spin_mode;
    c->is_complex = is_complex;
    c->precision = precision;
    if (const char* fa = std::getenv("HUB_FAIL_ALLOC")) c->fail_alloc = std::max(0LL, std::atoll(fa));
    *out = c;
    return HUB_OK;
}

int hub_set_kpoints(hub_ctx* c, int nk, const double* k_red, const double* w) {
    if (!c || nk < 1 || !k_red || !w) return HUB_EINVAL;
    if (c->built_host) return HUB_ESTATE;
    for (int i = 0; i < 3 * nk; ++i) {
        if (!std::isfinite(k_red[i])) return HUB_EINVAL;
        if (!c->is_complex && k_red[i] != 0.0) return HUB_EINVAL;
    }
    for (int i = 0; i < nk; ++i)
        if (!std::isfinite(w[i])) return HUB_EINVAL;
    c->nk = nk;
    c->kred.assign(k_red, k_red + 3 * nk);
    c->kw.assign(w, w + nk);
    return HUB_OK;
}

int hub_add_site(hub_ctx* c, const double R[3], int l, double zeta, double rc, int species, int* site_id) {
    if (!c || !R) return HUB_EINVAL;
    if (c->built_host) return HUB_ESTATE;
    if (l < 0 || l > 3 || !(zeta > 0.0) || !(rc > 0.0) || !std::isfinite(zeta) || !std::isfinite(rc)) return HUB_EINVAL;
    if (species < 0 || species >= HUB_MAX_SPECIES) return HUB_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(R[i])) return HUB_EINVAL;
    SiteDef s;
    for (int i = 0; i < 3; ++i) s.R[i] = R[i];
    s.l = l;
    s.zeta = zeta;
    s.rc = rc;
    s.species = species;
    s.ueff_fixed = std::nan("");
    s.zeta_dn = std::nan("");
    c->sites.push_back(s);
    if (site_id) *site_id = static_cast<int>(c->sites.size()) - 1;
    return HUB_OK;
}

int hub_set_site_spin_orbital(hub_ctx* c, int site, double zeta_dn) {
    if (!c || site < 0 || site >= static_cast<int>(c->sites.size())) return HUB_EINVAL;
    if (c->built_host) return HUB_ESTATE;
    if (c->spin_mode != HUB_SPINOR || !(zeta_dn > 0.0) || !std::isfinite(zeta_dn)) return HUB_EINVAL;
    c->sites[site].zeta_dn = zeta_dn;
    return HUB_OK;
}

int hub_set_fixed_ueff(hub_ctx* c, int site, double ueff) {
    if (!c || site < 0 || site >= static_cast<int>(c->sites.size())) return HUB_EINVAL;
    if (std::isinf(ueff)) return HUB_EINVAL;
    c->sites[site].ueff_fixed = ueff;
    if (c->built_dev) {
        hipError_t e = hipMemcpyAsync(c->d_ueff_fixed + site, &c->sites[site].ueff_fixed, sizeof(double),
                                      hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        drop_graph(c);
        return map_err(e);
    }
    return HUB_OK;
}

int hub_set_chunk(hub_ctx* c, int chunk_entries) {
    if (!c || chunk_entries < 64 || chunk_entries > 65536) return HUB_EINVAL;
    if (c->built_host) return HUB_ESTATE;
    c->chunk_entries = chunk_entries;
    return HUB_OK;
}

int hub_set_worklist(hub_ctx* c, int grouped_list) {
    if (!c || (grouped_list != 0 && grouped_list != 1)) return HUB_EINVAL;
    c->use_grouped = grouped_list == 1;
    drop_graph(c);
    return HUB_OK;
}

int hub_set_class_launch(hub_ctx* c, int policy) {
    if (!c || policy < HUB_CLASSES_MERGED || policy > HUB_CLASSES_CONCURRENT) return HUB_EINVAL;
    if (c->class_policy != policy) drop_graph(c);
    c->class_policy = policy;
    return HUB_OK;
}

int hub_set_tuning(hub_ctx* c, int which, int cpl, int waves, int layout) {
    if (!c || (which != 0 && which != 1)) return HUB_EINVAL;
    if (cpl != 0 && cpl != 1 && cpl != 2 && cpl != 4) return HUB_EINVAL;
    if (waves != 1 && waves != 2 && waves != 4) return HUB_EINVAL;
    if (layout < -1 || layout > 1) return HUB_EINVAL;
    c->tune_cpl[which] = cpl;
    c->tune_waves[which] = waves;
    c->tune_layout[which] = layout;
    drop_graph(c);
    return HUB_OK;
}

int hub_finalize_host(hub_ctx* c) {
    if (!c) return HUB_EINVAL;
    if (c->built_host) return HUB_OK;
    if (c->sites.empty()) return HUB_EINVAL;
    int st;
    try {
        st = hub_build_host(c->cell, c->ngrid, c->sites, c->chunk_entries, c->T);
    } catch (const std::bad_alloc&) {
        return HUB_ENOMEM;
    } catch (...) {
        return HUB_EINVAL;
    }
    if (st) return st;
    c->have_tensor.assign(c->sites.size(), 0);
    c->built_host = true;
    return HUB_OK;
}

namespace {
int gauge_tables(hub_ctx* c);
}  // namespace

int hub_finalize(hub_ctx* c, void* stream) {
    if (!c) return HUB_EINVAL;
    int st = hub_finalize_host(c);
    if (st) return st;
    if (c->built_dev) return HUB_OK;
    HUB_TRY(hipGetDevice(&c->device));
    HUB_TRY(scratch_address(c->device));
    c->stream = reinterpret_cast<hipStream_t>(stream);
    const HostTables& T = c->T;
    std::vector<int32_t> all(T.chunks.size());
    for (size_t i = 0; i < all.size(); ++i) all[i] = static_cast<int32_t>(i);
    const int nimg = static_cast<int>(T.images.size() / 3);
    std::vector<double> phase(static_cast<size_t>(c->nk) * nimg * 2);
    for (int k = 0; k < c->nk; ++k)
        for (int i = 0; i < nimg; ++i) {
            const double t = c->kred[3 * k] * T.images[3 * i] + c->kred[3 * k + 1] * T.images[3 * i + 1] +
                             c->kred[3 * k + 2] * T.images[3 * i + 2];
            phase[(static_cast<size_t>(k) * nimg + i) * 2] = std::cos(kTwoPi * t);
            phase[(static_cast<size_t>(k) * nimg + i) * 2 + 1] = std::sin(kTwoPi * t);
        }
    std::vector<double> fixed(c->sites.size());
    for (size_t s = 0; s < fixed.size(); ++s) fixed[s] = c->sites[s].ueff_fixed;
    size_t& b = c->table_bytes;
    b = 0;
    hipError_t e = hipSuccess;
    auto up = [&](auto** dst, const auto& src) {
        if (e == hipSuccess) e = upload(c, dst, src, b);
    };
    up(&c->d_chunks, T.chunks);
    up(&c->d_all, all);
    up(&c->d_gidx, T.gidx);
    up(&c->d_img, T.img);
    up(&c->d_phi, T.phi);
    up(&c->d_gphi, T.gphi);
    if (T.spindep) {
        up(&c->d_phi2, T.phi2);
        up(&c->d_gphi_dn, T.gphi_dn);
        up(&c->d_mphi_dn, T.mphi_dn);
    }
    up(&c->d_mphi, T.mphi);
    up(&c->d_images, T.images);
    up(&c->d_kred, c->kred);
    up(&c->d_phase, phase);
    up(&c->d_site_chunk_ptr, T.site_chunk_ptr);
    up(&c->d_site_chunk_ids, T.site_chunk_ids);
    up(&c->d_orb_site, T.orb_site);
    up(&c->d_site_L, T.site_L);
    up(&c->d_site_orb0, T.site_orb0);
    up(&c->d_site_species, T.site_species);
    up(&c->d_species_orb_ptr, T.species_orb_ptr);
    up(&c->d_species_orb_ids, T.species_orb_ids);
    up(&c->d_kw, c->kw);
    up(&c->d_ueff_fixed, fixed);
    if (T.grouped.ok) {
        // launch order: chunks sorted by function-count class
        std::vector<int32_t> gall;
        gall.reserve(T.grouped.chunks.size());
        c->gcls_ptr[0] = 0;
        for (int k = 1; k <= HUB_NCLASS; ++k) {
            for (size_t i = 0; i < T.grouped.chunks.size(); ++i)
                if (hub_nf_class(T.grouped.chunks[i].L) == k) gall.push_back(static_cast<int32_t>(i));
            c->gcls_ptr[k] = static_cast<int>(gall.size());
        }
        up(&c->d_gchunks, T.grouped.chunks);
        up(&c->d_gall, gall);
        // merged launch, pass by pass: chunks with more functions (fewer
        // entries per batch, longer entry loops) and more entries first
        std::vector<int32_t> gm(gall);
        std::stable_sort(gm.begin(), gm.end(), [&T](int32_t x, int32_t y) {
            const HubChunk &X = T.grouped.chunks[x], &Y = T.grouped.chunks[y];
            if (X.layer != Y.layer) return X.layer < Y.layer;
            const int kx = hub_nf_class(X.L) > 2, ky = hub_nf_class(Y.L) > 2;
            return kx != ky ? kx > ky : X.ne > Y.ne;
        });
        c->gpass_ptr.assign(T.grouped.npass + 1, 0);
        for (int32_t i : gm) ++c->gpass_ptr[T.grouped.chunks[i].layer + 1];
        for (int p = 0; p < T.grouped.npass; ++p) c->gpass_ptr[p + 1] += c->gpass_ptr[p];
        up(&c->d_gall_m, gm);
        // moment projection: one item per half of a chunk's functions, the
        // costliest (entries times the FP64 instructions per entry) first
        std::vector<int32_t> items;
        std::vector<int64_t> cost;
        for (int32_t i : gm) {
            const HubChunk& C = T.grouped.chunks[i];
            for (int h = 0; h * HUB_MOM_NFW < C.L; ++h) {
                const int nfw = std::min(HUB_MOM_NFW, C.L - h * HUB_MOM_NFW);
                items.push_back(2 * i + h);
                cost.push_back(static_cast<int64_t>(C.ne) * (8 * nfw + 12));
            }
        }
        std::vector<int32_t> order(items.size());
        for (size_t x = 0; x < order.size(); ++x) order[x] = static_cast<int32_t>(x);
        std::stable_sort(order.begin(), order.end(), [&cost](int32_t x, int32_t y) { return cost[x] > cost[y]; });
        std::vector<int32_t> mom(items.size());
        for (size_t x = 0; x < order.size(); ++x) mom[x] = items[order[x]];
        c->nmom = static_cast<int>(mom.size());
        up(&c->d_gmom, mom);
        up(&c->d_ggidx, T.grouped.gidx);
        up(&c->d_gtab, T.grouped.tab);
        up(&c->d_gf_orb, T.grouped.f_orb);
        up(&c->d_gf_img, T.grouped.f_img);
        up(&c->d_gred_ptr, T.grouped.red_ptr);
        up(&c->d_gred_row, T.grouped.red_row);
        up(&c->d_gred_img, T.grouped.red_img);
        if (T.spindep) {
            std::vector<int32_t> shift(T.J);
            for (int s = 0; s < T.nsites; ++s)
                for (int m = 0; m < T.site_L[s]; ++m) shift[T.site_orb0[s] + m] = T.site_L[s];
            up(&c->d_gspin_shift, shift);
        }
    }
    if (e == hipSuccess) {
        e = dev_malloc(c, &c->d_tensor, c->sites.size() * 2401 * sizeof(double));
        b += c->sites.size() * 2401 * sizeof(double);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    for (int k = 0; k < HUB_NCLASS && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join_ev[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        release(c);
        return map_err(e);
    }
    c->phase_host = phase;
    c->built_dev = true;
    if (c->gauge) return gauge_tables(c);
    return HUB_OK;
}

int hub_set_stream(hub_ctx* c, void* stream) {
    if (!c) return HUB_EINVAL;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    return HUB_OK;
}

int hub_query(const hub_ctx* c, int what, int64_t* v) {
    if (!c || !v) return HUB_EINVAL;
    if (!c->built_host) return HUB_ESTATE;
    const HostTables& T = c->T;
    switch (what) {
    case 0: *v = T.nsites; break;
    case 1: *v = T.J; break;
    case 2: *v = c->nsets(); break;
    case 3: *v = T.nlayers; break;
    case 4: *v = T.nentries; break;
    case 5: *v = static_cast<int64_t>(T.chunks.size()); break;
    case 6: *v = T.nspecies; break;
    case 7: *v = c->nk; break;
    case 8: *v = c->nblk(); break;
    case 9: *v = static_cast<int64_t>(c->table_bytes); break;
    case 10: *v = T.part_rows; break;
    case 11: *v = T.grouped.ok ? static_cast<int64_t>(T.grouped.chunks.size()) : 0; break;
    case 12: *v = T.grouped.nfmax; break;
    case 13: *v = c->stencil_entries; break;
    case 14: *v = T.grouped.ok ? T.grouped.npass : 0; break;
    case 15: *v = c->nalloc; break;
    case 16: *v = c->ncapture; break;
    default: return HUB_EINVAL;
    }
    return HUB_OK;
}

int hub_site_info(const hub_ctx* c, int site, int* L, int* orb_offset, int64_t* npoints, int* species) {
    if (!c) return HUB_EINVAL;
    if (!c->built_host) return HUB_ESTATE;
    if (site < 0 || site >= c->T.nsites) return HUB_EINVAL;
    if (L) *L = c->T.site_L[site];
    if (orb_offset) *orb_offset = c->T.site_orb0[site];
    if (npoints) *npoints = static_cast<int64_t>(c->T.spheres[site].g.size());
    if (species) *species = c->T.site_species[site];
    return HUB_OK;
}

int hub_site_points(const hub_ctx* c, int site, int32_t* g, int32_t* image3, double* phi, double* grad) {
    if (!c) return HUB_EINVAL;
    if (!c->built_host) return HUB_ESTATE;
    if (site < 0 || site >= c->T.nsites) return HUB_EINVAL;
    const SiteSphere& s = c->T.spheres[site];
    if (g) std::memcpy(g, s.g.data(), s.g.size() * sizeof(int32_t));
    if (image3) std::memcpy(image3, s.img3.data(), s.img3.size() * sizeof(int32_t));
    if (phi) std::memcpy(phi, s.phi.data(), s.phi.size() * sizeof(double));
    if (grad) std::memcpy(grad, s.grad.data(), s.grad.size() * sizeof(double));
    return HUB_OK;
}

int hub_project(hub_ctx* c, const void* psi, int64_t ld, int nstates, double* cout) {
    if (!c || !cout) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (!valid_states(c, psi, ld, nstates)) return HUB_EINVAL;
    return do_project(c, psi, ld, nstates, cout, false);
}

int hub_project_sets(hub_ctx* c, const void* psi, int64_t ld, int nstates, int set0, int nsets, double* cout) {
    if (!c || !cout) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (!valid_states(c, psi, ld, nstates)) return HUB_EINVAL;
    if (set0 < 0 || nsets < 1 || set0 + nsets > c->nsets()) return HUB_EINVAL;
    return do_project(c, psi, ld, nstates, cout, false, TAB_PHI, set0, nsets);
}

int hub_occupations(hub_ctx* c, const double* cc, int nstates, const double* f, double* n, double* pbar,
                    double* nbar) {
    if (!c || !cc || !f || !n || nstates < 1) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    return do_occupations(c, cc, nstates, f, n, pbar, nbar, false);
}

int hub_coulomb(hub_ctx* c, int site, double* tensor) {
    if (!c) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    const int ns = c->T.nsites;
    if (site < -1 || site >= ns) return HUB_EINVAL;
    if (site == -1 && tensor) return HUB_EINVAL;
    // sites with spin-dependent orbitals take a fixed U_eff (no ACBN0 tensor)
    if (site >= 0 && std::isfinite(c->sites[site].zeta_dn)) return HUB_EINVAL;
    const int s0 = site < 0 ? 0 : site, s1 = site < 0 ? ns : site + 1;
    size_t maxp = 1;
    for (int s = s0; s < s1; ++s) maxp = std::max(maxp, c->T.spheres[s].g.size());
    int32_t* d_ijk = nullptr;
    double *d_phi = nullptr, *d_rho = nullptr, *d_W = nullptr;
    hipError_t e = dev_malloc(c, &d_ijk, maxp * 3 * sizeof(int32_t));
    if (e == hipSuccess) e = dev_malloc(c, &d_phi, maxp * 7 * sizeof(double));
    if (e == hipSuccess) e = dev_malloc(c, &d_rho, maxp * 28 * sizeof(double));
    if (e == hipSuccess) e = dev_malloc(c, &d_W, maxp * 28 * sizeof(double));
    double h[3];
    for (int i = 0; i < 3; ++i) h[i] = c->cell[i] / c->ngrid[i];
    const double g0 = hub_g0_cell_average(h);
    for (int s = s0; s < s1 && e == hipSuccess; ++s) {
        if (std::isfinite(c->sites[s].zeta_dn)) continue;
        const SiteSphere& sp = c->T.spheres[s];
        const int L = c->T.site_L[s];
        e = hipMemcpyAsync(d_ijk, sp.ijk.data(), sp.ijk.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_phi, sp.phi.data(), sp.phi.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) break;
        CoulombArgs a{};
        a.ijk = d_ijk;
        a.phi = d_phi;
        a.P = static_cast<int>(sp.g.size());
        a.L = L;
        a.npair = L * (L + 1) / 2;
        a.rho = d_rho;
        a.W = d_W;
        a.tensor = c->d_tensor + static_cast<size_t>(s) * 2401;
        for (int i = 0; i < 3; ++i) a.h[i] = h[i];
        a.g0 = g0;
        a.dV = h[0] * h[1] * h[2];
        e = launch_coulomb(a, c->stream);
        if (e == hipSuccess && tensor)
            e = hipMemcpyAsync(tensor, a.tensor, static_cast<size_t>(L) * L * L * L * sizeof(double),
                               hipMemcpyDeviceToDevice, c->stream);
        // host arrays are reused next iteration: wait for the copies
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) c->have_tensor[s] = 1;
    }
    if (d_ijk) (void)hipFree(d_ijk);
    if (d_phi) (void)hipFree(d_phi);
    if (d_rho) (void)hipFree(d_rho);
    if (d_W) (void)hipFree(d_W);
    return map_err(e);
}

int hub_get_coulomb(hub_ctx* c, int site, double* tensor) {
    if (!c || !tensor) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (site < 0 || site >= c->T.nsites) return HUB_EINVAL;
    if (!c->have_tensor[site]) return HUB_ESTATE;
    const int L = c->T.site_L[site];
    HUB_TRY(hipMemcpyAsync(tensor, c->d_tensor + static_cast<size_t>(site) * 2401,
                           static_cast<size_t>(L) * L * L * L * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return HUB_OK;
}

int hub_set_coulomb(hub_ctx* c, int site, const double* tensor) {
    if (!c || !tensor) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (site < 0 || site >= c->T.nsites) return HUB_EINVAL;
    if (std::isfinite(c->sites[site].zeta_dn)) return HUB_EINVAL;
    const int L = c->T.site_L[site];
    HUB_TRY(hipMemcpyAsync(c->d_tensor + static_cast<size_t>(site) * 2401, tensor,
                           static_cast<size_t>(L) * L * L * L * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    c->have_tensor[site] = 1;
    return HUB_OK;
}

int hub_acbn0_uj(hub_ctx* c, const double* n, const double* pbar, double* U, double* J, double* Ueff,
                 int* status) {
    if (!c || !n || !pbar || !U || !J || !Ueff) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (need_tensors(c)) return HUB_ESTATE;
    return do_acbn0(c, n, pbar, U, J, Ueff, reinterpret_cast<int32_t*>(status), false);
}

int hub_apply(hub_ctx* c, const double* Ueff, const double* n, const double* cc, int nstates,
              const double* colscale, double alpha, void* hpsi, int64_t ld) {
    if (!c || !Ueff || !n || !cc) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (!valid_states(c, hpsi, ld, nstates) || !std::isfinite(alpha)) return HUB_EINVAL;
    return do_apply(c, Ueff, n, cc, nstates, colscale, alpha, hpsi, ld, false);
}

int hub_apply_sets(hub_ctx* c, const double* Ueff, const double* n, const double* cc, int nstates,
                   const double* colscale, double alpha, void* hpsi, int64_t ld, int set0, int nsets) {
    if (!c || !Ueff || !n || !cc) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (!valid_states(c, hpsi, ld, nstates) || !std::isfinite(alpha)) return HUB_EINVAL;
    if (set0 < 0 || nsets < 1 || set0 + nsets > c->nsets()) return HUB_EINVAL;
    return do_apply(c, Ueff, n, cc, nstates, colscale, alpha, hpsi, ld, false, set0, nsets);
}

int hub_energy(hub_ctx* c, const double* Ueff, const double* n, double* EU) {
    if (!c || !Ueff || !n || !EU) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    EnergyArgs a{};
    a.n = n;
    a.Ueff = Ueff;
    a.EU = EU;
    a.site_L = c->d_site_L;
    a.nsites = c->T.nsites;
    a.nblk = c->nblk();
    HUB_TRY(launch_energy(a, c->stream));
    return HUB_OK;
}

int hub_energy_fll(hub_ctx* c, const double* U, const double* J, const double* n, double* out) {
    if (!c || !U || !J || !n || !out) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    FllArgs a{};
    a.n = n;
    a.U = U;
    a.J = J;
    a.out = out;
    a.site_L = c->d_site_L;
    a.nsites = c->T.nsites;
    a.nblk = c->nblk();
    HUB_TRY(launch_fll(a, c->stream));
    return HUB_OK;
}

namespace {

// Forces (table TAB_GRAD, real part) or velocity-gauge current (TAB_MOMENT,
// imaginary part): out[site][i] = 2 g sum w f Re/Im sum_a conj(d_{a,i}) B_a,
// with d the projections of the psi on the table's 3L functions per site.
// fscale multiplies the result (1: forces or current; -g: g dE_U/dR).
int contract_moments(hub_ctx* c, const void* psi, int64_t ld, int nstates, const double* cc, const double* f,
                     const double* Ueff, const double* n, double* out, int table, double fscale) {
    if (!c || !cc || !f || !Ueff || !n || !out) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (!valid_states(c, psi, ld, nstates)) return HUB_EINVAL;
    const int ncol = c->ncol(nstates);
    const size_t need = static_cast<size_t>(c->nsets()) * c->T.J * 3 * ncol * c->ncplx();
    int st = ensure(&c->d_grad, &c->grad_cap, need, c);
    if (st) return st;
    if (c->T.spindep) {
        // spin-dependent orbitals: the spin-up tables give the even columns,
        // the spin-down tables the odd ones
        const int dn = table == TAB_GRAD ? TAB_GRAD_DN : (table == TAB_MOMENT ? TAB_MOMENT_DN : TAB_STENCIL_DN);
        st = do_project(c, psi, ld, nstates, c->d_grad, false, table, 0, -1, 0);
        if (!st) st = do_project(c, psi, ld, nstates, c->d_grad, false, dn, 0, -1, 1);
    } else {
        st = do_project(c, psi, ld, nstates, c->d_grad, false, table);
    }
    if (st) return st;
    return moment_contraction(c, cc, f, Ueff, n, c->d_grad, nstates, out, table == TAB_MOMENT, fscale);
}

// out[site][i] = fscale 2 g sum w f Re (imag: Im) sum_a conj(d_{a,i}) B_a
// from the moment projections d[q][3 j + i][col] (k_forces).
int moment_contraction(hub_ctx* c, const double* cc, const double* f, const double* Ueff, const double* n,
                       const double* d, int nstates, double* out, bool imag, double fscale) {
    const int ncol = c->ncol(nstates);
    ForceArgs a{};
    a.c = cc;
    a.d = d;
    a.f = f;
    a.n = n;
    a.ueff = Ueff;
    a.kweights = c->d_kw;
    a.F = out;
    a.site_L = c->d_site_L;
    a.site_orb0 = c->d_site_orb0;
    a.nsites = c->T.nsites;
    a.J = c->T.J;
    a.ncol = ncol;
    a.nstates = nstates;
    a.ncplx = c->ncplx();
    a.spinor = c->spin_mode == HUB_SPINOR;
    a.nspin = c->nspin();
    a.nq = c->nsets();
    a.nblk = c->nblk();
    a.imag = imag ? 1 : 0;
    a.scale = fscale;
    StageTimer tm(c, HUB_STAGE_FORCES);
    HUB_TRY(launch_forces(a, c->stream));
    return HUB_OK;
}

// Gauge tables on the device: with a field, the image phases at k + A and
// the grid-point phases; without one, the plain image phases again.
int gauge_tables(hub_ctx* c) {
    if (!c->gauge) {
        HUB_TRY(hipMemcpyAsync(c->d_phase, c->phase_host.data(), c->phase_host.size() * sizeof(double),
                               hipMemcpyHostToDevice, c->stream));
        return HUB_OK;
    }
    if (!c->d_pg) HUB_TRY(dev_malloc(c, &c->d_pg, static_cast<size_t>(c->G()) * 2 * sizeof(double)));
    GaugeArgs g{};
    for (int i = 0; i < 3; ++i) {
        g.A[i] = c->A[i];
        g.cell[i] = c->cell[i];
        g.h[i] = c->cell[i] / c->ngrid[i];
        g.ngrid[i] = c->ngrid[i];
    }
    g.images = c->d_images;
    g.nimg = static_cast<int>(c->T.images.size() / 3);
    g.kred = c->d_kred;
    g.nk = c->nk;
    g.phase = c->d_phase;
    g.pg = c->d_pg;
    HUB_TRY(launch_gauge_tables(g, c->stream));
    return HUB_OK;
}

// Dilated-sphere work list of the state-gradient force form, built on the
// host and uploaded at the first call that needs it.
int build_stencil(hub_ctx* c) {
    StencilTables S;
    const int st = hub_build_stencil(c->cell, c->ngrid, c->sites, c->T, c->chunk_entries, S);
    if (st) return st;
    std::vector<int32_t> all(S.chunks.size());
    std::iota(all.begin(), all.end(), 0);
    // a failed earlier attempt may have left some of the tables allocated
    for (void** p : {reinterpret_cast<void**>(&c->d_st_chunks), reinterpret_cast<void**>(&c->d_st_all),
                     reinterpret_cast<void**>(&c->d_st_gidx), reinterpret_cast<void**>(&c->d_st_tab),
                     reinterpret_cast<void**>(&c->d_st_site_ptr), reinterpret_cast<void**>(&c->d_st_site_ids),
                     reinterpret_cast<void**>(&c->d_st_tab_dn)}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    size_t bytes = 0;
    HUB_TRY(upload(c, &c->d_st_chunks, S.chunks, bytes));
    HUB_TRY(upload(c, &c->d_st_all, all, bytes));
    HUB_TRY(upload(c, &c->d_st_gidx, S.gidx, bytes));
    HUB_TRY(upload(c, &c->d_st_tab, S.tab, bytes));
    HUB_TRY(upload(c, &c->d_st_site_ptr, S.site_chunk_ptr, bytes));
    HUB_TRY(upload(c, &c->d_st_site_ids, S.site_chunk_ids, bytes));
    if (c->T.spindep) HUB_TRY(upload(c, &c->d_st_tab_dn, S.tab_dn, bytes));
    c->table_bytes += bytes;
    c->stencil_nchunks = static_cast<int>(S.chunks.size());
    c->stencil_part_rows = S.part_rows;
    c->stencil_entries = S.nentries;
    c->stencil_built = true;
    return HUB_OK;
}

}  // namespace

int hub_forces(hub_ctx* c, const void* psi, int64_t ld, int nstates, const double* cc, const double* f,
               const double* Ueff, const double* n, double* F) {
    return contract_moments(c, psi, ld, nstates, cc, f, Ueff, n, F, TAB_GRAD);
}

int hub_forces_state_gradient(hub_ctx* c, const void* psi, int64_t ld, int nstates, const double* cc,
                              const double* f, const double* Ueff, const double* n, double* F) {
    if (!c) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (!c->stencil_built) {
        const int st = build_stencil(c);
        if (st) return st;
    }
    return contract_moments(c, psi, ld, nstates, cc, f, Ueff, n, F, TAB_STENCIL);
}

int hub_current(hub_ctx* c, const void* psi, int64_t ld, int nstates, const double* cc, const double* f,
                const double* Ueff, const double* n, double* J) {
    return contract_moments(c, psi, ld, nstates, cc, f, Ueff, n, J, TAB_MOMENT);
}

int hub_energy_gradient(hub_ctx* c, const void* psi, int64_t ld, int nstates, const double* cc, const double* f,
                        const double* Ueff, const double* n, double scale, void* grad_psi, int64_t ldg,
                        double* grad_R) {
    if (!c || !cc || !f || !Ueff || !n || !std::isfinite(scale)) return HUB_EINVAL;
    if (!built(c)) return HUB_ESTATE;
    if (!grad_psi && !grad_R) return HUB_EINVAL;
    if (grad_psi && !valid_states(c, grad_psi, ldg, nstates)) return HUB_EINVAL;
    if (grad_R && !valid_states(c, psi, ld, nstates)) return HUB_EINVAL;
    if (grad_psi) {
        // every used column of every row starts at zero (the apply writes
        // sphere points only), then grad += scale 2 g_s dV w_k f V_U psi
        const int ncol = c->ncol(nstates);
        HUB_TRY(launch_zero_cols(grad_psi, static_cast<int>(c->elem() / c->ncplx()),
                                 static_cast<int64_t>(c->nsets()) * c->G(), ldg * c->ncplx(), ncol * c->ncplx(),
                                 c->stream));
        const double gs = c->spin_mode == HUB_UNPOLARIZED ? 2.0 : 1.0;
        const double dV = (c->cell[0] / c->ngrid[0]) * (c->cell[1] / c->ngrid[1]) * (c->cell[2] / c->ngrid[2]);
        const int st = do_apply(c, Ueff, n, cc, nstates, nullptr, scale * 2.0 * gs * dV, grad_psi, ldg, false, 0, -1,
                                f);
        if (st) return st;
    }
    if (grad_R) return contract_moments(c, psi, ld, nstates, cc, f, Ueff, n, grad_R, TAB_GRAD, -scale);
    return HUB_OK;
}

int hub_step_noalloc(hub_ctx* c, const hub_step_io* io) {
    int st = check_step(c, io);
    if (st) return st;
    void* base = scratch_ptr(c->device);
    if (!base) return HUB_ESTATE;
    // slices of the scratch array: projection partial sums, occupation
    // partial sums, N-bar (when the caller passes none), the apply's sink row
    const int ncol = c->ncol(io->nstates);
    const size_t n_part = slice256(part_need(c, ncol, c->T.spindep ? 2 : 1));
    const size_t n_occ = slice256(occ_need(c, io->nstates));
    const size_t n_nbar = io->nbar ? 0 : slice256(static_cast<size_t>(c->nsets()) * c->T.nspecies * io->nstates);
    const size_t n_sink = slice256(static_cast<size_t>(io->ldh) * c->ncplx());
    if ((n_part + n_occ + n_nbar + n_sink) * sizeof(double) > HUB_SCRATCH_BYTES) return HUB_ESCRATCH;
    double* p = static_cast<double*>(base);
    const hub_ctx::FixedWs ws{p, p + n_part, p + n_part + n_occ, p + n_part + n_occ + n_nbar};
    c->ws_fixed = &ws;
    st = run_step(c, io, false);
    c->ws_fixed = nullptr;
    return st;
}

int hub_set_vector_potential(hub_ctx* c, const double* A) {
    if (!c) return HUB_EINVAL;
    if (A) {
        // the kernels address the grid-point phase table with 32-bit byte
        // offsets (16 bytes per point)
        if (!c->is_complex || c->G() > static_cast<int64_t>(UINT32_MAX / 16)) return HUB_EINVAL;
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(A[i])) return HUB_EINVAL;
    }
    const bool on = A != nullptr;
    if (on != c->gauge) drop_graph(c);
    c->gauge = on;
    for (int i = 0; i < 3; ++i) c->A[i] = on ? A[i] : 0.0;
    if (!c->built_dev) return HUB_OK;
    return gauge_tables(c);
}

int hub_step(hub_ctx* c, const hub_step_io* io, int mode) { return step_impl(c, io, mode, nullptr); }

int hub_step_current(hub_ctx* c, const hub_step_io* io, double* J, int mode) {
    if (!J) return HUB_EINVAL;
    return step_impl(c, io, mode, J);
}

int hub_profile(hub_ctx* c, int enable) {
    if (!c || (enable != 0 && enable != 1)) return HUB_EINVAL;
    c->prof = enable == 1;
    return HUB_OK;
}

int hub_profile_read(hub_ctx* c, double* ms, int64_t* counts) {
    if (!c) return HUB_EINVAL;
    if (!c->ev_pending.empty()) HUB_TRY(hipStreamSynchronize(c->stream));
    for (auto& p : c->ev_pending) {
        float t = 0.0f;
        HUB_TRY(hipEventElapsedTime(&t, p.second.first, p.second.second));
        c->prof_ms[p.first] += t;
        c->prof_n[p.first] += 1;
        c->ev_pool.push_back(p.second.first);
        c->ev_pool.push_back(p.second.second);
    }
    c->ev_pending.clear();
    for (int i = 0; i < HUB_NSTAGES; ++i) {
        if (ms) ms[i] = c->prof_ms[i];
        if (counts) counts[i] = c->prof_n[i];
        c->prof_ms[i] = 0.0;
        c->prof_n[i] = 0;
    }
    return HUB_OK;
}

int hub_destroy(hub_ctx* c) {
    if (!c) return HUB_EINVAL;
    if (c->built_dev) (void)hipStreamSynchronize(c->stream);
    for (auto& p : c->ev_pending) {
        c->ev_pool.push_back(p.second.first);
        c->ev_pool.push_back(p.second.second);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    release(c);
    delete c;
    return HUB_OK;
}

}  // extern "C"
