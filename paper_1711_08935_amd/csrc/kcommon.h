// Device-side helpers and launch argument blocks of the Hubbard kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hub_internal.h"

#define HUB_WAVE 64

// Launch arguments of the projection kernel (gather + contraction).
struct ProjArgs {
    const void* psi;          // states, T[nq][G][ld] (x2 for complex)
    int64_t ld;               // columns per grid point
    int64_t qstride;          // scalars between state sets (G * ld * ncplx)
    int ncol;                 // columns used (nstates or 2 nstates)
    int ncplx;                // 1 real, 2 complex
    int nq;                   // state sets
    const HubChunk* chunks;
    const int32_t* chunk_list;
    const int32_t* gidx;
    const double* tab;        // orbital table (or gradient table)
    int tabmult;              // 1: phi, 3: grad phi or position moments
    int wide;                 // 1: one state set per wave; 0: sets packed across lanes
    int nchunks;              // chunks in chunk_list (set by the launcher)
    int tiles;                // column tiles per chunk (set by the launcher)
    const double* pg;         // velocity gauge: [G] exp(i A.r_g) (re, im), or null
    double* part;             // [nq][prows][ncol] (x2 complex)
    int64_t prows;            // rows per state set = part_rows * tabmult
    // position-moment launch (k_project_mom) only: per grouped point the
    // displacement d0[3] from its chunk's first cover, per chunk and function
    // the offset fdel[HUB_GF_MAX][3] to its own cover; component i (0: the
    // orbitals, 1-3: the moments) is written to part + i * pplane
    const double* d0;
    const double* fdel;
    int64_t pplane;
};

// Launch arguments of the apply kernel (coefficients + scatter).
struct ApplyArgs {
    void* hpsi;
    int64_t ld;
    int64_t qstride;
    int ncol;
    int nstates;
    int nq;                   // state sets
    int nspin;
    int spinor;
    int nblk;                 // blocks per site in n
    const HubChunk* chunks;
    const int32_t* chunk_list;
    const int32_t* gidx;
    const double* tab;
    const double* phase;      // [nk][nimg] (re, im) of exp(+i k.T)
    int nimg;
    const double* c;          // [nq][J][ncol] (x2 complex)
    int J;
    const double* n;          // [site][nblk][7][7][2]
    const double* ueff;       // [site]
    const double* colscale;   // [nq][nstates] or null
    const double* occ;        // [context sets][nstates] occupations f, or null: then each column is
                              // also weighted by w_k f_s (energy gradient)
    const double* kw;         // [nk] k-point weights (with occ)
    double alpha;
    int wide;                 // 1: one state set per wave; 0: sets packed across lanes
    int nchunks;              // chunks in chunk_list (set by the launcher)
    int tiles;                // column tiles per chunk (set by the launcher)
    const double* pg;         // velocity gauge: [G] exp(i A.r_g) (re, im), or null
    int spindep;              // per-site chunks with 2L functions [sigma][m] (spinor orbitals)
    int q0;                   // context index of the first state set of the launch (k-point, spin)
    // grouped chunks: per chunk HUB_GF_MAX (orbital j, image) pairs
    const int32_t* f_orb;
    const int32_t* f_img;
    const int32_t* orb_site;
    const int32_t* site_orb0;
    const int32_t* site_L;
    // one row (ld x ncplx values) of scratch that the padding entries of a
    // chunk read and write instead of a state row; its contents are garbage
    void* sink;
};

template <typename T, int N>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&v)[N]) {
    if constexpr (sizeof(T) * N >= 16) {
        constexpr int per = 16 / sizeof(T);
        using V16 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
#pragma unroll
        for (int i = 0; i < N / per; ++i) {
            const V16 t = *reinterpret_cast<const V16*>(p + i * per);
            if constexpr (sizeof(T) == 4) {
                v[i * per + 0] = t.x; v[i * per + 1] = t.y; v[i * per + 2] = t.z; v[i * per + 3] = t.w;
            } else {
                v[i * per + 0] = t.x; v[i * per + 1] = t.y;
            }
        }
    } else if constexpr (sizeof(T) == 4 && N == 2) {
        const float2 t = *reinterpret_cast<const float2*>(p);
        v[0] = t.x; v[1] = t.y;
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = p[i];
    }
}

template <typename T, int N>
__device__ __forceinline__ void store_vec(T* __restrict__ p, const T (&v)[N]) {
    if constexpr (sizeof(T) * N >= 16) {
        constexpr int per = 16 / sizeof(T);
        using V16 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
#pragma unroll
        for (int i = 0; i < N / per; ++i) {
            V16 t;
            if constexpr (sizeof(T) == 4) {
                t.x = v[i * per + 0]; t.y = v[i * per + 1]; t.z = v[i * per + 2]; t.w = v[i * per + 3];
            } else {
                t.x = v[i * per + 0]; t.y = v[i * per + 1];
            }
            *reinterpret_cast<V16*>(p + i * per) = t;
        }
    } else if constexpr (sizeof(T) == 4 && N == 2) {
        float2 t;
        t.x = v[0]; t.y = v[1];
        *reinterpret_cast<float2*>(p) = t;
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) p[i] = v[i];
    }
}

// Row access of the entry loops.  The projection streams its state rows
// with non-temporal loads: each element is read once per step, and loads
// that do not allocate in the caches leave the chunk tables there and do
// not evict the apply's pending writes into the projection's time.  The
// apply reads and writes hpsi with ordinary accesses (non-temporal ones
// measured slower there).
typedef float hub_f2 __attribute__((ext_vector_type(2)));
typedef float hub_f4 __attribute__((ext_vector_type(4)));
typedef double hub_d2 __attribute__((ext_vector_type(2)));

template <typename T, int N>
__device__ __forceinline__ void load_row_stream(const T* __restrict__ p, T (&v)[N]) {
    if constexpr (sizeof(T) * N == 8 && sizeof(T) == 4) {
        const hub_f2 t = __builtin_nontemporal_load(reinterpret_cast<const hub_f2*>(p));
        v[0] = t[0];
        v[1] = t[1];
    } else if constexpr (sizeof(T) * N == 8) {
        v[0] = __builtin_nontemporal_load(p);
    } else if constexpr (sizeof(T) * N >= 16) {
        constexpr int per = 16 / sizeof(T);
        using V = typename std::conditional<sizeof(T) == 4, hub_f4, hub_d2>::type;
#pragma unroll
        for (int i = 0; i < N / per; ++i) {
            const V t = __builtin_nontemporal_load(reinterpret_cast<const V*>(p + i * per));
#pragma unroll
            for (int k = 0; k < per; ++k) v[i * per + k] = t[k];
        }
    } else {
        load_vec<T, N>(p, v);
    }
}

template <typename T, int N>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&v)[N]) {
    load_vec<T, N>(p, v);
}

template <typename T, int N>
__device__ __forceinline__ void store_row(T* __restrict__ p, const T (&v)[N]) {
    store_vec<T, N>(p, v);
}

// Rows per batch of the software-pipelined entry loops: the two batches of
// U rows of NV values per lane stay within 32 values, and the orbital values
// of one batch (U x NF doubles, uniform, held in scalar registers) within
// HUB_TAB_BUDGET.
#ifndef HUB_TAB_BUDGET
#define HUB_TAB_BUDGET 32
#endif
__host__ __device__ constexpr int hub_batch_rows(int nv, int nf) {
    int u = 8;
    while (u > 1 && (u * nv > 16 || u * nf > HUB_TAB_BUDGET)) u /= 2;
    return u;
}

// Function-count classes of the grouped work list: class k (1..HUB_NCLASS)
// holds the chunks with 4(k-1) < NF <= 4k and is launched on its own, so a
// kernel's registers follow the largest NF of its class.  Class 0 is the
// per-site work list (L in {1, 3, 5, 7}).
#define HUB_NCLASS 4
static_assert(HUB_GF_MAX == 4 * HUB_NCLASS, "the classes cover every grouped function count");
__host__ __device__ constexpr int hub_nf_class(int nf) { return (nf + 3) / 4; }
// Merged launches cover the chunks of every function count up to a bound:
// class HUB_NCLASS + m holds NF 1..4m; the kernels are built for m = 2 (a
// work list whose points carry at most 8 functions: registers sized for 8)
// and m = 4 (every grouped chunk).
#define HUB_MERGED8 (HUB_NCLASS + 2)
#define HUB_MERGED16 (HUB_NCLASS + 4)
// Waves per SIMD asked of the compiler for a merged kernel: the launches
// bounded at 8 functions with up to 4 values per lane fit in 128 registers,
// which gives four waves per SIMD; 1 leaves the allocation free.
__host__ __device__ constexpr int hub_waves_hint(int cls, int nv) { return cls == HUB_NCLASS + 2 && nv <= 4 ? 4 : 1; }
// largest function count of a launch class (0: per-site chunks, L <= 7)
__host__ __device__ constexpr int hub_cls_nfmax(int cls) {
    return cls > HUB_NCLASS ? 4 * (cls - HUB_NCLASS) : (cls == 0 ? 7 : 4 * cls);
}

// Work-groups are dispatched to the XCDs round-robin (work-group w runs on
// XCD w mod 8), and each XCD has its own L2.  The 1-D launch grid maps w to
// (chunk slot, column tile) so that the tiles of one chunk are consecutive
// work-groups of one XCD: the chunk's indexes and orbital values are read
// from HBM once and from that XCD's L2 by the other tiles.
#define HUB_NXCD 8
struct HubSlot {
    int chunk;                // index into the launch's chunk list
    int tile;                 // column tile
};
__device__ __forceinline__ HubSlot hub_slot(int tiles) {
    const int w = blockIdx.x;
    const int wl = w / HUB_NXCD;
    return {(wl / tiles) * HUB_NXCD + (w - wl * HUB_NXCD), wl % tiles};
}
// work-groups of such a launch (chunk slots past nchunks exit at once)
inline int64_t hub_slot_grid(int nchunks, int64_t tiles) {
    return static_cast<int64_t>((nchunks + HUB_NXCD - 1) / HUB_NXCD) * HUB_NXCD * tiles;
}

// Splits [0, n) into nw contiguous ranges; range w is [lo, lo + len).
__device__ __forceinline__ void hub_wave_range(int n, int nw, int w, int& lo, int& len) {
    const int per = (n + nw - 1) / nw;
    lo = w * per;
    const int hi = lo + per < n ? lo + per : n;
    len = hi > lo ? hi - lo : 0;
}

// Launchers, one translation unit per storage precision (and work list).
hipError_t launch_project_f32(const ProjArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, int cls,
                              hipStream_t st);
hipError_t launch_project_f64(const ProjArgs& a, int nchunks, int nq, int cplx, int cpl, int waves, int cls,
                              hipStream_t st);
// orbital and position-moment projections of complex states over grouped
// chunks (k_project_mom.h).  Work items: chunk * 2 + h, h the half of the
// chunk's functions (h = 1 only for chunks with more than HUB_MOM_NFW
// functions); a.chunk_list holds nitems of them.
#define HUB_MOM_NFW 8
hipError_t launch_project_mom_f32(const ProjArgs& a, int nitems, int nq, hipStream_t st);
hipError_t launch_project_mom_f64(const ProjArgs& a, int nitems, int nq, hipStream_t st);
hipError_t launch_apply_f32(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves,
                            hipStream_t st);
hipError_t launch_apply_f64(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves,
                            hipStream_t st);
hipError_t launch_apply_grouped_f32(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves,
                                    int cls, hipStream_t st);
hipError_t launch_apply_grouped_f64(const ApplyArgs& a, int nchunks, int nq, int cplx, int cpl, int waves,
                                    int cls, hipStream_t st);

// cls: function-count class of the chunks in a.chunk_list (0: per-site list)
inline hipError_t launch_project(const ProjArgs& a, int nchunks, int nq, int prec, int cplx, int cpl, int waves,
                                 int cls, hipStream_t st) {
    return prec == HUB_F64 ? launch_project_f64(a, nchunks, nq, cplx, cpl, waves, cls, st)
                           : launch_project_f32(a, nchunks, nq, cplx, cpl, waves, cls, st);
}
inline hipError_t launch_apply(const ApplyArgs& a, int nchunks, int nq, int prec, int cplx, int cpl, int waves,
                               hipStream_t st) {
    return prec == HUB_F64 ? launch_apply_f64(a, nchunks, nq, cplx, cpl, waves, st)
                           : launch_apply_f32(a, nchunks, nq, cplx, cpl, waves, st);
}
inline hipError_t launch_apply_grouped(const ApplyArgs& a, int nchunks, int nq, int prec, int cplx, int cpl,
                                       int waves, int cls, hipStream_t st) {
    return prec == HUB_F64 ? launch_apply_grouped_f64(a, nchunks, nq, cplx, cpl, waves, cls, st)
                           : launch_apply_grouped_f32(a, nchunks, nq, cplx, cpl, waves, cls, st);
}
