// Device side of the UTIL-table engine for gfx950 (CDNA4, wave64).
//
// UTIL kernel: for a mini-bucket with joint scope U = (u_0..u_{nv-1}, x),
// every output row s (an assignment of u_0..u_{nv-1}, row-major) gets
//     g[s] = min_{v in D_x} (+)_{f} f[ sum_j stride_f(u_j) * digit_j(s) + v ]
// i.e. the aggregation of Sec. 5.3 (Eq. (1): mixed-radix decode of the output
// row, re-encoded over each input table's scope) fused with the elimination
// of Sec. 5.4 (x is the last scope variable of every table, so its D entries
// are contiguous).  Nothing is materialised over the joint scope: each
// output row is written once, each table entry read from HBM/L2.
// (+) is the saturating int32 sum (infinity = INT32_MAX) or the float sum.
//
// Two code paths per tile:
//   tiled: row = o * p_in + r.  The decode of Eq. (1) is split in two: the
//          outer part of every table offset is computed once per outer index
//          (one thread each) into LDS, the inner part once per thread into
//          registers; functions that do not depend on the inner variables
//          are pre-summed per outer index (LDS).  The row loop is then one
//          LDS broadcast + one vector load of D entries per remaining function.
//   row:   full decode per row (any D, any number of functions).
//
// Schedules: one launch per mini-bucket, or one launch per dependency level
// (all instances and all independent mini-buckets of the level together);
// either sequence can be captured once into a hipGraph and replayed.
//
// VALUE kernel: back-substitution of Alg. 1/2 (second loop) along value
// levels, then the bound (constants left after elimination) and the cost of
// the assignment over the input functions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>

#include "bx_internal.h"

namespace bx {

bx_status dev_upload_tiles(Plan &P, void *ws, hipStream_t st);

namespace {

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return set_error(BX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------ cost algebra
// Integers accumulate as uint32 with a clamping add (v_add_u32 ... clamp); for
// non-negative int32 inputs min(INF, exact sum) is recovered at the end, the
// same value as a step-by-step saturating sum, whatever the order.
struct CostI {
    using T = int32_t;
    using A = uint32_t;
    __device__ static A zero() { return 0u; }
    __device__ static A add(A a, T v) { return __builtin_elementwise_add_sat(a, (uint32_t)v); }
    __device__ static A add2(A a, A b) { return __builtin_elementwise_add_sat(a, b); }
    __device__ static A mn(A a, A b) { return a < b ? a : b; }
    __device__ static T fin(A a) { return (T)(a < (uint32_t)kInfI32 ? a : (uint32_t)kInfI32); }
    __device__ static uint32_t bits(A a) { return a; }
    __device__ static A from_bits(uint32_t b) { return b; }
};
struct CostF {
    using T = float;
    using A = float;
    __device__ static A zero() { return 0.f; }
    __device__ static A add(A a, T v) { return a + v; }
    __device__ static A add2(A a, A b) { return a + b; }
    __device__ static A mn(A a, A b) { return fminf(a, b); }
    __device__ static T fin(A a) { return a; }
    __device__ static uint32_t bits(A a) { return __float_as_uint(a); }
    __device__ static A from_bits(uint32_t b) { return __uint_as_float(b); }
};

struct Descs {
    const DevMb *mb;
    const DevFn *fn;
    const DevTile *tile;
    char *ws;
    const char *zeros;   // 256 zero bytes of the workspace
    int32_t n_tiles;
    int32_t nt;          // blocked rows stored non-temporally (per launch)
};

// ------------------------------------------------------------ row path
// One thread per output row, full mixed-radix decode per row (Eq. (1)).  The
// eliminated domain is a template parameter so the D accumulators stay in
// registers; DT == 0 handles any D with a running minimum.
template <class C, int DT>
__device__ __forceinline__ void rows_tile(const Descs &d, const DevMb &mb, int64_t begin,
                                          int64_t end) {
    using T = typename C::T;
    using A = typename C::A;
    const T *tab = reinterpret_cast<const T *>(d.ws);
    T *out = reinterpret_cast<T *>(d.ws) + mb.out_off;
    const int nv = mb.nv, nf = mb.nf;
    const DevFn *fns = d.fn + mb.f_begin;
    for (int64_t r = begin + threadIdx.x; r < end; r += blockDim.x) {
        uint32_t dig[kMaxVars];
        uint32_t rem = (uint32_t)r;
#pragma unroll
        for (int j = kMaxVars - 1; j >= 0; --j) {
            if (j < nv) {
                const uint32_t dj = (uint32_t)mb.dims[j];
                const uint32_t q = rem / dj;
                dig[j] = rem - q * dj;
                rem = q;
            } else {
                dig[j] = 0;
            }
        }
        if constexpr (DT > 0) {
            A acc[DT];
#pragma unroll
            for (int x = 0; x < DT; ++x) acc[x] = C::zero();
            for (int f = 0; f < nf; ++f) {
                int32_t base = 0;
#pragma unroll
                for (int j = 0; j < kMaxVars; ++j)
                    if (j < nv) base += (int32_t)dig[j] * fns[f].stride[j];
                const T *p = tab + fns[f].tab_off + base;
#pragma unroll
                for (int x = 0; x < DT; ++x) acc[x] = C::add(acc[x], p[x]);
            }
            A best = acc[0];
#pragma unroll
            for (int x = 1; x < DT; ++x) best = C::mn(best, acc[x]);
            out[r] = C::fin(best);
        } else {
            A best = C::zero();
            for (int x = 0; x < mb.D; ++x) {
                A s = C::zero();
                for (int f = 0; f < nf; ++f) {
                    int32_t base = x;
#pragma unroll
                    for (int j = 0; j < kMaxVars; ++j)
                        if (j < nv) base += (int32_t)dig[j] * fns[f].stride[j];
                    s = C::add(s, tab[fns[f].tab_off + base]);
                }
                best = x == 0 ? s : C::mn(best, s);
            }
            out[r] = C::fin(best);
        }
    }
}

template <class C>
__device__ __forceinline__ void run_rows(const Descs &d, const DevMb &mb, int64_t b, int64_t e) {
    switch (mb.D) {
    case 1: rows_tile<C, 1>(d, mb, b, e); break;
    case 2: rows_tile<C, 2>(d, mb, b, e); break;
    case 3: rows_tile<C, 3>(d, mb, b, e); break;
    case 4: rows_tile<C, 4>(d, mb, b, e); break;
    case 5: rows_tile<C, 5>(d, mb, b, e); break;
    case 6: rows_tile<C, 6>(d, mb, b, e); break;
    case 7: rows_tile<C, 7>(d, mb, b, e); break;
    case 8: rows_tile<C, 8>(d, mb, b, e); break;
    default: rows_tile<C, 0>(d, mb, b, e); break;
    }
}

// ------------------------------------------------------------ tiled path
// LDS of one workgroup.  The staging buffer exists only in the kernel that
// stages (it costs occupancy: 33 KB against 17 KB per workgroup).
template <bool kStage>
struct TileSmem {
    int32_t outer[kTileMaxOuter][kTileLaneFns];   // outer part of lane-function offsets
    uint32_t usum[kTileMaxOuter][kTileMaxD];      // pre-summed outer-only functions
    uint32_t stage[kStage ? kStageEntries : 1];   // rows of small lane tables (raw bits)
    int32_t lo[kStageMaxFns], hi[kStageMaxFns];    // min / max outer offset in the tile
};

// N consecutive entries starting at p, where p is a multiple of N entries from
// a 256-byte boundary: use the widest vector access that alignment allows.
template <int N, class T>
__device__ __forceinline__ void load_run(const T *p, T (&v)[N]) {
    using V4 = typename std::conditional<std::is_same<T, float>::value, float4, int4>::type;
    using V2 = typename std::conditional<std::is_same<T, float>::value, float2, int2>::type;
    if constexpr (N % 4 == 0) {
#pragma unroll
        for (int i = 0; i < N / 4; ++i) {
            const V4 w = reinterpret_cast<const V4 *>(p)[i];
            v[4 * i] = w.x; v[4 * i + 1] = w.y; v[4 * i + 2] = w.z; v[4 * i + 3] = w.w;
        }
    } else if constexpr (N % 2 == 0) {
#pragma unroll
        for (int i = 0; i < N / 2; ++i) {
            const V2 w = reinterpret_cast<const V2 *>(p)[i];
            v[2 * i] = w.x; v[2 * i + 1] = w.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = p[i];
    }
}

// Row loop of the tiled path.  Each thread owns inner position r of outer
// slots qs, qs + q, ...; for each it adds the pre-summed outer-only
// functions (LDS broadcast) and the KL lane functions (one run of DT entries
// each), takes the minimum over the DT values and writes one row.  The first
// KS lane functions are read from their rows staged in LDS (sb[f] = position
// of the staged copy minus the first staged offset, plus io[f]), the others
// from HBM / cache.  U outer slots per trip: all their loads are issued
// together, and before the previous trip's stores -- the vector-memory
// counter covers loads and stores in issue order, so waiting for a trip's
// loads then never waits for stores.  Table bases are uniform (scalar
// registers) and offsets 32-bit byte counts, so loads use a scalar base plus
// a vector offset.  Slots past the end of the tile re-read the last outer
// index (in range) and skip the store.
template <class C, int DT, int KL, int KS, class SM>
__device__ __forceinline__ void tiled_rows(const Descs &d, const DevMb &mb, const DevFn *fns,
                                           int64_t o_begin, int n_o, const SM &sm,
                                           const int32_t (&io)[kTileLaneFns], const int32_t (&sb)[kStageMaxFns],
                                           const typename C::A (&cv)[DT], int qs, int r) {
    using T = typename C::T;
    using A = typename C::A;
    constexpr int KLD = (KL > 0 ? KL : 1) * DT;
    constexpr int U = KLD > 16 ? 1 : (KLD > 8 ? 2 : 4);   // U * KLD <= 32 loaded registers
    const int P = mb.p_in, Q = mb.q;
    const char *tb[KL > 0 ? KL : 1];
    uint32_t iob[KL > 0 ? KL : 1];
#pragma unroll
    for (int f = 0; f < KL; ++f) {
        tb[f] = d.ws + fns[f].tab_off * (int64_t)sizeof(T);
        iob[f] = (uint32_t)io[f] * (uint32_t)sizeof(T);
    }
    char *ob = d.ws + (mb.out_off + o_begin * P) * (int64_t)sizeof(T);
    const uint32_t rb = (uint32_t)r * (uint32_t)sizeof(T);
    const uint32_t pb = (uint32_t)P * (uint32_t)sizeof(T);
    T v[U][KL > 0 ? KL : 1][DT];
    A best[U];
    auto issue = [&](int ol0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ol = min(ol0 + u * Q, n_o - 1);
#pragma unroll
            for (int f = 0; f < KL; ++f) {
                if (f < KS)
                    load_run<DT>(reinterpret_cast<const T *>(sm.stage) + (sm.outer[ol][f] + sb[f]), v[u][f]);
                else
                    load_run<DT>(reinterpret_cast<const T *>(
                                     tb[f] + ((uint32_t)sm.outer[ol][f] * (uint32_t)sizeof(T) + iob[f])),
                                 v[u][f]);
            }
        }
    };
    auto compute = [&](int ol0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ol = min(ol0 + u * Q, n_o - 1);
            A acc[DT];
#pragma unroll
            for (int x = 0; x < DT; ++x) acc[x] = C::add2(C::from_bits(sm.usum[ol][x]), cv[x]);
#pragma unroll
            for (int f = 0; f < KL; ++f)
#pragma unroll
                for (int x = 0; x < DT; ++x) acc[x] = C::add(acc[x], v[u][f][x]);
            best[u] = acc[0];
#pragma unroll
            for (int x = 1; x < DT; ++x) best[u] = C::mn(best[u], acc[x]);
        }
    };
    auto store = [&](int ol0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ol = ol0 + u * Q;
            if (ol < n_o) *reinterpret_cast<T *>(ob + ((uint32_t)ol * pb + rb)) = C::fin(best[u]);
        }
    };
    if (qs >= n_o) return;
    issue(qs);
    compute(qs);
    int prev = qs;
    for (int ol0 = qs + U * Q; ol0 < n_o; ol0 += U * Q) {
        issue(ol0);
        store(prev);
        compute(ol0);
        prev = ol0;
    }
    store(prev);
}

// Register-blocked row loop.  The tile's outer indices are visited with the
// two box variables a (da <= kBlockMaxDa values) and b (DB values) fastest,
// so outer slot l = (box * da + ia) * DB + ib.  Thread (qs, r) takes boxes
// qs, qs + q, ... and computes all da * DB rows of each.  A blocked
// mini-bucket has at most three lane functions: one depending on neither
// box variable (loaded once per box), one on b only (once per ib), one on a
// only (once per ia); the partial sums stay in registers and each row adds
// the pre-summed outer-only functions (LDS) before the minimum over D.  All
// loads of a box are issued together, and the next box's before this box's
// stores: the vector-memory counter covers loads and stores in issue order,
// so waiting for a box's loads never waits for the previous box's stores.
// Loads for ia >= da re-read ia = da - 1 (in range); those rows are not
// stored, non-temporally when the launch says so (the autotuner's choice per
// level).  The output outer index of slot l was stored by phase 1 in LDS
// column kBlockRowCol.
template <class C, int DT, int DA, int DB, bool kNT, class SM>
__device__ __forceinline__ void blocked_rows(const Descs &d, const DevMb &mb, const DevFn *fns, int n_o,
                                             const SM &sm, const int32_t (&dig)[kBlockMaxInner],
                                             const typename C::A (&cv)[DT], int qs, int r) {
    using T = typename C::T;
    using A = typename C::A;
    const int P = mb.p_in, Q = mb.q;
    const int da = mb.da, box = da * DB;
    const int nb = n_o / box;
    const int nvo = mb.nv - mb.n_inner, n_in = mb.n_inner;
    char *ob = d.ws + mb.out_off * (int64_t)sizeof(T);
    const uint32_t rb = (uint32_t)r * (uint32_t)sizeof(T);
    const uint32_t pb = (uint32_t)P * (uint32_t)sizeof(T);
    // table base (uniform) and this thread's inner offset (bytes) of lane function f
    auto lane = [&](int f, uint32_t &iob) -> const char * {
        int32_t io = 0;
#pragma unroll
        for (int k = 0; k < kBlockMaxInner; ++k)
            if (k < n_in) io += dig[k] * fns[f].stride[nvo + k];
        iob = (uint32_t)io * (uint32_t)sizeof(T);
        return d.ws + fns[f].tab_off * (int64_t)sizeof(T);
    };
    // first function of each group; a group without a function reads zeros
    // (the workspace's zero block, offset masked to 0) -- no branch, no phi
    const bool h0 = mb.g0 > 0, h1 = mb.ga > mb.g0, h2 = mb.gb > mb.ga;
    const int f0 = 0, f1 = h1 ? mb.g0 : 0, f2 = h2 ? mb.ga : 0;
    const int32_t m0 = h0 ? -1 : 0, m1 = h1 ? -1 : 0, m2 = h2 ? -1 : 0;
    uint32_t io0 = 0, io1 = 0, io2 = 0;
    const char *tb0 = h0 ? lane(f0, io0) : d.zeros;
    const char *tb1 = h1 ? lane(f1, io1) : d.zeros;
    const char *tb2 = h2 ? lane(f2, io2) : d.zeros;
    auto at = [&](const char *tb, uint32_t iob, int32_t m, int l, int f) -> const T * {
        return reinterpret_cast<const T *>(tb + ((uint32_t)(sm.outer[l][f] & m) * (uint32_t)sizeof(T) + iob));
    };
    T v0[DT], v1[DB][DT], v2[DA][DT];
    auto issue = [&](int l0) {
        load_run<DT>(at(tb0, io0, m0, l0, f0), v0);
#pragma unroll
        for (int b = 0; b < DB; ++b) load_run<DT>(at(tb1, io1, m1, l0 + b, f1), v1[b]);
#pragma unroll
        for (int ia = 0; ia < DA; ++ia) load_run<DT>(at(tb2, io2, m2, l0 + min(ia, da - 1) * DB, f2), v2[ia]);
    };
    A best[DA][DB];
    auto compute = [&](int l0) {
#pragma unroll
        for (int ia = 0; ia < DA; ++ia) {
            const int la = l0 + min(ia, da - 1) * DB;
#pragma unroll
            for (int b = 0; b < DB; ++b) {
                A acc[DT];
#pragma unroll
                for (int x = 0; x < DT; ++x)
                    acc[x] = C::add(C::add(C::add(C::add2(C::from_bits(sm.usum[la + b][x]), cv[x]), v0[x]),
                                           v1[b][x]),
                                    v2[ia][x]);
                best[ia][b] = acc[0];
#pragma unroll
                for (int x = 1; x < DT; ++x) best[ia][b] = C::mn(best[ia][b], acc[x]);
            }
        }
    };
    auto store = [&](int l0) {
#pragma unroll
        for (int ia = 0; ia < DA; ++ia) {
            if (ia >= da) break;
#pragma unroll
            for (int b = 0; b < DB; ++b) {
                const uint32_t orow = (uint32_t)sm.outer[l0 + ia * DB + b][kBlockRowCol];
                T *dst = reinterpret_cast<T *>(ob + (orow * pb + rb));
                if constexpr (kNT)
                    __builtin_nontemporal_store(C::fin(best[ia][b]), dst);
                else
                    *dst = C::fin(best[ia][b]);
            }
        }
    };
    if (qs >= nb) return;
    // a box's loads are issued before the previous box's stores
    issue(qs * box);
    compute(qs * box);
    int prev = qs * box;
    for (int bq = qs + Q; bq < nb; bq += Q) {
        const int l0 = bq * box;
        issue(l0);
        store(prev);
        compute(l0);
        prev = l0;
    }
    store(prev);
}

template <class C, int DT, bool kNT, class SM>
__device__ __forceinline__ void run_blocked(const Descs &d, const DevMb &mb, const DevFn *fns, int n_o,
                                            const SM &sm, const int32_t (&dig)[kBlockMaxInner],
                                            const typename C::A (&cv)[DT], int qs, int r) {
    // register copies of the a loads: 1 without an a variable, else 4 (a
    // domain of 2 or 3 re-reads its last value)
    if (mb.da == 1) {
        switch (mb.db) {
        case 2: blocked_rows<C, DT, 1, 2, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        case 3: blocked_rows<C, DT, 1, 3, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        default: blocked_rows<C, DT, 1, 4, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        }
    } else {
        switch (mb.db) {
        case 2: blocked_rows<C, DT, kBlockMaxDa, 2, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        case 3: blocked_rows<C, DT, kBlockMaxDa, 3, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        default: blocked_rows<C, DT, kBlockMaxDa, 4, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        }
    }
}

// Row loop with the number of staged lane functions as a template argument
// (staging only for D <= kStageMaxD).
template <class C, int DT, int KL, class SM>
__device__ __forceinline__ void rows_ks(int KS, const Descs &d, const DevMb &mb, const DevFn *fns,
                                        int64_t o_begin, int n_o, const SM &sm,
                                        const int32_t (&io)[kTileLaneFns], const int32_t (&sb)[kStageMaxFns],
                                        const typename C::A (&cv)[DT], int qs, int r) {
    if constexpr (DT > kStageMaxD || sizeof(sm.stage) < sizeof(uint32_t) * kStageEntries) {
        tiled_rows<C, DT, KL, 0>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r);
    } else {
        switch (KS) {
        case 0: tiled_rows<C, DT, KL, 0>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 1: tiled_rows<C, DT, KL, 1>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 2: if constexpr (KL >= 2) tiled_rows<C, DT, KL, 2>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 3: if constexpr (KL >= 3) tiled_rows<C, DT, KL, 3>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        default: if constexpr (KL >= 4) tiled_rows<C, DT, KL, 4>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        }
    }
}

template <class C, int DT, bool kStage, bool kNT>
__device__ __forceinline__ void tiled_tile(const Descs &d, const DevMb &mb, int64_t o_begin,
                                           int64_t o_end, TileSmem<kStage> &sm) {
    using T = typename C::T;
    using A = typename C::A;
    const T *tab = reinterpret_cast<const T *>(d.ws);
    const int tid = threadIdx.x;
    const int nv = mb.nv, KL = mb.nfl, NI = mb.nfi, NC = mb.nfc, NU = mb.nf - KL - NI - NC;
    const int nvo = nv - mb.n_inner;
    const int n_o = (int)(o_end - o_begin);
    const DevFn *fns = d.fn + mb.f_begin;
    const int P = mb.p_in;
    const int qs = tid / P;
    const int r = tid - qs * P;
    // functions of the eliminated variable alone, and functions of inner
    // variables only: for a thread (fixed inner position) the same D entries
    // on every row of the tile, summed once into registers (loads issued
    // before phase 1, so their latency overlaps it)
    A cv[DT];
#pragma unroll
    for (int x = 0; x < DT; ++x) cv[x] = C::zero();
    for (int g = 0; g < NI + NC; ++g) {
        const DevFn &fn = fns[KL + NU + g];
        int32_t off = 0;
        if (g < NI) {
            uint32_t rem = (uint32_t)r;
            for (int j = nv - 1; j >= nvo; --j) {
                const uint32_t dj = (uint32_t)mb.dims[j];
                const uint32_t q = rem / dj;
                off += (int32_t)(rem - q * dj) * fn.stride[j];
                rem = q;
            }
        }
        T v[DT];
        load_run<DT>(tab + fn.tab_off + off, v);
#pragma unroll
        for (int x = 0; x < DT; ++x) cv[x] = C::add(cv[x], v[x]);
    }

    // staging candidates need the smallest and largest outer offset of each
    // lane function over the tile
    const bool stage_ok = kStage && DT <= kStageMaxD && KL <= kStageMaxFns && !mb.blk;
    if (stage_ok) {
        if (tid < KL) {
            sm.lo[tid] = 0x7fffffff;
            sm.hi[tid] = 0;
        }
        __syncthreads();
    }
    // phase 1: one outer index per thread -- the outer part of each lane
    // function's offset, and the sum of the functions without inner
    // variables; the digits of Eq. (1) are folded into the offsets as they
    // are produced, last variable first
    for (int ol = tid; ol < n_o; ol += kUtilThreads) {
        int32_t lo[kTileLaneFns], uo[kTileOuterFns];
#pragma unroll
        for (int f = 0; f < kTileLaneFns; ++f) lo[f] = 0;
#pragma unroll
        for (int g = 0; g < kTileOuterFns; ++g) uo[g] = 0;
        uint32_t rem = (uint32_t)(o_begin + ol);
        int32_t orow = 0;   // blocked: outer index of the output row
        for (int j = nvo - 1; j >= 0; --j) {
            const uint32_t dj = (uint32_t)mb.dims[j];
            const uint32_t q = rem / dj;
            const int32_t dg = (int32_t)(rem - q * dj);
            rem = q;
            orow += dg * mb.ostr[j];
#pragma unroll
            for (int f = 0; f < kTileLaneFns; ++f)
                if (f < KL) lo[f] += dg * fns[f].stride[j];
#pragma unroll
            for (int g = 0; g < kTileOuterFns; ++g)
                if (g < NU) uo[g] += dg * fns[KL + g].stride[j];
        }
#pragma unroll
        for (int f = 0; f < kTileLaneFns; ++f)
            if (f < KL) sm.outer[ol][f] = lo[f];
        if (mb.blk) sm.outer[ol][kBlockRowCol] = orow;
        if (stage_ok) {
#pragma unroll
            for (int f = 0; f < kStageMaxFns; ++f) {
                if (f < KL) {
                    atomicMin(&sm.lo[f], lo[f]);
                    atomicMax(&sm.hi[f], lo[f]);
                }
            }
        }
        A us[DT];
#pragma unroll
        for (int x = 0; x < DT; ++x) us[x] = C::zero();
#pragma unroll
        for (int g = 0; g < kTileOuterFns; ++g) {
            if (g < NU) {
                T v[DT];
                load_run<DT>(tab + fns[KL + g].tab_off + uo[g], v);
#pragma unroll
                for (int x = 0; x < DT; ++x) us[x] = C::add(us[x], v[x]);
            }
        }
#pragma unroll
        for (int x = 0; x < DT; ++x) sm.usum[ol][x] = C::bits(us[x]);
    }
    // phase 2: the inner part of each lane function's offset
    int32_t io[kTileLaneFns];
#pragma unroll
    for (int f = 0; f < kTileLaneFns; ++f) io[f] = 0;
    int32_t dig[kBlockMaxInner];   // inner digits, fastest last (blocked loop)
#pragma unroll
    for (int k = 0; k < kBlockMaxInner; ++k) dig[k] = 0;
    {
        uint32_t rem = (uint32_t)r;
        for (int j = nv - 1; j >= nvo; --j) {
            const uint32_t dj = (uint32_t)mb.dims[j];
            const uint32_t q = rem / dj;
            const int32_t dg = (int32_t)(rem - q * dj);
            rem = q;
#pragma unroll
            for (int k = 0; k < kBlockMaxInner; ++k)
                if (k == j - nvo) dig[k] = dg;
#pragma unroll
            for (int f = 0; f < kTileLaneFns; ++f)
                if (f < KL) io[f] += dg * fns[f].stride[j];
        }
    }
    __syncthreads();
    // phase 3: staging.  Every entry a tile reads from a lane table lies
    // between its smallest outer offset (inner part 0) and its largest outer
    // offset plus the largest inner part plus D - 1: one contiguous range of
    // the table.  The first lane functions whose ranges fit the LDS buffer
    // together, and whose staged entries are read kStageReuse times each on
    // average, are copied in.
    int32_t sb[kStageMaxFns];
#pragma unroll
    for (int f = 0; f < kStageMaxFns; ++f) sb[f] = 0;
    int KS = 0;
    if constexpr (kStage && DT <= kStageMaxD) {
        if (stage_ok) {
            const int64_t reads = (int64_t)n_o * P * DT;   // entries read per lane function
            int used = 0;
            for (int f = 0; f < KL; ++f) {
                const int32_t lo = sm.lo[f];
                const int32_t range = sm.hi[f] + fns[f].io_max + DT - lo;
                if (used + range > kStageEntries || reads < (int64_t)kStageReuse * range) break;
                const uint32_t *src = reinterpret_cast<const uint32_t *>(tab + fns[f].tab_off + lo);
                for (int e = tid; e < range; e += kUtilThreads) sm.stage[used + e] = src[e];
                sb[f] = used - lo + io[f];
                used += range;
                ++KS;
            }
        }
    }
    KS = __builtin_amdgcn_readfirstlane(KS);
    __syncthreads();
    // phase 4: the rows
    if (qs < mb.q && mb.blk) {
        if constexpr (DT <= kBlockMaxD) run_blocked<C, DT, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r);
    } else if (qs < mb.q) {
        switch (KL) {
        case 0: tiled_rows<C, DT, 0, 0>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 1: rows_ks<C, DT, 1>(KS, d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 2: rows_ks<C, DT, 2>(KS, d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 3: rows_ks<C, DT, 3>(KS, d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 4: rows_ks<C, DT, 4>(KS, d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 5: if constexpr (5 * DT <= kTileMaxRun) tiled_rows<C, DT, 5, 0>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 6: if constexpr (6 * DT <= kTileMaxRun) tiled_rows<C, DT, 6, 0>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        case 7: if constexpr (7 * DT <= kTileMaxRun) tiled_rows<C, DT, 7, 0>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        default: if constexpr (8 * DT <= kTileMaxRun) tiled_rows<C, DT, 8, 0>(d, mb, fns, o_begin, n_o, sm, io, sb, cv, qs, r); break;
        }
    }
    __syncthreads();   // the LDS tables are rewritten by the next tile
}

// Tiles of the tiled path, one workgroup each (PER_BUCKET and LEVEL
// schedules); kStage: with the LDS staging of lane tables.  At least 6 waves
// per SIMD (<= 80 VGPRs) where LDS allows it: the row loops are
// latency-bound and occupancy is what hides the latency.
template <class C, bool kStage, bool kNT>
__global__ __launch_bounds__(kUtilThreads, 6) void util_tiles_kernel(Descs d, int32_t tile0) {
    __shared__ TileSmem<kStage> sm;
    const DevTile t = d.tile[tile0 + blockIdx.x];
    const DevMb &mb = d.mb[t.mb];
    switch (mb.D) {
    case 1: tiled_tile<C, 1, kStage, kNT>(d, mb, t.begin, t.end, sm); break;
    case 2: tiled_tile<C, 2, kStage, kNT>(d, mb, t.begin, t.end, sm); break;
    case 3: tiled_tile<C, 3, kStage, kNT>(d, mb, t.begin, t.end, sm); break;
    case 4: tiled_tile<C, 4, kStage, kNT>(d, mb, t.begin, t.end, sm); break;
    case 5: tiled_tile<C, 5, kStage, kNT>(d, mb, t.begin, t.end, sm); break;
    case 6: tiled_tile<C, 6, kStage, kNT>(d, mb, t.begin, t.end, sm); break;
    case 7: tiled_tile<C, 7, kStage, kNT>(d, mb, t.begin, t.end, sm); break;
    default: tiled_tile<C, 8, kStage, kNT>(d, mb, t.begin, t.end, sm); break;
    }
}

// Tiles of the row path, one workgroup each.
template <class C>
__global__ __launch_bounds__(kUtilThreads) void util_rows_kernel(Descs d, int32_t tile0) {
    const DevTile t = d.tile[tile0 + blockIdx.x];
    run_rows<C>(d, d.mb[t.mb], t.begin, t.end);
}

// ------------------------------------------------------------ value kernel
constexpr int kValueThreads = 256;
constexpr int kSigmaCap = 16384;   // variables per problem (uint16 in LDS)
constexpr int kPairCap = kValuePairCap;  // candidate values per value step

struct VDescs {
    const DevInst *inst;
    const DevVar *var;
    const DevVFn *vfn;
    const int32_t *term;
    const DevPair *pair;
    const int32_t *vlv;
    const int32_t *vlp;
    const int64_t *cst;
    DevResult *res;
    char *ws;
    char *sigma_base;
};

// one workgroup per problem
template <class C>
__global__ __launch_bounds__(kValueThreads) void value_kernel(VDescs d) {
    using T = typename C::T;
    constexpr bool kF = std::is_same<T, float>::value;
    using S = typename std::conditional<kF, double, uint32_t>::type;   // comparison type
    __shared__ uint16_t sigma[kSigmaCap];
    __shared__ S cost[kPairCap];
    __shared__ S red[kValueThreads];
    const DevInst I = d.inst[blockIdx.x];
    const T *tab = reinterpret_cast<const T *>(d.ws);
    const int tid = threadIdx.x;
    for (int v = tid; v < I.n; v += blockDim.x) sigma[v] = 0;
    __syncthreads();
    auto add = [](S a, T v) -> S {
        if constexpr (kF) return a + (double)v;
        else return __builtin_elementwise_add_sat(a, (uint32_t)v);
    };
    auto cap = [](S a) -> S {
        if constexpr (kF) return a;
        else return a < (uint32_t)kInfI32 ? a : (uint32_t)kInfI32;
    };
    // the problem's function descriptors and (var, stride) terms, copied to
    // LDS when they fit (they do not depend on the assignment)
    __shared__ uint4 vstage[kValueStageBytes / 16];
    const bool staged = (int64_t)I.vfn_n * 16 + (int64_t)I.term_n * 8 <= kValueStageBytes;
    DevVFn *vfn_l = reinterpret_cast<DevVFn *>(vstage);
    int2 *term_l = reinterpret_cast<int2 *>(vfn_l + I.vfn_n);
    const int2 *terms_g = reinterpret_cast<const int2 *>(d.term);
    if (staged) {
        for (int i = tid; i < I.vfn_n; i += blockDim.x) vfn_l[i] = d.vfn[I.vfn_begin + i];
        for (int i = tid; i < I.term_n; i += blockDim.x) term_l[i] = terms_g[I.term_begin + i];
    }
    __syncthreads();
    S u = 0;
    auto pass = [&](auto staged_tag) {
        constexpr bool kStaged = decltype(staged_tag)::value;
        auto vfn_at = [&](int f) -> DevVFn {
            if constexpr (kStaged) return vfn_l[f - I.vfn_begin];
            else return d.vfn[f];
        };
        auto term_at = [&](int t) -> int2 {
            if constexpr (kStaged) return term_l[t - I.term_begin];
            else return terms_g[t];
        };
        // one entry of function e for value x under the current assignment
        // (terms four at a time, so that their loads are in flight together)
        auto lookup = [&](const DevVFn &e, int32_t x) -> T {
            int64_t idx = e.tab_off + x;
            int t = e.t_begin;
            const int te = e.t_begin + e.nt;
            for (; t + 4 <= te; t += 4) {
                const int2 a = term_at(t), b = term_at(t + 1), c = term_at(t + 2), g = term_at(t + 3);
                idx += (int64_t)sigma[a.x] * a.y + (int64_t)sigma[b.x] * b.y + (int64_t)sigma[c.x] * c.y +
                       (int64_t)sigma[g.x] * g.y;
            }
            for (; t < te; ++t) {
                const int2 a = term_at(t);
                idx += (int64_t)sigma[a.x] * a.y;
            }
            return tab[idx];
        };
        for (int s = I.lvl_begin; s < I.lvl_begin + I.n_lvl; ++s) {
            const int pb = d.vlp[s], pe = d.vlp[s + 1];
            const int vb = d.vlv[s], ve = d.vlv[s + 1];
            // the argmin below needs no assignment: fetch its descriptor now
            DevVar mine{};
            if (vb + tid < ve) mine = d.var[vb + tid];
            for (int p = pb + tid; p < pe; p += blockDim.x) {
                const DevPair pr = d.pair[p];
                S c = 0;
                int f = pr.f_begin;
                const int fe = pr.f_begin + pr.nf;
                // four functions at a time: their lookups are independent
                for (; f + 4 <= fe; f += 4) {
                    const DevVFn e0 = vfn_at(f), e1 = vfn_at(f + 1), e2 = vfn_at(f + 2), e3 = vfn_at(f + 3);
                    const T v0 = lookup(e0, pr.x), v1 = lookup(e1, pr.x), v2 = lookup(e2, pr.x),
                            v3 = lookup(e3, pr.x);
                    c = add(add(add(add(c, v0), v1), v2), v3);
                }
                for (; f < fe; ++f) c = add(c, lookup(vfn_at(f), pr.x));
                cost[p - pb] = cap(c);
            }
            __syncthreads();
            for (int q = vb + tid; q < ve; q += blockDim.x) {
                const DevVar dv = q == vb + tid ? mine : d.var[q];
                const int o = dv.pair_begin - pb;
                S best = cost[o];
                int bx = 0;
                for (int x = 1; x < dv.D; ++x)
                    if (cost[o + x] < best) { best = cost[o + x]; bx = x; }
                sigma[dv.var] = (uint16_t)bx;
            }
            __syncthreads();
        }
        // cost of the assignment over the input functions
        for (int f = I.ub_begin + tid; f < I.ub_begin + I.ub_n; f += blockDim.x) u = add(u, lookup(vfn_at(f), 0));
    };
    if (staged) pass(std::true_type{});
    else pass(std::false_type{});
    int32_t *sig_out = reinterpret_cast<int32_t *>(d.sigma_base + I.sigma_off);
    for (int v = tid; v < I.n; v += blockDim.x) sig_out[v] = sigma[v];
    red[tid] = u;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) {
            if constexpr (kF) red[tid] = red[tid] + red[tid + w];
            else red[tid] = __builtin_elementwise_add_sat(red[tid], red[tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        // bound: constant inputs plus the scalar outputs of elimination
        S b;
        if constexpr (kF) b = I.host_const;
        else b = (uint32_t)(int32_t)I.host_const;
        for (int c = I.const_begin; c < I.const_begin + I.const_n; ++c) b = add(b, tab[d.cst[c]]);
        DevResult r{};
        S ub = red[0];
        if constexpr (kF) {
            r.bound = b;
            r.ub = ub + I.host_const;
        } else {
            ub = __builtin_elementwise_add_sat(ub, (uint32_t)(int32_t)I.host_const);
            r.bound = (double)cap(b);
            r.ub = (double)cap(ub);
        }
        r.status = 0;
        d.res[blockIdx.x] = r;
    }
}

Descs make_descs(const Plan &P, void *ws) {
    char *w = static_cast<char *>(ws);
    Descs d;
    d.mb = reinterpret_cast<const DevMb *>(w + P.off_mb);
    d.fn = reinterpret_cast<const DevFn *>(w + P.off_fn);
    d.tile = reinterpret_cast<const DevTile *>(w + P.off_tile);
    d.ws = w;
    d.zeros = w + P.off_zeros;
    d.n_tiles = (int32_t)P.dtile.size();
    d.nt = 0;
    return d;
}

VDescs make_vdescs(const Plan &P, void *ws) {
    char *w = static_cast<char *>(ws);
    VDescs d;
    d.inst = reinterpret_cast<const DevInst *>(w + P.off_inst);
    d.var = reinterpret_cast<const DevVar *>(w + P.off_var);
    d.vfn = reinterpret_cast<const DevVFn *>(w + P.off_vfn);
    d.term = reinterpret_cast<const int32_t *>(w + P.off_term);
    d.pair = reinterpret_cast<const DevPair *>(w + P.off_pair);
    d.vlv = reinterpret_cast<const int32_t *>(w + P.off_vlv);
    d.vlp = reinterpret_cast<const int32_t *>(w + P.off_vlp);
    d.cst = reinterpret_cast<const int64_t *>(w + P.off_const);
    d.res = reinterpret_cast<DevResult *>(w + P.off_results);
    d.ws = w;
    d.sigma_base = w + P.off_sigma;
    return d;
}

template <class C>
void launch_range(Descs d, int32_t t0, int32_t t_row, int32_t t1, bool stage, bool nt, hipStream_t st) {
    d.nt = nt ? 1 : 0;
    if (t_row > t0) {
        const dim3 grid(t_row - t0), block(kUtilThreads);
        if (stage && nt)
            hipLaunchKernelGGL((util_tiles_kernel<C, true, true>), grid, block, 0, st, d, t0);
        else if (stage)
            hipLaunchKernelGGL((util_tiles_kernel<C, true, false>), grid, block, 0, st, d, t0);
        else if (nt)
            hipLaunchKernelGGL((util_tiles_kernel<C, false, true>), grid, block, 0, st, d, t0);
        else
            hipLaunchKernelGGL((util_tiles_kernel<C, false, false>), grid, block, 0, st, d, t0);
    }
    if (t1 > t_row)
        hipLaunchKernelGGL(util_rows_kernel<C>, dim3(t1 - t_row), dim3(kUtilThreads), 0, st, d, t_row);
}

template <class C>
bx_status launch_util(Plan &P, void *ws, bx_schedule sched, hipStream_t st) {
    Descs d = make_descs(P, ws);
    if (P.dtile.empty()) return BX_OK;
    if (sched == BX_SCHED_PER_BUCKET) {
        for (const PInst &I : P.inst)
            for (int32_t g : I.mbs) {
                const PMb &mb = P.mbs[g];
                if (mb.n_tiles == 0) continue;
                const int32_t t0 = mb.first_tile, t1 = mb.first_tile + mb.n_tiles;
                launch_range<C>(d, t0, P.dmb[g].path == 0 ? t1 : t0, t1, P.level_stage[mb.level] != 0,
                                P.level_nt[mb.level] != 0, st);
            }
    } else if (sched == BX_SCHED_LEVEL) {
        const bool ev = P.timing && !P.capturing;
        for (int l = 0; l < P.n_levels; ++l) {
            const int32_t t0 = P.level_tile_begin[l], t1 = P.level_tile_begin[l + 1];
            if (t1 <= t0) continue;
            if (ev) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.lev_ev[2 * l]), st));
            launch_range<C>(d, t0, P.level_row_begin[l], t1, P.level_stage[l] != 0, P.level_nt[l] != 0, st);
            if (ev) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.lev_ev[2 * l + 1]), st));
        }
    } else {
        return set_error(BX_E_UNSUPPORTED, "the dataflow schedule is disabled in this build");
    }
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

template <class C>
bx_status launch_value(Plan &P, void *ws, hipStream_t st) {
    VDescs d = make_vdescs(P, ws);
    hipLaunchKernelGGL(value_kernel<C>, dim3((unsigned)P.inst.size()), dim3(kValueThreads), 0, st, d);
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

template <class V>
void put(std::vector<uint8_t> &img, size_t off, const std::vector<V> &v) {
    if (!v.empty()) std::memcpy(img.data() + off, v.data(), v.size() * sizeof(V));
}

bx_status run(Plan &P, void *ws, bx_schedule sched, hipStream_t st) {
    bx_status s = P.ct == BX_COST_I32 ? launch_util<CostI>(P, ws, sched, st)
                                      : launch_util<CostF>(P, ws, sched, st);
    if (s != BX_OK) return s;
    if (P.timing && !P.capturing) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[1]), st));
    return P.ct == BX_COST_I32 ? launch_value<CostI>(P, ws, st) : launch_value<CostF>(P, ws, st);
}

bx_status ensure_events(Plan &P) {
    for (int i = 0; i < 3; ++i)
        if (!P.ev[i]) HIP_TRY(hipEventCreate(reinterpret_cast<hipEvent_t *>(&P.ev[i])));
    if (P.lev_ev.size() != 2 * (size_t)P.n_levels) {
        for (void *e : P.lev_ev) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
        P.lev_ev.assign(2 * (size_t)P.n_levels, nullptr);
        for (void *&e : P.lev_ev) HIP_TRY(hipEventCreate(reinterpret_cast<hipEvent_t *>(&e)));
    }
    return BX_OK;
}

// Per level, the tile goal (one of kTuneGoals) and the tiled kernel (with or
// without LDS staging) that ran the level fastest: minimum over reps of the
// level's own events, every combination timed on the whole level pass.  Then
// plain or non-temporal stores of the blocked rows for the whole pass,
// whichever ran it faster (the choice changes what the next level finds in
// the caches, so it is timed on whole passes, not per level).
bx_status tune_levels(Plan &P, void *ws, int32_t reps, hipStream_t st) {
    bx_status s = ensure_events(P);
    if (s != BX_OK) return s;
    std::vector<float> best(P.n_levels, 1e30f);
    std::vector<int32_t> goal(P.n_levels, kDefaultTilesGoal);
    std::vector<uint8_t> stage(P.n_levels, 1);
    const bool was_timing = P.timing;
    P.timing = true;
    for (int32_t g : kTuneGoals) {
        retile(P, g);
        s = dev_upload_tiles(P, ws, st);
        if (s != BX_OK) { P.timing = was_timing; return s; }
        std::fill(P.level_nt.begin(), P.level_nt.end(), (uint8_t)0);
        for (int pass = 0; pass < 2 * reps; ++pass) {
            const int v = pass & 1;
            std::fill(P.level_stage.begin(), P.level_stage.end(), (uint8_t)v);
            s = P.ct == BX_COST_I32 ? launch_util<CostI>(P, ws, BX_SCHED_LEVEL, st)
                                    : launch_util<CostF>(P, ws, BX_SCHED_LEVEL, st);
            if (s != BX_OK) { P.timing = was_timing; return s; }
            HIP_TRY(hipStreamSynchronize(st));
            for (int l = 0; l < P.n_levels; ++l) {
                if (P.level_tile_begin[l + 1] <= P.level_tile_begin[l]) continue;
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, static_cast<hipEvent_t>(P.lev_ev[2 * l]),
                                            static_cast<hipEvent_t>(P.lev_ev[2 * l + 1])));
                if (ms < best[l]) {
                    best[l] = ms;
                    goal[l] = g;
                    stage[l] = (uint8_t)v;
                }
            }
        }
    }
    P.timing = was_timing;
    P.level_goal = goal;
    P.level_stage = stage;
    retile_levels(P);
    s = dev_upload_tiles(P, ws, st);
    if (s != BX_OK) return s;
    float pass_ms[2] = {1e30f, 1e30f};
    hipEvent_t e0 = static_cast<hipEvent_t>(P.ev[0]), e1 = static_cast<hipEvent_t>(P.ev[2]);
    P.timing = false;
    for (int pass = 0; pass < 2 * reps; ++pass) {
        const int w = pass & 1;
        std::fill(P.level_nt.begin(), P.level_nt.end(), (uint8_t)w);
        HIP_TRY(hipEventRecord(e0, st));
        s = P.ct == BX_COST_I32 ? launch_util<CostI>(P, ws, BX_SCHED_LEVEL, st)
                                : launch_util<CostF>(P, ws, BX_SCHED_LEVEL, st);
        if (s != BX_OK) { P.timing = was_timing; return s; }
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        pass_ms[w] = std::min(pass_ms[w], ms);
    }
    P.timing = was_timing;
    std::fill(P.level_nt.begin(), P.level_nt.end(), (uint8_t)(pass_ms[1] < pass_ms[0] ? 1 : 0));
    return BX_OK;
}

}  // namespace

bx_status dev_upload(Plan &P, void *ws, size_t bytes, void *stream) {
    if (!ws) return set_error(BX_E_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return set_error(BX_E_INVALID, "workspace must be 256-byte aligned");
    if (bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    for (const PInst &I : P.inst)
        if (I.n > kSigmaCap) return set_error(BX_E_UNSUPPORTED, "more than 16384 variables in one problem");
    if (P.dtile.size() > P.tile_cap)
        return set_error(BX_E_INVALID, "internal: the tile list exceeds its workspace region");
    std::vector<uint8_t> img(P.static_bytes, 0);
    put(img, P.off_mb, P.dmb);
    put(img, P.off_fn, P.dfn);
    put(img, P.off_tile, P.dtile);
    put(img, P.off_var, P.dvar);
    put(img, P.off_vfn, P.dvfn);
    put(img, P.off_term, P.dterm);
    put(img, P.off_pair, P.dpair);
    put(img, P.off_vlv, P.vlevel_var_begin);
    put(img, P.off_vlp, P.vlevel_pair_begin);
    put(img, P.off_inst, P.dinst);
    put(img, P.off_const, P.dconst);
    put(img, P.off_tables, P.tables);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    P.executed = false;
    return BX_OK;
}

// Re-uploads only the tile list and the mini-bucket descriptors (after a retile).
bx_status dev_upload_tiles(Plan &P, void *ws, hipStream_t st) {
    if (P.dtile.size() > P.tile_cap)
        return set_error(BX_E_INVALID, "internal: the tile list exceeds its workspace region");
    char *w = static_cast<char *>(ws);
    HIP_TRY(hipMemcpyAsync(w + P.off_mb, P.dmb.data(), P.dmb.size() * sizeof(DevMb), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + P.off_fn, P.dfn.data(), P.dfn.size() * sizeof(DevFn), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + P.off_tile, P.dtile.data(), P.dtile.size() * sizeof(DevTile),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return BX_OK;
}

bx_status dev_execute(Plan &P, void *ws, size_t bytes, bx_schedule sched, void *stream) {
    if (!ws) return set_error(BX_E_INVALID, "workspace is NULL");
    if (bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (sched == BX_SCHED_AUTO) sched = P.tuned_valid ? P.tuned : BX_SCHED_LEVEL;
    if (sched == BX_SCHED_DATAFLOW)
        return set_error(BX_E_UNSUPPORTED, "the dataflow schedule is disabled in this build");
    const bool timed = P.timing && !P.capturing;
    if (timed) {
        bx_status es = ensure_events(P);
        if (es != BX_OK) return es;
        HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[0]), st));
    }
    bx_status s = run(P, ws, sched, st);
    if (s != BX_OK) return s;
    if (timed) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[2]), st));
    P.executed = true;
    P.timed_sched = timed ? sched : BX_SCHED_AUTO;
    return BX_OK;
}

bx_status dev_results(Plan &P, const void *ws, int32_t prob, double *bound, double *ub,
                      int32_t *assignment, void *stream) {
    if (!P.executed) return set_error(BX_E_STATE, "results requested before execute");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *w = static_cast<const char *>(ws);
    DevResult r{};
    HIP_TRY(hipMemcpyAsync(&r, w + P.off_results + sizeof(DevResult) * prob, sizeof r,
                           hipMemcpyDeviceToHost, st));
    const PInst &I = P.inst[prob];
    if (assignment && I.n > 0)
        HIP_TRY(hipMemcpyAsync(assignment, w + P.off_sigma + P.dinst[prob].sigma_off,
                               sizeof(int32_t) * I.n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (P.timed_sched != BX_SCHED_AUTO) {
        HIP_TRY(hipEventElapsedTime(&P.last_util_ms, static_cast<hipEvent_t>(P.ev[0]),
                                    static_cast<hipEvent_t>(P.ev[1])));
        HIP_TRY(hipEventElapsedTime(&P.last_value_ms, static_cast<hipEvent_t>(P.ev[1]),
                                    static_cast<hipEvent_t>(P.ev[2])));
        P.last_util_kernel_ms = P.last_util_ms;
        if (P.timed_sched == BX_SCHED_LEVEL) {
            float sum = 0.f;
            for (int l = 0; l < P.n_levels; ++l) {
                if (P.level_tile_begin[l + 1] <= P.level_tile_begin[l]) continue;
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, static_cast<hipEvent_t>(P.lev_ev[2 * l]),
                                            static_cast<hipEvent_t>(P.lev_ev[2 * l + 1])));
                sum += ms;
            }
            P.last_util_kernel_ms = sum;
        }
        P.timed_sched = BX_SCHED_AUTO;
    }
    if (r.status != 0) return set_error(BX_E_DEVICE, "device reported a failure");
    if (bound) *bound = r.bound;
    if (ub) *ub = r.ub;
    return BX_OK;
}

// Captures one execute (UTIL launches + value kernel) into a hipGraph bound
// to this workspace; dev_graph_launch replays it.  The captured kernels
// contain no memset nodes.
bx_status dev_graph_create(Plan &P, void *ws, size_t bytes, bx_schedule sched, void *stream) {
    if (!ws) return set_error(BX_E_INVALID, "workspace is NULL");
    if (bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    if (!stream) return set_error(BX_E_INVALID, "graph capture needs a non-null stream");
    if (sched == BX_SCHED_AUTO) sched = P.tuned_valid ? P.tuned : BX_SCHED_LEVEL;
    if (sched == BX_SCHED_DATAFLOW)
        return set_error(BX_E_UNSUPPORTED, "the dataflow schedule is disabled in this build");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (P.graph_exec) { (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(P.graph_exec)); P.graph_exec = nullptr; }
    if (P.graph) { (void)hipGraphDestroy(static_cast<hipGraph_t>(P.graph)); P.graph = nullptr; }
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    P.capturing = true;
    bx_status s = run(P, ws, sched, st);
    P.capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != BX_OK) { if (g) (void)hipGraphDestroy(g); return s; }
    if (e != hipSuccess) return set_error(BX_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return set_error(BX_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    P.graph = g;
    P.graph_exec = ge;
    P.graph_ws = ws;
    return BX_OK;
}

bx_status dev_graph_launch(Plan &P, void *stream) {
    if (!P.graph_exec) return set_error(BX_E_STATE, "no graph: call bx_plan_graph_create first");
    HIP_TRY(hipGraphLaunch(static_cast<hipGraphExec_t>(P.graph_exec), static_cast<hipStream_t>(stream)));
    P.executed = true;
    return BX_OK;
}

bx_status dev_copy_table(const Plan &P, const void *ws, int64_t off, int64_t n, void *host,
                         void *stream) {
    (void)P;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *w = static_cast<const char *>(ws);
    HIP_TRY(hipMemcpyAsync(host, w + off * 4, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return BX_OK;
}

// Times every (schedule, tile size) candidate on this plan and keeps the
// fastest for BX_SCHED_AUTO.  Results are cached by the plan's shape class.
bx_status dev_autotune(Plan &P, void *ws, size_t bytes, int32_t reps, void *stream) {
    if (!ws || bytes < P.total_bytes) return set_error(BX_E_INVALID, "workspace missing or too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (reps < 1) reps = 1;
    const bx_schedule best_sched = BX_SCHED_LEVEL;
    bx_status s = run(P, ws, best_sched, st);   // warm-up
    if (s == BX_OK) s = tune_levels(P, ws, reps + 1, st);
    if (s != BX_OK) return s;
    P.tuned = best_sched;
    P.tuned_valid = true;
    P.executed = true;
    return BX_OK;
}

void dev_release(Plan &P) {
    for (void *&e : P.ev)
        if (e) { (void)hipEventDestroy(static_cast<hipEvent_t>(e)); e = nullptr; }
    for (void *e : P.lev_ev) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    P.lev_ev.clear();
    if (P.graph_exec) { (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(P.graph_exec)); P.graph_exec = nullptr; }
    if (P.graph) { (void)hipGraphDestroy(static_cast<hipGraph_t>(P.graph)); P.graph = nullptr; }
}

}  // namespace bx
