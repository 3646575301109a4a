// UTIL kernels: for a mini-bucket with joint scope U = (u_0..u_{nv-1}, x),
// every output row s (an assignment of u_0..u_{nv-1}, row-major) gets
//     g[s] = min_{v in D_x} (+)_{f} f[ sum_j stride_f(u_j) * digit_j(s) + v ]
// i.e. the aggregation of Sec. 6.3 (Eq. (3): mixed-radix decode of the output
// row, re-encoded over each input table's scope) fused with the elimination
// of Sec. 6.4 (x is the last scope variable of every table, so its D entries
// are contiguous).  Nothing is materialised over the joint scope: each
// output row is written once, each table entry read from HBM/L2.
// (+) is the saturating int32 sum (infinity = INT32_MAX) or the float sum.
//
// Two code paths per tile:
//   tiled: row = o * p_in + r.  The decode of Eq. (3) is split in two: the
//          outer part of every table offset is computed once per outer index
//          (one thread each) into LDS, the inner part once per thread into
//          registers; functions that do not depend on the inner variables
//          are pre-summed per outer index (LDS).  The row loop is then one
//          LDS broadcast + one vector load of D entries per remaining function.
//   row:   full decode per row (any D, any number of functions).
//   lanes: D > 8, G lanes per row share the values of the eliminated
//          variable and reduce their minima by lane exchanges.
//   packed: small mini-buckets, one row per thread, rows of several
//          mini-buckets (and of a connected part of the bucket tree, stage
//          by stage) in one workgroup.
//
// Kernel templates only: the translation units bx_k_*.hip instantiate them.
#pragma once

#include "bx_device.h"

namespace bx {
namespace {

// ------------------------------------------------------------ row path
// One thread per output row, full mixed-radix decode per row (Eq. (3)),
// redone for every function (no per-row digit array: this path shares the
// kernel, and so the register budget, of the tiled path).  The eliminated
// domain is a template parameter so the D accumulators stay in registers;
// DT == 0 handles any D with a running minimum.
template <class C>
__device__ __forceinline__ int32_t row_offset(const DevMb &mb, const DevFn &fn, uint32_t r) {
    int32_t base = 0;
    for (int j = mb.nv - 1; j >= 0; --j) {
        const uint32_t dj = (uint32_t)mb.dims[j];
        const uint32_t q = r / dj;
        base += (int32_t)(r - q * dj) * fn.stride[j];
        r = q;
    }
    return base;
}

template <class C, int DT>
__device__ __forceinline__ void rows_tile(const Descs &d, const DevMb &mb, int64_t begin,
                                          int64_t end) {
    using T = typename C::T;
    using A = typename C::A;
    const T *tab = reinterpret_cast<const T *>(d.ws);
    T *out = reinterpret_cast<T *>(d.ws) + mb.out_off;
    const int nf = mb.nf;
    const DevFn *fns = d.fn + mb.f_begin;
    for (int64_t r = begin + threadIdx.x; r < end; r += blockDim.x) {
        if constexpr (DT > 0) {
            A acc[DT];
#pragma unroll
            for (int x = 0; x < DT; ++x) acc[x] = C::zero();
            for (int f = 0; f < nf; ++f) {
                T v[DT];
                const T *p = tab + fns[f].tab_off + row_offset<C>(mb, fns[f], (uint32_t)r);
#pragma unroll
                for (int x = 0; x < DT; ++x) v[x] = p[x];
#pragma unroll
                for (int x = 0; x < DT; ++x) acc[x] = C::add(acc[x], v[x]);
            }
            A best = acc[0];
#pragma unroll
            for (int x = 1; x < DT; ++x) best = C::mn(best, acc[x]);
            if constexpr (C::kSum)
                if (mb.red) best = soft_min(acc, best);
            out[r] = C::fin(best);
        } else {
            A best = C::ident();
            SoftAcc sa;
            for (int x = 0; x < mb.D; ++x) {
                A s = C::zero();
                for (int f = 0; f < nf; ++f)
                    s = C::add(s, tab[fns[f].tab_off + row_offset<C>(mb, fns[f], (uint32_t)r) + x]);
                best = C::mn(best, s);
                if constexpr (C::kSum) sa.add(s);
            }
            if constexpr (C::kSum)
                if (mb.red) best = sa.fin();
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
// index (in range) and store its value again.
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
    const bool sum = C::kSum && mb.red;   // sum-product elimination (uniform)
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
            if constexpr (C::kSum)
                if (sum) best[u] = soft_min(acc, best[u]);
        }
    };
    // a slot past the end holds the value of the tile's last outer index (at
    // this inner position) and writes it there again: every trip issues U
    // stores, so the wait for a trip's loads never includes the previous
    // trip's stores (a conditional store would give the compiler a path
    // without them and a wait for everything)
    auto store = [&](int ol0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ol = min(ol0 + u * Q, n_o - 1);
            *reinterpret_cast<T *>(ob + ((uint32_t)ol * pb + rb)) = C::fin(best[u]);
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
    const bool sum = C::kSum && mb.red;   // sum-product elimination (uniform)
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
                if constexpr (C::kSum)
                    if (sum) best[ia][b] = soft_min(acc, best[ia][b]);
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
    // domain of 2 or 3 re-reads its last value); b alone may have domain 5,
    // and D = 5 comes with b alone (the planner keeps to these shapes)
    if (mb.da == 1) {
        switch (mb.db) {
        case 2: blocked_rows<C, DT, 1, 2, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        case 3: blocked_rows<C, DT, 1, 3, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        case 4: blocked_rows<C, DT, 1, 4, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        default: blocked_rows<C, DT, 1, kBlockMaxDb1, kNT>(d, mb, fns, n_o, sm, dig, cv, qs, r); break;
        }
    } else if constexpr (DT <= kBlockMaxD2) {
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
    // variables; the digits of Eq. (3) are folded into the offsets as they
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

// ------------------------------------------------------------ lane-group path
// Eliminated domains above the tiled path's (D > 8): G lanes cooperate on
// one output row, lane j taking the values j, j + G, ... of the eliminated
// variable.  The row is decoded (Eq. (3)) once per lane, not once per value;
// each function's D consecutive entries are read by the G lanes together
// (consecutive addresses); the minimum over the group is a butterfly of lane
// exchanges.  Lanes past D keep the identity of the minimum.  Slots past the
// end of the tile decode the tile's last row (in range) and store nothing.
template <class C, int G>
__device__ __forceinline__ void lanes_tile(const Descs &d, const DevMb &mb, int64_t begin, int64_t end) {
    using T = typename C::T;
    using A = typename C::A;
    constexpr int R = kUtilThreads / G;   // rows per pass
    const T *tab = reinterpret_cast<const T *>(d.ws);
    T *out = reinterpret_cast<T *>(d.ws) + mb.out_off;
    const int nv = mb.nv, nf = mb.nf, D = mb.D;
    const DevFn *fns = d.fn + mb.f_begin;
    const int lane = (int)threadIdx.x % G;
    const int slot = (int)threadIdx.x / G;
    for (int64_t r0 = begin; r0 < end; r0 += R) {
        const int64_t r = r0 + slot;
        uint32_t rem = (uint32_t)(r < end ? r : end - 1);
        int32_t base[kLaneMaxFns];
#pragma unroll
        for (int f = 0; f < kLaneMaxFns; ++f) base[f] = 0;
        for (int j = nv - 1; j >= 0; --j) {
            const uint32_t dj = (uint32_t)mb.dims[j];
            const uint32_t q = rem / dj;
            const int32_t dg = (int32_t)(rem - q * dj);
            rem = q;
#pragma unroll
            for (int f = 0; f < kLaneMaxFns; ++f)
                if (f < nf) base[f] += dg * fns[f].stride[j];
        }
        A best = C::ident();
        SoftAcc sa;
        for (int x = lane; x < D; x += G) {
            A s = C::zero();
#pragma unroll
            for (int f = 0; f < kLaneMaxFns; ++f)
                if (f < nf) s = C::add(s, tab[fns[f].tab_off + base[f] + x]);
            best = C::mn(best, s);
            if constexpr (C::kSum) sa.add(s);
        }
        if constexpr (C::kSum) {
            if (mb.red) {   // sum-product: lanes exchange (least value, scaled sum) pairs
#pragma unroll
                for (int m = G / 2; m > 0; m >>= 1)
                    sa.merge(__shfl_xor(sa.m, m, G), __shfl_xor(sa.s, m, G));
                best = sa.fin();
            }
        }
        if (!(C::kSum && mb.red)) {
#pragma unroll
            for (int m = G / 2; m > 0; m >>= 1)
                best = C::mn(best, C::from_bits((uint32_t)__shfl_xor((int)C::bits(best), m, G)));
        }
        if (r < end && lane == 0) out[r] = C::fin(best);
    }
}

// Tiles of the lane-group path, one workgroup each.
template <class C>
__global__ __launch_bounds__(kUtilThreads) void util_lanes_kernel(Descs d, int32_t tile0) {
    const DevTile t = d.tile[tile0 + blockIdx.x];
    const DevMb &mb = d.mb[t.mb];
    switch (mb.lanes) {
    case 8: lanes_tile<C, 8>(d, mb, t.begin, t.end); break;
    case 16: lanes_tile<C, 16>(d, mb, t.begin, t.end); break;
    case 32: lanes_tile<C, 32>(d, mb, t.begin, t.end); break;
    default: lanes_tile<C, 64>(d, mb, t.begin, t.end); break;
    }
}


// ------------------------------------------------------------ packed path
// One output row r of a packed mini-bucket, from its descriptor record in
// LDS: the mixed-radix decode of Eq. (3) folded into every function's offset
// (right-aligned dims and strides, so every slot is decoded alike), then the
// values of the eliminated variable XB at a time: the loads of all functions
// for those values are issued together (absent functions and values past D
// read the workspace's zero block instead, so nothing branches), and the
// minimum is taken over the D real values.
template <class C>
__device__ __forceinline__ void pack_row(const Descs &d, const DevSeg &sg, uint32_t r) {
    using T = typename C::T;
    using A = typename C::A;
    constexpr int XB = 4;
    const int nf = sg.nf, D = sg.D;
    const T *tab = reinterpret_cast<const T *>(d.ws);
    const T *zero = reinterpret_cast<const T *>(d.zeros);
    int32_t base[kPackMaxFns];
#pragma unroll
    for (int f = 0; f < kPackMaxFns; ++f) base[f] = 0;
    // the row's digits, fastest slot first, over the nv slots in use (the
    // leading ones have dim 1, stride 0).  r < kPackRowLimit = 2^16: the
    // quotient from a single-precision reciprocal is off by at most one
    // (relative error below 2^-21 on a value below 2^16), and one
    // correction step each way makes it exact
    uint32_t rem = r;
    const int nv = sg.nv;
#pragma unroll
    for (int j = kPackMaxVars - 1; j >= 0; --j) {
        if (j >= kPackMaxVars - nv) {
            const uint32_t dj = sg.dims[j];
            uint32_t q = (uint32_t)((float)rem * __builtin_amdgcn_rcpf((float)dj));
            int32_t dg = (int32_t)rem - (int32_t)(q * dj);
            if (dg < 0) { --q; dg += (int32_t)dj; }
            if (dg >= (int32_t)dj) { ++q; dg -= (int32_t)dj; }
            rem = q;
#pragma unroll
            for (int f = 0; f < kPackMaxFns; ++f) base[f] += dg * (int32_t)sg.stride[f][j];
        }
    }
    const T *tp[kPackMaxFns];
#pragma unroll
    for (int f = 0; f < kPackMaxFns; ++f) tp[f] = tab + sg.tab_off[f] + base[f];
    A best = C::ident();
    SoftAcc sa;
    for (int x0 = 0; x0 < D; x0 += XB) {
        T v[kPackMaxFns][XB];
#pragma unroll
        for (int f = 0; f < kPackMaxFns; ++f)
#pragma unroll
            for (int x = 0; x < XB; ++x) v[f][x] = *((f < nf && x0 + x < D) ? tp[f] + (x0 + x) : zero);
        // every load of the chunk is issued before any of them is used
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int x = 0; x < XB; ++x) {
            A s = C::zero();
#pragma unroll
            for (int f = 0; f < kPackMaxFns; ++f) s = C::add(s, v[f][x]);
            best = C::mn(best, x0 + x < D ? s : C::ident());
            if constexpr (C::kSum)
                if (x0 + x < D) sa.add(s);
        }
    }
    if constexpr (C::kSum)
        if (sg.red) best = sa.fin();
    reinterpret_cast<T *>(d.ws)[sg.out_off + r] = C::fin(best);
}

// A packed tile.  Its descriptor records (at most kPackMaxSegs) are copied to
// LDS (`seg`, the workgroup's LDS reused) first; then stage by stage, thread
// t takes the stage's rows t, t + 256, ...; a row belongs to the last record
// of the stage starting at or before it (binary search in LDS).  A
// workgroup barrier separates the stages: a later stage reads what an
// earlier one wrote, and every wave of a workgroup runs on one compute
// unit, behind one vector L1 cache.
template <class C>
__device__ __forceinline__ void pack_tile(const Descs &d, const DevTile &t, DevSeg *seg) {
    const int32_t s0 = (int32_t)t.begin;
    const int32_t nseg = min((int32_t)(t.end - t.begin), kPackMaxSegs);   // the planner keeps it within
    {
        constexpr int W = (int)(sizeof(DevSeg) / sizeof(int4));
        const int4 *src = reinterpret_cast<const int4 *>(d.seg + s0);
        int4 *dst = reinterpret_cast<int4 *>(seg);
        for (int32_t k = (int32_t)threadIdx.x; k < nseg * W; k += kUtilThreads) dst[k] = src[k];
    }
    __syncthreads();
    int32_t s = 0;
    while (s < nseg) {
        const int32_t n = seg[s].stage_segs, total = seg[s].stage_rows;
        for (int32_t p = (int32_t)threadIdx.x; p < total; p += kUtilThreads) {
            int32_t lo = s, hi = s + n - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (seg[mid].first <= p) lo = mid;
                else hi = mid - 1;
            }
            pack_row<C>(d, seg[lo], (uint32_t)(p - seg[lo].first));
        }
        s += n;
        if (s < nseg) __syncthreads();
    }
}


// Descriptor warm-up, run by the kWarmBlocks workgroups after a launch's tiles
// (workgroup b runs on XCD b % 8): the tile, mini-bucket and function
// descriptors (or packed records) of the next launch's tiles that will run on
// this XCD are loaded once, so that the next launch finds them in this XCD's
// L2 instead of HBM -- its first steps are a chain of dependent descriptor
// loads, which is most of a small level's time.  One word of each 128-byte
// line is enough; the loads feed a value stored only if it equals a constant
// (so that they are kept).
__device__ __forceinline__ void warm_descriptors(const Descs &d, int32_t x) {
    int32_t j0 = x + 8 * (int32_t)threadIdx.x, step = 8 * kUtilThreads, j1 = d.pf_n;
    if (d.pf_xcd) {   // XCD x takes the x-th contiguous part of the next launch's tiles
        int32_t start = 0;
        for (int32_t y = 0; y < x; ++y) start += (d.pf_n - y + 7) >> 3;
        j0 = start + (int32_t)threadIdx.x;
        step = kUtilThreads;
        j1 = start + ((d.pf_n - x + 7) >> 3);
    }
    uint32_t acc = 0;
    for (int32_t j = j0; j < j1; j += step) {
        const DevTile t = d.tile[d.pf_t0 + j];
        acc ^= (uint32_t)t.begin;
        if (t.mb >= 0) {
            const int32_t *m = reinterpret_cast<const int32_t *>(d.mb + t.mb);
            acc ^= (uint32_t)(m[0] ^ m[32] ^ m[64]);
            const int32_t fb = d.mb[t.mb].f_begin, nf = d.mb[t.mb].nf;
            for (int32_t f = 0; f < nf; ++f) {
                const int32_t *w = reinterpret_cast<const int32_t *>(d.fn + fb + f);
                acc ^= (uint32_t)(w[0] ^ w[32]);
            }
        } else {
            for (int64_t s = t.begin; s < t.end; ++s) {
                const int32_t *w = reinterpret_cast<const int32_t *>(d.seg + s);
                acc ^= (uint32_t)(w[0] ^ w[32]);
            }
        }
    }
    if (acc == 0x9e3779b9u) d.sink[0] = (int32_t)acc;
}
static_assert(sizeof(DevMb) >= 65 * 4 && sizeof(DevFn) >= 33 * 4 && sizeof(DevSeg) >= 33 * 4,
              "warm-up reads stay inside the descriptors");

// One launch per level runs the level's tiles, each workgroup on the path its
// tile names: packed tiles (mb < 0), the tiled path and the row path (also
// the per-bucket tiles of packed mini-buckets).  One launch instead of one
// per path: kernels of one stream run one after another, so a level with
// several paths would wait for each in turn.  (Lane-group tiles, D > 8, have
// a kernel of their own: their registers would spill the tiled path's.)  At
// least 5 waves per SIMD (<= 102 VGPRs): with 6 (<= 80) the compiler spilled
// inside the register-blocked loop, and a spill reload there is a vector
// memory load like any other -- waiting for it waits for every store issued
// before it.  kStage: the variant with LDS staging of lane tables; kNT:
// blocked rows stored non-temporally.
template <class C, bool kStage, bool kNT>
__global__ __launch_bounds__(kUtilThreads, 5) void util_tiles_kernel(Descs d, int32_t tile0) {
    __shared__ TileSmem<kStage> sm;
    static_assert(sizeof(TileSmem<kStage>) >= sizeof(DevSeg) * kPackMaxSegs, "packed tiles reuse the LDS");
    int32_t ti = (int32_t)blockIdx.x;
    const int32_t n_own = (int32_t)gridDim.x - d.pf_extra;   // the launch's own tiles
    if (ti >= n_own) {
        warm_descriptors(d, ti & 7);
        return;
    }
    if (d.xcd) {   // XCD x = b % 8 takes the x-th contiguous part of the tiles
        const int32_t n = n_own, x = ti & 7;
        int32_t start = 0;
        for (int32_t y = 0; y < x; ++y) start += (n - y + 7) >> 3;
        ti = start + (ti >> 3);
    }
    const DevTile t = d.tile[tile0 + ti];
    if (t.mb < 0) {
        pack_tile<C>(d, t, reinterpret_cast<DevSeg *>(&sm));
        return;
    }
    const DevMb &mb = d.mb[t.mb];
    if (mb.path == 1 || mb.path == 3) {
        run_rows<C>(d, mb, t.begin, t.end);
        return;
    }
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

}  // namespace
}  // namespace bx
