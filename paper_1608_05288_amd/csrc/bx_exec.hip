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
// VALUE kernel: back-substitution of Alg. 1/2 (second loop) along value
// levels, then the bound (constants left after elimination) and the cost of
// the assignment over the input functions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

#include "bx_internal.h"

namespace bx {

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
};
struct CostF {
    using T = float;
    using A = float;
    __device__ static A zero() { return 0.f; }
    __device__ static A add(A a, T v) { return a + v; }
    __device__ static A add2(A a, A b) { return a + b; }
    __device__ static A mn(A a, A b) { return fminf(a, b); }
    __device__ static T fin(A a) { return a; }
};

struct Descs {
    const DevMb *mb;
    const DevFn *fn;
    const DevTile *tile;
    char *ws;
};

// ------------------------------------------------------------ row kernel
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
                int64_t base = fns[f].tab_off;
#pragma unroll
                for (int j = 0; j < kMaxVars; ++j)
                    if (j < nv) base += (int64_t)dig[j] * fns[f].stride[j];
#pragma unroll
                for (int x = 0; x < DT; ++x) acc[x] = C::add(acc[x], tab[base + x]);
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
                    int64_t base = fns[f].tab_off + x;
#pragma unroll
                    for (int j = 0; j < kMaxVars; ++j)
                        if (j < nv) base += (int64_t)dig[j] * fns[f].stride[j];
                    s = C::add(s, tab[base]);
                }
                best = x == 0 ? s : C::mn(best, s);
            }
            out[r] = C::fin(best);
        }
    }
}

template <class C>
__device__ __forceinline__ void run_row_tile(const Descs &d, const DevTile &t) {
    const DevMb &mb = d.mb[t.mb];
    switch (mb.D) {
    case 1: rows_tile<C, 1>(d, mb, t.begin, t.end); break;
    case 2: rows_tile<C, 2>(d, mb, t.begin, t.end); break;
    case 3: rows_tile<C, 3>(d, mb, t.begin, t.end); break;
    case 4: rows_tile<C, 4>(d, mb, t.begin, t.end); break;
    case 5: rows_tile<C, 5>(d, mb, t.begin, t.end); break;
    case 6: rows_tile<C, 6>(d, mb, t.begin, t.end); break;
    case 7: rows_tile<C, 7>(d, mb, t.begin, t.end); break;
    case 8: rows_tile<C, 8>(d, mb, t.begin, t.end); break;
    default: rows_tile<C, 0>(d, mb, t.begin, t.end); break;
    }
}

// A range of tiles, one workgroup each (PER_BUCKET and LEVEL schedules).
template <class C>
__global__ __launch_bounds__(256) void util_rows_kernel(Descs d, int32_t tile0) {
    const DevTile t = d.tile[tile0 + blockIdx.x];
    run_row_tile<C>(d, t);
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
    for (int s = I.lvl_begin; s < I.lvl_begin + I.n_lvl; ++s) {
        const int pb = d.vlp[s], pe = d.vlp[s + 1];
        for (int p = pb + tid; p < pe; p += blockDim.x) {
            const DevPair pr = d.pair[p];
            const DevVar dv = d.var[pr.var_entry];
            S c = 0;
            for (int f = dv.f_begin; f < dv.f_begin + dv.nf; ++f) {
                const DevVFn e = d.vfn[f];
                int64_t idx = e.tab_off + pr.x;
                for (int t = e.t_begin; t < e.t_begin + e.nt; ++t)
                    idx += (int64_t)sigma[d.term[2 * t]] * d.term[2 * t + 1];
                c = add(c, tab[idx]);
            }
            cost[p - pb] = cap(c);
        }
        __syncthreads();
        const int vb = d.vlv[s], ve = d.vlv[s + 1];
        for (int q = vb + tid; q < ve; q += blockDim.x) {
            const DevVar dv = d.var[q];
            const int o = dv.pair_begin - pb;
            S best = cost[o];
            int bx = 0;
            for (int x = 1; x < dv.D; ++x)
                if (cost[o + x] < best) { best = cost[o + x]; bx = x; }
            sigma[dv.var] = (uint16_t)bx;
        }
        __syncthreads();
    }
    int32_t *sig_out = reinterpret_cast<int32_t *>(d.sigma_base + I.sigma_off);
    for (int v = tid; v < I.n; v += blockDim.x) sig_out[v] = sigma[v];
    // cost of the assignment over the input functions
    S u = 0;
    for (int f = I.ub_begin + tid; f < I.ub_begin + I.ub_n; f += blockDim.x) {
        const DevVFn e = d.vfn[f];
        int64_t idx = e.tab_off;
        for (int t = e.t_begin; t < e.t_begin + e.nt; ++t)
            idx += (int64_t)sigma[d.term[2 * t]] * d.term[2 * t + 1];
        u = add(u, tab[idx]);
    }
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
            if constexpr (true) ub = ub + I.host_const;
            r.bound = b;
            r.ub = ub;
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
bx_status launch_util(Plan &P, void *ws, bx_schedule sched, hipStream_t st) {
    Descs d = make_descs(P, ws);
    if (sched == BX_SCHED_PER_BUCKET) {
        for (const PInst &I : P.inst)
            for (int32_t g : I.mbs) {
                const PMb &mb = P.mbs[g];
                if (mb.n_tiles == 0) continue;
                hipLaunchKernelGGL(util_rows_kernel<C>, dim3(mb.n_tiles), dim3(P.block), 0, st, d,
                                   mb.first_tile);
            }
    } else {
        for (int l = 0; l < P.n_levels; ++l) {
            int32_t t0 = P.level_tile_begin[l], t1 = P.level_tile_begin[l + 1];
            if (t1 > t0)
                hipLaunchKernelGGL(util_rows_kernel<C>, dim3(t1 - t0), dim3(P.block), 0, st, d, t0);
        }
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

}  // namespace

bx_status dev_upload(Plan &P, void *ws, size_t bytes, void *stream) {
    if (!ws) return set_error(BX_E_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return set_error(BX_E_INVALID, "workspace must be 256-byte aligned");
    if (bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    for (const PInst &I : P.inst)
        if (I.n > kSigmaCap) return set_error(BX_E_UNSUPPORTED, "more than 16384 variables in one problem");
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

bx_status dev_execute(Plan &P, void *ws, size_t bytes, bx_schedule sched, void *stream) {
    if (!ws) return set_error(BX_E_INVALID, "workspace is NULL");
    if (bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (sched == BX_SCHED_AUTO) sched = P.tuned_valid ? P.tuned : BX_SCHED_LEVEL;
    if (sched == BX_SCHED_DATAFLOW) sched = BX_SCHED_LEVEL;
    if (P.timing) {
        for (int i = 0; i < 3; ++i)
            if (!P.ev[i]) HIP_TRY(hipEventCreate(reinterpret_cast<hipEvent_t *>(&P.ev[i])));
        HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[0]), st));
    }
    bx_status s = P.ct == BX_COST_I32 ? launch_util<CostI>(P, ws, sched, st)
                                      : launch_util<CostF>(P, ws, sched, st);
    if (s != BX_OK) return s;
    if (P.timing) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[1]), st));
    s = P.ct == BX_COST_I32 ? launch_value<CostI>(P, ws, st) : launch_value<CostF>(P, ws, st);
    if (s != BX_OK) return s;
    if (P.timing) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[2]), st));
    P.executed = true;
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
    if (P.timing) {
        HIP_TRY(hipEventElapsedTime(&P.last_util_ms, static_cast<hipEvent_t>(P.ev[0]),
                                    static_cast<hipEvent_t>(P.ev[1])));
        HIP_TRY(hipEventElapsedTime(&P.last_value_ms, static_cast<hipEvent_t>(P.ev[1]),
                                    static_cast<hipEvent_t>(P.ev[2])));
    }
    if (r.status != 0) return set_error(BX_E_DEVICE, "device reported a failed dependency wait");
    if (bound) *bound = r.bound;
    if (ub) *ub = r.ub;
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

bx_status dev_autotune(Plan &P, void *ws, size_t bytes, int32_t reps, void *stream) {
    (void)ws; (void)bytes; (void)reps; (void)stream;
    P.tuned = BX_SCHED_LEVEL;
    P.tuned_valid = true;
    return BX_OK;
}

void dev_release(Plan &P) {
    for (void *&e : P.ev)
        if (e) { (void)hipEventDestroy(static_cast<hipEvent_t>(e)); e = nullptr; }
}

}  // namespace bx
