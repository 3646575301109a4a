// Row-path UTIL kernel and the value kernel (both cost types), and the
// dispatch of the tiled-kernel launchers.
#include "bx_util_kernels.h"

namespace bx {
namespace {

// Copies n elements from global memory to LDS with eight loads in flight per
// thread (a plain strided loop waits for each load before the next).
template <class E>
__device__ inline void stage_copy(E *dst, const E *src, int n) {
    const int B = blockDim.x;
    int i = threadIdx.x;
    for (; i + 7 * B < n; i += 8 * B) {
        E a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = src[i + u * B];
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[i + u * B] = a[u];
    }
    for (; i < n; i += B) dst[i] = src[i];
}

// comparison type of the value kernel: sums of FP32 costs in double,
// saturating sums of integer costs in uint32
template <class C>
using ValueSum = typename std::conditional<std::is_same<typename C::T, float>::value, double, uint32_t>::type;

// VALUE kernel: back-substitution of Alg. 1/2 (second loop) along value
// levels, then the bound (constants left after elimination) and the cost of
// the assignment over the input functions.  One workgroup per problem.
//
// Nothing but the table entries depends on the assignment, so the problem's
// value levels, variable and candidate-value descriptors (kLv) and function
// descriptors with the occurrences of each variable in them (kFn) are copied
// to LDS first when they fit the arena.  A value level is then two steps:
// each candidate value sums its functions' entries (one thread per
// candidate, one round trip to the tables), and each variable takes its
// first minimum.  With the function data in LDS, a function's entry offset
// is kept up to date instead of recomputed: the lanes that pick a
// variable's value add value x stride into every function that has the
// variable in its scope (LDS atomics: variables of one level share
// functions), and a function is read only after all of its scope but its
// bucket variable has a value.  Without it, each lookup sums its
// (variable, stride) terms from HBM.
template <class C, bool kLv, bool kFn>
__device__ void value_body(const VDescs &d, const DevInst &I, uint4 *arena, ValueSum<C> *cost, ValueSum<C> *red) {
    using T = typename C::T;
    constexpr bool kF = std::is_same<T, float>::value;
    using S = ValueSum<C>;
    const T *tab = reinterpret_cast<const T *>(d.ws);
    const int tid = threadIdx.x;
    const int2 *terms_g = reinterpret_cast<const int2 *>(d.term);
    // arena layout, 16-byte sections: sigma | level bounds | vars | pairs | vfns | occurrences
    char *a = reinterpret_cast<char *>(arena);
    uint16_t *sigma = reinterpret_cast<uint16_t *>(a);
    a += ((int64_t)I.n * 2 + 15) / 16 * 16;
    // var bounds and pair bounds of the levels (n_lvl + 1 each)
    int32_t *lv_l = reinterpret_cast<int32_t *>(a);
    DevVar *var_l = reinterpret_cast<DevVar *>(a + (kLv ? ((int64_t)(I.n_lvl + 1) * 8 + 15) / 16 * 16 : 0));
    DevPair *pair_l = reinterpret_cast<DevPair *>(var_l + (kLv ? I.var_n : 0));
    DevVFn *vfn_l = reinterpret_cast<DevVFn *>(pair_l + (kLv ? I.pair_n : 0));
    int2 *occ_l = reinterpret_cast<int2 *>(vfn_l + (kFn ? I.vfn_n : 0));
    for (int v = tid; v < I.n; v += blockDim.x) sigma[v] = 0;
    if constexpr (kLv) {
        for (int i = tid; i <= I.n_lvl; i += blockDim.x) {
            lv_l[i] = d.vlv[I.lvl_begin + i];
            lv_l[I.n_lvl + 1 + i] = d.vlp[I.lvl_begin + i];
        }
        stage_copy(reinterpret_cast<uint4 *>(var_l), reinterpret_cast<const uint4 *>(d.var + I.var_begin),
                   I.var_n * (int)(sizeof(DevVar) / 16));
        stage_copy(reinterpret_cast<uint4 *>(pair_l), reinterpret_cast<const uint4 *>(d.pair + I.pair_begin),
                   I.pair_n * (int)(sizeof(DevPair) / 16));
    }
    if constexpr (kFn) {
        // every offset starts at its table's first entry (all digits 0)
        stage_copy(reinterpret_cast<uint4 *>(vfn_l), reinterpret_cast<const uint4 *>(d.vfn + I.vfn_begin),
                   I.vfn_n * (int)(sizeof(DevVFn) / 16));
        stage_copy(occ_l, reinterpret_cast<const int2 *>(d.occ) + I.occ_begin, I.occ_n);
    }
    __syncthreads();
    auto add = [](S x, T v) -> S {
        if constexpr (kF) return x + (double)v;
        else return __builtin_elementwise_add_sat(x, (uint32_t)v);
    };
    auto cap = [](S x) -> S {
        if constexpr (kF) return x;
        else return x < (uint32_t)kInfI32 ? x : (uint32_t)kInfI32;
    };
    auto var_at = [&](int q) -> DevVar {
        if constexpr (kLv) return var_l[q - I.var_begin];
        else return d.var[q];
    };
    auto pair_at = [&](int p) -> DevPair {
        if constexpr (kLv) return pair_l[p - I.pair_begin];
        else return d.pair[p];
    };
    // entry offset of function f (global index) under the current assignment,
    // the bucket variable at 0
    auto offset_of = [&](int f) -> int64_t {
        if constexpr (kFn) {
            return vfn_l[f - I.vfn_begin].tab_off;
        } else {
            // terms four at a time, the last group padded with repeats of its
            // last term that add nothing
            const DevVFn e = d.vfn[f];
            int64_t idx = e.tab_off;
            const int te = e.t_begin + e.nt;
            for (int t = e.t_begin; t < te; t += 4) {
                const int l = te - 1;
                const int2 p0 = terms_g[t], p1 = terms_g[min(t + 1, l)], p2 = terms_g[min(t + 2, l)],
                           p3 = terms_g[min(t + 3, l)];
                const int64_t s0 = sigma[p0.x], s1 = sigma[p1.x], s2 = sigma[p2.x], s3 = sigma[p3.x];
                idx += s0 * p0.y + (t + 1 < te ? s1 * p1.y : 0) + (t + 2 < te ? s2 * p2.y : 0) +
                       (t + 3 < te ? s3 * p3.y : 0);
            }
            return idx;
        }
    };
    for (int s = 0; s < I.n_lvl; ++s) {
        int pb, pe, vb, ve;
        if constexpr (kLv) {
            vb = lv_l[s]; ve = lv_l[s + 1];
            pb = lv_l[I.n_lvl + 1 + s]; pe = lv_l[I.n_lvl + 2 + s];
        } else {
            vb = d.vlv[I.lvl_begin + s]; ve = d.vlv[I.lvl_begin + s + 1];
            pb = d.vlp[I.lvl_begin + s]; pe = d.vlp[I.lvl_begin + s + 1];
        }
        for (int p = pb + tid; p < pe; p += blockDim.x) {
            const DevPair pr = pair_at(p);
            S c = 0;
            const int fe = pr.f_begin + pr.nf;
            // four functions at a time, the last group padded with repeats of
            // its last function (looked up, not added): the lookups of a group
            // are independent, so their table loads are in flight together
            for (int f = pr.f_begin; f < fe; f += 4) {
                const int l = fe - 1;
                const T v0 = tab[offset_of(f) + pr.x], v1 = tab[offset_of(min(f + 1, l)) + pr.x],
                        v2 = tab[offset_of(min(f + 2, l)) + pr.x], v3 = tab[offset_of(min(f + 3, l)) + pr.x];
                c = add(c, v0);
                if (f + 1 < fe) c = add(c, v1);
                if (f + 2 < fe) c = add(c, v2);
                if (f + 3 < fe) c = add(c, v3);
            }
            cost[p - pb] = cap(c);
        }
        __syncthreads();
        // argmin step: G lanes per variable (as many as the level leaves,
        // up to a wave) each take the same first minimum; one writes the
        // value, and with the function data in LDS the G lanes share the
        // variable's occurrences (a zero digit adds nothing)
        const int nv = ve - vb;
        int lg = 0;
        while (lg < 6 && (nv << (lg + 1)) <= (int)blockDim.x) ++lg;
        const int G = 1 << lg;
        for (int t = tid; t < (nv << lg); t += blockDim.x) {
            const DevVar dv = var_at(vb + (t >> lg));
            const int j = t & (G - 1);
            const int o = dv.pair_begin - pb;
            S best = cost[o];
            int bx = 0;
            for (int x = 1; x < dv.D; ++x)
                if (cost[o + x] < best) { best = cost[o + x]; bx = x; }
            if (j == 0) sigma[dv.var] = (uint16_t)bx;
            if constexpr (kFn) {
                if (bx != 0) {
                    const int oe = dv.occ_begin + dv.occ_n;
                    for (int k = dv.occ_begin + j; k < oe; k += G) {
                        const int2 oc = occ_l[k - I.occ_begin];
                        atomicAdd(reinterpret_cast<unsigned long long *>(&vfn_l[oc.x].tab_off),
                                  (unsigned long long)((int64_t)bx * oc.y));
                    }
                }
            }
        }
        __syncthreads();
    }
    // cost of the assignment over the input functions
    // (four functions per thread at a time, as above)
    S u = 0;
    const int ube = I.ub_begin + I.ub_n, B = blockDim.x;
    for (int f = I.ub_begin + tid; f < ube; f += 4 * B) {
        const int f1 = f + B < ube ? f + B : f, f2 = f + 2 * B < ube ? f + 2 * B : f,
                  f3 = f + 3 * B < ube ? f + 3 * B : f;
        const T v0 = tab[offset_of(f)], v1 = tab[offset_of(f1)], v2 = tab[offset_of(f2)], v3 = tab[offset_of(f3)];
        u = add(u, v0);
        if (f1 != f) u = add(u, v1);
        if (f2 != f) u = add(u, v2);
        if (f3 != f) u = add(u, v3);
    }
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
        if constexpr (kF) b = I.host_const + I.bound_const;
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

template <class C>
__global__ __launch_bounds__(kValueThreads) void value_kernel(VDescs d) {
    using S = ValueSum<C>;
    __shared__ uint4 arena[kValueArenaBytes / 16];
    __shared__ S cost[kPairCap];
    __shared__ S red[kValueThreads];
    const DevInst I = d.inst[blockIdx.x];
    const int64_t sig = ((int64_t)I.n * 2 + 15) / 16 * 16;
    const int64_t lvb = ((int64_t)(I.n_lvl + 1) * 8 + 15) / 16 * 16 + (int64_t)I.var_n * sizeof(DevVar) +
                        (int64_t)I.pair_n * sizeof(DevPair);
    const int64_t fnb = (int64_t)I.vfn_n * sizeof(DevVFn) + ((int64_t)I.occ_n * 8 + 15) / 16 * 16;
    // the function data is the larger and the more often read: it goes first
    const bool fn = sig + fnb <= kValueArenaBytes;
    const bool lv = sig + (fn ? fnb : 0) + lvb <= kValueArenaBytes;
    if (fn && lv) value_body<C, true, true>(d, I, arena, cost, red);
    else if (fn) value_body<C, false, true>(d, I, arena, cost, red);
    else if (lv) value_body<C, true, false>(d, I, arena, cost, red);
    else value_body<C, false, false>(d, I, arena, cost, red);
}

// Bandwidth references for the roofline of the UTIL kernels: a streaming
// copy, a streaming write and a streaming read (sum into one word per
// workgroup) of 16-byte vectors, grid-stride over the whole buffer.
__global__ __launch_bounds__(256) void stream_copy_kernel(int4 *__restrict__ dst, const int4 *__restrict__ src,
                                                          int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void stream_write_kernel(int4 *__restrict__ dst, int64_t n, int32_t v) {
    const int4 w = make_int4(v, v + 1, v + 2, v + 3);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = w;
}

__global__ __launch_bounds__(256) void stream_read_kernel(const int4 *__restrict__ src, int64_t n,
                                                          int32_t *__restrict__ out) {
    int32_t acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int4 w = src[i];
        acc ^= w.x ^ w.y ^ w.z ^ w.w;
    }
    __shared__ int32_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] ^= red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace

// kind 0: copy src -> dst; 1: write dst; 2: read src (one int32 per
// workgroup into dst).  n16: 16-byte vectors; grid: workgroups.
void launch_stream(int kind, void *dst, const void *src, int64_t n16, int32_t grid, hipStream_t st) {
    if (kind == 0)
        hipLaunchKernelGGL(stream_copy_kernel, dim3(grid), dim3(256), 0, st, static_cast<int4 *>(dst),
                           static_cast<const int4 *>(src), n16);
    else if (kind == 1)
        hipLaunchKernelGGL(stream_write_kernel, dim3(grid), dim3(256), 0, st, static_cast<int4 *>(dst), n16, 7);
    else
        hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(256), 0, st, static_cast<const int4 *>(src), n16,
                           static_cast<int32_t *>(dst));
}

void launch_tiles_i32(const Descs &d, int32_t t0, int32_t n, bool stage, bool nt, hipStream_t st) {
    if (stage) launch_tiles_i32_s1(d, t0, n, nt, st);
    else launch_tiles_i32_s0(d, t0, n, nt, st);
}

void launch_tiles_fs(const Descs &d, int32_t t0, int32_t n, bool stage, bool nt, hipStream_t st) {
    if (stage) launch_tiles_fs_s1(d, t0, n, nt, st);
    else launch_tiles_fs_s0(d, t0, n, nt, st);
}

void launch_lanes_fs(const Descs &d, int32_t t0, int32_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(util_lanes_kernel<CostFS>, dim3(n), dim3(kUtilThreads), 0, st, d, t0);
}

void launch_tiles_f32(const Descs &d, int32_t t0, int32_t n, bool stage, bool nt, hipStream_t st) {
    if (stage) launch_tiles_f32_s1(d, t0, n, nt, st);
    else launch_tiles_f32_s0(d, t0, n, nt, st);
}

void launch_lanes_i32(const Descs &d, int32_t t0, int32_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(util_lanes_kernel<CostI>, dim3(n), dim3(kUtilThreads), 0, st, d, t0);
}

void launch_lanes_f32(const Descs &d, int32_t t0, int32_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(util_lanes_kernel<CostF>, dim3(n), dim3(kUtilThreads), 0, st, d, t0);
}

void launch_value_i32(const VDescs &d, int32_t n_inst, hipStream_t st) {
    hipLaunchKernelGGL(value_kernel<CostI>, dim3((unsigned)n_inst), dim3(kValueThreads), 0, st, d);
}

void launch_value_f32(const VDescs &d, int32_t n_inst, hipStream_t st) {
    hipLaunchKernelGGL(value_kernel<CostF>, dim3((unsigned)n_inst), dim3(kValueThreads), 0, st, d);
}

}  // namespace bx
