// Row-path UTIL kernel and the value kernel (both cost types), and the
// dispatch of the tiled-kernel launchers.
#include "bx_util_kernels.h"

namespace bx {
namespace {

// VALUE kernel: back-substitution of Alg. 1/2 (second loop) along value
// levels, then the bound (constants left after elimination) and the cost of
// the assignment over the input functions.
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
