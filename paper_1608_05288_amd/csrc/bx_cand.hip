// Candidate values: a sampled estimate, on the tables of an executed plan, of
// what each recorded partition candidate of an over-full bucket would
// contribute to the mini-bucket bound.
//
// The partition step of Alg. 2 replaces min_x sum_{f in B} f by
// sum_k min_x sum_{f in Q_k} f over the parts Q_k; the second never exceeds
// the first (Sec. 2.2), and the larger it is the less the bound loses at this
// bucket.  For decision d with bucket variables u (other than the eliminated
// x) and candidate c, the pass computes
//     value[c] = (1/S) sum_{s<S} sum_k min_x sum_{f in Q_k(c)} f(u = s, x)
// with the digit of variable u in sample s taken as rnd[d][s][slot(u)] mod
// |D_u|, slot(u) = rank of u among the bucket variables in increasing id.
// Integer costs add with saturation at INF (Sec. 2), the sum over the parts
// included, and enter the mean as their int32 value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>

#include "bx_internal.h"

namespace bx {

namespace {

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return set_error(BX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kCandThreads = 256;

struct CDescs {
    const DevCDec *dec;
    const DevCFn *fn;
    const int32_t *term;     // (slot, stride) pairs
    const int32_t *dom;      // domain size per slot
    const uint8_t *part;     // part of each function, per candidate
    const uint32_t *rnd;     // [decision][sample][kCandSlots]
    const char *ws;
    double *out;
    int32_t samples;
};

template <bool kInt>
__global__ __launch_bounds__(kCandThreads) void cand_values_kernel(CDescs d) {
    using T = typename std::conditional<kInt, int32_t, float>::type;
    const DevCDec dec = d.dec[blockIdx.x];
    if (!dec.valid) {                            // unsupported bucket: NaN values
        if ((int)threadIdx.x < dec.ncand) d.out[dec.out_begin + threadIdx.x] = __builtin_nan("");
        return;
    }
    __shared__ double red[kCandThreads];
    __shared__ uint32_t dig[kCandThreads][kCandSlots + 1];
    const T *tab = reinterpret_cast<const T *>(d.ws);
    const int tid = threadIdx.x;
    for (int c = 0; c < dec.ncand; ++c) {
        const uint8_t *pc = d.part + dec.part_begin + (int64_t)c * dec.nfn;
        int np = 0;
        for (int f = 0; f < dec.nfn; ++f) np = max(np, (int)pc[f] + 1);
        double acc = 0.0;
        for (int s = tid; s < d.samples; s += kCandThreads) {
            const uint32_t *rs = d.rnd + ((int64_t)blockIdx.x * d.samples + s) * kCandSlots;
            for (int j = 0; j < dec.nslot; ++j) dig[tid][j] = rs[j] % (uint32_t)d.dom[dec.slot_begin + j];
            double tot = 0.0;
            for (int k = 0; k < np; ++k) {
                typename std::conditional<kInt, uint32_t, float>::type a[kCandMaxD];
#pragma unroll
                for (int x = 0; x < kCandMaxD; ++x) a[x] = 0;
                for (int f = 0; f < dec.nfn; ++f) {
                    if (pc[f] != k) continue;
                    const DevCFn fn = d.fn[dec.fn_begin + f];
                    int64_t off = fn.tab_off;
                    for (int t = 0; t < fn.nterm; ++t)
                        off += (int64_t)dig[tid][d.term[2 * (fn.term_begin + t)]] * d.term[2 * (fn.term_begin + t) + 1];
#pragma unroll
                    for (int x = 0; x < kCandMaxD; ++x) {
                        if (x < dec.D) {
                            if constexpr (kInt)
                                a[x] = __builtin_elementwise_add_sat(a[x], (uint32_t)tab[off + x]);
                            else
                                a[x] += tab[off + x];
                        }
                    }
                }
                auto best = a[0];
#pragma unroll
                for (int x = 1; x < kCandMaxD; ++x)
                    if (x < dec.D) best = a[x] < best ? a[x] : best;
                if constexpr (kInt)
                    tot += (double)(best < (uint32_t)kInfI32 ? best : (uint32_t)kInfI32);
                else
                    tot += (double)best;
            }
            if constexpr (kInt) tot = tot < (double)kInfI32 ? tot : (double)kInfI32;
            acc += tot;
        }
        red[tid] = acc;
        __syncthreads();
        for (int w = kCandThreads / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) d.out[dec.out_begin + c] = red[0] / (double)d.samples;
        __syncthreads();
    }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// host image: DevCDec[n_dec] | DevCFn[...] | terms | doms | parts
struct CandLayout {
    size_t off_dec, off_fn, off_term, off_dom, off_part, total;
};

CandLayout build_cand_image(const Plan &P, std::vector<uint8_t> &image) {
    std::vector<DevCDec> dec;
    std::vector<DevCFn> fns;
    std::vector<int32_t> term, dom;
    std::vector<uint8_t> part;
    int64_t out = 0;
    for (const Decision &D : P.decisions) {
        const PInst &I = P.inst[D.inst];
        DevCDec e{};
        e.D = I.dom[D.var];
        e.nfn = (int32_t)D.B.size();
        e.fn_begin = (int32_t)fns.size();
        e.slot_begin = (int32_t)dom.size();
        e.ncand = (int32_t)D.cands.size();
        e.part_begin = (int32_t)part.size();
        e.out_begin = (int32_t)out;
        out += e.ncand;
        // bucket variables other than the eliminated one, increasing id
        std::vector<int32_t> vars;
        for (int32_t id : D.B)
            for (int32_t u : I.fns[id].scope)
                if (u != D.var) vars.push_back(u);
        std::sort(vars.begin(), vars.end());
        vars.erase(std::unique(vars.begin(), vars.end()), vars.end());
        e.nslot = (int32_t)vars.size();
        e.valid = e.D <= kCandMaxD && e.nfn <= kCandMaxFns && e.nslot <= kCandSlots;
        if (e.valid) {
            for (int32_t u : vars) dom.push_back(I.dom[u]);
            for (int32_t id : D.B) {
                const PFn &f = I.fns[id];
                DevCFn cf{};
                cf.tab_off = f.off;
                cf.term_begin = (int32_t)(term.size() / 2);
                // row-major over f.scope, the eliminated variable last (stride 1)
                int64_t st = 1;
                for (int j = (int)f.scope.size() - 1; j >= 0; --j) {
                    const int32_t u = f.scope[j];
                    if (u != D.var) {
                        term.push_back((int32_t)(std::lower_bound(vars.begin(), vars.end(), u) - vars.begin()));
                        term.push_back((int32_t)st);
                        ++cf.nterm;
                    }
                    st *= I.dom[u];
                }
                fns.push_back(cf);
            }
            for (const Candidate &c : D.cands) {
                std::vector<uint8_t> po(D.B.size(), 0);
                for (size_t k = 0; k < c.parts.size(); ++k)
                    for (int32_t id : c.parts[k])
                        po[std::find(D.B.begin(), D.B.end(), id) - D.B.begin()] = (uint8_t)k;
                part.insert(part.end(), po.begin(), po.end());
            }
        } else {
            e.nfn = 0;
            e.nslot = 0;
        }
        dec.push_back(e);
    }
    CandLayout L{};
    L.off_dec = 0;
    L.off_fn = align256(L.off_dec + dec.size() * sizeof(DevCDec));
    L.off_term = align256(L.off_fn + fns.size() * sizeof(DevCFn));
    L.off_dom = align256(L.off_term + term.size() * sizeof(int32_t));
    L.off_part = align256(L.off_dom + dom.size() * sizeof(int32_t));
    L.total = align256(L.off_part + part.size());
    image.assign(L.total, 0);
    std::memcpy(image.data() + L.off_dec, dec.data(), dec.size() * sizeof(DevCDec));
    std::memcpy(image.data() + L.off_fn, fns.data(), fns.size() * sizeof(DevCFn));
    std::memcpy(image.data() + L.off_term, term.data(), term.size() * sizeof(int32_t));
    std::memcpy(image.data() + L.off_dom, dom.data(), dom.size() * sizeof(int32_t));
    std::memcpy(image.data() + L.off_part, part.data(), part.size());
    return L;
}

}  // namespace

size_t cand_scratch_bytes(const Plan &P) {
    std::vector<uint8_t> image;
    return build_cand_image(P, image).total;
}

bx_status dev_candidate_values(Plan &P, const void *ws, size_t ws_bytes, int32_t samples, const uint32_t *rnd,
                               double *out, void *scratch, size_t scratch_bytes, void *stream) {
    if (!ws || !rnd || !out || (!scratch && !P.decisions.empty()))
        return set_error(BX_E_INVALID, "NULL device pointer");
    if (ws_bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    if (samples < 1) return set_error(BX_E_INVALID, "samples must be >= 1");
    if (P.decisions.empty()) return BX_OK;
    const CandLayout L = build_cand_image(P, P.cand_image);
    if (scratch_bytes < L.total) return set_error(BX_E_NOMEM, "scratch smaller than bx_plan_candidate_scratch_bytes");
    if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0) return set_error(BX_E_INVALID, "scratch must be 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(scratch, P.cand_image.data(), L.total, hipMemcpyHostToDevice, st));
    const char *b = static_cast<const char *>(scratch);
    CDescs d;
    d.dec = reinterpret_cast<const DevCDec *>(b + L.off_dec);
    d.fn = reinterpret_cast<const DevCFn *>(b + L.off_fn);
    d.term = reinterpret_cast<const int32_t *>(b + L.off_term);
    d.dom = reinterpret_cast<const int32_t *>(b + L.off_dom);
    d.part = reinterpret_cast<const uint8_t *>(b + L.off_part);
    d.rnd = rnd;
    d.ws = static_cast<const char *>(ws);
    d.out = out;
    d.samples = samples;
    const dim3 grid((unsigned)P.decisions.size());
    if (P.ct == BX_COST_I32)
        hipLaunchKernelGGL(cand_values_kernel<true>, grid, dim3(kCandThreads), 0, st, d);
    else
        hipLaunchKernelGGL(cand_values_kernel<false>, grid, dim3(kCandThreads), 0, st, d);
    HIP_TRY(hipGetLastError());
    // the host image must outlive the copy
    HIP_TRY(hipStreamSynchronize(st));
    return BX_OK;
}

}  // namespace bx
