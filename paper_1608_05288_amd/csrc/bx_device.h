// Device-side definitions shared by the UTIL-table kernels (gfx950, wave64):
// the cost algebra, the descriptor bundles the kernels receive, vector loads
// of runs of table entries, and the launchers each kernel translation unit
// provides to the host code.  Only .hip translation units include this.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "bx_internal.h"

namespace bx {

// ------------------------------------------------------------ cost algebra
// Integers accumulate as uint32 with a clamping add (v_add_u32 ... clamp); for
// non-negative int32 inputs min(INF, exact sum) is recovered at the end, the
// same value as a step-by-step saturating sum, whatever the order.
struct CostI {
    using T = int32_t;
    using A = uint32_t;
    static constexpr bool kSum = false;   // integer costs: minimum only
    __device__ static A zero() { return 0u; }
    __device__ static A ident() { return 0xffffffffu; }   // identity of mn
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
    static constexpr bool kSum = false;   // minimum only (MPE, float WCSPs)
    __device__ static A zero() { return 0.f; }
    __device__ static A ident() { return __builtin_huge_valf(); }
    __device__ static A add(A a, T v) { return a + v; }
    __device__ static A add2(A a, A b) { return a + b; }
    __device__ static A mn(A a, A b) { return fminf(a, b); }
    __device__ static T fin(A a) { return a; }
    __device__ static uint32_t bits(A a) { return __float_as_uint(a); }
    __device__ static A from_bits(uint32_t b) { return __uint_as_float(b); }
};

// Float costs of a sum-product plan: mini-buckets flagged `red` eliminate
// by summation (their own kernel instances, so that the min-only kernels
// keep their register budget).
struct CostFS : CostF {
    static constexpr bool kSum = true;
};

// Sum-product elimination (float costs): -ln sum_x exp(-a_x), taken as
// m - ln sum_x exp(m - a_x) with m the least a_x, so that every exponential
// is at most 1 and the largest is exactly 1; +inf when every a_x is +inf.
// `m` is the least of a[0..N), already computed by the caller.
template <int N>
__device__ __forceinline__ float soft_min(const float (&a)[N], float m) {
    if (m == __builtin_huge_valf()) return m;
    float s = 0.f;
#pragma unroll
    for (int x = 0; x < N; ++x) s += expf(m - a[x]);
    return m - logf(s);
}

// The same over values arriving one at a time (and from other lanes):
// m = least value so far, s = sum of exp(m - a) over the values so far.
struct SoftAcc {
    float m = __builtin_huge_valf();
    float s = 0.f;
    __device__ void add(float a) {
        if (a < m) {
            s = s * expf(a - m) + 1.f;     // m = +inf: exp(-inf) = 0
            m = a;
        } else if (a != __builtin_huge_valf()) {
            s += expf(m - a);
        }
    }
    __device__ void merge(float m2, float s2) {
        if (m2 == __builtin_huge_valf()) return;
        if (m == __builtin_huge_valf()) { m = m2; s = s2; return; }
        if (m2 < m) { s = s * expf(m2 - m) + s2; m = m2; }
        else s += s2 * expf(m - m2);
    }
    __device__ float fin() const { return m == __builtin_huge_valf() ? m : m - logf(s); }
};

struct Descs {
    const DevMb *mb;
    const DevFn *fn;
    const DevTile *tile;
    const DevSeg *seg;   // segments of the packed tiles
    char *ws;
    const char *zeros;   // 256 zero bytes of the workspace
    int32_t n_tiles;
    int32_t nt;          // blocked rows stored non-temporally (per launch)
    int32_t xcd;         // tiles taken XCD by XCD (per launch): workgroup b runs on
                         //   XCD b % 8, and XCD x takes the x-th contiguous part
                         //   of the launch's tiles, so the tiles of one
                         //   mini-bucket share that XCD's L2
    // descriptor warm-up (per launch): pf_extra (0 or kWarmBlocks) workgroups
    // after the launch's tiles load the descriptors of the next launch's
    // tiles [pf_t0, pf_t0 + pf_n) into the L2 of the XCD each will run on
    // (pf_xcd: the next launch takes its tiles XCD by XCD)
    int32_t pf_t0, pf_n, pf_extra, pf_xcd;
    int32_t *sink;       // a word the warm-up writes only to keep its loads
};
constexpr int kWarmBlocks = 8;        // one warm-up workgroup per XCD
constexpr int kWarmMaxTiles = 4096;   // next launches with more tiles are not warmed


// ------------------------------------------------------------ value kernel
constexpr int kValueThreads = 256;
constexpr int kSigmaCap = 16384;   // variables per problem (uint16 in LDS)
// value kernel: LDS arena for the assignment and the staged descriptors (the
// comparison buffer and the reduction buffer sit beside it, 160 KB in all)
constexpr int kValueArenaBytes = 140 * 1024;
constexpr int kPairCap = kValuePairCap;  // candidate values per value step

struct VDescs {
    const DevInst *inst;
    const DevVar *var;
    const DevVFn *vfn;
    const int32_t *term;
    const int32_t *occ;
    const DevPair *pair;
    const int32_t *vlv;
    const int32_t *vlp;
    const int64_t *cst;
    DevResult *res;
    char *ws;
    char *sigma_base;
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

// ------------------------------------------------------------ launchers
// Defined in the kernel translation units (one per cost type and tiled-kernel
// variant, so that they compile in parallel).  Tiles [t0, t0 + n) of the
// descriptor bundle; nothing is launched when n <= 0.
void launch_tiles_i32(const Descs &d, int32_t t0, int32_t n, bool stage, bool nt, hipStream_t st);
void launch_tiles_f32(const Descs &d, int32_t t0, int32_t n, bool stage, bool nt, hipStream_t st);
void launch_tiles_fs(const Descs &d, int32_t t0, int32_t n, bool stage, bool nt, hipStream_t st);
void launch_tiles_fs_s0(const Descs &d, int32_t t0, int32_t n, bool nt, hipStream_t st);
void launch_tiles_fs_s1(const Descs &d, int32_t t0, int32_t n, bool nt, hipStream_t st);
void launch_lanes_fs(const Descs &d, int32_t t0, int32_t n, hipStream_t st);
void launch_tiles_i32_s0(const Descs &d, int32_t t0, int32_t n, bool nt, hipStream_t st);
void launch_tiles_i32_s1(const Descs &d, int32_t t0, int32_t n, bool nt, hipStream_t st);
void launch_tiles_f32_s0(const Descs &d, int32_t t0, int32_t n, bool nt, hipStream_t st);
void launch_tiles_f32_s1(const Descs &d, int32_t t0, int32_t n, bool nt, hipStream_t st);
void launch_lanes_i32(const Descs &d, int32_t t0, int32_t n, hipStream_t st);
void launch_lanes_f32(const Descs &d, int32_t t0, int32_t n, hipStream_t st);
void launch_value_i32(const VDescs &d, int32_t n_inst, hipStream_t st);
void launch_value_f32(const VDescs &d, int32_t n_inst, hipStream_t st);
void launch_stream(int kind, void *dst, const void *src, int64_t n16, int32_t grid, hipStream_t st);

}  // namespace bx
