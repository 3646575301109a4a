// Streamed execution: tables that do not have to stay in device memory.
//
// The paper overlaps the transfer of one chunk of a bucket-table with the
// kernel working on the previous chunk (Sec. 6.3, the concurrent host /
// device computation).  Here every table -- the normalised inputs and every
// UTIL message -- lives in a caller-provided pinned host buffer laid out like
// the table and message regions of the plan's workspace, and the device
// holds only what one mini-bucket needs at a time:
//   - its input tables, copied in (host -> device) before it runs, except
//     the problem's own tables when they take no more room than one
//     mini-bucket's inputs: those are copied in once for the whole pass;
//   - its output, computed in chunks of rows into two device buffers: while
//     the kernel fills one, the previous chunk is copied out (device ->
//     host) on a second stream, events ordering the two streams;
//   - one small descriptor set per chunk (the mini-bucket with its output
//     offset moved onto the chunk buffer, its functions moved onto the
//     staged inputs, the chunk's tiles); all of them are built before the
//     pass and copied to the device in one copy, so the pass itself is only
//     table copies and launches, enqueued without waiting for the device.
// Mini-buckets run one after another in creation order (producers first); a
// consumer's input copies wait for the event recorded after its producers'
// last copy-outs, so a message is back in host memory before it is read.  The
// device workspace is then bounded by the largest mini-bucket's inputs plus
// two chunks, whatever the total size of the tables.  Scalar outputs (empty
// scope) stay on the device, and a last kernel adds them up per problem into
// the bound.  The value phase needs every table on the device and is not
// run: the result is the bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "bx_device.h"

namespace bx {

namespace {

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return set_error(BX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Rows of a chunk of mini-bucket d: a multiple of the rows one outer index
// covers on the tiled path.
int64_t chunk_of(const DevMb &d, int64_t chunk_rows) {
    if (d.path != 0) return std::max<int64_t>(1, chunk_rows);
    return std::max<int64_t>(1, chunk_rows / d.p_in) * d.p_in;
}

struct Layout {
    size_t zeros, tile_off, stage, stage_bytes, chunk[2], chunk_bytes;
    size_t inputs;                     // the input tables, when resident (inputs_resident)
    bool inputs_resident;
    size_t scal, bdesc, bout, total;   // the descriptor pool follows `total`
    int32_t max_tiles;
};

// Tiles of one chunk with at most this many rows each (row path: 256 rows;
// lane groups: their passes; tiled path: whole outer indices).
int32_t max_tiles_per_chunk(int64_t chunk_rows) { return (int32_t)(chunk_rows / 32 + 2); }

Layout layout_for(const Plan &P, int64_t chunk_rows) {
    Layout L{};
    size_t max_in = 0;
    for (size_t g = 0; g < P.mbs.size(); ++g) {
        size_t in = 0;
        const PInst &I = P.inst[P.mbs[g].inst];
        for (int32_t id : P.mbs[g].members) in += up((size_t)I.fns[id].size * 4);
        max_in = std::max(max_in, in);
    }
    L.max_tiles = max_tiles_per_chunk(chunk_rows);
    size_t o = 0;
    L.zeros = o;
    o = up(o + 256);
    L.tile_off = up(sizeof(DevMb));   // in a chunk's descriptor image: the mini-bucket, then the tiles
    L.stage = o;
    L.stage_bytes = std::max<size_t>(max_in, 256);
    o = up(o + L.stage_bytes);
    // the input tables stay on the device for the whole pass when they take
    // no more room than one mini-bucket's inputs already do
    L.inputs_resident = P.tables.size() <= L.stage_bytes;
    L.inputs = o;
    if (L.inputs_resident) o = up(o + std::max<size_t>(P.tables.size(), 256));
    L.chunk_bytes = up((size_t)chunk_rows * 4);
    for (int k = 0; k < 2; ++k) {
        L.chunk[k] = o;
        o = up(o + L.chunk_bytes);
    }
    L.scal = o;
    o = up(o + 4 * std::max<size_t>(P.dconst.size(), 1));
    L.bdesc = o;
    o = up(o + 32 * std::max<size_t>(P.inst.size(), 1));
    L.bout = o;
    o = up(o + 8 * std::max<size_t>(P.inst.size(), 1));
    L.total = o;
    return L;
}

// The bound of every problem: its constant plus its scalar outputs
// (saturating for integers), one thread per problem.
struct BoundDesc {
    int32_t begin, n;   // scalar outputs [begin, begin + n) of the scalar region
    int32_t pad[2];
    double base;        // constant inputs (and, for sums, -ln |D| of unconstrained variables)
};

template <class T>
__global__ void stream_bound_kernel(const BoundDesc *bd, const T *scal, double *out, int32_t n_inst) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_inst) return;
    const BoundDesc b = bd[i];
    if constexpr (std::is_same<T, int32_t>::value) {
        uint32_t a = (uint32_t)(int32_t)b.base;
        for (int32_t c = b.begin; c < b.begin + b.n; ++c) a = __builtin_elementwise_add_sat(a, (uint32_t)scal[c]);
        out[i] = (double)(a < (uint32_t)kInfI32 ? a : (uint32_t)kInfI32);
    } else {
        double a = b.base;
        for (int32_t c = b.begin; c < b.begin + b.n; ++c) a += (double)scal[c];
        out[i] = a;
    }
}

}  // namespace

// The pass, described before it runs: every descriptor image (function
// descriptors per mini-bucket, mini-bucket and tiles per chunk) in one pool
// that goes to the device in one copy, and per mini-bucket its input copies.
struct Chunk {
    size_t img;          // chunk image in the pool: DevMb, then the tiles at tile_off
    int32_t n_tiles;
    int64_t r0, r1;
};
struct In {
    size_t dst, src, bytes;
    int32_t producer;    // mini-bucket that wrote it, -1: an input table
};
struct MbPass {
    size_t fn_img = 0;
    std::vector<In> in;
    std::vector<Chunk> chunks;
};
struct PassPlan {
    std::vector<uint8_t> img;
    std::vector<MbPass> mb;
    std::vector<int32_t> scal_of;    // scalar outputs: their slot in the scalar region
    std::vector<uint8_t> consumed;   // mini-buckets whose output another one reads
};

bx_status build_pass(const Plan &P, int64_t chunk_rows, const Layout &L, PassPlan &pp) {
    const int64_t tab0 = (int64_t)(P.off_tables / 4);   // element offset of the table region
    pp.img.clear();
    pp.mb.assign(P.mbs.size(), MbPass{});
    pp.scal_of.assign(P.mbs.size(), -1);
    pp.consumed.assign(P.mbs.size(), 0);
    for (size_t c = 0; c < P.dconst.size(); ++c)
        for (size_t g = 0; g < P.mbs.size(); ++g)
            if (P.mbs[g].out_id < 0 && P.mbs[g].out_off == P.dconst[c]) pp.scal_of[g] = (int32_t)c;
    auto put = [&](const void *src, size_t n) -> size_t {
        const size_t at = pp.img.size();
        pp.img.resize(up(at + n), 0);
        std::memcpy(pp.img.data() + at, src, n);
        return at;
    };
    int64_t no = 0;   // chunk number over the pass: chunk buffers alternate
    for (size_t g = 0; g < P.mbs.size(); ++g) {
        const PMb &mb = P.mbs[g];
        const DevMb &d0 = P.dmb[g];
        const PInst &I = P.inst[mb.inst];
        if (d0.nf <= 0) return set_error(BX_E_INVALID, "internal: a mini-bucket without functions");
        std::vector<DevFn> fns(P.dfn.begin() + d0.f_begin, P.dfn.begin() + d0.f_begin + d0.nf);
        size_t so = 0;
        for (DevFn &f : fns) {
            int64_t size = 0;
            for (int32_t id : mb.members)
                if (I.fns[id].off == f.tab_off) size = I.fns[id].size;
            if (size <= 0) return set_error(BX_E_INVALID, "internal: input table not found");
            if (f.src_mb >= 0) pp.consumed[f.src_mb] = 1;
            if (f.src_mb < 0 && L.inputs_resident) {   // read in place
                f.tab_off = (int64_t)(L.inputs / 4) + (f.tab_off - tab0);
                continue;
            }
            pp.mb[g].in.push_back(In{L.stage + so, (size_t)(f.tab_off - tab0) * 4, (size_t)size * 4, f.src_mb});
            f.tab_off = (int64_t)((L.stage + so) / 4);
            so += up((size_t)size * 4);
        }
        pp.mb[g].fn_img = put(fns.data(), sizeof(DevFn) * fns.size());
        const int64_t step = chunk_of(d0, chunk_rows);
        for (int64_t r0 = 0; r0 < mb.out_rows; r0 += step, ++no) {
            const int64_t r1 = std::min<int64_t>(mb.out_rows, r0 + step);
            DevMb d = d0;
            d.f_begin = 0;
            d.level = 0;
            // row r lands at chunk buffer (no & 1) + (r - r0); a scalar stays on the device
            d.out_off = pp.scal_of[g] >= 0 ? (int64_t)(L.scal / 4) + pp.scal_of[g]
                                           : (int64_t)(L.chunk[no & 1] / 4) - r0;
            std::vector<DevTile> tiles;
            if (d.path == 0) {
                const int64_t o0 = r0 / d.p_in, o1 = r1 / d.p_in;
                const int64_t per = outer_per_tile(d, 4096);
                for (int64_t o = o0; o < o1; o += per) tiles.push_back(DevTile{0, 0, o, std::min(o1, o + per)});
            } else {
                const int64_t per = d.path == 2 ? (int64_t)(kUtilThreads / d.lanes) * kLanePasses : kRowTileRows;
                for (int64_t r = r0; r < r1; r += per) tiles.push_back(DevTile{0, 0, r, std::min(r1, r + per)});
            }
            if ((int32_t)tiles.size() > L.max_tiles) return set_error(BX_E_INVALID, "internal: chunk tiles exceed their bound");
            std::vector<uint8_t> slot(L.tile_off + sizeof(DevTile) * tiles.size(), 0);
            std::memcpy(slot.data(), &d, sizeof d);
            std::memcpy(slot.data() + L.tile_off, tiles.data(), sizeof(DevTile) * tiles.size());
            pp.mb[g].chunks.push_back(Chunk{put(slot.data(), slot.size()), (int32_t)tiles.size(), r0, r1});
        }
    }
    return BX_OK;
}

bx_status stream_bytes(const Plan &P, int64_t chunk_rows, size_t *dev_bytes, size_t *host_bytes) {
    if (chunk_rows < 256) return set_error(BX_E_INVALID, "chunk_rows must be >= 256");
    for (const DevMb &d : P.dmb)
        if (d.blk) return set_error(BX_E_UNSUPPORTED, "streamed execution needs a plan made with BX_FLAG_NO_BLOCKING");
    const Layout L = layout_for(P, chunk_rows);
    PassPlan pp;
    bx_status s = build_pass(P, chunk_rows, L, pp);
    if (s != BX_OK) return s;
    if (dev_bytes) *dev_bytes = L.total + up(std::max<size_t>(pp.img.size(), 256));   // + the descriptor pool
    if (host_bytes) *host_bytes = P.off_results - P.off_tables;   // the table and message regions
    return BX_OK;
}

bx_status dev_execute_streamed(Plan &P, void *ws, size_t bytes, void *host, size_t host_bytes, int64_t chunk_rows,
                               void *stream, double *bounds) {
    size_t need = 0, hneed = 0;
    bx_status s = stream_bytes(P, chunk_rows, &need, &hneed);
    if (s != BX_OK) return s;
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256) return set_error(BX_E_INVALID, "workspace must be 256-byte aligned");
    if (bytes < need) return set_error(BX_E_NOMEM, "workspace smaller than the streamed execution needs");
    if (!host || host_bytes < hneed) return set_error(BX_E_NOMEM, "host buffer smaller than the tables need");
    const Layout L = layout_for(P, chunk_rows);
    char *w = static_cast<char *>(ws);
    char *h = static_cast<char *>(host);
    hipStream_t sa = static_cast<hipStream_t>(stream);
    // the input tables into their place in the host buffer
    std::memcpy(h, P.tables.data(), P.tables.size());
    hipStream_t sb = nullptr;
    // events: kernel of chunk buffer k done, copy-out of chunk buffer k done,
    // and per mini-bucket whose output goes back to the host: its last
    // copy-out done (its consumers copy it in after that)
    hipEvent_t done_k[2] = {nullptr, nullptr}, done_c[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> out_done(P.mbs.size(), nullptr);
    // the pinned host image of the descriptor pool (copied in once)
    uint8_t *pin = nullptr;
    auto cleanup = [&]() {
        for (int k = 0; k < 2; ++k) {
            if (done_k[k]) (void)hipEventDestroy(done_k[k]);
            if (done_c[k]) (void)hipEventDestroy(done_c[k]);
        }
        for (hipEvent_t e : out_done)
            if (e) (void)hipEventDestroy(e);
        if (sb) (void)hipStreamDestroy(sb);
        if (pin) (void)hipHostFree(pin);
    };
    auto fail = [&](bx_status st) {
        (void)hipStreamSynchronize(sa);
        if (sb) (void)hipStreamSynchronize(sb);
        cleanup();
        return st;
    };
#define S_TRY(expr)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(set_error(BX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
    } while (0)
    const int64_t tab0 = (int64_t)(P.off_tables / 4);   // element offset of the table region
    PassPlan pp;
    {
        bx_status st = build_pass(P, chunk_rows, L, pp);
        if (st != BX_OK) return fail(st);
    }
    const std::vector<int32_t> &scal_of = pp.scal_of;
    const size_t pool = L.total;   // the descriptor pool's place in the workspace
    S_TRY(hipStreamCreateWithFlags(&sb, hipStreamNonBlocking));
    for (int k = 0; k < 2; ++k) {
        S_TRY(hipEventCreateWithFlags(&done_k[k], hipEventDisableTiming));
        S_TRY(hipEventCreateWithFlags(&done_c[k], hipEventDisableTiming));
    }
    for (size_t g = 0; g < P.mbs.size(); ++g)
        if (pp.consumed[g] && scal_of[g] < 0) S_TRY(hipEventCreateWithFlags(&out_done[g], hipEventDisableTiming));
    // every descriptor of the pass to the device in one copy
    S_TRY(hipHostMalloc(reinterpret_cast<void **>(&pin), std::max<size_t>(pp.img.size(), 256), hipHostMallocDefault));
    std::memcpy(pin, pp.img.data(), pp.img.size());
    S_TRY(hipMemcpyAsync(w + pool, pin, pp.img.size(), hipMemcpyHostToDevice, sa));
    if (L.inputs_resident && !P.tables.empty())
        S_TRY(hipMemcpyAsync(w + L.inputs, h, P.tables.size(), hipMemcpyHostToDevice, sa));
    S_TRY(hipMemsetAsync(w + L.zeros, 0, 256, sa));
    Descs base{};
    base.ws = w;
    base.zeros = w + L.zeros;
    base.nt = 0;
    base.xcd = 0;
    // ---- the pass: mini-buckets in creation order (producers first)
    // held[k]: the mini-bucket whose whole output chunk buffer k holds (-1:
    // none or part of one); a consumer then copies it device to device on
    // stream a, after the producer's kernel and before the buffer's next
    // kernel, instead of waiting for the copy-out and copying it back in
    int32_t held[2] = {-1, -1};
    int64_t chunk_no = 0;
    for (size_t g = 0; g < P.mbs.size(); ++g) {
        const PMb &mb = P.mbs[g];
        const DevMb &d0 = P.dmb[g];
        auto in_buffer = [&](int32_t p) -> int { return p < 0 ? -1 : held[0] == p ? 0 : held[1] == p ? 1 : -1; };
        // the messages it reads from host memory are back there (their
        // copy-outs on stream b), then its inputs come in
        for (const In &in : pp.mb[g].in)
            if (in.producer >= 0 && in_buffer(in.producer) < 0 && out_done[in.producer])
                S_TRY(hipStreamWaitEvent(sa, out_done[in.producer], 0));
        for (const In &in : pp.mb[g].in) {
            const int k = in_buffer(in.producer);
            if (k >= 0) S_TRY(hipMemcpyAsync(w + in.dst, w + L.chunk[k], in.bytes, hipMemcpyDeviceToDevice, sa));
            else S_TRY(hipMemcpyAsync(w + in.dst, h + in.src, in.bytes, hipMemcpyHostToDevice, sa));
        }
        for (const Chunk &c : pp.mb[g].chunks) {
            const int k = (int)(chunk_no & 1);
            // chunk buffer k is free once chunk_no - 2 is copied out
            if (chunk_no >= 2) S_TRY(hipStreamWaitEvent(sa, done_c[k], 0));
            Descs dd = base;
            dd.mb = reinterpret_cast<const DevMb *>(w + pool + c.img);
            dd.fn = reinterpret_cast<const DevFn *>(w + pool + pp.mb[g].fn_img);
            dd.tile = reinterpret_cast<const DevTile *>(w + pool + c.img + L.tile_off);
            dd.seg = nullptr;
            dd.n_tiles = c.n_tiles;
            if (d0.path == 2) {
                if (P.ct == BX_COST_I32) launch_lanes_i32(dd, 0, c.n_tiles, sa);
                else if (P.sum_mode) launch_lanes_fs(dd, 0, c.n_tiles, sa);
                else launch_lanes_f32(dd, 0, c.n_tiles, sa);
            } else {
                if (P.ct == BX_COST_I32) launch_tiles_i32(dd, 0, c.n_tiles, false, false, sa);
                else if (P.sum_mode) launch_tiles_fs(dd, 0, c.n_tiles, false, false, sa);
                else launch_tiles_f32(dd, 0, c.n_tiles, false, false, sa);
            }
            S_TRY(hipGetLastError());
            S_TRY(hipEventRecord(done_k[k], sa));
            // copy the chunk out on stream b once its kernel is done
            S_TRY(hipStreamWaitEvent(sb, done_k[k], 0));
            if (scal_of[g] < 0)
                S_TRY(hipMemcpyAsync(h + (mb.out_off - tab0 + c.r0) * 4, w + L.chunk[k], (size_t)(c.r1 - c.r0) * 4,
                                     hipMemcpyDeviceToHost, sb));
            S_TRY(hipEventRecord(done_c[k], sb));
            // a scalar output leaves the buffer as it was
            if (scal_of[g] < 0) held[k] = (c.r0 == 0 && c.r1 == mb.out_rows) ? (int32_t)g : -1;
            ++chunk_no;
        }
        if (out_done[g]) S_TRY(hipEventRecord(out_done[g], sb));
    }
    // the bound of every problem: constants plus scalar outputs (a kernel)
    std::vector<BoundDesc> bd(P.inst.size());
    for (size_t ii = 0; ii < P.inst.size(); ++ii) {
        const DevInst &di = P.dinst[ii];
        bd[ii] = BoundDesc{di.const_begin, di.const_n, {0, 0},
                           di.host_const + (P.ct == BX_COST_F32 ? di.bound_const : 0.0)};
    }
    S_TRY(hipMemcpyAsync(w + L.bdesc, bd.data(), sizeof(BoundDesc) * bd.size(), hipMemcpyHostToDevice, sa));
    const int32_t ni = (int32_t)P.inst.size();
    if (P.ct == BX_COST_I32)
        hipLaunchKernelGGL(stream_bound_kernel<int32_t>, dim3((ni + 255) / 256), dim3(256), 0, sa,
                           reinterpret_cast<const BoundDesc *>(w + L.bdesc),
                           reinterpret_cast<const int32_t *>(w + L.scal), reinterpret_cast<double *>(w + L.bout), ni);
    else
        hipLaunchKernelGGL(stream_bound_kernel<float>, dim3((ni + 255) / 256), dim3(256), 0, sa,
                           reinterpret_cast<const BoundDesc *>(w + L.bdesc),
                           reinterpret_cast<const float *>(w + L.scal), reinterpret_cast<double *>(w + L.bout), ni);
    S_TRY(hipGetLastError());
    S_TRY(hipMemcpyAsync(bounds, w + L.bout, sizeof(double) * P.inst.size(), hipMemcpyDeviceToHost, sa));
    S_TRY(hipStreamSynchronize(sb));
    S_TRY(hipStreamSynchronize(sa));
    cleanup();
    return BX_OK;
#undef S_TRY
}

}  // namespace bx
