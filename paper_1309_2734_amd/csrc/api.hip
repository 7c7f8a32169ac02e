// Host side of the C-ABI in include/cgh.h: argument checks, device
// workspace, planning and the kernel sequence of each evaluation mode.
//
// Evaluation sequence of one hologram (Section 2.1, Eq. (2) and (5)):
//   a1 per-point constants (FP64)          k_point_consts
//   a2 line phases reduced mod 1 (FP64)    k_phase_tables   (direct mode)
//   a3 direct FP32 accumulation            k_direct
// or
//   a4 hi/lo line factors                  k_factors        (matrix-core modes)
//   a5 split GEMM (+ fixed-order split-K)  k_gemm, k_splitk_reduce
// Large clouds are cut into point chunks that fit the workspace budget; the
// chunks accumulate into the output in order.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cgh.h"
#include "common.h"

using namespace cgh;

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_last_error;

cgh_status fail(cgh_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

cgh_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? CGH_ENOMEM : CGH_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define CGH_HIP(call, what)                                                                   \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return hip_fail(e_, what);                                                        \
    } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    hipError_t set(int dev)
    {
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess)
            return e;
        ok = true;
        return prev == dev ? hipSuccess : hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (ok) {
            int cur = -1;
            if (hipGetDevice(&cur) == hipSuccess && cur != prev)
                (void)hipSetDevice(prev);
        }
    }
};

// Grow-only device buffer.  `shadow` keeps the bytes last copied into a
// small table, so an unchanged table is not copied (or waited for) again.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    std::vector<char> shadow;
    hipError_t ensure(size_t bytes, bool *moved = nullptr)
    {
        if (bytes <= cap)
            return hipSuccess;
        shadow.clear();
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            cap = 0;
            if (e != hipSuccess)
                return e;
        }
        size_t want = bytes < 256 ? 256 : bytes;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = want;
        if (moved)
            *moved = true;
        return hipSuccess;
    }
    void release()
    {
        shadow.clear();
        if (p)
            (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Bytes of device workspace one class of intermediate (tables or factors)
// may take; larger clouds are processed in point chunks.
size_t workspace_budget()
{
    const char *env = std::getenv("CGH_WORKSPACE_BYTES");
    if (env && *env) {
        char *end = nullptr;
        unsigned long long v = std::strtoull(env, &end, 10);
        if (end && *end == '\0' && v >= (1ull << 20))
            return (size_t)v;
    }
    return (size_t)4 << 30;
}

struct ProfRecord {
    const char *name;
    hipEvent_t start, stop;
};
struct ProfTotal {
    const char *name;
    int64_t launches;
    double ms;
};

}  // namespace

// ------------------------------------------------------------------ context
struct cgh_ctx {
    int width = 0, height = 0, device = 0;
    double pitch = 0.0, wavelength = 0.0;
    int wpad = 0, hpad = 0;           // line tables padded to kLinePad

    // uploaded cloud: float SoA x | y | z | amp, each n_cap long
    DevBuf points;
    int64_t n = 0, n_cap = 0;
    bool uploaded = false;

    // workspace
    DevBuf consts;                    // beta | cx | cy (double) | amp (float)
    int64_t consts_cap = 0;           // slots
    DevBuf tab_u, tab_v;              // a2 tables
    DevBuf fac[4];                    // Lh, Ll, Rh, Rl
    DevBuf partials;                  // split-K partial tiles
    DevBuf segs, frames;              // small device tables
    uint64_t ws_generation = 0;       // bumps when a buffer moves

    // batch graph cache
    hipGraphExec_t graph_exec = nullptr;
    std::vector<cgh_frame> graph_frames;
    int graph_mode = -1;
    float *graph_out = nullptr;
    hipStream_t graph_stream = nullptr;
    uint64_t graph_generation = 0;
    uint64_t points_generation = 0;
    uint64_t graph_points_generation = 0;

    // profiling
    bool profiling = false;
    std::vector<ProfRecord> prof_pending;
    std::vector<hipEvent_t> prof_free;
    std::vector<ProfTotal> prof_totals;
};

namespace {

void drop_graph(cgh_ctx *c)
{
    if (c->graph_exec)
        (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    c->graph_frames.clear();
}

hipError_t ensure_ws(cgh_ctx *c, DevBuf &b, size_t bytes)
{
    bool moved = false;
    hipError_t e = b.ensure(bytes, &moved);
    if (moved) {
        ++c->ws_generation;
        drop_graph(c);
    }
    return e;
}

hipEvent_t take_event(cgh_ctx *c)
{
    if (!c->prof_free.empty()) {
        hipEvent_t e = c->prof_free.back();
        c->prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Launch bracket for profiling: record a start event before and a stop
// event after a launch on stream s.
struct Bracket {
    cgh_ctx *c;
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    Bracket(cgh_ctx *c_, const char *n, hipStream_t s_) : c(c_), name(n), s(s_)
    {
        if (c->profiling) {
            a = take_event(c);
            b = take_event(c);
            if (a && b)
                (void)hipEventRecord(a, s);
        }
    }
    void done()
    {
        if (a && b) {
            (void)hipEventRecord(b, s);
            c->prof_pending.push_back({name, a, b});
            a = b = nullptr;
        }
    }
    ~Bracket()
    {
        if (a)
            c->prof_free.push_back(a);
        if (b)
            c->prof_free.push_back(b);
    }
};

PointConsts consts_view(cgh_ctx *c, int64_t slots)
{
    char *base = (char *)c->consts.p;
    PointConsts pc;
    pc.beta = (double *)base;
    pc.cx = (double *)(base + 8 * slots);
    pc.cy = (double *)(base + 16 * slots);
    pc.amp = (float *)(base + 24 * slots);
    return pc;
}

hipError_t ensure_consts(cgh_ctx *c, int64_t slots)
{
    // 8 + 8 + 8 + 4 bytes per slot; the view is laid out for `slots`
    hipError_t e = ensure_ws(c, c->consts, (size_t)slots * 28 + 256);
    if (e == hipSuccess)
        c->consts_cap = slots;
    return e;
}

// Segment and frame tables (small) go to device memory with a synchronous
// copy, after the stream has drained (queued kernels may still read the old
// contents).  A table whose bytes did not change since the last copy is left
// alone, so repeated evaluations of one workload never block the host.
hipError_t upload_small(cgh_ctx *c, DevBuf &b, const void *src, size_t bytes, hipStream_t s)
{
    if (b.p && b.shadow.size() == bytes && std::memcmp(b.shadow.data(), src, bytes) == 0)
        return hipSuccess;
    hipError_t e = ensure_ws(c, b, bytes);
    if (e != hipSuccess)
        return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return e;
    e = hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        b.shadow.clear();
        return e;
    }
    b.shadow.assign((const char *)src, (const char *)src + bytes);
    return hipSuccess;
}

const float *pts_x(cgh_ctx *c) { return (const float *)c->points.p; }
const float *pts_y(cgh_ctx *c) { return pts_x(c) + c->n_cap; }
const float *pts_z(cgh_ctx *c) { return pts_x(c) + 2 * c->n_cap; }
const float *pts_a(cgh_ctx *c) { return pts_x(c) + 3 * c->n_cap; }

// ---------------------------------------------------------------- planning
struct Plan {
    GemmPlan g;
    int tiles_m = 0, tiles_n = 0;
};

// Tile shape and split count for an M x N output over `slots` points.
// CGH_GEMM_PLAN="bm,bn,waves_m,waves_n,stages,splits" overrides the choice
// (used to sweep shapes; an unsupported shape is ignored, splits 0 = auto).
Plan plan_gemm(int M, int N, int64_t slots, int products)
{
    struct Shape {
        int bm, bn, wm, wn, stages;
    };
    static const Shape cand[] = {{192, 384, 2, 4, 2}, {384, 192, 4, 2, 2}, {192, 256, 2, 4, 2},
                                 {256, 256, 2, 4, 2}, {128, 256, 2, 4, 2}};
    Plan best;
    int forced_splits = 0;
    Shape forced = {0, 0, 0, 0, 0};
    const char *env = std::getenv("CGH_GEMM_PLAN");
    if (env && std::sscanf(env, "%d,%d,%d,%d,%d,%d", &forced.bm, &forced.bn, &forced.wm,
                           &forced.wn, &forced.stages, &forced_splits) >= 5 &&
        gemm_tile_supported(forced.bm, forced.bn, forced.wm, forced.wn, forced.stages)) {
        best.g.bm = forced.bm;
        best.g.bn = forced.bn;
        best.g.waves_m = forced.wm;
        best.g.waves_n = forced.wn;
        best.g.stages = forced.stages;
    } else {
        forced_splits = 0;
        double best_cost = 1e300;
        for (auto &t : cand) {
            const int tm = (M + t.bm - 1) / t.bm, tn = (N + t.bn - 1) / t.bn;
            const double padded = (double)tm * t.bm * (double)tn * t.bn;
            // operand bytes per flop fall with the tile's harmonic size
            const double reuse = 2.0 * t.bm * t.bn / (t.bm + t.bn);
            const double cost = padded * (1.0 + 64.0 / reuse);
            if (cost < best_cost) {
                best_cost = cost;
                best.g.bm = t.bm;
                best.g.bn = t.bn;
                best.g.waves_m = t.wm;
                best.g.waves_n = t.wn;
                best.g.stages = t.stages;
            }
        }
    }
    best.tiles_m = (M + best.g.bm - 1) / best.g.bm;
    best.tiles_n = (N + best.g.bn - 1) / best.g.bn;
    const int tiles = best.tiles_m * best.tiles_n;
    const int64_t kblocks = slots / kFragPoints;
    // as many K splits as fit the device (one workgroup per CU) in one wave
    int splits = forced_splits > 0 ? forced_splits : std::max(1, 256 / tiles);
    while (splits > 1 && kblocks / splits < 8)
        --splits;
    best.g.splits = splits;
    best.g.mblocks = best.tiles_m * (best.g.bm / kFragLines);
    best.g.nblocks = best.tiles_n * (best.g.bn / kFragLines);
    best.g.kblocks = kblocks;
    best.g.products = products;
    return best;
}

cgh_status check_mode(int mode)
{
    if (mode < CGH_DIRECT_FP32 || mode > CGH_SEPARABLE_FP32)
        return fail(CGH_EINVAL, "unknown mode");
    return CGH_OK;
}

// ------------------------------------------------------- one set of frames
// Direct kernel over frames whose constants occupy slots [0, total_slots)
// (tables built here).  `fd_dev` points at the device copy of the frames.
cgh_status run_direct(cgh_ctx *c, const FrameDesc *fd_dev, int n_frames, int64_t total_slots,
                      float *out, bool accumulate, hipStream_t s)
{
    const size_t tu = (size_t)std::max<int64_t>(total_slots, 1) * c->wpad * sizeof(float);
    const size_t tv = (size_t)std::max<int64_t>(total_slots, 1) * c->hpad * sizeof(float);
    CGH_HIP(ensure_ws(c, c->tab_u, tu), "table allocation");
    CGH_HIP(ensure_ws(c, c->tab_v, tv), "table allocation");
    if (total_slots > 0) {
        Bracket br(c, "phase_tables", s);
        CGH_HIP(launch_phase_tables(consts_view(c, c->consts_cap), total_slots, c->wpad, c->hpad,
                                    (float *)c->tab_u.p, (float *)c->tab_v.p, s),
                "phase_tables launch");
        br.done();
    }
    Bracket br(c, "direct_fp32", s);
    CGH_HIP(launch_direct((const float *)c->tab_u.p, (const float *)c->tab_v.p,
                          consts_view(c, c->consts_cap).amp, fd_dev, n_frames, c->width,
                          c->height, c->wpad, c->hpad, 16, out, accumulate, s),
            "direct launch");
    br.done();
    return CGH_OK;
}

// Matrix-core modes for one frame whose constants are slots [slot0, slot0 + slots).
cgh_status run_gemm(cgh_ctx *c, int mode, int64_t slot0, int64_t slots, float *out,
                    bool accumulate, hipStream_t s)
{
    const bool split = mode == CGH_SPLIT_BF16 || mode == CGH_SPLIT_FP16;
    const FactorType ft = mode == CGH_SPLIT_BF16 ? FactorType::BF16 : FactorType::FP16;
    const Plan p = plan_gemm(c->height, c->width, slots, split ? 3 : 1);
    const int hl = split ? 2 : 1;
    // 2 K-columns (cos, sin) of 2 bytes per line and point
    const size_t lbytes = (size_t)p.g.mblocks * kFragLines * (size_t)slots * 2 * 2;
    const size_t rbytes = (size_t)p.g.nblocks * kFragLines * (size_t)slots * 2 * 2;
    CGH_HIP(ensure_ws(c, c->fac[0], lbytes), "factor allocation");
    CGH_HIP(ensure_ws(c, c->fac[2], rbytes), "factor allocation");
    if (hl == 2) {
        CGH_HIP(ensure_ws(c, c->fac[1], lbytes), "factor allocation");
        CGH_HIP(ensure_ws(c, c->fac[3], rbytes), "factor allocation");
    }
    if (p.g.splits > 1)
        CGH_HIP(ensure_ws(c, c->partials,
                          (size_t)p.g.splits * c->height * (size_t)c->width * sizeof(float)),
                "split-K workspace allocation");
    PointConsts pc = consts_view(c, c->consts_cap);
    {
        Bracket br(c, split ? "factors_split" : "factors", s);
        CGH_HIP(launch_factors(pc, slot0, slots, c->width, c->height, p.g.kblocks, p.g.mblocks,
                               p.g.nblocks, ft, c->fac[0].p, hl == 2 ? c->fac[1].p : nullptr,
                               c->fac[2].p, hl == 2 ? c->fac[3].p : nullptr, s),
                "factor launch");
        br.done();
    }
    {
        Bracket br(c, split ? "gemm_split_mfma" : "gemm_mfma", s);
        CGH_HIP(launch_gemm(p.g, ft, c->fac[0].p, hl == 2 ? c->fac[1].p : nullptr, c->fac[2].p,
                            hl == 2 ? c->fac[3].p : nullptr, c->height, c->width, out, c->width,
                            (float *)c->partials.p, accumulate, s),
                "gemm launch");
        br.done();
    }
    if (p.g.splits > 1) {
        Bracket br(c, "splitk_reduce", s);
        CGH_HIP(launch_splitk_reduce((const float *)c->partials.p, p.g.splits, c->height,
                                     c->width, out, c->width, accumulate, s),
                "split-K reduce launch");
        br.done();
    }
    return CGH_OK;
}

// Bytes of workspace per constant slot for a mode (tables or factors).
size_t bytes_per_slot(cgh_ctx *c, int mode)
{
    if (mode == CGH_DIRECT_FP32)
        return (size_t)(c->wpad + c->hpad) * sizeof(float);
    const int hl = (mode == CGH_SPLIT_BF16 || mode == CGH_SPLIT_FP16) ? 2 : 1;
    return (size_t)(round_up(c->width, 384) + round_up(c->height, 384)) * 2 * 2 * hl;
}

int64_t chunk_slots(cgh_ctx *c, int mode)
{
    int64_t chunk = (int64_t)(workspace_budget() / bytes_per_slot(c, mode));
    return std::max<int64_t>(kSlotAlign, chunk / kSlotAlign * kSlotAlign);
}

// Per-point constants of segment `seg_index` of the uploaded segment table.
cgh_status point_consts(cgh_ctx *c, int seg_index, int n_segs, int64_t max_count, int64_t slots,
                        hipStream_t s)
{
    CGH_HIP(ensure_consts(c, slots), "constant allocation");
    Bracket br(c, "point_consts", s);
    CGH_HIP(launch_point_consts(pts_x(c), pts_y(c), pts_z(c), pts_a(c),
                                (const Segment *)c->segs.p + seg_index, n_segs,
                                std::max<int64_t>(max_count, 1), c->width, c->height, c->pitch,
                                consts_view(c, slots), s),
            "point constant launch");
    br.done();
    return CGH_OK;
}

// Hologram of points [p0, p0 + count) at wavelength lam into out (H x W),
// cut into point chunks that fit the workspace budget.  Chunk i's segment
// and frame descriptors are entry i of the two small tables.
cgh_status eval_one(cgh_ctx *c, int mode, int64_t p0, int64_t count, double lam, float *out,
                    hipStream_t s)
{
    const int64_t chunk = chunk_slots(c, mode);
    std::vector<Segment> segs;
    std::vector<FrameDesc> fds;
    for (int64_t off = 0; off < count || segs.empty(); off += chunk) {
        const int64_t cnt = std::min(chunk, count - off);
        segs.push_back({p0 + off, cnt, 0, lam});
        fds.push_back({0, round_up(cnt, kSlotAlign) / kGroup, 0});
    }
    CGH_HIP(upload_small(c, c->segs, segs.data(), segs.size() * sizeof(Segment), s),
            "segment table upload");
    CGH_HIP(upload_small(c, c->frames, fds.data(), fds.size() * sizeof(FrameDesc), s),
            "frame table upload");
    for (size_t i = 0; i < segs.size(); ++i) {
        const int64_t slots = std::max<int64_t>(round_up(segs[i].count, kSlotAlign), kSlotAlign);
        cgh_status st = point_consts(c, (int)i, 1, segs[i].count, slots, s);
        if (st != CGH_OK)
            return st;
        const bool acc = i > 0;
        if (mode == CGH_DIRECT_FP32 || segs[i].count == 0)
            st = run_direct(c, (const FrameDesc *)c->frames.p + i, 1,
                            round_up(segs[i].count, kSlotAlign), out, acc, s);
        else
            st = run_gemm(c, mode, 0, slots, out, acc, s);
        if (st != CGH_OK)
            return st;
    }
    return CGH_OK;
}

// Direct mode over many frames with one launch per stage: all frames'
// constants and tables side by side, the direct kernel's grid covering every
// frame (largest first, so the longest workgroups start first).
cgh_status eval_batch_direct(cgh_ctx *c, const cgh_frame *frames, int n_frames, float *out,
                             hipStream_t s)
{
    const int64_t plane = (int64_t)c->width * c->height;
    std::vector<int> order(n_frames);
    for (int f = 0; f < n_frames; ++f)
        order[f] = f;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return frames[a].point_count > frames[b].point_count;
    });
    std::vector<Segment> segs(n_frames);
    std::vector<FrameDesc> fds(n_frames);
    int64_t slot = 0, max_count = 0;
    for (int k = 0; k < n_frames; ++k) {
        const cgh_frame &fr = frames[order[k]];
        const int64_t padded = round_up(fr.point_count, kSlotAlign);
        segs[k] = {fr.point_offset, fr.point_count, slot, fr.wavelength};
        fds[k] = {slot, padded / kGroup, order[k] * plane};
        slot += padded;
        max_count = std::max(max_count, fr.point_count);
    }
    CGH_HIP(upload_small(c, c->segs, segs.data(), segs.size() * sizeof(Segment), s),
            "segment table upload");
    CGH_HIP(upload_small(c, c->frames, fds.data(), fds.size() * sizeof(FrameDesc), s),
            "frame table upload");
    const int64_t slots = std::max<int64_t>(slot, kSlotAlign);
    cgh_status st = point_consts(c, 0, n_frames, max_count, slots, s);
    if (st != CGH_OK)
        return st;
    return run_direct(c, (const FrameDesc *)c->frames.p, n_frames, slot, out, false, s);
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char *cgh_strerror(cgh_status s)
{
    switch (s) {
    case CGH_OK: return "success";
    case CGH_EINVAL: return "invalid argument";
    case CGH_ENOMEM: return "out of memory";
    case CGH_EDEVICE: return "device error";
    case CGH_ENOTSUP: return "not supported";
    case CGH_ESTATE: return "invalid call order";
    }
    return "unknown status";
}

const char *cgh_last_error(void) { return g_last_error.c_str(); }

int32_t cgh_version(void) { return 10000; }

cgh_status cgh_create(cgh_ctx **out, int32_t width, int32_t height, double pitch_m,
                      double wavelength_m, int32_t device)
{
    g_last_error.clear();
    if (!out)
        return fail(CGH_EINVAL, "out is NULL");
    *out = nullptr;
    if (width < 1 || width > 65536 || height < 1 || height > 65536)
        return fail(CGH_EINVAL, "width and height must be in [1, 65536]");
    if (!finite_pos(pitch_m))
        return fail(CGH_EINVAL, "pitch must be finite and > 0");
    if (!finite_pos(wavelength_m))
        return fail(CGH_EINVAL, "wavelength must be finite and > 0");
    if (device < 0)
        return fail(CGH_EINVAL, "device index must be >= 0");

    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0)
        return fail(CGH_EDEVICE, std::string("no HIP device: ") +
                                     (e != hipSuccess ? hipGetErrorString(e) : "none visible"));
    if (device >= count)
        return fail(CGH_EDEVICE, "device index out of range");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CGH_EDEVICE, std::string("device is ") + prop.gcnArchName +
                                     ", this library is built for gfx950");

    cgh_ctx *c = new (std::nothrow) cgh_ctx();
    if (!c)
        return fail(CGH_ENOMEM, "context allocation");
    c->width = width;
    c->height = height;
    c->pitch = pitch_m;
    c->wavelength = wavelength_m;
    c->device = device;
    c->wpad = (int)round_up(width, kLinePad);
    c->hpad = (int)round_up(height, kLinePad);
    *out = c;
    return CGH_OK;
}

void cgh_destroy(cgh_ctx *c)
{
    if (!c)
        return;
    DeviceGuard g;
    if (g.set(c->device) == hipSuccess)
        (void)hipDeviceSynchronize();
    drop_graph(c);
    for (auto &r : c->prof_pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : c->prof_free)
        (void)hipEventDestroy(e);
    c->points.release();
    c->consts.release();
    c->tab_u.release();
    c->tab_v.release();
    for (auto &f : c->fac)
        f.release();
    c->partials.release();
    c->segs.release();
    c->frames.release();
    delete c;
}

cgh_status cgh_points_upload(cgh_ctx *c, const float *x, const float *y, const float *z,
                             const float *amp, int64_t n, cgh_mem where, void *stream)
{
    g_last_error.clear();
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    if (n < 0)
        return fail(CGH_EINVAL, "n must be >= 0");
    if (where != CGH_MEM_HOST && where != CGH_MEM_DEVICE)
        return fail(CGH_EINVAL, "unknown memory kind");
    if (n > 0 && (!x || !y || !z || !amp))
        return fail(CGH_EINVAL, "point arrays must be non-NULL when n > 0");
    if (n > ((int64_t)1 << 34))
        return fail(CGH_EINVAL, "too many points");
    if (where == CGH_MEM_HOST) {
        for (int64_t i = 0; i < n; ++i) {
            if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(z[i]) ||
                !std::isfinite(amp[i]))
                return fail(CGH_EINVAL, "point " + std::to_string(i) + " has a non-finite value");
            if (!(z[i] > 0.0f))
                return fail(CGH_EINVAL, "point " + std::to_string(i) + " has z <= 0");
        }
    }
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const int64_t cap = std::max<int64_t>(n, 1);
    if (cap > c->n_cap || !c->points.p) {
        // the old cloud may still be read by queued work on this stream
        CGH_HIP(hipStreamSynchronize(s), "stream synchronise");
        c->points.release();
        CGH_HIP(c->points.ensure((size_t)cap * 4 * sizeof(float)), "point allocation");
        c->n_cap = cap;
        ++c->ws_generation;
        drop_graph(c);
    }
    float *d = (float *)c->points.p;
    const float *src[4] = {x, y, z, amp};
    if (n > 0) {
        for (int k = 0; k < 4; ++k) {
            if (where == CGH_MEM_HOST) {
                CGH_HIP(hipStreamSynchronize(s), "stream synchronise");
                CGH_HIP(hipMemcpy(d + k * c->n_cap, src[k], (size_t)n * sizeof(float),
                                  hipMemcpyHostToDevice),
                        "point upload");
            } else {
                CGH_HIP(hipMemcpyAsync(d + k * c->n_cap, src[k], (size_t)n * sizeof(float),
                                       hipMemcpyDeviceToDevice, s),
                        "point upload");
            }
        }
    }
    c->n = n;
    c->uploaded = true;
    ++c->points_generation;
    return CGH_OK;
}

cgh_status cgh_compute(cgh_ctx *c, cgh_mode mode, float *out_dev, void *stream)
{
    g_last_error.clear();
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    if (!out_dev)
        return fail(CGH_EINVAL, "output is NULL");
    cgh_status st = check_mode(mode);
    if (st != CGH_OK)
        return st;
    if (!c->uploaded)
        return fail(CGH_ESTATE, "no points uploaded");
    if (mode == CGH_SEPARABLE_FP32)
        return fail(CGH_ENOTSUP, "CGH_SEPARABLE_FP32 is not built yet");
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    return eval_one(c, mode, 0, c->n, c->wavelength, out_dev, (hipStream_t)stream);
}

cgh_status cgh_batch_compute(cgh_ctx *c, const cgh_frame *frames, int32_t n_frames,
                             cgh_mode mode, float *out_dev, void *stream)
{
    g_last_error.clear();
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    if (!frames)
        return fail(CGH_EINVAL, "frames is NULL");
    if (n_frames < 1 || n_frames > 65535)
        return fail(CGH_EINVAL, "n_frames must be in [1, 65535]");
    if (!out_dev)
        return fail(CGH_EINVAL, "output is NULL");
    cgh_status st = check_mode(mode);
    if (st != CGH_OK)
        return st;
    if (!c->uploaded)
        return fail(CGH_ESTATE, "no points uploaded");
    for (int f = 0; f < n_frames; ++f) {
        const cgh_frame &fr = frames[f];
        if (fr.point_offset < 0 || fr.point_count < 0 || fr.point_offset > c->n ||
            fr.point_count > c->n - fr.point_offset)
            return fail(CGH_EINVAL, "frame " + std::to_string(f) + " is outside the upload");
        if (!finite_pos(fr.wavelength))
            return fail(CGH_EINVAL, "frame " + std::to_string(f) + " has a bad wavelength");
    }
    if (mode == CGH_SEPARABLE_FP32)
        return fail(CGH_ENOTSUP, "CGH_SEPARABLE_FP32 is not built yet");
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const int64_t plane = (int64_t)c->width * c->height;
    if (mode == CGH_DIRECT_FP32) {
        int64_t total = 0;
        for (int f = 0; f < n_frames; ++f)
            total += round_up(frames[f].point_count, kSlotAlign);
        if (total <= chunk_slots(c, mode))
            return eval_batch_direct(c, frames, n_frames, out_dev, s);
    }
    for (int f = 0; f < n_frames; ++f) {
        st = eval_one(c, mode, frames[f].point_offset, frames[f].point_count,
                      frames[f].wavelength, out_dev + f * plane, s);
        if (st != CGH_OK)
            return st;
    }
    return CGH_OK;
}

cgh_status cgh_profile_enable(cgh_ctx *c, int32_t on)
{
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    c->profiling = on != 0;
    return CGH_OK;
}

cgh_status cgh_profile_reset(cgh_ctx *c)
{
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    for (auto &r : c->prof_pending) {
        (void)hipEventSynchronize(r.stop);
        c->prof_free.push_back(r.start);
        c->prof_free.push_back(r.stop);
    }
    c->prof_pending.clear();
    c->prof_totals.clear();
    return CGH_OK;
}

cgh_status cgh_profile_read(cgh_ctx *c, const char **names, int64_t *launches, double *total_ms,
                            int32_t capacity, int32_t *count)
{
    if (!c || !count || capacity < 0 || (capacity > 0 && (!names || !launches || !total_ms)))
        return fail(CGH_EINVAL, "bad profile_read arguments");
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    for (auto &r : c->prof_pending) {
        CGH_HIP(hipEventSynchronize(r.stop), "hipEventSynchronize");
        float ms = 0.0f;
        CGH_HIP(hipEventElapsedTime(&ms, r.start, r.stop), "hipEventElapsedTime");
        auto it = std::find_if(c->prof_totals.begin(), c->prof_totals.end(),
                               [&](const ProfTotal &t) { return std::strcmp(t.name, r.name) == 0; });
        if (it == c->prof_totals.end())
            c->prof_totals.push_back({r.name, 1, (double)ms});
        else {
            it->launches += 1;
            it->ms += ms;
        }
        c->prof_free.push_back(r.start);
        c->prof_free.push_back(r.stop);
    }
    c->prof_pending.clear();
    int32_t k = 0;
    for (auto &t : c->prof_totals) {
        if (k >= capacity)
            break;
        names[k] = t.name;
        launches[k] = t.launches;
        total_ms[k] = t.ms;
        ++k;
    }
    *count = k;
    return CGH_OK;
}

}  // extern "C"
