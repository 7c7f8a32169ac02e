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
// Large clouds are cut into point chunks that fit the workspace; the chunks
// accumulate into the output in order.
//
// Streams.  Every call only enqueues work on its stream.  A single
// hologram's segment and frame descriptors travel in the kernel arguments; a
// batch's tables go to device memory through a page-locked staging ring with
// asynchronous copies.  Calls on one context share its workspace, so each
// call's stream first waits for an event recorded behind the previous call
// (on whatever stream that ran).  The host blocks only where a workspace
// buffer must grow (the allocator synchronises the device).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
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

#define CGH_TRY(call)                                                                         \
    do {                                                                                      \
        cgh_status s_ = (call);                                                               \
        if (s_ != CGH_OK)                                                                     \
            return s_;                                                                        \
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
// small table, so an unchanged table is not copied again.  Growing waits for
// the device first: queued work may still read the old allocation.
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
            hipError_t e = hipDeviceSynchronize();
            if (e == hipSuccess)
                e = hipFree(p);
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
    return (size_t)16 << 30;
}

// True while `s` records into a graph.
bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return st != hipStreamCaptureStatusNone;
}

// Page-locked staging ring for the small device tables of batch calls.  A
// table is written into the ring and copied to the device asynchronously on
// the call's stream; an event recorded behind the copy tells when its ring
// region may be written again.  Enqueuing a copy never waits for earlier
// kernels, only (after the ring wraps) for earlier copies still pending.
struct Staging {
    char *host = nullptr;
    size_t cap = 0, head = 0;
    struct Use {
        size_t off, len;
        hipEvent_t ev;
    };
    std::deque<Use> busy;
    std::vector<hipEvent_t> spare;

    hipError_t wait_all()
    {
        for (auto &u : busy) {
            hipError_t e = hipEventSynchronize(u.ev);
            if (e != hipSuccess)
                return e;
            spare.push_back(u.ev);
        }
        busy.clear();
        return hipSuccess;
    }
    // A region of `len` bytes no pending copy reads; *off receives its offset.
    hipError_t reserve(size_t len, size_t *off)
    {
        len = (len + 255) / 256 * 256;
        if (len > cap) {
            hipError_t e = wait_all();
            if (e != hipSuccess)
                return e;
            const size_t want = std::max({len, 2 * cap, (size_t)1 << 20});
            if (host)
                (void)hipHostFree(host);
            host = nullptr;
            cap = head = 0;
            e = hipHostMalloc((void **)&host, want, hipHostMallocDefault);
            if (e != hipSuccess) {
                host = nullptr;
                return e;
            }
            cap = want;
        }
        if (head + len > cap)
            head = 0;
        for (auto it = busy.begin(); it != busy.end();) {
            const bool overlap = it->off < head + len && head < it->off + it->len;
            const hipError_t e = overlap ? hipEventSynchronize(it->ev) : hipEventQuery(it->ev);
            if (e == hipSuccess) {
                spare.push_back(it->ev);
                it = busy.erase(it);
            } else if (e == hipErrorNotReady) {
                ++it;
            } else {
                return e;
            }
        }
        *off = head;
        head += len;
        return hipSuccess;
    }
    // The copy out of [off, off + len) was enqueued on s.
    hipError_t mark(size_t off, size_t len, hipStream_t s)
    {
        hipEvent_t ev = nullptr;
        if (!spare.empty()) {
            ev = spare.back();
            spare.pop_back();
        } else {
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess)
                return e;
        }
        hipError_t e = hipEventRecord(ev, s);
        if (e != hipSuccess) {
            spare.push_back(ev);
            return e;
        }
        busy.push_back({off, len, ev});
        return hipSuccess;
    }
    void release()
    {
        (void)wait_all();
        for (auto ev : spare)
            (void)hipEventDestroy(ev);
        spare.clear();
        if (host)
            (void)hipHostFree(host);
        host = nullptr;
        cap = head = 0;
    }
};

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
// One autotuned choice: a GEMM shape + split count, or (direct mode) the rows
// each lane owns.  Keyed by device arch, hologram size, mode and the K-size
// bucket (ceil(log2(K blocks))).
struct TuneEntry {
    std::string key;
    int bm = 0, bn = 0, wm = 0, wn = 0, stages = 0, splits = 0, rows = 0;
    double us = 0.0;
};

struct cgh_ctx {
    int width = 0, height = 0, device = 0;
    double pitch = 0.0, wavelength = 0.0;
    int wpad = 0, hpad = 0;           // line tables padded to kLinePad

    // uploaded cloud: float SoA x | y | z | amp, each n_cap long
    DevBuf points;
    int64_t n = 0, n_cap = 0;
    bool uploaded = false;

    // workspace, shared by all evaluations (each call rewrites what it reads)
    DevBuf consts;                    // beta | cx | cy | zlam (double) | amp | zhalf (float)
    DevBuf tab_u, tab_v;              // a2 tables
    DevBuf tab_x, tab_y;              // a2s offset tables (exact spherical wave)
    DevBuf fac;                       // Lh | Ll | Rh | Rl in one allocation
    DevBuf partials;                  // split-K partial tiles / point-split planes
    DevBuf tune_out;                  // scratch hologram for cgh_tune
    DevBuf field;                     // complex object wave for cgh_kinoform
    // device tables of batch calls only (a captured batch graph reads them;
    // no other call writes them)
    DevBuf bsegs, bframes, items, counter;
    Staging staging;                  // host side of the batch tables' copies
    uint64_t ws_generation = 0;       // bumps when a buffer moves

    // ordering of calls made on different streams
    hipEvent_t order_ev = nullptr;
    hipStream_t order_stream = nullptr;
    bool order_valid = false;

    // batch graph cache
    hipGraphExec_t graph_exec = nullptr;
    std::vector<cgh_frame> graph_frames;
    int graph_mode = -1;
    float *graph_out = nullptr;
    uint64_t graph_generation = 0;

    // autotuned plans (from cgh_tune or the cache file), see plan lookup
    std::string arch;
    std::vector<struct TuneEntry> tuned;

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

// Calls on one context share its workspace: a call's stream waits for the
// end of the previous call when that ran on another stream (nothing is
// recorded or waited for inside a stream capture).
struct CallOrder {
    cgh_ctx *c;
    hipStream_t s;
    bool active;
    CallOrder(cgh_ctx *c_, hipStream_t s_) : c(c_), s(s_), active(!capturing(s_)) {}
    hipError_t enter()
    {
        if (!active || !c->order_valid || c->order_stream == s)
            return hipSuccess;
        return hipStreamWaitEvent(s, c->order_ev, 0);
    }
    ~CallOrder()
    {
        if (!active)
            return;
        if (!c->order_ev &&
            hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming) != hipSuccess) {
            c->order_ev = nullptr;
            return;
        }
        if (hipEventRecord(c->order_ev, s) == hipSuccess) {
            c->order_stream = s;
            c->order_valid = true;
        } else {
            // without the marker a later stream cannot wait for this call
            (void)hipStreamSynchronize(s);
            c->order_valid = false;
        }
    }
};

// Copy a small host table into device buffer b, ordered on stream s, unless
// b already holds those bytes (or will once s reaches the copy that put them
// there).  Inside a stream capture a table that would change is refused,
// which abandons the capture.
cgh_status upload_small(cgh_ctx *c, DevBuf &b, const void *src, size_t bytes, hipStream_t s,
                        const char *what)
{
    if (bytes == 0)
        return CGH_OK;
    if (b.p && b.shadow.size() == bytes && std::memcmp(b.shadow.data(), src, bytes) == 0)
        return CGH_OK;
    if (capturing(s))
        return fail(CGH_ESTATE, std::string(what) + " would change inside a stream capture");
    CGH_HIP(ensure_ws(c, b, bytes), what);
    size_t off = 0;
    CGH_HIP(c->staging.reserve(bytes, &off), what);
    std::memcpy(c->staging.host + off, src, bytes);
    b.shadow.clear();
    CGH_HIP(hipMemcpyAsync(b.p, c->staging.host + off, bytes, hipMemcpyHostToDevice, s), what);
    if (c->staging.mark(off, bytes, s) != hipSuccess)
        CGH_HIP(hipStreamSynchronize(s), what);   // the region must not be reused early
    b.shadow.assign((const char *)src, (const char *)src + bytes);
    return CGH_OK;
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
// event after a launch on stream s (nothing without a profiling context).
struct Bracket {
    cgh_ctx *c;
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    Bracket(cgh_ctx *c_, const char *n, hipStream_t s_) : c(c_), name(n), s(s_)
    {
        if (c && c->profiling) {
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

// Constants of `slots` slots laid out from `base`: 4 x 8 + 2 x 4 bytes per slot.
PointConsts consts_at(char *base, int64_t slots)
{
    PointConsts pc;
    pc.beta = (double *)base;
    pc.cx = (double *)(base + 8 * slots);
    pc.cy = (double *)(base + 16 * slots);
    pc.zlam = (double *)(base + 24 * slots);
    pc.amp = (float *)(base + 32 * slots);
    pc.zhalf = (float *)(base + 36 * slots);
    return pc;
}
size_t consts_bytes(int64_t slots) { return (size_t)slots * 40 + 256; }

cgh_status check_mode(int mode)
{
    if (mode < CGH_DIRECT_FP32 || mode > CGH_SPHERICAL_FP32)
        return fail(CGH_EINVAL, "unknown mode");
    return CGH_OK;
}

// Modes evaluated by the direct kernels (a cosine per point and pixel).
bool is_direct(int mode) { return mode == CGH_DIRECT_FP32 || mode == CGH_SPHERICAL_FP32; }

// How a matrix-core mode stores and multiplies its factors.
struct ModeInfo {
    FactorType ft;
    int products;        // 3 = hi*hi + hi*lo + lo*hi, 1 = one product
    int hl;              // factor arrays per side (hi, lo)
    int elem;            // bytes per factor value
    int kbp;             // points per K block
    const char *fac_name, *gemm_name, *batch_name;   // profiling labels
    // bytes of factors per line (row or column) and point
    int line_bytes() const { return 2 * elem * hl; }
};

ModeInfo mode_info(int mode)
{
    switch (mode) {
    case CGH_SPLIT_BF16:
        return {FactorType::BF16, 3, 2, 2, kblock_points(FactorType::BF16), "factors_split",
                "gemm_split_mfma", "gemm_split_mfma_batch"};
    case CGH_SPLIT_FP16:
        return {FactorType::FP16, 3, 2, 2, kblock_points(FactorType::FP16), "factors_split",
                "gemm_split_mfma", "gemm_split_mfma_batch"};
    case CGH_SEPARABLE_FP32:
        return {FactorType::FP32, 1, 1, 4, kblock_points(FactorType::FP32), "factors_fp32",
                "gemm_fp32_mfma", "gemm_fp32_mfma_batch"};
    default:   // CGH_FP16
        return {FactorType::FP16, 1, 1, 2, kblock_points(FactorType::FP16), "factors",
                "gemm_mfma", "gemm_mfma_batch"};
    }
}

// ---------------------------------------------------------------- planning
// GEMM launch shapes the tuner tries: (BM, BN, waves along M, waves along N,
// LDS ring depth); each must be built in gemm.hip.
const int kShapes[][5] = {{192, 384, 2, 4, 2}, {384, 192, 4, 2, 2}, {192, 320, 2, 4, 2},
                          {192, 256, 2, 4, 2}, {256, 256, 2, 4, 2}, {192, 192, 2, 2, 3},
                          {192, 192, 2, 4, 3}, {128, 256, 2, 4, 2}, {192, 128, 2, 2, 2},
                          {128, 192, 2, 2, 2}};

// Lines padded to whole tiles of every shape (factor sets are sized for any
// of them).
int64_t pad_all_shapes(int64_t lines, bool rows)
{
    int64_t p = lines;
    for (auto &sh : kShapes)
        p = std::max(p, round_up(lines, rows ? sh[0] : sh[1]));
    return p;
}
struct Plan {
    GemmPlan g;
    int tiles_m = 0, tiles_n = 0;
};

int kblock_bucket(int64_t kblocks)
{
    int b = 0;
    while (((int64_t)1 << b) < kblocks)
        ++b;
    return b;
}

// `m_lines` = output rows of the product: the height, or twice it for a
// complex evaluation (real and imaginary planes stacked).
std::string tune_key(const cgh_ctx *c, int mode, int64_t kblocks, int m_lines)
{
    return c->arch + "/" + std::to_string(c->width) + "x" + std::to_string(m_lines) + "/mode" +
           std::to_string(mode) + "/kb" + std::to_string(kblock_bucket(kblocks));
}

const TuneEntry *find_tuned(const cgh_ctx *c, const std::string &key)
{
    if (!c)
        return nullptr;
    for (auto &t : c->tuned)
        if (t.key == key)
            return &t;
    return nullptr;
}

// Key of a batch's tuned launch: hologram size, mode and the K bucket of its
// largest frame.
std::string batch_tune_key(const cgh_ctx *c, int mode, int64_t max_kblocks)
{
    return c->arch + "/" + std::to_string(c->width) + "x" + std::to_string(c->height) + "/mode" +
           std::to_string(mode) + "/batch/kb" + std::to_string(kblock_bucket(max_kblocks));
}

// Tile shape and split count for an M x N output over `slots` points: the
// tuned plan `tuned` when there is one, else
// CGH_GEMM_PLAN="bm,bn,waves_m,waves_n,stages,splits" (used to sweep shapes;
// an unsupported shape is ignored, splits 0 = auto), else the default choice.
Plan plan_gemm(int M, int N, int64_t slots, const ModeInfo &mi, const TuneEntry *tuned = nullptr)
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
    if (tuned && gemm_tile_supported(tuned->bm, tuned->bn, tuned->wm, tuned->wn, tuned->stages)) {
        forced = {tuned->bm, tuned->bn, tuned->wm, tuned->wn, tuned->stages};
        forced_splits = tuned->splits;
    }
    if ((tuned && forced.bm) ||
        (env && std::sscanf(env, "%d,%d,%d,%d,%d,%d", &forced.bm, &forced.bn, &forced.wm,
                            &forced.wn, &forced.stages, &forced_splits) >= 5 &&
         gemm_tile_supported(forced.bm, forced.bn, forced.wm, forced.wn, forced.stages))) {
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
    const int64_t kblocks = slots / mi.kbp;
    // as many K splits as fit the device in one wave of workgroups
    const int resident = 256 * gemm_groups_per_cu(best.g.bm, best.g.bn, best.g.waves_m,
                                                  best.g.waves_n, best.g.stages, mi.products);
    int splits = forced_splits > 0 ? forced_splits : std::max(1, resident / tiles);
    while (splits > 1 && kblocks / splits < 8)
        --splits;
    best.g.splits = splits;
    best.g.mblocks = best.tiles_m * (best.g.bm / kFragLines);
    best.g.nblocks = best.tiles_n * (best.g.bn / kFragLines);
    best.g.kblocks = kblocks;
    best.g.products = mi.products;
    return best;
}

// --------------------------------------------------------- evaluation core
// Hologram geometry of one evaluation.
struct Geo {
    int width = 0, height = 0, wpad = 0, hpad = 0;
    double pitch = 0.0;
};

Geo ctx_geo(const cgh_ctx *c) { return {c->width, c->height, c->wpad, c->hpad, c->pitch}; }

// Where an evaluation's intermediates live.
enum class Role { Consts = 0, TabU, TabV, TabX, TabY, Factors, Partials, Count };

struct Ws {
    virtual ~Ws() = default;
    // at least `bytes` of device memory for `role`; stable for the evaluation
    virtual cgh_status get(Role role, size_t bytes, void **p) = 0;
};

// The context's grow-only buffers.
struct CtxWs final : Ws {
    cgh_ctx *c;
    explicit CtxWs(cgh_ctx *c_) : c(c_) {}
    cgh_status get(Role role, size_t bytes, void **p) override
    {
        DevBuf *b = nullptr;
        switch (role) {
        case Role::Consts: b = &c->consts; break;
        case Role::TabU: b = &c->tab_u; break;
        case Role::TabV: b = &c->tab_v; break;
        case Role::TabX: b = &c->tab_x; break;
        case Role::TabY: b = &c->tab_y; break;
        case Role::Factors: b = &c->fac; break;
        default: b = &c->partials; break;
        }
        CGH_HIP(ensure_ws(c, *b, std::max<size_t>(bytes, 1)), "workspace allocation");
        *p = b->p;
        return CGH_OK;
    }
};

// One evaluation: geometry, the points (device SoA), the workspace and, with
// a context, its tuned plans and profiling.
struct Eval {
    cgh_ctx *c = nullptr;     // nullptr: default plans, no profiling
    Geo g;
    const float *x = nullptr, *y = nullptr, *z = nullptr, *a = nullptr;
    Ws *ws = nullptr;
    size_t partial_cap = SIZE_MAX;   // bytes of split partials allowed
    int rows = 0;             // direct rows per lane chosen by the caller (0: own choice)
    PointConsts pc{};         // set by ev_consts
    float *tu = nullptr, *tv = nullptr, *tx = nullptr, *ty = nullptr;   // set by ev_tables
};

const float *pts_x(cgh_ctx *c) { return (const float *)c->points.p; }
const float *pts_y(cgh_ctx *c) { return pts_x(c) + c->n_cap; }
const float *pts_z(cgh_ctx *c) { return pts_x(c) + 2 * c->n_cap; }
const float *pts_a(cgh_ctx *c) { return pts_x(c) + 3 * c->n_cap; }

Eval ctx_eval(cgh_ctx *c, Ws *ws)
{
    Eval ev;
    ev.c = c;
    ev.g = ctx_geo(c);
    ev.x = pts_x(c);
    ev.y = pts_y(c);
    ev.z = pts_z(c);
    ev.a = pts_a(c);
    ev.ws = ws;
    return ev;
}

// a1: per-point constants of the segments into `slots` slots.
cgh_status ev_consts(Eval &ev, const SegList &segs, int n_segs, int64_t max_count, int64_t slots,
                     hipStream_t s)
{
    void *p = nullptr;
    CGH_TRY(ev.ws->get(Role::Consts, consts_bytes(slots), &p));
    ev.pc = consts_at((char *)p, slots);
    Bracket br(ev.c, "point_consts", s);
    CGH_HIP(launch_point_consts(ev.x, ev.y, ev.z, ev.a, segs, n_segs,
                                std::max<int64_t>(max_count, 1), ev.g.width, ev.g.height,
                                ev.g.pitch, ev.pc, s),
            "point constant launch");
    br.done();
    return CGH_OK;
}

// a2 (Eq. (2)) or a2s (Eq. (1)) tables for constant slots [0, slots).
cgh_status ev_tables(Eval &ev, int mode, int64_t slots, hipStream_t s)
{
    const bool sph = mode == CGH_SPHERICAL_FP32;
    const size_t tu = (size_t)std::max<int64_t>(slots, 1) * ev.g.wpad * sizeof(float);
    const size_t tv = (size_t)std::max<int64_t>(slots, 1) * ev.g.hpad * sizeof(float);
    void *p = nullptr;
    CGH_TRY(ev.ws->get(Role::TabU, tu, &p));
    ev.tu = (float *)p;
    CGH_TRY(ev.ws->get(Role::TabV, tv, &p));
    ev.tv = (float *)p;
    if (sph) {
        CGH_TRY(ev.ws->get(Role::TabX, tu, &p));
        ev.tx = (float *)p;
        CGH_TRY(ev.ws->get(Role::TabY, tv, &p));
        ev.ty = (float *)p;
    }
    if (slots <= 0)
        return CGH_OK;
    Bracket br(ev.c, sph ? "sphere_tables" : "phase_tables", s);
    if (sph)
        CGH_HIP(launch_sphere_tables(ev.pc, slots, ev.g.wpad, ev.g.hpad, ev.tu, ev.tv, ev.tx,
                                     ev.ty, s),
                "sphere_tables launch");
    else
        CGH_HIP(launch_phase_tables(ev.pc, slots, ev.g.wpad, ev.g.hpad, ev.tu, ev.tv, s),
                "phase_tables launch");
    br.done();
    return CGH_OK;
}

// Row counts per lane the direct kernels are built for.
bool direct_rows_ok(int mode, int rows)
{
    if (mode == CGH_SPHERICAL_FP32)
        return rows == 4 || rows == 8;
    return rows == 4 || rows == 8 || rows == 16;
}

hipError_t launch_direct_mode(const Eval &ev, int mode, const FrameList &frames, int n_frames,
                              int rows, float *out, float *out_im, bool accumulate, hipStream_t s)
{
    if (mode == CGH_SPHERICAL_FP32)
        return launch_direct_sphere(ev.tu, ev.tv, ev.tx, ev.ty, ev.pc.amp, ev.pc.zhalf, frames,
                                    n_frames, ev.g.width, ev.g.height, ev.g.wpad, ev.g.hpad, rows,
                                    out, out_im, accumulate, s);
    return launch_direct(ev.tu, ev.tv, ev.pc.amp, frames, n_frames, ev.g.width, ev.g.height,
                         ev.g.wpad, ev.g.hpad, rows, out, out_im, accumulate, s);
}

// Rows per lane of a direct launch: CGH_DIRECT_ROWS (4, 8 or 16; used to
// sweep), else the tuned choice, else the default.
int direct_rows(const Eval &ev, int mode)
{
    if (ev.rows && direct_rows_ok(mode, ev.rows))
        return ev.rows;
    const TuneEntry *t = ev.c ? find_tuned(ev.c, tune_key(ev.c, mode, 0, ev.g.height)) : nullptr;
    int rows = t && direct_rows_ok(mode, t->rows) ? t->rows
                                                   : (mode == CGH_SPHERICAL_FP32 ? 8 : 16);
    if (const char *env = std::getenv("CGH_DIRECT_ROWS")) {
        const int r = std::atoi(env);
        if (direct_rows_ok(mode, r))
            rows = r;
    }
    return rows;
}

// Point split of a direct evaluation: the K split count (CGH_DIRECT_SPLITS,
// 1, 2 or 4, used to sweep; else the tuned choice; else enough runs, up to 4,
// for about 2048 workgroups of four waves, eight waves per SIMD).
int direct_splits(const Eval &ev, int mode)
{
    const TuneEntry *t = ev.c ? find_tuned(ev.c, tune_key(ev.c, mode, 0, ev.g.height)) : nullptr;
    int sp = 1;
    if (t && t->splits > 0) {
        sp = t->splits;
    } else {
        const int rows = direct_rows(ev, mode);
        const int64_t wgs = (int64_t)((ev.g.width + 63) / 64) *
                            ((ev.g.height + 4 * rows - 1) / (4 * rows));
        while (sp < 4 && wgs * sp < 2048)
            sp *= 2;
    }
    if (const char *env = std::getenv("CGH_DIRECT_SPLITS")) {
        const int v = std::atoi(env);
        if (v == 1 || v == 2 || v == 4)
            sp = v;
    }
    return sp;
}

// One frame's points cut into at most `splits` (<= kInlineFrames) runs of
// whole group pairs (the direct kernel takes a frame's groups two at a
// time), run r writing partial planes r * planes .. (planes = 2 for a
// complex evaluation: real, then imaginary).  *runs receives the count.
FrameList split_frames(const FrameDesc &fd, int splits, int planes, int64_t plane, int *runs)
{
    FrameList fl{};
    fl.dev = nullptr;
    const int64_t pairs = fd.groups / 2;
    const int64_t per = std::max<int64_t>(1, (pairs + splits - 1) / splits);
    int r = 0;
    for (int64_t p = 0; p < pairs && r < kInlineFrames; p += per, ++r) {
        const int64_t np = std::min(per, pairs - p);
        fl.inl[r] = {fd.first + p * 2 * kGroup, 2 * np, (int64_t)r * planes * plane};
    }
    *runs = r;
    return fl;
}

// Direct kernel over frames whose constants occupy slots [0, total_slots)
// (tables built here).
cgh_status ev_run_direct(Eval &ev, int mode, const FrameList &frames, int n_frames,
                         int64_t total_slots, float *out, float *out_im, bool accumulate,
                         hipStream_t s)
{
    CGH_TRY(ev_tables(ev, mode, total_slots, s));
    const bool sph = mode == CGH_SPHERICAL_FP32;
    const int rows = direct_rows(ev, mode);
    const char *name = sph ? (out_im ? "direct_sphere_complex" : "direct_sphere")
                           : (out_im ? "direct_fp32_complex" : "direct_fp32");
    Bracket br(ev.c, name, s);
    CGH_HIP(launch_direct_mode(ev, mode, frames, n_frames, rows, out, out_im, accumulate, s),
            "direct launch");
    br.done();
    return CGH_OK;
}

// Direct mode for one frame, split over its points when the split count asks
// for it: the runs write partial planes, summed in a fixed order (more
// workgroups for a small hologram, the same numbers on every run).
cgh_status ev_run_direct_one(Eval &ev, int mode, const FrameDesc &fd, int64_t total_slots,
                             float *out, float *out_im, bool accumulate, hipStream_t s)
{
    const int64_t plane = (int64_t)ev.g.width * ev.g.height;
    // a complex evaluation's planes [Re; Im] are consecutive: each run writes
    // its own pair, and the pairs are summed as planes of 2H rows
    const int planes = out_im ? 2 : 1;
    int splits = out_im && out_im != out + plane ? 1 : direct_splits(ev, mode);
    while (splits > 1 && (size_t)splits * planes * plane * sizeof(float) > ev.partial_cap)
        splits /= 2;
    if (splits <= 1 || fd.groups < 4) {
        FrameList fl{};
        fl.dev = nullptr;
        fl.inl[0] = fd;
        return ev_run_direct(ev, mode, fl, 1, total_slots, out, out_im, accumulate, s);
    }
    int runs = 0;
    const FrameList fl = split_frames(fd, splits, planes, plane, &runs);
    void *p = nullptr;
    CGH_TRY(ev.ws->get(Role::Partials, (size_t)runs * planes * plane * sizeof(float), &p));
    float *part = (float *)p;
    CGH_TRY(ev_run_direct(ev, mode, fl, runs, total_slots, part, out_im ? part + plane : nullptr,
                          false, s));
    Bracket br(ev.c, "splitk_reduce", s);
    CGH_HIP(launch_splitk_reduce(part, runs, planes * ev.g.height, ev.g.width, out, ev.g.width,
                                 accumulate, s),
            "split-K reduce launch");
    br.done();
    return CGH_OK;
}

// Matrix-core modes for `slots` constant slots from slot 0.  With `cplx`, L
// holds the real- and imaginary-part rows stacked (M = 2H) and `out`
// receives [Re; Im] as two consecutive H x W planes.  With `raw` the factor
// kernel evaluates the points' constants itself (ev.pc is not read).
cgh_status ev_run_gemm(Eval &ev, int mode, int64_t slots, float *out, bool cplx, bool accumulate,
                       hipStream_t s, const RawPoints *raw = nullptr)
{
    const ModeInfo mi = mode_info(mode);
    const int M = cplx ? 2 * ev.g.height : ev.g.height;
    const int N = ev.g.width;
    Plan p = plan_gemm(M, N, slots, mi,
                       ev.c ? find_tuned(ev.c, tune_key(ev.c, mode, slots / mi.kbp, M)) : nullptr);
    const size_t per_split = (size_t)M * N * sizeof(float);
    while (p.g.splits > 1 && (size_t)p.g.splits * per_split > ev.partial_cap)
        --p.g.splits;
    FactorSet fs;
    fs.hl = mi.hl;
    fs.amb = p.g.mblocks;
    fs.anb = p.g.nblocks;
    fs.kblocks = p.g.kblocks;
    void *fp = nullptr;
    CGH_TRY(ev.ws->get(Role::Factors, (size_t)std::max<int64_t>(fs.bytes(), 1), &fp));
    fs.base = (char *)fp;
    float *part = nullptr;
    if (p.g.splits > 1) {
        void *pp = nullptr;
        CGH_TRY(ev.ws->get(Role::Partials, (size_t)p.g.splits * per_split, &pp));
        part = (float *)pp;
    }
    {
        Bracket br(ev.c, mi.fac_name, s);
        if (raw)
            CGH_HIP(launch_factors_points(*raw, ev.g.width, ev.g.height, cplx, p.g.kblocks,
                                          p.g.mblocks, p.g.nblocks, mi.ft, fs, s),
                    "factor launch");
        else
            CGH_HIP(launch_factors(ev.pc, 0, ev.g.width, ev.g.height, cplx, p.g.kblocks,
                                   p.g.mblocks, p.g.nblocks, mi.ft, fs, s),
                    "factor launch");
        br.done();
    }
    {
        Bracket br(ev.c, mi.gemm_name, s);
        CGH_HIP(launch_gemm(p.g, mi.ft, fs, M, N, out, N, part, accumulate, s), "gemm launch");
        br.done();
    }
    if (p.g.splits > 1) {
        Bracket br(ev.c, "splitk_reduce", s);
        CGH_HIP(launch_splitk_reduce(part, p.g.splits, M, N, out, N, accumulate, s),
                "split-K reduce launch");
        br.done();
    }
    return CGH_OK;
}

// Bytes of workspace per constant slot for a mode (tables or factors).
size_t bytes_per_slot(const Geo &g, int mode, bool cplx)
{
    if (is_direct(mode))
        return (size_t)(g.wpad + g.hpad) * sizeof(float) * (mode == CGH_SPHERICAL_FP32 ? 2 : 1);
    const int64_t m = cplx ? 2 * (int64_t)g.height : g.height;
    const int64_t w = pad_all_shapes(g.width, false);
    const int64_t h = pad_all_shapes(m, true);
    return (size_t)(w + h) * mode_info(mode).line_bytes();
}

int64_t chunk_slots(const Geo &g, int mode, bool cplx = false)
{
    int64_t chunk = (int64_t)(workspace_budget() / bytes_per_slot(g, mode, cplx));
    return std::max<int64_t>(kSlotAlign, chunk / kSlotAlign * kSlotAlign);
}

// Hologram of points [p0, p0 + count) at wavelength lam into out (H x W, or
// [Re; Im] with cplx), in point chunks of `chunk` slots that accumulate into
// the output in order.  Each chunk's segment travels in the kernel arguments.
cgh_status ev_one(Eval &ev, int mode, int64_t p0, int64_t count, double lam, float *out,
                  bool cplx, int64_t chunk, hipStream_t s)
{
    float *out_im = cplx ? out + (int64_t)ev.g.width * ev.g.height : nullptr;
    int64_t off = 0;
    do {
        const int64_t cnt = std::min(chunk, count - off);
        const int64_t padded = round_up(cnt, kSlotAlign);
        const int64_t slots = std::max<int64_t>(padded, kSlotAlign);
        const bool acc = off > 0;
        if (is_direct(mode) || cnt == 0) {
            SegList sl{};
            sl.dev = nullptr;
            sl.one = {p0 + off, cnt, 0, lam};
            CGH_TRY(ev_consts(ev, sl, 1, cnt, slots, s));
            const FrameDesc fd{0, padded / kGroup, 0};
            CGH_TRY(ev_run_direct_one(ev, is_direct(mode) ? mode : CGH_DIRECT_FP32, fd, padded,
                                      out, out_im, acc, s));
        } else {
            // the factor kernel takes the points themselves: no constants launch
            const RawPoints rp{ev.x, ev.y, ev.z, ev.a, p0 + off, cnt, lam,
                               0.5 * (double)(ev.g.width - 1), 0.5 * (double)(ev.g.height - 1),
                               ev.g.pitch};
            CGH_TRY(ev_run_gemm(ev, mode, slots, out, cplx, acc, s, &rp));
        }
        off += chunk;
    } while (off < count);
    return CGH_OK;
}

// A single hologram of the context's whole cloud.
cgh_status eval_ctx(cgh_ctx *c, int mode, float *out, bool cplx, hipStream_t s)
{
    CtxWs ws(c);
    Eval ev = ctx_eval(c, &ws);
    return ev_one(ev, mode, 0, c->n, c->wavelength, out, cplx, chunk_slots(ev.g, mode, cplx), s);
}

// ------------------------------------------------------------------ batches
// Direct mode over many frames with one launch per stage: all frames'
// constants and tables side by side, the direct kernel's grid covering every
// frame (largest first, so the longest workgroups start first).
cgh_status eval_batch_direct(cgh_ctx *c, int mode, const cgh_frame *frames, int n_frames,
                             float *out, hipStream_t s, const TuneEntry *force = nullptr)
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
    CGH_TRY(upload_small(c, c->bsegs, segs.data(), segs.size() * sizeof(Segment), s,
                         "segment table upload"));
    CGH_TRY(upload_small(c, c->bframes, fds.data(), fds.size() * sizeof(FrameDesc), s,
                         "frame table upload"));
    CtxWs ws(c);
    Eval ev = ctx_eval(c, &ws);
    const TuneEntry *t =
        force ? force : find_tuned(c, batch_tune_key(c, mode, round_up(max_count, kSlotAlign)));
    if (t)
        ev.rows = t->rows;
    const int64_t slots = std::max<int64_t>(slot, kSlotAlign);
    SegList sl{};
    sl.dev = (const Segment *)c->bsegs.p;
    CGH_TRY(ev_consts(ev, sl, n_frames, max_count, slots, s));
    FrameList fl{};
    fl.dev = (const FrameDesc *)c->bframes.p;
    return ev_run_direct(ev, mode, fl, n_frames, slot, out, nullptr, false, s);
}

// Matrix-core modes over many frames: frames are grouped so that each
// group's factors fit the workspace budget; per group one constants launch,
// one factor launch (all frames side by side along K) and one persistent
// GEMM launch over (frame, tile) items, largest K first.
cgh_status eval_batch_gemm(cgh_ctx *c, int mode, const cgh_frame *frames, int n_frames,
                           float *out, hipStream_t s, const TuneEntry *force = nullptr)
{
    const ModeInfo mi = mode_info(mode);
    const int64_t plane = (int64_t)c->width * c->height;
    // tile shape: the batch's tuned shape, else the single-hologram tuned (or
    // default) shape of its largest frame
    int64_t max_count = 0;
    for (int f = 0; f < n_frames; ++f)
        max_count = std::max(max_count, frames[f].point_count);
    const int64_t max_slots = std::max<int64_t>(round_up(max_count, kSlotAlign), kSlotAlign);
    const TuneEntry *t = force ? force : find_tuned(c, batch_tune_key(c, mode, max_slots / mi.kbp));
    if (!t)
        t = find_tuned(c, tune_key(c, mode, max_slots / mi.kbp, c->height));
    Plan p = plan_gemm(c->height, c->width, max_slots, mi, t);
    const size_t per_slot = (size_t)(p.g.mblocks + p.g.nblocks) * kFragLines * mi.line_bytes();
    const int64_t budget = std::max<int64_t>(
        (int64_t)workspace_budget() / (int64_t)per_slot / kSlotAlign * kSlotAlign, kSlotAlign);

    // Frames into groups whose padded slots fit the budget (a frame larger
    // than the budget is a group of its own): as few groups as the budget
    // allows, filled largest frame first, each frame into the least-loaded
    // group with room, so that every group holds a balanced share of large
    // and small frames and its (frame, tile) items spread evenly over the
    // workgroups (consecutive runs of frames could leave a last group of a
    // few large frames, whose launch is one item long).  All groups' segments
    // and work items go to the device in one table each, so a repeated call
    // (and its graph capture) copies nothing.
    auto padded_slots = [&](int f) { return round_up(frames[f].point_count, kSlotAlign); };
    std::vector<int> order(n_frames);
    for (int f = 0; f < n_frames; ++f)
        order[f] = f;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return frames[a].point_count > frames[b].point_count;
    });
    int64_t all_slots = 0;
    for (int f = 0; f < n_frames; ++f)
        all_slots += padded_slots(f);
    std::vector<std::vector<int>> members((size_t)std::max<int64_t>(
        1, std::min<int64_t>(n_frames, (all_slots + budget - 1) / budget)));
    std::vector<int64_t> load(members.size(), 0);
    for (int f : order) {
        const int64_t ps = padded_slots(f);
        int best = -1;
        for (int g = 0; g < (int)members.size(); ++g)
            if ((members[g].empty() || load[g] + ps <= budget) &&
                (best < 0 || load[g] < load[best]))
                best = g;
        if (best < 0) {
            members.emplace_back();
            load.push_back(0);
            best = (int)members.size() - 1;
        }
        members[best].push_back(f);
        load[best] += ps;
    }

    struct Group {
        int seg0, nseg;
        int item0, nitem;
        int64_t slots, max_count;
    };
    std::vector<Group> groups;
    std::vector<Segment> segs;
    std::vector<BatchItem> items;
    for (auto &mem : members) {
        if (mem.empty())
            continue;
        std::sort(mem.begin(), mem.end());
        Group gr{(int)segs.size(), 0, (int)items.size(), 0, 0, 0};
        for (int f : mem) {
            const int64_t ps = padded_slots(f);
            segs.push_back({frames[f].point_offset, frames[f].point_count, gr.slots,
                            frames[f].wavelength});
            for (int tm = 0; tm < p.tiles_m; ++tm)
                for (int tn = 0; tn < p.tiles_n; ++tn)
                    items.push_back({gr.slots / mi.kbp, ps / mi.kbp, f * plane, tm, tn});
            gr.slots += ps;
            gr.max_count = std::max(gr.max_count, frames[f].point_count);
        }
        gr.nseg = (int)segs.size() - gr.seg0;
        gr.nitem = (int)items.size() - gr.item0;
        std::stable_sort(items.begin() + gr.item0, items.end(),
                         [](const BatchItem &x, const BatchItem &y) { return x.kblocks > y.kblocks; });
        groups.push_back(gr);
    }
    CGH_TRY(upload_small(c, c->bsegs, segs.data(), segs.size() * sizeof(Segment), s,
                         "segment table upload"));
    CGH_TRY(upload_small(c, c->items, items.data(), items.size() * sizeof(BatchItem), s,
                         "work list upload"));
    CGH_HIP(ensure_ws(c, c->counter, sizeof(int)), "counter allocation");
    int64_t max_group_slots = kSlotAlign;
    for (auto &gr : groups)
        max_group_slots = std::max(max_group_slots, gr.slots);
    CtxWs ws(c);
    Eval ev = ctx_eval(c, &ws);
    FactorSet fs;
    fs.hl = mi.hl;
    fs.amb = p.g.mblocks;
    fs.anb = p.g.nblocks;
    fs.kblocks = max_group_slots / mi.kbp;
    void *fp = nullptr, *cp = nullptr;
    CGH_TRY(ws.get(Role::Factors, (size_t)fs.bytes(), &fp));
    fs.base = (char *)fp;
    // the largest group's constants first, so no group grows the buffer
    CGH_TRY(ws.get(Role::Consts, consts_bytes(max_group_slots), &cp));
    for (auto &gr : groups) {
        const int64_t total = std::max<int64_t>(gr.slots, kSlotAlign);
        SegList sl{};
        sl.dev = (const Segment *)c->bsegs.p + gr.seg0;
        CGH_TRY(ev_consts(ev, sl, gr.nseg, gr.max_count, total, s));
        GemmPlan g = p.g;
        g.kblocks = total / mi.kbp;
        FactorSet gfs = fs;            // this group's K extent
        gfs.kblocks = g.kblocks;
        {
            Bracket br(c, mi.fac_name, s);
            CGH_HIP(launch_factors(ev.pc, 0, c->width, c->height, false, g.kblocks, g.mblocks,
                                   g.nblocks, mi.ft, gfs, s),
                    "factor launch");
            br.done();
        }
        {
            Bracket br(c, mi.batch_name, s);
            CGH_HIP(launch_gemm_batch(g, mi.ft, gfs, (const BatchItem *)c->items.p + gr.item0,
                                      gr.nitem, (int *)c->counter.p, c->height, c->width, out,
                                      std::min(256, gr.nitem), s),
                    "batched gemm launch");
            br.done();
        }
    }
    return CGH_OK;
}

// The kernel sequence of one batch call, without graph handling.
cgh_status batch_sequence(cgh_ctx *c, const cgh_frame *frames, int n_frames, int mode, float *out,
                          hipStream_t s, const TuneEntry *force = nullptr)
{
    const int64_t plane = (int64_t)c->width * c->height;
    if (is_direct(mode)) {
        int64_t total = 0;
        for (int f = 0; f < n_frames; ++f)
            total += round_up(frames[f].point_count, kSlotAlign);
        if (total <= chunk_slots(ctx_geo(c), mode))
            return eval_batch_direct(c, mode, frames, n_frames, out, s, force);
        CtxWs ws(c);
        Eval ev = ctx_eval(c, &ws);
        const int64_t chunk = chunk_slots(ev.g, mode);
        for (int f = 0; f < n_frames; ++f)
            CGH_TRY(ev_one(ev, mode, frames[f].point_offset, frames[f].point_count,
                           frames[f].wavelength, out + f * plane, false, chunk, s));
        return CGH_OK;
    }
    return eval_batch_gemm(c, mode, frames, n_frames, out, s, force);
}

bool same_frames(const std::vector<cgh_frame> &a, const cgh_frame *b, int n)
{
    if ((int)a.size() != n)
        return false;
    for (int i = 0; i < n; ++i)
        if (a[i].point_offset != b[i].point_offset || a[i].point_count != b[i].point_count ||
            a[i].wavelength != b[i].wavelength)
            return false;
    return true;
}

// ------------------------------------------------------------ tune cache
// JSON lines, one choice per line:
// {"key": "gfx950/1920x1080/mode1/kb10", "bm": 192, "bn": 384, "wm": 2, "wn": 4,
//  "stages": 2, "splits": 8, "rows": 0, "us": 220.3}
const char *tune_cache_path()
{
    const char *p = std::getenv("CGH_TUNE_CACHE");
    return p && *p ? p : nullptr;
}

void put_tuned(cgh_ctx *c, const TuneEntry &e)
{
    for (auto &t : c->tuned)
        if (t.key == e.key) {
            t = e;
            return;
        }
    c->tuned.push_back(e);
}

void load_tune_cache(cgh_ctx *c)
{
    const char *path = tune_cache_path();
    if (!path)
        return;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char key[256];
        TuneEntry e;
        if (std::sscanf(line,
                        " {\"key\": \"%255[^\"]\", \"bm\": %d, \"bn\": %d, \"wm\": %d, \"wn\": %d, "
                        "\"stages\": %d, \"splits\": %d, \"rows\": %d, \"us\": %lf",
                        key, &e.bm, &e.bn, &e.wm, &e.wn, &e.stages, &e.splits, &e.rows,
                        &e.us) == 9) {
            e.key = key;
            put_tuned(c, e);   // later lines win
        }
    }
    std::fclose(f);
}

void append_tune_cache(const TuneEntry &e)
{
    const char *path = tune_cache_path();
    if (!path)
        return;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"bm\": %d, \"bn\": %d, \"wm\": %d, \"wn\": %d, "
                 "\"stages\": %d, \"splits\": %d, \"rows\": %d, \"us\": %.3f}\n",
                 e.key.c_str(), e.bm, e.bn, e.wm, e.wn, e.stages, e.splits, e.rows, e.us);
    std::fclose(f);
}

// Average duration (us) of `reps` launches of fn on stream s, after one warm-up.
template <typename F>
cgh_status time_launches(F fn, int reps, hipStream_t s, double *us)
{
    hipEvent_t a = nullptr, b = nullptr;
    CGH_HIP(hipEventCreate(&a), "hipEventCreate");
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    e = fn();
    if (e == hipSuccess)
        e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
        e = fn();
    if (e == hipSuccess)
        e = hipEventRecord(b, s);
    if (e == hipSuccess)
        e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess)
        return hip_fail(e, "tuning launch");
    *us = 1e3 * ms / reps;
    return CGH_OK;
}

// The device exists and is a gfx950; `arch` receives its name.
cgh_status check_device(int32_t device, std::string &arch)
{
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
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    return CGH_OK;
}

// ------------------------------------------- evaluation without allocation
// Fixed workspace of cgh_compute_noalloc: one array per device (each device
// holds its own copy, at its own address, until the process ends).  In host
// code the name is only a stand-in: kernels get the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxDevices] = {};   // device address per device, once resolved

// This device's scratch address (the device is current).  The first call on
// a device checks it is a gfx950, resolves the address and raises the GEMM
// kernels' LDS limit.
cgh_status scratch_on(int device, char **p)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        int count = 0;
        CGH_HIP(hipGetDeviceCount(&count), "hipGetDeviceCount");
        if (device >= count)
            return fail(CGH_EDEVICE, "device index out of range");
        hipDeviceProp_t prop;
        CGH_HIP(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(CGH_EDEVICE, "this library is built for gfx950");
        void *ptr = nullptr;
        CGH_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static scratch address");
        if (!ptr)
            return fail(CGH_EDEVICE, "static scratch address is NULL");
        CGH_HIP(gemm_prepare_kernels(), "GEMM kernel attributes");
        g_scratch_dev[device] = (char *)ptr;
    }
    *p = g_scratch_dev[device];
    return CGH_OK;
}

// Regions of the scratch array, handed out in order of first request; a
// later request of a role must fit the region it got first.
struct ArenaWs final : Ws {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    size_t off[(int)Role::Count] = {}, len[(int)Role::Count] = {};
    bool set[(int)Role::Count] = {};
    cgh_status get(Role role, size_t bytes, void **p) override
    {
        const int r = (int)role;
        bytes = (bytes + 255) / 256 * 256;
        if (!set[r]) {
            if (bytes > cap - used)
                return fail(CGH_EINVAL, "evaluation does not fit the static scratch");
            off[r] = used;
            len[r] = bytes;
            set[r] = true;
            used += bytes;
        } else if (bytes > len[r]) {
            return fail(CGH_EINVAL, "evaluation does not fit the static scratch");
        }
        *p = base + off[r];
        return CGH_OK;
    }
};

// Point chunk (slots) and bytes of split partials of a no-allocation
// evaluation, both within kScratchBytes: at most half of it for the partial
// planes of the split counts the default plan would use, the rest for the
// constants and the tables or factors of one chunk.  *chunk = 0 when not even
// one slot group fits.
void noalloc_plan(const Geo &g, int mode, int64_t *chunk, size_t *partial_cap)
{
    const size_t plane = (size_t)g.width * g.height * sizeof(float);
    int splits = 1;
    if (is_direct(mode)) {
        Eval probe;
        probe.g = g;
        splits = direct_splits(probe, mode);
    } else {
        splits = plan_gemm(g.height, g.width, (int64_t)1 << 20, mode_info(mode)).g.splits;
    }
    const size_t want = splits > 1 ? (size_t)splits * plane : 0;
    const size_t per_slot = 40 + bytes_per_slot(g, mode, false);
    const size_t slack = 8 * 256;        // 256-byte rounding of every region
    for (int attempt = 0; attempt < 2; ++attempt) {
        size_t part = attempt == 0 ? std::min(want, kScratchBytes / 2) / plane * plane : 0;
        if (part < 2 * plane)
            part = 0;
        const int64_t ch =
            (int64_t)((kScratchBytes - part - slack) / per_slot) / kSlotAlign * kSlotAlign;
        if (ch >= kSlotAlign) {
            *chunk = ch;
            *partial_cap = part;
            return;
        }
    }
    *chunk = 0;
    *partial_cap = 0;
}

// First step of the wavefront-recording method for the context's cloud: the
// per-point constants in the constants workspace, then the n x n plane.
cgh_status wrm_record(cgh_ctx *c, double zw, int n, float2 *field, hipStream_t s)
{
    const int64_t np = c->n;
    const size_t cap = (size_t)std::max<int64_t>(np, 1);
    void *p = nullptr;
    const size_t groups = (cap + kWrmGroup - 1) / kWrmGroup;
    CGH_HIP(ensure_ws(c, c->consts, cap * kWrmBytesPerPoint + groups * sizeof(float4) + 4 * 256),
            "workspace allocation");
    p = c->consts.p;
    char *b = (char *)p;
    auto take = [&](size_t bytes) {
        char *r = b;
        b += (bytes + 255) / 256 * 256;
        return r;
    };
    WrmConsts wc;
    wc.box = (float4 *)take(cap * sizeof(float4));
    wc.raw = (float4 *)take(cap * sizeof(float4));
    wc.gbox = (float4 *)take(groups * sizeof(float4));
    wc.next_tile = (int *)take(sizeof(int));
    {
        Bracket br(c, "wrm_consts", s);
        CGH_HIP(launch_wrm_consts(pts_x(c), pts_y(c), pts_z(c), pts_a(c), np, n, c->pitch,
                                  c->wavelength, zw, wc, s),
                "recording constants launch");
        br.done();
    }
    int chunks = wrm_record_chunks(np, n);
    if (const char *env = std::getenv("CGH_WRM_CHUNKS")) {
        const int v = std::atoi(env);
        if (v >= 1 && v <= 16 && np > kWrmQueueMinPoints)
            chunks = v;
    }
    // chunks 1 .. chunks-1 take an n x n plane of workspace each, within the budget
    const size_t plane = (size_t)n * n * sizeof(float2);
    chunks = (int)std::min<size_t>((size_t)chunks, 1 + workspace_budget() / plane);
    float2 *parts = nullptr;
    if (chunks > 1) {
        CGH_HIP(ensure_ws(c, c->partials, (size_t)(chunks - 1) * n * n * sizeof(float2)),
                "workspace allocation");
        parts = (float2 *)c->partials.p;
    }
    Bracket br(c, "wrm_record", s);
    CGH_HIP(launch_wrm_record(wc, np, n, c->pitch, c->wavelength, zw, chunks, field, parts, s),
            "recording launch");
    br.done();
    return CGH_OK;
}

// Common checks of the single-hologram compute calls.
cgh_status check_compute(cgh_ctx *c, int mode, const void *out)
{
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    if (!out)
        return fail(CGH_EINVAL, "output is NULL");
    CGH_TRY(check_mode(mode));
    if (!c->uploaded)
        return fail(CGH_ESTATE, "no points uploaded");
    return CGH_OK;
}

}  // namespace

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

int32_t cgh_version(void) { return 10100; }

// ------------------------------------------------------ Fresnel diffraction
struct cgh_fresnel {
    int device = 0;
    int n = 0, m = 0;              // field size, log2 of the padded size 2n
    double pitch = 0.0, wavelength = 0.0, z = 0.0;
    float2 scale{0.0f, 0.0f};      // exp(i 2 pi z / lambda) / (i lambda z) p^2 / (2n)^2
    DevBuf tw, hc, x, y;          // y only for the pipeline with transposes
};

cgh_status cgh_fresnel_create(cgh_fresnel **out, int32_t n, double pitch_m, double wavelength_m,
                              double z_m, int32_t device)
{
    g_last_error.clear();
    if (!out)
        return fail(CGH_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 16 || n > 8192 || (n & (n - 1)) != 0)
        return fail(CGH_EINVAL, "n must be a power of two in [16, 8192]");
    if (!finite_pos(pitch_m))
        return fail(CGH_EINVAL, "pitch must be finite and > 0");
    if (!finite_pos(wavelength_m))
        return fail(CGH_EINVAL, "wavelength must be finite and > 0");
    if (!std::isfinite(z_m) || z_m == 0.0)
        return fail(CGH_EINVAL, "z must be finite and non-zero");
    if (device < 0)
        return fail(CGH_EINVAL, "device index must be >= 0");
    std::string arch;
    CGH_TRY(check_device(device, arch));
    DeviceGuard g;
    CGH_HIP(g.set(device), "hipSetDevice");
    cgh_fresnel *f = new (std::nothrow) cgh_fresnel();
    if (!f)
        return fail(CGH_ENOMEM, "plan allocation");
    f->device = device;
    f->n = n;
    f->pitch = pitch_m;
    f->wavelength = wavelength_m;
    f->z = z_m;
    int m = 0;
    while ((1 << m) < 2 * n)
        ++m;
    f->m = m;
    const int64_t L = (int64_t)1 << m;
    // exp(i 2 pi frac(z / lambda)) (-i) p^2 / (lambda z L^2), in FP64
    const double two_pi = 6.28318530717958647692;
    const double zr = z_m / wavelength_m - std::floor(z_m / wavelength_m);
    const double mag = pitch_m * pitch_m / (wavelength_m * z_m) / ((double)L * (double)L);
    f->scale = float2{(float)(mag * std::sin(two_pi * zr)), (float)(-mag * std::cos(two_pi * zr))};
    hipError_t e = fresnel_prepare_kernels();
    if (e == hipSuccess)
        e = f->tw.ensure(fresnel_twiddle_bytes(m));
    if (e == hipSuccess)
        e = f->hc.ensure((size_t)L * sizeof(float2));
    if (e == hipSuccess)
        e = f->x.ensure((size_t)n * n * sizeof(float2));
    if (e == hipSuccess && fresnel_workspace_planes(m) > 1)
        e = f->y.ensure((size_t)n * n * sizeof(float2));
    if (e == hipSuccess)
        e = fresnel_tables(n, m, pitch_m * pitch_m / (2.0 * wavelength_m * z_m),
                           (float2 *)f->tw.p, (float2 *)f->hc.p, nullptr);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        f->tw.release();
        f->hc.release();
        f->x.release();
        f->y.release();
        delete f;
        return hip_fail(e, "Fresnel plan set-up");
    }
    *out = f;
    return CGH_OK;
}

cgh_status cgh_fresnel_run(cgh_fresnel *f, const float *u_dev, float *out_dev, void *stream)
{
    g_last_error.clear();
    if (!f)
        return fail(CGH_EINVAL, "plan is NULL");
    if (!u_dev || !out_dev)
        return fail(CGH_EINVAL, "field or output is NULL");
    if ((uintptr_t)u_dev % 8 != 0 || (uintptr_t)out_dev % 8 != 0)
        return fail(CGH_EINVAL, "field and output must be 8-byte aligned (complex float pairs)");
    DeviceGuard g;
    CGH_HIP(g.set(f->device), "hipSetDevice");
    CGH_HIP(fresnel_run(f->n, f->m, (const float2 *)f->tw.p, (const float2 *)f->hc.p, f->scale,
                        (const float2 *)u_dev, (float2 *)out_dev, (float2 *)f->x.p,
                        (float2 *)f->y.p, (hipStream_t)stream),
            "Fresnel diffraction launch");
    return CGH_OK;
}

void cgh_fresnel_destroy(cgh_fresnel *f)
{
    if (!f)
        return;
    DeviceGuard g;
    if (g.set(f->device) == hipSuccess)
        (void)hipDeviceSynchronize();
    f->tw.release();
    f->hc.release();
    f->x.release();
    f->y.release();
    delete f;
}

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

    std::string arch;
    CGH_TRY(check_device(device, arch));
    {
        DeviceGuard g;
        CGH_HIP(g.set(device), "hipSetDevice");
        CGH_HIP(gemm_prepare_kernels(), "GEMM kernel attributes");
    }

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
    c->arch = arch;
    load_tune_cache(c);
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
    if (c->order_ev)
        (void)hipEventDestroy(c->order_ev);
    c->staging.release();
    for (DevBuf *b : {&c->points, &c->consts, &c->tab_u, &c->tab_v, &c->tab_x, &c->tab_y,
                      &c->fac, &c->partials, &c->tune_out, &c->field, &c->bsegs, &c->bframes,
                      &c->items, &c->counter})
        b->release();
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
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    const int64_t cap = std::max<int64_t>(n, 1);
    if (cap > c->n_cap || !c->points.p) {
        // queued work (on any stream) may still read the old cloud
        CGH_HIP(hipDeviceSynchronize(), "device synchronise");
        c->points.release();
        CGH_HIP(c->points.ensure((size_t)cap * 4 * sizeof(float)), "point allocation");
        c->n_cap = cap;
        ++c->ws_generation;
        drop_graph(c);
    }
    float *d = (float *)c->points.p;
    const float *src[4] = {x, y, z, amp};
    if (n > 0) {
        if (where == CGH_MEM_HOST)   // queued work may still read the old cloud
            CGH_HIP(hipStreamSynchronize(s), "stream synchronise");
        for (int k = 0; k < 4; ++k) {
            if (where == CGH_MEM_HOST)
                CGH_HIP(hipMemcpy(d + k * c->n_cap, src[k], (size_t)n * sizeof(float),
                                  hipMemcpyHostToDevice),
                        "point upload");
            else
                CGH_HIP(hipMemcpyAsync(d + k * c->n_cap, src[k], (size_t)n * sizeof(float),
                                       hipMemcpyDeviceToDevice, s),
                        "point upload");
        }
    }
    c->n = n;
    c->uploaded = true;
    return CGH_OK;
}

cgh_status cgh_compute(cgh_ctx *c, cgh_mode mode, float *out_dev, void *stream)
{
    g_last_error.clear();
    CGH_TRY(check_compute(c, mode, out_dev));
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    return eval_ctx(c, mode, out_dev, false, s);
}

cgh_status cgh_compute_complex(cgh_ctx *c, cgh_mode mode, float *out_dev, void *stream)
{
    g_last_error.clear();
    CGH_TRY(check_compute(c, mode, out_dev));
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    return eval_ctx(c, mode, out_dev, true, s);
}

cgh_status cgh_kinoform(cgh_ctx *c, cgh_mode mode, uint8_t *out_dev, void *stream)
{
    g_last_error.clear();
    CGH_TRY(check_compute(c, mode, out_dev));
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    const int64_t plane = (int64_t)c->width * c->height;
    CGH_HIP(ensure_ws(c, c->field, (size_t)plane * 2 * sizeof(float)), "field allocation");
    float *field = (float *)c->field.p;
    CGH_TRY(eval_ctx(c, mode, field, true, s));
    Bracket br(c, "kinoform", s);
    CGH_HIP(launch_kinoform(field, field + plane, plane, out_dev, s), "kinoform launch");
    br.done();
    return CGH_OK;
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
    CGH_TRY(check_mode(mode));
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
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s))
        return fail(CGH_ESTATE, "the stream is capturing: cgh_batch_compute records its own "
                                "graph");
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    // Replay: same mode, frames and output as the captured call, and no
    // workspace buffer moved since (a move drops the graph).  The graph reads
    // only the batch tables, which no other call writes.
    if (c->graph_exec && !c->profiling && c->graph_mode == (int)mode && c->graph_out == out_dev &&
        c->graph_generation == c->ws_generation && same_frames(c->graph_frames, frames, n_frames)) {
        CGH_HIP(hipGraphLaunch(c->graph_exec, s), "hipGraphLaunch");
        return CGH_OK;
    }
    drop_graph(c);
    CGH_TRY(batch_sequence(c, frames, n_frames, (int)mode, out_dev, s));
    if (c->profiling || s == nullptr)
        return CGH_OK;
    // Capture the same sequence for replay.  Its tables and workspace are now
    // in place, so the captured pass issues kernel launches only; if anything
    // else would be recorded, the capture is abandoned and later calls run
    // eagerly.
    const uint64_t gen = c->ws_generation;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return CGH_OK;
    }
    const cgh_status cst = batch_sequence(c, frames, n_frames, (int)mode, out_dev, s);
    const hipError_t ce = hipStreamEndCapture(s, &graph);
    hipGraphExec_t exec = nullptr;
    if (cst == CGH_OK && ce == hipSuccess && graph && c->ws_generation == gen &&
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
        c->graph_exec = exec;
        c->graph_mode = (int)mode;
        c->graph_out = out_dev;
        c->graph_generation = c->ws_generation;
        c->graph_frames.assign(frames, frames + n_frames);
    }
    if (graph)
        (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    g_last_error.clear();
    return CGH_OK;
}

cgh_status cgh_compute_noalloc(int32_t width, int32_t height, double pitch_m,
                               double wavelength_m, const float *x_dev, const float *y_dev,
                               const float *z_dev, const float *amp_dev, int64_t n, cgh_mode mode,
                               float *out_dev, int32_t device, void *stream)
{
    g_last_error.clear();
    if (width < 1 || width > 65536 || height < 1 || height > 65536)
        return fail(CGH_EINVAL, "width and height must be in [1, 65536]");
    if (!finite_pos(pitch_m))
        return fail(CGH_EINVAL, "pitch must be finite and > 0");
    if (!finite_pos(wavelength_m))
        return fail(CGH_EINVAL, "wavelength must be finite and > 0");
    if (n < 0 || n > ((int64_t)1 << 34))
        return fail(CGH_EINVAL, "n must be in [0, 2^34]");
    if (n > 0 && (!x_dev || !y_dev || !z_dev || !amp_dev))
        return fail(CGH_EINVAL, "point arrays must be non-NULL when n > 0");
    if (!out_dev)
        return fail(CGH_EINVAL, "output is NULL");
    CGH_TRY(check_mode(mode));
    if (device < 0 || device >= kMaxDevices)
        return fail(CGH_EINVAL, "device index must be in [0, 64)");
    Geo g;
    g.width = width;
    g.height = height;
    g.wpad = (int)round_up(width, kLinePad);
    g.hpad = (int)round_up(height, kLinePad);
    g.pitch = pitch_m;
    int64_t chunk = 0;
    size_t part = 0;
    noalloc_plan(g, mode, &chunk, &part);
    if (chunk == 0)
        return fail(CGH_EINVAL, "the hologram is too large for the 32 MiB static scratch in this "
                                "mode (one group of 32 points does not fit)");
    DeviceGuard dg;
    CGH_HIP(dg.set(device), "hipSetDevice");
    char *base = nullptr;
    CGH_TRY(scratch_on(device, &base));
    ArenaWs ws;
    ws.base = base;
    ws.cap = kScratchBytes;
    Eval ev;
    ev.g = g;
    ev.x = x_dev;
    ev.y = y_dev;
    ev.z = z_dev;
    ev.a = amp_dev;
    ev.ws = &ws;
    ev.partial_cap = part;
    return ev_one(ev, mode, 0, n, wavelength_m, out_dev, false, chunk, (hipStream_t)stream);
}

cgh_status cgh_wrm_record(cgh_ctx *c, double plane_z_m, int32_t n, float *field_dev,
                          void *stream)
{
    g_last_error.clear();
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    if (!field_dev || (uintptr_t)field_dev % 8 != 0)
        return fail(CGH_EINVAL, "field must be a non-NULL, 8-byte aligned device buffer");
    if (!std::isfinite(plane_z_m))
        return fail(CGH_EINVAL, "plane distance must be finite");
    if (n < 16 || n > 8192 || (n & (n - 1)) != 0)
        return fail(CGH_EINVAL, "n must be a power of two in [16, 8192]");
    if (!c->uploaded)
        return fail(CGH_ESTATE, "no points uploaded");
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    return wrm_record(c, plane_z_m, n, (float2 *)field_dev, s);
}

cgh_status cgh_wrm_compute(cgh_ctx *c, cgh_fresnel *plan, float *field_dev, float *out_dev,
                           void *stream)
{
    g_last_error.clear();
    if (!c || !plan)
        return fail(CGH_EINVAL, "context or plan is NULL");
    if (!field_dev || (uintptr_t)field_dev % 8 != 0)
        return fail(CGH_EINVAL, "field must be a non-NULL, 8-byte aligned device buffer");
    if (!out_dev)
        return fail(CGH_EINVAL, "output is NULL");
    if (plan->device != c->device)
        return fail(CGH_EINVAL, "the plan and the context are on different devices");
    if (plan->pitch != c->pitch || plan->wavelength != c->wavelength)
        return fail(CGH_EINVAL, "the plan's pitch and wavelength must equal the context's");
    if (!(plan->z > 0.0))
        return fail(CGH_EINVAL, "the plan's distance (the virtual plane's) must be > 0");
    if (plan->n < c->width || plan->n < c->height || (plan->n - c->width) % 2 != 0 ||
        (plan->n - c->height) % 2 != 0)
        return fail(CGH_EINVAL, "the plane must hold the hologram centred: n >= width, height, "
                                "with n - width and n - height even");
    if (!c->uploaded)
        return fail(CGH_ESTATE, "no points uploaded");
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    float2 *field = (float2 *)field_dev;
    CGH_TRY(wrm_record(c, plan->z, plan->n, field, s));
    {
        Bracket br(c, "fresnel_diffraction", s);
        CGH_HIP(fresnel_run(plan->n, plan->m, (const float2 *)plan->tw.p,
                            (const float2 *)plan->hc.p, plan->scale, field, field,
                            (float2 *)plan->x.p, (float2 *)plan->y.p, s),
                "Fresnel diffraction launch");
        br.done();
    }
    Bracket br(c, "hologram_window", s);
    CGH_HIP(launch_window_real(field, plan->n, (plan->n - c->width) / 2,
                               (plan->n - c->height) / 2, c->width, c->height, out_dev, s),
            "window launch");
    br.done();
    return CGH_OK;
}

cgh_status cgh_tune_batch(cgh_ctx *c, const cgh_frame *frames, int32_t n_frames, cgh_mode mode,
                          float *out_dev, int32_t repeats, char *report, int32_t report_len,
                          void *stream)
{
    g_last_error.clear();
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    if (!frames || n_frames < 1 || n_frames > 65535)
        return fail(CGH_EINVAL, "frames must be non-NULL with n_frames in [1, 65535]");
    if (!out_dev)
        return fail(CGH_EINVAL, "output is NULL");
    CGH_TRY(check_mode(mode));
    if (repeats < 1 || repeats > 1000)
        return fail(CGH_EINVAL, "repeats must be in [1, 1000]");
    if (report_len < 0 || (report_len > 0 && !report))
        return fail(CGH_EINVAL, "bad report buffer");
    if (!c->uploaded)
        return fail(CGH_ESTATE, "no points uploaded");
    int64_t max_count = 0, total = 0;
    for (int f = 0; f < n_frames; ++f) {
        const cgh_frame &fr = frames[f];
        if (fr.point_offset < 0 || fr.point_count < 0 || fr.point_offset > c->n ||
            fr.point_count > c->n - fr.point_offset)
            return fail(CGH_EINVAL, "frame " + std::to_string(f) + " is outside the upload");
        if (!finite_pos(fr.wavelength))
            return fail(CGH_EINVAL, "frame " + std::to_string(f) + " has a bad wavelength");
        max_count = std::max(max_count, fr.point_count);
        total += round_up(fr.point_count, kSlotAlign);
    }
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s))
        return fail(CGH_ESTATE, "the stream is capturing");
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    drop_graph(c);
    const int64_t max_slots = round_up(std::max<int64_t>(max_count, 1), kSlotAlign);
    TuneEntry best;
    int tried = 0;
    auto try_one = [&](const TuneEntry &cand) -> cgh_status {
        double us = 0;
        cgh_status bst = CGH_OK;
        std::string msg;
        const cgh_status tst = time_launches(
            [&] {
                bst = batch_sequence(c, frames, n_frames, (int)mode, out_dev, s, &cand);
                if (bst == CGH_OK)
                    return hipSuccess;
                msg = g_last_error;
                return hipErrorLaunchFailure;
            },
            repeats, s, &us);
        if (bst != CGH_OK)
            return fail(bst, msg);
        if (tst != CGH_OK)
            return tst;
        ++tried;
        if (tried == 1 || us < best.us) {
            best = cand;
            best.us = us;
        }
        return CGH_OK;
    };
    if (is_direct(mode)) {
        if (total > chunk_slots(ctx_geo(c), mode))
            return fail(CGH_ENOTSUP, "the batch's tables exceed the workspace budget");
        best.key = batch_tune_key(c, mode, max_slots);
        for (int rows : {4, 8, 16}) {
            if (!direct_rows_ok(mode, rows))
                continue;
            TuneEntry cand;
            cand.key = best.key;
            cand.rows = rows;
            CGH_TRY(try_one(cand));
        }
    } else {
        const ModeInfo mi = mode_info(mode);
        const std::string key = batch_tune_key(c, mode, max_slots / mi.kbp);
        for (auto &sh : kShapes) {
            if (!gemm_tile_supported(sh[0], sh[1], sh[2], sh[3], sh[4]))
                continue;
            TuneEntry cand;
            cand.key = key;
            cand.bm = sh[0];
            cand.bn = sh[1];
            cand.wm = sh[2];
            cand.wn = sh[3];
            cand.stages = sh[4];
            CGH_TRY(try_one(cand));
        }
    }
    if (tried == 0)
        return fail(CGH_ENOTSUP, "no launch shape fits this batch");
    put_tuned(c, best);
    append_tune_cache(best);
    if (report_len > 0)
        std::snprintf(report, (size_t)report_len,
                      "%s: bm=%d bn=%d waves=%dx%d stages=%d rows=%d %.1f us per batch "
                      "(%d candidates)",
                      best.key.c_str(), best.bm, best.bn, best.wm, best.wn, best.stages,
                      best.rows, best.us, tried);
    return CGH_OK;
}

cgh_status cgh_tune(cgh_ctx *c, cgh_mode mode, int32_t repeats, char *report, int32_t report_len,
                    void *stream)
{
    g_last_error.clear();
    if (!c)
        return fail(CGH_EINVAL, "context is NULL");
    CGH_TRY(check_mode(mode));
    if (repeats < 1 || repeats > 1000)
        return fail(CGH_EINVAL, "repeats must be in [1, 1000]");
    if (report_len < 0 || (report_len > 0 && !report))
        return fail(CGH_EINVAL, "bad report buffer");
    if (!c->uploaded)
        return fail(CGH_ESTATE, "no points uploaded");
    DeviceGuard g;
    CGH_HIP(g.set(c->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    CallOrder order(c, s);
    CGH_HIP(order.enter(), "stream ordering");
    CGH_HIP(ensure_ws(c, c->tune_out, (size_t)c->width * c->height * sizeof(float)),
            "tuning output allocation");
    float *out = (float *)c->tune_out.p;
    CtxWs ws(c);
    Eval ev = ctx_eval(c, &ws);

    // the first point chunk of the cloud (at least one slot group)
    const int64_t count = std::min(c->n, chunk_slots(ev.g, mode));
    const int64_t slots = std::max<int64_t>(round_up(count, kSlotAlign), kSlotAlign);
    SegList sl{};
    sl.dev = nullptr;
    sl.one = {0, count, 0, c->wavelength};
    CGH_TRY(ev_consts(ev, sl, 1, count, slots, s));
    const FrameDesc fd{0, slots / kGroup, 0};

    TuneEntry best;
    int tried = 0;
    if (is_direct(mode)) {
        best.key = tune_key(c, mode, 0, c->height);
        CGH_TRY(ev_tables(ev, mode, slots, s));
        for (int splits : {1, 2, 4}) {
            int runs = 1;
            FrameList fl{};
            fl.dev = nullptr;
            fl.inl[0] = fd;
            if (splits > 1) {
                if (fd.groups < 4)
                    continue;
                fl = split_frames(fd, splits, 1, (int64_t)c->width * c->height, &runs);
                CGH_HIP(ensure_ws(c, c->partials,
                                  (size_t)runs * c->height * (size_t)c->width * sizeof(float)),
                        "split-K workspace allocation");
            }
            for (int rows : {4, 8, 16}) {
                if (!direct_rows_ok(mode, rows))
                    continue;
                double us = 0;
                CGH_TRY(time_launches(
                    [&] {
                        if (splits == 1)
                            return launch_direct_mode(ev, mode, fl, 1, rows, out, nullptr, false,
                                                      s);
                        hipError_t e = launch_direct_mode(ev, mode, fl, runs, rows,
                                                          (float *)c->partials.p, nullptr, false,
                                                          s);
                        if (e == hipSuccess)
                            e = launch_splitk_reduce((const float *)c->partials.p, runs,
                                                     c->height, c->width, out, c->width, false, s);
                        return e;
                    },
                    repeats, s, &us));
                ++tried;
                if (best.rows == 0 || us < best.us) {
                    best.rows = rows;
                    best.splits = splits;
                    best.us = us;
                }
            }
        }
    } else {
        const ModeInfo mi = mode_info(mode);
        const int64_t kblocks = slots / mi.kbp;
        best.key = tune_key(c, mode, kblocks, c->height);
        // factors padded to whole tiles of every candidate shape
        FactorSet fs;
        fs.hl = mi.hl;
        fs.kblocks = kblocks;
        for (auto &sh : kShapes) {
            fs.amb = std::max(fs.amb, (int)(round_up(c->height, sh[0]) / kFragLines));
            fs.anb = std::max(fs.anb, (int)(round_up(c->width, sh[1]) / kFragLines));
        }
        void *fp = nullptr;
        CGH_TRY(ws.get(Role::Factors, (size_t)fs.bytes(), &fp));
        fs.base = (char *)fp;
        CGH_HIP(launch_factors(ev.pc, 0, c->width, c->height, false, kblocks, fs.amb, fs.anb,
                               mi.ft, fs, s),
                "factor launch");
        for (auto &sh : kShapes) {
            if (!gemm_tile_supported(sh[0], sh[1], sh[2], sh[3], sh[4]))
                continue;
            const int tiles = (int)((c->height + sh[0] - 1) / sh[0] * ((c->width + sh[1] - 1) / sh[1]));
            // split counts around "one wave of workgroups fills the device",
            // each split >= 8 K blocks
            const int resident =
                256 * gemm_groups_per_cu(sh[0], sh[1], sh[2], sh[3], sh[4], mi.products);
            const int smax = (int)std::max<int64_t>(1, kblocks / 8);
            const int s0 = std::min(std::max(1, resident / tiles), smax);
            std::vector<int> cands{s0};
            for (int sp : {s0 - 1, s0 / 2, 2 * s0, 1}) {
                if (sp < 1 || sp > smax || sp * tiles > 2 * resident ||
                    std::find(cands.begin(), cands.end(), sp) != cands.end())
                    continue;
                cands.push_back(sp);
            }
            for (int sp : cands) {
                GemmPlan gp;
                gp.bm = sh[0];
                gp.bn = sh[1];
                gp.waves_m = sh[2];
                gp.waves_n = sh[3];
                gp.stages = sh[4];
                gp.splits = sp;
                gp.mblocks = (c->height + sh[0] - 1) / sh[0] * (sh[0] / kFragLines);
                gp.nblocks = (c->width + sh[1] - 1) / sh[1] * (sh[1] / kFragLines);
                gp.kblocks = kblocks;
                gp.products = mi.products;

                if (sp > 1)
                    CGH_HIP(ensure_ws(c, c->partials,
                                      (size_t)sp * c->height * (size_t)c->width * sizeof(float)),
                            "split-K workspace allocation");
                double us = 0;
                CGH_TRY(time_launches(
                    [&] {
                        hipError_t e = launch_gemm(gp, mi.ft, fs, c->height, c->width, out,
                                                   c->width, (float *)c->partials.p, false, s);
                        if (e == hipSuccess && sp > 1)
                            e = launch_splitk_reduce((const float *)c->partials.p, sp, c->height,
                                                     c->width, out, c->width, false, s);
                        return e;
                    },
                    repeats, s, &us));
                ++tried;
                if (best.bm == 0 || us < best.us) {
                    best.bm = sh[0];
                    best.bn = sh[1];
                    best.wm = sh[2];
                    best.wn = sh[3];
                    best.stages = sh[4];
                    best.splits = sp;
                    best.us = us;
                }
            }
        }
    }
    if (tried == 0)
        return fail(CGH_ENOTSUP, "no launch shape fits this hologram");
    put_tuned(c, best);
    append_tune_cache(best);
    if (report_len > 0)
        std::snprintf(report, (size_t)report_len,
                      "%s: bm=%d bn=%d waves=%dx%d stages=%d splits=%d rows=%d %.1f us "
                      "(%d candidates)",
                      best.key.c_str(), best.bm, best.bn, best.wm, best.wn, best.stages,
                      best.splits, best.rows, best.us, tried);
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
