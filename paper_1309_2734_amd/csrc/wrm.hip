// First step of the wavefront-recording method (Section 2.3): the object wave
// of the cloud recorded on a virtual plane between the points and the
// hologram, each point only over the disc its light crosses.
//
// The plane is an n x n grid of pitch p centred like the hologram, at
// distance zw from it; point j lies d_j = z_j - zw beyond it.  Its wave on
// the plane is the Fresnel form of Eq. (2) at depth d_j (without the constant
// per-point phase, as for the hologram itself), written over the disc of
// radius r_j = lambda d_j / (2 p) -- beyond it the chirp's local frequency
// r / (lambda d_j) exceeds the grid's 1 / (2 p) -- so
//     u_w[m][c] = sum over j with d_j > 0 and dx^2 + dy^2 <= r_j^2 of
//                 A_j exp(i 2 pi beta_j ((c - cx_j)^2 + (m - cy_j)^2)),
//     dx = (c - (n-1)/2) p - x_j,  dy = (m - (n-1)/2) p - y_j,
//     beta_j = p^2 / (2 lambda d_j),  cx_j = (n-1)/2 + x_j / p,  cy_j likewise.
//
// Membership of a sample in a disc is a decision floating point takes, so it
// is taken exactly as the definition states it: differences in metres,
// squared and summed in FP64, against r_j^2 in FP64, with no fused
// multiply-add anywhere in this file (the contraction pragma below).  The
// phase is reduced per (point, column) and per (point, row) in FP64, as for
// the hologram; each reduced part gets its FP32 cosine and sine, and a
// sample takes their product:
//     A cos(2 pi (U + V)) = A cos 2piU cos 2piV - A sin 2piU sin 2piV,
//     A sin(2 pi (U + V)) = A sin 2piU cos 2piV + A cos 2piU sin 2piV.
//
// Mapping: a workgroup of eight waves owns a tile of 64 columns x 32 rows;
// a wave owns a 16 x 16 sub-tile, a lane 4 rows of one column of it.  The
// workgroup walks the cloud in index order, one group of 1024 points per
// round, skipping groups whose disc bounding box (made by the constants
// kernel) misses the tile: each thread tests two points' discs against the
// tile's box (a conservative FP32 test that only decides what to skip; the
// next round's boxes and raw inputs load meanwhile), and the hit points,
// compacted in index order (their places from a shuffle scan of the
// round's 16 hit-mask counts), go to LDS in batches of up to 32.  The first
// wave evaluates a batch's FP64 constants, one lane per hit, from the raw
// inputs (by the one function the culling box also uses), and the set of
// sub-tiles each hit's disc can reach (the same FP32 test per sub-tile).
// Per batch the workgroup tabulates in LDS each hit's column terms (dx^2,
// A cos 2piU, A sin 2piU) for the 64 columns and row terms (dy^2, cos 2piV,
// sin 2piV) for the 32 rows; then every wave adds to its 16 x 16 samples,
// in index order, the hits that can reach them, branch-free (a sample
// outside the disc adds zero products).  Every sample's sum is formed in
// point order by one lane: deterministic, with no atomics.  Large clouds
// reach few tiles with a lot of work each, so their tiles come from a
// queue drained by persistent workgroups (row-major order, the next free
// workgroup takes the next item), and their points are cut into a few
// chunks of consecutive groups: a (tile, chunk) item is one workgroup's,
// each chunk is recorded as a plane of its own, and the planes are added
// in chunk order afterwards (still one fixed order per sample).
#pragma clang fp contract(off)

#include <algorithm>

#include "common.h"

namespace cgh {
namespace {

constexpr int kTileCols = 64;
constexpr int kTileRows = 32;
constexpr int kSub = 16;                           // a wave's sub-tile: 16 x 16 samples
constexpr int kSubX = kTileCols / kSub;            // sub-tiles per tile row
constexpr int kLaneRows = kSub * kSub / 64;        // samples (rows) per lane
constexpr int kWaves = kSubX * (kTileRows / kSub);
constexpr int kThreads = 64 * kWaves;
static_assert(kWaves == 8 && kLaneRows == 4, "eight waves of 16 x 16 samples");
constexpr int kPerThread = 2;                      // points a thread tests per round
constexpr int kRound = kPerThread * kThreads;      // points per round = per group
static_assert(kRound == kWrmGroup, "a recording round covers one point group");
constexpr int kMasks = kPerThread * kWaves;        // hit masks of a round
static_assert((kMasks & (kMasks - 1)) == 0 && kMasks <= 64, "a round's masks are scanned in a wave");
constexpr int kBatch = 32;                         // hits tabulated at once
static_assert(kBatch <= 64, "a batch's constants are one wave's");

// Disc of the point with box b (cx, cy, radius in samples, -) against a
// sample box: a conservative FP32 test that only decides what to skip.
__device__ __forceinline__ float reach_of(float4 b) { return b.z * 1.0001f + 0.05f; }
__device__ __forceinline__ bool box_hit(float4 b, float bx0, float bx1, float by0, float by1)
{
    const float ex = fmaxf(fmaxf(bx0 - b.x, b.x - bx1), 0.0f);
    const float ey = fmaxf(fmaxf(by0 - b.y, b.y - by1), 0.0f);
    const float reach = reach_of(b);
    return b.z >= 0.0f && ex * ex + ey * ey <= reach * reach;
}

// FP64 constants of a point (x, y, z, A as uploaded): disc radius rj and
// its square r2 (metres; r2 < 0 when the point is not beyond the plane),
// beta (revolutions per sample^2) and the disc centre in samples.  The one
// place they are computed, so the culling box and the disc test agree.
struct PointFp64 {
    double x, y, rj, r2, beta, cx, cy;
};
__device__ __forceinline__ PointFp64 point_fp64(float4 raw, double pitch, double lam, double zw,
                                                double half)
{
    PointFp64 p;
    p.x = (double)raw.x;
    p.y = (double)raw.y;
    const double d = (double)raw.z - zw;
    p.rj = 0.0;
    p.r2 = -1.0;
    p.beta = 0.0;
    if (d > 0.0) {
        p.rj = lam * d / (2.0 * pitch);      // disc radius, metres
        p.r2 = p.rj * p.rj;
        p.beta = pitch * pitch / (2.0 * lam * d);
    }
    p.cx = half + p.x / pitch;
    p.cy = half + p.y / pitch;
    return p;
}

// a1 of the recording: the culling box and raw inputs of point i (see
// WrmConsts in common.h), and per group of kRound points (one workgroup)
// the box of their discs.
constexpr int kConstsThreads = 1024;
static_assert(kRound % kConstsThreads == 0, "a group is whole passes of the constants block");

__global__ __launch_bounds__(kConstsThreads) void k_wrm_consts(const float *__restrict__ x,
                                                               const float *__restrict__ y,
                                                               const float *__restrict__ z,
                                                               const float *__restrict__ amp,
                                                               int64_t n_points, double pitch,
                                                               double lam, double zw, double half,
                                                               WrmConsts wc)
{
    __shared__ float4 part[kConstsThreads / 64];
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *wc.next_tile = 0;   // the recording's tile queue starts empty
    // (x lo, x hi, y lo, y hi) of this thread's discs, widened by a sample;
    // empty for points outside the cloud or not beyond the plane
    float4 ext{__builtin_inff(), -__builtin_inff(), __builtin_inff(), -__builtin_inff()};
    for (int k = 0; k < kRound / kConstsThreads; ++k) {
        const int64_t i = (int64_t)blockIdx.x * kRound + k * kConstsThreads + threadIdx.x;
        if (i >= n_points)
            break;
        const float4 raw{x[i], y[i], z[i], amp[i]};
        const PointFp64 pt = point_fp64(raw, pitch, lam, zw, half);
        const float rho = pt.r2 < 0.0 ? -1.0f : (float)(pt.rj / pitch);   // radius, samples
        const float4 b{(float)pt.cx, (float)pt.cy, rho, 0.0f};
        wc.box[i] = b;
        wc.raw[i] = raw;
        if (rho >= 0.0f) {
            const float r = reach_of(b) + 1.0f;
            ext.x = fminf(ext.x, b.x - r);
            ext.y = fmaxf(ext.y, b.x + r);
            ext.z = fminf(ext.z, b.y - r);
            ext.w = fmaxf(ext.w, b.y + r);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        ext.x = fminf(ext.x, __shfl_xor(ext.x, o));
        ext.y = fmaxf(ext.y, __shfl_xor(ext.y, o));
        ext.z = fminf(ext.z, __shfl_xor(ext.z, o));
        ext.w = fmaxf(ext.w, __shfl_xor(ext.w, o));
    }
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = ext;
    __syncthreads();
    if (threadIdx.x == 0 && (int64_t)blockIdx.x * kRound < n_points) {
        float4 g = part[0];
        for (int w = 1; w < kConstsThreads / 64; ++w) {
            g.x = fminf(g.x, part[w].x);
            g.y = fmaxf(g.y, part[w].y);
            g.z = fminf(g.z, part[w].z);
            g.w = fmaxf(g.w, part[w].w);
        }
        wc.gbox[blockIdx.x] = g;
    }
}

// A hit's terms for one row: dy^2 (metres^2, FP64) and the cosine and sine
// of its reduced row phase; for one column: dx^2 and A times the cosine and
// sine of its reduced column phase.  Kept as separate arrays of 8-byte
// values, so lanes reading or writing consecutive entries touch consecutive
// 8-byte words (no LDS bank conflicts; 16-byte records are accessed as two
// 8-byte halves with a 16-byte stride).
// LDS of a recording workgroup.
struct RecordLds {
    uint64_t gmask[4];                   // groups of the window (256) reaching the tile
    uint64_t masks[kPerThread][kWaves];  // points of the round hitting the tile
    // constants of the batch's hits
    double h_x[kBatch], h_y[kBatch], h_r2[kBatch], h_beta[kBatch], h_cx[kBatch], h_cy[kBatch];
    float h_a[kBatch];
    uint32_t h_sub[kBatch];              // sub-tiles (waves) the hit's disc can reach
    float4 h_raw[kBatch], h_box[kBatch]; // the hits' raw inputs and culling boxes
    double rt_dy2[kBatch][kTileRows];
    float2 rt_cs[kBatch][kTileRows];    // (cos 2piV, sin 2piV)
    double ct_dx2[kBatch][kTileCols];
    float2 ct_acs[kBatch][kTileCols];   // A (cos 2piU, sin 2piU)
};

// One tile (64 columns from col0, 32 rows from trow0) of the plane, summed
// over the points of groups [g_lo, g_hi) into dst (an n x n plane).
__device__ __forceinline__ void record_tile(const WrmConsts &wc, int64_t n_points, int n,
                                            double pitch, double lam, double zw, double half,
                                            int col0, int trow0, int64_t g_lo, int64_t g_hi,
                                            float2 *__restrict__ dst, RecordLds &L)
{
    auto &gmask = L.gmask;
    auto &masks = L.masks;
    auto &h_x = L.h_x;
    auto &h_y = L.h_y;
    auto &h_r2 = L.h_r2;
    auto &h_beta = L.h_beta;
    auto &h_cx = L.h_cx;
    auto &h_cy = L.h_cy;
    auto &h_a = L.h_a;
    auto &h_sub = L.h_sub;
    auto &h_raw = L.h_raw;
    auto &h_box = L.h_box;
    auto &rt_dy2 = L.rt_dy2;
    auto &rt_cs = L.rt_cs;
    auto &ct_dx2 = L.ct_dx2;
    auto &ct_acs = L.ct_acs;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // the wave's sub-tile, and the lane's column and first row in it (the
    // lane's samples: kLaneRows consecutive rows of one column)
    const int sub_c = (wave % kSubX) * kSub, sub_r = (wave / kSubX) * kSub;
    const int lc = sub_c + (lane % kSub), lr = sub_r + (lane / kSub) * kLaneRows;
    const int row0 = trow0 + lr;
    const int col = col0 + lc;

    // the tile's sample centres span [col0, col0 + 63] x [trow0, trow0 + 31]
    const float bx0 = (float)col0, bx1 = (float)(col0 + kTileCols - 1);
    const float by0 = (float)trow0, by1 = (float)(trow0 + kTileRows - 1);
    float acc_re[kLaneRows], acc_im[kLaneRows];
#pragma unroll
    for (int r = 0; r < kLaneRows; ++r) {
        acc_re[r] = 0.0f;
        acc_im[r] = 0.0f;
    }

    // a round's boxes and raw inputs, loaded a round ahead
    float4 box[kPerThread], raw[kPerThread];
    auto load_boxes = [&](int64_t base) {
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const int64_t i = base + k * kThreads + tid;
            box[k] = i < n_points ? wc.box[i] : float4{0.0f, 0.0f, -1.0f, 0.0f};
            raw[k] = i < n_points ? wc.raw[i] : float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    // windows of 256 groups: which of them can reach the tile (one test per
    // thread), then the rounds of those in order
    for (int64_t w0 = g_lo; w0 < g_hi; w0 += 256) {
        {
            const int64_t g = w0 + tid;
            bool reach = false;
            if (tid < 256 && g < g_hi) {
                const float4 gb = wc.gbox[g];
                reach = !(gb.y < bx0 || gb.x > bx1 || gb.w < by0 || gb.z > by1);
            }
            const uint64_t m = __ballot(reach);
            if (lane == 0 && wave < 4)
                gmask[wave] = m;
        }
        __syncthreads();
        uint64_t gm[4];   // the same in every lane, made scalar
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint64_t v = gmask[w];
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
            gm[w] = ((uint64_t)hi << 32) | (uint64_t)lo;
        }
        __syncthreads();   // gmask is read before the next window rewrites it
        // first reaching group at or after q of the window (256: none)
        auto next_group = [&](int q) {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if (q < (w + 1) * 64) {
                    const int sh = q > w * 64 ? q - w * 64 : 0;
                    const uint64_t v = gm[w] & (~0ull << sh);
                    if (v)
                        return w * 64 + (int)__builtin_ctzll(v);
                }
            }
            return 256;
        };
        int q = next_group(0);
        if (q < 256)
            load_boxes((w0 + q) * kRound);
        while (q < 256) {
            const int64_t base = (w0 + q) * kRound;
            bool hit[kPerThread];
            // this round's boxes and raw inputs (the prefetch reuses box and raw)
            float4 hbox[kPerThread], hraw[kPerThread];
            uint64_t own[kPerThread];   // this wave's hit masks
#pragma unroll
            for (int k = 0; k < kPerThread; ++k) {
                hit[k] = box_hit(box[k], bx0, bx1, by0, by1);
                hbox[k] = box[k];
                hraw[k] = raw[k];
                own[k] = __ballot(hit[k]);
                if (lane == 0)
                    masks[k][wave] = own[k];
            }
            q = q + 1 < 256 ? next_group(q + 1) : 256;
            if (q < 256)
                load_boxes((w0 + q) * kRound);   // in flight while this round's hits add
            __syncthreads();
            // this thread's places among the round's hits (index order
            // (k, wave, lane)), and their count: lane j of every wave counts
            // mask j mod 16 (k kWaves + w order) and the counts are scanned
            // across the lanes
            const int mi = lane & (kMasks - 1);
            const int cnt = __builtin_popcountll((&masks[0][0])[mi]);
            int incl = cnt;
#pragma unroll
            for (int o = 1; o < kMasks; o <<= 1) {
                const int t = __shfl_up(incl, o, kMasks);
                if (mi >= o)
                    incl += t;
            }
            const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, kMasks - 1));
            int pos[kPerThread];
#pragma unroll
            for (int k = 0; k < kPerThread; ++k)
                pos[k] = __shfl(incl - cnt, k * kWaves + wave) +
                         (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(own[k] >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)own[k], 0));
            __syncthreads();   // the masks are read before the next round rewrites them
            for (int b0 = 0; b0 < total; b0 += kBatch) {
                const int nb = total - b0 < kBatch ? total - b0 : kBatch;
                // the batch's hits: raw inputs and culling boxes from their
                // owners, then the FP64 constants and sub-tile sets of all of
                // them in one pass of the first wave (one lane per hit), not
                // once in every wave that owns one
#pragma unroll
                for (int k = 0; k < kPerThread; ++k) {
                    if (hit[k] && pos[k] >= b0 && pos[k] < b0 + kBatch) {
                        h_raw[pos[k] - b0] = hraw[k];
                        h_box[pos[k] - b0] = hbox[k];
                    }
                }
                __syncthreads();
                if (tid < nb) {
                    const float4 rw = h_raw[tid], bx = h_box[tid];
                    const PointFp64 pt = point_fp64(rw, pitch, lam, zw, half);
                    h_x[tid] = pt.x;
                    h_y[tid] = pt.y;
                    h_r2[tid] = pt.r2;
                    h_beta[tid] = pt.beta;
                    h_cx[tid] = pt.cx;
                    h_cy[tid] = pt.cy;
                    h_a[tid] = rw.w;
                    uint32_t sub = 0;
#pragma unroll
                    for (int w = 0; w < kWaves; ++w) {
                        const float sx0 = bx0 + (float)((w % kSubX) * kSub);
                        const float sy0 = by0 + (float)((w / kSubX) * kSub);
                        if (box_hit(bx, sx0, sx0 + (float)(kSub - 1), sy0, sy0 + (float)(kSub - 1)))
                            sub |= 1u << w;
                    }
                    h_sub[tid] = sub;
                }
                __syncthreads();
                // the batch's column terms (hits x 64) and row terms (hits x 32)
                for (int e = tid; e < nb * (kTileCols + kTileRows); e += kThreads) {
                    if (e < nb * kTileCols) {
                        const int h = e / kTileCols, c = e % kTileCols;
                        const double dx = ((double)(col0 + c) - half) * pitch - h_x[h];
                        const double uc = (double)(col0 + c) - h_cx[h];
                        const float u = (float)__builtin_amdgcn_fract(h_beta[h] * (uc * uc));
                        const float a = h_a[h];
                        ct_dx2[h][c] = dx * dx;
                        ct_acs[h][c] =
                            float2{a * __builtin_amdgcn_cosf(u), a * __builtin_amdgcn_sinf(u)};
                    } else {
                        const int f = e - nb * kTileCols;
                        const int h = f / kTileRows, r = f % kTileRows;
                        const double dy = ((double)(trow0 + r) - half) * pitch - h_y[h];
                        const double vr = (double)(trow0 + r) - h_cy[h];
                        const float v = (float)__builtin_amdgcn_fract(h_beta[h] * (vr * vr));
                        rt_dy2[h][r] = dy * dy;
                        rt_cs[h][r] = float2{__builtin_amdgcn_cosf(v), __builtin_amdgcn_sinf(v)};
                    }
                }
                __syncthreads();
                // The wave's hits: those whose disc can reach its sub-tile,
                // in index order; within them branch-free (samples outside
                // the disc add zero products).
                uint32_t mine = (uint32_t)__ballot(lane < nb && ((h_sub[lane & (kBatch - 1)] >> wave) & 1u));
                while (mine) {
                    const int h = __builtin_ctz(mine);
                    mine &= mine - 1u;
                    const double dx2 = ct_dx2[h][lc];
                    const float2 acs = ct_acs[h][lc];
                    const double r2 = h_r2[h];
                    double dy2[kLaneRows];
                    float2 cs[kLaneRows];
#pragma unroll
                    for (int r = 0; r < kLaneRows; ++r) {
                        dy2[r] = rt_dy2[h][lr + r];
                        cs[r] = rt_cs[h][lr + r];
                    }
#pragma unroll
                    for (int r = 0; r < kLaneRows; ++r) {
                        const bool in = dx2 + dy2[r] <= r2;
                        const float c = in ? acs.x : 0.0f, sn = in ? acs.y : 0.0f;
                        acc_re[r] =
                            __builtin_fmaf(-sn, cs[r].y, __builtin_fmaf(c, cs[r].x, acc_re[r]));
                        acc_im[r] =
                            __builtin_fmaf(c, cs[r].y, __builtin_fmaf(sn, cs[r].x, acc_im[r]));
                    }
                }
                __syncthreads();   // the batch is consumed before the next one is written
            }
        }
    }
    if (col < n) {
#pragma unroll
        for (int r = 0; r < kLaneRows; ++r)
            if (row0 + r < n)
                dst[(int64_t)(row0 + r) * n + col] = float2{acc_re[r], acc_im[r]};
    }
}

// Work items are (tile, point chunk) pairs, tile-major: the points' groups
// are cut into `chunks` consecutive ranges, chunk 0 recorded into `field`
// and chunk c > 0 into plane c - 1 of `parts`, which k_wrm_sum then adds to
// the field in chunk order.  Items go one per workgroup (`queue` false: the
// grid covers them; chunks is then 1), or, for clouds of more than a few
// point groups, come from a queue (the counter reset by the constants
// kernel) that persistent workgroups drain: the few tiles the cloud
// reaches, each hundreds of times the work of an empty one, run side by
// side on all CUs as soon as a workgroup is free, and their chunks spread
// one tile's work over several workgroups.
__global__ __launch_bounds__(kThreads) void k_wrm_record(WrmConsts wc, int64_t n_points, int n,
                                                         double pitch, double lam, double zw,
                                                         double half, int queue, int chunks,
                                                         float2 *__restrict__ field,
                                                         float2 *__restrict__ parts)
{
    __shared__ RecordLds L;
    __shared__ int next;
    const int tiles_x = (n + kTileCols - 1) / kTileCols;
    const int items = tiles_x * ((n + kTileRows - 1) / kTileRows) * chunks;
    const int64_t n_groups = (n_points + kRound - 1) / kRound;
    for (int t = blockIdx.x;;) {
        if (queue) {
            if (threadIdx.x == 0)
                next = atomicAdd(wc.next_tile, 1);
            __syncthreads();        // next is visible; the previous tile's LDS use is over
            t = next;
            __syncthreads();        // everyone has read next before thread 0 rewrites it
        }
        if (t >= items)
            break;
        const int tile = t / chunks, chunk = t - tile * chunks;
        float2 *dst = chunk == 0 ? field : parts + (int64_t)(chunk - 1) * n * n;
        record_tile(wc, n_points, n, pitch, lam, zw, half, (tile % tiles_x) * kTileCols,
                    (tile / tiles_x) * kTileRows, n_groups * chunk / chunks,
                    n_groups * (chunk + 1) / chunks, dst, L);
        if (!queue)
            break;
    }
}

// field[i] += parts[0][i] + ... in chunk order, two samples per thread, as
// one 16-byte access each when `wide` (field and planes 16-byte aligned).
__global__ __launch_bounds__(256) void k_wrm_sum(float2 *__restrict__ field,
                                                 const float2 *__restrict__ parts, int planes,
                                                 int64_t samples, int wide)
{
    const int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= samples)
        return;
    if (!wide) {
        const int64_t end = i + 2 < samples ? i + 2 : samples;
        for (int64_t k = i; k < end; ++k) {
            float2 a = field[k];
            for (int c = 0; c < planes; ++c) {
                const float2 b = parts[(int64_t)c * samples + k];
                a.x += b.x;
                a.y += b.y;
            }
            field[k] = a;
        }
    } else if (i + 1 < samples) {
        float4 a = *(const float4 *)(field + i);
        for (int c = 0; c < planes; ++c) {
            const float4 b = *(const float4 *)(parts + (int64_t)c * samples + i);
            a.x += b.x;
            a.y += b.y;
            a.z += b.z;
            a.w += b.w;
        }
        *(float4 *)(field + i) = a;
    } else {
        float2 a = field[i];
        for (int c = 0; c < planes; ++c) {
            const float2 b = parts[(int64_t)c * samples + i];
            a.x += b.x;
            a.y += b.y;
        }
        field[i] = a;
    }
}

// Re O over the hologram's W x H window of an n x n field, the window's
// first sample at column ox, row oy.
__global__ __launch_bounds__(256) void k_window_real(const float2 *__restrict__ field, int n,
                                                     int ox, int oy, int width, int height,
                                                     float *__restrict__ out)
{
    const int ix = blockIdx.x * blockDim.x + threadIdx.x;
    const int iy = blockIdx.y;
    if (ix >= width)
        return;
    out[(int64_t)iy * width + ix] = field[(int64_t)(iy + oy) * n + ix + ox].x;
}

}  // namespace

hipError_t launch_wrm_consts(const float *x, const float *y, const float *z, const float *amp,
                             int64_t n_points, int n, double pitch, double lam, double zw,
                             const WrmConsts &wc, hipStream_t s)
{
    // at least one block: it also resets the recording's tile queue
    const int64_t blocks = n_points > 0 ? (n_points + kRound - 1) / kRound : 1;
    hipLaunchKernelGGL(k_wrm_consts, dim3((unsigned)blocks), dim3(kConstsThreads), 0, s, x, y, z,
                       amp, n_points, pitch, lam, zw, 0.5 * (double)(n - 1), wc);
    return hipGetLastError();
}

int wrm_record_chunks(int64_t n_points, int n)
{
    if (n <= 0 || n_points <= kWrmQueueMinPoints)
        return 1;
    const int64_t n_groups = (n_points + kRound - 1) / kRound;
    return (int)std::min<int64_t>({kWrmMaxChunks, n_groups, std::max<int64_t>(1, n_points / kWrmPointsPerChunk)});
}

hipError_t launch_wrm_record(const WrmConsts &wc, int64_t n_points, int n, double pitch,
                             double lam, double zw, int chunks, float2 *field, float2 *parts,
                             hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int queue = n_points > kWrmQueueMinPoints ? 1 : 0;
    if (chunks < 1 || (!queue && chunks != 1) || (chunks > 1 && !parts))
        return hipErrorInvalidValue;
    const int64_t items = (int64_t)((n + kTileCols - 1) / kTileCols) *
                          ((n + kTileRows - 1) / kTileRows) * chunks;
    int64_t grid = items;
    if (queue) {
        // persistent: as many workgroups as are resident at once
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_wrm_record, kThreads, 0);
        if (e != hipSuccess)
            return e;
        grid = std::min<int64_t>(items, (int64_t)cus * std::max(per_cu, 1));
    }
    hipLaunchKernelGGL(k_wrm_record, dim3((unsigned)grid), dim3(kThreads), 0, s, wc, n_points,
                       n, pitch, lam, zw, 0.5 * (double)(n - 1), queue, chunks, field, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || chunks == 1)
        return e;
    const int64_t samples = (int64_t)n * n;
    const int64_t threads = (samples + 1) / 2;
    // the caller's field need only be 8-byte aligned
    const int wide = (uintptr_t)field % 16 == 0 && (uintptr_t)parts % 16 == 0 && samples % 2 == 0;
    hipLaunchKernelGGL(k_wrm_sum, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, field,
                       parts, chunks - 1, samples, wide);
    return hipGetLastError();
}

hipError_t launch_window_real(const float2 *field, int n, int ox, int oy, int width, int height,
                              float *out, hipStream_t s)
{
    if (width <= 0 || height <= 0)
        return hipSuccess;
    const dim3 grid((unsigned)((width + 255) / 256), (unsigned)height);
    hipLaunchKernelGGL(k_window_real, grid, dim3(256), 0, s, field, n, ox, oy, width, height,
                       out);
    return hipGetLastError();
}

}  // namespace cgh
