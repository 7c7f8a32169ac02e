// Split complex-GEMM of the separable hologram form on the matrix cores.
//
// I[iy, ix] = sum_k L[iy, k] R[ix, k] (K = 2N, see factors.hip), evaluated as
//     Lh Rh^T + Lh Rl^T + Ll Rh^T        (3 products; Ll Rl^T is below FP32 noise)
// or Lh Rh^T alone, in BF16 or FP16 with FP32 accumulation, using
// v_mfma_f32_16x16x32_{bf16,f16} (the 16x16 shape keeps the matrix pipe
// busier than the 32x32 one on gfx950); or L R^T in FP32 with
// v_mfma_f32_16x16x4_f32, four per 1 KB block.  In FP32 lane l holds K-columns
// 4 (l / 16) .. + 3 of a block and the m-th instruction takes its m-th value,
// so instruction m sums K-columns m, 4 + m, 8 + m, 12 + m: the four together
// cover the block's 16 K-columns once, in an order both operands share.
//
// Tiling:
//   - a workgroup of WM x WN waves computes a BM x BN output tile over one
//     K range (split-K); each wave owns a (BM/WM) x (BN/WN) sub-tile of
//     16 x 16 MFMA blocks, its accumulators in registers;
//   - one stage = one K block (16 points in bf16/f16, 8 in FP32).  Its operand
//     blocks (1 KB each, already in MFMA lane order in memory) are copied
//     straight into LDS with buffer_load_dwordx4 ... lds (no register staging;
//     a buffer rather than a global load, so the compiler can count the LDS
//     reads that follow precisely instead of waiting for all of them)
//     into a ring of STAGES slots, STAGES-1 stages ahead of the MFMAs.  The
//     copies of a stage are dealt evenly to all waves.  One barrier per
//     stage; its per-wave vmcnt wait lets later stages' copies stay in flight
//     (a __syncthreads() fence would drain them);
//   - each wave reads its fragments with conflict-free ds_read_b128 (lane l
//     reads bytes 16 l .. 16 l + 15 of a block) in product order -- A hi and
//     B hi for hi*hi, then B lo for hi*lo, then A lo for lo*hi -- so reads
//     overlap the MFMAs of the previous product, and issues the MFMAs of each
//     product over all its blocks before the next, so consecutive MFMAs never
//     write the same accumulator.
// Eight-wave shapes put two waves on each SIMD; one wave's waits are covered
// by the other's MFMAs.
// Workgroup order: consecutive workgroup ids are dispatched round-robin over
// the 8 XCDs, so ids are remapped to give each XCD a contiguous run of
// (split, tile) work -- same K range, neighbouring tiles -- whose operands
// its L2 shares.  Tiles are numbered down the columns of tiles, so a run
// that ends or starts part of the way through a split's tiles (splits that do
// not divide evenly over the XCDs) covers whole tile columns, sharing their
// B blocks.
// Split-K partial tiles go to a workspace and are summed in a fixed order by
// k_splitk_reduce, so results are bitwise reproducible (no float atomics).
#include <algorithm>

#include "common.h"

namespace cgh {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;
constexpr int kBlockBytes = 1024;   // one 16-line x 32-K operand block

template <typename T>
struct Frag;
template <>
struct Frag<__bf16> {
    typedef bf16x8 type;
    static constexpr int kSub = 1;
    static __device__ __forceinline__ f32x4 mfma(type a, type b, f32x4 c, int)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Frag<_Float16> {
    typedef f16x8 type;
    static constexpr int kSub = 1;
    static __device__ __forceinline__ f32x4 mfma(type a, type b, f32x4 c, int)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Frag<float> {
    typedef f32x4 type;
    static constexpr int kSub = 4;    // instructions per block (m = 0 .. 3)
    static __device__ __forceinline__ f32x4 mfma(type a, type b, f32x4 c, int m)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b[m], c, 0, 0, 0);
    }
};

// Buffer resource over one K slab of the factor set (loads past it return
// zeros), raw addressing (word 3 as for gfx9 raw buffers).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const char *slab, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(slab), (short)0, bytes,
                                             0x00020000);
}

// One 1 KB block: lane l copies bytes voff .. voff + 15 (voff includes 16 l)
// of the buffer to lds_block + 16 l.
__device__ __forceinline__ void copy_block_to_lds(__amdgpu_buffer_rsrc_t rsrc, uint32_t voff,
                                                  char *lds_block)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        rsrc, (__attribute__((address_space(3))) void *)lds_block, 16, voff, 0, 0, 0);
}

// Wait until at most N of this wave's vector-memory loads are outstanding
// (s_waitcnt vmcnt(N), expcnt and lgkmcnt fields left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// `ahead` = later stages whose copies may stay in flight (0 .. 3).
template <int LPS>
__device__ __forceinline__ void wait_stages_ahead(int64_t ahead)
{
    if (ahead <= 0)
        wait_vm<0>();
    else if (ahead == 1)
        wait_vm<(LPS < 64 ? LPS : 63)>();
    else if (ahead == 2)
        wait_vm<(2 * LPS < 64 ? 2 * LPS : 63)>();
    else
        wait_vm<(3 * LPS < 64 ? 3 * LPS : 63)>();
}

// Workgroup barrier for the copy ring.  It does not wait for this wave's
// outstanding copies (the caller has waited for the stage it needs); it does
// wait for this wave's LDS reads, since other waves may overwrite the slot
// they read once past the barrier.  The empty asm statements keep the
// compiler from moving memory operations across it.
__device__ __forceinline__ void ring_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt, expcnt at their maxima
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One output tile: line blocks tm (of L) and tn (of R), K blocks
// [kb_begin, kb_begin + n_st) of the factor set; the result goes to
// dst[row * ld + col] for row < M, col < N (added to what is there when
// acc_old).  All threads of the workgroup call it.
template <int BM, int BN, int WM, int WN, int PRODUCTS, typename T, int STAGES>
__device__ __forceinline__ void gemm_tile(const FactorSet &fs, int64_t kb_begin, int64_t n_st,
                                          int tm, int tn, int M, int N, float *__restrict__ dst,
                                          int64_t ld, bool acc_old, char *lds)
{
    constexpr int NW = WM * WN;
    constexpr int HL = PRODUCTS == 3 ? 2 : 1;
    constexpr int MB = BM / kFragLines;          // line blocks per tile
    constexpr int NB = BN / kFragLines;
    constexpr int FM = MB / WM;                  // MFMA blocks per wave along M
    constexpr int FN = NB / WN;                  // ... along N
    static_assert(MB % WM == 0 && NB % WN == 0, "tile splits evenly over waves");
    constexpr int SLOT_BLOCKS = HL * (MB + NB);  // [A hi: MB][A lo: MB][B hi: NB][B lo: NB]
    constexpr int SLOT_BYTES = SLOT_BLOCKS * kBlockBytes;
    constexpr int P = STAGES - 1;                // copy distance in stages
    static_assert(P >= 1 && P <= 4, "ring depth");
    // copies per stage per wave (at most); with copies more than one stage
    // ahead every wave must issue the same number, for its vmcnt waits
    constexpr int LPS = (SLOT_BLOCKS + NW - 1) / NW;
    static_assert(SLOT_BLOCKS % NW == 0 || P == 1, "stage copies deal evenly");
    static_assert((P - 1) * LPS < 64, "vmcnt range");
    static_assert(PRODUCTS == 1 || Frag<T>::kSub == 1, "split products are 16-bit only");
    typedef typename Frag<T>::type frag_t;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / WN, wn = wave % WN;

    // ---- this wave's copies: slot blocks wave, wave + NW, ..., as byte
    // offsets into a K slab of the factor set
    const int slab_bytes = fs.slab_blocks() * kBlockBytes;
    const char *slab0 = fs.base + kb_begin * (int64_t)slab_bytes;
    uint32_t voff[LPS];
#pragma unroll
    for (int c = 0; c < LPS; ++c) {
        const int b = (wave + NW * c) % SLOT_BLOCKS;   // wrapped entries are not copied
        int blk;
        if (b < HL * MB)
            blk = fs.first_l(HL == 2 && b >= MB) + tm * MB + b % MB;
        else
            blk = fs.first_r(HL == 2 && b - HL * MB >= NB) + tn * NB + (b - HL * MB) % NB;
        voff[c] = (uint32_t)(blk * kBlockBytes + lane * 16);
    }
    auto issue = [&](int64_t i, int slot) {     // stage i (relative) into ring slot
        char *dst_slot = lds + slot * SLOT_BYTES;
        const __amdgpu_buffer_rsrc_t rsrc = slab_rsrc(slab0 + i * slab_bytes, slab_bytes);
#pragma unroll
        for (int c = 0; c < LPS; ++c)
            if (SLOT_BLOCKS % NW == 0 || wave + NW * c < SLOT_BLOCKS)
                copy_block_to_lds(rsrc, voff[c], dst_slot + (wave + NW * c) * kBlockBytes);
    };

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

#pragma unroll
    for (int i = 0; i < P; ++i)
        if (i < n_st)
            issue(i, i);
    int slot = 0;
    for (int64_t i = 0; i < n_st; ++i) {
        // this wave's copies of stage i landed; later stages may stay in flight
        const int64_t ahead = (n_st - 1 - i) < (P - 1) ? (n_st - 1 - i) : (P - 1);
        wait_stages_ahead<LPS>(ahead);
        // every wave's copies of stage i landed, and every wave is done with
        // stage i-1's slot, which the next copy overwrites
        ring_barrier();
        if (i + P < n_st)
            issue(i + P, slot == 0 ? P : slot - 1);
        const char *sb = lds + slot * SLOT_BYTES + lane * 16;
        auto blk = [&](int b) { return *reinterpret_cast<const frag_t *>(sb + b * kBlockBytes); };
        const int a_hi = wm * FM, a_lo = MB + wm * FM;          // this wave's A blocks
        const int b_hi = HL * MB + wn * FN, b_lo = HL * MB + NB + wn * FN;
        // B fragments for the whole stage; A fragments one row block at a
        // time, the next one read while the current one's MFMAs issue
        frag_t bh[FN];
        frag_t a_cur = blk(a_hi);
#pragma unroll
        for (int c = 0; c < FN; ++c)
            bh[c] = blk(b_hi + c);
        if (PRODUCTS == 3) {
            frag_t bl[FN];
#pragma unroll
            for (int c = 0; c < FN; ++c)
                bl[c] = blk(b_lo + c);
            // hi * hi and hi * lo, row block by row block
#pragma unroll
            for (int r = 0; r < FM; ++r) {
                const frag_t a_nxt = blk(r + 1 < FM ? a_hi + r + 1 : a_lo);
#pragma unroll
                for (int c = 0; c < FN; ++c)
                    acc[r][c] = Frag<T>::mfma(a_cur, bh[c], acc[r][c], 0);
#pragma unroll
                for (int c = 0; c < FN; ++c)
                    acc[r][c] = Frag<T>::mfma(a_cur, bl[c], acc[r][c], 0);
                a_cur = a_nxt;
                __builtin_amdgcn_sched_barrier(0);   // keep the next read ahead of these MFMAs
            }
            // lo * hi
#pragma unroll
            for (int r = 0; r < FM; ++r) {
                const frag_t a_nxt = blk(r + 1 < FM ? a_lo + r + 1 : a_lo);
#pragma unroll
                for (int c = 0; c < FN; ++c)
                    acc[r][c] = Frag<T>::mfma(a_cur, bh[c], acc[r][c], 0);
                a_cur = a_nxt;
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int r = 0; r < FM; ++r) {
                const frag_t a_nxt = blk(r + 1 < FM ? a_hi + r + 1 : a_hi);
#pragma unroll
                for (int m = 0; m < Frag<T>::kSub; ++m)
#pragma unroll
                    for (int c = 0; c < FN; ++c)
                        acc[r][c] = Frag<T>::mfma(a_cur, bh[c], acc[r][c], m);
                a_cur = a_nxt;
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        slot = slot == P ? 0 : slot + 1;
    }

    // ---- epilogue: accumulator register r of a 16x16 block holds row
    // 4 (lane / 16) + r, column lane mod 16.
    const int row_base = tm * BM + wm * FM * kFragLines;
    const int col_base = tn * BN + wn * FN * kFragLines;
#pragma unroll
    for (int r0 = 0; r0 < FM; ++r0)
#pragma unroll
        for (int c0 = 0; c0 < FN; ++c0) {
            const int col = col_base + c0 * kFragLines + (lane & 15);
            if (col >= N)
                continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row_base + r0 * kFragLines + 4 * (lane >> 4) + r;
                if (row < M) {
                    float *p = dst + (int64_t)row * ld + col;
                    *p = acc_old ? *p + acc[r0][c0][r] : acc[r0][c0][r];
                }
            }
        }
}

// One hologram, split-K: workgroup -> (split, tile).
template <int BM, int BN, int WM, int WN, int PRODUCTS, typename T, int STAGES>
__global__ __launch_bounds__(64 * WM * WN, 2) void k_gemm(
    FactorSet fs, int64_t kblocks, int tiles_m, int tiles_n, int splits, int64_t kb_per_split,
    int M, int N, float *__restrict__ out, int64_t ldo, float *__restrict__ partials,
    int accumulate)
{
    extern __shared__ __attribute__((aligned(1024))) char lds[];
    const int total = tiles_m * tiles_n * splits;
    const int per_xcd = gridDim.x / kXcds;
    const int work = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (work >= total)
        return;
    const int tiles = tiles_m * tiles_n;
    const int split = work / tiles;
    const int tile = work % tiles;
    const int64_t kb_begin = (int64_t)split * kb_per_split;
    int64_t kb_end = kb_begin + kb_per_split;
    if (kb_end > kblocks)
        kb_end = kblocks;
    const int64_t n_st = kb_end > kb_begin ? kb_end - kb_begin : 0;
    float *dst = splits == 1 ? out : partials + (int64_t)split * M * N;
    const int64_t ld = splits == 1 ? ldo : (int64_t)N;
    gemm_tile<BM, BN, WM, WN, PRODUCTS, T, STAGES>(fs, kb_begin, n_st, tile % tiles_m,
                                                   tile / tiles_m, M, N, dst, ld,
                                                   splits == 1 && accumulate != 0, lds);
}

// Many holograms, persistent: every workgroup takes (frame, tile) items from
// a shared counter until none is left; an item covers its frame's whole K
// range and writes its tile of that frame's output.  Items are ordered
// largest K first.  The counter starts at 0 (k_reset_counter).
template <int BM, int BN, int WM, int WN, int PRODUCTS, typename T, int STAGES>
__global__ __launch_bounds__(64 * WM * WN, 2) void k_gemm_batch(
    FactorSet fs, const BatchItem *__restrict__ items, int n_items, int *__restrict__ counter,
    int M, int N, float *__restrict__ out)
{
    extern __shared__ __attribute__((aligned(1024))) char lds[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0)
            next = atomicAdd(counter, 1);
        __syncthreads();            // next is visible; the previous tile's LDS use is over
        const int it = next;
        __syncthreads();            // everyone has read next before thread 0 rewrites it
        if (it >= n_items)
            break;
        const BatchItem w = items[it];
        gemm_tile<BM, BN, WM, WN, PRODUCTS, T, STAGES>(fs, w.kb_begin, w.kblocks, w.tm, w.tn, M,
                                                       N, out + w.out_off, N, false, lds);
    }
}

__global__ void k_reset_counter(int *counter) { *counter = 0; }

// out[i] = (accumulate ? out[i] : 0) + partials[0][i] + ... + partials[S-1][i], in that
// order; four consecutive elements per thread when N allows.
__global__ __launch_bounds__(256) void k_splitk_reduce(const float *__restrict__ partials,
                                                       int splits, int M, int N,
                                                       float *__restrict__ out, int64_t ldo,
                                                       int accumulate, int vec4)
{
    const int64_t total = (int64_t)M * N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (vec4) {
        const int64_t q = total / 4;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < q; e += stride) {
            float4 s = reinterpret_cast<const float4 *>(partials)[e];
            for (int k = 1; k < splits; ++k) {
                const float4 v = reinterpret_cast<const float4 *>(partials + (int64_t)k * total)[e];
                s.x += v.x;
                s.y += v.y;
                s.z += v.z;
                s.w += v.w;
            }
            const int64_t row = (4 * e) / N, col = (4 * e) % N;
            float4 *p = reinterpret_cast<float4 *>(out + row * ldo + col);
            if (accumulate) {
                const float4 o = *p;
                s = float4{o.x + s.x, o.y + s.y, o.z + s.z, o.w + s.w};
            }
            *p = s;
        }
        return;
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t row = e / N, col = e % N;
        float s = partials[e];
        for (int k = 1; k < splits; ++k)
            s += partials[(int64_t)k * total + e];
        float *p = out + row * ldo + col;
        *p = accumulate ? *p + s : s;
    }
}

// LDS of a workgroup: the copy ring, STAGES x (hi, lo) x (BM + BN) / 16 blocks.
template <int BM, int BN, int PRODUCTS, int STAGES>
constexpr int ring_bytes()
{
    return STAGES * (PRODUCTS == 3 ? 2 : 1) * (BM + BN) / kFragLines * kBlockBytes;
}

// The plan's tiles and K range stay inside the factor set, whose halves
// match the product count.
bool plan_fits(const GemmPlan &plan, int BM, int BN, int M, int N, const FactorSet &fs)
{
    return plan.mblocks % (BM / kFragLines) == 0 && plan.nblocks % (BN / kFragLines) == 0 &&
           plan.mblocks <= fs.amb && plan.nblocks <= fs.anb &&
           (int64_t)plan.mblocks * kFragLines >= M && (int64_t)plan.nblocks * kFragLines >= N &&
           plan.kblocks <= fs.kblocks && fs.base != nullptr &&
           fs.hl == (plan.products == 3 ? 2 : 1) &&
           (int64_t)fs.slab_blocks() * kBlockBytes < ((int64_t)1 << 31);
}

template <int BM, int BN, int WM, int WN, int PRODUCTS, typename T, int STAGES>
hipError_t launch_tile(const GemmPlan &plan, const FactorSet &fs, int M, int N, float *out,
                       int64_t ldo, float *partials, bool accumulate, hipStream_t s)
{
    if (!plan_fits(plan, BM, BN, M, N, fs))
        return hipErrorInvalidValue;     // tiles would read past the factor set
    const int lds_bytes = ring_bytes<BM, BN, PRODUCTS, STAGES>();
    auto kern = k_gemm<BM, BN, WM, WN, PRODUCTS, T, STAGES>;
    const int tiles_m = plan.mblocks / (BM / kFragLines);
    const int tiles_n = plan.nblocks / (BN / kFragLines);
    const int64_t per = (plan.kblocks + plan.splits - 1) / plan.splits;
    const int total = tiles_m * tiles_n * plan.splits;
    const int grid = (total + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WM * WN), lds_bytes, s, fs, plan.kblocks,
                       tiles_m, tiles_n, plan.splits, per, M, N, out, ldo, partials,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, int PRODUCTS, typename T, int STAGES>
hipError_t launch_tile_batch(const GemmPlan &plan, const FactorSet &fs, const BatchItem *items,
                             int n_items, int *counter, int M, int N, float *out, int grid,
                             hipStream_t s)
{
    if (!plan_fits(plan, BM, BN, M, N, fs))
        return hipErrorInvalidValue;     // tiles would read past the factor set
    const int lds_bytes = ring_bytes<BM, BN, PRODUCTS, STAGES>();
    auto kern = k_gemm_batch<BM, BN, WM, WN, PRODUCTS, T, STAGES>;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WM * WN), lds_bytes, s, fs, items, n_items,
                       counter, M, N, out);
    return hipGetLastError();
}

// Built shapes: (BM, BN, waves along M, waves along N, LDS ring depth).  The
// ring holds STAGES x 2 (hi, lo) x (BM + BN) / 16 KB with three products
// (half of that with one) and must fit the 160 KB of LDS.
#define CGH_GEMM_SHAPES(X)                                                                     \
    X(192, 384, 2, 4, 2)                                                                       \
    X(384, 192, 4, 2, 2)                                                                       \
    X(192, 320, 2, 4, 2)                                                                       \
    X(192, 256, 2, 4, 2)                                                                       \
    X(256, 256, 2, 4, 2)                                                                       \
    X(192, 192, 2, 2, 3)                                                                       \
    X(192, 192, 2, 4, 3)                                                                       \
    X(192, 192, 2, 4, 2)                                                                       \
    X(128, 256, 2, 4, 2)                                                                       \
    X(192, 128, 2, 2, 2)                                                                       \
    X(128, 192, 2, 2, 2)

template <int PRODUCTS, typename T>
hipError_t launch_products(const GemmPlan &plan, const FactorSet &fs, int M, int N, float *out,
                           int64_t ldo, float *partials, bool accumulate, hipStream_t s)
{
#define CGH_TILE(TBM, TBN, TWM, TWN, TST)                                                     \
    if (plan.bm == TBM && plan.bn == TBN && plan.waves_m == TWM && plan.waves_n == TWN &&     \
        plan.stages == TST)                                                                   \
        return launch_tile<TBM, TBN, TWM, TWN, PRODUCTS, T, TST>(plan, fs, M, N, out, ldo,    \
                                                                 partials, accumulate, s);
    CGH_GEMM_SHAPES(CGH_TILE)
#undef CGH_TILE
    return hipErrorInvalidValue;
}

template <int PRODUCTS, typename T>
hipError_t launch_products_batch(const GemmPlan &plan, const FactorSet &fs,
                                 const BatchItem *items, int n_items, int *counter, int M, int N,
                                 float *out, int grid, hipStream_t s)
{
#define CGH_TILE(TBM, TBN, TWM, TWN, TST)                                                     \
    if (plan.bm == TBM && plan.bn == TBN && plan.waves_m == TWM && plan.waves_n == TWN &&     \
        plan.stages == TST)                                                                   \
        return launch_tile_batch<TBM, TBN, TWM, TWN, PRODUCTS, T, TST>(                       \
            plan, fs, items, n_items, counter, M, N, out, grid, s);
    CGH_GEMM_SHAPES(CGH_TILE)
#undef CGH_TILE
    return hipErrorInvalidValue;
}

// Raise the LDS limit of both kernels of every built shape and operand type
// on the current device (the ring exceeds the default 64 KB).
template <int BM, int BN, int WM, int WN, int STAGES, int PRODUCTS, typename T>
hipError_t prepare_one()
{
    const int lds = ring_bytes<BM, BN, PRODUCTS, STAGES>();
    hipError_t e = hipFuncSetAttribute((const void *)k_gemm<BM, BN, WM, WN, PRODUCTS, T, STAGES>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_gemm_batch<BM, BN, WM, WN, PRODUCTS, T, STAGES>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    return e;
}

template <int BM, int BN, int WM, int WN, int STAGES>
hipError_t prepare_shape()
{
    hipError_t e = prepare_one<BM, BN, WM, WN, STAGES, 3, __bf16>();
    if (e == hipSuccess)
        e = prepare_one<BM, BN, WM, WN, STAGES, 3, _Float16>();
    if (e == hipSuccess)
        e = prepare_one<BM, BN, WM, WN, STAGES, 1, __bf16>();
    if (e == hipSuccess)
        e = prepare_one<BM, BN, WM, WN, STAGES, 1, _Float16>();
    if (e == hipSuccess)
        e = prepare_one<BM, BN, WM, WN, STAGES, 1, float>();
    return e;
}

}  // namespace

hipError_t gemm_prepare_kernels()
{
#define CGH_TILE(TBM, TBN, TWM, TWN, TST)                                                     \
    if (hipError_t e = prepare_shape<TBM, TBN, TWM, TWN, TST>(); e != hipSuccess)            \
        return e;
    CGH_GEMM_SHAPES(CGH_TILE)
#undef CGH_TILE
    return hipSuccess;
}

hipError_t launch_gemm_batch(const GemmPlan &plan, FactorType ft, const FactorSet &fs,
                             const BatchItem *items, int n_items, int *counter, int M, int N,
                             float *out, int grid, hipStream_t s)
{
    if (ft == FactorType::FP32)
        return plan.products == 1 ? launch_products_batch<1, float>(plan, fs, items, n_items,
                                                                    counter, M, N, out, grid, s)
                                  : hipErrorInvalidValue;
    if (plan.products == 3) {
        if (ft == FactorType::BF16)
            return launch_products_batch<3, __bf16>(plan, fs, items, n_items, counter, M, N, out,
                                                    grid, s);
        return launch_products_batch<3, _Float16>(plan, fs, items, n_items, counter, M, N, out,
                                                  grid, s);
    }
    if (ft == FactorType::BF16)
        return launch_products_batch<1, __bf16>(plan, fs, items, n_items, counter, M, N, out,
                                                grid, s);
    return launch_products_batch<1, _Float16>(plan, fs, items, n_items, counter, M, N, out, grid,
                                              s);
}

int gemm_groups_per_cu(int bm, int bn, int waves_m, int waves_n, int stages, int products)
{
    // two waves per SIMD (the register budget) and the 160 KB of LDS
    const int ring = stages * (products == 3 ? 2 : 1) * (bm + bn) / kFragLines * kBlockBytes;
    const int by_waves = 8 / (waves_m * waves_n);
    const int by_lds = (160 * 1024) / ring;
    return std::max(1, std::min(by_waves, by_lds));
}

bool gemm_tile_supported(int bm, int bn, int waves_m, int waves_n, int stages)
{
#define CGH_TILE(TBM, TBN, TWM, TWN, TST)                                                     \
    if (bm == TBM && bn == TBN && waves_m == TWM && waves_n == TWN && stages == TST)          \
        return true;
    CGH_GEMM_SHAPES(CGH_TILE)
#undef CGH_TILE
    return false;
}

hipError_t launch_gemm(const GemmPlan &plan, FactorType ft, const FactorSet &fs, int M, int N,
                       float *out, int64_t ldo, float *partials, bool accumulate, hipStream_t s)
{
    if (ft == FactorType::FP32)
        return plan.products == 1 ? launch_products<1, float>(plan, fs, M, N, out, ldo, partials,
                                                              accumulate, s)
                                  : hipErrorInvalidValue;
    if (plan.products == 3) {
        if (ft == FactorType::BF16)
            return launch_products<3, __bf16>(plan, fs, M, N, out, ldo, partials, accumulate, s);
        return launch_products<3, _Float16>(plan, fs, M, N, out, ldo, partials, accumulate, s);
    }
    if (ft == FactorType::BF16)
        return launch_products<1, __bf16>(plan, fs, M, N, out, ldo, partials, accumulate, s);
    return launch_products<1, _Float16>(plan, fs, M, N, out, ldo, partials, accumulate, s);
}

hipError_t launch_splitk_reduce(const float *partials, int splits, int M, int N, float *out,
                                int64_t ldo, bool accumulate, hipStream_t s)
{
    const int64_t total = (int64_t)M * N;
    if (total <= 0)
        return hipSuccess;
    int64_t blocks = (total / 4 + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    if (blocks < 1)
        blocks = 1;
    // float4 path: rows of whole float4s, 16-byte aligned buffers
    const int vec4 = (N % 4 == 0) && (ldo % 4 == 0) && ((uintptr_t)out % 16 == 0) &&
                     ((uintptr_t)partials % 16 == 0);
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, s, partials, splits,
                       M, N, out, ldo, accumulate ? 1 : 0, vec4);
    return hipGetLastError();
}

}  // namespace cgh
