// Split complex-GEMM of the separable hologram form on the matrix cores.
//
// I[iy, ix] = sum_k L[iy, k] R[ix, k] (K = 2N, see factors.hip), evaluated as
//     Lh Rh^T + Lh Rl^T + Ll Rh^T        (3 products; Ll Rl^T is below FP32 noise)
// or Lh Rh^T alone, in BF16 or FP16 with FP32 accumulation, using
// v_mfma_f32_32x32x16_{bf16,f16}.
//
// Tiling (256 threads = 4 waves as 2 x 2):
//   - a workgroup computes a BM x BN output tile over one K range (split-K);
//     each wave owns a (BM/2) x (BN/2) sub-tile of 32 x 32 MFMA blocks;
//   - one stage = one K block (16 K-columns = 8 points).  Its operand blocks
//     (1 KB each, already in MFMA lane order in memory) are copied straight
//     into LDS with global_load_lds_dwordx4 (no register staging) into a ring
//     of STAGES slots, STAGES stages ahead of the MFMAs; one barrier per
//     stage, with per-wave vmcnt waits that let the later stages' copies stay
//     in flight;
//   - each wave reads its fragments with conflict-free ds_read_b128 (lane l
//     reads bytes 16 l .. 16 l + 15 of a block) and issues 3 x (BM/64) x
//     (BN/64) MFMAs per stage, product-major, so consecutive MFMAs never write
//     the same accumulator.  Fragments are double-buffered in registers: the
//     barrier and the next stage's LDS reads sit in the middle of the current
//     stage's MFMAs;
//   - shapes with MINWG = 2 fit two workgroups per CU (<= 80 KB LDS and <= 256
//     registers per lane each), so one workgroup's barrier and LDS waits are
//     covered by the other's MFMAs.
// Workgroup order: consecutive workgroup ids are dispatched round-robin over
// the 8 XCDs, so ids are remapped to give each XCD a contiguous run of
// (split, tile) work -- same K range, neighbouring tiles -- whose operands
// its L2 shares.
// Split-K partial tiles go to a workspace and are summed in a fixed order by
// k_splitk_reduce, so results are bitwise reproducible (no float atomics).
#include "common.h"

namespace cgh {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kXcds = 8;
constexpr int kBlockBytes = 1024;   // one 32 x 16 operand block

template <typename T>
struct Frag;
template <>
struct Frag<__bf16> {
    typedef bf16x8 type;
    static __device__ __forceinline__ f32x16 mfma(type a, type b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Frag<_Float16> {
    typedef f16x8 type;
    static __device__ __forceinline__ f32x16 mfma(type a, type b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

__device__ __forceinline__ void copy_block_to_lds(const char *gsrc, char *lds_block, int lane)
{
    // Each lane copies its 16 bytes; the hardware writes lane l's data at
    // lds_block + 16 l.
    __builtin_amdgcn_global_load_lds(
        (const __attribute__((address_space(1))) void *)(gsrc + lane * 16),
        (__attribute__((address_space(3))) void *)lds_block, 16, 0, 0);
}

// Wait until at most N of this wave's vector-memory loads are outstanding
// (s_waitcnt vmcnt(N), expcnt and lgkmcnt fields left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// `ahead` = later stages whose copies may stay in flight (0 .. 4).
template <int LPS>
__device__ __forceinline__ void wait_stages_ahead(int64_t ahead)
{
    if (ahead <= 0)
        wait_vm<0>();
    else if (ahead == 1)
        wait_vm<LPS>();
    else if (ahead == 2)
        wait_vm<(2 * LPS < 64 ? 2 * LPS : 63)>();
    else if (ahead == 3)
        wait_vm<(3 * LPS < 64 ? 3 * LPS : 63)>();
    else
        wait_vm<(4 * LPS < 64 ? 4 * LPS : 63)>();
}

// Workgroup barrier for the copy ring.  It does not wait for this wave's
// outstanding copies (a __syncthreads() fence would drain them all): the
// caller has already waited for the stage it needs with wait_vm.  It does
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

// LDS stage layout (blocks of 1 KB, one K block per stage):
// [A hi: MB][A lo: MB][B hi: NB][B lo: NB]   (lo parts only with 3 products)
template <int BM, int BN, int HL>
struct StageLayout {
    static constexpr int MB = BM / 32;
    static constexpr int NB = BN / 32;
    static constexpr int blocks = HL * (MB + NB);
    static constexpr int bytes = blocks * kBlockBytes;
};

// One stage's operand fragments of a wave: hi (and lo) parts of its FM
// line blocks of L and FN line blocks of R.
template <typename T, int HL, int FM, int FN>
struct Frags {
    typedef typename Frag<T>::type frag_t;
    frag_t a[HL][FM], b[HL][FN];
    // slot layout [A hi: MB][A lo: MB][B hi: NB][B lo: NB]
    __device__ __forceinline__ void read(const char *slot, int MB, int NB, int wm, int wn, int lane)
    {
#pragma unroll
        for (int r = 0; r < FM; ++r)
            a[0][r] = *reinterpret_cast<const frag_t *>(slot + (wm * FM + r) * kBlockBytes + lane * 16);
#pragma unroll
        for (int c = 0; c < FN; ++c)
            b[0][c] = *reinterpret_cast<const frag_t *>(slot + (HL * MB + wn * FN + c) * kBlockBytes +
                                                        lane * 16);
        if (HL == 2) {
#pragma unroll
            for (int c = 0; c < FN; ++c)
                b[HL - 1][c] = *reinterpret_cast<const frag_t *>(
                    slot + (HL * MB + NB + wn * FN + c) * kBlockBytes + lane * 16);
#pragma unroll
            for (int r = 0; r < FM; ++r)
                a[HL - 1][r] = *reinterpret_cast<const frag_t *>(
                    slot + (MB + wm * FM + r) * kBlockBytes + lane * 16);
        }
    }
};

// MFMAs [LO, HI) of a stage's list, ordered product-major -- hi*hi, hi*lo,
// lo*hi -- then by line block, so consecutive MFMAs never write the same
// accumulator.
template <int LO, int HI, typename T, int HL, int FM, int FN>
__device__ __forceinline__ void mfma_list(f32x16 (&acc)[FM][FN], const Frags<T, HL, FM, FN> &f)
{
#pragma unroll
    for (int k = LO; k < HI; ++k) {
        const int p = k / (FM * FN), r = (k / FN) % FM, c = k % FN;
        const int ha = p == 2 ? HL - 1 : 0;   // lo * hi takes A's lo part
        const int hb = p == 1 ? HL - 1 : 0;   // hi * lo takes B's lo part
        acc[r][c] = Frag<T>::mfma(f.a[ha][r], f.b[hb][c], acc[r][c]);
    }
}

template <int BM, int BN, int PRODUCTS, typename T, int STAGES, int MINWG>
__global__ __launch_bounds__(256, MINWG) void k_gemm(const char *__restrict__ Lh,
                                                     const char *__restrict__ Ll,
                                                     const char *__restrict__ Rh,
                                                     const char *__restrict__ Rl, int64_t kblocks,
                                                     int tiles_m, int tiles_n, int splits,
                                                     int64_t kb_per_split, int M, int N,
                                                     float *__restrict__ out, int64_t ldo,
                                                     float *__restrict__ partials, int accumulate)
{
    constexpr int HL = PRODUCTS == 3 ? 2 : 1;
    typedef StageLayout<BM, BN, HL> SL;
    constexpr int FM = BM / 64;   // 32x32 blocks per wave along M
    constexpr int FN = BN / 64;   // ... along N
    constexpr int P = STAGES;     // ring slots = copy distance in stages
    static_assert(P >= 2 && P <= 5, "ring depth");
    // Copies per stage per wave: waves 0, 1 take L, waves 2, 3 take R -- the
    // hi and lo parts with 3 products, else the two halves of the line blocks.
    constexpr int LPS_A = HL == 2 ? SL::MB : SL::MB / 2;
    constexpr int LPS_B = HL == 2 ? SL::NB : SL::NB / 2;
    static_assert(HL == 2 || (SL::MB % 2 == 0 && SL::NB % 2 == 0), "even line blocks");
    static_assert((P - 1) * (LPS_A > LPS_B ? LPS_A : LPS_B) < 64, "vmcnt range");
    static_assert(P - 1 <= 4, "wait_stages_ahead covers up to 4 stages");
    constexpr int kTotal = PRODUCTS * FM * FN;   // MFMAs per stage per wave
    constexpr int kHalf = (kTotal + 1) / 2;
    extern __shared__ __attribute__((aligned(1024))) char lds[];

    // ---- which (split, tile) this workgroup computes
    const int total = tiles_m * tiles_n * splits;
    const int per_xcd = gridDim.x / kXcds;
    const int work = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (work >= total)
        return;
    const int tiles = tiles_m * tiles_n;
    const int split = work / tiles;
    const int tile = work % tiles;
    const int tm = tile / tiles_n;
    const int tn = tile % tiles_n;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave >> 1, wn = wave & 1;

    const int64_t kb_begin = (int64_t)split * kb_per_split;
    int64_t kb_end = kb_begin + kb_per_split;
    if (kb_end > kblocks)
        kb_end = kblocks;
    const int64_t n_st = kb_end > kb_begin ? kb_end - kb_begin : 0;

    // ---- this wave's copies: LPS line blocks from `src`, K block by K block
    const int64_t row_bytes = kblocks * kBlockBytes;   // one line block across all K
    const int mat = wave >> 1, part = wave & 1;
    const char *src;
    int dst_block0;
    if (mat == 0) {
        src = (HL == 2 && part ? Ll : Lh) +
              ((int64_t)tm * SL::MB + (HL == 2 ? 0 : part * LPS_A)) * row_bytes;
        dst_block0 = HL == 2 ? part * SL::MB : part * LPS_A;
    } else {
        src = (HL == 2 && part ? Rl : Rh) +
              ((int64_t)tn * SL::NB + (HL == 2 ? 0 : part * LPS_B)) * row_bytes;
        dst_block0 = HL * SL::MB + (HL == 2 ? part * SL::NB : part * LPS_B);
    }
    src += kb_begin * kBlockBytes;
    auto issue = [&](int64_t i, int slot) {     // stage i (relative) into ring slot
        char *dst = lds + slot * SL::bytes + dst_block0 * kBlockBytes;
        const char *s0 = src + i * kBlockBytes;
        if (mat == 0) {
#pragma unroll
            for (int b = 0; b < LPS_A; ++b)
                copy_block_to_lds(s0 + b * row_bytes, dst + b * kBlockBytes, lane);
        } else {
#pragma unroll
            for (int b = 0; b < LPS_B; ++b)
                copy_block_to_lds(s0 + b * row_bytes, dst + b * kBlockBytes, lane);
        }
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[i][j][r] = 0.0f;

    // Software pipeline.  Fragments of stage i sit in registers while stage
    // i's MFMAs run; in the middle of them the workgroup passes the barrier
    // for stage i+1, re-fills stage i's LDS slot with stage i+P's copies, and
    // reads stage i+1's fragments into the other register set, so LDS latency
    // hides behind the second half of stage i's MFMAs.
    Frags<T, HL, FM, FN> f0, f1;
    if (n_st > 0) {
#pragma unroll
        for (int i = 0; i < P; ++i)
            if (i < n_st)
                issue(i, i);
        const int64_t ahead0 = (n_st - 1) < (P - 1) ? (n_st - 1) : (P - 1);
        if (mat == 0)
            wait_stages_ahead<LPS_A>(ahead0);
        else
            wait_stages_ahead<LPS_B>(ahead0);
        ring_barrier();
        f0.read(lds, SL::MB, SL::NB, wm, wn, lane);
    }
    auto step = [&](int64_t i, Frags<T, HL, FM, FN> &cur, Frags<T, HL, FM, FN> &nxt) {
        mfma_list<0, kHalf>(acc, cur);
        if (i + 1 < n_st) {
            // copies of stage i+1 landed (this wave's: stages i+2 .. i+P-1 may
            // stay in flight); after the barrier every wave's did, and every
            // wave has consumed its reads of stage i's slot
            const int64_t ahead = (n_st - 2 - i) < (P - 2) ? (n_st - 2 - i) : (P - 2);
            if (mat == 0)
                wait_stages_ahead<LPS_A>(ahead);
            else
                wait_stages_ahead<LPS_B>(ahead);
            ring_barrier();
            if (i + P < n_st)
                issue(i + P, (int)(i % P));
            nxt.read(lds + (int)((i + 1) % P) * SL::bytes, SL::MB, SL::NB, wm, wn, lane);
        }
        mfma_list<kHalf, kTotal>(acc, cur);
    };
    int64_t i = 0;
    for (; i + 1 < n_st; i += 2) {
        step(i, f0, f1);
        step(i + 1, f1, f0);
    }
    if (i < n_st)
        step(i, f0, f1);

    // ---- epilogue: accumulator register r of a 32x32 block holds row
    // 8 (r / 4) + 4 (lane / 32) + (r mod 4), column lane mod 32.
    const int row_base = tm * BM + wm * (BM / 2);
    const int col_base = tn * BN + wn * (BN / 2);
    float *dst = splits == 1 ? out : partials + (int64_t)split * M * N;
    const int64_t ld = splits == 1 ? ldo : (int64_t)N;
    const bool acc_old = splits == 1 && accumulate != 0;
#pragma unroll
    for (int r0 = 0; r0 < FM; ++r0)
#pragma unroll
        for (int c0 = 0; c0 < FN; ++c0) {
            const int col = col_base + c0 * 32 + (lane & 31);
            if (col >= N)
                continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = row_base + r0 * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < M) {
                    float *p = dst + (int64_t)row * ld + col;
                    *p = acc_old ? *p + acc[r0][c0][r] : acc[r0][c0][r];
                }
            }
        }
}

// out[i] = (accumulate ? out[i] : 0) + partials[0][i] + ... + partials[S-1][i], in that order.
__global__ __launch_bounds__(256) void k_splitk_reduce(const float *__restrict__ partials,
                                                       int splits, int M, int N,
                                                       float *__restrict__ out, int64_t ldo,
                                                       int accumulate)
{
    const int64_t total = (int64_t)M * N;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t row = e / N, col = e % N;
        float s = partials[e];
        for (int k = 1; k < splits; ++k)
            s += partials[(int64_t)k * total + e];
        float *p = out + row * ldo + col;
        *p = accumulate ? *p + s : s;
    }
}

template <int BM, int BN, int PRODUCTS, typename T, int STAGES, int MINWG>
hipError_t launch_tile(const GemmPlan &plan, const void *Lh, const void *Ll, const void *Rh,
                       const void *Rl, int M, int N, float *out, int64_t ldo, float *partials,
                       bool accumulate, hipStream_t s)
{
    constexpr int HL = PRODUCTS == 3 ? 2 : 1;
    const int lds_bytes = STAGES * StageLayout<BM, BN, HL>::bytes;
    auto kern = k_gemm<BM, BN, PRODUCTS, T, STAGES, MINWG>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess)
        return e;
    const int tiles_m = plan.mblocks / (BM / 32);
    const int tiles_n = plan.nblocks / (BN / 32);
    const int64_t per = (plan.kblocks + plan.splits - 1) / plan.splits;
    const int total = tiles_m * tiles_n * plan.splits;
    const int grid = (total + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds_bytes, s, (const char *)Lh,
                       (const char *)Ll, (const char *)Rh, (const char *)Rl, plan.kblocks,
                       tiles_m, tiles_n, plan.splits, per, M, N, out, ldo, partials,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

// Built shapes: (BM, BN, ring depth, workgroups per CU).
#define CGH_GEMM_SHAPES(X)                                                                     \
    X(192, 192, 3, 2)                                                                          \
    X(192, 192, 5, 1)                                                                          \
    X(256, 192, 4, 1)                                                                          \
    X(192, 256, 4, 1)                                                                          \
    X(256, 128, 5, 1)                                                                          \
    X(128, 256, 5, 1)                                                                          \
    X(128, 128, 4, 2)                                                                          \
    X(128, 256, 3, 2)                                                                          \
    X(256, 128, 3, 2)

template <int PRODUCTS, typename T>
hipError_t launch_products(const GemmPlan &plan, const void *Lh, const void *Ll, const void *Rh,
                           const void *Rl, int M, int N, float *out, int64_t ldo,
                           float *partials, bool accumulate, hipStream_t s)
{
#define CGH_TILE(TBM, TBN, TST, TWG)                                                          \
    if (plan.bm == TBM && plan.bn == TBN && plan.stages == TST && plan.wg_per_cu == TWG)      \
        return launch_tile<TBM, TBN, PRODUCTS, T, TST, TWG>(plan, Lh, Ll, Rh, Rl, M, N, out,  \
                                                            ldo, partials, accumulate, s);
    CGH_GEMM_SHAPES(CGH_TILE)
#undef CGH_TILE
    return hipErrorInvalidValue;
}

}  // namespace

bool gemm_tile_supported(int bm, int bn, int stages, int wg_per_cu)
{
#define CGH_TILE(TBM, TBN, TST, TWG)                                                          \
    if (bm == TBM && bn == TBN && stages == TST && wg_per_cu == TWG)                          \
        return true;
    CGH_GEMM_SHAPES(CGH_TILE)
#undef CGH_TILE
    return false;
}

hipError_t launch_gemm(const GemmPlan &plan, FactorType ft, const void *Lh, const void *Ll,
                       const void *Rh, const void *Rl, int M, int N, float *out, int64_t ldo,
                       float *partials, bool accumulate, hipStream_t s)
{
    if (plan.products == 3) {
        if (ft == FactorType::BF16)
            return launch_products<3, __bf16>(plan, Lh, Ll, Rh, Rl, M, N, out, ldo, partials,
                                              accumulate, s);
        return launch_products<3, _Float16>(plan, Lh, Ll, Rh, Rl, M, N, out, ldo, partials,
                                            accumulate, s);
    }
    if (ft == FactorType::BF16)
        return launch_products<1, __bf16>(plan, Lh, Ll, Rh, Rl, M, N, out, ldo, partials,
                                          accumulate, s);
    return launch_products<1, _Float16>(plan, Lh, Ll, Rh, Rl, M, N, out, ldo, partials,
                                        accumulate, s);
}

hipError_t launch_splitk_reduce(const float *partials, int splits, int M, int N, float *out,
                                int64_t ldo, bool accumulate, hipStream_t s)
{
    const int64_t total = (int64_t)M * N;
    if (total <= 0)
        return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, s, partials, splits,
                       M, N, out, ldo, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace cgh
