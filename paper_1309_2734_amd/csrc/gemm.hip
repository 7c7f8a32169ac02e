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
//   - a stage covers 2 K blocks (32 K-columns = 16 points); its operand
//     blocks (1 KB each, already in MFMA lane order in memory) are copied
//     straight into LDS with global_load_lds_dwordx4 (no register staging),
//     two stages in flight (double buffer, one barrier per stage);
//   - each wave reads its fragments with conflict-free ds_read_b128 (lane l
//     reads bytes 16 l .. 16 l + 15 of a block) and issues, per K block,
//     3 x (BM/64) x (BN/64) MFMAs, ordered product-major so that consecutive
//     MFMAs never write the same accumulator.
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
constexpr int kStageK = 2;          // K blocks per stage

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

// LDS stage layout (blocks of 1 KB): [A hi: MB x kStageK][A lo][B hi: NB x kStageK][B lo]
template <int BM, int BN, int HL>
struct StageLayout {
    static constexpr int MB = BM / 32;
    static constexpr int NB = BN / 32;
    static constexpr int a_blocks = MB * kStageK;
    static constexpr int b_blocks = NB * kStageK;
    static constexpr int blocks = HL * (a_blocks + b_blocks);
    static constexpr int bytes = blocks * kBlockBytes;
};

template <int BM, int BN, int PRODUCTS, typename T>
__global__ __launch_bounds__(256, 1) void k_gemm(const char *__restrict__ Lh,
                                                 const char *__restrict__ Ll,
                                                 const char *__restrict__ Rh,
                                                 const char *__restrict__ Rl, int64_t kblocks,
                                                 int tiles_m, int tiles_n, int splits,
                                                 int64_t stages_per_split, int M, int N,
                                                 float *__restrict__ out, int64_t ldo,
                                                 float *__restrict__ partials, int accumulate)
{
    constexpr int HL = PRODUCTS == 3 ? 2 : 1;
    typedef StageLayout<BM, BN, HL> SL;
    constexpr int FM = BM / 64;   // 32x32 blocks per wave along M
    constexpr int FN = BN / 64;   // ... along N
    typedef typename Frag<T>::type frag_t;
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

    const int64_t total_stages = kblocks / kStageK;
    const int64_t s_begin = (int64_t)split * stages_per_split;
    int64_t s_end = s_begin + stages_per_split;
    if (s_end > total_stages)
        s_end = total_stages;

    // operand row-block bases (bytes) for this tile
    const int64_t row_bytes = kblocks * kBlockBytes;   // one line block across all K
    const char *a_src[2] = {Lh + (int64_t)tm * SL::MB * row_bytes,
                            HL == 2 ? Ll + (int64_t)tm * SL::MB * row_bytes : nullptr};
    const char *b_src[2] = {Rh + (int64_t)tn * SL::NB * row_bytes,
                            HL == 2 ? Rl + (int64_t)tn * SL::NB * row_bytes : nullptr};

    // Issue the copies of stage `st` into LDS buffer `buf`.  Waves 0, 1 copy
    // L blocks, waves 2, 3 copy R blocks; with hi and lo factors, the odd wave
    // takes the lo copy, otherwise the two waves split the line blocks.
    const int mat = wave >> 1, part = wave & 1;
    auto issue = [&](int64_t st, int buf) {
        char *base = lds + buf * SL::bytes;
        const int64_t kofs = st * kStageK * (int64_t)kBlockBytes;
        if (mat == 0) {
            constexpr int n = HL == 2 ? SL::a_blocks : SL::a_blocks / 2;
            const char *src = (HL == 2 ? a_src[part] : a_src[0]) + kofs;
            char *dst = base + (HL == 2 ? part * SL::a_blocks : 0) * kBlockBytes;
            const int first = HL == 2 ? 0 : part * n;
#pragma unroll
            for (int it = 0; it < n; ++it) {
                const int i = first + it;             // i = rb * kStageK + kk
                copy_block_to_lds(src + (int64_t)(i / kStageK) * row_bytes +
                                      (i % kStageK) * kBlockBytes,
                                  dst + i * kBlockBytes, lane);
            }
        } else {
            constexpr int n = HL == 2 ? SL::b_blocks : SL::b_blocks / 2;
            const char *src = (HL == 2 ? b_src[part] : b_src[0]) + kofs;
            char *dst = base + (HL * SL::a_blocks + (HL == 2 ? part * SL::b_blocks : 0)) * kBlockBytes;
            const int first = HL == 2 ? 0 : part * n;
#pragma unroll
            for (int it = 0; it < n; ++it) {
                const int i = first + it;
                copy_block_to_lds(src + (int64_t)(i / kStageK) * row_bytes +
                                      (i % kStageK) * kBlockBytes,
                                  dst + i * kBlockBytes, lane);
            }
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

    if (s_begin < s_end)
        issue(s_begin, 0);
    for (int64_t st = s_begin; st < s_end; ++st) {
        const int buf = (int)((st - s_begin) & 1);
        // own copies of this stage landed; then every wave's did, and every
        // wave is done reading the other buffer
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (st + 1 < s_end)
            issue(st + 1, buf ^ 1);
        const char *base = lds + buf * SL::bytes;
#pragma unroll
        for (int kk = 0; kk < kStageK; ++kk) {
            frag_t a[HL][FM], b[HL][FN];
#pragma unroll
            for (int h = 0; h < HL; ++h) {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int blk = h * SL::a_blocks + (wm * FM + i) * kStageK + kk;
                    a[h][i] = *reinterpret_cast<const frag_t *>(base + blk * kBlockBytes + lane * 16);
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int blk = HL * SL::a_blocks + h * SL::b_blocks + (wn * FN + j) * kStageK + kk;
                    b[h][j] = *reinterpret_cast<const frag_t *>(base + blk * kBlockBytes + lane * 16);
                }
            }
            // hi * hi
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = Frag<T>::mfma(a[0][i], b[0][j], acc[i][j]);
            if (PRODUCTS == 3) {
                // hi * lo, then lo * hi
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = Frag<T>::mfma(a[0][i], b[HL - 1][j], acc[i][j]);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = Frag<T>::mfma(a[HL - 1][i], b[0][j], acc[i][j]);
            }
        }
    }

    // ---- epilogue: accumulator register r of a 32x32 block holds row
    // 8 (r / 4) + 4 (lane / 32) + (r mod 4), column lane mod 32.
    const int row_base = tm * BM + wm * (BM / 2);
    const int col_base = tn * BN + wn * (BN / 2);
    float *dst = splits == 1 ? out : partials + (int64_t)split * M * N;
    const int64_t ld = splits == 1 ? ldo : (int64_t)N;
    const bool acc_old = splits == 1 && accumulate != 0;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = col_base + j * 32 + (lane & 31);
            if (col >= N)
                continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = row_base + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < M) {
                    float *p = dst + (int64_t)row * ld + col;
                    *p = acc_old ? *p + acc[i][j][r] : acc[i][j][r];
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

template <int BM, int BN, int PRODUCTS, typename T>
hipError_t launch_tile(const GemmPlan &plan, const void *Lh, const void *Ll, const void *Rh,
                       const void *Rl, int M, int N, float *out, int64_t ldo, float *partials,
                       bool accumulate, hipStream_t s)
{
    constexpr int HL = PRODUCTS == 3 ? 2 : 1;
    const int lds_bytes = 2 * StageLayout<BM, BN, HL>::bytes;
    auto kern = k_gemm<BM, BN, PRODUCTS, T>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess)
        return e;
    const int tiles_m = plan.mblocks / (BM / 32);
    const int tiles_n = plan.nblocks / (BN / 32);
    const int64_t total_stages = plan.kblocks / kStageK;
    const int64_t per = (total_stages + plan.splits - 1) / plan.splits;
    const int total = tiles_m * tiles_n * plan.splits;
    const int grid = (total + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds_bytes, s, (const char *)Lh,
                       (const char *)Ll, (const char *)Rh, (const char *)Rl, plan.kblocks,
                       tiles_m, tiles_n, plan.splits, per, M, N, out, ldo, partials,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

template <int PRODUCTS, typename T>
hipError_t launch_products(const GemmPlan &plan, const void *Lh, const void *Ll, const void *Rh,
                           const void *Rl, int M, int N, float *out, int64_t ldo,
                           float *partials, bool accumulate, hipStream_t s)
{
#define CGH_TILE(TBM, TBN)                                                                    \
    if (plan.bm == TBM && plan.bn == TBN)                                                     \
        return launch_tile<TBM, TBN, PRODUCTS, T>(plan, Lh, Ll, Rh, Rl, M, N, out, ldo,         \
                                                  partials, accumulate, s);
    CGH_TILE(256, 192)
    CGH_TILE(192, 256)
    CGH_TILE(192, 192)
    CGH_TILE(128, 256)
    CGH_TILE(256, 128)
    CGH_TILE(128, 128)
#undef CGH_TILE
    return hipErrorInvalidValue;
}

}  // namespace

bool gemm_tile_supported(int bm, int bn)
{
    return (bm == 256 && (bn == 192 || bn == 128)) ||
           (bm == 192 && (bn == 256 || bn == 192)) || (bm == 128 && (bn == 256 || bn == 128));
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
