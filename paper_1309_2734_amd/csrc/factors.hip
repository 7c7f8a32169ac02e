// Complex line factors of the separable form, split into hi + lo halves.
//
// With the FP64-reduced line phases U[ix, j], V[iy, j] (revolutions),
//     A_j cos(2 pi (U + V)) = A_j cos(2 pi V) cos(2 pi U) - A_j sin(2 pi V) sin(2 pi U),
// so the hologram of Eq. (5) is the real matrix product I = L R^T over
// K = 2N interleaved columns:
//     L[iy, 2j] =  A_j cos(2 pi V[iy, j]),   L[iy, 2j+1] = -A_j sin(2 pi V[iy, j]),
//     R[ix, 2j] =      cos(2 pi U[ix, j]),   R[ix, 2j+1] =      sin(2 pi U[ix, j]).
// The imaginary part of the object wave of Eq. (2),
//     A_j sin(2 pi (U + V)) = A_j sin(2 pi V) cos(2 pi U) + A_j cos(2 pi V) sin(2 pi U),
// uses the same R with the rows
//     L'[iy, 2j] = A_j sin(2 pi V[iy, j]),   L'[iy, 2j+1] =  A_j cos(2 pi V[iy, j]);
// for a complex evaluation L' is stacked under L (lines H .. 2H-1).
// In the 16-bit types each value v is stored as hi = round(v) and
// lo = round(v - hi) (round to nearest even; v - hi is exact in FP32), or as
// hi alone; FP32 factors are stored as computed.
//
// Storage order = the operand order of the matrix instructions: the matrix
// is cut into 1 KB blocks of 16 lines, a block being 64 lanes x 16 bytes;
// lane l holds line (l mod 16) and the next 16 bytes of K-columns of group
// l / 16.  In bf16/f16 (v_mfma_f32_16x16x32_*) that is K-columns
// 8 (l / 16) .. + 7, 4 points' (cos, sin) pairs, 16 points a block; in FP32
// (four v_mfma_f32_16x16x4_f32 per block, see gemm.hip) K-columns
// 4 (l / 16) .. + 3, 2 points, 8 points a block.  Blocks are ordered
// whole 1 KB units, so a GEMM stage copies whole 1 KB blocks straight
// into LDS.  Blocks are stored K-major (one slab of every array's line
// blocks per K block; FactorSet in common.h).  Lines past the hologram are
// written as zeros.
#include "common.h"

namespace cgh {
namespace {

// A (cos, sin) pair in the storage type, converted as one two-wide vector
// (round to nearest even; one packed convert where the target has it).
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename T>
struct PairOf {
    typedef T type __attribute__((ext_vector_type(2)));
};

// one lane's 16 bytes of a block: consecutive (cos, sin) pairs
template <typename T>
struct alignas(16) Vec16B {
    static constexpr int kValues = 16 / sizeof(T);
    typename PairOf<T>::type pair[kValues / 2];
};

// Grid: x = (group of kKBlocks consecutive K blocks) * 64 + lane, y = line
// block (L blocks first, then R).  A thread loads the constants of all its
// points first, then computes and stores block by block, so one wave has
// several blocks' loads in flight and its stores follow back to back.
constexpr int kKBlocks = 2;

// With RAW, the per-point constants come from the points themselves instead
// of precomputed arrays: the workgroup's threads first evaluate those of its
// own points (4 waves x kKBlocks K blocks) into LDS, with the formulas of the
// point-constant kernel, so a single hologram needs no separate constants
// launch.
template <typename T, bool SPLIT, bool RAW>
__global__ __launch_bounds__(256) void k_factors(PointConsts pc, RawPoints rp, int64_t slot0,
                                                 int64_t kblocks, int height, int width, int cplx,
                                                 int mblocks, FactorSet fs)
{
    constexpr int kLanePoints = Vec16B<T>::kValues / 2;      // (cos, sin) pairs per lane
    constexpr int kBlockPoints = 4 * kLanePoints;
    constexpr int kWgPoints = 4 * kKBlocks * kBlockPoints;   // points of the workgroup
    __shared__ double s_ctr[RAW ? kWgPoints : 1], s_beta[RAW ? kWgPoints : 1];
    __shared__ float s_amp[RAW ? kWgPoints : 1];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t kb0 = (t >> 6) * kKBlocks;
    const bool is_l = (int)blockIdx.y < mblocks;
    if (RAW) {
        if ((int)threadIdx.x < kWgPoints) {
            const int64_t slot = (int64_t)blockIdx.x * kWgPoints + threadIdx.x;
            double ctr = 0.0, beta = 0.0;
            float a = 0.0f;
            if (slot < rp.count) {   // padding slots: zero amplitude, zero phase
                const int64_t src = rp.src + slot;
                beta = rp.pitch * rp.pitch / (2.0 * rp.wavelength * (double)rp.z[src]);
                ctr = is_l ? rp.half_h + (double)rp.y[src] / rp.pitch
                           : rp.half_w + (double)rp.x[src] / rp.pitch;
                a = rp.amp[src];
            }
            s_ctr[threadIdx.x] = ctr;
            s_beta[threadIdx.x] = beta;
            s_amp[threadIdx.x] = a;
        }
        __syncthreads();
    }
    if (kb0 >= kblocks)
        return;
    const int lane = (int)(t & 63);
    const int rb = is_l ? (int)blockIdx.y : (int)blockIdx.y - mblocks;
    const int line = rb * kFragLines + (lane & (kFragLines - 1));
    const int lines = is_l ? (cplx ? 2 * height : height) : width;
    const bool valid = line < lines;
    const bool im_part = is_l && line >= height;           // rows of L' (complex only)
    const int src_line = im_part ? line - height : line;
    const double dline = (double)src_line;
    const int nkb = kblocks - kb0 < kKBlocks ? (int)(kblocks - kb0) : kKBlocks;

    // constants of this lane's points in the group's blocks (blocks past
    // kblocks re-read the last one; their results are not stored)
    double ctr[kKBlocks][kLanePoints], beta[kKBlocks][kLanePoints];
    float amp[kKBlocks][kLanePoints];
#pragma unroll
    for (int b = 0; b < kKBlocks; ++b) {
        const int64_t kb = kb0 + (b < nkb ? b : nkb - 1);
        const int64_t j0 = slot0 + kb * kBlockPoints + kLanePoints * (lane / kFragLines);
#pragma unroll
        for (int p = 0; p < kLanePoints; ++p) {
            if (RAW) {
                const int64_t q = j0 - slot0 - (int64_t)blockIdx.x * kWgPoints + p;
                ctr[b][p] = s_ctr[q];
                beta[b][p] = s_beta[q];
                amp[b][p] = s_amp[q];
            } else {
                ctr[b][p] = is_l ? pc.cy[j0 + p] : pc.cx[j0 + p];
                beta[b][p] = pc.beta[j0 + p];
                amp[b][p] = pc.amp[j0 + p];
            }
        }
    }

    Vec16B<T> *out = reinterpret_cast<Vec16B<T> *>(fs.base);
    const int hi_blk = (is_l ? fs.first_l(false) : fs.first_r(false)) + rb;
    const int lo_blk = (is_l ? fs.first_l(true) : fs.first_r(true)) + rb;
#pragma unroll
    for (int b = 0; b < kKBlocks; ++b) {
        if (b >= nkb)
            break;
        Vec16B<T> hi, lo;
#pragma unroll
        for (int p = 0; p < kLanePoints; ++p) {
            const double d = dline - ctr[b][p];
            const float ph = (float)__builtin_amdgcn_fract(beta[b][p] * (d * d));
            float c = __builtin_amdgcn_cosf(ph);     // cos(2 pi ph)
            float s = __builtin_amdgcn_sinf(ph);     // sin(2 pi ph)
            if (im_part) {
                const float a = amp[b][p];
                const float ac = a * c;
                c = a * s;
                s = ac;
            } else if (is_l) {
                const float a = amp[b][p];
                c = a * c;
                s = -a * s;
            }
            if (!valid) {
                c = 0.0f;
                s = 0.0f;
            }
            using P2 = typename PairOf<T>::type;
            const f32x2 v = {c, s};
            const P2 h = __builtin_convertvector(v, P2);
            hi.pair[p] = h;
            if (SPLIT)   // v - hi is exact in FP32
                lo.pair[p] = __builtin_convertvector(v - __builtin_convertvector(h, f32x2), P2);
        }
        const int64_t slab = (kb0 + b) * fs.slab_blocks();
        out[(slab + hi_blk) * 64 + lane] = hi;
        if (SPLIT)
            out[(slab + lo_blk) * 64 + lane] = lo;
    }
}

template <typename T, bool RAW>
hipError_t launch_t(PointConsts pc, const RawPoints &rp, int64_t slot0, int width, int height,
                    int cplx, int64_t kblocks, int mblocks, int nblocks, const FactorSet &fs,
                    hipStream_t s)
{
    const int64_t groups = (kblocks + kKBlocks - 1) / kKBlocks;
    const dim3 grid((unsigned)((groups * 64 + 255) / 256), (unsigned)(mblocks + nblocks));
    if (fs.hl == 2)
        hipLaunchKernelGGL((k_factors<T, sizeof(T) == 2, RAW>), grid, dim3(256), 0, s, pc, rp,
                           slot0, kblocks, height, width, cplx, mblocks, fs);
    else
        hipLaunchKernelGGL((k_factors<T, false, RAW>), grid, dim3(256), 0, s, pc, rp, slot0,
                           kblocks, height, width, cplx, mblocks, fs);
    return hipGetLastError();
}

bool factors_fit(int64_t kblocks, int mblocks, int nblocks, FactorType ft, const FactorSet &fs)
{
    return fs.base != nullptr && kblocks <= fs.kblocks && mblocks <= fs.amb &&
           nblocks <= fs.anb && (fs.hl == 1 || fs.hl == 2) &&
           !(ft == FactorType::FP32 && fs.hl != 1);
}

}  // namespace

hipError_t launch_factors(PointConsts pc, int64_t slot0, int width, int height, bool cplx,
                          int64_t kblocks, int mblocks, int nblocks, FactorType ft,
                          const FactorSet &fs, hipStream_t s)
{
    if (kblocks <= 0 || mblocks + nblocks <= 0)
        return hipSuccess;
    if (!factors_fit(kblocks, mblocks, nblocks, ft, fs))   // the written blocks must lie in the set
        return hipErrorInvalidValue;
    const int cx = cplx ? 1 : 0;
    const RawPoints none{};
    if (ft == FactorType::BF16)
        return launch_t<__bf16, false>(pc, none, slot0, width, height, cx, kblocks, mblocks,
                                       nblocks, fs, s);
    if (ft == FactorType::FP32)
        return launch_t<float, false>(pc, none, slot0, width, height, cx, kblocks, mblocks,
                                      nblocks, fs, s);
    return launch_t<_Float16, false>(pc, none, slot0, width, height, cx, kblocks, mblocks,
                                     nblocks, fs, s);
}

hipError_t launch_factors_points(const RawPoints &rp, int width, int height, bool cplx,
                                 int64_t kblocks, int mblocks, int nblocks, FactorType ft,
                                 const FactorSet &fs, hipStream_t s)
{
    if (kblocks <= 0 || mblocks + nblocks <= 0)
        return hipSuccess;
    if (!factors_fit(kblocks, mblocks, nblocks, ft, fs))
        return hipErrorInvalidValue;
    const int cx = cplx ? 1 : 0;
    const PointConsts none{};
    if (ft == FactorType::BF16)
        return launch_t<__bf16, true>(none, rp, 0, width, height, cx, kblocks, mblocks, nblocks,
                                      fs, s);
    if (ft == FactorType::FP32)
        return launch_t<float, true>(none, rp, 0, width, height, cx, kblocks, mblocks, nblocks,
                                     fs, s);
    return launch_t<_Float16, true>(none, rp, 0, width, height, cx, kblocks, mblocks, nblocks,
                                    fs, s);
}

}  // namespace cgh
