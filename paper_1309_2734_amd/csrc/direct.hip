// Direct FP32 evaluation of the amplitude hologram (Section 2.1, Eq. (5) with
// the Fresnel phase of Eq. (2)): one cosine per point and pixel.
//
// Mapping on gfx950.  A wave's 64 lanes own 64 consecutive pixel columns
// (coalesced loads of the column table and coalesced stores), and each lane
// owns R rows.  Points are taken 16 at a time (one table group):
//   - the lane loads its column's 16 reduced column phases U[ix, j] with four
//     16-byte loads (table blocked as [group][column][16]);
//   - lane l also loads, for each of its R rows, the row phase V[iy, j] of
//     point j = 16 g + (l mod 16); each 16-lane DPP row thus holds the row
//     phases of all 16 points.  The 16 amplitudes are wave-uniform and go to
//     scalar registers;
//   - for point k of the group, the row phase is broadcast from lane k of
//     each 16-lane row with DPP row_newbcast, folded into the add:
//         t = V[row, k] (broadcast) + U[col, k]      v_add_f32_dpp
//         c = cos(2 pi t)                            v_cos_f32 (input in revolutions)
//         acc = fma(A_k (scalar), c, acc)            v_fmac_f32
//     t lies in [0, 2] because U and V were reduced in FP64, which is inside
//     the hardware cosine's domain and keeps its absolute error ~1e-7.
// No LDS, no barrier: the four waves of a workgroup take the same 64 columns
// and consecutive row bands, so their column-table loads hit in L1.
// Accumulation: a fresh FP32 partial per 32 points, added to the running sum.
// The complex variant (CPLX) also accumulates the imaginary part of the
// object wave of Eq. (2), A_k sin(2 pi t) with v_sin_f32, for the phase-only
// hologram of Eq. (3).
#include "common.h"

namespace cgh {
namespace {

constexpr int kWaves = 4;

template <int R>
struct GroupRegs {
    float4 u[4];      // U[col, 16g + 0..15]
    float v[R];       // V[row_r, 16g + lane%16]
    float a[kGroup];  // A[16g + 0..15]: wave-uniform, held in scalar registers
};

// Tables are padded to whole 64-column / 64-row blocks, so no load needs a
// bounds clamp: the R row phases of a lane are R consecutive table lines.
template <int R>
__device__ __forceinline__ void load_group(GroupRegs<R> &G, const float *__restrict__ Ug,
                                           const float *__restrict__ Vg,
                                           const float *__restrict__ Ag)
{
    const float4 *up = reinterpret_cast<const float4 *>(Ug);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        G.u[i] = up[i];
#pragma unroll
    for (int r = 0; r < R; ++r)
        G.v[r] = Vg[r * kGroup];
#pragma unroll
    for (int k = 0; k < kGroup; ++k)
        G.a[k] = Ag[k];
}

template <int K, int R, bool CPLX>
__device__ __forceinline__ void point_step(const GroupRegs<R> &G, float *part, float *part_im)
{
    const float uk = reinterpret_cast<const float *>(G.u)[K];
    const float ak = G.a[K];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float t = row_bcast<K>(G.v[r]) + uk;
        part[r] = __builtin_fmaf(ak, __builtin_amdgcn_cosf(t), part[r]);
        if (CPLX)
            part_im[r] = __builtin_fmaf(ak, __builtin_amdgcn_sinf(t), part_im[r]);
    }
}

template <int R, bool CPLX>
__device__ __forceinline__ void group_step(const GroupRegs<R> &G, float *p, float *q)
{
    point_step<0, R, CPLX>(G, p, q);   point_step<1, R, CPLX>(G, p, q);
    point_step<2, R, CPLX>(G, p, q);   point_step<3, R, CPLX>(G, p, q);
    point_step<4, R, CPLX>(G, p, q);   point_step<5, R, CPLX>(G, p, q);
    point_step<6, R, CPLX>(G, p, q);   point_step<7, R, CPLX>(G, p, q);
    point_step<8, R, CPLX>(G, p, q);   point_step<9, R, CPLX>(G, p, q);
    point_step<10, R, CPLX>(G, p, q);  point_step<11, R, CPLX>(G, p, q);
    point_step<12, R, CPLX>(G, p, q);  point_step<13, R, CPLX>(G, p, q);
    point_step<14, R, CPLX>(G, p, q);  point_step<15, R, CPLX>(G, p, q);
}

// Grid: x = column blocks of 64, y = row bands of kWaves * R rows, z = frame.
// Tables: U [groups][wpad][16], V [groups][hpad][16]; wpad, hpad multiples of
// 64; every frame's group count is even.  CPLX: the imaginary part goes to
// out_im (same layout and offsets as out).
template <int R, bool CPLX>
__global__ __launch_bounds__(256) void k_direct(const float *__restrict__ U,
                                                const float *__restrict__ V,
                                                const float *__restrict__ amp,
                                                FrameList frames, int width,
                                                int height, int wpad, int hpad,
                                                float *__restrict__ out,
                                                float *__restrict__ out_im, int accumulate)
{
    const FrameDesc fd = frame_at(frames, blockIdx.z);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = blockIdx.x * 64 + lane;
    const int row0 = (blockIdx.y * kWaves + wave) * R;

    // group g of this frame: U at Ug + g*ustep, V at Vg + g*vstep, A at Ag + 16 g
    const int64_t ustep = (int64_t)wpad * kGroup;
    const int64_t vstep = (int64_t)hpad * kGroup;
    const float *Ug = U + fd.first * wpad + (int64_t)col * kGroup;
    const float *Vg = V + fd.first * hpad + (int64_t)row0 * kGroup + (lane & (kGroup - 1));
    const float *Ag = amp + fd.first;

    float acc[R], part[R];
    float acc_im[CPLX ? R : 1], part_im[CPLX ? R : 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[r] = 0.0f;
        part[r] = 0.0f;
        if (CPLX) {
            acc_im[r] = 0.0f;
            part_im[r] = 0.0f;
        }
    }
    // Two register sets in ping-pong: the loads of the next group are in
    // flight while the current one is evaluated.  The last prefetch re-reads
    // the final group (in bounds, unused) so the loop body has no branch.
    const int64_t G = fd.groups;
    GroupRegs<R> ga, gb;
    if (G > 0)
        load_group<R>(ga, Ug, Vg, Ag);
    // G is even (slots are padded to kSlotAlign = 2 groups); the clamp only
    // keeps the loads inside the frame's tables should that ever not hold.
    for (int64_t g = 0; g < G; g += 2) {
        const int64_t g1 = g + 1 < G ? g + 1 : G - 1;
        load_group<R>(gb, Ug + g1 * ustep, Vg + g1 * vstep, Ag + g1 * kGroup);
        group_step<R, CPLX>(ga, part, part_im);
        const int64_t gn = g + 2 < G ? g + 2 : G - 1;
        load_group<R>(ga, Ug + gn * ustep, Vg + gn * vstep, Ag + gn * kGroup);
        group_step<R, CPLX>(gb, part, part_im);
        // a fresh partial every 32 points keeps the FP32 running sum's
        // rounding error small
#pragma unroll
        for (int r = 0; r < R; ++r) {
            acc[r] += part[r];
            part[r] = 0.0f;
            if (CPLX) {
                acc_im[r] += part_im[r];
                part_im[r] = 0.0f;
            }
        }
    }
    if (col < width) {
        float *o = out + fd.out_off;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (row0 + r < height) {
                float *p = o + (int64_t)(row0 + r) * width + col;
                *p = accumulate ? *p + acc[r] : acc[r];
            }
        if (CPLX) {
            float *oi = out_im + fd.out_off;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (row0 + r < height) {
                    float *p = oi + (int64_t)(row0 + r) * width + col;
                    *p = accumulate ? *p + acc_im[r] : acc_im[r];
                }
        }
    }
}

template <int R>
void launch_rows(const float *U, const float *V, const float *amp, const FrameList &frames,
                 int n_frames, int width, int height, int wpad, int hpad, float *out,
                 float *out_im, int acc, hipStream_t s)
{
    const dim3 grid((unsigned)((width + 63) / 64),
                    (unsigned)((height + kWaves * R - 1) / (kWaves * R)), (unsigned)n_frames);
    if (out_im != nullptr)
        hipLaunchKernelGGL((k_direct<R, true>), grid, dim3(256), 0, s, U, V, amp, frames,
                           width, height, wpad, hpad, out, out_im, acc);
    else
        hipLaunchKernelGGL((k_direct<R, false>), grid, dim3(256), 0, s, U, V, amp, frames,
                           width, height, wpad, hpad, out, (float *)nullptr, acc);
}

}  // namespace

hipError_t launch_direct(const float *U, const float *V, const float *amp,
                         const FrameList &frames, int n_frames, int width, int height,
                         int wpad, int hpad, int rows_per_wave, float *out, float *out_im,
                         bool accumulate, hipStream_t s)
{
    const int acc = accumulate ? 1 : 0;
    if (n_frames <= 0)
        return hipSuccess;
    if (rows_per_wave == 8)
        launch_rows<8>(U, V, amp, frames, n_frames, width, height, wpad, hpad, out, out_im,
                       acc, s);
    else if (rows_per_wave == 16)
        launch_rows<16>(U, V, amp, frames, n_frames, width, height, wpad, hpad, out, out_im,
                        acc, s);
    else
        launch_rows<4>(U, V, amp, frames, n_frames, width, height, wpad, hpad, out, out_im,
                       acc, s);
    return hipGetLastError();
}

}  // namespace cgh
