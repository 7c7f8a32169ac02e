// Direct FP32 evaluation of the exact spherical wave of Eq. (1) (Section
// 2.1): O = sum_j A_j exp(i 2 pi d_j / lambda), d_j = sqrt(r_j^2 + z_j^2),
// r_j^2 = (x_h - x_j)^2 + (y_h - y_j)^2; the hologram is its real part (the
// first line of Eq. (5) with phi_r = 0 and without the constant 2 A_r).
//
// d / lambda reaches ~10^6 revolutions, far beyond FP32.  It is split into
// the Fresnel phase of Eq. (2) and a small non-separable remainder:
//     d / lambda = z / lambda + r^2 / (2 z lambda) - (d - z)^2 / (2 z lambda),
// an identity, since d^2 = r^2 + z^2.  The first two terms are the separable
// part, reduced modulo one revolution in FP64 per line as for Eq. (2) (z /
// lambda folded into the row table).  The remainder has no cancellation when
// written with rho = r^2 / z^2:
//     (d - z)^2 / (2 z lambda) = (z / (2 lambda)) w^2,   w = (d - z) / z = rho / (1 + sqrt(1 + rho)),
// so it is evaluated per point and pixel in FP32 with a relative error of a
// few 1e-7 (of a term below 0.1 revolution at paraxial geometries).
//
// Mapping as the direct kernel of Eq. (5) (direct.hip): lanes = 64 columns,
// R rows per lane, 16 points per group; the row tables V and Y are broadcast
// from lane k of each 16-lane row by DPP, folded into the adds.  Per point
// and pixel:
//     rho = Y[row, k] (bcast) + X[col, k]         v_add_f32_dpp
//     s   = sqrt(1 + rho)                         v_add_f32, v_sqrt_f32
//     w   = rho / (1 + s)                         v_add_f32, v_rcp_f32, v_mul_f32
//     t   = V[row, k] (bcast) + U[col, k]         v_add_f32_dpp
//     t   = t - zhalf_k w^2                       v_mul_f32, v_fma_f32 (zhalf_k scalar)
//     acc = fma(A_k, cos(2 pi t), acc)            v_cos_f32, v_fmac_f32 (A_k scalar)
// and for the complex variant a sine and a second accumulator.
#include "common.h"

namespace cgh {
namespace {

constexpr int kWaves = 4;

template <int R>
struct SphereRegs {
    float4 u[4];        // U[col, 16g + 0..15]
    float4 x[4];        // X[col, 16g + 0..15]
    float v[R];         // V[row_r, 16g + lane%16]
    float y[R];         // Y[row_r, 16g + lane%16]
    float a[kGroup];    // A_j: wave-uniform (scalar registers)
    float zh[kGroup];   // z_j / (2 lambda): wave-uniform
};

template <int R>
__device__ __forceinline__ void load_group(SphereRegs<R> &G, const float *__restrict__ Ug,
                                           const float *__restrict__ Xg,
                                           const float *__restrict__ Vg,
                                           const float *__restrict__ Yg,
                                           const float *__restrict__ Ag,
                                           const float *__restrict__ Zg)
{
    const float4 *up = reinterpret_cast<const float4 *>(Ug);
    const float4 *xp = reinterpret_cast<const float4 *>(Xg);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        G.u[i] = up[i];
        G.x[i] = xp[i];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        G.v[r] = Vg[r * kGroup];
        G.y[r] = Yg[r * kGroup];
    }
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
        G.a[k] = Ag[k];
        G.zh[k] = Zg[k];
    }
}

template <int K, int R, bool CPLX>
__device__ __forceinline__ void point_step(const SphereRegs<R> &G, float *part, float *part_im)
{
    const float uk = reinterpret_cast<const float *>(G.u)[K];
    const float xk = reinterpret_cast<const float *>(G.x)[K];
    const float ak = G.a[K];
    const float zk = G.zh[K];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float rho = row_bcast<K>(G.y[r]) + xk;
        const float s = __builtin_amdgcn_sqrtf(1.0f + rho);
        const float w = rho * __builtin_amdgcn_rcpf(1.0f + s);
        float t = row_bcast<K>(G.v[r]) + uk;
        t = __builtin_fmaf(-zk, w * w, t);
        part[r] = __builtin_fmaf(ak, __builtin_amdgcn_cosf(t), part[r]);
        if (CPLX)
            part_im[r] = __builtin_fmaf(ak, __builtin_amdgcn_sinf(t), part_im[r]);
    }
}

template <int R, bool CPLX>
__device__ __forceinline__ void group_step(const SphereRegs<R> &G, float *p, float *q)
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
// Tables: U, X [groups][wpad][16]; V, Y [groups][hpad][16]; wpad, hpad
// multiples of 64; every frame's group count is even.
template <int R, bool CPLX>
__global__ __launch_bounds__(256) void k_direct_sphere(
    const float *__restrict__ U, const float *__restrict__ V, const float *__restrict__ X,
    const float *__restrict__ Y, const float *__restrict__ amp, const float *__restrict__ zhalf,
    FrameList frames, int width, int height, int wpad, int hpad,
    float *__restrict__ out, float *__restrict__ out_im, int accumulate)
{
    const FrameDesc fd = frame_at(frames, blockIdx.z);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = blockIdx.x * 64 + lane;
    const int row0 = (blockIdx.y * kWaves + wave) * R;

    const int64_t ustep = (int64_t)wpad * kGroup;
    const int64_t vstep = (int64_t)hpad * kGroup;
    const int64_t coff = fd.first * wpad + (int64_t)col * kGroup;
    const int64_t roff = fd.first * hpad + (int64_t)row0 * kGroup + (lane & (kGroup - 1));
    const float *Ug = U + coff, *Xg = X + coff;
    const float *Vg = V + roff, *Yg = Y + roff;
    const float *Ag = amp + fd.first, *Zg = zhalf + fd.first;

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
    // ping-pong register sets as in the Eq. (5) kernel; G is even
    const int64_t G = fd.groups;
    SphereRegs<R> ga, gb;
    if (G > 0)
        load_group<R>(ga, Ug, Xg, Vg, Yg, Ag, Zg);
    for (int64_t g = 0; g < G; g += 2) {
        const int64_t g1 = g + 1 < G ? g + 1 : G - 1;
        load_group<R>(gb, Ug + g1 * ustep, Xg + g1 * ustep, Vg + g1 * vstep, Yg + g1 * vstep,
                      Ag + g1 * kGroup, Zg + g1 * kGroup);
        group_step<R, CPLX>(ga, part, part_im);
        const int64_t gn = g + 2 < G ? g + 2 : G - 1;
        load_group<R>(ga, Ug + gn * ustep, Xg + gn * ustep, Vg + gn * vstep, Yg + gn * vstep,
                      Ag + gn * kGroup, Zg + gn * kGroup);
        group_step<R, CPLX>(gb, part, part_im);
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

// a2s: a thread writes four consecutive entries of one table line of a
// group in each of its two tables (16-byte stores; consecutive threads write
// consecutive 16 bytes); blockIdx.y strides over the groups.  Padding slots
// (zlam = 0, amplitude 0) get zero offsets.
__global__ __launch_bounds__(256) void k_sphere_tables(PointConsts pc, int64_t n_groups,
                                                       int wpad, int hpad,
                                                       float *__restrict__ U,
                                                       float *__restrict__ V,
                                                       float *__restrict__ X,
                                                       float *__restrict__ Y)
{
    constexpr int kQuads = kGroup / 4;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int line_all = idx / kQuads;
    const int q0 = 4 * (idx % kQuads);
    if (line_all >= wpad + hpad)
        return;
    const bool is_u = line_all < wpad;
    const int line = is_u ? line_all : line_all - wpad;
    const double *ctr = is_u ? pc.cx : pc.cy;
    float *phase = is_u ? U : V;
    float *offset = is_u ? X : Y;
    const int64_t lines = is_u ? wpad : hpad;
    for (int64_t g = blockIdx.y; g < n_groups; g += gridDim.y) {
        const int64_t j0 = g * kGroup + q0;
        float ph[4], off[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = j0 + u;
            const double beta = pc.beta[j], zl = pc.zlam[j];
            const double d = (double)line - ctr[j];
            const double d2 = d * d;
            // (p / z)^2 = 2 beta / (z / lambda)
            const double rs = zl > 0.0 ? 2.0 * beta / zl : 0.0;
            off[u] = (float)(d2 * rs);
            ph[u] = (float)__builtin_amdgcn_fract(is_u ? beta * d2 : beta * d2 + zl);
        }
        const int64_t e = (g * lines + line) * kGroup + q0;
        *reinterpret_cast<float4 *>(phase + e) = float4{ph[0], ph[1], ph[2], ph[3]};
        *reinterpret_cast<float4 *>(offset + e) = float4{off[0], off[1], off[2], off[3]};
    }
}

template <int R>
void launch_rows(const float *U, const float *V, const float *X, const float *Y,
                 const float *amp, const float *zhalf, const FrameList &frames, int n_frames,
                 int width, int height, int wpad, int hpad, float *out, float *out_im, int acc,
                 hipStream_t s)
{
    const dim3 grid((unsigned)((width + 63) / 64),
                    (unsigned)((height + kWaves * R - 1) / (kWaves * R)), (unsigned)n_frames);
    if (out_im != nullptr)
        hipLaunchKernelGGL((k_direct_sphere<R, true>), grid, dim3(256), 0, s, U, V, X, Y, amp,
                           zhalf, frames, width, height, wpad, hpad, out, out_im, acc);
    else
        hipLaunchKernelGGL((k_direct_sphere<R, false>), grid, dim3(256), 0, s, U, V, X, Y, amp,
                           zhalf, frames, width, height, wpad, hpad, out, (float *)nullptr,
                           acc);
}

}  // namespace

hipError_t launch_sphere_tables(PointConsts pc, int64_t n_slots, int wpad, int hpad, float *U,
                                float *V, float *X, float *Y, hipStream_t s)
{
    if (n_slots <= 0)
        return hipSuccess;
    const int64_t groups = n_slots / kGroup;
    const unsigned bx = (unsigned)(((int64_t)(wpad + hpad) * (kGroup / 4) + 255) / 256);
    const unsigned by = (unsigned)(groups < 65535 ? groups : 65535);
    hipLaunchKernelGGL(k_sphere_tables, dim3(bx, by), dim3(256), 0, s, pc, groups, wpad, hpad, U,
                       V, X, Y);
    return hipGetLastError();
}

hipError_t launch_direct_sphere(const float *U, const float *V, const float *X, const float *Y,
                                const float *amp, const float *zhalf,
                                const FrameList &frames, int n_frames, int width, int height,
                                int wpad, int hpad, int rows_per_wave, float *out,
                                float *out_im, bool accumulate, hipStream_t s)
{
    const int acc = accumulate ? 1 : 0;
    if (n_frames <= 0)
        return hipSuccess;
    if (rows_per_wave == 8)
        launch_rows<8>(U, V, X, Y, amp, zhalf, frames, n_frames, width, height, wpad, hpad,
                       out, out_im, acc, s);
    else
        launch_rows<4>(U, V, X, Y, amp, zhalf, frames, n_frames, width, height, wpad, hpad,
                       out, out_im, acc, s);
    return hipGetLastError();
}

}  // namespace cgh
