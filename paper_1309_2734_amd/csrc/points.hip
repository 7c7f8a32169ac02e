// Per-point constants and FP64-reduced line-phase tables.
//
// Eq. (2) (Section 2.1) in pixel units: the phase of point j at pixel
// (ix, iy) is beta_j ((ix - cx_j)^2 + (iy - cy_j)^2) revolutions.  At the
// hologram sizes of interest it reaches several hundred revolutions, where a
// float32 phase has lost ~1e-4 rad; so it is reduced modulo one revolution in
// FP64, one line at a time, and only the reduced value is rounded to float32.
#include "common.h"

namespace cgh {
namespace {

// a1: one thread per constant slot of one segment (blockIdx.y = segment).
__global__ __launch_bounds__(256) void k_point_consts(const float *__restrict__ x,
                                                      const float *__restrict__ y,
                                                      const float *__restrict__ z,
                                                      const float *__restrict__ amp,
                                                      SegList segs, double half_w,
                                                      double half_h, double pitch,
                                                      PointConsts pc)
{
    const Segment sg = segs.dev ? segs.dev[blockIdx.y] : segs.one;
    const int64_t padded = (sg.count + kSlotAlign - 1) / kSlotAlign * kSlotAlign;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= padded)
        return;
    const int64_t d = sg.dst + i;
    if (i < sg.count) {
        const int64_t s = sg.src + i;
        // beta = p^2 / (2 lambda z): revolutions per pixel^2
        pc.beta[d] = pitch * pitch / (2.0 * sg.wavelength * (double)z[s]);
        pc.cx[d] = half_w + (double)x[s] / pitch;
        pc.cy[d] = half_h + (double)y[s] / pitch;
        pc.zlam[d] = (double)z[s] / sg.wavelength;
        pc.amp[d] = amp[s];
        pc.zhalf[d] = (float)(0.5 * (double)z[s] / sg.wavelength);
    } else {
        // padding slot: zero amplitude, zero phase
        pc.beta[d] = 0.0;
        pc.cx[d] = 0.0;
        pc.cy[d] = 0.0;
        pc.zlam[d] = 0.0;
        pc.amp[d] = 0.0f;
        pc.zhalf[d] = 0.0f;
    }
}

// frac(beta * d^2) in FP64, rounded once to float32.  v_fract_f64 returns a
// value in [0, 1); the float32 rounding can give 1.0f, which is the same
// angle as 0.
__device__ __forceinline__ float reduce_line(double beta, double d)
{
    return (float)__builtin_amdgcn_fract(beta * (d * d));
}

// a2: U blocked as [group][column][kGroup], V as [group][row][kGroup].  A
// thread writes four consecutive entries of one table line of a group (one
// 16-byte store; consecutive threads write consecutive 16 bytes);
// blockIdx.y strides over the groups.
__global__ __launch_bounds__(256) void k_phase_tables(PointConsts pc, int64_t n_groups, int width,
                                                      int height, float *__restrict__ U,
                                                      float *__restrict__ V)
{
    constexpr int kQuads = kGroup / 4;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int line_all = idx / kQuads;
    const int q0 = 4 * (idx % kQuads);
    if (line_all >= width + height)
        return;
    const bool is_u = line_all < width;
    const int line = is_u ? line_all : line_all - width;
    const double *ctr = is_u ? pc.cx : pc.cy;
    float *tab = is_u ? U : V;
    const int64_t lines = is_u ? width : height;
    for (int64_t g = blockIdx.y; g < n_groups; g += gridDim.y) {
        const int64_t j = g * kGroup + q0;
        float4 t;
        t.x = reduce_line(pc.beta[j], (double)line - ctr[j]);
        t.y = reduce_line(pc.beta[j + 1], (double)line - ctr[j + 1]);
        t.z = reduce_line(pc.beta[j + 2], (double)line - ctr[j + 2]);
        t.w = reduce_line(pc.beta[j + 3], (double)line - ctr[j + 3]);
        *reinterpret_cast<float4 *>(tab + (g * lines + line) * kGroup + q0) = t;
    }
}

}  // namespace

hipError_t launch_point_consts(const float *x, const float *y, const float *z, const float *amp,
                               const SegList &segs, int n_segs, int64_t max_count,
                               int width, int height, double pitch, PointConsts pc,
                               hipStream_t s)
{
    if (n_segs <= 0 || max_count <= 0)
        return hipSuccess;
    if (!segs.dev && n_segs != 1)
        return hipErrorInvalidValue;
    const int64_t padded = (max_count + kSlotAlign - 1) / kSlotAlign * kSlotAlign;
    dim3 grid((unsigned)((padded + 255) / 256), (unsigned)n_segs);
    hipLaunchKernelGGL(k_point_consts, grid, dim3(256), 0, s, x, y, z, amp, segs,
                       0.5 * (double)(width - 1), 0.5 * (double)(height - 1), pitch, pc);
    return hipGetLastError();
}

hipError_t launch_phase_tables(PointConsts pc, int64_t n_slots, int width, int height,
                               float *U, float *V, hipStream_t s)
{
    if (n_slots <= 0)
        return hipSuccess;
    const int64_t groups = n_slots / kGroup;
    const unsigned bx = (unsigned)(((int64_t)(width + height) * (kGroup / 4) + 255) / 256);
    const unsigned by = (unsigned)(groups < 65535 ? groups : 65535);
    hipLaunchKernelGGL(k_phase_tables, dim3(bx, by), dim3(256), 0, s, pc, groups, width, height,
                       U, V);
    return hipGetLastError();
}

}  // namespace cgh
