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
// the hologram, and the FP32 cosine and sine see the sum of the two reduced
// parts, in [0, 2) revolutions.
//
// Mapping: a workgroup of four waves owns a tile of 64 columns x 32 rows;
// a wave owns 8 rows, a lane one column of them.  The workgroup walks the
// points in index order, 256 at a time: each wave tests 64 points' discs
// against the tile's box (a conservative FP32 test that only decides what to
// skip), the hit masks meet in LDS, and every wave then adds the hit points
// to its 8 x 64 samples in index order.  Every sample's sum is therefore
// formed in point order by one lane: deterministic, with no atomics.
#pragma clang fp contract(off)

#include "common.h"

namespace cgh {
namespace {

constexpr int kTileCols = 64;
constexpr int kWaveRows = 8;
constexpr int kWaves = 4;
constexpr int kTileRows = kWaveRows * kWaves;

// a1 of the recording: constants of point i (see WrmConsts in common.h).
__global__ __launch_bounds__(256) void k_wrm_consts(const float *__restrict__ x,
                                                    const float *__restrict__ y,
                                                    const float *__restrict__ z,
                                                    const float *__restrict__ amp,
                                                    int64_t n_points, double pitch, double lam,
                                                    double zw, double half, WrmConsts wc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_points)
        return;
    const double xj = (double)x[i], yj = (double)y[i];
    const double d = (double)z[i] - zw;
    double r2 = -1.0, beta = 0.0;
    float rho = -1.0f;
    if (d > 0.0) {
        const double rj = lam * d / (2.0 * pitch);   // disc radius, metres
        r2 = rj * rj;
        beta = pitch * pitch / (2.0 * lam * d);      // revolutions per sample^2
        rho = (float)(rj / pitch);                   // disc radius, samples
    }
    const double cx = half + xj / pitch, cy = half + yj / pitch;
    wc.x[i] = xj;
    wc.y[i] = yj;
    wc.r2[i] = r2;
    wc.beta[i] = beta;
    wc.cx[i] = cx;
    wc.cy[i] = cy;
    wc.amp[i] = amp[i];
    wc.box[i] = float4{(float)cx, (float)cy, rho, 0.0f};
}

__global__ __launch_bounds__(256) void k_wrm_record(WrmConsts wc, int64_t n_points, int n,
                                                    double pitch, double half,
                                                    float2 *__restrict__ field)
{
    __shared__ uint64_t hits[kWaves];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col0 = blockIdx.x * kTileCols;
    const int trow0 = blockIdx.y * kTileRows;
    const int row0 = trow0 + wave * kWaveRows;
    const int col = col0 + lane;

    // the tile's sample centres span [col0, col0 + 63] x [trow0, trow0 + 31]
    const float bx0 = (float)col0, bx1 = (float)(col0 + kTileCols - 1);
    const float by0 = (float)trow0, by1 = (float)(trow0 + kTileRows - 1);
    const double xw = ((double)col - half) * pitch;
    double yw[kWaveRows];
#pragma unroll
    for (int r = 0; r < kWaveRows; ++r)
        yw[r] = ((double)(row0 + r) - half) * pitch;
    float acc_re[kWaveRows], acc_im[kWaveRows];
#pragma unroll
    for (int r = 0; r < kWaveRows; ++r) {
        acc_re[r] = 0.0f;
        acc_im[r] = 0.0f;
    }

    for (int64_t base = 0; base < n_points; base += kWaves * 64) {
        const int64_t i = base + wave * 64 + lane;
        bool hit = false;
        if (i < n_points) {
            const float4 b = wc.box[i];
            const float ex = fmaxf(fmaxf(bx0 - b.x, b.x - bx1), 0.0f);
            const float ey = fmaxf(fmaxf(by0 - b.y, b.y - by1), 0.0f);
            const float reach = b.z * 1.0001f + 0.05f;   // margin over FP32 rounding
            hit = b.z >= 0.0f && ex * ex + ey * ey <= reach * reach;
        }
        const uint64_t m = __ballot(hit);
        if (lane == 0)
            hits[wave] = m;
        __syncthreads();
#pragma unroll 1
        for (int w = 0; w < kWaves; ++w) {
            // the same mask in every lane: made scalar, so the loop and the
            // point loads below are scalar too (readfirstlane returns int:
            // each half goes through uint32_t so the low one is not
            // sign-extended into the high bits)
            const uint64_t hw = hits[w];
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)hw);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(hw >> 32));
            uint64_t mm = ((uint64_t)hi << 32) | (uint64_t)lo;
            while (mm) {
                const int bit = __builtin_ctzll(mm);
                mm &= mm - 1;
                const int64_t j = base + w * 64 + bit;
                const double xj = wc.x[j], yj = wc.y[j], r2 = wc.r2[j];
                const double beta = wc.beta[j], cx = wc.cx[j], cy = wc.cy[j];
                const float a = wc.amp[j];
                const double dx = xw - xj;
                const double dx2 = dx * dx;
                const double uc = (double)col - cx;
                const float u = (float)__builtin_amdgcn_fract(beta * (uc * uc));
#pragma unroll
                for (int r = 0; r < kWaveRows; ++r) {
                    const double dy = yw[r] - yj;
                    const double rr = dx2 + dy * dy;
                    if (rr <= r2) {
                        const double vr = (double)(row0 + r) - cy;
                        const float t = u + (float)__builtin_amdgcn_fract(beta * (vr * vr));
                        acc_re[r] = __builtin_fmaf(a, __builtin_amdgcn_cosf(t), acc_re[r]);
                        acc_im[r] = __builtin_fmaf(a, __builtin_amdgcn_sinf(t), acc_im[r]);
                    }
                }
            }
        }
        __syncthreads();   // every wave has read the masks before they are rewritten
    }
    if (col < n) {
#pragma unroll
        for (int r = 0; r < kWaveRows; ++r)
            if (row0 + r < n)
                field[(int64_t)(row0 + r) * n + col] = float2{acc_re[r], acc_im[r]};
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
    if (n_points <= 0)
        return hipSuccess;
    const int64_t blocks = (n_points + 255) / 256;
    hipLaunchKernelGGL(k_wrm_consts, dim3((unsigned)blocks), dim3(256), 0, s, x, y, z, amp,
                       n_points, pitch, lam, zw, 0.5 * (double)(n - 1), wc);
    return hipGetLastError();
}

hipError_t launch_wrm_record(const WrmConsts &wc, int64_t n_points, int n, double pitch,
                             float2 *field, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const dim3 grid((unsigned)((n + kTileCols - 1) / kTileCols),
                    (unsigned)((n + kTileRows - 1) / kTileRows));
    hipLaunchKernelGGL(k_wrm_record, grid, dim3(64 * kWaves), 0, s, wc, n_points, n, pitch,
                       0.5 * (double)(n - 1), field);
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
