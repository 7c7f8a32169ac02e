// Phase-only hologram (kinoform) of Eq. (3): the argument of the complex
// object wave, wrapped to [0, 2 pi) and quantised to 256 levels,
//     theta = atan2(Im O, Re O) (+ 2 pi if negative),  code = floor(theta * 255 / (2 pi)),
// in FP32, the precision the paper's program takes the argument in (Section 4.1).
// Memory-bound: 8 bytes read and 1 byte written per pixel; each thread takes
// four consecutive pixels (two 16-byte loads, one 4-byte store).
#include "common.h"

namespace cgh {
namespace {

__device__ __forceinline__ uint32_t phase_code(float re, float im)
{
    constexpr float kTwoPi = 6.28318530717958647692f;
    constexpr float kCodesPerRad = 255.0f / 6.28318530717958647692f;
    float theta = atan2f(im, re);
    if (theta < 0.0f)
        theta += kTwoPi;
    const float q = floorf(theta * kCodesPerRad);
    return (uint32_t)fminf(fmaxf(q, 0.0f), 255.0f);
}

// re, im: n floats each; out: n bytes.  Vector path when all three are
// 16-byte (re, im) and 4-byte (out) aligned; the last n mod 4 pixels, or all
// of them otherwise, one per thread.
__global__ __launch_bounds__(256) void k_kinoform(const float *__restrict__ re,
                                                  const float *__restrict__ im, int64_t n,
                                                  uint8_t *__restrict__ out, int vec4)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tail = 0;
    if (vec4) {
        const int64_t q = n / 4;
        for (int64_t e = t0; e < q; e += stride) {
            const float4 a = reinterpret_cast<const float4 *>(re)[e];
            const float4 b = reinterpret_cast<const float4 *>(im)[e];
            const uint32_t w = phase_code(a.x, b.x) | (phase_code(a.y, b.y) << 8) |
                               (phase_code(a.z, b.z) << 16) | (phase_code(a.w, b.w) << 24);
            reinterpret_cast<uint32_t *>(out)[e] = w;
        }
        tail = q * 4;
    }
    for (int64_t e = tail + t0; e < n; e += stride)
        out[e] = (uint8_t)phase_code(re[e], im[e]);
}

}  // namespace

hipError_t launch_kinoform(const float *re, const float *im, int64_t n, uint8_t *out,
                           hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n / 4 + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    if (blocks < 1)
        blocks = 1;
    const int vec4 = ((uintptr_t)re % 16 == 0) && ((uintptr_t)im % 16 == 0) &&
                     ((uintptr_t)out % 4 == 0);
    hipLaunchKernelGGL(k_kinoform, dim3((unsigned)blocks), dim3(256), 0, s, re, im, n, out, vec4);
    return hipGetLastError();
}

}  // namespace cgh
