// Fresnel diffraction of a sampled field (Section 2.3, Eq. (10)) on gfx950.
//
// The n x n complex field u (pitch p) propagates by z to
//     O[m][c] = C p^2 sum_k sum_l u[k][l] h(m - k, c - l),
//     h(a, b) = exp(i pi p^2 (a^2 + b^2) / (lambda z)),  C = exp(i 2 pi z / lambda) / (i lambda z),
// evaluated, as the second line of Eq. (10) writes it, as F^-1[F[u] F[h]] on
// the grid zero-padded to L x L, L = 2n (no wrap-around), cropped to n x n.
//
// Design for this chip:
//   - h is separable, h(a, b) = h1(a) h1(b), so F[h] is the outer product of
//     one length-L transform of the chirp h1: computed once per plan, and the
//     2-D transform of h never exists.  The chirp phase (revolutions,
//     p^2 a^2 / (2 lambda z), up to ~1e5) is reduced in FP64 before the FP32
//     exponential.
//   - 2-D transforms are row transforms with transposes between them; every
//     row transform runs in LDS (a whole row, up to L = 16384 complex = 128 KB,
//     in one workgroup) as a Stockham autosort FFT of radix-16 passes (plus one
//     radix-2/4/8 pass), the small DFTs in registers.  Twiddles come from an
//     FP64-computed table, kept in LDS as two factors, w^t = w^(64 t_hi)
//     w^t_lo (64 + L/64 entries), so a pass reads none from global memory.
//     Inverse transforms are conj(F[conj(x)]).
//   - Zero padding and cropping are pruned: rows that are all zero are never
//     transformed, zeros are never loaded, and outputs outside the crop are
//     never stored.  The forward column transform, the spectrum product and
//     the inverse column transform of a column are one kernel, so the L x L
//     spectrum never reaches HBM.  Five kernels, HBM traffic 18 n^2 x 8 bytes.
#include "common.h"

namespace cgh {
namespace {

// threads per row transform: 1024 for long rows (one or two rows fill a CU's
// LDS, so the waves of one row must hide the LDS latency), 256 otherwise
constexpr int kFftThreadsLong = 1024;
constexpr int kFftThreadsShort = 256;
constexpr int kLongLog2 = 13;
constexpr int kMaxLog2 = 14;               // L <= 16384: a row is 128 KB of LDS
constexpr int kMaxL = 1 << kMaxLog2;

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return float2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return float2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return float2{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ float2 conjf2(float2 a) { return float2{a.x, -a.y}; }

// exp(-2 pi i q / 16), q = 0 .. 15: cos and -sin of multiples of pi / 8
constexpr float kC8 = 0.923879532511286756f;   // cos(pi / 8)
constexpr float kS8 = 0.382683432365089772f;   // sin(pi / 8)
constexpr float kR2 = 0.707106781186547524f;   // cos(pi / 4)

__device__ __forceinline__ float2 root16(int q)
{
    constexpr float c[16] = {1.0f, kC8, kR2, kS8, 0.0f, -kS8, -kR2, -kC8,
                             -1.0f, -kC8, -kR2, -kS8, 0.0f, kS8, kR2, kC8};
    return float2{c[q & 15], -c[(q + 12) & 15]};   // sin(x) = cos(x - pi/2)
}

// x * exp(-2 pi i Q / 16) with the exact forms of the multiples of pi / 2
// (a swap and a sign) and pi / 4 (two products) spelled out.
template <int Q>
__device__ __forceinline__ float2 mul_root16(float2 x)
{
    constexpr int q = Q & 15;
    if constexpr (q == 0)
        return x;
    else if constexpr (q == 4)
        return float2{x.y, -x.x};                           // * (-i)
    else if constexpr (q == 8)
        return float2{-x.x, -x.y};                          // * (-1)
    else if constexpr (q == 12)
        return float2{-x.y, x.x};                           // * i
    else if constexpr (q == 2)
        return float2{kR2 * (x.x + x.y), kR2 * (x.y - x.x)};   // * (1 - i) / sqrt 2
    else if constexpr (q == 6)
        return float2{kR2 * (x.y - x.x), -kR2 * (x.x + x.y)};  // * (-1 - i) / sqrt 2
    else if constexpr (q == 10)
        return float2{-kR2 * (x.x + x.y), kR2 * (x.x - x.y)};  // * (-1 + i) / sqrt 2
    else if constexpr (q == 14)
        return float2{kR2 * (x.x - x.y), kR2 * (x.x + x.y)};   // * (1 + i) / sqrt 2
    else
        return cmul(x, root16(q));
}

template <int R, int Q>
__device__ __forceinline__ void dft_combine(float2 *v, const float2 *e, const float2 *o)
{
    if constexpr (Q < R / 2) {
        const float2 t = mul_root16<Q *(16 / R)>(o[Q]);
        v[Q] = cadd(e[Q], t);
        v[Q + R / 2] = csub(e[Q], t);
        dft_combine<R, Q + 1>(v, e, o);
    }
}

// In-register forward DFT of size R (R = 1, 2, 4, 8, 16): v[q] <- sum_r v[r]
// exp(-2 pi i r q / R), by radix-2 decimation in time.
template <int R>
__device__ __forceinline__ void dft(float2 *v)
{
    if constexpr (R > 1) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int r = 0; r < R / 2; ++r) {
            e[r] = v[2 * r];
            o[r] = v[2 * r + 1];
        }
        dft<R / 2>(e);
        dft<R / 2>(o);
        dft_combine<R, 0>(v, e, o);
    }
}

// One Stockham pass of radix R over s[0 .. L) (L = 2^m) with sub-transform
// size ns (2^lns): butterfly j (k = j mod ns) takes s[j + r L/R], multiplies
// input r by w_L^(r k L/(ns R)) (w_L = exp(-2 pi i / L), table tw), applies
// the size-R DFT and writes output q to s[(j - k) R + k + q ns].  In place:
// every thread reads all its inputs before the barrier, writes after it.
// Twiddle w_L^t from the two LDS factor tables (t < L).
__device__ __forceinline__ float2 twiddle(const float2 *tw_hi, const float2 *tw_lo, int t)
{
    return cmul(tw_hi[t >> 6], tw_lo[t & 63]);
}

// The twiddles w^(r e), r = 1 .. R-1, of one butterfly: table lookups for
// r = 1, 2, 4, 8 and products of those (at most three) for the rest, so each
// carries at most a few roundings; e (R - 1) < L.
template <int R>
__device__ __forceinline__ void butterfly_twiddles(const float2 *tw_hi, const float2 *tw_lo,
                                                   int e, int lmask, float2 *w)
{
    float2 p[4];
#pragma unroll
    for (int b = 0; (1 << b) < R; ++b)
        p[b] = twiddle(tw_hi, tw_lo, (e << b) & lmask);
#pragma unroll
    for (int r = 1; r < R; ++r) {
        float2 acc{1.0f, 0.0f};
        bool first = true;
#pragma unroll
        for (int b = 0; (1 << b) < R; ++b)
            if (r & (1 << b)) {
                acc = first ? p[b] : cmul(acc, p[b]);
                first = false;
            }
        w[r] = acc;
    }
}

template <int R, int LR, int T>
__device__ __forceinline__ void stockham_pass(float2 *s, int m, int lns, const float2 *tw_hi,
                                              const float2 *tw_lo)
{
    // the long-row launch covers L >= 2^kLongLog2, the short one L below it
    constexpr int LMAX = T == kFftThreadsLong ? kMaxL : (1 << (kLongLog2 - 1));
    constexpr int BMAX = (LMAX / R + T - 1) / T;
    const int nb = (1 << m) / R;                 // butterflies
    const int ns = 1 << lns;
    const int tshift = m - lns - LR;             // log2(L / (ns R))
    float2 v[BMAX][R];
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int j = threadIdx.x + b * T;
        if (j < nb) {
            const int k = j & (ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[b][r] = s[j + r * nb];
            if (k > 0) {
                float2 w[R];
                butterfly_twiddles<R>(tw_hi, tw_lo, k << tshift, (1 << m) - 1, w);
#pragma unroll
                for (int r = 1; r < R; ++r)
                    v[b][r] = cmul(v[b][r], w[r]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int j = threadIdx.x + b * T;
        if (j < nb) {
            const int k = j & (ns - 1);
            dft<R>(v[b]);
            const int base = ((j - k) << LR) + k;
#pragma unroll
            for (int q = 0; q < R; ++q)
                s[base + q * ns] = v[b][q];
        }
    }
    __syncthreads();
}

// Forward FFT of s[0 .. 2^m) in LDS, natural order in and out.  The caller
// has synchronised after filling s.
template <int T>
__device__ __forceinline__ void fft_lds(float2 *s, int m, const float2 *tw_hi,
                                        const float2 *tw_lo)
{
    int lns = 0;
    switch (m & 3) {
    case 1:
        stockham_pass<2, 1, T>(s, m, 0, tw_hi, tw_lo);
        lns = 1;
        break;
    case 2:
        stockham_pass<4, 2, T>(s, m, 0, tw_hi, tw_lo);
        lns = 2;
        break;
    case 3:
        stockham_pass<8, 3, T>(s, m, 0, tw_hi, tw_lo);
        lns = 3;
        break;
    default:
        break;
    }
    for (; lns < m; lns += 4)
        stockham_pass<16, 4, T>(s, m, lns, tw_hi, tw_lo);
}

// LDS of a row transform: the row (L values), then the twiddle factors w^t
// (t < 64) and w^(64 t) (t < L / 64).
constexpr size_t row_lds_bytes(int m)
{
    return sizeof(float2) * ((size_t(1) << m) + 64 + ((size_t(1) << m) / 64 + 1));
}

enum class RowOp { Forward, Fresnel, Inverse };

// One row per workgroup.  Loads in[row][0 .. in_len) (zeros beyond), then
//   Forward: F;   Inverse: conj F conj;
//   Fresnel: F, times hc[i] hc[row] scale (the spectrum of the separable
//            impulse response at frequency (row, i), and the constant), then
//            conj F conj;
// and stores the first out_len outputs to out[row].  in and out may be the
// same rows (the row is in LDS before anything is stored).
template <RowOp OP, int T>
__global__ __launch_bounds__(T) void k_fft_rows(const float2 *in, int64_t in_ld,
                                                          int in_len, float2 *out, int64_t out_ld,
                                                          int out_len, int m,
                                                          const float2 *__restrict__ tw,
                                                          const float2 *__restrict__ hc,
                                                          float2 scale)
{
    extern __shared__ float2 s[];
    const int L = 1 << m;
    float2 *tw_lo = s + L;
    float2 *tw_hi = tw_lo + 64;
    for (int t = threadIdx.x; t < 64; t += T)
        tw_lo[t] = tw[t & (L - 1)];
    for (int t = threadIdx.x; t * 64 < L; t += T)
        tw_hi[t] = tw[t * 64];
    const int64_t row = blockIdx.x;
    const float2 *src = in + row * in_ld;
    for (int i = threadIdx.x; i < L; i += T) {
        const float2 x = i < in_len ? src[i] : float2{0.0f, 0.0f};
        s[i] = OP == RowOp::Inverse ? conjf2(x) : x;
    }
    __syncthreads();
    fft_lds<T>(s, m, tw_hi, tw_lo);
    if (OP == RowOp::Fresnel) {
        const float2 hr = cmul(hc[row], scale);
        for (int i = threadIdx.x; i < L; i += T)
            s[i] = conjf2(cmul(s[i], cmul(hc[i], hr)));
        __syncthreads();
        fft_lds<T>(s, m, tw_hi, tw_lo);
    }
    float2 *dst = out + row * out_ld;
    for (int i = threadIdx.x; i < out_len; i += T)
        dst[i] = OP == RowOp::Forward ? s[i] : conjf2(s[i]);
}

// out[c][r] = in[r][c] for r < rows, c < cols; 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose(const float2 *__restrict__ in, int64_t in_ld,
                                                   float2 *__restrict__ out, int64_t out_ld,
                                                   int rows, int cols)
{
    __shared__ float2 tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int r = r0 + ty + k, c = c0 + tx;
        if (r < rows && c < cols)
            tile[ty + k][tx] = in[(int64_t)r * in_ld + c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int c = c0 + ty + k, r = r0 + tx;
        if (r < rows && c < cols)
            out[(int64_t)c * out_ld + r] = tile[tx][ty + k];
    }
}

// tw[t] = exp(-2 pi i t / L), computed in FP64.
__global__ void k_twiddles(int m, float2 *tw)
{
    const int L = 1 << m;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < L; t += gridDim.x * blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)t / (double)L, &sn, &cs);
        tw[t] = float2{(float)cs, (float)-sn};
    }
}

// The chirp h1 at the circular offsets of the padded grid: sample d is the
// offset d (d < n) or d - L, h1 = exp(2 pi i frac(q d^2)), q = p^2 / (2 lambda z)
// revolutions per pixel^2 (FP64 before the reduction).
__global__ void k_chirp(int m, int n, double q, float2 *h)
{
    const int L = 1 << m;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < L; t += gridDim.x * blockDim.x) {
        const double d = t < n ? (double)t : (double)(t - L);
        const double rev = q * d * d;
        const double fr = rev - floor(rev);
        double sn, cs;
        sincospi(2.0 * fr, &sn, &cs);
        h[t] = float2{(float)cs, (float)sn};
    }
}

template <RowOp OP>
hipError_t rows(const float2 *in, int64_t in_ld, int in_len, float2 *out, int64_t out_ld,
                int out_len, int n_rows, int m, const float2 *tw, const float2 *hc, float2 scale,
                hipStream_t s)
{
    const size_t lds = row_lds_bytes(m);
    if (m >= kLongLog2)
        hipLaunchKernelGGL((k_fft_rows<OP, kFftThreadsLong>), dim3((unsigned)n_rows),
                           dim3(kFftThreadsLong), lds, s, in, in_ld, in_len, out, out_ld, out_len,
                           m, tw, hc, scale);
    else
        hipLaunchKernelGGL((k_fft_rows<OP, kFftThreadsShort>), dim3((unsigned)n_rows),
                           dim3(kFftThreadsShort), lds, s, in, in_ld, in_len, out, out_ld,
                           out_len, m, tw, hc, scale);
    return hipGetLastError();
}

hipError_t transpose(const float2 *in, int64_t in_ld, float2 *out, int64_t out_ld, int r, int c,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)((c + 31) / 32), (unsigned)((r + 31) / 32)),
                       dim3(256), 0, s, in, in_ld, out, out_ld, r, c);
    return hipGetLastError();
}

}  // namespace

hipError_t fresnel_prepare_kernels()
{
    const int lds = (int)row_lds_bytes(kMaxLog2);
    const void *kernels[] = {
        (const void *)k_fft_rows<RowOp::Forward, kFftThreadsLong>,
        (const void *)k_fft_rows<RowOp::Fresnel, kFftThreadsLong>,
        (const void *)k_fft_rows<RowOp::Inverse, kFftThreadsLong>,
        (const void *)k_fft_rows<RowOp::Forward, kFftThreadsShort>,
        (const void *)k_fft_rows<RowOp::Fresnel, kFftThreadsShort>,
        (const void *)k_fft_rows<RowOp::Inverse, kFftThreadsShort>};
    for (const void *k : kernels) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t fresnel_tables(int n, int m, double q, float2 *tw, float2 *hc, hipStream_t s)
{
    if (n < 1 || m < 1 || m > kMaxLog2 || (2 * n) != (1 << m))
        return hipErrorInvalidValue;
    const int L = 1 << m;
    const unsigned blocks = (unsigned)((L + 255) / 256);
    hipLaunchKernelGGL(k_twiddles, dim3(blocks), dim3(256), 0, s, m, tw);
    hipLaunchKernelGGL(k_chirp, dim3(blocks), dim3(256), 0, s, m, n, q, hc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // hc <- F[h1], in place (one row)
    return rows<RowOp::Forward>(hc, L, L, hc, L, L, 1, m, tw, nullptr, float2{0.0f, 0.0f}, s);
}

hipError_t fresnel_run(int n, int m, const float2 *tw, const float2 *hc, float2 scale,
                       const float2 *u, float2 *out, float2 *x, float2 *y, hipStream_t s)
{
    if (n < 1 || m < 1 || m > kMaxLog2 || (2 * n) != (1 << m))
        return hipErrorInvalidValue;
    const int L = 1 << m;
    const float2 none{0.0f, 0.0f};
    hipError_t e;
    // rows of u, zero-padded: X[k][0 .. L) = F_row(u[k]), k < n (rows >= n are zero)
    e = rows<RowOp::Forward>(u, n, n, x, L, L, n, m, tw, nullptr, none, s);
    if (e != hipSuccess)
        return e;
    e = transpose(x, L, y, n, n, L, s);                       // Y = X^T: L x n
    if (e != hipSuccess)
        return e;
    // columns: forward transform (n nonzeros), spectrum product, inverse, crop to n
    e = rows<RowOp::Fresnel>(y, n, n, y, n, n, L, m, tw, hc, scale, s);
    if (e != hipSuccess)
        return e;
    e = transpose(y, n, x, L, L, n, s);                       // X = Y^T: n x L
    if (e != hipSuccess)
        return e;
    // rows: inverse transform, crop to n
    e = rows<RowOp::Inverse>(x, L, L, out, n, n, n, m, tw, nullptr, none, s);
    return e;
}

}  // namespace cgh
