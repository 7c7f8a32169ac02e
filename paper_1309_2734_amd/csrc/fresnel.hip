// Fresnel diffraction of a sampled field (Section 2.3, Eq. (10)) on gfx950.
//
// The n x n complex field u (pitch p) propagates by z to
//     O[m][c] = C p^2 sum_k sum_l u[k][l] h(m - k, c - l),
//     h(a, b) = exp(i pi p^2 (a^2 + b^2) / (lambda z)),  C = exp(i 2 pi z / lambda) / (i lambda z),
// evaluated, as the second line of Eq. (10) writes it, as F^-1[F[u] F[h]] on
// the grid zero-padded to L x L, L = 2n (no wrap-around), cropped to n x n.
//
// Design for this chip:
//   - h is separable, h(a, b) = h1(a) h1(b), so the 2-D linear convolution
//     is a 1-D one along every row followed by one along every column, each
//     zero-padded to L and cropped to n: F[h1] (one length-L transform of the
//     chirp, computed once per plan) is the only spectrum there is.  The
//     chirp phase (revolutions, p^2 a^2 / (2 lambda z), up to ~1e5) is
//     reduced in FP64 before the FP32 exponential.
//   - A line (up to L = 16384 complex) is one workgroup's: each thread
//     holds 16 of its values (32 for lines of 8192 and more) in registers
//     through a Stockham autosort FFT of radix-16 (radix-32) passes plus one
//     smaller pass, and LDS only carries the exchange between two passes
//     (the first pass runs on the values as loaded, the last leaves the
//     results in registers).  Twiddles come from an FP64-computed table of
//     log2 V values per butterfly and pass (w^e, w^2e, w^4e, ..; the other
//     twiddles are products of these), expanded into LDS for the early
//     passes and held in registers for the last one.  Workgroups are
//     persistent, and the loads of a workgroup's next line are in flight
//     while it transforms the current one (its barriers order LDS only).
//     Inverse transforms are conj(F[conj(x)]).
//   - Up to n = 1024 there are no transposes: both passes read their lines
//     as columns (lane j of a wave loads element j + r L/V of its column,
//     one 8-byte load per row) and store them as contiguous rows.  The
//     first pass convolves the columns of u and stores Z^T; the second
//     convolves the columns of Z^T, which are the rows of Z, and stores the
//     rows of O.  A turn of the persistent grid gives each XCD adjacent
//     columns, so the row segments its workgroups read are whole cache
//     lines of its own L2.  Two kernels, HBM traffic 4 n^2 x 8 bytes.
//   - From n = 2048 on, column loads cost more than a transpose (strided
//     rows of 16-64 KB: n = 8192 takes 0.8-1.0 ms per column pass against
//     0.5 ms per row pass and 0.2 ms per transpose), so the rows of u are
//     convolved, transposed, convolved as rows again and transposed back:
//     four kernels, 8 n^2 x 8 bytes.
//   - Zero padding and cropping are pruned: zeros are never loaded, and
//     outputs outside the crop are never stored.  A line's forward
//     transform, spectrum product and inverse transform are one kernel, so
//     no padded plane or spectrum ever reaches HBM.
#include <atomic>

#include "common.h"

namespace cgh {
namespace {

constexpr int kMinLog2 = 5;                // L >= 32 (n >= 16)
constexpr int kMaxLog2 = 14;               // L <= 16384: a row is 136 KB of LDS, 512 threads
constexpr int kColsMaxLog2 = 11;           // column-load pipeline up to L = 2048 (n = 1024)

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return float2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return float2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return float2{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ float2 conjf2(float2 a) { return float2{a.x, -a.y}; }

// cos(2 pi q / 32), q = 0 .. 8
constexpr float kCos32[9] = {1.0f,
                             0.980785280403230449f,    // cos(pi / 16)
                             0.923879532511286756f,    // cos(pi / 8)
                             0.831469612302545237f,    // cos(3 pi / 16)
                             0.707106781186547524f,    // cos(pi / 4)
                             0.555570233019602225f,    // cos(5 pi / 16)
                             0.382683432365089772f,    // cos(3 pi / 8)
                             0.195090322016128268f,    // cos(7 pi / 16)
                             0.0f};
constexpr float kR2 = 0.707106781186547524f;           // cos(pi / 4)

constexpr float cos32(int q)
{
    q &= 31;
    return q <= 8 ? kCos32[q] : q <= 16 ? -kCos32[16 - q] : q <= 24 ? -kCos32[q - 16]
                                                                    : kCos32[32 - q];
}

// x * exp(-2 pi i Q / 32) with the exact forms of the multiples of pi / 2
// (a swap and a sign) and pi / 4 (two products) spelled out.
template <int Q>
__device__ __forceinline__ float2 mul_root32(float2 x)
{
    constexpr int q = Q & 31;
    if constexpr (q == 0)
        return x;
    else if constexpr (q == 8)
        return float2{x.y, -x.x};                           // * (-i)
    else if constexpr (q == 16)
        return float2{-x.x, -x.y};                          // * (-1)
    else if constexpr (q == 24)
        return float2{-x.y, x.x};                           // * i
    else if constexpr (q == 4)
        return float2{kR2 * (x.x + x.y), kR2 * (x.y - x.x)};   // * (1 - i) / sqrt 2
    else if constexpr (q == 12)
        return float2{kR2 * (x.y - x.x), -kR2 * (x.x + x.y)};  // * (-1 - i) / sqrt 2
    else if constexpr (q == 20)
        return float2{-kR2 * (x.x + x.y), kR2 * (x.x - x.y)};  // * (-1 + i) / sqrt 2
    else if constexpr (q == 28)
        return float2{kR2 * (x.x - x.y), kR2 * (x.x + x.y)};   // * (1 + i) / sqrt 2
    else {
        constexpr float c = cos32(q), sn = cos32(q + 24);      // sin(x) = cos(x - pi/2)
        return cmul(x, float2{c, -sn});
    }
}

template <int R, int Q>
__device__ __forceinline__ void dft_combine(float2 *v, const float2 *e, const float2 *o)
{
    if constexpr (Q < R / 2) {
        const float2 t = mul_root32<Q *(32 / R)>(o[Q]);
        v[Q] = cadd(e[Q], t);
        v[Q + R / 2] = csub(e[Q], t);
        dft_combine<R, Q + 1>(v, e, o);
    }
}

// In-register forward DFT of size R (R = 1, 2, 4, .., 32): v[q] <- sum_r v[r]
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

// The twiddles w^(r e), r = 1 .. 2^LV - 1, of one radix-2^LV butterfly from
// the LV table values p[b] = w^(2^b e): products of at most LV table values,
// so each carries a few roundings at most.
template <int LV>
__device__ __forceinline__ void butterfly_twiddles(const float2 *p, float2 *w)
{
#pragma unroll
    for (int r = 1; r < (1 << LV); ++r) {
        float2 acc{1.0f, 0.0f};
        bool first = true;
#pragma unroll
        for (int b = 0; b < LV; ++b)
            if (r & (1 << b)) {
                acc = first ? p[b] : cmul(acc, p[b]);
                first = false;
            }
        w[r] = acc;
    }
}

// log2 of the values a thread holds for a row of length 2^m: 32 for the
// longest rows (one exchange fewer per transform), else 16
constexpr int values_log2(int m) { return m >= 13 ? 5 : 4; }

// Shape of a row transform of length L = 2^M.  Every thread holds V values
// of its row in registers (V = 16, or 32 for the longest rows), so a row
// takes TR = L / V threads and a workgroup takes ROWS rows (at least one
// wave).  The transform is a Stockham autosort FFT: one radix-R0 pass
// (R0 = 2^(M mod log2 V), or V), then radix-V passes.  Pass with
// sub-transform size ns and radix R: butterfly b (k = b mod ns) takes
// X[b + r L/R], multiplies input r by w^(r k L/(ns R)) (w = exp(-2 pi i / L)),
// applies the size-R DFT and puts output q at (b - k) R + k + q ns.  Thread
// j's values are X[j + r TR] (r < V): exactly the inputs of its butterflies
// in every pass, and, after the last pass (ns = TR), the outputs X[j + q TR]
// in natural order.  So the first pass runs on the values as loaded, the
// last one leaves results in registers, and LDS only carries the exchange
// between two passes.
template <int M>
struct Fft {
    static_assert(M >= kMinLog2 && M <= kMaxLog2, "row length");
    static constexpr int L = 1 << M;
    static constexpr int LV = values_log2(M);
    static constexpr int V = 1 << LV;                        // values per thread
    static constexpr int TR = L / V;                         // threads per row
    static constexpr int ROWS = TR >= 64 ? 1 : 64 / TR;      // rows per workgroup
    static constexpr int T = TR * ROWS;                      // threads per workgroup
    static constexpr int LR0 = M % LV == 0 ? LV : M % LV;    // log2 of the first radix
    static constexpr int R0 = 1 << LR0;
    static constexpr int NB0 = V / R0;                       // first-pass butterflies per thread
    static constexpr int PASSES = 1 + (M - LR0) / LV;
    static constexpr int ROW_SLOTS = L + L / 16;             // padded row in LDS
    static constexpr int NP = PASSES - 1;                    // radix-V passes
    // sub-transform size of radix-V pass p >= 1, and the first entry of its
    // twiddle sets in the pass table (one set per k < ns)
    static constexpr int ns(int p) { return 1 << (LR0 + LV * (p - 1)); }
    static constexpr int tw_first(int p) { return p <= 1 ? 0 : tw_first(p - 1) + ns(p - 1); }
    // LDS: the rows, then the V - 1 twiddles of every set of passes
    // 1 .. NP-1 (the last pass's set of a thread, k = j, stays in its
    // registers as the LV table values)
    static constexpr int LDS_SETS = tw_first(NP);
    static constexpr size_t lds_bytes = sizeof(float2) * (ROWS * ROW_SLOTS + (V - 1) * LDS_SETS);
    // LDS addressing with constant offsets needs TR to be a multiple of 16
    static constexpr bool FAST_SLOTS = TR % 16 == 0;
    // waves per SIMD the register budget is sized for
    static constexpr int WAVES_PER_EU = V == 32 ? 2 : 4;
};

// Entries of the pass twiddle table of a length-2^m transform: one per
// (radix-V pass p >= 1, k < ns(p)), each the LV = log2 V values w^e, w^(2e),
// .., w^(2^(LV-1) e), e = k L / (V ns(p)).
int pass_table_entries(int m)
{
    const int lv = values_log2(m);
    const int lr0 = m % lv == 0 ? lv : m % lv;
    int total = 0;
    for (int lns = lr0; lns + lv <= m; lns += lv)
        total += 1 << lns;
    return total;
}

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (a full barrier would wait for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS slot of row position i: one spare slot after every 16 values spreads
// the strided stores of the early passes over the banks.
__device__ __forceinline__ int slot(int i) { return i + (i >> 4); }

// Row position of thread j's value idx once pass p (p = 0: the first pass)
// has produced it.
template <int M>
__device__ __forceinline__ int out_pos(int p, int j, int idx)
{
    using F = Fft<M>;
    if (p == 0)   // butterfly j + b TR, output q, held in x[b + q NB0]
        return (j + (idx % F::NB0) * F::TR) * F::R0 + idx / F::NB0;
    const int ns = F::ns(p);
    const int k = j & (ns - 1);
    return (j - k) * F::V + k + idx * ns;
}

// Forward transform of one row; x[r] = X[j + r TR] in, x[q] = F[X][j + q TR]
// out.  s is the row's LDS, sets the V - 1 twiddles of each set of passes
// 1 .. NP-1 (in LDS), lt the LV table values of this thread's set of the last
// pass.  Every thread of the workgroup calls it (it holds barriers).
template <int M>
__device__ __forceinline__ void fft_row(float2 (&x)[Fft<M>::V], float2 *s, int j,
                                        const float2 *sets, const float2 (&lt)[Fft<M>::LV])
{
    using F = Fft<M>;
    constexpr int V = F::V;
    // Opaque copy of j: the addresses of two transforms in one kernel are
    // then computed twice instead of being held through both.
    asm volatile("" : "+v"(j));
    constexpr int NP = F::NP;
#pragma unroll
    for (int b = 0; b < F::NB0; ++b) {
        float2 v[F::R0];
#pragma unroll
        for (int a = 0; a < F::R0; ++a)
            v[a] = x[b + a * F::NB0];
        dft<F::R0>(v);
#pragma unroll
        for (int q = 0; q < F::R0; ++q)
            x[b + q * F::NB0] = v[q];
    }
#pragma unroll
    for (int p = 1; p <= NP; ++p) {
        lds_barrier();   // the previous exchange's reads are done
        if constexpr (F::FAST_SLOTS) {
            // slot(out_pos(p - 1, j, idx)) = base + a constant per idx
            if (p == 1) {
                float2 *w = s + F::R0 * j + ((F::R0 * j) >> 4);
#pragma unroll
                for (int idx = 0; idx < V; ++idx) {
                    const int q = idx / F::NB0, b = idx % F::NB0;
                    w[q + (F::R0 >= 16 ? q >> 4 : 0) + b * (F::R0 * F::TR / 16 * 17)] = x[idx];
                }
            } else {
                const int ns = F::ns(p - 1);
                const int k = j & (ns - 1);
                float2 *w = s + (V / 16 * 17) * (j - k) + k + (k >> 4);
#pragma unroll
                for (int idx = 0; idx < V; ++idx)
                    w[idx * ns + ((idx * ns) >> 4)] = x[idx];
            }
            lds_barrier();
            const float2 *r0 = s + j + (j >> 4);
#pragma unroll
            for (int r = 0; r < V; ++r)
                x[r] = r0[r * (F::TR / 16 * 17)];
        } else {
#pragma unroll
            for (int idx = 0; idx < V; ++idx)
                s[slot(out_pos<M>(p - 1, j, idx))] = x[idx];
            lds_barrier();
#pragma unroll
            for (int r = 0; r < V; ++r)
                x[r] = s[slot(j + r * F::TR)];
        }
        float2 w[V];
        if (p < NP) {
            const float2 *te = sets + (V - 1) * (F::tw_first(p) + (j & (F::ns(p) - 1)));
#pragma unroll
            for (int r = 1; r < V; ++r)
                w[r] = te[r - 1];
        } else {
            butterfly_twiddles<F::LV>(lt, w);
        }
#pragma unroll
        for (int r = 1; r < V; ++r)
            x[r] = cmul(x[r], w[r]);
        dft<V>(x);
    }
}

enum class RowOp { Forward, Fresnel };

// Inputs of this thread for one line: x[r] = element j + r TR of the line
// for r < NIN, zeros beyond.  A line is a row of `in` (element i at
// in[line * ld + i]) or, if COLS, a column (element i at in[i * ld + line]).
// No branch: a load under a branch is waited for where the branch joins,
// which would serialise the loads and end the prefetch.
template <int M, int NIN, bool COLS>
__device__ __forceinline__ void load_line(float2 (&x)[Fft<M>::V], const float2 *in, int64_t ld,
                                          int64_t line, int j)
{
    using F = Fft<M>;
    if constexpr (COLS) {
        // Buffer loads over the NIN TR rows of `in` (fewer than 2^31 bytes,
        // which the launch checks): one offset register per thread, and the
        // distance between a thread's loads, TR rows, in a scalar register.
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float2 *>(in), (short)0, (int)((int64_t)NIN * F::TR * ld * 8), 0x00020000);
        const uint32_t voff = (uint32_t)((line + (int64_t)j * ld) * 8);
        const uint32_t step = (uint32_t)((int64_t)F::TR * ld * 8);
#pragma unroll
        for (int r = 0; r < F::V; ++r)
            x[r] = r < NIN ? __builtin_bit_cast(
                                 float2, __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff, r * step, 0))
                           : float2{0.0f, 0.0f};
    } else {
        const float2 *src = in + line * ld;
#pragma unroll
        for (int r = 0; r < F::V; ++r)
            x[r] = r < NIN ? src[j + r * F::TR] : float2{0.0f, 0.0f};
    }
}

// Line group of workgroup b's k-th turn (G = gridDim.x workgroups, `full`
// = the number of turns in which all G take a group): b + k G in general.
// The hardware deals consecutive workgroups to the eight XCDs in turn; when
// the lines are columns, a full turn is dealt so that each XCD takes G/8
// adjacent groups, whose loads then share cache lines in that XCD's L2 (a
// row's segment of G/8 columns) instead of every line reaching all eight.
template <bool COLS>
__device__ __forceinline__ int group_of(int b, int k, int G, int full)
{
    if (!COLS || G % 8 != 0 || k >= full)
        return b + k * G;
    return k * G + (b % 8) * (G / 8) + b / 8;
}

// Persistent over line groups (ROWS lines each): workgroup b takes groups
// b, b + G, b + 2G, ... (G = gridDim.x, sized to what is resident at once),
// and the loads of its next group are in flight while it transforms the
// current one.  Per line (a row of `in`, or a column if COLS): loads its
// elements 0 .. n_in) (zeros beyond; n_in = L/2 if HALF_IN, else L), then
//   Forward: F (all L outputs stored);
//   Fresnel: F, times hc[i] (the spectrum of the one-dimensional impulse
//            response at frequency i), then conj F conj (outputs 0 .. L/2
//            stored, times `scale`): the line's linear convolution with h1;
// into row `line` of out, lines < n_lines.  Without COLS, in and out may
// be the same rows (a thread's loads of a row precede its stores, and a row
// is read by its own threads only); with COLS they must not overlap.  Lines
// of a last, partial group are computed from a repeated line and not
// stored.
template <RowOp OP, int M, bool HALF_IN, bool COLS>
__global__ __launch_bounds__(Fft<M>::T) __attribute__((amdgpu_waves_per_eu(
    Fft<M>::WAVES_PER_EU))) void k_fft_rows(const float2 *in, int64_t in_ld, float2 *out,
                                            int64_t out_ld, int n_rows,
                                            const float2 *__restrict__ twp,
                                            const float2 *__restrict__ hc, float2 scale)
{
    using F = Fft<M>;
    constexpr int V = F::V;
    constexpr int NIN = HALF_IN ? V / 2 : V;
    constexpr int NOUT = OP == RowOp::Forward ? V : V / 2;
    extern __shared__ float2 lds[];
    const int rl = threadIdx.x / F::TR;
    const int j = threadIdx.x % F::TR;
    float2 *s = lds + rl * F::ROW_SLOTS;
    float2 *sets = lds + F::ROWS * F::ROW_SLOTS;
    const int groups = (n_rows + F::ROWS - 1) / F::ROWS;
    const int G = (int)gridDim.x, b0 = (int)blockIdx.x;
    const int full = groups / G;
    auto row_of = [&](int k) -> int64_t {
        const int r = group_of<COLS>(b0, k, G, full) * F::ROWS + rl;
        return F::ROWS == 1 || r < n_rows ? r : n_rows - 1;
    };

    // twiddle sets of passes 1 .. NP-1, expanded to their V - 1 values in
    // LDS (ordered before their first use by the transform's first barrier);
    // the last pass's set stays in registers
    for (int t = threadIdx.x; t < F::LDS_SETS; t += F::T) {
        float2 w[V];
        butterfly_twiddles<F::LV>(twp + F::LV * t, w);
#pragma unroll
        for (int r = 1; r < V; ++r)
            sets[(V - 1) * t + r - 1] = w[r];
    }
    float2 lt[F::LV];
#pragma unroll
    for (int b = 0; b < F::LV; ++b)
        lt[b] = twp[F::LV * (F::tw_first(F::NP) + j) + b];

    float2 xn[V];
    load_line<M, NIN, COLS>(xn, in, in_ld, row_of(0), j);
    for (int k = 0; b0 + k * G < groups; ++k) {
        const int64_t row = (int64_t)group_of<COLS>(b0, k, G, full) * F::ROWS + rl;
        const bool live = F::ROWS == 1 || row < n_rows;
        const bool more = b0 + (k + 1) * G < groups;
        float2 x[V];
#pragma unroll
        for (int r = 0; r < V; ++r)
            x[r] = xn[r];
        // The next group's loads, in flight through this group's transforms
        // (their barriers wait for LDS operations only).  The Fresnel row
        // issues them after its spectrum loads, which it waits for mid-row.
        if (OP != RowOp::Fresnel && more)
            load_line<M, NIN, COLS>(xn, in, in_ld, row_of(k + 1), j);
        fft_row<M>(x, s, j, sets, lt);
        float2 crow{1.0f, 0.0f};
        if (OP == RowOp::Fresnel) {
            // All V spectrum loads in flight at once, then the products.
            // The empty asm hides the index from the compiler, so the loads
            // cannot be hoisted into the transform, where they would hold
            // 2 V more registers.  The constant `scale` commutes with the
            // inverse transform and is applied to the stored outputs.
            int jj = j;
            asm volatile("" : "+v"(jj));
            float2 h[V];
#pragma unroll
            for (int r = 0; r < V; ++r)
                h[r] = hc[jj + r * F::TR];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int r = 0; r < V; ++r)
                x[r] = conjf2(cmul(x[r], h[r]));
            crow = scale;
            if (more)
                load_line<M, NIN, COLS>(xn, in, in_ld, row_of(k + 1), j);
            fft_row<M>(x, s, j, sets, lt);
        }
        if (live) {
            // store addresses from here on (hoisted, they would hold 2 V registers)
            int jo = j;
            asm volatile("" : "+v"(jo));
            float2 *dst = out + row * out_ld + jo;
#pragma unroll
            for (int q = 0; q < NOUT; ++q) {
                float2 v = x[q];
                if (OP == RowOp::Fresnel)
                    v = cmul(conjf2(v), crow);
                dst[q * F::TR] = v;
            }
        }
    }
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

// The pass twiddle table of a length-2^m transform (layout at
// pass_table_entries), computed in FP64: w = exp(-2 pi i / L).
__global__ void k_twiddles(int m, int entries, float2 *tw)
{
    const int L = 1 << m;
    const int lv = values_log2(m);
    const int lr0 = m % lv == 0 ? lv : m % lv;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < entries;
         t += gridDim.x * blockDim.x) {
        int first = 0, lns = lr0;
        while (t >= first + (1 << lns)) {
            first += 1 << lns;
            lns += lv;
        }
        const int e = (t - first) << (m - lns - lv);
        for (int b = 0; b < lv; ++b) {
            double sn, cs;
            sincospi(2.0 * (double)((e << b) & (L - 1)) / (double)L, &sn, &cs);
            tw[lv * t + b] = float2{(float)cs, (float)-sn};
        }
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

// Workgroups of a row kernel resident at once on the current device (the
// persistent grid), queried once per kernel and device: at plan set-up, so a
// run that is being captured into a graph makes no query.
constexpr int kMaxDevices = 64;

template <RowOp OP, int M, bool HALF_IN, bool COLS>
hipError_t resident_groups(int *out)
{
    static std::atomic<int> cached[kMaxDevices];   // zero-initialised (static storage)
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    int r = cached[dev].load(std::memory_order_relaxed);
    if (r == 0) {
        int cus = 0, per_cu = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, (const void *)k_fft_rows<OP, M, HALF_IN, COLS>, Fft<M>::T,
                Fft<M>::lds_bytes);
        if (e != hipSuccess)
            return e;
        r = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
        cached[dev].store(r, std::memory_order_relaxed);
    }
    *out = r;
    return hipSuccess;
}

// The two line kernels of a length 2^M: Forward over rows with all L inputs
// (the chirp's transform), and Fresnel with L/2 inputs, over columns for
// M <= kColsMaxLog2 and over rows above.
template <RowOp OP>
constexpr bool fresnel_op = OP == RowOp::Fresnel;
constexpr bool cols_pipeline(int m) { return m <= kColsMaxLog2; }
template <RowOp OP, int M>
constexpr bool line_cols = fresnel_op<OP> && cols_pipeline(M);

template <RowOp OP, int M>
hipError_t launch_rows(const float2 *in, int64_t in_ld, float2 *out, int64_t out_ld, int n_rows,
                       int64_t groups, const float2 *tw, const float2 *hc, float2 scale,
                       hipStream_t s)
{
    using F = Fft<M>;
    constexpr bool FR = fresnel_op<OP>, COLS = line_cols<OP, M>;
    int resident = 0;
    hipError_t e = resident_groups<OP, M, FR, COLS>(&resident);
    if (e != hipSuccess)
        return e;
    const unsigned grid = (unsigned)(groups < resident ? groups : resident);
    hipLaunchKernelGGL((k_fft_rows<OP, M, FR, COLS>), dim3(grid), dim3(F::T), F::lds_bytes, s,
                       in, in_ld, out, out_ld, n_rows, tw, hc, scale);
    return hipGetLastError();
}

// Line transforms of n_rows lines of length L = 2^m into rows of out:
// Forward takes rows of `in` with all L inputs and stores all L outputs;
// Fresnel takes L/2 inputs per line and stores L/2 outputs, its lines being
// columns of `in` (element i of column c at in[i * in_ld + c]) if
// cols_pipeline(m), else rows.
template <RowOp OP, int M = kMinLog2>
hipError_t rows(const float2 *in, int64_t in_ld, int n_in, float2 *out, int64_t out_ld,
                int n_rows, int m, const float2 *tw, const float2 *hc, float2 scale,
                hipStream_t s)
{
    if constexpr (M > kMaxLog2) {
        return hipErrorInvalidValue;
    } else {
        if (m != M)
            return rows<OP, M + 1>(in, in_ld, n_in, out, out_ld, n_rows, m, tw, hc, scale, s);
        using F = Fft<M>;
        if (n_in != (fresnel_op<OP> ? F::L / 2 : F::L))
            return hipErrorInvalidValue;
        if (n_rows <= 0)
            return hipSuccess;
        // column lines c < n_rows of an n_in-row input are read through one
        // buffer resource (a 31-bit byte range)
        if (line_cols<OP, M> &&
            (n_rows > in_ld || (int64_t)n_in * in_ld * (int64_t)sizeof(float2) > INT32_MAX))
            return hipErrorInvalidValue;
        const int64_t groups = ((int64_t)n_rows + F::ROWS - 1) / F::ROWS;
        return launch_rows<OP, M>(in, in_ld, out, out_ld, n_rows, groups, tw, hc, scale, s);
    }
}

template <int M = kMinLog2>
hipError_t prepare_rows()
{
    if constexpr (M > kMaxLog2) {
        return hipSuccess;
    } else {
        const int lds = (int)Fft<M>::lds_bytes;
        constexpr bool COLS = line_cols<RowOp::Fresnel, M>;
        const void *kernels[] = {(const void *)k_fft_rows<RowOp::Forward, M, false, false>,
                                 (const void *)k_fft_rows<RowOp::Fresnel, M, true, COLS>};
        for (const void *k : kernels) {
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e != hipSuccess)
                return e;
        }
        int r = 0;
        hipError_t e = resident_groups<RowOp::Forward, M, false, false>(&r);
        if (e == hipSuccess)
            e = resident_groups<RowOp::Fresnel, M, true, COLS>(&r);
        if (e != hipSuccess)
            return e;
        return prepare_rows<M + 1>();
    }
}

hipError_t transpose(const float2 *in, int64_t in_ld, float2 *out, int64_t out_ld, int r, int c,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)((c + 31) / 32), (unsigned)((r + 31) / 32)),
                       dim3(256), 0, s, in, in_ld, out, out_ld, r, c);
    return hipGetLastError();
}

}  // namespace

hipError_t fresnel_prepare_kernels() { return prepare_rows(); }

size_t fresnel_workspace_planes(int m) { return cols_pipeline(m) ? 1 : 2; }

size_t fresnel_twiddle_bytes(int m)
{
    return m < kMinLog2 || m > kMaxLog2
               ? 0
               : (size_t)pass_table_entries(m) * values_log2(m) * sizeof(float2);
}

hipError_t fresnel_tables(int n, int m, double q, float2 *tw, float2 *hc, hipStream_t s)
{
    if (n < 1 || m < kMinLog2 || m > kMaxLog2 || (2 * n) != (1 << m))
        return hipErrorInvalidValue;
    const int L = 1 << m;
    const unsigned blocks = (unsigned)((L + 255) / 256);
    hipLaunchKernelGGL(k_twiddles, dim3(blocks), dim3(256), 0, s, m, pass_table_entries(m), tw);
    hipLaunchKernelGGL(k_chirp, dim3(blocks), dim3(256), 0, s, m, n, q, hc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // hc <- F[h1], in place (one row)
    return rows<RowOp::Forward>(hc, L, L, hc, L, 1, m, tw, nullptr, float2{0.0f, 0.0f}, s);
}

hipError_t fresnel_run(int n, int m, const float2 *tw, const float2 *hc, float2 scale,
                       const float2 *u, float2 *out, float2 *x, float2 *y, hipStream_t s)
{
    if (n < 1 || m < kMinLog2 || m > kMaxLog2 || (2 * n) != (1 << m))
        return hipErrorInvalidValue;
    const float2 one{1.0f, 0.0f};
    hipError_t e;
    // h(a, b) = h1(a) h1(b): the 2-D linear convolution is the 1-D one along
    // every column and then along every row, or the other way round.
    if (cols_pipeline(m)) {
        // Columns of u: x = Z^T, Z = (u * h1 along the first index) C p^2,
        // a column of Z per row of x; then the columns of x (the rows of Z):
        // O = Z * h1 along the second index, row by row.
        e = rows<RowOp::Fresnel>(u, n, n, x, n, n, m, tw, hc, scale, s);
        if (e != hipSuccess)
            return e;
        return rows<RowOp::Fresnel>(x, n, n, out, n, n, m, tw, hc, one, s);
    }
    // Rows of u: V = (u * h1 along the second index) C p^2; W = V^T; the rows
    // of W (the columns of V) convolved in place; O = W^T.
    e = rows<RowOp::Fresnel>(u, n, n, x, n, n, m, tw, hc, scale, s);
    if (e != hipSuccess)
        return e;
    e = transpose(x, n, y, n, n, n, s);
    if (e != hipSuccess)
        return e;
    e = rows<RowOp::Fresnel>(y, n, n, y, n, n, m, tw, hc, one, s);
    if (e != hipSuccess)
        return e;
    return transpose(y, n, out, n, n, n, s);
}

}  // namespace cgh
