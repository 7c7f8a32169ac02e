// Microbenchmarks of the gfx950 rates the kernels' rooflines rest on.
//
//     paper_1309_2734_amd/cgh_microbench        (built by paper_1309_2734_amd/build.py)
//
// Prints one line per measurement:
//   - accuracy and bias of the hardware cosine and sine (v_cos_f32 /
//     v_sin_f32, argument in revolutions) over the argument ranges the direct
//     and factor kernels use, against FP64 on the host;
//   - issue rates: v_cos_f32, v_fma_f32, v_fma_f64, and the direct kernel's
//     per-term sequence (add, cosine, multiply-add), per clock and CU at the
//     device's nominal clock;
//   - matrix-core rates of the instructions the GEMM uses
//     (v_mfma_f32_16x16x32_bf16 / _f16, v_mfma_f32_16x16x4_f32);
//   - HBM: a plain write and a plain copy of 1 GiB;
//   - LDS: ds_read_b128 bandwidth per CU.
// Rates are averaged over launches repeated for ~0.3 s, while a second
// thread samples the shader clock the driver reports (pp_dpm_sclk), so each
// rate is also given per clock at that clock.  Every kernel works in
// registers or on buffers it allocates; grids and indices are fixed and in
// bounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#define CK(x)                                                                                  \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) {                                                                \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);        \
            std::exit(1);                                                                      \
        }                                                                                      \
    } while (0)

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// out[i] = hardware cosine (or sine) of lo + span * i / n, i < n
__global__ __launch_bounds__(256) void k_trig(float *out, long n, float lo, float span, int sine)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float t = lo + span * ((float)i * (1.0f / (float)n));
    out[i] = sine ? __builtin_amdgcn_sinf(t) : __builtin_amdgcn_cosf(t);
}

// Issue-rate loops: 8 independent chains per thread, `iters` iterations.
// op 0: v_cos_f32; 1: v_fma_f32; 2: per-term sequence t = v + u, c = cos(t),
// acc = fma(a, c, acc) with u advanced once per iteration.
template <int OP>
__global__ __launch_bounds__(256) void k_rate(float *out, int iters, float seed)
{
    float x[8], acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = seed + 0.01f * k + 1e-6f * threadIdx.x;
        acc[k] = 0.0f;
    }
    float u = 0.37f * seed;
    for (int it = 0; it < iters; ++it) {
        if (OP == 2)
            u += 1.0e-7f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (OP == 0)
                x[k] = __builtin_amdgcn_cosf(x[k]);
            else if (OP == 1)
                x[k] = __builtin_fmaf(x[k], 0.999f, 0.001f);
            else
                acc[k] = __builtin_fmaf(x[k], __builtin_amdgcn_cosf(x[k] + u), acc[k]);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        s += x[k] + acc[k];
    out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_rate_f64(double *out, int iters, double seed)
{
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        x[k] = seed + 0.01 * k + 1e-6 * threadIdx.x;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int k = 0; k < 8; ++k)
            x[k] = __builtin_fma(x[k], 0.999, 0.001);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        s += x[k];
    out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Matrix-core loops: 4 independent accumulators per wave, each instruction
// taking the same operands.  T 0: 16x16x32 bf16; 1: 16x16x32 f16;
// 2: 16x16x4 f32.
template <int T>
struct MfmaOp;
template <>
struct MfmaOp<0> {
    typedef bf16x8 op_t;
    static __device__ op_t make(float v)
    {
        op_t a;
        for (int k = 0; k < 8; ++k)
            a[k] = (__bf16)(v + 0.001f * k);
        return a;
    }
    static __device__ f32x4 run(op_t a, op_t b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct MfmaOp<1> {
    typedef f16x8 op_t;
    static __device__ op_t make(float v)
    {
        op_t a;
        for (int k = 0; k < 8; ++k)
            a[k] = (_Float16)(v + 0.001f * k);
        return a;
    }
    static __device__ f32x4 run(op_t a, op_t b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct MfmaOp<2> {
    typedef float op_t;
    static __device__ op_t make(float v) { return v; }
    static __device__ f32x4 run(op_t a, op_t b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <int T>
__global__ void k_mfma(float *out, int iters)
{
    typedef MfmaOp<T> Op;
    const typename Op::op_t a = Op::make(0.001f * threadIdx.x), b = Op::make(0.002f);
    f32x4 c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        c[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            c[j] = Op::run(a, b, c[j]);
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
    out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_write(float4 *p, long n, float v)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = float4{v, v + 1.0f, v + 2.0f, v + 3.0f};
}

__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ a, float4 *__restrict__ b,
                                              long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        b[i] = a[i];
}

// Every lane reads 16 B per ds_read_b128 from a 64 KB buffer at
// conflict-free addresses; the values are kept live by empty asm uses.
__global__ __launch_bounds__(512) void k_lds(int *out, int iters)
{
    __shared__ float4 buf[4096];
    for (int i = threadIdx.x; i < 4096; i += 512)
        buf[i] = make_float4((float)i, (float)i, (float)i, (float)i);
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = buf[(threadIdx.x + u * 512 + it) & 4095];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            asm volatile("" ::"v"(v[u].x), "v"(v[u].y), "v"(v[u].z), "v"(v[u].w));
    }
    if (threadIdx.x == 0)
        out[blockIdx.x] = 1;
}

// The shader clock the driver reports as current (the starred level of
// pp_dpm_sclk, largest over the cards), sampled every ~2 ms from a second
// thread while a measurement repeats.  0 where the files are unreadable.
int current_sclk_mhz()
{
    int best = 0;
    for (int card = 0; card < 64; ++card) {
        char path[96];
        std::snprintf(path, sizeof(path), "/sys/class/drm/card%d/device/pp_dpm_sclk", card);
        FILE *f = std::fopen(path, "r");
        if (!f)
            continue;
        char line[128];
        while (std::fgets(line, sizeof(line), f)) {
            if (!std::strchr(line, '*'))
                continue;
            const char *colon = std::strchr(line, ':');
            const int mhz = colon ? std::atoi(colon + 1) : 0;
            best = std::max(best, mhz);
        }
        std::fclose(f);
    }
    return best;
}

struct ClockSampler {
    std::atomic<bool> stop{false};
    std::vector<int> samples;
    std::thread th;
    void start()
    {
        stop = false;
        samples.clear();
        th = std::thread([this] {
            while (!stop) {
                const int mhz = current_sclk_mhz();
                if (mhz >= 500)          // idle gaps read ~100 MHz
                    samples.push_back(mhz);
                std::this_thread::sleep_for(std::chrono::milliseconds(2));
            }
        });
    }
    int finish_median()
    {
        stop = true;
        th.join();
        if (samples.empty())
            return 0;
        std::sort(samples.begin(), samples.end());
        return samples[samples.size() / 2];
    }
};

}  // namespace

int main()
{
    hipDeviceProp_t prop;
    CK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const double clk_hz = prop.clockRate * 1e3;       // nominal shader clock
    std::printf("device %s (%s), %d CUs, nominal clock %.0f MHz\n", prop.name, prop.gcnArchName,
                cus, clk_hz / 1e6);
    std::fflush(stdout);
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    // seconds per launch, averaged over launches repeated for ~0.3 s, and the
    // median sampled shader clock (MHz) meanwhile
    int last_mhz = 0;
    auto timed = [&](auto launch) {
        launch();                                    // warm-up and length probe
        CK(hipDeviceSynchronize());
        CK(hipEventRecord(e0, 0));
        launch();
        CK(hipEventRecord(e1, 0));
        CK(hipEventSynchronize(e1));
        CK(hipGetLastError());
        float ms = 0.0f;
        CK(hipEventElapsedTime(&ms, e0, e1));
        const int reps = std::max(1, std::min(1000, (int)(300.0 / std::max(ms, 1e-3f))));
        ClockSampler clk;
        clk.start();
        CK(hipEventRecord(e0, 0));
        for (int r = 0; r < reps; ++r)
            launch();
        CK(hipEventRecord(e1, 0));
        CK(hipEventSynchronize(e1));
        last_mhz = clk.finish_median();
        CK(hipGetLastError());
        CK(hipEventElapsedTime(&ms, e0, e1));
        return (double)ms * 1e-3 / reps;
    };
    auto at_clock = [&](double per_s) {
        static char buf[64];
        if (last_mhz > 0)
            std::snprintf(buf, sizeof(buf), "; %.1f at the sampled %d MHz",
                          per_s / cus / (last_mhz * 1e6), last_mhz);
        else
            std::snprintf(buf, sizeof(buf), "; clock not readable");
        return buf;
    };

    // ---- hardware cosine / sine accuracy
    {
        const long n = 1L << 24;
        float *d = nullptr;
        CK(hipMalloc(&d, n * sizeof(float)));
        std::vector<float> h(n);
        struct Case {
            const char *name;
            float lo, span;
            int sine;
        } cases[] = {{"v_cos_f32 on [0, 2) rev", 0.0f, 2.0f, 0},
                     {"v_cos_f32 on [0, 1) rev", 0.0f, 1.0f, 0},
                     {"v_sin_f32 on [0, 1) rev", 0.0f, 1.0f, 1}};
        for (const Case &c : cases) {
            hipLaunchKernelGGL(k_trig, dim3((unsigned)(n / 256)), dim3(256), 0, 0, d, n, c.lo,
                               c.span, c.sine);
            CK(hipDeviceSynchronize());
            CK(hipGetLastError());
            CK(hipMemcpy(h.data(), d, n * sizeof(float), hipMemcpyDeviceToHost));
            double mx = 0.0, sum = 0.0, sq = 0.0;
            for (long i = 0; i < n; ++i) {
                const float t = c.lo + c.span * ((float)i * (1.0f / (float)n));
                const double a = 6.283185307179586 * (double)t;
                const double e = (double)h[i] - (c.sine ? std::sin(a) : std::cos(a));
                mx = std::fmax(mx, std::fabs(e));
                sum += e;
                sq += e * e;
            }
            std::printf("%-26s max abs err %.3e  mean err %.3e  rms err %.3e  (%ld points)\n",
                        c.name, mx, sum / n, std::sqrt(sq / n), n);
        }
        CK(hipFree(d));
        std::fflush(stdout);
    }

    // ---- issue rates
    {
        const int blocks = cus * 8, threads = 256, iters = 16384;   // launches of ~1 ms
        void *o = nullptr;
        CK(hipMalloc(&o, (size_t)blocks * threads * sizeof(double)));
        const double lanes = (double)blocks * threads * iters;
        auto report = [&](const char *name, double s, double per_iter, const char *unit) {
            const double r = lanes * per_iter / s;
            std::printf("%-34s %.3e %s/s  %.1f per clock per CU at the nominal clock%s\n", name,
                        r, unit, r / cus / clk_hz, at_clock(r));
        };
        report("v_cos_f32 (8 chains)", timed([&] {
                   hipLaunchKernelGGL(k_rate<0>, dim3(blocks), dim3(threads), 0, 0, (float *)o,
                                      iters, 0.1f);
               }), 8, "lane-op");
        report("v_fma_f32 (8 chains)", timed([&] {
                   hipLaunchKernelGGL(k_rate<1>, dim3(blocks), dim3(threads), 0, 0, (float *)o,
                                      iters, 0.1f);
               }), 8, "lane-op");
        report("term: add + cos + fma", timed([&] {
                   hipLaunchKernelGGL(k_rate<2>, dim3(blocks), dim3(threads), 0, 0, (float *)o,
                                      iters, 0.1f);
               }), 8, "term");
        report("v_fma_f64 (8 chains)", timed([&] {
                   hipLaunchKernelGGL(k_rate_f64, dim3(blocks), dim3(threads), 0, 0, (double *)o,
                                      iters, 0.1);
               }), 8, "lane-op");
        // matrix cores: flops per instruction / 64 lanes, 4 instructions per iteration
        const int mi = iters;
        const double lanes_m = (double)blocks * threads * mi;
        auto mreport = [&](const char *name, double s, double flop_per_instr) {
            const double r = lanes_m * 4.0 * flop_per_instr / 64.0 / s;
            std::printf("%-34s %.1f TFLOP/s  (%.0f flop per clock per CU at the nominal clock%s)\n",
                        name, r / 1e12, r / cus / clk_hz, at_clock(r));
        };
        mreport("v_mfma_f32_16x16x32_bf16", timed([&] {
                    hipLaunchKernelGGL(k_mfma<0>, dim3(blocks), dim3(threads), 0, 0, (float *)o, mi);
                }), 16.0 * 16 * 32 * 2);
        mreport("v_mfma_f32_16x16x32_f16", timed([&] {
                    hipLaunchKernelGGL(k_mfma<1>, dim3(blocks), dim3(threads), 0, 0, (float *)o, mi);
                }), 16.0 * 16 * 32 * 2);
        mreport("v_mfma_f32_16x16x4_f32", timed([&] {
                    hipLaunchKernelGGL(k_mfma<2>, dim3(blocks), dim3(threads), 0, 0, (float *)o, mi);
                }), 16.0 * 16 * 4 * 2);
        CK(hipFree(o));
        std::fflush(stdout);
    }

    // ---- HBM
    {
        const size_t bytes = (size_t)1 << 30;   // 4x the 256 MB memory-side cache
        const long n = (long)(bytes / sizeof(float4));
        float4 *a = nullptr, *b = nullptr;
        CK(hipMalloc(&a, bytes));
        CK(hipMalloc(&b, bytes));
        const unsigned blocks = (unsigned)((n + 255) / 256);
        const double tw = timed([&] { hipLaunchKernelGGL(k_write, dim3(blocks), dim3(256), 0, 0, a, n, 1.0f); });
        const double tc = timed([&] { hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, 0, a, b, n); });
        std::printf("HBM write, 1 GiB                   %.2f TB/s\n", bytes / tw / 1e12);
        std::printf("HBM copy, 1 GiB (read + write)     %.2f TB/s\n", 2.0 * bytes / tc / 1e12);
        CK(hipFree(a));
        CK(hipFree(b));
        std::fflush(stdout);
    }

    // ---- LDS
    {
        int *d = nullptr;
        CK(hipMalloc(&d, (size_t)cus * 2 * sizeof(int)));
        for (int per_cu = 1; per_cu <= 2; ++per_cu) {
            const int blocks = cus * per_cu, iters = 20000;
            const double s = timed([&] {
                hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(512), 0, 0, d, iters);
            });
            const double bytes = (double)blocks * 512 * iters * 8 * 16;
            std::printf("LDS ds_read_b128, %d x 512 threads/CU %.1f B per clock per CU at the "
                        "nominal clock%s\n", per_cu, bytes / s / cus / clk_hz, at_clock(bytes / s));
        }
        CK(hipFree(d));
    }
    std::printf("done\n");
    return 0;
}
