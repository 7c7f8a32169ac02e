// Internal declarations shared by the host library and the gfx950 kernels.
//
// Notation (Section 2.1, Eq. (2)): pixel (ix, iy), point j with (x_j, y_j,
// z_j, A_j), wavelength lambda, pitch p.  In pixel units the Fresnel phase of
// point j at pixel (ix, iy), in revolutions, is
//
//     phi_j(ix, iy) = beta_j (ix - cx_j)^2 + beta_j (iy - cy_j)^2,
//     beta_j = p^2 / (2 lambda z_j),  cx_j = (W-1)/2 + x_j / p,  cy_j = (H-1)/2 + y_j / p,
//
// because pi r^2 / (lambda z) radians = r^2 / (2 lambda z) revolutions.  The
// sum of Eq. (5) is I = sum_j A_j cos(2 pi phi_j).  The square splits into a
// column part and a row part; every kernel here works on those two "line
// phases", reduced modulo one revolution in FP64:
//
//     U[ix, j] = frac(beta_j (ix - cx_j)^2),   V[iy, j] = frac(beta_j (iy - cy_j)^2),
//
// so that cos(2 pi phi_j) = cos(2 pi (U + V)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cgh {

// Points are processed in groups of this many (tables are blocked by group).
constexpr int kGroup = 16;
// Every segment's slots are padded (with zero-amplitude points) to a multiple
// of this, so each frame has an even number of groups.
constexpr int kSlotAlign = 32;
// Line tables are padded to a multiple of this many columns / rows.
constexpr int kLinePad = 64;
// Matrix-core operand blocks (factors.hip, gemm.hip) are 1 KB of 16 lines:
// 32 K-columns = 16 points in bf16/f16, 16 K-columns = 8 points in FP32.
constexpr int kFragLines = 16;

// Per-point constants of one evaluation segment, structure of arrays.
struct PointConsts {
    double *beta;  // revolutions per pixel^2
    double *cx;    // point position in pixel units along x
    double *cy;    // ... along y
    double *zlam;  // z_j / lambda: the on-axis distance in revolutions
    float *amp;    // A_j
    float *zhalf;  // z_j / (2 lambda), rounded to float
};

// DPP row_newbcast:K -- every lane of a 16-lane row reads lane K of that row.
// The compiler folds the move into a consuming VOP2 instruction (v_add_f32).
template <int K>
__device__ __forceinline__ float row_bcast(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x150 + K, 0xF, 0xF, false));
}

// A run of points to prepare: source points [src, src + count) of the
// uploaded cloud, seen at wavelength `wavelength`, written to constant slots
// [dst, dst + count) and zero-padded to a multiple of kSlotAlign.
struct Segment {
    int64_t src;
    int64_t count;
    int64_t dst;       // multiple of kSlotAlign
    double wavelength;
};

// One hologram of a (possibly batched) evaluation.
struct FrameDesc {
    int64_t first;     // first constant slot (multiple of kSlotAlign)
    int64_t groups;    // point groups: count padded to kSlotAlign, / kGroup (even)
    int64_t out_off;   // offset of the frame's output in floats
};

// Segments of a launch: a device table (dev != nullptr, entry blockIdx.y),
// or one segment passed by value in the kernel arguments, so that a single
// hologram's evaluation needs no table in device memory.
struct SegList {
    const Segment *dev;
    Segment one;
};

// Frames of a direct launch: a device table, or up to kInlineFrames frames in
// the kernel arguments (a single hologram, whole or cut into point runs).
constexpr int kInlineFrames = 4;
struct FrameList {
    const FrameDesc *dev;
    FrameDesc inl[kInlineFrames];
};

// A 64-bit value every lane holds, made scalar (each half through uint32_t:
// readfirstlane returns int).
__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Frame i (i the same in every lane).  The fields are made scalar
// explicitly: the compiler does not prove a value chosen between the device
// table and the kernel arguments uniform, and would otherwise keep the
// frame's per-point loads (amplitudes) in vector registers.
__device__ __forceinline__ FrameDesc frame_at(const FrameList &f, int i)
{
    const FrameDesc d = f.dev ? f.dev[i] : f.inl[i];
    return FrameDesc{uniform_i64(d.first), uniform_i64(d.groups), uniform_i64(d.out_off)};
}

// ---------------------------------------------------------------- launchers
// Each returns the hipError_t of the launch.

// a1: per-point constants for a list of segments.
hipError_t launch_point_consts(const float *x, const float *y, const float *z, const float *amp,
                               const SegList &segs, int n_segs, int64_t max_count,
                               int width, int height, double pitch, PointConsts pc,
                               hipStream_t s);

// a2: line-phase tables for the direct kernel, blocked as [group][line][kGroup]:
// U over `wpad` columns, V over `hpad` rows (lines past the hologram are
// evaluated like the others and never stored), for slots [0, n_slots).
hipError_t launch_phase_tables(PointConsts pc, int64_t n_slots, int wpad, int hpad,
                               float *U, float *V, hipStream_t s);

// a2s: tables of the exact spherical wave (Eq. (1)), blocked like a2's:
// U, V as a2's with z_j / lambda added to V before the reduction, and the
// squared offsets in units of z_j, X = ((ix - cx_j) p / z_j)^2 and
// Y = ((iy - cy_j) p / z_j)^2.
hipError_t launch_sphere_tables(PointConsts pc, int64_t n_slots, int wpad, int hpad, float *U,
                                float *V, float *X, float *Y, hipStream_t s);

// a3s: direct FP32 accumulation of the exact spherical wave (tables from a2s).
hipError_t launch_direct_sphere(const float *U, const float *V, const float *X, const float *Y,
                                const float *amp, const float *zhalf,
                                const FrameList &frames, int n_frames, int width, int height,
                                int wpad, int hpad, int rows_per_wave, float *out,
                                float *out_im, bool accumulate, hipStream_t s);

// a3: direct FP32 accumulation for frames[0 .. n_frames) (tables from a2,
// padded to wpad columns and hpad rows, multiples of kLinePad).  With out_im
// != nullptr the imaginary part of the object wave goes there as well.
hipError_t launch_direct(const float *U, const float *V, const float *amp,
                         const FrameList &frames, int n_frames, int width, int height,
                         int wpad, int hpad, int rows_per_wave, float *out, float *out_im,
                         bool accumulate, hipStream_t s);

// a4/a5 factor set, K-major: for every K block kb one contiguous slab of
// slab_blocks() 1 KB operand blocks -- the line blocks of Lh [0, amb), of Ll
// [amb, 2 amb) (with lo halves), then those of Rh and Rl (anb each).  Block b
// of an array sits at base + (kb * slab_blocks() + first + b) KB, so a GEMM
// stage reads one slab and addresses it with small 32-bit offsets.
struct FactorSet {
    char *base = nullptr;
    int hl = 1;            // 2: hi and lo halves
    int amb = 0, anb = 0;  // L / R line blocks allocated
    int64_t kblocks = 0;   // K blocks allocated
    __host__ __device__ int slab_blocks() const { return hl * (amb + anb); }
    __host__ __device__ int first_l(bool lo) const { return lo ? amb : 0; }
    __host__ __device__ int first_r(bool lo) const { return hl * amb + (lo ? anb : 0); }
    int64_t bytes() const { return kblocks * slab_blocks() * (int64_t)1024; }
};

// a4: factor build.  Writes K blocks [0, kblocks) of the hi (and, with
// fs.hl == 2, lo) factors of L (rows; mblocks line blocks) and R (columns;
// nblocks) in the MFMA fragment order described in factors.hip; a K block
// holds kblock_points(ft) points starting at constant slot slot0.  FP32
// factors have no lo half.  With `cplx`, L has 2 * height lines: the
// real-part factors of rows 0 .. height-1, then the imaginary-part factors of
// the same rows, so that L R^T is [Re O; Im O].
enum class FactorType { BF16 = 0, FP16 = 1, FP32 = 2 };
// Points [src, src + count) of a cloud seen at `wavelength`, for kernels that
// evaluate the per-point constants themselves (half_w = (W-1)/2, half_h =
// (H-1)/2).  Slots past `count` are padding (zero amplitude).
struct RawPoints {
    const float *x, *y, *z, *amp;
    int64_t src, count;
    double wavelength, half_w, half_h, pitch;
};
constexpr int kblock_points(FactorType ft) { return ft == FactorType::FP32 ? 8 : 16; }
hipError_t launch_factors(PointConsts pc, int64_t slot0, int width, int height, bool cplx,
                          int64_t kblocks, int mblocks, int nblocks, FactorType ft,
                          const FactorSet &fs, hipStream_t s);
// a1 + a4 in one launch for a single hologram: the same factors from the
// points (constants evaluated in the kernel, as k_point_consts does).
hipError_t launch_factors_points(const RawPoints &rp, int width, int height, bool cplx,
                                 int64_t kblocks, int mblocks, int nblocks, FactorType ft,
                                 const FactorSet &fs, hipStream_t s);

// a5: split GEMM on MFMA.  See gemm.hip for the tiling.
struct GemmPlan {
    int bm, bn;          // macro tile (multiples of 32)
    int waves_m, waves_n;// wave grid of a workgroup (4 or 8 waves)
    int stages;          // LDS ring depth (copies run stages-1 K blocks ahead)
    int splits;          // K splits (1 = write the output directly)
    int64_t kblocks;     // K blocks of kblock_points(factor type) points
    int mblocks, nblocks;// line blocks of kFragLines (padded to whole tiles)
    int products;        // 3 = hi*hi + hi*lo + lo*hi, 1 = hi*hi only
};
// Launches whose tiles or K range fall outside the factor set are refused
// (hipErrorInvalidValue).
hipError_t launch_gemm(const GemmPlan &plan, FactorType ft, const FactorSet &fs, int M, int N,
                       float *out, int64_t ldo, float *partials, bool accumulate, hipStream_t s);
bool gemm_tile_supported(int bm, int bn, int waves_m, int waves_n, int stages);
// Workgroups of a shape that fit one CU at once (registers for two waves per
// SIMD, LDS for the copy ring).
int gemm_groups_per_cu(int bm, int bn, int waves_m, int waves_n, int stages, int products);
// Raises the GEMM kernels' LDS limit on the current device; called once per
// context, before any launch or capture.
hipError_t gemm_prepare_kernels();

// a6: one (frame, tile) work item of the persistent batched GEMM.  The
// factors of all frames sit side by side along K in one factor set; an
// item's K blocks are [kb_begin, kb_begin + kblocks).
struct BatchItem {
    int64_t kb_begin;
    int64_t kblocks;
    int64_t out_off;   // floats: frame index * height * width
    int32_t tm, tn;    // tile indices
};
// plan.kblocks = the factor set's K blocks; grid = persistent workgroups;
// counter = one int of device memory (reset by the launch).
hipError_t launch_gemm_batch(const GemmPlan &plan, FactorType ft, const FactorSet &fs,
                             const BatchItem *items, int n_items, int *counter, int M, int N,
                             float *out, int grid, hipStream_t s);
// a8: phase-only hologram (Eq. (3)) from the real and imaginary planes.
hipError_t launch_kinoform(const float *re, const float *im, int64_t n, uint8_t *out,
                           hipStream_t s);
// F4: Fresnel diffraction of a sampled n x n field (Eq. (10)), n a power of
// two, L = 2n <= 16384 (m = log2 L).  fresnel_tables fills the transforms'
// twiddle table tw (fresnel_twiddle_bytes(m) bytes) and the transform hc[L]
// of the 1-D chirp for q = p^2 / (2 lambda z) revolutions per pixel^2;
// fresnel_run propagates u (n x n complex) to out (n x n), scale =
// exp(i 2 pi z / lambda) / (i lambda z) p^2 / L^2, with workspaces x and y
// of n * n complex each (y only if fresnel_workspace_planes(m) is 2) that
// overlap neither u nor out (u and out may be the same buffer).
// fresnel_prepare_kernels raises the kernels' LDS limit (once, before any
// capture).
hipError_t fresnel_prepare_kernels();
size_t fresnel_twiddle_bytes(int m);
size_t fresnel_workspace_planes(int m);
hipError_t fresnel_tables(int n, int m, double q, float2 *tw, float2 *hc, hipStream_t s);
hipError_t fresnel_run(int n, int m, const float2 *tw, const float2 *hc, float2 scale,
                       const float2 *u, float2 *out, float2 *x, float2 *y, hipStream_t s);

hipError_t launch_splitk_reduce(const float *partials, int splits, int M, int N, float *out,
                                int64_t ldo, bool accumulate, hipStream_t s);

// Wavefront recording, first step (wrm.hip): per-point data of the recording
// on an n x n virtual plane at distance zw from the hologram.  box.z < 0 marks
// a point not beyond the plane.
struct WrmConsts {
    float4 *box;          // (cx, cy, disc radius in samples, 0) in FP32, for culling
    float4 *raw;          // (x, y, z, A) as uploaded; the FP64 constants of a point
                          // are evaluated from these where it is used
    // per group of kWrmGroup consecutive points: (x lo, x hi, y lo, y hi) in
    // samples bounding their discs (a sample wider), for culling whole groups
    float4 *gbox;
    int *next_tile;       // the recording kernel's tile queue (reset by the constants kernel)
};
constexpr int64_t kWrmGroup = 1024;
constexpr size_t kWrmBytesPerPoint = 2 * sizeof(float4);
hipError_t launch_wrm_consts(const float *x, const float *y, const float *z, const float *amp,
                             int64_t n_points, int n, double pitch, double lam, double zw,
                             const WrmConsts &wc, hipStream_t s);
// Clouds above kWrmQueueMinPoints points are recorded by persistent
// workgroups from a tile queue, their groups cut into `chunks` ranges of
// about kWrmPointsPerChunk points (at most kWrmMaxChunks), recorded as
// separate planes and summed in chunk order.
constexpr int64_t kWrmQueueMinPoints = 4 * kWrmGroup;
constexpr int64_t kWrmPointsPerChunk = 15000;
constexpr int kWrmMaxChunks = 4;
int wrm_record_chunks(int64_t n_points, int n);
// The recorded plane, n x n complex (re, im) pairs, every sample written;
// parts holds chunks - 1 further n x n planes (unused when chunks is 1).
hipError_t launch_wrm_record(const WrmConsts &wc, int64_t n_points, int n, double pitch,
                             double lam, double zw, int chunks, float2 *field, float2 *parts,
                             hipStream_t s);
// out[iy][ix] = Re field[iy + oy][ix + ox] for the width x height window.
hipError_t launch_window_real(const float2 *field, int n, int ox, int oy, int width, int height,
                              float *out, hipStream_t s);

}  // namespace cgh
