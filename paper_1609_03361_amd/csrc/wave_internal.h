// Internal interface between the host orchestration (wave_host.cpp) and the
// gfx950 kernels (wave_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wave {

constexpr int kMaxHalf = 8;        // space order 16 -> half-width 8

// One injection contribution.  Entries are sorted by (row, z, point) and a
// per-row CSR gives each row's range: the owner of grid node (row, z) adds
// alpha * w * val[pt] to its update, row = x*ny + y (3D) or x (2D).  Twelve
// bytes (the row is implied by the CSR), one dwordx3 load.
struct InjEntry {
    int32_t z;
    int32_t pt;
    float w;
};

// Device view of a set of sparse points used for sampling: flat index of the
// cell's lowest corner and the 2^d multilinear weights (corner bit a selects
// +1 along axis a, axis 0 most significant).
struct SampleSet {
    const int64_t* base;   // [npts]
    const float* w;        // [npts][2^d]
    int32_t npts;
};

struct InjectSet {
    const int32_t* row_ptr;   // [nrows + 1]
    const InjEntry* ent;      // [nent]
};

// Everything one time step needs.  `out` may alias `other` (in-place
// leapfrog: u^{n+1} overwrites u^{n-1}, each point is read then written by
// the same thread only).
struct StepArgs {
    const float* cur;      // u^n (forward) / v^k (adjoint)
    const float* other;    // u^{n-1} / v^{k+1}
    float* out;            // u^{n+1} / v^{k-1}
    const float* alpha;    // dt^2 / (m + eta dt/2)
    const float* beta;     // (m - eta dt/2) / (m + eta dt/2)
    int64_t nx, ny, nz;    // 2D: ny = 1
    float cx[kMaxHalf + 1], cy[kMaxHalf + 1], cz[kMaxHalf + 1];   // c_j / h^2, j >= 1
    // injection into `out` (values for this step)
    InjectSet inj;
    const float* inj_val;  // [npts of the injected set] for this step, or nullptr
    // optional: this step's weighted values already gathered into entry
    // order, inj_ev[e] = ent[e].w * inj_val[ent[e].pt] (rounded product; the
    // direct path forms the same product), or nullptr
    const float* inj_ev;
    // optional gather for the next step, done by extra blocks at the end of
    // the launch: ev_out[e] = ent[e].w * ev_src[ent[e].pt] for e < nent
    float* ev_out;
    const float* ev_src;
    int32_t nent;
    // sampling of `cur` (values for this step)
    SampleSet smp;
    float* smp_out;        // [npts] for this step, or nullptr
    // injected nodes lie in planes [inj_x0, inj_x1] and rows [inj_y0, inj_y1]
    // (empty when inj_x1 < inj_x0): blocks outside skip injection without a
    // memory lookup
    int64_t inj_x0, inj_x1, inj_y0, inj_y1;
    int64_t stencil_blocks;
    // streaming-kernel tiling (set by the launcher): tiles along z and y,
    // x-chunk length, and whether the single-shot grid pads its tile part to
    // a multiple of 8 and remaps block ids so that consecutive tiles land on
    // the same XCD
    int32_t ntz, nty, xchunk, remap;
    // imaging condition (adjoint with gradient): g -= fwd * (other - 2 cur + out) / dt^2
    const float* img_fwd;  // u^k, or nullptr
    float* img_grad;
    float inv_dt2;
    // 1 when beta is zero everywhere (forward-Euler diffusion): the step then
    // reads neither `other` nor beta (12 instead of 20 bytes per update); the
    // update is unchanged, since beta (cur - other) is then zero
    int32_t no_prev;
};

// One shot of a batched launch: the static step arguments plus the base
// pointers that the step index selects from.
struct ShotDesc {
    StepArgs a;          // cur/other/out/inj_val/smp_out are set per step
    float* buf[4];       // wavefield pair: even steps read buf[0], odd steps buf[1];
                         // the two-step slab (2D) rotates through all four
    const float* q;      // [nt][nsrc]
    float* d;            // [nt][nrec] or nullptr
    int32_t nsrc, nrec;
};

// Tile configuration of the streaming kernel: block shape variant and x-chunk
// length (0 = chosen from the grid).  Public tile id: (variant << 16) | xchunk.
struct TileCfg {
    int variant = 0;
    int xchunk = 0;
};
inline TileCfg tile_from_id(int id) { TileCfg c; c.variant = (id >> 16) & 0xff; c.xchunk = id & 0xffff; return c; }
inline int tile_id(const TileCfg& c) { return (c.variant << 16) | c.xchunk; }

// Size of the device array that serves as the workspace of
// wave_forward_noalloc, and how many devices' addresses of it are kept.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
// Device address of that array on the current device (looked up once per
// device with hipGetSymbolAddress).
hipError_t noalloc_scratch(void** ptr);

// Rows of u^n a 2D slab block computes at most (its x-chunk); the LDS slab
// holds them with R halo rows on either side.
constexpr int kSlabRows = 16;
// The two-step body (2D tile variant kTwoStepVariant, batched shots only):
// the default column length and the threads per block (eight waves, one per
// row of a round of its walk along the column).
constexpr int kSlab2Column = 64;
constexpr int kSlab2Threads = 512;
constexpr int kTwoStepVariant = 4;

// Block shapes of the step kernel: z-points per lane, lanes along z and rows
// along y (2D: rows along x, computed by the slab body when > 1).
//   2D: one wave with four z-points per lane (256 z), 128 scalar lanes
//   (128 z), one wave with two z-points per lane (128 z), or the slab body
//   with eight waves of four-point lanes (256 z, chunks of up to 16 rows held
//   in LDS, two rows per wave; measured against four waves with four rows
//   each: 167 us against 170 us on the 48 batched shots, and 172 us for the
//   streaming body).
//   3D, four z-points per lane: 64 z x 16 rows, 64 z x 8 rows, 32 z x 32
//   rows, 100 z x 10 rows or 200 z x 5 rows (the last two cover grids such as
//   200^3 without a mostly empty last tile); two z-points per lane: 64 z x 8
//   rows (half the queue registers per lane).  Taller tiles for the high
//   orders, where the y halo (R rows on either side) is as large as a 16-row
//   tile: 64 z x 32 rows (four points per lane), 64 z x 16 and 64 z x 32 rows
//   (two points per lane), 128 z x 16 rows (four and two points per lane).
struct BlockShape {
    int vz, tzl, ty;
};
constexpr BlockShape kShapes2D[] = {{4, 64, 1}, {1, 128, 1}, {2, 64, 1}, {4, 64, 8}};
constexpr BlockShape kShapes3D[] = {{4, 16, 16}, {4, 16, 8}, {4, 8, 32}, {4, 25, 10}, {4, 50, 5},
                                    {2, 32, 8},  {4, 16, 32}, {2, 32, 16}, {2, 32, 32}, {4, 32, 16},
                                    {2, 64, 16}};

// The step kernels of one space order O (defined in wave_step.h, instantiated
// in wave_o<O>.hip); the launch_* functions below dispatch to them.
template <int O>
struct OrderOps {
    static int64_t plan(int ndim, TileCfg cfg, StepArgs& a, bool device);
    static hipError_t step(int ndim, const StepArgs& a, hipStream_t s, TileCfg cfg);
    static hipError_t batch(int ndim, int64_t nz_any, TileCfg cfg, const ShotDesc* shots,
                            const int64_t* begin, int32_t nshots, int64_t blocks, int32_t n,
                            hipStream_t s);
    static hipError_t batch2(const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                             int64_t blocks, int32_t n, int32_t bufs, int32_t flags, hipStream_t s);
    static hipError_t persistent(int ndim, int64_t nz_any, TileCfg cfg, const ShotDesc* shots,
                                 const int64_t* begin, int32_t nshots, int64_t items, int32_t nt,
                                 unsigned int* sync, int32_t spin_limit, int* grid_used,
                                 hipStream_t s);
    static hipError_t persistent_graph(int ndim, int64_t nz_any, TileCfg cfg,
                                       const ShotDesc* shots, const int64_t* begin,
                                       int32_t nshots, int64_t items, int32_t nt,
                                       unsigned int* sync, int32_t spin_limit, int* grid_used,
                                       hipGraph_t* graph);
};

// Number of single-step block-shape variants for a grid (2D: 4, 3D: 11; the
// row length handed to the kernels is always a multiple of 4).  Batched 2D
// shots also accept kTwoStepVariant.
int tile_variants(int ndim, int64_t nz);
// Longest x-chunk a block shape accepts (the 2D slab holds at most 16 rows;
// the streaming shapes have no limit below the grid).
int max_xchunk(int ndim, int variant);
// Block shape used when no tile is given or cached: in 2D the slab body; in
// 3D the one whose tiles waste the fewest lanes on the (ny, nz) plane, ties
// broken by a measured preference order that depends on the space order.
int default_variant(int ndim, int order, int64_t ny, int64_t nz);
// Fill the tiling fields of `a` (ntz, nty, xchunk, stencil_blocks, remap) for
// `cfg`; returns the block count of one launch including receiver samplers.
// With `device` the plan is the one a single-shot launch on the current
// device makes (x-chunks from the kernel's occupancy); without, the
// occupancy-free plan of the many-shot launches.
int64_t plan_tiles(int ndim, int order, TileCfg cfg, StepArgs& a, bool device = false);

// Launch one time step of the 2.5D streaming kernel (plans `a` for cfg).
hipError_t launch_step(int ndim, int order, const StepArgs& a, hipStream_t s, TileCfg cfg);
// One step of every shot in one launch; every shot must be planned with the
// same cfg; `begin` holds the first block of each shot and the total.
hipError_t launch_batch(int ndim, int order, int64_t nz_any, TileCfg cfg, const ShotDesc* shots,
                        const int64_t* begin, int32_t nshots, int64_t blocks, int32_t n,
                        hipStream_t s);
// Two steps of every shot in one launch (2D, tile variant kTwoStepVariant,
// shots planned with it): n, bufs and flags as k_step_batch2 documents them.
hipError_t launch_batch2(int order, const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                         int64_t blocks, int32_t n, int32_t bufs, int32_t flags, hipStream_t s);
// All nt steps of all shots in one cooperative (co-resident) launch with a
// device-wide barrier per step.  `sync` = {arrival counter, error word}, both
// zero at launch; the error word is set if a barrier wait exceeded
// `spin_limit` polls.  The grid is as many blocks as the kernel's occupancy
// lets every CU hold at once (never more than `items`); the cooperative
// launch is refused rather than run with fewer resident.  *grid_used
// receives the number of blocks.
hipError_t launch_batch_persistent(int ndim, int order, int64_t nz_any, TileCfg cfg,
                                   const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                                   int64_t items, int32_t nt, unsigned int* sync, int32_t spin_limit,
                                   int* grid_used, hipStream_t s);
// The same persistent kernel as a graph: a kernel node that zeroes `sync`
// followed by the persistent kernel as a node with the cooperative launch
// attribute (co-resident grid, sized by the kernel's occupancy).  *graph is
// created here and owned by the caller.
hipError_t graph_batch_persistent(int ndim, int order, int64_t nz_any, TileCfg cfg,
                                  const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                                  int64_t items, int32_t nt, unsigned int* sync, int32_t spin_limit,
                                  int* grid_used, hipGraph_t* graph);
// One pass over the model: per block {min m, min eta, count of invalid values}
// into `partial` (3 * nblocks floats) for the host-side validation, and the
// step coefficients alpha = dt^2/(m + eta dt/2), beta = (m - eta dt/2)/(m + eta dt/2).
// m and eta are [rows][nz]; alpha and beta are written as [rows][nzp] with
// zeros in the padding columns nz <= z < nzp.
hipError_t launch_check_fields(const float* m, const float* eta, int64_t rows, int64_t nz,
                               int64_t nzp, float* partial, int nblocks, float* alpha, float* beta,
                               double dt, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);
// ev[e] = ent[e].w * val[ent[e].pt] for e < nent (the first step of a
// gathered injection).
hipError_t launch_gather(float* ev, const float* val, const InjEntry* ent, int32_t nent, hipStream_t s);
// Diffusion coefficients alpha = dt a, beta = 0 and per block {max a, invalid count}
// into `partial` (2 * nblocks floats); a is [rows][nz], alpha and beta [rows][nzp].
hipError_t launch_diffusion_coef(const float* a, int64_t rows, int64_t nz, int64_t nzp,
                                 float* partial, int nblocks, float* alpha, float* beta, double dt,
                                 hipStream_t s);
// Reduced-precision checkpoint of (cur, prev): stores cur and cur - prev as
// BF16 (bf16 != 0) or FP16 with per-array power-of-two scales kept in `slot`
// (4 words: scale_u, scale_d, max|u| and max|d| bits).  The maxima go
// through `partial` (2 * nblocks floats of scratch, at most nblocks blocks)
// and a one-block pass, without atomics.  n is a multiple of 4 (fields use
// padded rows); four values per thread, 8-byte stores.
hipError_t launch_ckpt_encode(const float* cur, const float* prev, int64_t n, int bf16,
                              unsigned int* slot, float* partial, int nblocks,
                              unsigned short* out_u, unsigned short* out_d, hipStream_t s);
hipError_t launch_ckpt_decode(const unsigned short* in_u, const unsigned short* in_d,
                              const unsigned int* slot, int64_t n, int bf16, float* cur, float* prev,
                              hipStream_t s);
// r = d - dobs over n values and misfit[0] = 1/2 sum r^2 (deterministic two-pass
// reduction through `partial`, which holds nblocks floats).
hipError_t launch_residual(const float* d, const float* dobs, float* r, int64_t n, float* partial,
                           int nblocks, float* misfit, hipStream_t s);

}  // namespace wave
