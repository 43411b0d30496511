/*
 * wave.h — C ABI of the MI355X damped-acoustic finite-difference propagator.
 *
 * The method is the explicit scheme of the paper's seismic-inversion example
 * (Section "Seismic Inversion Example", equation "eqn:acoustic"):
 *
 *     m u_tt + eta u_t - lap(u) = q
 *
 * second order in time (central differences for u_tt and u_t), order 2..16
 * in space (Section "High-level API": u.laplace is the sum over axes of the
 * order-2k central second derivative), solved for the next time level as in
 * the forward listing ("lst:wave"):
 *
 *     u^{n+1} = (2 m u^n - (m - eta dt/2) u^{n-1} + dt^2 L u^n) / (m + eta dt/2)
 *
 * Sources are injected and receivers sampled by multilinear interpolation
 * over the 2^d nodes of the enclosing cell (Section "Sparse point
 * interpolation"): step n samples d^n from u^n and adds
 * dt^2 q^n w / (m + eta dt/2) to u^{n+1}.  Outside the grid the field is
 * zero.  The adjoint ("lst:adjoint") runs the same update backwards in time
 * with the roles of sources and receivers exchanged.
 *
 * Conventions for every entry point
 *   - Layout: C-contiguous, depth z fastest.  2D fields are [nx][nz], 3D
 *     fields [nx][ny][nz]; traces and wavelets are time-major [nt][npts].
 *   - Field, trace, wavelet, gradient and workspace pointers are DEVICE
 *     pointers (FP32 unless stated).  Coordinates are HOST FP64 [npts][ndim],
 *     metres from grid index 0, and are copied during the call.
 *   - The caller owns every buffer, including the workspace; the library
 *     allocates no device memory.  Buffers must not overlap unless stated.
 *   - Validation is synchronous and happens before any write to an output:
 *     on a non-zero return no output has been touched.  Validation reads
 *     m and eta on `stream` and waits for it once per call.  After that the
 *     work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns; faults surface at the caller's next synchronise.
 *   - Return codes are the wave_status values below; wave_last_error() gives
 *     a thread-local message for the last non-zero return.  Nothing throws
 *     or aborts across this interface.
 *   - Calls that share a workspace must be ordered on one stream.
 */
#ifndef WAVE_H
#define WAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WAVE_OK = 0,
    WAVE_EINVAL = -1,     /* bad argument: null pointer, ndim, order, nt, shape, dt, fields */
    WAVE_ECFL = -2,       /* dt above the stability bound of the scheme */
    WAVE_ERANGE = -3,     /* a sparse point lies outside [0, (n_a - 1) h_a] on some axis */
    WAVE_EWORKSPACE = -4, /* workspace missing, misaligned or too small */
    WAVE_EHIP = -5        /* the HIP runtime reported an error */
} wave_status;

/* Grid and time axis.  Section "High-level API" (space_order on the symbol,
 * u.laplace) and the listings' problem statement forward(model, nt, dt, h,
 * order).  2D: shape = {nx, nz, 0}, spacing = {hx, hz, 0}. */
typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t space_order;   /* 2, 4, ..., 16 */
    int64_t shape[3];      /* points per axis, each >= 2 */
    double spacing[3];     /* metres, > 0 */
    double dt;             /* seconds, > 0 */
    int32_t nt;            /* time steps, >= 1 */
    int32_t reserved;      /* set to 0 */
} wave_grid;

/* Sparse points (Section "Sparse point interpolation"). */
typedef struct {
    int32_t npts;          /* >= 0 */
    int32_t reserved;      /* set to 0 */
    const double* coords;  /* HOST [npts][ndim], metres; may be NULL when npts == 0 */
} wave_points;

typedef enum { WAVE_CKPT_FP32 = 0, WAVE_CKPT_BF16 = 1, WAVE_CKPT_FP16 = 2 } wave_ckpt_dtype;

/* Per-call options.  A zero-initialised struct plus a workspace is valid. */
typedef struct {
    void* workspace;          /* DEVICE, 256-byte aligned, >= wave_workspace_size() bytes */
    size_t workspace_bytes;
    int32_t ckpt_every;       /* gradient/checkpointing: steps per segment, 0 = 20 */
    int32_t ckpt_dtype;       /* wave_ckpt_dtype for stored snapshots */
    int32_t tile;             /* 0 = tuned if wave_tune has seen this grid, else automatic;
                                 > 0 = explicit tile id (variant << 16 | x-chunk planes, 0 =
                                 planned).  Variants (block shapes, z x rows of the (y, z)
                                 plane): 2D 0 = 256 z (4 per lane), 1 = 128 z (1 per lane),
                                 2 = 128 z (2 per lane), 3 = 256 z with x-chunks of at most
                                 16 rows held in LDS, 4 (wave_forward_batch, where it is
                                 the 2D default, and wave_forward without checkpoints,
                                 which then runs as a batch of one shot) = two time
                                 steps per pass over columns of x-chunk rows, 64 when
                                 planned (temporal blocking, 256 - 2 ceil4(R) owned z per
                                 block, see wave_forward_batch); 3D 0 = 64 x 16, 1 = 64 x 8,
                                 2 = 32 x 32, 3 = 100 x 10, 4 = 200 x 5 (4 z-points per
                                 lane), 5 = 64 x 8 (2 per lane), 6 = 64 x 32 (4 per lane),
                                 7 = 64 x 16, 8 = 64 x 32 (2 per lane), 9 = 128 x 16
                                 (4 per lane), 10 = 128 x 16 (2 per lane).  An unknown
                                 variant or a negative id is WAVE_EINVAL.  Results do not
                                 depend on it. */
    int32_t flags;            /* WAVE_FLAG_* bits */
} wave_opts;

#define WAVE_FLAG_NO_GRAPH 1    /* batch: launch directly instead of replaying a hipGraph */
#define WAVE_FLAG_PERSISTENT 2  /* batch: one persistent co-resident launch for all steps (see below) */
#define WAVE_FLAG_TUNE_IMAGING 4 /* wave_tune (and the workspace size of WAVE_OP_FORWARD): time
                                    the adjoint step with the imaging condition instead of the
                                    plain step; the result is cached for that kernel only.
                                    wave_tune runs without injected or sampled points, so a
                                    dense receiver set (the gradient's adjoint injects every
                                    receiver each step) can make its winner slower there than
                                    the planned tile; wave_tune_shot times the step with the
                                    shot's points. wave_tune_shot: the workspace is that of
                                    WAVE_OP_ADJOINT with this flag, else of WAVE_OP_FORWARD */

typedef enum {
    WAVE_OP_FORWARD = 0,      /* wave_forward without checkpoints, wave_diffusion, wave_tune */
    WAVE_OP_ADJOINT = 1,      /* wave_adjoint */
    WAVE_OP_GRADIENT = 2,     /* wave_gradient (includes the checkpoint storage) */
    WAVE_OP_FORWARD_CKPT = 3, /* wave_forward writing caller-owned checkpoints */
    WAVE_OP_BACKWARD = 4,     /* wave_backward (replay ring, adjoint pair, gradient accumulator) */
} wave_op;

/* Bytes of workspace an entry point needs for this grid and point sets
 * (checkpoint storage is separate: wave_checkpoint_size).  Fields inside the
 * workspace and the checkpoints use rows of nz rounded up to a multiple of 4
 * points; caller arrays never do.  Returns a wave_status; *bytes is written
 * on success. */
int wave_workspace_size(int32_t op, const wave_grid* grid, const wave_points* src,
                        const wave_points* rec, const wave_opts* opts, size_t* bytes);

/* Bytes of checkpoint storage for opts->ckpt_every / opts->ckpt_dtype.  One
 * checkpoint per segment of ckpt_every steps: FP32 keeps the pair (u^c,
 * u^{c-1}) exactly, so the backward replay is bitwise the forward run; BF16
 * and FP16 keep u^c and the increment u^c - u^{c-1}, each scaled by its own
 * power of two (largest magnitude mapped into [2^14, 2^15)) and rounded to
 * nearest even, so the replayed velocity carries one rounding of the
 * increment rather than of two nearly equal states. */
int wave_checkpoint_size(const wave_grid* grid, const wave_opts* opts, size_t* bytes);

/*
 * Forward modelling (listing "lst:wave" plus point-to-grid injection and
 * grid-to-point sampling).
 *   m      [shape]  squared slowness 1/v^2 (s^2/m^2), finite, > 0
 *   eta    [shape]  damping (s/m^2), finite, >= 0; NULL means eta = 0
 *   src, q          source positions and wavelets q [nt][nsrc]
 *   rec, d          receiver positions and traces d [nt][nrec] (written; d^n from u^n)
 *   u_final         NULL or [shape]: receives u^nt
 *   ckpt            NULL, or DEVICE checkpoint storage of at least
 *                   wave_checkpoint_size() bytes for the same opts->ckpt_every
 *                   and ckpt_dtype (the library cannot check its size):
 *                   receives the snapshots that wave_backward replays
 * Workspace: op WAVE_OP_FORWARD, or WAVE_OP_FORWARD_CKPT when ckpt is given.
 * In 2D without ckpt, an explicit tile of variant 4 runs the call as a batch
 * of one shot on the two-step body (wave_forward_batch, whose rules and
 * errors then apply; the 2D forward workspace covers it).  The result is
 * bitwise the same.
 */
int wave_forward(const wave_grid* grid, const float* m, const float* eta,
                 const wave_points* src, const float* q,
                 const wave_points* rec, float* d,
                 float* u_final, void* ckpt, const wave_opts* opts, void* stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * forward modelling as wave_forward without checkpoints and with the tuned or
 * default tile, bitwise the same results, but the workspace is a device array
 * of WAVE_NOALLOC_WORKSPACE_BYTES that the library holds on every device it
 * runs on until the process ends.  The call makes no device allocation and
 * pins no host memory (no hipMalloc, hipHostMalloc or hipFree; its host-side
 * tables use ordinary heap memory).  A grid and point set whose forward
 * workspace (wave_workspace_size, op WAVE_OP_FORWARD) exceeds that size is
 * rejected with WAVE_EWORKSPACE before anything runs.  Every call on one
 * device uses the same array: calls on one device must be ordered on one
 * stream (or synchronised); overlapping calls race.  Each call initialises
 * everything it reads from the array.
 */
#define WAVE_NOALLOC_WORKSPACE_BYTES (64u << 20)
int wave_forward_noalloc(const wave_grid* grid, const float* m, const float* eta,
                         const wave_points* src, const float* q,
                         const wave_points* rec, float* d, float* u_final, void* stream);

/*
 * Adjoint modelling (listing "lst:adjoint": the eta term enters with the
 * opposite sign and the update is solved for the backward level).  Driven by
 * receiver data, sampled at the sources; it is the exact transpose of the
 * map q -> d of wave_forward:
 *   for k = nt-1 .. 0:  q_adj^k = sample of v^k at the sources,
 *                       v^{k-1} = update(v^k, v^{k+1}) + dt^2 d^k w / (m + eta dt/2)
 *   d      [nt][nrec]  adjoint source
 *   q_adj  [nt][nsrc]  written
 *   v_final NULL or [shape]: receives v^0
 */
int wave_adjoint(const wave_grid* grid, const float* m, const float* eta,
                 const wave_points* rec, const float* d,
                 const wave_points* src, float* q_adj,
                 float* v_final, const wave_opts* opts, void* stream);

/*
 * Adjoint-state backward pass from stored checkpoints.  For the data map
 * d = F(m, q) of wave_forward and an adjoint source r = dJ/dd [nt][nrec]:
 *   grad_m [shape]      written: dJ/dm = -sum_n v^n (u^{n+1} - 2u^n + u^{n-1}) / dt^2
 *                       with v the adjoint field driven by r (eta held fixed)
 *   grad_q [nt][nsrc]   NULL or written: dJ/dq (the adjoint sampled at the sources)
 * `ckpt` must come from wave_forward with the same grid, fields, sources,
 * wavelets and opts->ckpt_every/ckpt_dtype.  Workspace: op WAVE_OP_BACKWARD.
 */
int wave_backward(const wave_grid* grid, const float* m, const float* eta,
                  const wave_points* src, const float* q,
                  const wave_points* rec, const float* r,
                  const void* ckpt, float* grad_m, float* grad_q,
                  const wave_opts* opts, void* stream);

/*
 * Misfit and gradient for one shot (the gradient test of Section
 * "Performance" of the seismic example): forward with checkpoints, residual
 * r = d - d_obs, J = 1/2 sum r^2, then wave_backward(r).
 *   d_obs  [nt][nrec]
 *   grad   [shape]   written, dJ/dm
 *   misfit DEVICE    one float, written: J
 *   d_syn  NULL or [nt][nrec]: receives the modelled data
 * The workspace (op WAVE_OP_GRADIENT) includes the checkpoint storage.
 */
int wave_gradient(const wave_grid* grid, const float* m, const float* eta,
                  const wave_points* src, const float* q,
                  const wave_points* rec, const float* d_obs,
                  float* grad, float* misfit, float* d_syn,
                  const wave_opts* opts, void* stream);

/*
 * Many shots at once (the paper's remark that an inversion workflow runs many
 * operators in parallel, Section "Discussion"): every shot is forward
 * modelled exactly as by wave_forward, but step n of all shots runs in one
 * launch over a flattened list of (shot, tile, x-chunk) blocks, and the nt
 * launches are captured once into a hipGraph that is replayed (and reused by
 * later calls with the same buffers).  Shots may differ in shape, spacing,
 * fields and points; they must share ndim, space_order, nt and dt.  Each
 * shot's results are bitwise those of wave_forward on the same shot.
 */
typedef struct {
    wave_grid grid;
    const float* m;           /* [shape] */
    const float* eta;         /* [shape] or NULL */
    wave_points src;
    const float* q;           /* [nt][nsrc] */
    wave_points rec;
    float* d;                 /* [nt][nrec], written */
    float* u_final;           /* NULL or [shape]: receives u^nt */
} wave_shot;

int wave_batch_workspace_size(int32_t nshots, const wave_shot* shots, const wave_opts* opts,
                              size_t* bytes);
/* 2D tile variant 4 (temporal blocking, Section "Loop Blocking" applied to
 * time as well; the default for 2D batches): each launch advances every
 * shot by two steps.  A block walks a column of x-chunk rows eight rows at a
 * time, computing level n+1 on its rows and R rows beyond them (and on its z
 * widened by ceil4(R)) and level n+2 on its own points, from one read of
 * u^n, u^{n-1}, alpha and beta.  The passes read one wavefield pair and
 * write the other, so the workspace of a 2D batch holds four wavefields per
 * shot; an odd nt starts with one step, and the receivers of level n-1 are
 * sampled by the pass that reads it.  Results are bitwise those of the
 * one-step variants.  With WAVE_FLAG_PERSISTENT the variant maps to 3 (the
 * persistent kernel takes one step at a time). */
/* With opts->flags & WAVE_FLAG_PERSISTENT the whole time loop of all shots is
 * one cooperative launch (all its blocks are resident at once; the grid is
 * what the kernel's occupancy allows), with a device-wide barrier between
 * steps.  By default that launch is the cooperative kernel node of a hipGraph
 * (built once and reused like the per-step graph); with WAVE_FLAG_NO_GRAPH as
 * well it is a direct cooperative launch.  The persistent mode waits for the
 * launch before returning and reports WAVE_EHIP if a barrier wait ever
 * exceeded its bound (every wait is bounded, so the launch always ends).
 * In every mode the blocks of the larger shots come first in the flattened
 * list; the order does not change any result. */
int wave_forward_batch(int32_t nshots, const wave_shot* shots, const wave_opts* opts, void* stream);
/* How this thread's last wave_forward_batch ran: 0 per-step launches replayed
 * from a hipGraph, 1 per-step launches, 2 one persistent launch, 3 one
 * persistent launch replayed from a hipGraph; -1 if none yet. */
int wave_last_batch_mode(void);

/*
 * Tile autotuner (the paper's brute-force search over loop-blocking sizes,
 * Section "Loop Blocking"): times every candidate tile of the step kernel
 * (block shape x x-chunk length) for `steps` launches on this grid (or batch)
 * using the workspace (size of WAVE_OP_FORWARD, resp. the batch), keeps the
 * fastest in a process-wide cache that calls with opts->tile == 0 consult
 * (mirrored to the file named by the environment variable WAVE_TUNE_CACHE),
 * and returns its id and its time per step in microseconds.  Candidates give
 * bitwise identical results; no output buffer is written.  With the
 * environment variable WAVE_TUNE_VERBOSE set, every candidate's time is
 * printed to stderr.
 */
int wave_tune(const wave_grid* grid, const wave_opts* opts, int32_t steps, void* stream,
              int32_t* tile, double* us_per_step);
int wave_tune_batch(int32_t nshots, const wave_shot* shots, const wave_opts* opts, int32_t steps,
                    void* stream, int32_t* tile, double* us_per_step);
/* The same search on one shot's own step: the model m/eta (device, as for
 * wave_forward) and both point sets (host) are set up as a forward run sets
 * them up, and every candidate launch injects the sources and samples the
 * receivers, or with WAVE_FLAG_TUNE_IMAGING runs the adjoint step with the
 * imaging condition, injecting the receivers and sampling the sources.  The
 * injected values are zeros and the samples go to a buffer of the tuner's
 * own (allocated and freed inside the call): the injection and sampling work
 * is that of a real step, their values do not change a launch's time.
 * Workspace: op WAVE_OP_FORWARD, or WAVE_OP_ADJOINT with
 * WAVE_FLAG_TUNE_IMAGING set in opts->flags, sized with the same points.
 * The winner is cached like wave_tune's; no caller buffer is written.  Like
 * wave_tune it relaunches the step on the same fields, which stay in the
 * last-level cache when they fit: its times are then lower than those of a
 * run that streams other fields between steps (the gradient's replay), and
 * its ranking of close candidates can differ from theirs. */
int wave_tune_shot(const wave_grid* grid, const float* m, const float* eta, const wave_points* src,
                   const wave_points* rec, const wave_opts* opts, int32_t steps, void* stream,
                   int32_t* tile, double* us_per_step);

/* The tile ids wave_tune times on this grid, in order: every block shape with
 * x-chunks of 2R, 4R, 8, 16, ..., 128 planes and of every split of the grid
 * into 2 .. 32 chunks, each clamped to what the shape accepts and to the
 * grid, so no two ids launch the same thing.  Writes up
 * to `cap` ids into `ids` and the number of candidates into *n.  Host only. */
int wave_tile_candidates(const wave_grid* grid, int32_t* ids, int32_t cap, int32_t* n);
/* The tile a step launch on this grid uses for the requested id (0 = the
 * tuned or default one): its block shape and its x-chunk after clamping and
 * planning.  For an x-chunk of 0, the plan depends on the kernel's occupancy
 * on the current device; without a device the occupancy-free plan is
 * returned. */
int wave_resolve_tile(const wave_grid* grid, int32_t tile, int32_t* resolved);

/*
 * Diffusion (Section "2D Diffusion Example", equation "eqn:diffusion"):
 * u_t = a lap(u) with forward Euler in time, the same order-2k Laplacian and
 * zero outside the grid, on the same step kernel (u^{n+1} = u^n + dt a L u^n).
 *   a       [shape]  diffusion coefficient, finite, >= 0
 *   u0      [shape]  initial state
 *   u_final [shape]  receives u^nt
 * Returns WAVE_ECFL when dt a_max max|lambda(L)| > 2.  Workspace: the size of
 * WAVE_OP_FORWARD with no points.
 */
int wave_diffusion(const wave_grid* grid, const float* a, const float* u0, float* u_final,
                   const wave_opts* opts, void* stream);

/*
 * Misfit of modelled against observed data (the objective of the gradient
 * test, Section "Performance" of the seismic example): r = d - d_obs and
 * J = 1/2 sum r^2, summed in a fixed order (per-block partial sums, then one
 * block), so the result is run-to-run reproducible.
 *   d, d_obs  DEVICE [n] FP32
 *   r         NULL or DEVICE [n]: receives the residual
 *   misfit    DEVICE, one float: receives J
 *   opts      workspace of at least WAVE_MISFIT_WORKSPACE_BYTES bytes (partials)
 */
#define WAVE_MISFIT_WORKSPACE_BYTES 4096
int wave_misfit(const float* d, const float* d_obs, int64_t n, float* r, float* misfit,
                const wave_opts* opts, void* stream);

/* Phase timing (a metrics aid).  With profiling on, each entry point called
 * by this thread records HIP events on its stream around its time loop(s),
 * from the first step launch to the last (set-up excluded).
 * wave_last_loop waits for the last call's end event and reports the
 * elapsed milliseconds and the number of step launches it made. */
int wave_set_profiling(int32_t enable);
int wave_last_loop(double* ms, int64_t* launches);

/* Releases what the library keeps for the calling thread: the last
 * instantiated batch graph and its capture stream, the timing events and the
 * pinned host staging buffer (after its last copy has finished).  Later calls
 * recreate them on demand.  Call it before the HIP runtime shuts down (the
 * Python binding does so at interpreter exit); returns WAVE_EHIP if the
 * runtime refused a release. */
int wave_release(void);

/* Thread-local message describing the last non-zero return ("" if none). */
const char* wave_last_error(void);

/* Library version string. */
const char* wave_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WAVE_H */
