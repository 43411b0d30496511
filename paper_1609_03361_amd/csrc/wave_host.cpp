// Host side of the C ABI declared in include/wave.h: argument validation,
// finite-difference weights, stability bound, sparse-point tables, workspace
// layout and the time loops that enqueue the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wave.h"
#include "wave_internal.h"

using namespace wave;

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(WAVE_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                          \
    } while (0)

// Per-thread state: phase timing (wave_set_profiling / wave_last_loop), the
// pinned host staging buffer for the per-call uploads and the validation
// read-back, the last instantiated batch graph with its capture stream, and
// the mode of the last batched call.  Every thread's state is registered so
// that wave_release can destroy the HIP objects of all of them (torch runs
// the autograd backward on a thread of its own).  The small host structs are
// never freed.
struct Prof {
    bool on = false;
    bool have = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int64_t launches = 0;
};

// Staging: grown on demand; an event marks the last use so that the buffer is
// never rewritten while a copy reads it.
struct Staging {
    char* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipStream_t capture = nullptr;
    std::vector<char> key;
};

struct ThreadState {
    Prof prof;
    Staging stage;
    GraphCache graph;
    // How the last batched call ran: 0 = per-step launches replayed from a
    // hipGraph, 1 = per-step launches, 2 = one persistent launch, 3 = one
    // persistent launch replayed from a hipGraph.
    int batch_mode = -1;
};

std::mutex g_threads_mu;
std::vector<ThreadState*> g_threads;

ThreadState& TS()
{
    thread_local ThreadState* st = nullptr;
    if (!st) {
        st = new ThreadState;
        std::lock_guard<std::mutex> lk(g_threads_mu);
        g_threads.push_back(st);
    }
    return *st;
}

int prof_begin(hipStream_t s)
{
    TS().prof.launches = 0;
    TS().prof.have = false;
    if (!TS().prof.on) return 0;
    if (!TS().prof.t0 && hipEventCreate(&TS().prof.t0) != hipSuccess) return -1;
    if (!TS().prof.t1 && hipEventCreate(&TS().prof.t1) != hipSuccess) return -1;
    return hipEventRecord(TS().prof.t0, s) == hipSuccess ? 0 : -1;
}

int prof_end(hipStream_t s)
{
    if (!TS().prof.on) return 0;
    if (hipEventRecord(TS().prof.t1, s) != hipSuccess) return -1;
    TS().prof.have = true;
    return 0;
}

constexpr size_t kAlign = 256;
constexpr int kCheckBlocks = 2048;
constexpr int kRedFloats = 1024;   // reduction scratch: misfit partials, checkpoint maxima

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Grid description
// ---------------------------------------------------------------------------
struct Geo {
    int ndim = 0, order = 0, half = 0, nt = 0;
    int64_t n[3] = {0, 0, 0};     // 3D view: (nx, ny, nz); 2D: (nx, 1, nz)
    double h[3] = {0, 0, 0};      // spacing in the 3D view (2D: hy unused)
    double dt = 0;
    // Fields inside the library (coefficients, wavefields, checkpoints,
    // gradient accumulator) use rows of nzp = nz rounded up to a multiple of
    // 4, so that every row starts 16-byte aligned and the step kernel can
    // load four z-points per lane.  The padding points hold alpha = beta = 0
    // and wavefield values 0, which the update keeps at 0, so to the stencil
    // they are the zero halo outside the grid.  Caller arrays are unpadded.
    int64_t nzp = 0;
    int64_t npts() const { return n[0] * n[1] * n[2]; }
    int64_t npad() const { return n[0] * n[1] * nzp; }
    int64_t nrows() const { return n[0] * n[1]; }
};

int make_geo(const wave_grid* g, Geo* G)
{
    if (!g) return fail(WAVE_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(WAVE_EINVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->space_order < 2 || g->space_order > 16 || (g->space_order & 1))
        return fail(WAVE_EINVAL, "space_order must be even in [2, 16] (got %d)", g->space_order);
    if (g->nt < 1) return fail(WAVE_EINVAL, "nt must be >= 1 (got %d)", g->nt);
    if (!(g->dt > 0.0) || !std::isfinite(g->dt)) return fail(WAVE_EINVAL, "dt must be finite and > 0");
    for (int a = 0; a < g->ndim; ++a) {
        if (g->shape[a] < 2) return fail(WAVE_EINVAL, "shape[%d] must be >= 2", a);
        if (g->shape[a] > (int64_t)1 << 31) return fail(WAVE_EINVAL, "shape[%d] too large", a);
        if (!(g->spacing[a] > 0.0) || !std::isfinite(g->spacing[a]))
            return fail(WAVE_EINVAL, "spacing[%d] must be finite and > 0", a);
    }
    G->ndim = g->ndim;
    G->order = g->space_order;
    G->half = g->space_order / 2;
    G->nt = g->nt;
    G->dt = g->dt;
    if (g->ndim == 3) {
        for (int a = 0; a < 3; ++a) { G->n[a] = g->shape[a]; G->h[a] = g->spacing[a]; }
    } else {
        G->n[0] = g->shape[0]; G->n[1] = 1; G->n[2] = g->shape[1];
        G->h[0] = g->spacing[0]; G->h[1] = 1.0; G->h[2] = g->spacing[1];
    }
    G->nzp = (G->n[2] + 3) / 4 * 4;
    const double total = (double)G->n[0] * (double)G->n[1] * (double)G->nzp;
    if (total > 4.0e10) return fail(WAVE_EINVAL, "grid has too many points");
    if ((double)G->n[0] * (double)G->n[1] >= 2147483647.0)
        return fail(WAVE_EINVAL, "nx * ny must be below 2^31");
    if ((double)G->n[1] * (double)G->nzp >= 2147483647.0)
        return fail(WAVE_EINVAL, "ny * nz must be below 2^31");
    return WAVE_OK;
}

// Caller arrays [rows][nz] <-> library fields [rows][nzp].
hipError_t copy_out(float* dst, const float* src, const Geo& G, hipStream_t s)
{
    if (G.nzp == G.n[2])
        return hipMemcpyAsync(dst, src, (size_t)G.npts() * 4, hipMemcpyDeviceToDevice, s);
    return hipMemcpy2DAsync(dst, (size_t)G.n[2] * 4, src, (size_t)G.nzp * 4, (size_t)G.n[2] * 4,
                            (size_t)G.nrows(), hipMemcpyDeviceToDevice, s);
}

// The padding of dst must already be zero.
hipError_t copy_in(float* dst, const float* src, const Geo& G, hipStream_t s)
{
    if (G.nzp == G.n[2])
        return hipMemcpyAsync(dst, src, (size_t)G.npts() * 4, hipMemcpyDeviceToDevice, s);
    return hipMemcpy2DAsync(dst, (size_t)G.nzp * 4, src, (size_t)G.n[2] * 4, (size_t)G.n[2] * 4,
                            (size_t)G.nrows(), hipMemcpyDeviceToDevice, s);
}

// Central second-derivative weights of order 2k (Section "High-level API":
// f.dx2 with space_order = 2k), closed form
//   c_j = 2 (-1)^(j+1) (k!)^2 / (j^2 (k-j)! (k+j)!),  j = 1..k,
// evaluated as an exact integer ratio in double (every factor < 2^53 for
// k <= 8), so each c_j is the correctly rounded value.
void fd_weights(int k, double* c)
{
    auto fact = [](int v) { double f = 1; for (int i = 2; i <= v; ++i) f *= i; return f; };
    const double kf = fact(k);
    for (int j = 1; j <= k; ++j) {
        const double num = 2.0 * kf * kf;
        const double den = (double)j * j * fact(k - j) * fact(k + j);
        c[j] = ((j & 1) ? 1.0 : -1.0) * (num / den);
    }
    double s = 0;
    for (int j = 1; j <= k; ++j) s += c[j];
    c[0] = -2.0 * s;
}

// Leapfrog stability (eta = 0; damping does not tighten it): the largest
// eigenvalue of -L is at most sum_a S/h_a^2 with S = sum_j |c_j| over the full
// stencil, and the scheme is stable when vmax^2 dt^2 max|lambda| <= 4.
double cfl_dt_max(const Geo& G, double vmax)
{
    double c[kMaxHalf + 1];
    fd_weights(G.half, c);
    double S = std::fabs(c[0]);
    for (int j = 1; j <= G.half; ++j) S += 2.0 * std::fabs(c[j]);
    double lam = 0;
    for (int a = 0; a < 3; ++a)
        if (G.ndim == 3 || a != 1) lam += S / (G.h[a] * G.h[a]);
    return 2.0 / (vmax * std::sqrt(lam));
}

// ---------------------------------------------------------------------------
// Sparse points: multilinear weights over the enclosing cell.
// ---------------------------------------------------------------------------
struct HostPoints {
    int npts = 0;
    std::vector<int64_t> base;     // flat index of the cell's lowest corner
    std::vector<float> w;          // [npts][2^d]
    std::vector<int64_t> cell;     // [npts][3] lowest-corner index per 3D-view axis
};

int make_points(const Geo& G, const wave_points* P, const char* what, HostPoints* out)
{
    out->npts = 0;
    if (!P || P->npts == 0) return WAVE_OK;
    if (P->npts < 0) return fail(WAVE_EINVAL, "%s: npts < 0", what);
    if (!P->coords) return fail(WAVE_EINVAL, "%s: coords is NULL", what);
    const int d = G.ndim, nc = 1 << d;
    const int np = P->npts;
    out->npts = np;
    out->base.resize(np);
    out->w.resize((size_t)np * nc);
    out->cell.resize((size_t)np * 3);
    // the caller's axes map onto the 3D view: 3D (x,y,z) -> 0,1,2; 2D (x,z) -> 0,2
    const int axis3[3] = {0, d == 3 ? 1 : 2, 2};
    for (int p = 0; p < np; ++p) {
        int64_t i0[3] = {0, 0, 0};
        double f[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
            const int A = axis3[a];
            const double c = P->coords[(size_t)p * d + a];
            const double top = (double)(G.n[A] - 1) * G.h[A];
            if (!(c >= 0.0) || !(c <= top))
                return fail(WAVE_ERANGE, "%s point %d: coordinate %d = %.17g outside [0, %.17g]",
                            what, p, a, c, top);
            const double x = std::min(c / G.h[A], (double)(G.n[A] - 1));
            int64_t i = (int64_t)std::floor(x);
            if (i > G.n[A] - 2) i = G.n[A] - 2;
            i0[A] = i;
            f[A] = x - (double)i;
        }
        out->base[p] = (i0[0] * G.n[1] + i0[1]) * G.nzp + i0[2];
        for (int A = 0; A < 3; ++A) out->cell[(size_t)p * 3 + A] = i0[A];
        for (int c = 0; c < nc; ++c) {
            double w = 1.0;
            for (int a = 0; a < d; ++a) {
                const int bit = (c >> (d - 1 - a)) & 1;
                const double fa = f[axis3[a]];
                w *= bit ? fa : 1.0 - fa;
            }
            out->w[(size_t)p * nc + c] = (float)w;
        }
    }
    return WAVE_OK;
}

// Owner-gather table for injection: every (point, corner) pair becomes one
// entry keyed by the grid row and z of its node; entries are sorted by (row,
// z, point) so each node sums its contributions in a fixed order.
struct HostInject {
    std::vector<int32_t> row_ptr;   // [nrows + 1]
    std::vector<InjEntry> ent;
};

void make_inject(const Geo& G, const HostPoints& P, HostInject* out)
{
    const int d = G.ndim, nc = 1 << d;
    struct Keyed {
        int32_t row;
        InjEntry e;
    };
    std::vector<Keyed> ent;
    ent.reserve((size_t)P.npts * nc);
    for (int p = 0; p < P.npts; ++p) {
        const int64_t* i0 = &P.cell[(size_t)p * 3];
        for (int c = 0; c < nc; ++c) {
            int64_t idx[3] = {i0[0], i0[1], i0[2]};
            if (d == 3) {
                idx[0] += (c >> 2) & 1; idx[1] += (c >> 1) & 1; idx[2] += c & 1;
            } else {
                idx[0] += (c >> 1) & 1; idx[2] += c & 1;
            }
            Keyed k;
            k.row = (int32_t)(idx[0] * G.n[1] + idx[1]);
            k.e.z = (int32_t)idx[2];
            k.e.pt = p;
            k.e.w = P.w[(size_t)p * nc + c];
            ent.push_back(k);
        }
    }
    // (row, z, point) is a total order: two corners of one point never share a node
    std::sort(ent.begin(), ent.end(), [](const Keyed& a, const Keyed& b) {
        if (a.row != b.row) return a.row < b.row;
        if (a.e.z != b.e.z) return a.e.z < b.e.z;
        return a.e.pt < b.e.pt;
    });
    const int64_t nrows = G.nrows();
    out->row_ptr.assign(nrows + 1, 0);
    out->ent.resize(ent.size());
    for (size_t i = 0; i < ent.size(); ++i) {
        out->row_ptr[ent[i].row + 1]++;
        out->ent[i] = ent[i].e;
    }
    for (int64_t r = 0; r < nrows; ++r) out->row_ptr[r + 1] += out->row_ptr[r];
}

// ---------------------------------------------------------------------------
// Workspace layout (one function for sizing and for carving).
// ---------------------------------------------------------------------------
struct Plan {
    size_t alpha = 0, beta = 0, check = 0;
    size_t wf[2] = {0, 0};                  // forward wavefield pair
    size_t smp_base[2] = {0, 0}, smp_w[2] = {0, 0};   // [0]: receivers, [1]: sources
    size_t inj_ptr[2] = {0, 0}, inj_ent[2] = {0, 0};  // [0]: sources, [1]: receivers
    size_t ring = 0; int nring = 0;         // backward: forward replay buffers
    size_t gacc = 0;                        // backward: gradient accumulator
    size_t adj[2] = {0, 0};                 // adjoint wavefield pair
    size_t resid = 0, dsyn = 0, red = 0;    // gradient: residual, modelled data, reduction
    size_t ckpt = 0;                        // gradient: checkpoint storage
    // injection values gathered into entry order, double-buffered, for
    // point sets of at least kDenseEntries entries: [0] sources, [1] receivers
    size_t ev[2][2] = {{0, 0}, {0, 0}};
    size_t total = 0;
};

// Injected point sets with this many entries (2^d per point) or more have
// their values gathered into entry order one step ahead, by extra blocks of
// the previous launch: the owner's lookup then costs one memory round trip
// instead of two.  Sparser sets (a few sources) read the values directly.
constexpr int kDenseEntries = 256;

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) { size_t o = off; off = round_up(off + std::max<size_t>(bytes, 1), kAlign); return o; }
};

int ckpt_every(const wave_opts* o) { return (o && o->ckpt_every > 0) ? o->ckpt_every : 20; }

int ckpt_elem(const wave_opts* o)
{
    if (!o || o->ckpt_dtype == WAVE_CKPT_FP32) return 4;
    return 2;
}

size_t ckpt_bytes(const Geo& G, const wave_opts* o)
{
    const int K = ckpt_every(o);
    const int64_t nck = (G.nt + K - 1) / K;
    const size_t snap = round_up((size_t)G.npad() * ckpt_elem(o), kAlign);
    return (size_t)nck * 2 * snap + round_up((size_t)nck * 4 * sizeof(float), kAlign);
}

// What each op keeps in its workspace.  Forward: coefficients, tables and the
// wavefield pair.  Forward with checkpoints: the same plus the codec's
// reduction scratch (the checkpoints themselves are the caller's).  Adjoint:
// coefficients, tables and the adjoint pair.  Backward from checkpoints: the
// replay ring, the adjoint pair and the gradient accumulator.  Gradient: all
// of it, plus residual, modelled data and the checkpoint storage.
Plan make_plan(int op, const Geo& G, int nsrc, int nrec, const wave_opts* o)
{
    Plan P;
    Carver c;
    const size_t N = (size_t)G.npad();
    const int nc = 1 << G.ndim;
#ifdef WAVE_EXP_TABLES_LAST
    Carver big;
    P.alpha = big.take(N * 4 + WAVE_EXP_FIELD_GAP);
    P.beta = big.take(N * 4 + WAVE_EXP_FIELD_GAP);
    P.wf[0] = big.take(N * 4 + WAVE_EXP_FIELD_GAP);
    P.wf[1] = big.take(N * 4 + WAVE_EXP_FIELD_GAP);
    c.off = big.off;
#else
    P.alpha = c.take(N * 4);
    P.beta = c.take(N * 4);
#endif
    P.check = c.take((size_t)kCheckBlocks * 3 * 4);
    // sparse tables: the forward (and the backward's replay) samples receivers
    // and injects sources, the adjoint the other way round
    const bool fwd = op != WAVE_OP_ADJOINT;
    const bool adj = op == WAVE_OP_ADJOINT || op == WAVE_OP_GRADIENT || op == WAVE_OP_BACKWARD;
    const bool samples_rec = fwd && op != WAVE_OP_BACKWARD;
    const int npt[2] = {samples_rec ? nrec : 0, adj ? nsrc : 0};
    for (int s = 0; s < 2; ++s) {
        P.smp_base[s] = c.take((size_t)npt[s] * 8);
        P.smp_w[s] = c.take((size_t)npt[s] * nc * 4);
    }
    const int ipt[2] = {fwd ? nsrc : 0, adj ? nrec : 0};
    const bool iuse[2] = {fwd, adj};
    for (int s = 0; s < 2; ++s) {
        P.inj_ptr[s] = c.take(iuse[s] ? ((size_t)G.nrows() + 1) * 4 : 0);
        P.inj_ent[s] = c.take((size_t)ipt[s] * nc * sizeof(InjEntry));
    }
#ifndef WAVE_EXP_TABLES_LAST
    if (op == WAVE_OP_FORWARD || op == WAVE_OP_FORWARD_CKPT || op == WAVE_OP_GRADIENT) {
        P.wf[0] = c.take(N * 4);
        P.wf[1] = c.take(N * 4);
    }
#endif
    if (adj) {
        P.adj[0] = c.take(N * 4);
        P.adj[1] = c.take(N * 4);
    }
    if (op == WAVE_OP_GRADIENT || op == WAVE_OP_BACKWARD) {
        P.nring = std::min(ckpt_every(o), G.nt) + 1;
        P.ring = c.take(N * 4 * (size_t)P.nring);
        P.gacc = c.take(N * 4);
    }
    if ((op == WAVE_OP_FORWARD || op == WAVE_OP_ADJOINT) && o && (o->flags & WAVE_FLAG_TUNE_IMAGING)) {
        // wave_tune (forward plan) or wave_tune_shot (adjoint plan) of the
        // imaging step: a forward-field plane and a gradient
        P.nring = 1;
        P.ring = c.take(N * 4);
        P.gacc = c.take(N * 4);
    }
    const int nent[2] = {fwd ? nsrc * nc : 0, adj ? nrec * nc : 0};
    for (int s = 0; s < 2; ++s)
        if (nent[s] >= kDenseEntries)
            for (int b = 0; b < 2; ++b) P.ev[s][b] = c.take((size_t)nent[s] * 4);
    if (op == WAVE_OP_GRADIENT || op == WAVE_OP_FORWARD_CKPT) P.red = c.take(kRedFloats * 4);
    if (op == WAVE_OP_GRADIENT) {
        P.resid = c.take((size_t)G.nt * nrec * 4);
        P.dsyn = c.take((size_t)G.nt * nrec * 4);
        P.ckpt = c.take(ckpt_bytes(G, o));
    }
    P.total = c.off;
    return P;
}

// ---------------------------------------------------------------------------
// Tile cache: the fastest tile found by wave_tune / wave_tune_batch for a
// grid, consulted when opts->tile == 0.  Process-wide; mirrored to the file
// named by WAVE_TUNE_CACHE (lines "key tile_id") when that is set.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("WAVE_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[256];
    int id;
    while (std::fscanf(f, "%255s %d", key, &id) == 2) g_tune[key] = id;
    std::fclose(f);
}

// Everything a tile's timing depends on: dimension, order, shape, spacing
// (through the weights, not the traffic, but kept apart to be safe) and
// whether the launch is the adjoint step with the imaging condition, which
// moves 32 instead of 20 bytes per point and holds more registers.
std::string tune_key(const Geo& G, bool imaging)
{
    char b[192];
    std::snprintf(b, sizeof b, "d%do%d:%lldx%lldx%lld:h%.9gx%.9gx%.9g%s", G.ndim, G.order,
                  (long long)G.n[0], (long long)G.n[1], (long long)G.n[2], G.h[0], G.h[1], G.h[2],
                  imaging ? ":img" : "");
    return b;
}

// The tuned tile for `key`, else the default block shape for G with the
// x-chunk chosen by the planner (batched 2D shots: the two-step body; on the
// 48 batched 2001 x 801 order-8 shots 140 us per step against 167 us for the
// one-step slab).
TileCfg cached_tile(const std::string& key, const Geo& G, bool batch)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return tile_from_id(it->second);
    TileCfg c;
    c.variant = (batch && G.ndim == 2) ? kTwoStepVariant : default_variant(G.ndim, G.order, G.n[1], G.nzp);
    return c;
}

// opts->tile: 0 = cached or default, else an explicit id that must name an
// existing block shape.  The two-step 2D body is accepted where `two_step`
// (the batched forward, and the single-shot forward without checkpoints),
// and is the default of the batched forward (`batch`).
int pick_tile(const wave_opts* o, const std::string& key, const Geo& G, TileCfg* out, bool batch = false,
              bool two_step = false)
{
    if (o->tile < 0) return fail(WAVE_EINVAL, "tile id %d is negative", o->tile);
    if (o->tile == 0) {
        *out = cached_tile(key, G, batch);
        return WAVE_OK;
    }
    const TileCfg c = tile_from_id(o->tile);
    if ((batch || two_step) && G.ndim == 2 && c.variant == kTwoStepVariant) {
        *out = c;
        return WAVE_OK;
    }
    if (c.variant >= tile_variants(G.ndim, G.nzp))
        return fail(WAVE_EINVAL, "tile variant %d does not exist (%dD has %d%s)", c.variant, G.ndim,
                    tile_variants(G.ndim, G.nzp),
                    G.ndim == 2 ? "; the two-step variant 4 runs in wave_forward_batch and in "
                                  "wave_forward without checkpoints only" : "");
    *out = c;
    return WAVE_OK;
}

void store_tile(const std::string& key, int id)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[key] = id;
    if (const char* path = std::getenv("WAVE_TUNE_CACHE")) {
        if (FILE* f = std::fopen(path, "a")) {
            std::fprintf(f, "%s %d\n", key.c_str(), id);
            std::fclose(f);
        }
    }
}

// ---------------------------------------------------------------------------
// Per-call device context
// ---------------------------------------------------------------------------
struct Ctx {
    Geo G;
    Plan P;
    char* ws = nullptr;
    hipStream_t s = nullptr;
    float cx[kMaxHalf + 1] = {}, cy[kMaxHalf + 1] = {}, cz[kMaxHalf + 1] = {};
    HostPoints rec, src;
    HostInject inj_src, inj_rec;
    TileCfg cfg;            // block shape and x-chunk of the streaming kernel
    TileCfg cfg_img;        // the same for the adjoint step with the imaging condition
    template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

int check_ws(const Plan& P, const wave_opts* o)
{
    if (!o) return fail(WAVE_EWORKSPACE, "opts is NULL (it carries the workspace)");
    if (o->ckpt_dtype < WAVE_CKPT_FP32 || o->ckpt_dtype > WAVE_CKPT_FP16)
        return fail(WAVE_EINVAL, "unknown ckpt_dtype %d", o->ckpt_dtype);
    if (o->ckpt_every < 0) return fail(WAVE_EINVAL, "ckpt_every must be >= 0");
    if (!o->workspace) return fail(WAVE_EWORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(o->workspace) % kAlign)
        return fail(WAVE_EWORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    if (o->workspace_bytes < P.total)
        return fail(WAVE_EWORKSPACE, "workspace too small: %zu bytes given, %zu needed",
                    o->workspace_bytes, P.total);
    return WAVE_OK;
}

void set_weights(Ctx& C)
{
    double c[kMaxHalf + 1];
    fd_weights(C.G.half, c);
    for (int j = 1; j <= C.G.half; ++j) {
        C.cx[j] = (float)(c[j] / (C.G.h[0] * C.G.h[0]));
        C.cy[j] = C.G.ndim == 3 ? (float)(c[j] / (C.G.h[1] * C.G.h[1])) : 0.f;
        C.cz[j] = (float)(c[j] / (C.G.h[2] * C.G.h[2]));
    }
}

int staging(size_t bytes, char** out)
{
    if (TS().stage.done) HIP_TRY(hipEventSynchronize(TS().stage.done));
    else HIP_TRY(hipEventCreateWithFlags(&TS().stage.done, hipEventDisableTiming));
    if (bytes > TS().stage.cap) {
        if (TS().stage.host) HIP_TRY(hipHostFree(TS().stage.host));
        TS().stage.host = nullptr;
        TS().stage.cap = 0;
        const size_t cap = round_up(std::max<size_t>(bytes, 1 << 20), 1 << 20);
        HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&TS().stage.host), cap, hipHostMallocDefault));
        TS().stage.cap = cap;
    }
    *out = TS().stage.host;
    return WAVE_OK;
}

// Common set-up: sparse tables, uploads, field validation and coefficients
// (one pass over m and eta), then the only wait of the call.  With `noalloc`
// the workspace is the library's own device array (wave_forward_noalloc) and
// the uploads and the read-back go through ordinary host memory instead of
// the pinned staging buffer, so that nothing is allocated on the device or
// pinned on the host.
int setup(Ctx& C, int op, const wave_grid* grid, const float* m, const float* eta,
          const wave_points* src, const wave_points* rec, const wave_opts* o, void* stream,
          bool noalloc = false)
{
    int rc = make_geo(grid, &C.G);
    if (rc) return rc;
    if (!m) return fail(WAVE_EINVAL, "m is NULL");
    if ((rc = make_points(C.G, rec, "receiver", &C.rec))) return rc;
    if ((rc = make_points(C.G, src, "source", &C.src))) return rc;
    C.P = make_plan(op, C.G, C.src.npts, C.rec.npts, o);
    if (noalloc) {
        if (C.P.total > kNoAllocBytes)
            return fail(WAVE_EWORKSPACE,
                        "this grid and point set need %zu bytes of workspace; the no-allocation "
                        "entry point has %zu (use wave_forward with a caller workspace)",
                        C.P.total, kNoAllocBytes);
        void* p = nullptr;
        HIP_TRY(noalloc_scratch(&p));
        C.ws = static_cast<char*>(p);
    } else {
        if ((rc = check_ws(C.P, o))) return rc;
        C.ws = static_cast<char*>(o->workspace);
    }
    C.s = static_cast<hipStream_t>(stream);
    if ((rc = pick_tile(o, tune_key(C.G, false), C.G, &C.cfg))) return rc;
    if ((rc = pick_tile(o, tune_key(C.G, true), C.G, &C.cfg_img))) return rc;
    set_weights(C);
    const bool fwd = op != WAVE_OP_ADJOINT;
    const bool adj = op == WAVE_OP_ADJOINT || op == WAVE_OP_GRADIENT || op == WAVE_OP_BACKWARD;
    if (fwd) make_inject(C.G, C.src, &C.inj_src);
    if (adj) make_inject(C.G, C.rec, &C.inj_rec);

    // gather every upload into the pinned staging buffer
    struct Up { size_t dst; const void* src; size_t bytes; };
    std::vector<Up> ups;
    const int nc = 1 << C.G.ndim;
    // the plan holds receiver sampling tables only for ops that sample them
    const bool samples_rec = fwd && op != WAVE_OP_BACKWARD;
    const HostPoints* sp[2] = {samples_rec ? &C.rec : nullptr, adj ? &C.src : nullptr};
    for (int s = 0; s < 2; ++s) {
        if (!sp[s] || sp[s]->npts == 0) continue;
        ups.push_back({C.P.smp_base[s], sp[s]->base.data(), (size_t)sp[s]->npts * 8});
        ups.push_back({C.P.smp_w[s], sp[s]->w.data(), (size_t)sp[s]->npts * nc * 4});
    }
    const HostInject* ij[2] = {fwd ? &C.inj_src : nullptr, adj ? &C.inj_rec : nullptr};
    for (int s = 0; s < 2; ++s) {
        if (!ij[s]) continue;
        ups.push_back({C.P.inj_ptr[s], ij[s]->row_ptr.data(), ij[s]->row_ptr.size() * 4});
        if (!ij[s]->ent.empty())
            ups.push_back({C.P.inj_ent[s], ij[s]->ent.data(), ij[s]->ent.size() * sizeof(InjEntry)});
    }
    const size_t part_bytes = (size_t)kCheckBlocks * 3 * 4;
    size_t total = part_bytes;
    for (const Up& u : ups) total += round_up(u.bytes, 64);
    char* host = nullptr;
    std::vector<char> pageable;
    if (noalloc) {
        // pageable memory: the copies complete by the wait below, while it lives
        pageable.resize(total);
        host = pageable.data();
    } else if ((rc = staging(total, &host))) {
        return rc;
    }
    float* part = reinterpret_cast<float*>(host);
    size_t off = part_bytes;
    for (const Up& u : ups) {
        std::memcpy(host + off, u.src, u.bytes);
        HIP_TRY(hipMemcpyAsync(C.ws + u.dst, host + off, u.bytes, hipMemcpyHostToDevice, C.s));
        off += round_up(u.bytes, 64);
    }
    HIP_TRY(launch_check_fields(m, eta, C.G.nrows(), C.G.n[2], C.G.nzp, C.at<float>(C.P.check),
                                kCheckBlocks, C.at<float>(C.P.alpha), C.at<float>(C.P.beta),
                                C.G.dt, C.s));
    HIP_TRY(hipMemcpyAsync(part, C.at<float>(C.P.check), part_bytes, hipMemcpyDeviceToHost, C.s));
    if (!noalloc) HIP_TRY(hipEventRecord(TS().stage.done, C.s));
    HIP_TRY(hipStreamSynchronize(C.s));
    float mmin = INFINITY, bad = 0;
    for (int b = 0; b < kCheckBlocks; ++b) {
        mmin = std::min(mmin, part[3 * b]);
        bad += part[3 * b + 2];
    }
    if (bad > 0)
        return fail(WAVE_EINVAL, "%.0f entries of m/eta are invalid (need m finite > 0, eta finite >= 0)", bad);
    const double vmax = 1.0 / std::sqrt((double)mmin);
    const double dtmax = cfl_dt_max(C.G, vmax);
    if (C.G.dt > dtmax)
        return fail(WAVE_ECFL, "dt = %.9g exceeds the stability bound %.9g (vmax = %.6g, order %d)",
                    C.G.dt, dtmax, vmax, C.G.order);
    return WAVE_OK;
}

StepArgs base_args(const Ctx& C)
{
    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.alpha = C.at<float>(C.P.alpha);
    a.beta = C.at<float>(C.P.beta);
    a.nx = C.G.n[0]; a.ny = C.G.n[1]; a.nz = C.G.nzp;
    std::memcpy(a.cx, C.cx, sizeof a.cx);
    std::memcpy(a.cy, C.cy, sizeof a.cy);
    std::memcpy(a.cz, C.cz, sizeof a.cz);
    a.inv_dt2 = (float)(1.0 / (C.G.dt * C.G.dt));
    return a;
}

// set = 0: sources inject (forward), receivers sample; set = 1: receivers
// inject (adjoint), sources sample.
// The planes x and rows y that an injected point set touches: every corner
// node lies in [min x0, max x0 + 1] x [min y0, max y0 + 1] over the points'
// cells (2D: rows are all 0; empty set: x1 < x0).
void inj_planes(const HostPoints& P, StepArgs& a)
{
    a.inj_x0 = a.inj_y0 = 1;
    a.inj_x1 = a.inj_y1 = 0;
    for (int p = 0; p < P.npts; ++p) {
        const int64_t x = P.cell[(size_t)p * 3], y = P.cell[(size_t)p * 3 + 1];
        const int64_t y1 = a.ny > 1 ? y + 1 : y;
        if (p == 0 || x < a.inj_x0) a.inj_x0 = x;
        if (p == 0 || x + 1 > a.inj_x1) a.inj_x1 = x + 1;
        if (p == 0 || y < a.inj_y0) a.inj_y0 = y;
        if (p == 0 || y1 > a.inj_y1) a.inj_y1 = y1;
    }
}

void bind_sparse(const Ctx& C, StepArgs& a, int set)
{
    const int inj = set == 0 ? 0 : 1;
    const int smp = set == 0 ? 0 : 1;
    a.inj.row_ptr = C.at<int32_t>(C.P.inj_ptr[inj]);
    a.inj.ent = C.at<InjEntry>(C.P.inj_ent[inj]);
    inj_planes(set == 0 ? C.src : C.rec, a);
    a.smp.base = C.at<int64_t>(C.P.smp_base[smp]);
    a.smp.w = C.at<float>(C.P.smp_w[smp]);
    a.smp.npts = set == 0 ? C.rec.npts : C.src.npts;
}

// Gathered injection for one step: `set` 0 = sources, 1 = receivers; step
// `n` reads the buffer of parity n and, when `next_vals` is given, the launch
// gathers the next step's values into the other buffer.  No-op for sparse sets.
void gathered(const Ctx& C, StepArgs& a, int set, int n, const float* next_vals)
{
    if (!C.P.ev[set][0]) return;
    const int nent = (set == 0 ? C.src.npts : C.rec.npts) << C.G.ndim;
    a.inj_ev = C.at<float>(C.P.ev[set][n & 1]);
    a.ev_out = next_vals ? C.at<float>(C.P.ev[set][(n + 1) & 1]) : nullptr;
    a.ev_src = next_vals;
    a.nent = next_vals ? nent : 0;
}

// The first gathered step's values (parity of step n).
hipError_t gather_first(const Ctx& C, const StepArgs& a, int set, int n, const float* vals)
{
    if (!C.P.ev[set][0]) return hipSuccess;
    const int nent = (set == 0 ? C.src.npts : C.rec.npts) << C.G.ndim;
    return launch_gather(C.at<float>(C.P.ev[set][n & 1]), vals, a.inj.ent, nent, C.s);
}

hipError_t step(const Ctx& C, const StepArgs& a)
{
    ++TS().prof.launches;
    return launch_step(C.G.ndim, C.G.order, a, C.s, a.img_grad ? C.cfg_img : C.cfg);
}

// Checkpoint storage: per checkpoint c two snapshot arrays (FP32: u^c and
// u^{c-1}; BF16/FP16: u^c and u^c - u^{c-1}, scaled) and a 4-word slot with
// the two scales.
struct CkptView {
    char* base = nullptr;
    int K = 20, elem = 4, nck = 0, dtype = WAVE_CKPT_FP32;
    size_t snap = 0;
    void* snapshot(int c, int which) const { return base + ((size_t)c * 2 + which) * snap; }
    unsigned int* slot(int c) const
    {
        return reinterpret_cast<unsigned int*>(base + (size_t)nck * 2 * snap) + (size_t)c * 4;
    }
};

CkptView ckpt_view(const Geo& G, const wave_opts* o, void* base)
{
    CkptView v;
    v.base = static_cast<char*>(base);
    v.K = ckpt_every(o);
    v.elem = ckpt_elem(o);
    v.dtype = o ? o->ckpt_dtype : WAVE_CKPT_FP32;
    v.nck = (G.nt + v.K - 1) / v.K;
    v.snap = round_up((size_t)G.npad() * v.elem, kAlign);
    return v;
}

int store_checkpoint(const Ctx& C, const CkptView& v, int c, const float* cur, const float* prev)
{
    const int64_t N = C.G.npad();
    if (v.dtype == WAVE_CKPT_FP32) {
        HIP_TRY(hipMemcpyAsync(v.snapshot(c, 0), cur, (size_t)N * 4, hipMemcpyDeviceToDevice, C.s));
        HIP_TRY(hipMemcpyAsync(v.snapshot(c, 1), prev, (size_t)N * 4, hipMemcpyDeviceToDevice, C.s));
        return WAVE_OK;
    }
    HIP_TRY(launch_ckpt_encode(cur, prev, N, v.dtype == WAVE_CKPT_BF16, v.slot(c),
                               C.at<float>(C.P.red), kRedFloats / 2,
                               static_cast<unsigned short*>(v.snapshot(c, 0)),
                               static_cast<unsigned short*>(v.snapshot(c, 1)), C.s));
    return WAVE_OK;
}

int load_checkpoint(const Ctx& C, const CkptView& v, int c, float* cur, float* prev)
{
    const int64_t N = C.G.npad();
    if (v.dtype == WAVE_CKPT_FP32) {
        HIP_TRY(hipMemcpyAsync(cur, v.snapshot(c, 0), (size_t)N * 4, hipMemcpyDeviceToDevice, C.s));
        HIP_TRY(hipMemcpyAsync(prev, v.snapshot(c, 1), (size_t)N * 4, hipMemcpyDeviceToDevice, C.s));
        return WAVE_OK;
    }
    HIP_TRY(launch_ckpt_decode(static_cast<const unsigned short*>(v.snapshot(c, 0)),
                               static_cast<const unsigned short*>(v.snapshot(c, 1)), v.slot(c), N,
                               v.dtype == WAVE_CKPT_BF16, cur, prev, C.s));
    return WAVE_OK;
}

// Forward time loop over the two-buffer in-place leapfrog.  If `ck` is set,
// the pair (u^c, u^{c-1}) is stored before step c for c = 0, K, 2K, ...
int run_forward(const Ctx& C, const float* q, float* d, float* u_final, const CkptView* ck,
                bool close_prof)
{
    const int64_t N = C.G.npad();
    float* buf[2] = {C.at<float>(C.P.wf[0]), C.at<float>(C.P.wf[1])};
    HIP_TRY(launch_fill(buf[0], N, 0.f, C.s));
    HIP_TRY(launch_fill(buf[1], N, 0.f, C.s));
    StepArgs a = base_args(C);
    bind_sparse(C, a, 0);
    if (C.src.npts) HIP_TRY(gather_first(C, a, 0, 0, q));
    int cur = 0;   // buf[cur] = u^n, buf[1-cur] = u^{n-1}
    if (prof_begin(C.s)) return fail(WAVE_EHIP, "profiling event failed");
    for (int n = 0; n < C.G.nt; ++n) {
        if (ck && n % ck->K == 0) {
            const int rc = store_checkpoint(C, *ck, n / ck->K, buf[cur], buf[1 - cur]);
            if (rc) return rc;
        }
        a.cur = buf[cur];
        a.other = buf[1 - cur];
        a.out = buf[1 - cur];
        a.inj_val = C.src.npts ? q + (size_t)n * C.src.npts : nullptr;
        if (C.src.npts)
            gathered(C, a, 0, n, n + 1 < C.G.nt ? q + (size_t)(n + 1) * C.src.npts : nullptr);
        a.smp_out = C.rec.npts ? d + (size_t)n * C.rec.npts : nullptr;
        HIP_TRY(step(C, a));
        cur = 1 - cur;
    }
    if (close_prof && prof_end(C.s)) return fail(WAVE_EHIP, "profiling event failed");
    if (u_final) HIP_TRY(copy_out(u_final, buf[cur], C.G, C.s));
    return WAVE_OK;
}

// Backward pass: replay each checkpoint segment forward into the ring, then
// step the adjoint through it with the imaging condition fused.
int run_backward(const Ctx& C, const float* q, const float* r, const CkptView& ck, float* grad,
                 float* grad_q, bool open_prof)
{
    const int64_t N = C.G.npad();
    const int nt = C.G.nt;
    float* v[2] = {C.at<float>(C.P.adj[0]), C.at<float>(C.P.adj[1])};
    HIP_TRY(launch_fill(v[0], N, 0.f, C.s));
    HIP_TRY(launch_fill(v[1], N, 0.f, C.s));
    float* gacc = C.at<float>(C.P.gacc);
    HIP_TRY(launch_fill(gacc, N, 0.f, C.s));
    float* ring = C.at<float>(C.P.ring);
    auto slot = [&](int i) { return ring + (size_t)i * N; };
    StepArgs fa = base_args(C);
    bind_sparse(C, fa, 0);
    fa.smp_out = nullptr;       // the replay samples nothing (no receiver tables in this plan)
    fa.smp.npts = 0;
    StepArgs ba = base_args(C);
    bind_sparse(C, ba, 1);
    ba.img_grad = gacc;
    if (C.rec.npts) HIP_TRY(gather_first(C, ba, 1, nt - 1, r + (size_t)(nt - 1) * C.rec.npts));
    int vc = 0;    // v[vc] = v^k, v[1-vc] = v^{k+1}
    if (open_prof && prof_begin(C.s)) return fail(WAVE_EHIP, "profiling event failed");
    for (int seg = ck.nck - 1; seg >= 0; --seg) {
        const int c0 = seg * ck.K;
        const int c1 = std::min(c0 + ck.K, nt);
        // ring slot i holds u^{c0 - 1 + i}
        const int rc = load_checkpoint(C, ck, seg, slot(1), slot(0));
        if (rc) return rc;
        for (int n = c0; n < c1 - 1; ++n) {
            fa.cur = slot(n - c0 + 1);
            fa.other = slot(n - c0);
            fa.out = slot(n - c0 + 2);
            fa.inj_val = C.src.npts ? q + (size_t)n * C.src.npts : nullptr;
            HIP_TRY(step(C, fa));
        }
        for (int k = c1 - 1; k >= c0; --k) {
            ba.cur = v[vc];
            ba.other = v[1 - vc];
            ba.out = v[1 - vc];
            ba.inj_val = C.rec.npts ? r + (size_t)k * C.rec.npts : nullptr;
            if (C.rec.npts) gathered(C, ba, 1, k, k > 0 ? r + (size_t)(k - 1) * C.rec.npts : nullptr);
            ba.smp_out = (grad_q && C.src.npts) ? grad_q + (size_t)k * C.src.npts : nullptr;
            ba.img_fwd = slot(k - c0 + 1);
            HIP_TRY(step(C, ba));
            vc = 1 - vc;
        }
    }
    if (prof_end(C.s)) return fail(WAVE_EHIP, "profiling event failed");
    HIP_TRY(copy_out(grad, gacc, C.G, C.s));
    return WAVE_OK;
}

// ---------------------------------------------------------------------------
// Tile autotuner (the paper's brute-force search over block sizes, Section
// "Loop Blocking", applied to the streaming kernel's block shape and x-chunk):
// each candidate is launched `steps` times on zeroed workspace buffers and
// timed with HIP events; the fastest per-step time wins.  Timing does not
// depend on the field values, and every candidate gives bitwise the same
// result (the per-point arithmetic does not depend on the tiling).
// ---------------------------------------------------------------------------
// Candidate tiles: every block shape with x-chunks of 2R, 4R, 8 .. 128
// planes and of every split of the grid into 2 .. 32 chunks, each clamped to
// what the shape accepts (the 2D slabs hold at most 16 rows) and to the grid,
// so that no two candidates launch the same thing.  Batched 2D shots also
// try the two-step slab.
std::vector<TileCfg> tile_candidates(int ndim, int half, int64_t nx, int64_t nz, bool batch = false)
{
    std::vector<TileCfg> out;
    // fixed lengths, and the length of every split of x into 2 .. 32 chunks
    // (on 200^3 order 8 the step takes 26.3 us at 17 planes, 32.1 us at 16
    // and 29.1 us at 11: how chunk ends fall on XCDs matters as much as the
    // prologue, so the search is dense rather than a rule)
    std::vector<int64_t> xs = {2 * half, 4 * half, 8, 16, 32, 64, 128};
    for (int64_t k = 2; k <= 32; ++k) xs.push_back((nx + k - 1) / k);
    const int nv = tile_variants(ndim, nz) + ((batch && ndim == 2) ? 1 : 0);   // + the two-step slab
    for (int v = 0; v < nv; ++v)
        for (int64_t x : xs) {
            if (x < 2 * half) continue;
            TileCfg c;
            c.variant = v;
            c.xchunk = (int)std::min<int64_t>(std::min<int64_t>(x, max_xchunk(ndim, v)), std::min<int64_t>(nx, 0xffff));
            bool dup = false;
            for (const TileCfg& o : out) dup = dup || (o.variant == c.variant && o.xchunk == c.xchunk);
            if (!dup) out.push_back(c);
        }
    return out;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// ---------------------------------------------------------------------------
// Batched shots: every shot's step n runs in one launch over a flattened list
// of (shot, tile, x-chunk) blocks; the nt launches are captured once into a
// hipGraph (on a library-owned capture stream) and replayed on the caller's
// stream.  The instantiated graph is kept per thread and reused while the
// launch arguments are unchanged.
// ---------------------------------------------------------------------------
struct BatchShot {
    Geo G;
    HostPoints rec, src;
    HostInject inj;
    size_t alpha = 0, beta = 0, buf[4] = {0, 0, 0, 0}, smp_base = 0, smp_w = 0, inj_ptr = 0, inj_ent = 0;
};

struct BatchPlan {
    std::vector<BatchShot> shots;
    size_t desc = 0, begin = 0, check = 0, sync = 0, total = 0;
};

constexpr int kCheckBlocksShot = 256;

int batch_plan(int32_t nshots, const wave_shot* shots, BatchPlan* B, bool build_tables)
{
    if (nshots < 1 || !shots) return fail(WAVE_EINVAL, "need at least one shot");
    B->shots.assign(nshots, BatchShot{});
    Carver c;
    B->desc = c.take(sizeof(ShotDesc) * (size_t)nshots);
    B->begin = c.take(sizeof(int64_t) * ((size_t)nshots + 1));
    B->check = c.take((size_t)nshots * kCheckBlocksShot * 3 * 4);
    B->sync = c.take(64);
    for (int i = 0; i < nshots; ++i) {
        BatchShot& S = B->shots[i];
        int rc = make_geo(&shots[i].grid, &S.G);
        if (rc) return fail(rc, "shot %d: %s", i, g_error.c_str());
        const Geo& G0 = B->shots[0].G;
        if (S.G.ndim != G0.ndim || S.G.order != G0.order || S.G.nt != G0.nt || S.G.dt != G0.dt)
            return fail(WAVE_EINVAL, "shot %d: every shot needs the same ndim, space_order, nt and dt", i);
        if (!shots[i].m) return fail(WAVE_EINVAL, "shot %d: m is NULL", i);
        if (shots[i].src.npts > 0 && !shots[i].q) return fail(WAVE_EINVAL, "shot %d: q is NULL", i);
        if (shots[i].rec.npts > 0 && !shots[i].d) return fail(WAVE_EINVAL, "shot %d: d is NULL", i);
        if (build_tables) {
            if ((rc = make_points(S.G, &shots[i].rec, "receiver", &S.rec)))
                return fail(rc, "shot %d: %s", i, g_error.c_str());
            if ((rc = make_points(S.G, &shots[i].src, "source", &S.src)))
                return fail(rc, "shot %d: %s", i, g_error.c_str());
        }
        const int ns = shots[i].src.npts > 0 ? shots[i].src.npts : 0;
        const int nr = shots[i].rec.npts > 0 ? shots[i].rec.npts : 0;
        const size_t N = (size_t)S.G.npad();
        const int nc = 1 << S.G.ndim;
        S.alpha = c.take(N * 4);
        S.beta = c.take(N * 4);
        // 2D shots keep a second wavefield pair for the two-step slab, whose
        // passes read one pair and write the other
        for (int k = 0; k < (S.G.ndim == 2 ? 4 : 2); ++k) S.buf[k] = c.take(N * 4);
        S.smp_base = c.take((size_t)nr * 8);
        S.smp_w = c.take((size_t)nr * nc * 4);
        S.inj_ptr = c.take(((size_t)S.G.nrows() + 1) * 4);
        S.inj_ent = c.take((size_t)ns * nc * sizeof(InjEntry));
    }
    B->total = c.off;
    return WAVE_OK;
}

// Workspace of a batch of one shot with ns sources and nr receivers (the
// single-shot 2D forward on the two-step body runs as one); batch_plan only
// checks the pointers for presence here, it reads no data.
size_t one_shot_batch_bytes(const wave_grid& grid, int ns, int nr)
{
    static const float present = 0.f;
    wave_shot one;
    std::memset(&one, 0, sizeof one);
    one.grid = grid;
    one.m = &present;
    one.src.npts = ns;
    one.rec.npts = nr;
    one.q = &present;
    one.d = const_cast<float*>(&present);
    BatchPlan B;
    if (batch_plan(1, &one, &B, false)) return 0;
    return B.total;
}

StepArgs shot_args(const BatchShot& S, char* ws)
{
    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.alpha = reinterpret_cast<float*>(ws + S.alpha);
    a.beta = reinterpret_cast<float*>(ws + S.beta);
    a.nx = S.G.n[0]; a.ny = S.G.n[1]; a.nz = S.G.nzp;
    double c[kMaxHalf + 1];
    fd_weights(S.G.half, c);
    for (int j = 1; j <= S.G.half; ++j) {
        a.cx[j] = (float)(c[j] / (S.G.h[0] * S.G.h[0]));
        a.cy[j] = S.G.ndim == 3 ? (float)(c[j] / (S.G.h[1] * S.G.h[1])) : 0.f;
        a.cz[j] = (float)(c[j] / (S.G.h[2] * S.G.h[2]));
    }
    a.inv_dt2 = (float)(1.0 / (S.G.dt * S.G.dt));
    a.inj.row_ptr = reinterpret_cast<int32_t*>(ws + S.inj_ptr);
    a.inj.ent = reinterpret_cast<InjEntry*>(ws + S.inj_ent);
    inj_planes(S.src, a);
    a.smp.base = reinterpret_cast<int64_t*>(ws + S.smp_base);
    a.smp.w = reinterpret_cast<float*>(ws + S.smp_w);
    a.smp.npts = S.rec.npts;
    return a;
}

// Descriptors for a tile config; returns the total block count via *blocks.
// The flattened block list takes the shots largest first (longest work
// first: the last blocks of a launch, and the last items of each persistent
// block, are then the small ones).  The order does not change any result:
// each block computes one shot's tile, and shots are independent.
void build_descs(const BatchPlan& B, const wave_shot* shots, char* ws, TileCfg cfg,
                 std::vector<ShotDesc>* desc, std::vector<int64_t>* begin, int64_t* blocks)
{
    const int n = (int)B.shots.size();
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return B.shots[a].G.npad() > B.shots[b].G.npad(); });
    desc->assign(n, ShotDesc{});
    begin->assign(n + 1, 0);
    int64_t acc = 0;
    for (int k = 0; k < n; ++k) {
        const int i = order[k];
        const BatchShot& S = B.shots[i];
        ShotDesc& D = (*desc)[k];
        D.a = shot_args(S, ws);
        D.a.smp_out = S.rec.npts ? shots[i].d : nullptr;   // marks sampling as active for planning
        const int64_t nb = plan_tiles(S.G.ndim, S.G.order, cfg, D.a);
        D.a.smp_out = nullptr;
        for (int k = 0; k < 4; ++k)
            D.buf[k] = (k < 2 || S.G.ndim == 2) ? reinterpret_cast<float*>(ws + S.buf[k]) : nullptr;
        D.q = shots[i].q;
        D.d = S.rec.npts ? shots[i].d : nullptr;
        D.nsrc = S.src.npts;
        D.nrec = S.rec.npts;
        (*begin)[k] = acc;
        acc += nb;
    }
    (*begin)[n] = acc;
    *blocks = acc;
}

// Uploads, field checks (one wait for all shots), coefficient fields and
// zeroed wavefields.
int batch_setup(const BatchPlan& B, const wave_shot* shots, char* ws, hipStream_t st)
{
    const int n = (int)B.shots.size();
    struct Up { size_t dst; const void* src; size_t bytes; };
    std::vector<Up> ups;
    std::vector<HostInject> injs(n);
    const int nc = 1 << B.shots[0].G.ndim;
    for (int i = 0; i < n; ++i) {
        const BatchShot& S = B.shots[i];
        make_inject(S.G, S.src, &injs[i]);
        if (S.rec.npts) {
            ups.push_back({S.smp_base, S.rec.base.data(), (size_t)S.rec.npts * 8});
            ups.push_back({S.smp_w, S.rec.w.data(), (size_t)S.rec.npts * nc * 4});
        }
        ups.push_back({S.inj_ptr, injs[i].row_ptr.data(), injs[i].row_ptr.size() * 4});
        if (!injs[i].ent.empty())
            ups.push_back({S.inj_ent, injs[i].ent.data(), injs[i].ent.size() * sizeof(InjEntry)});
    }
    const size_t part_bytes = (size_t)n * kCheckBlocksShot * 3 * 4;
    size_t total = part_bytes;
    for (const Up& u : ups) total += round_up(u.bytes, 64);
    char* host = nullptr;
    int rc = staging(total, &host);
    if (rc) return rc;
    size_t off = part_bytes;
    for (const Up& u : ups) {
        std::memcpy(host + off, u.src, u.bytes);
        HIP_TRY(hipMemcpyAsync(ws + u.dst, host + off, u.bytes, hipMemcpyHostToDevice, st));
        off += round_up(u.bytes, 64);
    }
    float* part = reinterpret_cast<float*>(host);
    for (int i = 0; i < n; ++i) {
        const BatchShot& S = B.shots[i];
        HIP_TRY(launch_check_fields(shots[i].m, shots[i].eta, S.G.nrows(), S.G.n[2], S.G.nzp,
                                    reinterpret_cast<float*>(ws + B.check) + (size_t)i * kCheckBlocksShot * 3,
                                    kCheckBlocksShot, reinterpret_cast<float*>(ws + S.alpha),
                                    reinterpret_cast<float*>(ws + S.beta), S.G.dt, st));
    }
    HIP_TRY(hipMemcpyAsync(part, ws + B.check, part_bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(TS().stage.done, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
        const BatchShot& S = B.shots[i];
        float mmin = INFINITY, bad = 0;
        for (int b = 0; b < kCheckBlocksShot; ++b) {
            mmin = std::min(mmin, part[((size_t)i * kCheckBlocksShot + b) * 3]);
            bad += part[((size_t)i * kCheckBlocksShot + b) * 3 + 2];
        }
        if (bad > 0) return fail(WAVE_EINVAL, "shot %d: %.0f invalid entries in m/eta", i, bad);
        const double dtmax = cfl_dt_max(S.G, 1.0 / std::sqrt((double)mmin));
        if (S.G.dt > dtmax)
            return fail(WAVE_ECFL, "shot %d: dt = %.9g exceeds the stability bound %.9g", i, S.G.dt, dtmax);
    }
    for (int i = 0; i < n; ++i) {
        const BatchShot& S = B.shots[i];
        HIP_TRY(launch_fill(reinterpret_cast<float*>(ws + S.buf[0]), S.G.npad(), 0.f, st));
        HIP_TRY(launch_fill(reinterpret_cast<float*>(ws + S.buf[1]), S.G.npad(), 0.f, st));
    }
    return WAVE_OK;
}

int upload_descs(const std::vector<ShotDesc>& desc, const std::vector<int64_t>& begin, char* ws,
                 const BatchPlan& B, hipStream_t st)
{
    const size_t db = desc.size() * sizeof(ShotDesc), bb = begin.size() * sizeof(int64_t);
    char* host = nullptr;
    int rc = staging(db + bb, &host);
    if (rc) return rc;
    std::memcpy(host, desc.data(), db);
    std::memcpy(host + db, begin.data(), bb);
    HIP_TRY(hipMemcpyAsync(ws + B.desc, host, db, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ws + B.begin, host + db, bb, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(TS().stage.done, st));
    return WAVE_OK;
}

std::string batch_key(const BatchPlan& B)
{
    int64_t pts = 0, mx = 0;
    for (const BatchShot& S : B.shots) { pts += S.G.npts(); mx = std::max(mx, S.G.n[0]); }
    char b[224];
    const Geo& G = B.shots[0].G;
    std::snprintf(b, sizeof b, "batch:d%do%d:%zu:%lld:%lldx%lld:h%.9gx%.9gx%.9g", G.ndim, G.order,
                  B.shots.size(), (long long)pts, (long long)mx, (long long)G.n[2], G.h[0], G.h[1],
                  G.h[2]);
    return b;
}

// Everything the instantiated graph bakes in.
std::vector<char> graph_key(const ShotDesc* d_desc, const int64_t* d_begin, int64_t blocks,
                            const Geo& G, int nshots, TileCfg cfg, int persistent)
{
    std::vector<char> key(sizeof(void*) * 2 + sizeof(int64_t) * 2 + sizeof(int) * 7);
    char* k = key.data();
    auto put = [&](const void* p, size_t n) { std::memcpy(k, p, n); k += n; };
    put(&d_desc, sizeof(void*));
    put(&d_begin, sizeof(void*));
    put(&blocks, sizeof(int64_t));
    const int64_t nz = G.nzp;
    put(&nz, sizeof(int64_t));
    const int v[7] = {nshots, G.nt, G.ndim, G.order, cfg.variant, cfg.xchunk, persistent};
    put(v, sizeof v);
    return key;
}

int instantiate_cached(hipGraph_t graph, const std::vector<char>& key)
{
    if (TS().graph.exec) {
        HIP_TRY(hipGraphExecDestroy(TS().graph.exec));
        TS().graph.exec = nullptr;
        TS().graph.key.clear();
    }
    const hipError_t e = hipGraphInstantiate(&TS().graph.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        TS().graph.exec = nullptr;
        return fail(WAVE_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    TS().graph.key = key;
    return WAVE_OK;
}

// One persistent cooperative launch for all steps (directly, or as the
// cooperative node of a cached graph), then a wait and a check of the
// barrier error word, so a barrier that did not complete is reported, never
// left hanging.
int run_batch_persistent(const BatchPlan& B, char* ws, TileCfg cfg, int64_t items, hipStream_t st,
                         bool use_graph)
{
    const Geo& G = B.shots[0].G;
    const int nshots = (int)B.shots.size();
    const ShotDesc* d_desc = reinterpret_cast<const ShotDesc*>(ws + B.desc);
    const int64_t* d_begin = reinterpret_cast<const int64_t*>(ws + B.begin);
    unsigned int* sync = reinterpret_cast<unsigned int*>(ws + B.sync);
    const int32_t spin_limit = 2000000;   // a few seconds of polling per barrier at most
    int grid = 0;
    TS().prof.launches += 1;
    if (!use_graph) {
        HIP_TRY(launch_fill(reinterpret_cast<float*>(sync), 2, 0.f, st));
        HIP_TRY(launch_batch_persistent(G.ndim, G.order, G.nzp, cfg, d_desc, d_begin, nshots, items,
                                        G.nt, sync, spin_limit, &grid, st));
        TS().batch_mode = 2;
    } else {
        const std::vector<char> key = graph_key(d_desc, d_begin, items, G, nshots, cfg, 1);
        if (!TS().graph.exec || TS().graph.key != key) {
            hipGraph_t graph = nullptr;
            HIP_TRY(graph_batch_persistent(G.ndim, G.order, G.nzp, cfg, d_desc, d_begin, nshots,
                                           items, G.nt, sync, spin_limit, &grid, &graph));
            const int rc = instantiate_cached(graph, key);
            if (rc) return rc;
        }
        HIP_TRY(hipGraphLaunch(TS().graph.exec, st));
        TS().batch_mode = 3;
    }
    unsigned int words[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(words, sync, sizeof words, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (words[1])
        return fail(WAVE_EHIP, "persistent batch: a device-wide barrier timed out");
    return WAVE_OK;
}

// Launches of a two-step run of nt steps (2D slab, variant kTwoStepVariant).
// An odd nt starts with one step (u^1 into buffer 2); then passes of two
// steps alternate between two buffer pairs, each sampling u^n and the
// previous pass's intermediate u^{n-1}; a last launch samples u^{nt-1}.
// Every level 0 .. nt-1 is sampled once.  *final_buf receives the buffer
// that holds u^nt.
struct Launch2 {
    int32_t n, bufs, flags;
};

std::vector<Launch2> two_step_schedule(int nt, int* final_buf)
{
    auto pack = [](int c, int o, int o1, int o2) { return c | (o << 2) | (o1 << 4) | (o2 << 6); };
    std::vector<Launch2> L;
    const int s0 = nt & 1;
    int pair[2][2] = {{0, 1}, {2, 3}};           // {u^n, u^{n-1}} of the passes' input pairs
    if (s0) {
        L.push_back({0, pack(0, 1, 2, 3), 1 | 2 | 8});
        pair[0][0] = 2; pair[0][1] = 0;
        pair[1][0] = 1; pair[1][1] = 3;
    }
    const int P = (nt - s0) / 2;
    for (int p = 0; p < P; ++p) {
        const int* in = pair[p & 1];
        const int* out = pair[(p + 1) & 1];
        L.push_back({s0 + 2 * p, pack(in[0], in[1], out[1], out[0]), 1 | 2 | (p > 0 ? 4 : 0)});
    }
    if (P > 0) L.push_back({nt, pack(pair[P & 1][0], pair[P & 1][1], 0, 0), 4});
    *final_buf = pair[P & 1][0];
    return L;
}

hipError_t launch_schedule_entry(const Geo& G, TileCfg cfg, const ShotDesc* d_desc, const int64_t* d_begin,
                                 int nshots, int64_t blocks, int i, const std::vector<Launch2>& sched,
                                 hipStream_t st)
{
    if (cfg.variant == kTwoStepVariant && G.ndim == 2)
        return launch_batch2(G.order, d_desc, d_begin, nshots, blocks, sched[i].n, sched[i].bufs,
                             sched[i].flags, st);
    return launch_batch(G.ndim, G.order, G.nzp, cfg, d_desc, d_begin, nshots, blocks, i, st);
}

int run_batch_loop(const BatchPlan& B, char* ws, TileCfg cfg, int64_t blocks, hipStream_t st,
                   bool use_graph)
{
    const Geo& G = B.shots[0].G;
    const int nshots = (int)B.shots.size();
    const ShotDesc* d_desc = reinterpret_cast<const ShotDesc*>(ws + B.desc);
    const int64_t* d_begin = reinterpret_cast<const int64_t*>(ws + B.begin);
    TS().batch_mode = use_graph ? 0 : 1;
    const bool two = cfg.variant == kTwoStepVariant && G.ndim == 2;
    int final_buf = 0;
    const std::vector<Launch2> sched = two ? two_step_schedule(G.nt, &final_buf) : std::vector<Launch2>();
    const int nl = two ? (int)sched.size() : G.nt;
    if (!use_graph) {
        for (int i = 0; i < nl; ++i) {
            ++TS().prof.launches;
            HIP_TRY(launch_schedule_entry(G, cfg, d_desc, d_begin, nshots, blocks, i, sched, st));
        }
        return WAVE_OK;
    }
    const std::vector<char> key = graph_key(d_desc, d_begin, blocks, G, nshots, cfg, 0);
    if (!TS().graph.exec || TS().graph.key != key) {
        if (!TS().graph.capture) HIP_TRY(hipStreamCreateWithFlags(&TS().graph.capture, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(TS().graph.capture, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        for (int i = 0; i < nl && err == hipSuccess; ++i)
            err = launch_schedule_entry(G, cfg, d_desc, d_begin, nshots, blocks, i, sched,
                                        TS().graph.capture);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(TS().graph.capture, &graph);
        if (err != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(WAVE_EHIP, "graph capture of the batched loop failed: %s",
                        hipGetErrorString(err != hipSuccess ? err : e2));
        }
        const int rc = instantiate_cached(graph, key);
        if (rc) return rc;
    }
    TS().prof.launches += nl;
    HIP_TRY(hipGraphLaunch(TS().graph.exec, st));
    return WAVE_OK;
}

}  // namespace

extern "C" {

const char* wave_last_error(void) { return g_error.c_str(); }

const char* wave_version(void) { return "wavefd-mi355x 0.1 (gfx950)"; }

int wave_last_batch_mode(void) { return TS().batch_mode; }

int wave_release(void)
{
    // Per thread, in dependency order: the graph executable, its capture
    // stream, the timing events, then the pinned staging buffer after its
    // last copy.
    int rc = WAVE_OK;
    auto note = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == WAVE_OK)
            rc = fail(WAVE_EHIP, "wave_release: %s: %s", what, hipGetErrorString(e));
    };
    std::lock_guard<std::mutex> lk(g_threads_mu);
    for (ThreadState* t : g_threads) {
        if (t->graph.exec) note(hipGraphExecDestroy(t->graph.exec), "hipGraphExecDestroy");
        t->graph.exec = nullptr;
        t->graph.key.clear();
        if (t->graph.capture) note(hipStreamDestroy(t->graph.capture), "hipStreamDestroy");
        t->graph.capture = nullptr;
        if (t->prof.t0) note(hipEventDestroy(t->prof.t0), "hipEventDestroy");
        if (t->prof.t1) note(hipEventDestroy(t->prof.t1), "hipEventDestroy");
        t->prof.t0 = t->prof.t1 = nullptr;
        t->prof.have = false;
        if (t->stage.done) {
            note(hipEventSynchronize(t->stage.done), "hipEventSynchronize");
            note(hipEventDestroy(t->stage.done), "hipEventDestroy");
        }
        t->stage.done = nullptr;
        if (t->stage.host) note(hipHostFree(t->stage.host), "hipHostFree");
        t->stage.host = nullptr;
        t->stage.cap = 0;
    }
    return rc;
}

int wave_tile_candidates(const wave_grid* grid, int32_t* ids, int32_t cap, int32_t* n)
{
    try {
        if (!n || cap < 0 || (cap > 0 && !ids)) return fail(WAVE_EINVAL, "n is required, ids for cap > 0");
        Geo G;
        int rc = make_geo(grid, &G);
        if (rc) return rc;
        const std::vector<TileCfg> c = tile_candidates(G.ndim, G.half, G.n[0], G.nzp);
        *n = (int32_t)c.size();
        for (int32_t i = 0; i < cap && i < (int32_t)c.size(); ++i) ids[i] = tile_id(c[i]);
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    }
}

int wave_resolve_tile(const wave_grid* grid, int32_t tile, int32_t* resolved)
{
    try {
        if (!resolved) return fail(WAVE_EINVAL, "resolved is NULL");
        Geo G;
        int rc = make_geo(grid, &G);
        if (rc) return rc;
        wave_opts o;
        std::memset(&o, 0, sizeof o);
        o.tile = tile;
        TileCfg cfg;
        if ((rc = pick_tile(&o, tune_key(G, false), G, &cfg, false, true))) return rc;
        StepArgs a;
        std::memset(&a, 0, sizeof a);
        a.nx = G.n[0]; a.ny = G.n[1]; a.nz = G.nzp;
        // with a device present, the plan a launch on it makes (occupancy-sized
        // x-chunks); without one, the occupancy-free plan
        int ndev = 0;
        const bool device = hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0;
        if (plan_tiles(G.ndim, G.order, cfg, a, device) < 0)
            return fail(WAVE_EINVAL, "tile %d cannot be planned", tile);
        TileCfg out = cfg;
        out.xchunk = a.xchunk;
        *resolved = tile_id(out);
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    }
}

int wave_misfit(const float* d, const float* d_obs, int64_t n, float* r, float* misfit,
                const wave_opts* opts, void* stream)
{
    if (!misfit || n < 0 || (n > 0 && (!d || !d_obs)))
        return fail(WAVE_EINVAL, "misfit is required, n >= 0, and d and d_obs when n > 0");
    if (!opts || !opts->workspace || reinterpret_cast<uintptr_t>(opts->workspace) % kAlign)
        return fail(WAVE_EWORKSPACE, "workspace missing or not %zu-byte aligned", kAlign);
    if (opts->workspace_bytes < (size_t)WAVE_MISFIT_WORKSPACE_BYTES)
        return fail(WAVE_EWORKSPACE, "workspace too small: %zu bytes given, %d needed",
                    opts->workspace_bytes, WAVE_MISFIT_WORKSPACE_BYTES);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_residual(d, d_obs, r, n, static_cast<float*>(opts->workspace), kRedFloats, misfit, st));
    return WAVE_OK;
}

int wave_set_profiling(int32_t enable)
{
    TS().prof.on = enable != 0;
    TS().prof.have = false;
    return WAVE_OK;
}

int wave_last_loop(double* ms, int64_t* launches)
{
    if (!ms || !launches) return fail(WAVE_EINVAL, "ms and launches are required");
    if (!TS().prof.have) return fail(WAVE_EINVAL, "no profiled call on this thread");
    HIP_TRY(hipEventSynchronize(TS().prof.t1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, TS().prof.t0, TS().prof.t1));
    *ms = f;
    *launches = TS().prof.launches;
    return WAVE_OK;
}

int wave_workspace_size(int32_t op, const wave_grid* grid, const wave_points* src,
                        const wave_points* rec, const wave_opts* opts, size_t* bytes)
{
    try {
        if (!bytes) return fail(WAVE_EINVAL, "bytes is NULL");
        if (op < WAVE_OP_FORWARD || op > WAVE_OP_BACKWARD) return fail(WAVE_EINVAL, "unknown op %d", op);
        Geo G;
        int rc = make_geo(grid, &G);
        if (rc) return rc;
        const int ns = src ? src->npts : 0, nr = rec ? rec->npts : 0;
        if (ns < 0 || nr < 0) return fail(WAVE_EINVAL, "npts < 0");
        *bytes = make_plan(op, G, ns, nr, opts).total;
        if (op == WAVE_OP_FORWARD && G.ndim == 2) *bytes = std::max(*bytes, one_shot_batch_bytes(*grid, ns, nr));
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_checkpoint_size(const wave_grid* grid, const wave_opts* opts, size_t* bytes)
{
    if (!bytes) return fail(WAVE_EINVAL, "bytes is NULL");
    Geo G;
    int rc = make_geo(grid, &G);
    if (rc) return rc;
    if (opts && (opts->ckpt_dtype < WAVE_CKPT_FP32 || opts->ckpt_dtype > WAVE_CKPT_FP16))
        return fail(WAVE_EINVAL, "unknown ckpt_dtype %d", opts->ckpt_dtype);
    *bytes = ckpt_bytes(G, opts);
    return WAVE_OK;
}

int wave_forward(const wave_grid* grid, const float* m, const float* eta, const wave_points* src,
                 const float* q, const wave_points* rec, float* d, float* u_final, void* ckpt,
                 const wave_opts* opts, void* stream)
{
    try {
        Ctx C;
        const int op = ckpt ? WAVE_OP_FORWARD_CKPT : WAVE_OP_FORWARD;
        if (src && src->npts > 0 && !q) return fail(WAVE_EINVAL, "q is NULL with %d sources", src->npts);
        if (rec && rec->npts > 0 && !d) return fail(WAVE_EINVAL, "d is NULL with %d receivers", rec->npts);
        if (!ckpt && grid && grid->ndim == 2 && opts && opts->tile > 0 &&
            tile_from_id(opts->tile).variant == kTwoStepVariant) {
            // two steps per pass: the call runs as a batch of one shot
            wave_shot one;
            std::memset(&one, 0, sizeof one);
            one.grid = *grid;
            one.m = m;
            one.eta = eta;
            if (src) one.src = *src;
            one.q = q;
            if (rec) one.rec = *rec;
            one.d = d;
            one.u_final = u_final;
            wave_opts o = *opts;
            o.flags &= ~WAVE_FLAG_PERSISTENT;
            return wave_forward_batch(1, &one, &o, stream);
        }
        int rc = setup(C, op, grid, m, eta, src, rec, opts, stream);
        if (rc) return rc;
        CkptView ck;
        if (ckpt) ck = ckpt_view(C.G, opts, ckpt);
        return run_forward(C, q, d, u_final, ckpt ? &ck : nullptr, true);
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_forward_noalloc(const wave_grid* grid, const float* m, const float* eta,
                         const wave_points* src, const float* q, const wave_points* rec, float* d,
                         float* u_final, void* stream)
{
    try {
        Ctx C;
        wave_opts o;
        std::memset(&o, 0, sizeof o);
        if (src && src->npts > 0 && !q) return fail(WAVE_EINVAL, "q is NULL with %d sources", src->npts);
        if (rec && rec->npts > 0 && !d) return fail(WAVE_EINVAL, "d is NULL with %d receivers", rec->npts);
        int rc = setup(C, WAVE_OP_FORWARD, grid, m, eta, src, rec, &o, stream, true);
        if (rc) return rc;
        return run_forward(C, q, d, u_final, nullptr, true);
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_adjoint(const wave_grid* grid, const float* m, const float* eta, const wave_points* rec,
                 const float* d, const wave_points* src, float* q_adj, float* v_final,
                 const wave_opts* opts, void* stream)
{
    try {
        Ctx C;
        if (src && src->npts > 0 && !q_adj) return fail(WAVE_EINVAL, "q_adj is NULL with %d sources", src->npts);
        if (rec && rec->npts > 0 && !d) return fail(WAVE_EINVAL, "d is NULL with %d receivers", rec->npts);
        int rc = setup(C, WAVE_OP_ADJOINT, grid, m, eta, src, rec, opts, stream);
        if (rc) return rc;
        const int64_t N = C.G.npad();
        float* v[2] = {C.at<float>(C.P.adj[0]), C.at<float>(C.P.adj[1])};
        HIP_TRY(launch_fill(v[0], N, 0.f, C.s));
        HIP_TRY(launch_fill(v[1], N, 0.f, C.s));
        StepArgs a = base_args(C);
        bind_sparse(C, a, 1);
        if (C.rec.npts) HIP_TRY(gather_first(C, a, 1, C.G.nt - 1, d + (size_t)(C.G.nt - 1) * C.rec.npts));
        int vc = 0;
        if (prof_begin(C.s)) return fail(WAVE_EHIP, "profiling event failed");
        for (int k = C.G.nt - 1; k >= 0; --k) {
            a.cur = v[vc];
            a.other = v[1 - vc];
            a.out = v[1 - vc];
            a.inj_val = C.rec.npts ? d + (size_t)k * C.rec.npts : nullptr;
            if (C.rec.npts) gathered(C, a, 1, k, k > 0 ? d + (size_t)(k - 1) * C.rec.npts : nullptr);
            a.smp_out = C.src.npts ? q_adj + (size_t)k * C.src.npts : nullptr;
            HIP_TRY(step(C, a));
            vc = 1 - vc;
        }
        if (prof_end(C.s)) return fail(WAVE_EHIP, "profiling event failed");
        // v[1 - vc] holds v^0 (the state sampled last)
        if (v_final)
            HIP_TRY(copy_out(v_final, v[1 - vc], C.G, C.s));
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_backward(const wave_grid* grid, const float* m, const float* eta, const wave_points* src,
                  const float* q, const wave_points* rec, const float* r, const void* ckpt,
                  float* grad_m, float* grad_q, const wave_opts* opts, void* stream)
{
    try {
        Ctx C;
        if (!ckpt) return fail(WAVE_EINVAL, "ckpt is NULL");
        if (!grad_m) return fail(WAVE_EINVAL, "grad_m is NULL");
        if (src && src->npts > 0 && !q) return fail(WAVE_EINVAL, "q is NULL with %d sources", src->npts);
        if (rec && rec->npts > 0 && !r) return fail(WAVE_EINVAL, "r is NULL with %d receivers", rec->npts);
        int rc = setup(C, WAVE_OP_BACKWARD, grid, m, eta, src, rec, opts, stream);
        if (rc) return rc;
        CkptView ck = ckpt_view(C.G, opts, const_cast<void*>(ckpt));
        return run_backward(C, q, r, ck, grad_m, grad_q, true);
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_gradient(const wave_grid* grid, const float* m, const float* eta, const wave_points* src,
                  const float* q, const wave_points* rec, const float* d_obs, float* grad,
                  float* misfit, float* d_syn, const wave_opts* opts, void* stream)
{
    try {
        Ctx C;
        if (!grad || !misfit || !d_obs) return fail(WAVE_EINVAL, "grad, misfit and d_obs are required");
        if (!rec || rec->npts <= 0) return fail(WAVE_EINVAL, "the gradient needs receivers");
        if (src && src->npts > 0 && !q) return fail(WAVE_EINVAL, "q is NULL with %d sources", src->npts);
        int rc = setup(C, WAVE_OP_GRADIENT, grid, m, eta, src, rec, opts, stream);
        if (rc) return rc;
        CkptView ck = ckpt_view(C.G, opts, C.at<void>(C.P.ckpt));
        float* dsyn = d_syn ? d_syn : C.at<float>(C.P.dsyn);
        rc = run_forward(C, q, dsyn, nullptr, &ck, false);
        if (rc) return rc;
        const int64_t nd = (int64_t)C.G.nt * C.rec.npts;
        float* resid = C.at<float>(C.P.resid);
        HIP_TRY(launch_residual(dsyn, d_obs, resid, nd, C.at<float>(C.P.red), kRedFloats, misfit, C.s));
        return run_backward(C, q, resid, ck, grad, nullptr, false);
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}


int wave_batch_workspace_size(int32_t nshots, const wave_shot* shots, const wave_opts* opts,
                              size_t* bytes)
{
    try {
        (void)opts;
        if (!bytes) return fail(WAVE_EINVAL, "bytes is NULL");
        BatchPlan B;
        const int rc = batch_plan(nshots, shots, &B, false);
        if (rc) return rc;
        *bytes = B.total;
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_forward_batch(int32_t nshots, const wave_shot* shots, const wave_opts* opts, void* stream)
{
    try {
        BatchPlan B;
        int rc = batch_plan(nshots, shots, &B, true);
        if (rc) return rc;
        if (!opts || !opts->workspace || reinterpret_cast<uintptr_t>(opts->workspace) % kAlign)
            return fail(WAVE_EWORKSPACE, "workspace missing or not %zu-byte aligned", kAlign);
        if (opts->workspace_bytes < B.total)
            return fail(WAVE_EWORKSPACE, "workspace too small: %zu bytes given, %zu needed",
                        opts->workspace_bytes, B.total);
        char* ws = static_cast<char*>(opts->workspace);
        hipStream_t st = static_cast<hipStream_t>(stream);
        if ((rc = batch_setup(B, shots, ws, st))) return rc;
        TileCfg cfg;
        const Geo& G0 = B.shots[0].G;
        if ((rc = pick_tile(opts, batch_key(B), G0, &cfg, true))) return rc;
        const bool persistent = (opts->flags & WAVE_FLAG_PERSISTENT) != 0;
        // the persistent kernel takes single steps: the two-step slab maps
        // to the one-step slab there
        if (persistent && G0.ndim == 2 && cfg.variant == kTwoStepVariant) cfg = TileCfg{3, kSlabRows};
        std::vector<ShotDesc> desc;
        std::vector<int64_t> begin;
        int64_t blocks = 0;
        build_descs(B, shots, ws, cfg, &desc, &begin, &blocks);
        if ((rc = upload_descs(desc, begin, ws, B, st))) return rc;
        if (prof_begin(st)) return fail(WAVE_EHIP, "profiling event failed");
        if (persistent)
            rc = run_batch_persistent(B, ws, cfg, blocks, st, !(opts->flags & WAVE_FLAG_NO_GRAPH));
        else
            rc = run_batch_loop(B, ws, cfg, blocks, st, !(opts->flags & WAVE_FLAG_NO_GRAPH));
        if (rc) return rc;
        if (prof_end(st)) return fail(WAVE_EHIP, "profiling event failed");
        int last = G0.nt & 1;
        if (G0.ndim == 2 && cfg.variant == kTwoStepVariant) (void)two_step_schedule(G0.nt, &last);
        for (int i = 0; i < nshots; ++i)
            if (shots[i].u_final) {
                const BatchShot& S = B.shots[i];
                HIP_TRY(copy_out(shots[i].u_final, reinterpret_cast<const float*>(ws + S.buf[last]), S.G, st));
            }
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_tune(const wave_grid* grid, const wave_opts* opts, int32_t steps, void* stream,
              int32_t* tile, double* us_per_step)
{
    try {
        Ctx C;
        if (!tile || !us_per_step || steps < 1) return fail(WAVE_EINVAL, "tile, us_per_step and steps >= 1 are required");
        int rc = make_geo(grid, &C.G);
        if (rc) return rc;
        C.P = make_plan(WAVE_OP_FORWARD, C.G, 0, 0, opts);
        if ((rc = check_ws(C.P, opts))) return rc;
        const bool imaging = (opts->flags & WAVE_FLAG_TUNE_IMAGING) != 0;
        C.ws = static_cast<char*>(opts->workspace);
        C.s = static_cast<hipStream_t>(stream);
        set_weights(C);
        const int64_t N = C.G.npad();
        for (size_t off : {C.P.alpha, C.P.beta, C.P.wf[0], C.P.wf[1]})
            HIP_TRY(launch_fill(C.at<float>(off), N, 0.f, C.s));
        StepArgs a = base_args(C);
        a.cur = C.at<float>(C.P.wf[0]);
        a.other = a.out = C.at<float>(C.P.wf[1]);
        if (imaging) {
            HIP_TRY(launch_fill(C.at<float>(C.P.ring), N, 0.f, C.s));
            HIP_TRY(launch_fill(C.at<float>(C.P.gacc), N, 0.f, C.s));
            a.img_fwd = C.at<float>(C.P.ring);
            a.img_grad = C.at<float>(C.P.gacc);
        }
        EventPair ev;
        HIP_TRY(hipEventCreate(&ev.a));
        HIP_TRY(hipEventCreate(&ev.b));
        double best = 1e300;
        TileCfg best_cfg;
        const bool verbose = std::getenv("WAVE_TUNE_VERBOSE") != nullptr;
        for (const TileCfg& cfg : tile_candidates(C.G.ndim, C.G.half, C.G.n[0], C.G.nzp)) {
            for (int w = 0; w < 2; ++w) HIP_TRY(launch_step(C.G.ndim, C.G.order, a, C.s, cfg));
            double t = 1e300;
            for (int rep = 0; rep < 3; ++rep) {
                HIP_TRY(hipEventRecord(ev.a, C.s));
                for (int i = 0; i < steps; ++i) HIP_TRY(launch_step(C.G.ndim, C.G.order, a, C.s, cfg));
                HIP_TRY(hipEventRecord(ev.b, C.s));
                HIP_TRY(hipEventSynchronize(ev.b));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
                t = std::min(t, 1e3 * ms / steps);
            }
            if (verbose)
                std::fprintf(stderr, "wave_tune %s: variant %d x-chunk %d: %.2f us\n",
                             imaging ? "imaging" : "step", cfg.variant, cfg.xchunk, t);
            if (t < best) { best = t; best_cfg = cfg; }
        }
        *tile = tile_id(best_cfg);
        *us_per_step = best;
        store_tile(tune_key(C.G, imaging), *tile);
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_tune_shot(const wave_grid* grid, const float* m, const float* eta, const wave_points* src,
                   const wave_points* rec, const wave_opts* opts, int32_t steps, void* stream,
                   int32_t* tile, double* us_per_step)
{
    // zero injection values and a sink for the sampled ones, the tuner's own
    struct DevBuf {
        float* p = nullptr;
        ~DevBuf() { if (p) { (void)hipDeviceSynchronize(); (void)hipFree(p); } }
    } vals;
    try {
        if (!tile || !us_per_step || steps < 1) return fail(WAVE_EINVAL, "tile, us_per_step and steps >= 1 are required");
        if (!opts) return fail(WAVE_EWORKSPACE, "opts is NULL (it carries the workspace)");
        const bool imaging = (opts->flags & WAVE_FLAG_TUNE_IMAGING) != 0;
        Ctx C;
        int rc = setup(C, imaging ? WAVE_OP_ADJOINT : WAVE_OP_FORWARD, grid, m, eta, src, rec, opts, stream);
        if (rc) return rc;
        // the forward injects sources and samples receivers, the imaging
        // adjoint the other way round
        const int set = imaging ? 1 : 0;
        const int ninj = imaging ? C.rec.npts : C.src.npts;
        const int nsmp = imaging ? C.src.npts : C.rec.npts;
        const size_t nv = (size_t)ninj + (size_t)nsmp + 1;
        HIP_TRY(hipMalloc(reinterpret_cast<void**>(&vals.p), nv * sizeof(float)));
        HIP_TRY(launch_fill(vals.p, (int64_t)nv, 0.f, C.s));
        const int64_t N = C.G.npad();
        float* pair[2] = {C.at<float>(imaging ? C.P.adj[0] : C.P.wf[0]),
                          C.at<float>(imaging ? C.P.adj[1] : C.P.wf[1])};
        for (float* f : pair) HIP_TRY(launch_fill(f, N, 0.f, C.s));
        StepArgs a = base_args(C);
        bind_sparse(C, a, set);
        a.cur = pair[0];
        a.other = a.out = pair[1];
        a.inj_val = ninj ? vals.p : nullptr;
        a.smp_out = nsmp ? vals.p + ninj : nullptr;
        if (imaging) {
            HIP_TRY(launch_fill(C.at<float>(C.P.ring), N, 0.f, C.s));
            HIP_TRY(launch_fill(C.at<float>(C.P.gacc), N, 0.f, C.s));
            a.img_fwd = C.at<float>(C.P.ring);
            a.img_grad = C.at<float>(C.P.gacc);
        }
        if (ninj) {
            HIP_TRY(gather_first(C, a, set, 0, vals.p));
            gathered(C, a, set, 0, vals.p);
        }
        EventPair ev;
        HIP_TRY(hipEventCreate(&ev.a));
        HIP_TRY(hipEventCreate(&ev.b));
        double best = 1e300;
        TileCfg best_cfg;
        const bool verbose = std::getenv("WAVE_TUNE_VERBOSE") != nullptr;
        for (const TileCfg& cfg : tile_candidates(C.G.ndim, C.G.half, C.G.n[0], C.G.nzp)) {
            for (int w = 0; w < 2; ++w) HIP_TRY(launch_step(C.G.ndim, C.G.order, a, C.s, cfg));
            double t = 1e300;
            for (int rep = 0; rep < 3; ++rep) {
                HIP_TRY(hipEventRecord(ev.a, C.s));
                for (int i = 0; i < steps; ++i) HIP_TRY(launch_step(C.G.ndim, C.G.order, a, C.s, cfg));
                HIP_TRY(hipEventRecord(ev.b, C.s));
                HIP_TRY(hipEventSynchronize(ev.b));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
                t = std::min(t, 1e3 * ms / steps);
            }
            if (verbose)
                std::fprintf(stderr, "wave_tune_shot %s: variant %d x-chunk %d: %.2f us\n",
                             imaging ? "imaging" : "step", cfg.variant, cfg.xchunk, t);
            if (t < best) { best = t; best_cfg = cfg; }
        }
        *tile = tile_id(best_cfg);
        *us_per_step = best;
        store_tile(tune_key(C.G, imaging), *tile);
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

int wave_tune_batch(int32_t nshots, const wave_shot* shots, const wave_opts* opts, int32_t steps,
                    void* stream, int32_t* tile, double* us_per_step)
{
    try {
        if (!tile || !us_per_step || steps < 1) return fail(WAVE_EINVAL, "tile, us_per_step and steps >= 1 are required");
        BatchPlan B;
        int rc = batch_plan(nshots, shots, &B, true);
        if (rc) return rc;
        if (!opts || !opts->workspace || reinterpret_cast<uintptr_t>(opts->workspace) % kAlign ||
            opts->workspace_bytes < B.total)
            return fail(WAVE_EWORKSPACE, "workspace missing, misaligned or too small");
        char* ws = static_cast<char*>(opts->workspace);
        hipStream_t st = static_cast<hipStream_t>(stream);
        if ((rc = batch_setup(B, shots, ws, st))) return rc;
        const Geo& G = B.shots[0].G;
        int64_t maxnx = 0;
        for (const BatchShot& S : B.shots) maxnx = std::max(maxnx, S.G.n[0]);
        EventPair ev;
        HIP_TRY(hipEventCreate(&ev.a));
        HIP_TRY(hipEventCreate(&ev.b));
        double best = 1e300;
        TileCfg best_cfg;
        const ShotDesc* d_desc = reinterpret_cast<const ShotDesc*>(ws + B.desc);
        const int64_t* d_begin = reinterpret_cast<const int64_t*>(ws + B.begin);
        const bool verbose = std::getenv("WAVE_TUNE_VERBOSE") != nullptr;
        for (const TileCfg& cfg : tile_candidates(G.ndim, G.half, maxnx, G.nzp, true)) {
            std::vector<ShotDesc> desc;
            std::vector<int64_t> begin;
            int64_t blocks = 0;
            build_descs(B, shots, ws, cfg, &desc, &begin, &blocks);
            for (ShotDesc& D : desc) { D.nsrc = 0; D.nrec = 0; D.d = nullptr; }   // no outputs touched
            if ((rc = upload_descs(desc, begin, ws, B, st))) return rc;
            // a two-step launch advances two levels: pass n reads buffers 0/1
            // and writes 3/2, timed per level
            const bool two = G.ndim == 2 && cfg.variant == kTwoStepVariant;
            auto once = [&](int i) {
                return two ? launch_batch2(G.order, d_desc, d_begin, nshots, blocks, 2 * i,
                                             0 | (1 << 2) | (3 << 4) | (2 << 6), 1, st)
                           : launch_batch(G.ndim, G.order, G.nzp, cfg, d_desc, d_begin, nshots, blocks, i, st);
            };
            const int launches = two ? (steps + 1) / 2 : steps;
            const int levels = two ? 2 * launches : steps;
            for (int w = 0; w < 2; ++w) HIP_TRY(once(w));
            double t = 1e300;
            for (int rep = 0; rep < 3; ++rep) {
                HIP_TRY(hipEventRecord(ev.a, st));
                for (int i = 0; i < launches; ++i) HIP_TRY(once(i));
                HIP_TRY(hipEventRecord(ev.b, st));
                HIP_TRY(hipEventSynchronize(ev.b));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
                t = std::min(t, 1e3 * ms / levels);
            }
            if (verbose)
                std::fprintf(stderr, "wave_tune_batch: variant %d x-chunk %d: %.2f us per step\n",
                             cfg.variant, cfg.xchunk, t);
            if (t < best) { best = t; best_cfg = cfg; }
        }
        *tile = tile_id(best_cfg);
        *us_per_step = best;
        store_tile(batch_key(B), *tile);
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}


int wave_diffusion(const wave_grid* grid, const float* a, const float* u0, float* u_final,
                   const wave_opts* opts, void* stream)
{
    try {
        Ctx C;
        int rc = make_geo(grid, &C.G);
        if (rc) return rc;
        if (!a || !u0 || !u_final) return fail(WAVE_EINVAL, "a, u0 and u_final are required");
        C.P = make_plan(WAVE_OP_FORWARD, C.G, 0, 0, opts);
        if ((rc = check_ws(C.P, opts))) return rc;
        C.ws = static_cast<char*>(opts->workspace);
        C.s = static_cast<hipStream_t>(stream);
        if ((rc = pick_tile(opts, tune_key(C.G, false), C.G, &C.cfg))) return rc;
        set_weights(C);
        const int64_t N = C.G.npad();
        char* host = nullptr;
        if ((rc = staging((size_t)kCheckBlocks * 2 * 4, &host))) return rc;
        float* part = reinterpret_cast<float*>(host);
        HIP_TRY(launch_diffusion_coef(a, C.G.nrows(), C.G.n[2], C.G.nzp, C.at<float>(C.P.check),
                                      kCheckBlocks, C.at<float>(C.P.alpha), C.at<float>(C.P.beta),
                                      C.G.dt, C.s));
        HIP_TRY(hipMemcpyAsync(part, C.at<float>(C.P.check), (size_t)kCheckBlocks * 2 * 4,
                               hipMemcpyDeviceToHost, C.s));
        HIP_TRY(hipEventRecord(TS().stage.done, C.s));
        HIP_TRY(hipStreamSynchronize(C.s));
        float amax = 0.f, bad = 0.f;
        for (int b = 0; b < kCheckBlocks; ++b) {
            amax = std::max(amax, part[2 * b]);
            bad += part[2 * b + 1];
        }
        if (bad > 0) return fail(WAVE_EINVAL, "%.0f entries of a are invalid (need finite, >= 0)", bad);
        // forward Euler is stable while dt a max|lambda(L)| <= 2
        double c[kMaxHalf + 1];
        fd_weights(C.G.half, c);
        double S = std::fabs(c[0]);
        for (int j = 1; j <= C.G.half; ++j) S += 2.0 * std::fabs(c[j]);
        double lam = 0;
        for (int ax = 0; ax < 3; ++ax)
            if (C.G.ndim == 3 || ax != 1) lam += S / (C.G.h[ax] * C.G.h[ax]);
        if (C.G.dt * amax * lam > 2.0 * (1 + 1e-12))
            return fail(WAVE_ECFL, "dt = %.9g exceeds the forward-Euler bound %.9g", C.G.dt,
                        2.0 / (amax * lam));
        float* buf[2] = {C.at<float>(C.P.wf[0]), C.at<float>(C.P.wf[1])};
        if (C.G.nzp != C.G.n[2]) HIP_TRY(launch_fill(buf[0], N, 0.f, C.s));
        HIP_TRY(copy_in(buf[0], u0, C.G, C.s));
        HIP_TRY(launch_fill(buf[1], N, 0.f, C.s));
        StepArgs sa = base_args(C);
        sa.no_prev = 1;                      // beta = 0: neither u^{n-1} nor beta is read
        if (prof_begin(C.s)) return fail(WAVE_EHIP, "profiling event failed");
        for (int n = 0; n < C.G.nt; ++n) {
            sa.cur = buf[n & 1];
            sa.other = buf[(n + 1) & 1];
            sa.out = buf[(n + 1) & 1];
            HIP_TRY(step(C, sa));
        }
        if (prof_end(C.s)) return fail(WAVE_EHIP, "profiling event failed");
        HIP_TRY(copy_out(u_final, buf[C.G.nt & 1], C.G, C.s));
        return WAVE_OK;
    } catch (const std::exception& e) {
        return fail(WAVE_EINVAL, "exception: %s", e.what());
    } catch (...) {
        return fail(WAVE_EINVAL, "unknown exception");
    }
}

}  // extern "C"
