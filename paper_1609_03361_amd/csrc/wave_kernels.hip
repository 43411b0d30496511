// gfx950 kernels around the step: field checks and step coefficients, the
// diffusion coefficients, fills, the misfit reduction and the checkpoint
// codec, plus the dispatch over the space order to the step kernels (each
// order in its own translation unit, wave_o<order>.hip, from wave_step.h).
#include <algorithm>
#include <mutex>

#include <hip/hip_fp16.h>

#include "wave_internal.h"

namespace wave {

// Workspace of wave_forward_noalloc: a device array of the library's own, so
// that the call allocates nothing.  Host code never uses the array's name as
// an address (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[kNoAllocBytes];

hipError_t noalloc_scratch(void** ptr)
{
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

namespace {

constexpr int kBlock = 256;

template <int VZ>
using Vec = float __attribute__((ext_vector_type(VZ)));

template <int VZ>
__device__ __forceinline__ Vec<VZ> vload(const float* p)
{
    return *reinterpret_cast<const Vec<VZ>*>(p);
}

template <int VZ>
__device__ __forceinline__ void vstore(float* p, const Vec<VZ>& v)
{
    *reinterpret_cast<Vec<VZ>*>(p) = v;
}

// Index of padded element j ([rows][nzp]) in the unpadded caller array
// ([rows][nz]), or -1 for a padding column.
__device__ __forceinline__ int64_t unpadded(int64_t j, int64_t nz, int64_t nzp)
{
    if (nz == nzp) return j;
    const int64_t row = j / nzp, z = j - row * nzp;
    return z < nz ? row * nz + z : -1;
}

__global__ __launch_bounds__(kBlock) void k_check_fields(const float* __restrict__ m,
                                                         const float* __restrict__ eta,
                                                         int64_t rows, int64_t nz, int64_t nzp,
                                                         float* __restrict__ partial,
                                                         float* __restrict__ alpha,
                                                         float* __restrict__ beta, double dt)
{
    // The coefficients are formed in FP64 and rounded once to FP32: the same
    // rounding of dt^2 or of m + eta dt/2 at every point of a layer would act
    // as a small systematic change of velocity, whose phase error grows with
    // the number of steps.
    __shared__ float smin_m[kBlock], smin_e[kBlock], sbad[kBlock];
    float mn = INFINITY, en = INFINITY, bad = 0.f;
    const double hdt = 0.5 * dt, dt2 = dt * dt;
    const int64_t n = rows * nzp;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const int64_t i = unpadded(j, nz, nzp);
        if (i < 0) {
            alpha[j] = 0.f;
            beta[j] = 0.f;
            continue;
        }
        const float mm = m[i];
        if (!(mm > 0.f) || !isfinite(mm)) bad += 1.f;
        else mn = fminf(mn, mm);
        double e = 0.0;
        if (eta) {
            const float ef = eta[i];
            if (!(ef >= 0.f) || !isfinite(ef)) bad += 1.f;
            else en = fminf(en, ef);
            e = (double)ef * hdt;
        }
        const double am = (double)mm + e;
        alpha[j] = (float)(dt2 / am);
        beta[j] = (float)(((double)mm - e) / am);
    }
    smin_m[threadIdx.x] = mn;
    smin_e[threadIdx.x] = en;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smin_m[threadIdx.x] = fminf(smin_m[threadIdx.x], smin_m[threadIdx.x + w]);
            smin_e[threadIdx.x] = fminf(smin_e[threadIdx.x], smin_e[threadIdx.x + w]);
            sbad[threadIdx.x] += sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x + 0] = smin_m[0];
        partial[3 * blockIdx.x + 1] = smin_e[0];
        partial[3 * blockIdx.x + 2] = sbad[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_fill(float* __restrict__ p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

// Diffusion set-up: per block {max a, count of invalid a} and the step
// coefficients of forward Euler written in the leapfrog form of the step
// kernel: alpha = dt a, beta = 0, so out = cur + dt a L cur.
__global__ __launch_bounds__(kBlock) void k_diffusion_coef(const float* __restrict__ a, int64_t rows,
                                                           int64_t nz, int64_t nzp,
                                                           float* __restrict__ partial,
                                                           float* __restrict__ alpha,
                                                           float* __restrict__ beta, double dt)
{
    __shared__ float smax[kBlock], sbad[kBlock];
    float mx = 0.f, bad = 0.f;
    const int64_t n = rows * nzp;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const int64_t i = unpadded(j, nz, nzp);
        beta[j] = 0.f;
        if (i < 0) {
            alpha[j] = 0.f;
            continue;
        }
        const float v = a[i];
        if (!(v >= 0.f) || !isfinite(v)) bad += 1.f;
        else mx = fmaxf(mx, v);
        alpha[j] = (float)(dt * (double)v);
    }
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + w]);
            sbad[threadIdx.x] += sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x + 0] = smax[0];
        partial[2 * blockIdx.x + 1] = sbad[0];
    }
}

// r = d - d_obs and per-block partial sums of r^2 (grid-stride, fixed order).
__global__ __launch_bounds__(kBlock) void k_residual(const float* __restrict__ d,
                                                     const float* __restrict__ dobs,
                                                     float* __restrict__ r, int64_t n,
                                                     float* __restrict__ partial)
{
    __shared__ float sh[kBlock];
    float acc = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const float v = d[i] - dobs[i];
        if (r) r[i] = v;
        acc = fmaf(v, v, acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// J = 1/2 sum of the partials (one block, fixed order).
__global__ __launch_bounds__(kBlock) void k_sum_half(const float* __restrict__ partial, int np,
                                                     float* __restrict__ out)
{
    __shared__ float sh[kBlock];
    float acc = 0.f;
    for (int i = threadIdx.x; i < np; i += kBlock) acc += partial[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = 0.5f * sh[0];
}

// ---------------------------------------------------------------------------
// Checkpoint codec.  A reduced-precision checkpoint of the pair (u^c, u^{c-1})
// stores u^c and the increment d = u^c - u^{c-1}, each as BF16 or FP16 of
// (value * s) with its own power-of-two scale s, chosen so that max|value| * s
// lies in [2^14, 2^15): the products are exact and FP16 cannot overflow.
// Restoring gives u^c = stored_u / s_u and u^{c-1} = u^c - stored_d / s_d, so
// the restart velocity carries the relative error of one rounding of d.
// slot layout per checkpoint: {s_u, s_d, max|u| bits, max|d| bits}.
// ---------------------------------------------------------------------------
// FP32 -> BF16 with round to nearest, ties to even, by integer rounding of the
// bit pattern: add 0x7fff plus the lowest kept bit, then truncate to the upper
// 16 bits (a carry out of the mantissa moves to the exponent, as rounding up
// must).  NaN stays a quiet NaN; infinities pass unchanged.
__device__ __forceinline__ unsigned short f32_to_bf16_rn(float x)
{
    unsigned int b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u) return (unsigned short)((b >> 16) | ((b & 0xffffu) ? 0x40u : 0u));
    b += 0x7fffu + ((b >> 16) & 1u);
    return (unsigned short)(b >> 16);
}

__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

__device__ __forceinline__ float scale_for(unsigned int maxbits)
{
    const float mx = __uint_as_float(maxbits);
    if (!(mx > 0.f) || !isfinite(mx)) return 1.f;
    int k;
    (void)frexpf(mx, &k);          // mx = f 2^k, f in [0.5, 1)
    int e = 15 - k;                // mx 2^e in [2^14, 2^15)
    e = e < -120 ? -120 : (e > 120 ? 120 : e);
    return ldexpf(1.f, e);
}

// Per block {max |u|, max |u - prev|} into partial[2b], partial[2b+1].
__global__ __launch_bounds__(kBlock) void k_ckpt_max(const float* __restrict__ cur,
                                                     const float* __restrict__ prev, int64_t n,
                                                     float* __restrict__ partial)
{
    __shared__ float sa[kBlock], sd[kBlock];
    float ma = 0.f, md = 0.f;
    const int64_t n4 = n / 4;      // n is a multiple of 4 (padded rows)
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kBlock) {
        const Vec<4> c = vload<4>(cur + 4 * i), p = vload<4>(prev + 4 * i);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            ma = fmaxf(ma, fabsf(c[v]));
            md = fmaxf(md, fabsf(c[v] - p[v]));
        }
    }
    sa[threadIdx.x] = ma;
    sd[threadIdx.x] = md;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] = fmaxf(sa[threadIdx.x], sa[threadIdx.x + w]);
            sd[threadIdx.x] = fmaxf(sd[threadIdx.x], sd[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sa[0];
        partial[2 * blockIdx.x + 1] = sd[0];
    }
}

// One block: the maxima over the per-block partials, and the two scales,
// into the checkpoint's slot (no atomics, so the order never matters).
__global__ __launch_bounds__(kBlock) void k_ckpt_scale(const float* __restrict__ partial, int nb,
                                                       unsigned int* __restrict__ slot)
{
    __shared__ float sa[kBlock], sd[kBlock];
    float ma = 0.f, md = 0.f;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        ma = fmaxf(ma, partial[2 * b]);
        md = fmaxf(md, partial[2 * b + 1]);
    }
    sa[threadIdx.x] = ma;
    sd[threadIdx.x] = md;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] = fmaxf(sa[threadIdx.x], sa[threadIdx.x + w]);
            sd[threadIdx.x] = fmaxf(sd[threadIdx.x], sd[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned int bu = __float_as_uint(sa[0]), bd = __float_as_uint(sd[0]);
        reinterpret_cast<float*>(slot)[0] = scale_for(bu);
        reinterpret_cast<float*>(slot)[1] = scale_for(bd);
        slot[2] = bu;
        slot[3] = bd;
    }
}

template <bool BF16>
__global__ __launch_bounds__(kBlock) void k_ckpt_encode(const float* __restrict__ cur,
                                                        const float* __restrict__ prev, int64_t n,
                                                        const unsigned int* __restrict__ slot,
                                                        unsigned short* __restrict__ out_u,
                                                        unsigned short* __restrict__ out_d)
{
    const float su = reinterpret_cast<const float*>(slot)[0];
    const float sd = reinterpret_cast<const float*>(slot)[1];
    using U4 = unsigned short __attribute__((ext_vector_type(4)));
    const int64_t n4 = n / 4;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kBlock) {
        const Vec<4> c = vload<4>(cur + 4 * i), p = vload<4>(prev + 4 * i);
        U4 eu, ed;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float d = c[v] - p[v];
            if (BF16) {
                eu[v] = f32_to_bf16_rn(c[v] * su);
                ed[v] = f32_to_bf16_rn(d * sd);
            } else {
                eu[v] = __half_as_ushort(__float2half_rn(c[v] * su));
                ed[v] = __half_as_ushort(__float2half_rn(d * sd));
            }
        }
        *reinterpret_cast<U4*>(out_u + 4 * i) = eu;
        *reinterpret_cast<U4*>(out_d + 4 * i) = ed;
    }
}

template <bool BF16>
__global__ __launch_bounds__(kBlock) void k_ckpt_decode(const unsigned short* __restrict__ in_u,
                                                        const unsigned short* __restrict__ in_d,
                                                        const float* __restrict__ slot, int64_t n,
                                                        float* __restrict__ cur,
                                                        float* __restrict__ prev)
{
    const float iu = 1.f / slot[0], id = 1.f / slot[1];   // exact: powers of two
    using U4 = unsigned short __attribute__((ext_vector_type(4)));
    const int64_t n4 = n / 4;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kBlock) {
        const U4 eu = *reinterpret_cast<const U4*>(in_u + 4 * i);
        const U4 ed = *reinterpret_cast<const U4*>(in_d + 4 * i);
        Vec<4> c, p;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float u = BF16 ? bf16_to_f32(eu[v]) : __half2float(__ushort_as_half(eu[v]));
            const float d = BF16 ? bf16_to_f32(ed[v]) : __half2float(__ushort_as_half(ed[v]));
            c[v] = u * iu;
            p[v] = c[v] - d * id;
        }
        vstore<4>(cur + 4 * i, c);
        vstore<4>(prev + 4 * i, p);
    }
}

int grid_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

int tile_variants(int ndim, int64_t)
{
    return ndim == 2 ? (int)(sizeof kShapes2D / sizeof kShapes2D[0])
                     : (int)(sizeof kShapes3D / sizeof kShapes3D[0]);
}

int max_xchunk(int ndim, int variant)
{
    if (ndim == 2 && variant == 3) return kSlabRows;
    return 1 << 30;
}

int default_variant(int ndim, int order, int64_t ny, int64_t nz)
{
    if (ndim == 2) return 3;      // the slab body (2001 x 801 order 8: 8.7 us against 10.9 us per step)
    // Candidates in order of preference at equal lane waste: up to order 8
    // the two-point-lane tile first (256^3 order 8: 52.2 us against 53.8 us
    // for 64 z x 16 rows of four-point lanes); at orders 14 and 16 the
    // two-point-lane 64 z x 16 tile (512^3 order 16, real fields: 470 us with
    // x-chunks of 256 planes against 520 us for 64 z x 16 of four-point lanes).
    const int pref[] = {5, 0, 1, 2, 3, 4, 6, 7, 8, 9, 10};
    const int base[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10};
    const int high[] = {7, 0, 1, 2, 3, 4, 5, 6, 8, 9, 10};
    static_assert(sizeof pref / sizeof pref[0] == sizeof kShapes3D / sizeof kShapes3D[0], "");
    static_assert(sizeof high / sizeof high[0] == sizeof kShapes3D / sizeof kShapes3D[0], "");
    const int* order_of = order <= 8 ? pref : (order >= 14 ? high : base);
    int best = 0;
    double best_eff = -1.0;
    for (int k = 0; k < tile_variants(3, nz); ++k) {
        const int v = order_of[k];
        const BlockShape& S = kShapes3D[v];
        const int64_t TZ = (int64_t)S.vz * S.tzl, TY = S.ty, NT = (int64_t)S.tzl * S.ty;
        const double fz = (double)nz / (double)(((nz + TZ - 1) / TZ) * TZ);
        const double fy = (double)ny / (double)(((ny + TY - 1) / TY) * TY);
        const double fw = (double)NT / (double)(((NT + 63) / 64) * 64);
        const double eff = fz * fy * fw;
        if (eff > best_eff + 1e-9) { best_eff = eff; best = v; }
    }
    return best;
}

// Order dispatch: each space order's kernels live in their own translation unit.
#ifdef WAVE_ONLY_ORDER
#define WAVE_ORDERS(X) X(WAVE_ONLY_ORDER)      // experimental builds of one order
#else
#define WAVE_ORDERS(X) X(2) X(4) X(6) X(8) X(10) X(12) X(14) X(16)
#endif

int64_t plan_tiles(int ndim, int order, TileCfg cfg, StepArgs& a, bool device)
{
#define WAVE_CASE(O) case O: return OrderOps<O>::plan(ndim, cfg, a, device);
    switch (order) { WAVE_ORDERS(WAVE_CASE) default: return -1; }
#undef WAVE_CASE
}

hipError_t launch_step(int ndim, int order, const StepArgs& a, hipStream_t s, TileCfg cfg)
{
#define WAVE_CASE(O) case O: return OrderOps<O>::step(ndim, a, s, cfg);
    switch (order) { WAVE_ORDERS(WAVE_CASE) default: return hipErrorInvalidValue; }
#undef WAVE_CASE
}

hipError_t launch_batch(int ndim, int order, int64_t nz_any, TileCfg cfg, const ShotDesc* shots,
                        const int64_t* begin, int32_t nshots, int64_t blocks, int32_t n,
                        hipStream_t s)
{
#define WAVE_CASE(O) case O: return OrderOps<O>::batch(ndim, nz_any, cfg, shots, begin, nshots, blocks, n, s);
    switch (order) { WAVE_ORDERS(WAVE_CASE) default: return hipErrorInvalidValue; }
#undef WAVE_CASE
}

hipError_t launch_batch2(int order, const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                         int64_t blocks, int32_t n, int32_t bufs, int32_t flags, hipStream_t s)
{
#define WAVE_CASE(O) case O: return OrderOps<O>::batch2(shots, begin, nshots, blocks, n, bufs, flags, s);
    switch (order) { WAVE_ORDERS(WAVE_CASE) default: return hipErrorInvalidValue; }
#undef WAVE_CASE
}

hipError_t launch_batch_persistent(int ndim, int order, int64_t nz_any, TileCfg cfg,
                                   const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                                   int64_t items, int32_t nt, unsigned int* sync, int32_t spin_limit,
                                   int* grid_used, hipStream_t s)
{
#define WAVE_CASE(O) case O: return OrderOps<O>::persistent(ndim, nz_any, cfg, shots, begin, nshots, items, nt, sync, spin_limit, grid_used, s);
    switch (order) { WAVE_ORDERS(WAVE_CASE) default: return hipErrorInvalidValue; }
#undef WAVE_CASE
}

hipError_t graph_batch_persistent(int ndim, int order, int64_t nz_any, TileCfg cfg,
                                  const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                                  int64_t items, int32_t nt, unsigned int* sync, int32_t spin_limit,
                                  int* grid_used, hipGraph_t* graph)
{
#define WAVE_CASE(O) case O: return OrderOps<O>::persistent_graph(ndim, nz_any, cfg, shots, begin, nshots, items, nt, sync, spin_limit, grid_used, graph);
    switch (order) { WAVE_ORDERS(WAVE_CASE) default: return hipErrorInvalidValue; }
#undef WAVE_CASE
}

hipError_t launch_check_fields(const float* m, const float* eta, int64_t rows, int64_t nz,
                               int64_t nzp, float* partial, int nblocks, float* alpha, float* beta,
                               double dt, hipStream_t s)
{
    if (nzp < nz || nzp % 4 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_check_fields, dim3(nblocks), dim3(kBlock), 0, s, m, eta, rows, nz, nzp,
                       partial, alpha, beta, dt);
    return hipGetLastError();
}

hipError_t launch_residual(const float* d, const float* dobs, float* r, int64_t n, float* partial,
                           int nblocks, float* misfit, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, dim3(nblocks), dim3(kBlock), 0, s, d, dobs, r, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_half, dim3(1), dim3(kBlock), 0, s, partial, nblocks, misfit);
    return hipGetLastError();
}

hipError_t launch_ckpt_encode(const float* cur, const float* prev, int64_t n, int bf16,
                              unsigned int* slot, float* partial, int nblocks,
                              unsigned short* out_u, unsigned short* out_d, hipStream_t s)
{
    if (n % 4 != 0 || nblocks < 1) return hipErrorInvalidValue;
    const int nb = std::min(nblocks, grid_for(n / 4));
    hipLaunchKernelGGL(k_ckpt_max, dim3(nb), dim3(kBlock), 0, s, cur, prev, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ckpt_scale, dim3(1), dim3(kBlock), 0, s, partial, nb, slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (bf16)
        hipLaunchKernelGGL(k_ckpt_encode<true>, dim3(grid_for(n / 4)), dim3(kBlock), 0, s, cur, prev,
                           n, slot, out_u, out_d);
    else
        hipLaunchKernelGGL(k_ckpt_encode<false>, dim3(grid_for(n / 4)), dim3(kBlock), 0, s, cur, prev,
                           n, slot, out_u, out_d);
    return hipGetLastError();
}

hipError_t launch_ckpt_decode(const unsigned short* in_u, const unsigned short* in_d,
                              const unsigned int* slot, int64_t n, int bf16, float* cur, float* prev,
                              hipStream_t s)
{
    if (n % 4 != 0) return hipErrorInvalidValue;
    const float* sl = reinterpret_cast<const float*>(slot);
    if (bf16)
        hipLaunchKernelGGL(k_ckpt_decode<true>, dim3(grid_for(n / 4)), dim3(kBlock), 0, s, in_u,
                           in_d, sl, n, cur, prev);
    else
        hipLaunchKernelGGL(k_ckpt_decode<false>, dim3(grid_for(n / 4)), dim3(kBlock), 0, s, in_u,
                           in_d, sl, n, cur, prev);
    return hipGetLastError();
}

hipError_t launch_diffusion_coef(const float* a, int64_t rows, int64_t nz, int64_t nzp,
                                 float* partial, int nblocks, float* alpha, float* beta, double dt,
                                 hipStream_t s)
{
    if (nzp < nz || nzp % 4 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_diffusion_coef, dim3(nblocks), dim3(kBlock), 0, s, a, rows, nz, nzp,
                       partial, alpha, beta, dt);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_gather(float* __restrict__ ev, const float* __restrict__ val,
                                                   const InjEntry* __restrict__ ent, int32_t nent)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < nent) ev[e] = ent[e].w * val[ent[e].pt];
}

hipError_t launch_gather(float* ev, const float* val, const InjEntry* ent, int32_t nent, hipStream_t s)
{
    if (nent <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((nent + kBlock - 1) / kBlock), dim3(kBlock), 0, s, ev, val, ent, nent);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace wave
