// gfx950 kernels of the damped acoustic leapfrog step.
//
// One launch = one time step of the solved update (paper, Section "Seismic
// Inversion Example", listing "lst:wave"):
//   out = cur + beta (cur - other) + alpha L cur   (+ alpha sum w val at injected nodes)
// with alpha = dt^2/(m + eta dt/2), beta = (m - eta dt/2)/(m + eta dt/2);
// algebraically this is (2 m cur - (m - eta dt/2) other + dt^2 L cur)/(m + eta dt/2).
// L is evaluated as sum_axes sum_j c_j ((u[+j] + u[-j]) - 2 u[0]): the
// centre weight never appears, so the FP32 stencil annihilates constants
// exactly whatever the rounding of c_j.
// Blocks past `stencil_blocks` sample `cur` at the sparse points (Section
// "Sparse point interpolation"): `cur` is read-only during the step, so the
// sampling needs no ordering with the update.
#include "wave_internal.h"

namespace wave {

namespace {

constexpr int kBlock = 256;

template <int DIM>
__device__ __forceinline__ float sample_point(const SampleSet& s, const float* __restrict__ u,
                                              int64_t p, int64_t sy, int64_t sx)
{
    const int64_t b = s.base[p];
    const float* w = s.w + p * (1 << DIM);
    float acc = 0.f;
    if (DIM == 2) {
        // corners (x, z): 00, 01, 10, 11
        acc = fmaf(w[0], u[b], acc);
        acc = fmaf(w[1], u[b + 1], acc);
        acc = fmaf(w[2], u[b + sx], acc);
        acc = fmaf(w[3], u[b + sx + 1], acc);
    } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t off = ((c >> 2) & 1) * sx + ((c >> 1) & 1) * sy + (c & 1);
            acc = fmaf(w[c], u[b + off], acc);
        }
    }
    return acc;
}

template <int DIM, int R, bool IMG>
__global__ __launch_bounds__(kBlock) void k_step_naive(StepArgs a)
{
    const int64_t nz = a.nz, ny = a.ny, nx = a.nx;
    const int64_t sy = nz, sx = ny * nz;
    if ((int64_t)blockIdx.x >= a.stencil_blocks) {
        const int64_t p = ((int64_t)blockIdx.x - a.stencil_blocks) * kBlock + threadIdx.x;
        if (p < a.smp.npts) a.smp_out[p] = sample_point<DIM>(a.smp, a.cur, p, sy, sx);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nx * sx) return;
    const int64_t z = i % nz;
    const int64_t rest = i / nz;
    const int64_t y = rest % ny;
    const int64_t x = rest / ny;
    const float* __restrict__ u = a.cur;
    const float u0 = u[i];
    const float m2u0 = -2.f * u0;
    float lap = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        const float p = (x + j < nx) ? u[i + j * sx] : 0.f;
        const float m = (x - j >= 0) ? u[i - j * sx] : 0.f;
        lap = fmaf(a.cx[j], (p + m) + m2u0, lap);
    }
    if (DIM == 3) {
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const float p = (y + j < ny) ? u[i + j * sy] : 0.f;
            const float m = (y - j >= 0) ? u[i - j * sy] : 0.f;
            lap = fmaf(a.cy[j], (p + m) + m2u0, lap);
        }
    }
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        const float p = (z + j < nz) ? u[i + j] : 0.f;
        const float m = (z - j >= 0) ? u[i - j] : 0.f;
        lap = fmaf(a.cz[j], (p + m) + m2u0, lap);
    }
    const float prev = a.other[i];
    const float al = a.alpha[i];
    float v = fmaf(a.beta[i], u0 - prev, u0);
    v = fmaf(al, lap, v);
    if (a.inj_val) {
        const int64_t row = x * ny + y;
        const int32_t e0 = a.inj.row_ptr[row], e1 = a.inj.row_ptr[row + 1];
        if (e0 != e1) {
            float acc = 0.f;
            bool hit = false;
            for (int32_t e = e0; e < e1; ++e) {
                const InjEntry en = a.inj.ent[e];
                if (en.z == (int32_t)z) {
                    acc = fmaf(en.w, a.inj_val[en.pt], acc);
                    hit = true;
                }
            }
            if (hit) v = fmaf(al, acc, v);
        }
    }
    if (IMG) {
        const float d2 = (prev + v) + m2u0;
        a.img_grad[i] = fmaf(-a.img_fwd[i] * a.inv_dt2, d2, a.img_grad[i]);
    }
    a.out[i] = v;
}

template <int DIM, int R>
hipError_t launch_step_t(const StepArgs& a0, hipStream_t s)
{
    StepArgs a = a0;
    const int64_t n = a.nx * a.ny * a.nz;
    a.stencil_blocks = (n + kBlock - 1) / kBlock;
    int64_t nsb = 0;
    if (a.smp_out && a.smp.npts > 0) nsb = (a.smp.npts + kBlock - 1) / kBlock;
    else a.smp.npts = 0;
    const int64_t blocks = a.stencil_blocks + nsb;
    if (a.img_grad)
        hipLaunchKernelGGL((k_step_naive<DIM, R, true>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_step_naive<DIM, R, false>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_dim(int order, const StepArgs& a, hipStream_t s)
{
    switch (order) {
    case 2: return launch_step_t<DIM, 1>(a, s);
    case 4: return launch_step_t<DIM, 2>(a, s);
    case 6: return launch_step_t<DIM, 3>(a, s);
    case 8: return launch_step_t<DIM, 4>(a, s);
    case 10: return launch_step_t<DIM, 5>(a, s);
    case 12: return launch_step_t<DIM, 6>(a, s);
    case 14: return launch_step_t<DIM, 7>(a, s);
    case 16: return launch_step_t<DIM, 8>(a, s);
    default: return hipErrorInvalidValue;
    }
}

__global__ __launch_bounds__(kBlock) void k_coefficients(const float* __restrict__ m,
                                                         const float* __restrict__ eta,
                                                         float* __restrict__ alpha,
                                                         float* __restrict__ beta, int64_t n,
                                                         float dt)
{
    const float hdt = 0.5f * dt, dt2 = dt * dt;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const float mm = m[i];
        const float e = eta ? eta[i] * hdt : 0.f;
        const float a = mm + e;
        alpha[i] = dt2 / a;
        beta[i] = (mm - e) / a;
    }
}

__global__ __launch_bounds__(kBlock) void k_check_fields(const float* __restrict__ m,
                                                         const float* __restrict__ eta,
                                                         int64_t n, float* __restrict__ partial)
{
    __shared__ float smin_m[kBlock], smin_e[kBlock], sbad[kBlock];
    float mn = INFINITY, en = INFINITY, bad = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const float mm = m[i];
        if (!(mm > 0.f) || !isfinite(mm)) bad += 1.f;
        else mn = fminf(mn, mm);
        if (eta) {
            const float e = eta[i];
            if (!(e >= 0.f) || !isfinite(e)) bad += 1.f;
            else en = fminf(en, e);
        }
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
        r[i] = v;
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

int grid_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

hipError_t launch_step(int ndim, int order, const StepArgs& a, hipStream_t s)
{
    if (ndim == 2) return launch_dim<2>(order, a, s);
    if (ndim == 3) return launch_dim<3>(order, a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_coefficients(const float* m, const float* eta, float* alpha, float* beta,
                               int64_t n, float dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_coefficients, dim3(grid_for(n)), dim3(kBlock), 0, s, m, eta, alpha,
                       beta, n, dt);
    return hipGetLastError();
}

hipError_t launch_check_fields(const float* m, const float* eta, int64_t n, float* partial,
                               int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_fields, dim3(nblocks), dim3(kBlock), 0, s, m, eta, n, partial);
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

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace wave
