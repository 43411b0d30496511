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
#include <algorithm>
#include <atomic>
#include "wave_internal.h"

#include <hip/hip_fp16.h>

#include <utility>

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

// ---------------------------------------------------------------------------
// 2.5D streaming step.  A block owns a (TY x TZ) tile of the (y, z) plane and
// walks an x-chunk plane by plane.  Each thread keeps the 2R+1 x-neighbours of
// its VZ consecutive z-points in a register queue (plus one slot being
// filled), so the x part of the stencil costs no memory traffic; the current
// plane with its y and z halos is staged in a double-buffered LDS tile for the
// y and z parts.  The next plane's global loads are issued before the current
// plane is computed.  Arithmetic per point, in order: x terms, y terms, z terms,
// each lap = fma(c_j, (u[+j] + u[-j]) - 2 u[0], lap); then
// out = fma(alpha, lap, fma(beta, u - other, u)).
// ---------------------------------------------------------------------------
template <int VZ>
using Vec = float __attribute__((ext_vector_type(VZ)));

template <int VZ>
__device__ __forceinline__ Vec<VZ> vzero()
{
    return Vec<VZ>(0.f);
}

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

// Operands touched once per step (previous level, coefficients, output).
// With NT they carry the non-temporal hint, which keeps them from evicting
// wavefield planes that later tiles re-read; measured on gfx950 it pays only
// where the halos are not loaded early (see Tile::LEAD).
template <int VZ, bool NT>
__device__ __forceinline__ Vec<VZ> vload_once(const float* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const Vec<VZ>*>(p));
    else return *reinterpret_cast<const Vec<VZ>*>(p);
}

template <int VZ, bool NT>
__device__ __forceinline__ void vstore_once(float* p, const Vec<VZ>& v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<Vec<VZ>*>(p));
    else *reinterpret_cast<Vec<VZ>*>(p) = v;
}

// Wait for this wave's LDS traffic, then meet the block at the barrier.
// Outstanding global loads stay in flight across it (no vmcnt wait).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// smallest divisor of s that is at least want (s itself if none is smaller)
constexpr int pre_ring(int s, int want)
{
    for (int r = want; r < s; ++r)
        if (s % r == 0) return r;
    return s;
}

template <int DIM, int R, int VZ, int TZL, int TY>
struct Tile {
    static constexpr int NT = TZL * TY;
    static constexpr int TZ = TZL * VZ;
    static constexpr int RZ = (R + VZ - 1) / VZ * VZ;       // z halo, whole vectors
    static constexpr int PITCH = TZ + 2 * RZ;
    static constexpr int ROWS = DIM == 3 ? TY + 2 * R : TY;
    static constexpr int NHY = DIM == 3 ? 2 * R * TZL : 0;   // y-halo vectors per plane
    static constexpr int NHZ = TY * 2 * (RZ / VZ);          // z-halo vectors per plane
    static constexpr int KH = (NHY + NHZ + NT - 1) / NT;    // halo vectors per thread
    static constexpr int S = 2 * R + 2;                     // queue slots
    // Per-plane operands (previous level, alpha, beta) come from a ring of PR
    // slots, fetched PR-1 planes ahead.  In 2D a plane is one row of the
    // tile, too little work to cover a load issued one plane earlier, so the
    // ring is deeper there (measured: 2.5 % on the batched 2D shots).  PR
    // divides S so that the unrolled group of S planes addresses every slot
    // at a compile-time index.
    static constexpr int PR = DIM == 2 ? pre_ring(S, 4) : 2;
    // Halo lead: in 3D, the y/z halo of plane p is loaded together with the
    // queue load of p (R+1 planes before its use) and held in registers, so it
    // is read while the neighbouring tile's load of the same rows is still in
    // L2.  Above R = 6 the extra registers would cost occupancy.
    static constexpr bool LEAD = DIM == 3 && R <= 6;
    static constexpr bool HINT = !LEAD;
    // 2D with TY > 1: the slab body (TY waves share one x-chunk held in LDS)
    static constexpr bool SLAB = DIM == 2 && TY > 1;
};

// Rows of u^n a 2D slab block computes at most (its x-chunk); the LDS slab
// holds them with R halo rows on either side.
constexpr int kSlabRows = 16;

// z part of the Laplacian for the VZ points of one lane.  `Lc` points at the
// lane's first point in an LDS row that holds RZ halo points on either side.
// (Used by the slab body; the streaming body has the same terms inline.)
template <int R, int VZ, int RZ>
__device__ __forceinline__ void z_terms(const float* Lc, const Vec<VZ>& c, const float* m2c,
                                        const float* cz, float* lap)
{
    float zr[2 * RZ + VZ];
#pragma unroll
    for (int k = 0; k < RZ / VZ; ++k) {
        const Vec<VZ> lv = vload<VZ>(Lc - RZ + k * VZ);
        const Vec<VZ> rv = vload<VZ>(Lc + VZ + k * VZ);
#pragma unroll
        for (int v = 0; v < VZ; ++v) {
            zr[k * VZ + v] = lv[v];
            zr[RZ + VZ + k * VZ + v] = rv[v];
        }
    }
#pragma unroll
    for (int v = 0; v < VZ; ++v) zr[RZ + v] = c[v];
#pragma unroll
    for (int j = 1; j <= R; ++j)
#pragma unroll
        for (int v = 0; v < VZ; ++v)
            lap[v] = fmaf(cz[j], (zr[RZ + v + j] + zr[RZ + v - j]) + m2c[v], lap[v]);
}

// The leapfrog update of the VZ points of one lane, then the owner-gather
// injection of the sources on row (x, y) (only when the block's x-range holds
// any, `inj_any`, and plane x does).  The streaming body spells out the same
// operations inline (as a call here it held two more registers per lane,
// which cost a wave per SIMD); the tile tests check the two bit for bit.
template <int VZ>
__device__ __forceinline__ Vec<VZ> update_inject(const StepArgs& a, const Vec<VZ>& c, const float* lap,
                                                 const Vec<VZ>& uo, const Vec<VZ>& al, const Vec<VZ>& be,
                                                 bool inj_any, bool own, int64_t x, int64_t y, int64_t z)
{
    Vec<VZ> o;
#pragma unroll
    for (int v = 0; v < VZ; ++v) {
        const float w = fmaf(be[v], c[v] - uo[v], c[v]);
        o[v] = fmaf(al[v], lap[v], w);
    }
    if (inj_any) {
        // planes without injected nodes skip the per-row lookup (uniform test)
        const int64_t ny = a.ny;
        const int32_t* rp = a.inj.row_ptr;
        if (rp[(x + 1) * ny] != rp[x * ny] && own) {
            const int64_t row = x * ny + y;
            const int32_t e0 = rp[row], e1 = rp[row + 1];
            float acc[VZ];
            bool hit[VZ];
#pragma unroll
            for (int v = 0; v < VZ; ++v) { acc[v] = 0.f; hit[v] = false; }
            for (int32_t e = e0; e < e1; ++e) {
                const InjEntry en = a.inj.ent[e];
                const int64_t dz = (int64_t)en.z - z;
#pragma unroll
                for (int v = 0; v < VZ; ++v)
                    if (dz == v) {
                        acc[v] = fmaf(en.w, a.inj_val[en.pt], acc[v]);
                        hit[v] = true;
                    }
            }
#pragma unroll
            for (int v = 0; v < VZ; ++v)
                if (hit[v]) o[v] = fmaf(al[v], acc[v], o[v]);
        }
    }
    return o;
}

// One block's share of one time step: tile (tzi, tyi) of the (y, z) plane over
// x-chunk `chunk`, where L = (chunk * nty + tyi) * ntz + tzi.
template <int DIM, int R, int VZ, int TZL, int TY, bool IMG>
__device__ __forceinline__ void stream_body(const StepArgs& a, int64_t L)
{
    using T = Tile<DIM, R, VZ, TZL, TY>;
    constexpr int NT = T::NT, TZ = T::TZ, RZ = T::RZ, PITCH = T::PITCH, S = T::S, KH = T::KH;
    constexpr int PR = T::PR;
    __shared__ __attribute__((aligned(16))) float lds[2][T::ROWS * PITCH];

    const int64_t nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t sy = nz, sx = ny * nz;
    const int tid = threadIdx.x;
    const int tzi = (int)(L % a.ntz);
    const int64_t t1 = L / a.ntz;
    const int tyi = (int)(t1 % a.nty);
    const int64_t chunk = t1 / a.nty;
    const int tz = tid % TZL, ty = tid / TZL;
    const int64_t y0 = (int64_t)tyi * TY, z0 = (int64_t)tzi * TZ;
    const int64_t y = y0 + ty, z = z0 + (int64_t)tz * VZ;
    const bool own = (y < ny) && (z < nz);
    const int64_t col = y * sy + z;
    const int64_t xa = chunk * a.xchunk;
    const int64_t xb = xa + a.xchunk < nx ? xa + a.xchunk : nx;
    // Odd chunks walk x downwards: the 2R planes two neighbouring chunks both
    // read are then read by both at the same time (at both ends, or at both
    // starts), while they are in L2.  The stencil is symmetric in x and the
    // pair sums commute, so the result does not depend on the direction.
#ifndef WAVE_ALT_DIR
#define WAVE_ALT_DIR 1
#endif
    const int dir = (WAVE_ALT_DIR && (chunk & 1)) ? -1 : 1;
    const int64_t count = xb - xa;
    const int64_t x0 = dir > 0 ? xa : xb - 1;

    // halo items of this thread: plane offset (or -1 when outside the grid) and LDS slot
    int64_t hoff[KH];
    int hlds[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
        const int i = tid + k * NT;
        hoff[k] = -1;
        hlds[k] = -1;
        if (i < T::NHY) {
            const int hr = i / TZL, hz = i % TZL;
            const int64_t yy = hr < R ? y0 - R + hr : y0 + TY + (hr - R);
            const int64_t zz = z0 + (int64_t)hz * VZ;
            hlds[k] = (hr < R ? hr : hr + TY) * PITCH + RZ + hz * VZ;
            if (yy >= 0 && yy < ny && zz < nz) hoff[k] = yy * sy + zz;
        } else if (i < T::NHY + T::NHZ) {
            constexpr int PER = RZ / VZ;
            const int j = i - T::NHY;
            const int r = j / (2 * PER), side = (j / PER) % 2, kk = j % PER;
            const int64_t yy = y0 + r;
            const int64_t zz = side == 0 ? z0 - RZ + (int64_t)kk * VZ : z0 + TZ + (int64_t)kk * VZ;
            hlds[k] = (r + (DIM == 3 ? R : 0)) * PITCH + (side == 0 ? kk * VZ : RZ + TZ + kk * VZ);
            if (yy < ny && zz >= 0 && zz < nz) hoff[k] = yy * sy + zz;
        }
    }

    const float* __restrict__ u = a.cur;
    auto center = [&](int64_t xx) -> Vec<VZ> {
        Vec<VZ> r = vzero<VZ>();
        if (own && xx >= 0 && xx < nx) r = vload<VZ>(u + xx * sx + col);
        return r;
    };

    // queue slot (U + R + j) % S holds plane x + dir j of the plane x at position U
    Vec<VZ> Q[S];
#pragma unroll
    for (int k = 0; k < 2 * R + 1; ++k) Q[k] = center(x0 + dir * (k - R));
    Q[S - 1] = vzero<VZ>();

    // per-plane operands, fetched PR-1 planes ahead of their use
    struct Pre {
        Vec<VZ> halo[KH];
        Vec<VZ> uo, al, be;
        Vec<VZ> fw, gr;          // imaging: forward wavefield u^k and gradient
    };
    Pre pre[PR];
    // halo ring of the lead mode (one slot per plane of lead)
    constexpr int HS = T::LEAD ? R + 1 : 1;
    Vec<VZ> hring[HS][KH];
    auto load_halo = [&](Vec<VZ>* dst, int64_t xx) {
#pragma unroll
        for (int k = 0; k < KH; ++k) {
            dst[k] = vzero<VZ>();
            if (hoff[k] >= 0 && xx >= 0 && xx < nx) dst[k] = vload<VZ>(u + xx * sx + hoff[k]);
        }
    };
    auto fetch = [&](Pre& P, int64_t xx) {
#pragma unroll
        for (int k = 0; k < KH; ++k) {
            P.halo[k] = vzero<VZ>();
            if (!T::LEAD && hoff[k] >= 0) P.halo[k] = vload<VZ>(u + xx * sx + hoff[k]);
        }
        P.uo = P.al = P.be = vzero<VZ>();
        if (own) {
            P.uo = vload_once<VZ, T::HINT>(a.other + xx * sx + col);
            P.al = vload_once<VZ, T::HINT>(a.alpha + xx * sx + col);
            P.be = vload_once<VZ, T::HINT>(a.beta + xx * sx + col);
            if constexpr (IMG) {
                P.fw = vload_once<VZ, T::HINT>(a.img_fwd + xx * sx + col);
                P.gr = vload_once<VZ, T::HINT>(a.img_grad + xx * sx + col);
            }
        }
    };
#pragma unroll
    for (int k = 0; k < PR - 1; ++k)
        if (k < count) fetch(pre[k], x0 + dir * k);
    if (T::LEAD) {
#pragma unroll
        for (int k = 0; k < HS; ++k) load_halo(hring[k], k < count ? x0 + dir * k : -1);
    }

    const int row_c = (ty + (DIM == 3 ? R : 0)) * PITCH + RZ + tz * VZ;
    // does any injected node lie in this block's x-range? (uniform; most
    // blocks of a forward run have none and skip the per-plane lookup)
    const bool inj_any = a.inj_val && a.inj.row_ptr[xb * ny] != a.inj.row_ptr[xa * ny];

    // one plane; U is the position within the unrolled group of S planes
    auto plane = [&](auto UC, int64_t i) {
        constexpr int U = decltype(UC)::value;
        constexpr int B = U & 1;
        const int64_t x = x0 + dir * i;
        Pre& P = pre[U % PR];
        if (i + PR - 1 < count) fetch(pre[(U + PR - 1) % PR], x + dir * (PR - 1));
        Q[(U + 2 * R + 1) % S] = center(x + dir * (R + 1));
        float* Ls = lds[B];
        const Vec<VZ> c = Q[(U + R) % S];
        vstore<VZ>(Ls + row_c, c);
        if (T::LEAD) {
            Vec<VZ>* hr = hring[U % HS];
#pragma unroll
            for (int k = 0; k < KH; ++k)
                if (hlds[k] >= 0) vstore<VZ>(Ls + hlds[k], hr[k]);
            if (i + R + 1 < count) load_halo(hr, x + dir * (R + 1));
        } else {
#pragma unroll
            for (int k = 0; k < KH; ++k)
                if (hlds[k] >= 0) vstore<VZ>(Ls + hlds[k], P.halo[k]);
        }
        lds_barrier();

        float lap[VZ], m2c[VZ];
#pragma unroll
        for (int v = 0; v < VZ; ++v) {
            lap[v] = 0.f;
            m2c[v] = -2.f * c[v];
        }
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const Vec<VZ>& p = Q[(U + R + j) % S];
            const Vec<VZ>& m = Q[(U + R - j + S) % S];
#pragma unroll
            for (int v = 0; v < VZ; ++v) lap[v] = fmaf(a.cx[j], (p[v] + m[v]) + m2c[v], lap[v]);
        }
        if (DIM == 3) {
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                const Vec<VZ> p = vload<VZ>(Ls + row_c + j * PITCH);
                const Vec<VZ> m = vload<VZ>(Ls + row_c - j * PITCH);
#pragma unroll
                for (int v = 0; v < VZ; ++v)
                    lap[v] = fmaf(a.cy[j], (p[v] + m[v]) + m2c[v], lap[v]);
            }
        }
        {
            float zr[2 * RZ + VZ];
#pragma unroll
            for (int k = 0; k < RZ / VZ; ++k) {
                const Vec<VZ> lv = vload<VZ>(Ls + row_c - RZ + k * VZ);
                const Vec<VZ> rv = vload<VZ>(Ls + row_c + VZ + k * VZ);
#pragma unroll
                for (int v = 0; v < VZ; ++v) {
                    zr[k * VZ + v] = lv[v];
                    zr[RZ + VZ + k * VZ + v] = rv[v];
                }
            }
#pragma unroll
            for (int v = 0; v < VZ; ++v) zr[RZ + v] = c[v];
#pragma unroll
            for (int j = 1; j <= R; ++j)
#pragma unroll
                for (int v = 0; v < VZ; ++v)
                    lap[v] = fmaf(a.cz[j], (zr[RZ + v + j] + zr[RZ + v - j]) + m2c[v], lap[v]);
        }
        Vec<VZ> o;
#pragma unroll
        for (int v = 0; v < VZ; ++v) {
            const float w = fmaf(P.be[v], c[v] - P.uo[v], c[v]);
            o[v] = fmaf(P.al[v], lap[v], w);
        }
        if (inj_any) {
            // planes without injected nodes skip the per-row lookup (uniform test)
            const int32_t* rp = a.inj.row_ptr;
            if (rp[(x + 1) * ny] != rp[x * ny] && own) {
                const int64_t row = x * ny + y;
                const int32_t e0 = rp[row], e1 = rp[row + 1];
                float acc[VZ];
                bool hit[VZ];
#pragma unroll
                for (int v = 0; v < VZ; ++v) { acc[v] = 0.f; hit[v] = false; }
                for (int32_t e = e0; e < e1; ++e) {
                    const InjEntry en = a.inj.ent[e];
                    const int64_t dz = (int64_t)en.z - z;
#pragma unroll
                    for (int v = 0; v < VZ; ++v)
                        if (dz == v) {
                            acc[v] = fmaf(en.w, a.inj_val[en.pt], acc[v]);
                            hit[v] = true;
                        }
                }
#pragma unroll
                for (int v = 0; v < VZ; ++v)
                    if (hit[v]) o[v] = fmaf(P.al[v], acc[v], o[v]);
            }
        }
        if (own) {
            const int64_t off = x * sx + col;
            if constexpr (IMG) {
                Vec<VZ> g = P.gr;
#pragma unroll
                for (int v = 0; v < VZ; ++v) {
                    const float d2 = (P.uo[v] + o[v]) + m2c[v];
                    g[v] = fmaf(-P.fw[v] * a.inv_dt2, d2, g[v]);
                }
                vstore_once<VZ, T::HINT>(a.img_grad + off, g);
            }
            vstore_once<VZ, T::HINT>(a.out + off, o);
        }
    };

    for (int64_t i = 0; i < count; i += S) {
        bool go = true;
        [&]<int... Us>(std::integer_sequence<int, Us...>) {
            ((go = go && (i + Us < count), go ? (plane(std::integral_constant<int, Us>{}, i + Us), 0) : 0), ...);
        }(std::make_integer_sequence<int, S>{});
    }
}

// 2D slab body.  The block owns a z-tile of TZ points over an x-chunk of at
// most kSlabRows rows (16: 32 rows read 1.25 rows per row but ran 5-10 %
// slower, with fewer blocks resident).  It loads rows xa-R .. xb+R-1 of u^n (with the z halo)
// into LDS once, and the previous level, alpha and beta of its own points into
// registers, meets at one barrier, and then each wave computes rows
// tw, tw + TW, ... of the chunk.  Against the streaming body the halo rows
// are read once per chunk instead of filling a register queue per lane, and a
// chunk needs no prologue of its own: 16-row chunks read 24 rows of u^n.  The
// arithmetic per point is that of the streaming body, term for term and in
// the same order, so the two give bitwise the same result.
template <int R, int VZ, int TZL, int TW, bool IMG>
__device__ __forceinline__ void slab_body(const StepArgs& a, int64_t L)
{
    using T = Tile<2, R, VZ, TZL, TW>;
    constexpr int NT = T::NT, TZ = T::TZ, RZ = T::RZ, PITCH = T::PITCH;
    constexpr int XR = kSlabRows, ROWS = XR + 2 * R, NV = PITCH / VZ, RPT = XR / TW;
    static_assert(XR % TW == 0, "rows per wave must be whole");
    static_assert(TZL % 64 == 0, "one wave per row group keeps the row test uniform");
    __shared__ __attribute__((aligned(16))) float lds[ROWS * PITCH];

    const int64_t nx = a.nx, nz = a.nz;
    const int tid = threadIdx.x;
    const int tzi = (int)(L % a.ntz);
    const int64_t chunk = L / a.ntz;        // 2D: one tile row
    const int tz = tid % TZL, tw = tid / TZL;
    const int64_t z0 = (int64_t)tzi * TZ, z = z0 + (int64_t)tz * VZ;
    const bool own = z < nz;
    const int64_t xa = chunk * a.xchunk;
    const int64_t xb = xa + a.xchunk < nx ? xa + a.xchunk : nx;
    const int count = (int)(xb - xa);       // at most XR (planner)
    const float* __restrict__ u = a.cur;

    // rows xa-R .. xb+R-1 of u^n with the z halo; zero outside the grid
    for (int i = tid; i < (count + 2 * R) * NV; i += NT) {
        const int r = i / NV, k = i - r * NV;
        const int64_t xx = xa - R + r, zz = z0 - RZ + (int64_t)k * VZ;
        Vec<VZ> v = vzero<VZ>();
        if (xx >= 0 && xx < nx && zz >= 0 && zz < nz) v = vload<VZ>(u + xx * nz + zz);
        vstore<VZ>(lds + r * PITCH + k * VZ, v);
    }
    Vec<VZ> uo[RPT], al[RPT], be[RPT], fw[RPT], gr[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = tw + q * TW;
        uo[q] = al[q] = be[q] = fw[q] = gr[q] = vzero<VZ>();
        if (own && r < count) {
            const int64_t off = (xa + r) * nz + z;
            uo[q] = vload_once<VZ, T::HINT>(a.other + off);
            al[q] = vload_once<VZ, T::HINT>(a.alpha + off);
            be[q] = vload_once<VZ, T::HINT>(a.beta + off);
            if constexpr (IMG) {
                fw[q] = vload_once<VZ, T::HINT>(a.img_fwd + off);
                gr[q] = vload_once<VZ, T::HINT>(a.img_grad + off);
            }
        }
    }
    __syncthreads();

    const bool inj_any = a.inj_val && a.inj.row_ptr[xb] != a.inj.row_ptr[xa];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = tw + q * TW;
        if (r >= count) break;              // uniform within a wave
        const int64_t x = xa + r;
        const float* Lc = lds + (r + R) * PITCH + RZ + tz * VZ;
        const Vec<VZ> c = vload<VZ>(Lc);
        float lap[VZ], m2c[VZ];
#pragma unroll
        for (int v = 0; v < VZ; ++v) {
            lap[v] = 0.f;
            m2c[v] = -2.f * c[v];
        }
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const Vec<VZ> p = vload<VZ>(Lc + j * PITCH);
            const Vec<VZ> m = vload<VZ>(Lc - j * PITCH);
#pragma unroll
            for (int v = 0; v < VZ; ++v) lap[v] = fmaf(a.cx[j], (p[v] + m[v]) + m2c[v], lap[v]);
        }
        z_terms<R, VZ, RZ>(Lc, c, m2c, a.cz, lap);
        const Vec<VZ> o = update_inject<VZ>(a, c, lap, uo[q], al[q], be[q], inj_any, own, x, 0, z);
        if (own) {
            const int64_t off = x * nz + z;
            if constexpr (IMG) {
                Vec<VZ> g = gr[q];
#pragma unroll
                for (int v = 0; v < VZ; ++v) {
                    const float d2 = (uo[q][v] + o[v]) + m2c[v];
                    g[v] = fmaf(-fw[q][v] * a.inv_dt2, d2, g[v]);
                }
                vstore_once<VZ, T::HINT>(a.img_grad + off, g);
            }
            vstore_once<VZ, T::HINT>(a.out + off, o);
        }
    }
}

template <int DIM, int R, int VZ, int TZL, int TY, bool IMG>
__device__ __forceinline__ void stream_tile(const StepArgs& a, int64_t L)
{
    if constexpr (Tile<DIM, R, VZ, TZL, TY>::SLAB) slab_body<R, VZ, TZL, TY, IMG>(a, L);
    else stream_body<DIM, R, VZ, TZL, TY, IMG>(a, L);
}

// Single shot: the first blocks are tiles, the rest sample receivers.  With
// `remap` the tile part of the grid is padded to a multiple of 8 and block b
// takes tile L = (b mod 8) * (part / 8) + b / 8: blocks are dealt to the 8
// XCDs in turn, so each XCD gets a contiguous run of tiles, and neighbouring
// tiles and chunks, which read each other's halo, share one L2.  (2001 x 801
// order 8 with 2D slabs: 6.5 us per step with 504 tiles, 10.0 us with 1004
// tiles before the padding, which then ran without the remap.)
template <int DIM, int R, int VZ, int TZL, int TY, bool IMG>
__global__ __launch_bounds__(TZL* TY) void k_step_stream(StepArgs a)
{
    const int64_t b = blockIdx.x;
    const int64_t SB = a.stencil_blocks;
    const int64_t part = a.remap ? (SB + 7) / 8 * 8 : SB;
    if (b >= part) {
        const int64_t p = (b - part) * (TZL * TY) + threadIdx.x;
        if (p < a.smp.npts) a.smp_out[p] = sample_point<DIM>(a.smp, a.cur, p, a.nz, a.ny * a.nz);
        return;
    }
    int64_t L = b;
    if (a.remap) {
        L = (b & 7) * (part >> 3) + (b >> 3);
        if (L >= SB) return;                // padding
    }
    stream_tile<DIM, R, VZ, TZL, TY, IMG>(a, L);
}

// Many shots in one launch: block b belongs to the shot s with
// begin[s] <= b < begin[s+1]; within a shot the layout is that of the single
// shot kernel (tiles, then receiver samplers).  Step n of every shot: the
// wavefield pair alternates roles, q and d rows are those of step n.
template <int DIM, int R, int VZ, int TZL, int TY>
__global__ __launch_bounds__(TZL* TY) void k_step_batch(const ShotDesc* __restrict__ shots,
                                                        const int64_t* __restrict__ begin,
                                                        int32_t nshots, int32_t n)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nshots - 1;
    while (lo < hi) {                       // last shot with begin[s] <= b
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const ShotDesc& D = shots[lo];
    StepArgs a = D.a;
    float* even = D.buf[0];
    float* odd = D.buf[1];
    a.cur = (n & 1) ? odd : even;
    a.other = (n & 1) ? even : odd;
    a.out = (n & 1) ? even : odd;
    a.inj_val = D.nsrc ? D.q + (int64_t)n * D.nsrc : nullptr;
    a.smp_out = D.nrec ? D.d + (int64_t)n * D.nrec : nullptr;
    const int64_t lb = b - begin[lo];
    if (lb >= a.stencil_blocks) {
        const int64_t p = (lb - a.stencil_blocks) * (TZL * TY) + threadIdx.x;
        if (p < a.smp.npts && a.smp_out) a.smp_out[p] = sample_point<DIM>(a.smp, a.cur, p, a.nz, a.ny * a.nz);
        return;
    }
    stream_tile<DIM, R, VZ, TZL, TY, false>(a, lb);
}


// All nt steps of all shots in one persistent launch.  The grid is sized to
// be co-resident (cooperative launch); block b takes items b, b + G, ... of
// the flattened (shot, tile, x-chunk) list of each step, then the grid meets
// at a barrier: a monotone arrival counter (step n completes at (n+1) G
// arrivals) with agent-scope release/acquire fences so the next step sees
// every block's writes.  Every wait is bounded: past `spin_limit` polls a
// block raises the error word and the whole grid leaves at the next barrier,
// so the launch always drains.
template <int DIM, int R, int VZ, int TZL, int TY>
__global__ __launch_bounds__(TZL* TY) void k_batch_persistent(const ShotDesc* __restrict__ shots,
                                                             const int64_t* __restrict__ begin,
                                                             int32_t nshots, int64_t items,
                                                             int32_t nt, unsigned int* sync,
                                                             int32_t spin_limit)
{
    for (int32_t n = 0; n < nt; ++n) {
        for (int64_t b = blockIdx.x; b < items; b += gridDim.x) {
            int lo = 0, hi = nshots - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (begin[mid] <= b) lo = mid;
                else hi = mid - 1;
            }
            const ShotDesc& D = shots[lo];
            StepArgs a = D.a;
            float* even = D.buf[0];
            float* odd = D.buf[1];
            a.cur = (n & 1) ? odd : even;
            a.other = (n & 1) ? even : odd;
            a.out = (n & 1) ? even : odd;
            a.inj_val = D.nsrc ? D.q + (int64_t)n * D.nsrc : nullptr;
            a.smp_out = D.nrec ? D.d + (int64_t)n * D.nrec : nullptr;
            const int64_t lb = b - begin[lo];
            if (lb >= a.stencil_blocks) {
                const int64_t p = (lb - a.stencil_blocks) * (TZL * TY) + threadIdx.x;
                if (p < a.smp.npts && a.smp_out)
                    a.smp_out[p] = sample_point<DIM>(a.smp, a.cur, p, a.nz, a.ny * a.nz);
            } else {
                stream_tile<DIM, R, VZ, TZL, TY, false>(a, lb);
            }
            __syncthreads();    // the next item rewrites the block's LDS tile
        }
        if (n + 1 == nt) break;
        __shared__ int leave;
        // every wave waits for its own stores to reach L2; then one thread per
        // block releases them to the device (one L2 write-back per block, not
        // per wave) and arrives
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(&sync[0], 1u);
            const unsigned int target = (unsigned int)(n + 1) * gridDim.x;
            int spins = 0;
            while (__hip_atomic_load(&sync[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                __builtin_amdgcn_s_sleep(2);
                if (++spins > spin_limit) {
                    atomicOr(&sync[1], 1u);
                    break;
                }
            }
            __threadfence();    // acquire: invalidates this CU's caches for the next step's reads
            leave = __hip_atomic_load(&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        }
        __syncthreads();
        if (leave) return;
    }
}

template <int DIM_, int R_, int VZ_, int TZL_, int TY_>
struct Cfg {
    static constexpr int DIM = DIM_, R = R_, VZ = VZ_, TZL = TZL_, TY = TY_;
    using T = Tile<DIM_, R_, VZ_, TZL_, TY_>;
};

// Block shapes.  The row length nz is a multiple of 4 (the library pads its
// fields), so every row starts 16-byte aligned.  2D: one wave with four
// z-points per lane (256 z), 128 scalar lanes (128 z), one wave with two
// z-points per lane (128 z), or the slab body with eight waves of four-point
// lanes (256 z, chunks of up to 16 rows held in LDS, two rows per wave;
// measured against four waves with four rows each: 167 us against 170 us on
// the 48 batched shots, and 172 us for the streaming body); 3D, four z-points per lane: 64 z x 16 rows,
// 64 z x 8 rows, 32 z x 32 rows, 100 z x 10 rows or 200 z x 5 rows (the
// last two cover grids such as 200^3 without a mostly empty last tile); 3D,
// two z-points per lane: 64 z x 8 rows (half the queue registers per lane).
template <int DIM, int R, class F>
hipError_t with_shape(int variant, int64_t nz, F&& f)
{
    if (nz % 4 != 0) return hipErrorInvalidValue;
    if constexpr (DIM == 2) {
        if (variant == 1) return f(Cfg<2, R, 1, 128, 1>{});
        if (variant == 2) return f(Cfg<2, R, 2, 64, 1>{});
        if (variant == 3) return f(Cfg<2, R, 4, 64, 8>{});
        return f(Cfg<2, R, 4, 64, 1>{});
    } else {
        if (variant == 1) return f(Cfg<3, R, 4, 16, 8>{});
        if (variant == 2) return f(Cfg<3, R, 4, 8, 32>{});
        if (variant == 3) return f(Cfg<3, R, 4, 25, 10>{});
        if (variant == 4) return f(Cfg<3, R, 4, 50, 5>{});
        if (variant == 5) return f(Cfg<3, R, 2, 32, 8>{});
        return f(Cfg<3, R, 4, 16, 16>{});
    }
}

template <class F>
hipError_t with_cfg(int ndim, int order, int variant, int64_t nz, F&& f)
{
#define WAVE_CASE(O) \
    case O: return ndim == 2 ? with_shape<2, O / 2>(variant, nz, f) : with_shape<3, O / 2>(variant, nz, f);
    switch (order) {
        WAVE_CASE(2) WAVE_CASE(4) WAVE_CASE(6) WAVE_CASE(8)
        WAVE_CASE(10) WAVE_CASE(12) WAVE_CASE(14) WAVE_CASE(16)
    default: return hipErrorInvalidValue;
    }
#undef WAVE_CASE
}

template <class C>
int64_t plan_t(StepArgs& a, int xchunk, int64_t resident = 0, bool single = false)
{
    using T = typename C::T;
    a.ntz = (int32_t)((a.nz + T::TZ - 1) / T::TZ);
    a.nty = C::DIM == 3 ? (int32_t)((a.ny + C::TY - 1) / C::TY) : 1;
    const int64_t tiles = (int64_t)a.ntz * a.nty;
    // the longest chunk the slab holds (with the XCD remap of single-shot
    // launches, 16 rows beat 8 on 2001 x 801 order 8: 6.6 us against 7.8 us)
    if (T::SLAB && xchunk <= 0) xchunk = kSlabRows;
    if (xchunk <= 0) {
        // 3D: as many blocks as the chip holds at once (`resident`, from the
        // kernel's occupancy; 1024 up to order 12 and 2048 above when
        // unknown), so that no second, partly empty round of blocks follows
        // (512^3 order 16: 3 chunks of 171 planes, 561 us against 589 us at
        // 64 planes); 2D: about 2048 blocks.  No chunk is shorter than 2R
        // planes (3D: at least 8), which would spend most of the block on
        // its prologue.
        int64_t xc;
        if (C::DIM == 3) {
            int64_t want = resident > 0 ? resident : (C::R <= 6 ? 1024 : 2048);
            // two-point lanes: a block is half the work of a four-point one
            // at the same rows; two rounds of them measured fastest (256^3
            // order 8: 52.2 us at 16-plane chunks against 53.5 us at 32)
            if (C::VZ == 2) want *= 2;
            int64_t chunks = want / tiles;
            if (chunks < 1) chunks = 1;
            xc = (a.nx + chunks - 1) / chunks;
        } else {
            const int64_t want_chunks = (2048 + tiles - 1) / tiles;
            xc = (a.nx + want_chunks - 1) / want_chunks;
        }
        const int64_t xmin = C::DIM == 3 ? (2 * C::R > 8 ? 2 * C::R : 8) : 2 * C::R;
        if (xc < xmin) xc = xmin;
        xchunk = (int)(xc < a.nx ? xc : a.nx);
    }
    if (T::SLAB && xchunk > kSlabRows) xchunk = kSlabRows;
    if (xchunk > a.nx) xchunk = (int)a.nx;
    a.xchunk = xchunk;
    const int64_t nchunk = (a.nx + xchunk - 1) / xchunk;
    a.stencil_blocks = tiles * nchunk;
    // a single-shot launch pads its tile part to a multiple of 8 and remaps
    // (k_step_stream); the many-shot kernels index items directly
    a.remap = single ? 1 : 0;
    const int64_t part = single ? (a.stencil_blocks + 7) / 8 * 8 : a.stencil_blocks;
    int64_t nsb = 0;
    if (a.smp_out && a.smp.npts > 0) nsb = (a.smp.npts + T::NT - 1) / T::NT;
    return part + nsb;
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

// ---------------------------------------------------------------------------
// Checkpoint codec.  A reduced-precision checkpoint of the pair (u^c, u^{c-1})
// stores u^c and the increment d = u^c - u^{c-1}, each as BF16 or FP16 of
// (value * s) with its own power-of-two scale s, chosen so that max|value| * s
// lies in [2^14, 2^15): the products are exact and FP16 cannot overflow.
// Restoring gives u^c = stored_u / s_u and u^{c-1} = u^c - stored_d / s_d, so
// the restart velocity carries the relative error of one rounding of d.
// slot layout per checkpoint: {s_u, s_d, max|u| bits, max|d| bits}.
// ---------------------------------------------------------------------------
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
    return ndim == 2 ? 4 : 6;
}

int default_variant(int ndim, int order, int64_t ny, int64_t nz)
{
    if (ndim == 2) return 3;      // the slab body (2001 x 801 order 8: 8.7 us against 10.9 us per step)
    // Candidates in order of preference at equal lane waste: up to order 8
    // the two-point-lane tile first (256^3 order 8: 52.2 us against 53.8 us
    // for 64 z x 16 rows of four-point lanes); above, it is slower (512^3
    // order 16: 596 us against 561 us).
    const int pref[] = {5, 0, 1, 2, 3, 4};
    const int base[] = {0, 1, 2, 3, 4, 5};
    const int* order_of = order <= 8 ? pref : base;
    int best = 0;
    double best_eff = -1.0;
    for (int k = 0; k < tile_variants(3, nz); ++k) {
        const int v = order_of[k];
        double eff = 0.0;
        (void)with_shape<3, 1>(v, nz, [&](auto C) {
            using T = typename decltype(C)::T;
            const double fz = (double)nz / (double)(((nz + T::TZ - 1) / T::TZ) * T::TZ);
            const double fy = (double)ny / (double)(((ny + C.TY - 1) / C.TY) * C.TY);
            const double fw = (double)T::NT / (double)(((T::NT + 63) / 64) * 64);
            eff = fz * fy * fw;
            return hipSuccess;
        });
        if (eff > best_eff + 1e-9) { best_eff = eff; best = v; }
    }
    return best;
}

int64_t plan_tiles(int ndim, int order, TileCfg cfg, StepArgs& a)
{
    int64_t blocks = -1;
    (void)with_cfg(ndim, order, cfg.variant, a.nz, [&](auto C) {
        blocks = plan_t<decltype(C)>(a, cfg.xchunk);
        return hipSuccess;
    });
    return blocks;
}

// Blocks of `kern` (nt threads each) resident on the whole device at once;
// 0 if the runtime cannot say.  Cached per kernel (one device type).
template <class K>
int64_t resident_blocks(K kern, int nt, std::atomic<int64_t>& cache)
{
    int64_t r = cache.load(std::memory_order_relaxed);
    if (r >= 0) return r;
    int dev = 0, cus = 0, per_cu = 0;
    r = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), nt,
                                                     0) == hipSuccess)
        r = (int64_t)per_cu * cus;
    cache.store(r, std::memory_order_relaxed);
    return r;
}

hipError_t launch_step(int ndim, int order, const StepArgs& a0, hipStream_t s, TileCfg cfg)
{
    return with_cfg(ndim, order, cfg.variant, a0.nz, [&](auto C) {
        using CC = decltype(C);
        auto launch = [&](auto kern, std::atomic<int64_t>& cache) {
            StepArgs a = a0;
            const int64_t res = cfg.xchunk <= 0 ? resident_blocks(kern, CC::T::NT, cache) : 0;
            const int64_t blocks = plan_t<CC>(a, cfg.xchunk, res, true);
            if (!(a.smp_out && a.smp.npts > 0)) a.smp.npts = 0;
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(CC::T::NT), 0, s, a);
            return hipGetLastError();
        };
        static std::atomic<int64_t> res_img{-1}, res_plain{-1};
        if (a0.img_grad)
            return launch(k_step_stream<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY, true>, res_img);
        return launch(k_step_stream<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY, false>, res_plain);
    });
}

hipError_t launch_batch_persistent(int ndim, int order, int64_t nz_any, TileCfg cfg,
                                   const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                                   int64_t items, int32_t nt, unsigned int* sync, int32_t spin_limit,
                                   int max_per_cu, int* grid_used, hipStream_t s)
{
    return with_cfg(ndim, order, cfg.variant, nz_any, [&](auto C) {
        using CC = decltype(C);
        auto kern = k_batch_persistent<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY>;
        int dev = 0, per_cu = 0;
        hipDeviceProp_t prop;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                             CC::T::NT, 0);
        if (e != hipSuccess) return e;
        // The occupancy figure is an upper bound that the dispatcher does not
        // always reach for many small blocks; cap the grid at a few blocks per
        // CU so that all of them are resident (the barrier needs every one).
        if (per_cu > max_per_cu) per_cu = max_per_cu;
        int64_t grid = (int64_t)per_cu * prop.multiProcessorCount;
        if (grid > items) grid = items;
        if (grid < 1) return hipErrorInvalidConfiguration;
        *grid_used = (int)grid;
        void* args[] = {(void*)&shots, (void*)&begin, (void*)&nshots, (void*)&items, (void*)&nt,
                        (void*)&sync, (void*)&spin_limit};
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3((unsigned)grid),
                                          dim3(CC::T::NT), args, 0, s);
    });
}

hipError_t launch_batch(int ndim, int order, int64_t nz_any, TileCfg cfg, const ShotDesc* shots,
                        const int64_t* begin, int32_t nshots, int64_t blocks, int32_t n,
                        hipStream_t s)
{
    return with_cfg(ndim, order, cfg.variant, nz_any, [&](auto C) {
        using CC = decltype(C);
        hipLaunchKernelGGL((k_step_batch<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY>),
                           dim3((unsigned)blocks), dim3(CC::T::NT), 0, s, shots, begin, nshots, n);
        return hipGetLastError();
    });
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

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace wave
