// Step kernels of the damped acoustic leapfrog scheme (gfx950), as templates
// over the space order, the block shape and the imaging flag.  Each space
// order is instantiated in a translation unit of its own (wave_o<order>.hip)
// through OrderOps<order>; the rest of the library dispatches on the order.
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
#pragma once

#include <algorithm>
#include <atomic>
#include <utility>

#include "wave_internal.h"

// Build-time knobs of the streaming body (defaults measured best): planes of
// per-plane operands in flight in 3D (two at least), and the largest half-width with the
// halo lead.
#ifndef WAVE_PRE_RING_3D
#define WAVE_PRE_RING_3D 2
#endif
#ifndef WAVE_LEAD_MAX_R
#define WAVE_LEAD_MAX_R 6
#endif
#ifndef WAVE_SLAB2_WPE
#define WAVE_SLAB2_WPE 4
#endif

namespace wave {

namespace {


// Global memory is addressed through pointers in the global address space.
// A generic pointer that the compiler cannot trace to a kernel argument
// (the batch kernels read theirs from the shot descriptors) would otherwise
// compile to flat loads, which count against the LDS counter as well: every
// wait for an LDS result, and every LDS barrier, would then also wait for all
// outstanding global loads.
#define WAVE_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ const WAVE_GLOBAL T* G(const T* p)
{
    return (const WAVE_GLOBAL T*)p;
}

template <class T>
__device__ __forceinline__ WAVE_GLOBAL T* G(T* p)
{
    return (WAVE_GLOBAL T*)p;
}

// One injection entry read through a global-address-space pointer (member by
// member: the implicit copy does not take an address-space-qualified source).
__device__ __forceinline__ InjEntry load_entry(const InjEntry* ent, int64_t e)
{
    const WAVE_GLOBAL InjEntry* q = G(ent) + e;
    InjEntry r;
    r.z = q->z;
    r.pt = q->pt;
    r.w = q->w;
    return r;
}

constexpr int kBlock = 256;

template <int DIM>
__device__ __forceinline__ float sample_point(const SampleSet& s, const float* __restrict__ ug,
                                              int64_t p, int64_t sy, int64_t sx)
{
    const WAVE_GLOBAL float* u = G(ug);
    const int64_t b = G(s.base)[p];
    const WAVE_GLOBAL float* w = G(s.w) + p * (1 << DIM);
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

template <int VZ>
__device__ __forceinline__ Vec<VZ> vload(const WAVE_GLOBAL float* p)
{
    return *(const WAVE_GLOBAL Vec<VZ>*)p;
}

template <int VZ>
__device__ __forceinline__ void vstore(WAVE_GLOBAL float* p, const Vec<VZ>& v)
{
    *(WAVE_GLOBAL Vec<VZ>*)p = v;
}

// Operands touched once per step (previous level, coefficients, output).
// With NT they carry the non-temporal hint, which keeps them from evicting
// wavefield planes that later tiles re-read; measured on gfx950 it pays only
// where the halos are not loaded early (see Tile::LEAD).
template <int VZ, bool NT>
__device__ __forceinline__ Vec<VZ> vload_once(const float* p)
{
    const WAVE_GLOBAL Vec<VZ>* q = (const WAVE_GLOBAL Vec<VZ>*)p;
    if constexpr (NT) return __builtin_nontemporal_load(q);
    else return *q;
}

template <int VZ, bool NT>
__device__ __forceinline__ void vstore_once(float* p, const Vec<VZ>& v)
{
    WAVE_GLOBAL Vec<VZ>* q = (WAVE_GLOBAL Vec<VZ>*)p;
    if constexpr (NT) __builtin_nontemporal_store(v, q);
    else *q = v;
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
    static constexpr int PR = DIM == 2 ? pre_ring(S, 4) : WAVE_PRE_RING_3D;
    // a plane's injection range is read (for the early loads of its gathered
    // values) before that plane's own fetch is issued, so its operands must
    // come from a fetch at least one plane earlier: a one-slot ring would read
    // an unfetched range and index the entry arrays with it
    static_assert(PR >= 2, "the per-plane operand ring needs at least two slots");
    // Halo lead: in 3D, the y/z halo of plane p is loaded together with the
    // queue load of p (R+1 planes before its use) and held in registers, so it
    // is read while the neighbouring tile's load of the same rows is still in
    // L2.  Above R = 6 the extra registers would cost occupancy.
    static constexpr bool LEAD = DIM == 3 && R <= WAVE_LEAD_MAX_R;
    static constexpr bool HINT = !LEAD;
    // 2D with TY > 1: the slab body (TY waves share one x-chunk held in LDS)
    static constexpr bool SLAB = DIM == 2 && TY > 1;
};


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

// Owner-gather injection of the entries [e0, e1) of a lane's row into its VZ
// points z .. z+VZ-1: o += alpha * sum_e w_e val[pt_e] over the entries at
// each point, summed in entry order (sorted by point index).  One entry at a
// time: loading several ahead held enough registers to cost the 512^3
// order-16 step a wave per SIMD.
template <int VZ>
__device__ __forceinline__ void inject_core(const InjEntry* __restrict__ ent, const float* __restrict__ ev,
                                            const float* __restrict__ val, int32_t e0, int32_t e1,
                                            int64_t z, const Vec<VZ>& al, Vec<VZ>& o)
{
    float acc[VZ];
    bool hit[VZ];
#pragma unroll
    for (int v = 0; v < VZ; ++v) { acc[v] = 0.f; hit[v] = false; }
    for (int32_t e = e0; e < e1; ++e) {
        const InjEntry en = load_entry(ent, e);
        // w * val rounded, then added: the gathered values hold the same products
        const float wv = ev ? G(ev)[e] : en.w * G(val)[en.pt];
        const int64_t dz = (int64_t)en.z - z;
#pragma unroll
        for (int v = 0; v < VZ; ++v)
            if (dz == v) {
                acc[v] = acc[v] + wv;
                hit[v] = true;
            }
    }
#pragma unroll
    for (int v = 0; v < VZ; ++v)
        if (hit[v]) o[v] = fmaf(al[v], acc[v], o[v]);
}

template <int VZ>
__device__ __forceinline__ void inject_entries(const StepArgs& a, int32_t e0, int32_t e1, int64_t z,
                                               const Vec<VZ>& al, Vec<VZ>& o)
{
    inject_core<VZ>(a.inj.ent, a.inj_ev, a.inj_val, e0, e1, z, al, o);
}

// The leapfrog update of the VZ points of one lane:
// out = fma(alpha, lap, fma(beta, u - other, u)).
template <int VZ>
__device__ __forceinline__ Vec<VZ> update_core(const Vec<VZ>& c, const float* lap, const Vec<VZ>& uo,
                                               const Vec<VZ>& al, const Vec<VZ>& be)
{
    Vec<VZ> o;
#pragma unroll
    for (int v = 0; v < VZ; ++v) {
        const float w = fmaf(be[v], c[v] - uo[v], c[v]);
        o[v] = fmaf(al[v], lap[v], w);
    }
    return o;
}

// The leapfrog update of the VZ points of one lane, then the owner-gather
// injection of the entries [e0, e1) of the lane's row (e1 == e0 when the row
// holds no injected node; the range was fetched with the other per-row
// operands).  The streaming body spells out the same operations inline (as a
// call here it held two more registers per lane, which cost a wave per
// SIMD); the tile tests check the two bit for bit.
template <int VZ>
__device__ __forceinline__ Vec<VZ> update_inject(const StepArgs& a, const Vec<VZ>& c, const float* lap,
                                                 const Vec<VZ>& uo, const Vec<VZ>& al, const Vec<VZ>& be,
                                                 int32_t e0, int32_t e1, int64_t z)
{
    Vec<VZ> o = update_core<VZ>(c, lap, uo, al, be);
    if (e1 > e0) inject_entries<VZ>(a, e0, e1, z, al, o);
    return o;
}

// Planes of an x-chunk whose injection flags a streaming block keeps in LDS
// (one bit per plane); planes beyond them are looked up in the row pointers.
constexpr int kInjMaskWords = 64;

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
    // offsets within a (y, z) plane fit 32 bits (the library checks ny * nz < 2^31)
    const int32_t col = (int32_t)(y * sy + z);
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
    int32_t hoff[KH];
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
            if (yy >= 0 && yy < ny && zz < nz) hoff[k] = (int32_t)(yy * sy + zz);
        } else if (i < T::NHY + T::NHZ) {
            constexpr int PER = RZ / VZ;
            const int j = i - T::NHY;
            const int r = j / (2 * PER), side = (j / PER) % 2, kk = j % PER;
            const int64_t yy = y0 + r;
            const int64_t zz = side == 0 ? z0 - RZ + (int64_t)kk * VZ : z0 + TZ + (int64_t)kk * VZ;
            hlds[k] = (r + (DIM == 3 ? R : 0)) * PITCH + (side == 0 ? kk * VZ : RZ + TZ + kk * VZ);
            if (yy < ny && zz >= 0 && zz < nz) hoff[k] = (int32_t)(yy * sy + zz);
        }
    }

    const WAVE_GLOBAL float* __restrict__ u = G(a.cur);
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

    // Injection: does any injected node lie in this block's x-range (uniform;
    // most blocks of a forward run have none), and which planes hold one (a
    // bit per plane in LDS, filled once), so that a plane's row lookup is a
    // per-row operand fetched ahead with the others instead of a dependent
    // load on every plane.
    const WAVE_GLOBAL int32_t* rp = G(a.inj.row_ptr);
    const bool inj_any = a.inj_val && xb > a.inj_x0 && xa <= a.inj_x1 &&
                         y0 + TY > a.inj_y0 && y0 <= a.inj_y1;
    __shared__ uint32_t inj_mask[kInjMaskWords];
    if (inj_any) {
        for (int w = tid; w < kInjMaskWords; w += NT) inj_mask[w] = 0u;
        lds_barrier();
        for (int64_t i = tid; i < count && i < 32 * kInjMaskWords; i += NT) {
            const int64_t xx = xa + i;
            if (rp[(xx + 1) * ny] != rp[xx * ny]) atomicOr(&inj_mask[i >> 5], 1u << (i & 31));
        }
        lds_barrier();
    }
    auto plane_has_inj = [&](int64_t xx) -> bool {
        const int64_t i = xx - xa;
        if (i < 32 * kInjMaskWords) return (inj_mask[i >> 5] >> (i & 31)) & 1u;
        return rp[(xx + 1) * ny] != rp[xx * ny];
    };

    // per-plane operands, fetched PR-1 planes ahead of their use
    struct Pre {
        Vec<VZ> halo[KH];
        Vec<VZ> uo, al, be;
        Vec<VZ> fw, gr;          // imaging: forward wavefield u^k and gradient
        int32_t e0, e1;          // injection entries of the lane's row
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
            if (!a.no_prev) {
                P.uo = vload_once<VZ, T::HINT>(a.other + xx * sx + col);
                P.be = vload_once<VZ, T::HINT>(a.beta + xx * sx + col);
            }
            P.al = vload_once<VZ, T::HINT>(a.alpha + xx * sx + col);
            if constexpr (IMG) {
                P.fw = vload_once<VZ, T::HINT>(a.img_fwd + xx * sx + col);
                P.gr = vload_once<VZ, T::HINT>(a.img_grad + xx * sx + col);
            }
        }
        P.e0 = P.e1 = 0;
        if (inj_any && own && plane_has_inj(xx)) {
            const int64_t row = xx * ny + y;
            P.e0 = rp[row];
            P.e1 = rp[row + 1];
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

    // one plane; U is the position within the unrolled group of S planes
    auto plane = [&](auto UC, int64_t i) {
        constexpr int U = decltype(UC)::value;
        constexpr int B = U & 1;
        const int64_t x = x0 + dir * i;
        Pre& P = pre[U % PR];
        // gathered injection: the depth and the value of the row's first two
        // entries, loaded first (before the prefetch of later planes: loads
        // complete in order, so waiting for these does not wait for those)
        // and used after the stencil
        const bool inj_here = inj_any && P.e1 > P.e0;
        int32_t ez0 = -1, ez1 = -1;
        float ev0 = 0.f, ev1 = 0.f;
        if (inj_here && a.inj_ev) {
            ez0 = G(a.inj.ent)[P.e0].z;
            ev0 = G(a.inj_ev)[P.e0];
            if (P.e0 + 1 < P.e1) {
                ez1 = G(a.inj.ent)[P.e0 + 1].z;
                ev1 = G(a.inj_ev)[P.e0 + 1];
            }
        }
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
        if (inj_here) {
            if (a.inj_ev) {
                // same entries, same order as inject_entries
                float acc[VZ];
                bool hit[VZ];
#pragma unroll
                for (int v = 0; v < VZ; ++v) { acc[v] = 0.f; hit[v] = false; }
#pragma unroll
                for (int v = 0; v < VZ; ++v) {
                    if (ez0 - z == v) { acc[v] = acc[v] + ev0; hit[v] = true; }
                    if (ez1 >= 0 && ez1 - z == v) { acc[v] = acc[v] + ev1; hit[v] = true; }
                }
                for (int32_t e = P.e0 + 2; e < P.e1; ++e) {
                    const int64_t dz = (int64_t)G(a.inj.ent)[e].z - z;
                    const float wv = G(a.inj_ev)[e];
#pragma unroll
                    for (int v = 0; v < VZ; ++v)
                        if (dz == v) { acc[v] = acc[v] + wv; hit[v] = true; }
                }
#pragma unroll
                for (int v = 0; v < VZ; ++v)
                    if (hit[v]) o[v] = fmaf(P.al[v], acc[v], o[v]);
            } else {
                inject_entries<VZ>(a, P.e0, P.e1, z, P.al, o);
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
    static_assert(XR <= 64, "the injection rows of a chunk are one wave-wide ballot");
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
    const WAVE_GLOBAL float* __restrict__ u = G(a.cur);

    // rows xa-R .. xb+R-1 of u^n with the z halo; zero outside the grid
    for (int i = tid; i < (count + 2 * R) * NV; i += NT) {
        const int r = i / NV, k = i - r * NV;
        const int64_t xx = xa - R + r, zz = z0 - RZ + (int64_t)k * VZ;
        Vec<VZ> v = vzero<VZ>();
        if (xx >= 0 && xx < nx && zz >= 0 && zz < nz) v = vload<VZ>(u + xx * nz + zz);
        vstore<VZ>(lds + r * PITCH + k * VZ, v);
    }
    // rows of the chunk holding injected nodes: one flag per lane, one ballot
    // (a chunk has at most 64 rows), then each lane's entry range is fetched
    // with its other per-row operands
    const WAVE_GLOBAL int32_t* rp = G(a.inj.row_ptr);
    const bool inj_any = a.inj_val && xb > a.inj_x0 && xa <= a.inj_x1;
    uint64_t inj_rows = 0;
    if (inj_any) {
        const int lane = tid & 63;
        inj_rows = __ballot(lane < count && rp[xa + lane + 1] != rp[xa + lane]);
    }
    Vec<VZ> uo[RPT], al[RPT], be[RPT], fw[RPT], gr[RPT];
    int32_t e0[RPT], e1[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = tw + q * TW;
        e0[q] = e1[q] = 0;
        if (own && r < count && ((inj_rows >> r) & 1u)) {
            e0[q] = rp[xa + r];
            e1[q] = rp[xa + r + 1];
        }
        uo[q] = al[q] = be[q] = fw[q] = gr[q] = vzero<VZ>();
        if (own && r < count) {
            const int64_t off = (xa + r) * nz + z;
            if (!a.no_prev) {
                uo[q] = vload_once<VZ, T::HINT>(a.other + off);
                be[q] = vload_once<VZ, T::HINT>(a.beta + off);
            }
            al[q] = vload_once<VZ, T::HINT>(a.alpha + off);
            if constexpr (IMG) {
                fw[q] = vload_once<VZ, T::HINT>(a.img_fwd + off);
                gr[q] = vload_once<VZ, T::HINT>(a.img_grad + off);
            }
        }
    }
    __syncthreads();

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
        const Vec<VZ> o = update_inject<VZ>(a, c, lap, uo[q], al[q], be[q], e0[q], e1[q], z);
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

// Single shot: the first blocks are tiles, the last `sample_blocks` sample
// the receivers (they only read `cur`).  Placed first instead, they took
// resident slots from the tiles and pushed a share of them into a further
// partial round (512^3 order 16: 523 us against 488 us per step).  With
// `remap` the tile part of the grid is padded to a multiple of 8 and block b
// takes tile L = (b mod 8) * (part / 8) + b / 8: blocks are dealt to the 8
// XCDs in turn, so each XCD gets a contiguous run of tiles, and neighbouring
// tiles and chunks, which read each other's halo, share one L2.  (2001 x 801
// order 8 with 2D slabs: 6.5 us per step with 504 tiles, 10.0 us with 1004
// tiles before the padding, which then ran without the remap.)
// Waves per SIMD the plain 3D step asks the compiler to keep resident (the
// second launch bound): 3 with four z-points per lane, 4 with two.  At order
// 16 the 64 z x 16 tile otherwise takes 169 VGPRs, one above what 3 waves
// per SIMD allow, and runs at 2.  The imaging step is left to the compiler.
template <int DIM, int VZ, bool IMG>
constexpr int step_waves_per_eu()
{
    return (DIM == 3 && !IMG) ? (VZ == 4 ? 3 : 4) : 1;
}

template <int DIM, int R, int VZ, int TZL, int TY, bool IMG>
__global__ __launch_bounds__(TZL* TY, (step_waves_per_eu<DIM, VZ, IMG>())) void k_step_stream(StepArgs a)
{
    const int64_t b = blockIdx.x;
    const int64_t SB = a.stencil_blocks;
    const int64_t part = a.remap ? (SB + 7) / 8 * 8 : SB;
    if (b >= part) {
        const int64_t nsb = a.smp_out && a.smp.npts > 0 ? (a.smp.npts + TZL * TY - 1) / (TZL * TY) : 0;
        if (b - part < nsb) {
            const int64_t p = (b - part) * (TZL * TY) + threadIdx.x;
            if (p < a.smp.npts) G(a.smp_out)[p] = sample_point<DIM>(a.smp, a.cur, p, a.nz, a.ny * a.nz);
        } else {
            // gather of the next step's injection values into entry order
            const int64_t e = (b - part - nsb) * (TZL * TY) + threadIdx.x;
            if (e < a.nent) {
                const InjEntry en = load_entry(a.inj.ent, e);
                G(a.ev_out)[e] = en.w * G(a.ev_src)[en.pt];
            }
        }
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
        if (p < a.smp.npts && a.smp_out) G(a.smp_out)[p] = sample_point<DIM>(a.smp, a.cur, p, a.nz, a.ny * a.nz);
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
                    G(a.smp_out)[p] = sample_point<DIM>(a.smp, a.cur, p, a.nz, a.ny * a.nz);
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

// Two time steps per pass (temporal blocking, 2D): levels n+1 and n+2 from
// u^n and u^{n-1} with one read of the fields.  A block of XR waves owns
// TZO = 256 - 2 RZ z-points of a column of x-rows [X0, X1); its lanes cover
// the owned z plus RZ on either side.  It walks the column in rounds of XR
// rows:
//   - u^n rows enter a ring in LDS (z halo RZ beyond the lanes), fetched one
//     round ahead into registers; level n+1 rows enter a second ring;
//   - step 1 of round j computes level n+1 on rows X0 + R + XR j + [0, XR)
//     (before the first round, on the 2R rows around X0), at every lane,
//     zero outside the grid, with the level-n injection; rows inside
//     [X0, X1) at the owned lanes also go to `out1`;
//   - step 2 of round j computes level n+2 on the rows step 1 produced in
//     the previous round, with the level n+1 injection, into `a.out`.
// Wave w takes the rows congruent to w (mod XR) relative to X0 in both
// steps, so the coefficients a row's step 1 loaded serve its step 2 a round
// later from registers.
// Each point's arithmetic is that of the single step (same operations in the
// same order), and a point outside the block's own part is computed from the
// same inputs as by the block that owns it, so two steps here are bitwise two
// single steps.  The inputs are not written during the pass, so the outputs
// go to a second pair of buffers.  Per own point and pass the block reads
// u^n (1 + 4R/C) times and u^{n-1}, alpha, beta (1 + 2R/C) times for a
// column of C rows, and writes two levels: 24 B per two updates as C grows,
// against 2 x 20 B for single steps.  Loads are issued in the order they
// are consumed, so no wait for one also waits for a later one.
template <int R, int VZ, int TZL, int XR>
__device__ __forceinline__ void roll2_body(const StepArgs& a, int64_t L, const float* __restrict__ val0,
                                           const float* __restrict__ val1, float* __restrict__ out1,
                                           bool two)
{
    constexpr int NT = TZL * XR;                   // one wave per row of a round
    constexpr int RZ = (R + VZ - 1) / VZ * VZ;
    constexpr int TZE = TZL * VZ;                  // z the lanes cover
    constexpr int TZO = TZE - 2 * RZ;              // z a block owns
    constexpr int P = TZE + 2 * RZ;                // row pitch of both rings
    // rows held: u^n from the oldest row a step 2 still reads to the newest
    // prefetched one (and the prologue's 4R rows plus one round); level n+1
    // from the oldest row a step 2 reads to the newest step-1 row
    constexpr int RING1 = (R + 3 * XR > 4 * R + XR) ? R + 3 * XR : 4 * R + XR;
    constexpr int RING2 = R + 2 * XR;
    constexpr int NV = P / VZ;                     // vectors per u^n row
    constexpr int NPV = (XR * NV + NT - 1) / NT;   // u^n vectors per thread per round
    static_assert(R <= XR, "step 2 lags step 1 by one round");
    static_assert(TZL % 64 == 0, "one wave per row keeps the row tests uniform");
    static_assert(TZO > 0 && TZO % VZ == 0, "owned z must be whole vectors");
    __shared__ __attribute__((aligned(16))) float ring1[RING1 * P];
    __shared__ __attribute__((aligned(16))) float ring2[RING2 * P];

    const int64_t nx = a.nx, nz = a.nz;
    const int tid = threadIdx.x;
    const int tzi = (int)(L % a.ntz);
    const int64_t col = L / a.ntz;
    // the wave index is uniform: row arithmetic then stays scalar
    const int tz = tid % TZL, w = __builtin_amdgcn_readfirstlane(tid / TZL);
    const int64_t z0 = (int64_t)tzi * TZO;         // first owned z
    const int64_t z = z0 - RZ + (int64_t)tz * VZ;  // the lane's first point
    // nz and z are multiples of VZ: a lane's points are all inside or all out
    const bool zin = z >= 0 && z < nz;
    const bool zown = zin && tz >= RZ / VZ && tz < TZL - RZ / VZ;
    const int64_t X0 = col * a.xchunk;
    const int64_t X1 = X0 + a.xchunk < nx ? X0 + a.xchunk : nx;
    const int64_t base1 = X0 - 2 * R, base2 = X0 - R;   // rows of slot 0 (rows are never below)
    const int lane_off = RZ + tz * VZ;
    auto row1 = [&](int64_t r) { return ring1 + (int)((uint32_t)(r - base1) % RING1) * P + lane_off; };
    auto row2 = [&](int64_t r) { return ring2 + (int)((uint32_t)(r - base2) % RING2) * P + lane_off; };
    auto unload = [&](int64_t r, int k) {         // vector k of u^n row r (zero outside the grid)
        const int64_t zz = z0 - 2 * RZ + (int64_t)k * VZ;
        Vec<VZ> v = vzero<VZ>();
        if (r >= 0 && r < nx && zz >= 0 && zz < nz) v = vload<VZ>(G(a.cur) + r * nz + zz);
        return v;
    };
    const WAVE_GLOBAL int32_t* rp = G(a.inj.row_ptr);
    const bool inj_any = val0 && X1 + R > a.inj_x0 && X0 - R <= a.inj_x1;
    auto inj_range = [&](int64_t x, int32_t& e0, int32_t& e1) {   // x uniform per wave
        e0 = e1 = 0;
        if (inj_any && x >= a.inj_x0 && x <= a.inj_x1 && x >= 0 && x < nx) {
            e0 = rp[x];
            e1 = rp[x + 1];
        }
    };
    // step-1 operands of row x (zero outside the grid)
    struct Ops {
        Vec<VZ> uo, al, be;
        int32_t e0, e1;
    };
    auto fetch_ops = [&](int64_t x, Ops& o) {
        o.uo = o.al = o.be = vzero<VZ>();
        inj_range(x, o.e0, o.e1);
        if (x >= 0 && x < nx && zin) {
            const int64_t off = x * nz + z;
            if (!a.no_prev) {
                o.uo = vload<VZ>(G(a.other) + off);
                o.be = vload<VZ>(G(a.beta) + off);
            }
            o.al = vload<VZ>(G(a.alpha) + off);
        }
    };
    // Laplacian of the lane's points of row x from a ring
    auto laplace = [&](auto row, int64_t x, const Vec<VZ>& c, float* lap, float* m2c) {
#pragma unroll
        for (int v = 0; v < VZ; ++v) {
            lap[v] = 0.f;
            m2c[v] = -2.f * c[v];
        }
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            const Vec<VZ> p = vload<VZ>(row(x + j));
            const Vec<VZ> m = vload<VZ>(row(x - j));
#pragma unroll
            for (int v = 0; v < VZ; ++v) lap[v] = fmaf(a.cx[j], (p[v] + m[v]) + m2c[v], lap[v]);
        }
        z_terms<R, VZ, RZ>(row(x), c, m2c, a.cz, lap);
    };
    // level n+1 of row x into ring 2 (zero outside the grid) and, inside
    // [X0, X1) at the owned lanes, into out1
    auto step1 = [&](int64_t x, const Ops& q) {
        const Vec<VZ> c = vload<VZ>(row1(x));
        float lap[VZ], m2c[VZ];
        laplace(row1, x, c, lap, m2c);
        Vec<VZ> o = update_core<VZ>(c, lap, q.uo, q.al, q.be);
        if (q.e1 > q.e0) inject_core<VZ>(a.inj.ent, nullptr, val0, q.e0, q.e1, z, q.al, o);
        const bool in = x >= 0 && x < nx && zin;
        vstore<VZ>(row2(x), in ? o : vzero<VZ>());
        if (in && zown && x >= X0 && x < X1) vstore<VZ>(G(out1) + x * nz + z, o);
    };
    // level n+2 of row x (in [X0, X1)) with its step-1 coefficients
    auto step2 = [&](int64_t x, const Ops& q) {
        const Vec<VZ> c = vload<VZ>(row2(x));
        float lap[VZ], m2c[VZ];
        laplace(row2, x, c, lap, m2c);
        const Vec<VZ> un0 = vload<VZ>(row1(x));    // u^n of the point
        Vec<VZ> o = update_core<VZ>(c, lap, un0, q.al, q.be);
        if (q.e1 > q.e0) inject_core<VZ>(a.inj.ent, nullptr, val1, q.e0, q.e1, z, q.al, o);
        if (zown) vstore<VZ>(G(a.out) + x * nz + z, o);
    };

    // prologue: u^n rows [X0-2R, X0+2R) straight into the ring, the first
    // round's rows into registers, the step-1 operands of this wave's rows
    // among [X0-R, X0+R): X0 + w - XR (when >= X0 - R) and X0 + w (when < X0 + R)
    for (int i = tid; i < 4 * R * NV; i += NT) {
        const int r = i / NV, k = i - r * NV;
        vstore<VZ>(ring1 + r * P + k * VZ, unload(base1 + r, k));
    }
    const int64_t ulim = X1 + 2 * R;               // u^n rows needed end here
    // The XR u^n rows of a round: vector m of this thread is row pr[m] of the
    // round, vector pk[m] of that row.  Its global address advances by XR rows
    // per round and its ring slot by XR slots, so the loop does no index
    // arithmetic beyond two additions.
    const int64_t rlim = ulim < nx ? ulim : nx;    // rows loaded below this, zero above
    int pr[NPV], pk[NPV], ps[NPV];
    bool pin[NPV];
    const float* pp[NPV];
#pragma unroll
    for (int m = 0; m < NPV; ++m) {
        const int i = tid + m * NT;
        pin[m] = i < XR * NV;
        const int ii = pin[m] ? i : 0;
        pr[m] = ii / NV;
        pk[m] = ii - pr[m] * NV;
        const int64_t zz = z0 - 2 * RZ + (int64_t)pk[m] * VZ;
        pin[m] = pin[m] && zz >= 0 && zz < nz;
        ps[m] = (4 * R + pr[m]) % RING1;           // slot of row X0 + 2R + pr[m] (slot 0: X0 - 2R)
        pp[m] = a.cur + (X0 + 2 * R + pr[m]) * nz + (pin[m] ? zz : 0);
    }
    auto fetch_u = [&](Vec<VZ>* pv, int64_t un) {  // rows un .. un + XR - 1
#pragma unroll
        for (int m = 0; m < NPV; ++m) {
            pv[m] = (pin[m] && un + pr[m] < rlim) ? vload<VZ>(G(pp[m])) : vzero<VZ>();
            pp[m] += (int64_t)XR * nz;
        }
    };
    auto store_u = [&](const Vec<VZ>* pv) {        // the round's rows into their slots
#pragma unroll
        for (int m = 0; m < NPV; ++m) {
            if (tid + m * NT < XR * NV) vstore<VZ>(ring1 + ps[m] * P + pk[m] * VZ, pv[m]);
            ps[m] += XR;
            if (ps[m] >= RING1) ps[m] -= RING1;
        }
    };
    int64_t un = X0 + 2 * R;                       // next u^n rows to prefetch
    Vec<VZ> pv[NPV];
    fetch_u(pv, un);
    const int64_t xa = X0 + w - XR, xb = X0 + w;   // this wave's prologue rows
    const bool has_a = w >= XR - R, has_b = w < R;
    Ops qa, q, carry;
    if (has_a) fetch_ops(xa, qa);
    if (has_b) fetch_ops(xb, q);
    lds_barrier();                                 // prologue rows in the ring
    if (has_a) step1(xa, qa);
    if (has_b) step1(xb, q);
    // step 2 of the next round takes row xb (when inside the column)
    bool has2 = has_b && xb < X1;
    int64_t x2 = xb;
    carry = q;
    const int64_t lim1 = X1 + R;                   // step-1 rows needed end here
    int64_t x1 = X0 + R + (int64_t)((w - R + XR) % XR);   // this wave's row of round 0
    if (x1 < lim1) fetch_ops(x1, q);
    const int rounds = (int)((X1 - X0 + XR - 1) / XR);      // step-1 rounds; one more for step 2
    for (int j = 0; j <= rounds; ++j) {
        if (j < rounds) {
            store_u(pv);                           // slots of rows no wave reads any more
            un += XR;
            if (un < ulim) fetch_u(pv, un);
        }
        lds_barrier();                             // u^n rows in; the last step 2 is done with ring 2
        const bool act1 = j < rounds && x1 < lim1;
        if (act1) step1(x1, q);
        const Ops next = q;                        // its coefficients serve step 2 next round
        const bool next2 = act1 && x1 < X1;
        const int64_t nx2 = x1;
        x1 += XR;
        if (j + 1 < rounds && x1 < lim1) fetch_ops(x1, q);
        if (!two) continue;                        // uniform: a one-step launch
        lds_barrier();                             // level n+1 rows in
        if (has2) step2(x2, carry);
        has2 = next2;
        x2 = nx2;
        carry = next;
    }
}

// Two steps of every shot in one launch (2D, the rolling two-step body): levels n+1 and
// n+2 from buffers buf[bufs & 3] (u^n) and buf[(bufs >> 2) & 3] (u^{n-1})
// into buf[(bufs >> 4) & 3] (u^{n+1}) and buf[(bufs >> 6) & 3] (u^{n+2}),
// with the injection rows n and n+1.  Blocks past a shot's tiles sample
// u^n into row n of d (flags & 2) and u^{n-1} into row n-1 (flags & 4);
// flags & 1 runs the tiles (a launch with flags 4 only samples, after the
// last pass); with flags & 8 the tiles take one step only (u^{n+1} into
// buf[(bufs >> 4) & 3]), which starts a run with an odd number of steps.
template <int R>
__global__ __launch_bounds__(kSlab2Threads, WAVE_SLAB2_WPE) void k_step_batch2(const ShotDesc* __restrict__ shots,
                                                               const int64_t* __restrict__ begin,
                                                               int32_t nshots, int32_t n, int32_t bufs,
                                                               int32_t flags)
{
    constexpr int NT = kSlab2Threads;
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nshots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const ShotDesc& D = shots[lo];
    StepArgs a = D.a;
    const float* u0 = D.buf[bufs & 3];
    const float* um = D.buf[(bufs >> 2) & 3];
    WAVE_GLOBAL float* d = G(D.d);
    const int64_t lb = b - begin[lo];
    if (lb >= a.stencil_blocks) {
        const int64_t nsb = (a.smp.npts + NT - 1) / NT;
        const int64_t sb = lb - a.stencil_blocks;
        const bool second = sb >= nsb;
        const int64_t p = (second ? sb - nsb : sb) * NT + threadIdx.x;
        if (p < a.smp.npts && d) {
            if (!second && (flags & 2)) d[(int64_t)n * D.nrec + p] = sample_point<2>(a.smp, u0, p, a.nz, a.nz);
            if (second && (flags & 4) && n >= 1)
                d[(int64_t)(n - 1) * D.nrec + p] = sample_point<2>(a.smp, um, p, a.nz, a.nz);
        }
        return;
    }
    if (!(flags & 1)) return;
    a.cur = u0;
    a.other = um;
    a.out = D.buf[(bufs >> 6) & 3];
    const float* v0 = D.nsrc ? D.q + (int64_t)n * D.nsrc : nullptr;
    const float* v1 = D.nsrc ? D.q + (int64_t)(n + 1) * D.nsrc : nullptr;
    roll2_body<R, 4, 64, kSlab2Threads / 64>(a, lb, v0, v1, D.buf[(bufs >> 4) & 3], !(flags & 8));
}

template <int DIM_, int R_, int VZ_, int TZL_, int TY_>
struct Cfg {
    static constexpr int DIM = DIM_, R = R_, VZ = VZ_, TZL = TZL_, TY = TY_;
    using T = Tile<DIM_, R_, VZ_, TZL_, TY_>;
};

// Block shapes (kShapes2D / kShapes3D in wave_internal.h).  The row length
// nz is a multiple of 4 (the library pads its fields), so every row starts
// 16-byte aligned.
template <int DIM, int R, int K>
using ShapeCfg = Cfg<DIM, R, (DIM == 2 ? kShapes2D[K] : kShapes3D[K]).vz,
                     (DIM == 2 ? kShapes2D[K] : kShapes3D[K]).tzl,
                     (DIM == 2 ? kShapes2D[K] : kShapes3D[K]).ty>;

template <int DIM, int R, class F>
hipError_t with_shape(int variant, int64_t nz, F&& f)
{
    if (nz % 4 != 0) return hipErrorInvalidValue;
    if constexpr (DIM == 2) {
        switch (variant) {
        case 0: return f(ShapeCfg<2, R, 0>{});
        case 1: return f(ShapeCfg<2, R, 1>{});
        case 2: return f(ShapeCfg<2, R, 2>{});
        case 3: return f(ShapeCfg<2, R, 3>{});
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (variant) {
        case 0: return f(ShapeCfg<3, R, 0>{});
        case 1: return f(ShapeCfg<3, R, 1>{});
        case 2: return f(ShapeCfg<3, R, 2>{});
        case 3: return f(ShapeCfg<3, R, 3>{});
        case 4: return f(ShapeCfg<3, R, 4>{});
        case 5: return f(ShapeCfg<3, R, 5>{});
        case 6: return f(ShapeCfg<3, R, 6>{});
        case 7: return f(ShapeCfg<3, R, 7>{});
        case 8: return f(ShapeCfg<3, R, 8>{});
        case 9: return f(ShapeCfg<3, R, 9>{});
        case 10: return f(ShapeCfg<3, R, 10>{});
        default: return hipErrorInvalidValue;
        }
    }
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
            // at the same rows; up to order 12 two rounds of them measured
            // fastest (256^3 order 8: 52.2 us at 16-plane chunks against
            // 53.5 us at 32), at order 16 one round (512^3: 470 us at 256
            // planes against 508 us at 128)
            if (C::VZ == 2 && C::R <= 6) want *= 2;
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
    // single-shot launches may gather the next step's injection values
    int64_t ngb = 0;
    if (single && a.ev_out && a.ev_src && a.nent > 0) ngb = (a.nent + T::NT - 1) / T::NT;
    return part + nsb + ngb;
}

// Plan of the two-step body (2D): tiles of 256 - 2 RZ owned z, columns of
// `xchunk` rows (default kSlab2Column); two sampler groups per shot (u^n and
// u^{n-1}).
template <int R>
int64_t plan_t2(StepArgs& a, int xchunk)
{
    constexpr int RZ = (R + 3) / 4 * 4;
    constexpr int TZO = 256 - 2 * RZ;
    if (a.nz % 4 != 0) return -1;
    a.ntz = (int32_t)((a.nz + TZO - 1) / TZO);
    a.nty = 1;
    if (xchunk <= 0) xchunk = kSlab2Column;
    if (xchunk > a.nx) xchunk = (int)a.nx;
    a.xchunk = xchunk;
    const int64_t nchunk = (a.nx + xchunk - 1) / xchunk;
    a.stencil_blocks = (int64_t)a.ntz * nchunk;
    // no XCD remap: contiguous runs of columns per XCD measured no faster
    a.remap = 0;
    int64_t nsb = 0;
    if (a.smp_out && a.smp.npts > 0) nsb = 2 * ((a.smp.npts + kSlab2Threads - 1) / kSlab2Threads);
    return a.stencil_blocks + nsb;
}

// Zero fill (the persistent graph clears its barrier words with it: a kernel
// node, not a memset node).
__global__ __launch_bounds__(kBlock) void k_zero(float* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = 0.f;
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

// Grid of the persistent kernel: every block resident at once, as the
// kernel's occupancy allows (the cooperative launch refuses a larger grid),
// and never more blocks than items.
template <class K>
hipError_t persistent_grid(K kern, int nt_block, int64_t items, int* grid)
{
    int dev = 0, per_cu = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                         nt_block, 0);
    if (e != hipSuccess) return e;
    int64_t g = (int64_t)per_cu * cus;
    if (g > items) g = items;
    if (g < 1) return hipErrorInvalidConfiguration;
    *grid = (int)g;
    return hipSuccess;
}

}  // namespace

// Blocks of the step kernel of config CC (plain or imaging) resident on the
// device at once, cached per kernel (0 when the runtime cannot say).
template <class CC, bool IMG>
int64_t step_resident()
{
    static std::atomic<int64_t> cache{-1};
    return resident_blocks(k_step_stream<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY, IMG>, CC::T::NT, cache);
}

template <int O>
int64_t OrderOps<O>::plan(int ndim, TileCfg cfg, StepArgs& a, bool device)
{
    if (ndim == 2 && cfg.variant == kTwoStepVariant) return plan_t2<O / 2>(a, cfg.xchunk);
    int64_t blocks = -1;
    auto f = [&](auto C) {
        using CC = decltype(C);
        const int64_t res = (device && cfg.xchunk <= 0) ? step_resident<CC, false>() : 0;
        blocks = plan_t<CC>(a, cfg.xchunk, res, device);
        return hipSuccess;
    };
    (void)(ndim == 2 ? with_shape<2, O / 2>(cfg.variant, a.nz, f) : with_shape<3, O / 2>(cfg.variant, a.nz, f));
    return blocks;
}

template <int O>
hipError_t OrderOps<O>::step(int ndim, const StepArgs& a0, hipStream_t s, TileCfg cfg)
{
    auto f = [&](auto C) {
        using CC = decltype(C);
        auto launch = [&](auto kern, int64_t res) {
            StepArgs a = a0;
            const int64_t blocks = plan_t<CC>(a, cfg.xchunk, res, true);
            if (!(a.smp_out && a.smp.npts > 0)) a.smp.npts = 0;
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(CC::T::NT), 0, s, a);
            return hipGetLastError();
        };
        if (a0.img_grad)
            return launch(k_step_stream<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY, true>,
                          cfg.xchunk <= 0 ? step_resident<CC, true>() : 0);
        return launch(k_step_stream<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY, false>,
                      cfg.xchunk <= 0 ? step_resident<CC, false>() : 0);
    };
    return ndim == 2 ? with_shape<2, O / 2>(cfg.variant, a0.nz, f) : with_shape<3, O / 2>(cfg.variant, a0.nz, f);
}

template <int O>
hipError_t OrderOps<O>::batch(int ndim, int64_t nz_any, TileCfg cfg, const ShotDesc* shots,
                              const int64_t* begin, int32_t nshots, int64_t blocks, int32_t n,
                              hipStream_t s)
{
    auto f = [&](auto C) {
        using CC = decltype(C);
        hipLaunchKernelGGL((k_step_batch<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY>),
                           dim3((unsigned)blocks), dim3(CC::T::NT), 0, s, shots, begin, nshots, n);
        return hipGetLastError();
    };
    return ndim == 2 ? with_shape<2, O / 2>(cfg.variant, nz_any, f) : with_shape<3, O / 2>(cfg.variant, nz_any, f);
}

template <int O>
hipError_t OrderOps<O>::batch2(const ShotDesc* shots, const int64_t* begin, int32_t nshots,
                               int64_t blocks, int32_t n, int32_t bufs, int32_t flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_batch2<O / 2>, dim3((unsigned)blocks), dim3(kSlab2Threads), 0, s, shots,
                       begin, nshots, n, bufs, flags);
    return hipGetLastError();
}

template <int O>
hipError_t OrderOps<O>::persistent(int ndim, int64_t nz_any, TileCfg cfg, const ShotDesc* shots,
                                   const int64_t* begin, int32_t nshots, int64_t items, int32_t nt,
                                   unsigned int* sync, int32_t spin_limit, int* grid_used,
                                   hipStream_t s)
{
    auto f = [&](auto C) {
        using CC = decltype(C);
        auto kern = k_batch_persistent<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY>;
        int grid = 0;
        hipError_t e = persistent_grid(kern, CC::T::NT, items, &grid);
        if (e != hipSuccess) return e;
        *grid_used = grid;
        void* args[] = {(void*)&shots, (void*)&begin, (void*)&nshots, (void*)&items, (void*)&nt,
                        (void*)&sync, (void*)&spin_limit};
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3((unsigned)grid),
                                          dim3(CC::T::NT), args, 0, s);
    };
    return ndim == 2 ? with_shape<2, O / 2>(cfg.variant, nz_any, f) : with_shape<3, O / 2>(cfg.variant, nz_any, f);
}

template <int O>
hipError_t OrderOps<O>::persistent_graph(int ndim, int64_t nz_any, TileCfg cfg,
                                         const ShotDesc* shots, const int64_t* begin,
                                         int32_t nshots, int64_t items, int32_t nt,
                                         unsigned int* sync, int32_t spin_limit, int* grid_used,
                                         hipGraph_t* graph)
{
    auto f = [&](auto C) {
        using CC = decltype(C);
        auto kern = k_batch_persistent<CC::DIM, CC::R, CC::VZ, CC::TZL, CC::TY>;
        int grid = 0;
        hipError_t e = persistent_grid(kern, CC::T::NT, items, &grid);
        if (e != hipSuccess) return e;
        *grid_used = grid;
        hipGraph_t g = nullptr;
        if ((e = hipGraphCreate(&g, 0)) != hipSuccess) return e;
        // node 1: zero the barrier words
        float* sp = reinterpret_cast<float*>(sync);
        int64_t two = 2;
        void* zargs[] = {(void*)&sp, (void*)&two};
        hipKernelNodeParams zp{};
        zp.func = reinterpret_cast<void*>(k_zero);
        zp.gridDim = dim3(1);
        zp.blockDim = dim3(kBlock);
        zp.kernelParams = zargs;
        hipGraphNode_t nz = nullptr, nk = nullptr;
        e = hipGraphAddKernelNode(&nz, g, nullptr, 0, &zp);
        // node 2: the persistent kernel, with the cooperative attribute
        void* args[] = {(void*)&shots, (void*)&begin, (void*)&nshots, (void*)&items, (void*)&nt,
                        (void*)&sync, (void*)&spin_limit};
        hipKernelNodeParams kp{};
        kp.func = reinterpret_cast<void*>(kern);
        kp.gridDim = dim3((unsigned)grid);
        kp.blockDim = dim3(CC::T::NT);
        kp.kernelParams = args;
        if (e == hipSuccess) e = hipGraphAddKernelNode(&nk, g, &nz, 1, &kp);
        if (e == hipSuccess) {
            hipKernelNodeAttrValue v{};
            v.cooperative = 1;
            e = hipGraphKernelNodeSetAttribute(nk, hipKernelNodeAttributeCooperative, &v);
        }
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return e;
        }
        *graph = g;
        return hipSuccess;
    };
    return ndim == 2 ? with_shape<2, O / 2>(cfg.variant, nz_any, f) : with_shape<3, O / 2>(cfg.variant, nz_any, f);
}

}  // namespace wave
