// Density, gradient and force interaction loops (paper Sec. 2.1: per reference
// particle, a weighted sum over the neighbours inside its support radius).
//
// Mapping on gfx950.  One wave64 owns an i-tile: up to 64 consecutive packed
// particles of one cell, one per lane.  It walks the j-tiles of the partner
// cell(s) in three steps:
//   1. tile cull -- lane k tests j-tile k of the item's j-tile list against
//      the i-tile's box (tile boxes are written by the pack kernel), so one
//      ballot culls 64 tiles with one round trip to memory;
//   2. stage -- for each surviving tile lane k holds j-particle k (the next
//      tile's records are already in flight), drops it when it is beyond
//      reach of the i-tile's box, and the survivors are compacted (ballot +
//      mbcnt) into an LDS candidate window together with the per-particle
//      quantities the pair term needs (sound speed, A = P/(Omega rho^2),
//      Balsara-limited viscosity, ...), computed once per candidate;
//   3. when the window is full (or the tile list ends) every lane tests every
//      candidate (broadcast LDS reads, ~8 VALU each) and records the hits as
//      bits; then each lane walks only its own set bits and evaluates the pair
//      term, reading the candidate record from LDS.
// Sums stay in registers: no atomics, a fixed order per lane, so results are
// deterministic.  FP32 VALU throughout: pairwise kernel sums are not a dense
// contraction, so MFMA does not apply.
//
// Two work sources share the code:
//   per-task (MODE 0): an item is one 64-slot chunk of one side of a task; the
//     partner is the other side (the same side for a self task); results are
//     the task's partial sums per slot, reduced later by unpack;
//   batched (MODE 1): an item is one tile of one cell, pulled from a device
//     work queue in descending-cost order; the partners are all neighbour
//     cells of the cell, each translated into its frame; results are final.
#include <hip/hip_runtime.h>

#include "sph_internal.hpp"

namespace sph {

struct InteractArgs {
    const char *pack;
    int64_t P;
    const float4 *bounds;
    float *res;
    int32_t *counts;
    const Chunk *items_chunks;  // MODE 0: chunk table; MODE 1: tile table
    int64_t chunk_base;         // MODE 0
    int64_t slot_base;          // MODE 0
    int64_t nitems;
    const int32_t *items;       // MODE 1: tile order
    const CellRange *cellr;
    const Nbr *nbr;
    const int32_t *nbr_off;
    const int32_t *jt_off;      // MODE 1: per cell j-tile list
    const JTile *jt;
    int32_t *queue;
    int32_t use_queue;
    float gam, beta, eps;
};

__device__ __forceinline__ float wmin(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wmax(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// wave-scope ordering of LDS traffic between lanes of one wave
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// cubic spline pieces in q = r / H: w(q), w'(q) and w'(q)/q (clamped at q = 1)
__device__ __forceinline__ void spline_w_dw(float q, float &w, float &dw)
{
    const float t = fmaxf(1.0f - q, 0.0f), t2 = t * t, q2 = q * q;
    const bool in = q < 0.5f;
    w = in ? fmaf(6.0f * q2, q - 1.0f, 1.0f) : 2.0f * t2 * t;
    dw = in ? q * fmaf(18.0f, q, -12.0f) : -6.0f * t2;
}
// w'(q)/q given r and H / r (inner branch needs no division)
__device__ __forceinline__ float spline_f(float q, float H_over_r)
{
    const float t = fmaxf(1.0f - q, 0.0f);
    return q < 0.5f ? fmaf(18.0f, q, -12.0f) : -6.0f * t * t * H_over_r;
}

// ---------------------------------------------------------------------------
// per-loop data: i registers, LDS candidate window, pair terms
// ---------------------------------------------------------------------------
// LDS candidate window of one wave.  ph holds, per candidate, the position
// relative to the i-tile centre and -|x|^2 (the phase-1 test reads only ph,
// plus H^2 for the force loop); the other planes feed the pair term.
template <int LOOP, int WIN>
struct Lds;

template <int WIN>
struct Lds<0, WIN> {
    float4 ph[WIN];  // x y z -|x|^2
    float m[WIN];
    int32_t jslot[WIN];
    uint32_t mask[WIN / 32][64];
};
template <int WIN>
struct Lds<1, WIN> {
    float4 ph[WIN];  // x y z -|x|^2
    float4 c1[WIN];  // vx vy vz m
    float4 c2[WIN];  // u m/rho c -
    int32_t jslot[WIN];
    uint32_t mask[WIN / 32][64];
};
template <int WIN>
struct Lds<2, WIN> {
    float4 ph[WIN];  // x y z -|x|^2
    float4 c1[WIN];  // vx vy vz m
    float4 c2[WIN];  // H 1/H A c
    float4 c3[WIN];  // K5 alpha~ alpha_d rho
    float2 c4[WIN];  // u H^2
    int32_t jslot[WIN];
    uint32_t mask[WIN / 32][64];
};

struct IData {
    float x, y, z, H, H2, invH;    // position relative to the i-tile centre
    float vx, vy, vz, u, c;
    float K5, A, at, ad, rho;
    float nx2, ny2, nz2;            // -2 x, -2 y, -2 z (phase-1 test)
    float t0;                       // |x|^2 - delta - H^2 (density, gradient) or |x|^2 - delta (force)
    float ri, xi2;                  // |x| and |x|^2
    float rj;                       // bound on |x_j| of staged candidates (tile centre frame)
    int32_t slot;
};

// Rounding bound of the phase-1 test: every intermediate is at most 2 R^2 with
// R = |x_i| + max |x_j| >= the supports involved, and the test takes 13
// roundings, so 20 * 2^-24 R^2 bounds the error; delta uses 2^-17 R^2.
__device__ __forceinline__ float test_delta(float ri, float rj)
{
    const float R = ri + rj;
    return 0x1p-17f * R * R;
}

struct Acc {
    float s0, s1, s2, s3, s4, s5;
    int32_t n;
};

template <int LOOP>
__device__ __forceinline__ void load_i(const InteractArgs &a, int64_t slot, bool valid, IData &d)
{
    d.slot = (int32_t)slot;
    if (!valid) {
        d.x = d.y = d.z = 0.f;
        d.H = 0.f;
        d.H2 = -1.f;
        d.invH = 0.f;
        d.vx = d.vy = d.vz = d.u = d.c = d.K5 = d.A = d.at = d.ad = d.rho = 0.f;
        return;
    }
    const float4 p0 = ((const float4 *)a.pack)[slot];
    d.x = p0.x;
    d.y = p0.y;
    d.z = p0.z;
    d.H = kGammaK * p0.w;
    d.H2 = d.H * d.H;
    d.invH = 1.0f / d.H;
    const float g = a.gam;
    if constexpr (LOOP >= 1) {
        const float4 p1 = ((const float4 *)(a.pack + a.P * 16))[slot];
        d.vx = p1.x;
        d.vy = p1.y;
        d.vz = p1.z;
        if constexpr (LOOP == 1) {
            const float2 p2 = ((const float2 *)(a.pack + a.P * 32))[slot];
            d.u = p2.x;
        } else {
            const float4 p2 = ((const float4 *)(a.pack + a.P * 32))[slot];
            const float4 p3 = ((const float4 *)(a.pack + a.P * 48))[slot];
            const float ad = ((const float *)(a.pack + a.P * 64))[slot];
            const float h = p0.w, u = p2.x, rho = p2.y, rdh = p2.z, D = p2.w;
            d.u = u;
            d.rho = rho;
            d.ad = ad;
            const float ih = d.invH;
            d.K5 = kC3 * ih * ih * ih * ih * ih;
            const float omega_rho = rho + h * rdh * (1.0f / 3.0f);  // Omega * rho
            d.A = (g - 1.0f) * u / omega_rho;
            const float c = sqrtf(g * (g - 1.0f) * u);
            const float irho = 1.0f / rho;
            const float div = fabsf(D * irho);
            const float curl = sqrtf(p3.x * p3.x + p3.y * p3.y + p3.z * p3.z) * irho;
            d.at = p3.w * div / (div + curl + a.eps * c / h);
            d.c = c;
        }
        if constexpr (LOOP == 1) d.c = sqrtf(g * (g - 1.0f) * d.u);
    }
}

// the packed record of one j particle, held in registers between its load and
// its staging (loaded one tile ahead of use)
template <int LOOP>
struct JRec;
template <>
struct JRec<0> {
    float4 p0;
    float m;
};
template <>
struct JRec<1> {
    float4 p0, p1;
    float2 p2;
};
template <>
struct JRec<2> {
    float4 p0, p1, p2, p3;
    float ad;
};

template <int LOOP>
__device__ __forceinline__ void load_j(const InteractArgs &a, int64_t js, bool ok, JRec<LOOP> &r)
{
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (LOOP == 0) {
        r.p0 = ok ? ((const float4 *)a.pack)[js] : z4;
        r.m = ok ? ((const float *)(a.pack + a.P * 16))[js] : 0.f;
    } else if constexpr (LOOP == 1) {
        r.p0 = ok ? ((const float4 *)a.pack)[js] : z4;
        r.p1 = ok ? ((const float4 *)(a.pack + a.P * 16))[js] : z4;
        r.p2 = ok ? ((const float2 *)(a.pack + a.P * 32))[js] : make_float2(0.f, 0.f);
    } else {
        r.p0 = ok ? ((const float4 *)a.pack)[js] : z4;
        r.p1 = ok ? ((const float4 *)(a.pack + a.P * 16))[js] : z4;
        r.p2 = ok ? ((const float4 *)(a.pack + a.P * 32))[js] : z4;
        r.p3 = ok ? ((const float4 *)(a.pack + a.P * 48))[js] : z4;
        r.ad = ok ? ((const float *)(a.pack + a.P * 64))[js] : 0.f;
    }
}

// stage candidate j (record r, pack slot js, translated by (tx,ty,tz) and
// shifted to the i-tile centre (cx,cy,cz)) at LDS index k
template <int LOOP, int WIN>
__device__ __forceinline__ void stage_j(const InteractArgs &a, Lds<LOOP, WIN> &L, int k, int64_t js,
                                        const JRec<LOOP> &r, float tx, float ty, float tz, float cx, float cy,
                                        float cz)
{
    const float g = a.gam;
    const float x = (r.p0.x + tx) - cx, y = (r.p0.y + ty) - cy, z = (r.p0.z + tz) - cz;
    L.jslot[k] = (int32_t)js;
    L.ph[k] = make_float4(x, y, z, -fmaf(z, z, fmaf(y, y, x * x)));
    if constexpr (LOOP == 0) {
        L.m[k] = r.m;
    } else if constexpr (LOOP == 1) {
        L.c1[k] = r.p1;
        L.c2[k] = make_float4(r.p2.x, r.p1.w / r.p2.y, sqrtf(g * (g - 1.0f) * r.p2.x), 0.f);
    } else {
        const float h = r.p0.w, u = r.p2.x, rho = r.p2.y, rdh = r.p2.z, D = r.p2.w;
        const float H = kGammaK * h, ih = 1.0f / H;
        const float A = (g - 1.0f) * u / (rho + h * rdh * (1.0f / 3.0f));
        const float c = sqrtf(g * (g - 1.0f) * u);
        const float irho = 1.0f / rho;
        const float div = fabsf(D * irho);
        const float curl = sqrtf(r.p3.x * r.p3.x + r.p3.y * r.p3.y + r.p3.z * r.p3.z) * irho;
        const float at = r.p3.w * div / (div + curl + a.eps * c / h);
        L.c1[k] = r.p1;
        L.c2[k] = make_float4(H, ih, A, c);
        L.c3[k] = make_float4(kC3 * ih * ih * ih * ih * ih, at, r.ad, rho);
        L.c4[k] = make_float2(u, H * H);
    }
}

// Phase-1 test of candidate k, as a sign: the result is negative when
// |x_i - x_j|^2 < H^2 + delta_i, evaluated as |x_i|^2 - delta_i - H^2 + |x_j|^2 -
// 2 x_i.x_j with delta_i covering the rounding of these four operations, so the
// hits are a superset of the exact test that the pair term applies again.
template <int LOOP, int WIN>
__device__ __forceinline__ float test_sign(const Lds<LOOP, WIN> &L, int k, const IData &d)
{
    const float4 q = L.ph[k];
    float t;
    if constexpr (LOOP == 2) t = (d.t0 - fmaxf(d.H2, L.c4[k].y)) - q.w;
    else t = d.t0 - q.w;
    return fmaf(d.nx2, q.x, fmaf(d.ny2, q.y, fmaf(d.nz2, q.z, t)));
}

template <int LOOP, int WIN>
__device__ __forceinline__ void pair(const InteractArgs &a, const Lds<LOOP, WIN> &L, int k, const IData &d,
                                     Acc &acc)
{
    const float4 c0 = L.ph[k];
    const float rx = d.x - c0.x, ry = d.y - c0.y, rz = d.z - c0.z;
    const float r2 = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
    if constexpr (LOOP == 0) {
        if (!(r2 < d.H2)) return;  // the exact criterion
        const float mj = L.m[k];
        const float r = fast_sqrt(r2);
        const float q = r * d.invH;
        float w, dw;
        spline_w_dw(q, w, dw);
        acc.s0 = fmaf(mj, w, acc.s0);                      // sum m w
        acc.s1 = fmaf(mj, fmaf(q, dw, 3.0f * w), acc.s1);  // sum m (3w + q w')
        acc.s2 += w;                                       // sum w
        acc.n++;
    } else {
        if (L.jslot[k] == d.slot) return;  // j != i
        if constexpr (LOOP == 1) {
            if (!(r2 < d.H2)) return;
        } else {
            if (!(r2 < fmaxf(d.H2, L.c4[k].y))) return;
        }
        const float4 c1 = L.c1[k];
        const float vx = d.vx - c1.x, vy = d.vy - c1.y, vz = d.vz - c1.z;
        const float invr = r2 > 0.f ? fast_rsq(r2) : 0.f;
        const float r = r2 * invr;
        const float dot = fmaf(vz, rz, fmaf(vy, ry, vx * rx));
        const float mu = fminf(dot * invr, 0.0f);
        if constexpr (LOOP == 1) {
            const float4 c2 = L.c2[k];  // u m/rho c
            const float f = spline_f(r * d.invH, d.H * invr);    // w'/q
            const float mf = c1.w * f;
            acc.s0 = fmaf(mf, dot, acc.s0);                                   // D
            acc.s1 = fmaf(mf, fmaf(vy, rz, -vz * ry), acc.s1);                // R
            acc.s2 = fmaf(mf, fmaf(vz, rx, -vx * rz), acc.s2);
            acc.s3 = fmaf(mf, fmaf(vx, ry, -vy * rx), acc.s3);
            acc.s4 = fmaf(c2.y * (d.u - c2.x), f, acc.s4);                    // L / 2
            acc.s5 = fmaxf(acc.s5, d.c + c2.z - a.beta * mu);                 // V
            acc.n++;
        } else {
            const float4 c2 = L.c2[k];  // H 1/H A c
            const float4 c3 = L.c3[k];  // K5 at ad rho
            const float2 c4 = L.c4[k];  // u H^2
            const float uj = c4.x;
            const float fi = r2 < d.H2 ? d.K5 * spline_f(r * d.invH, d.H * invr) : 0.0f;
            const float fj = r2 < c4.y ? c3.x * spline_f(r * c2.y, c2.x * invr) : 0.0f;
            const float fb = 0.5f * (fi + fj);
            const float vsig = d.c + c2.w - a.beta * mu;
            const float irb = fast_rcp(0.5f * (d.rho + c3.w));
            const float Pi = -0.25f * (d.at + c3.y) * vsig * mu * irb;
            const float mj = c1.w;
            const float s = fmaf(d.A, fi, fmaf(c2.z, fj, Pi * fb));
            const float ms = mj * s;
            acc.s0 = fmaf(-ms, rx, acc.s0);
            acc.s1 = fmaf(-ms, ry, acc.s1);
            acc.s2 = fmaf(-ms, rz, acc.s2);
            const float cond = 0.5f * (d.ad + c3.z) * fabsf(dot) * (d.u - uj) * fb * irb;
            acc.s3 = fmaf(mj, fmaf(d.A * fi, dot, fmaf(0.5f * Pi * fb, dot, cond)), acc.s3);
            acc.n++;
        }
    }
}

template <int LOOP>
__device__ __forceinline__ void write_out(const InteractArgs &a, const IData &d, const Acc &acc)
{
    float *r = a.res;
    const int64_t P = a.P, s = d.slot;
    if constexpr (LOOP == 0) {
        const float ih3 = d.invH * d.invH * d.invH;
        r[s] = kC3 * ih3 * acc.s0;
        r[P + s] = -kGammaK * kC3 * ih3 * d.invH * acc.s1;
        r[2 * P + s] = kC3 * ih3 * acc.s2;
    } else if constexpr (LOOP == 1) {
        const float ih = d.invH, K = kC3 * ih * ih * ih * ih * ih;
        r[s] = K * acc.s0;
        r[P + s] = K * acc.s1;
        r[2 * P + s] = K * acc.s2;
        r[3 * P + s] = K * acc.s3;
        r[4 * P + s] = 2.0f * K * acc.s4;
        r[5 * P + s] = acc.s5;
    } else {
        r[s] = acc.s0;
        r[P + s] = acc.s1;
        r[2 * P + s] = acc.s2;
        r[3 * P + s] = acc.s3;
    }
    if (a.counts) a.counts[s] = acc.n;
}

// test every staged candidate against every lane, then walk each lane's hits
template <int LOOP, int WIN>
__device__ __forceinline__ void flush(const InteractArgs &a, Lds<LOOP, WIN> &L, int nc, const IData &d,
                                   bool valid, Acc &acc)
{
    const int lane = threadIdx.x & 63;
    wave_sync();
    nc = __builtin_amdgcn_readfirstlane(nc);
    const int nw = (nc + 31) >> 5;
    IData dd = d;
    if constexpr (LOOP == 2) dd.t0 = dd.xi2 - test_delta(dd.ri, dd.rj);
    for (int w = 0; w < nw; ++w) {
        uint32_t m = 0;
        const int kb = 32 * w;
        const int kn = __builtin_amdgcn_readfirstlane(min(32, nc - kb));
        // shift each candidate's sign bit in: candidate kb + b ends at bit 31 - b
        if (kn == 32) {
#pragma unroll 16
            for (int b = 0; b < 32; ++b)
                m = __builtin_amdgcn_alignbit(m, __float_as_uint(test_sign<LOOP, WIN>(L, kb + b, dd)), 31);
        } else {
            for (int b = 0; b < kn; ++b)
                m = __builtin_amdgcn_alignbit(m, __float_as_uint(test_sign<LOOP, WIN>(L, kb + b, dd)), 31);
            m <<= (32 - kn);
        }
        L.mask[w][lane] = valid ? m : 0u;
    }
    wave_sync();
    if (nw == 0) return;
    int w = 0;
    uint32_t cur = L.mask[0][lane];
    for (;;) {
        while (cur == 0 && w + 1 < nw) {
            ++w;
            cur = L.mask[w][lane];
        }
        const bool act = cur != 0;
        if (!__any(act)) break;
        if (act) {
            const int b = __builtin_clz(cur);
            cur &= ~(0x80000000u >> b);
            pair<LOOP, WIN>(a, L, 32 * w + b, d, acc);
        }
    }
    wave_sync();
}

// one j-tile as seen by one lane during the cull: slots, translation, box
struct TileInfo {
    int64_t js0;
    int32_t jn;
    float tx, ty, tz;
};

__device__ __forceinline__ TileInfo bcast(const TileInfo &t, int l)
{
    TileInfo o;
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(uint64_t)t.js0, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)t.js0 >> 32), l);
    o.js0 = (int64_t)(((uint64_t)hi << 32) | lo);
    o.jn = __builtin_amdgcn_readlane(t.jn, l);
    o.tx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t.tx), l));
    o.ty = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t.ty), l));
    o.tz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t.tz), l));
    return o;
}

// stage the j particles of one tile that reach the i box; flush when full
template <int LOOP, int WIN>
__device__ __forceinline__ void stage_tile(const InteractArgs &a, Lds<LOOP, WIN> &L, int &nc, const TileInfo &t,
                                           const JRec<LOOP> &r, const IData &d, bool valid, const float4 &lo,
                                           const float4 &hi, const float4 &cen, Acc &acc)
{
    const int lane = threadIdx.x & 63;
    const float hmi = lo.w;
    bool keep = false;
    if (lane < t.jn) {
        const float x = r.p0.x + t.tx, y = r.p0.y + t.ty, z = r.p0.z + t.tz;
        const float ex = fmaxf(fmaxf(lo.x - x, x - hi.x), 0.f);
        const float ey = fmaxf(fmaxf(lo.y - y, y - hi.y), 0.f);
        const float ez = fmaxf(fmaxf(lo.z - z, z - hi.z), 0.f);
        const float reach = LOOP == 2 ? fmaxf(hmi, kGammaK * r.p0.w) : hmi;
        keep = fmaf(ez, ez, fmaf(ey, ey, ex * ex)) < reach * reach * 1.0001f;
    }
    const uint64_t bal = __ballot(keep);
    const int cnt = __popcll(bal);
    if (cnt == 0) return;
    if (nc + cnt > WIN) {
        flush<LOOP, WIN>(a, L, nc, d, valid, acc);
        nc = 0;
    }
    if (keep) {
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        stage_j<LOOP, WIN>(a, L, nc + rank, t.js0 + lane, r, t.tx, t.ty, t.tz, cen.x, cen.y, cen.z);
    }
    nc = __builtin_amdgcn_readfirstlane(nc + cnt);
}

// gather the candidates of one item's j-tile list (nj tiles) into the window
template <int LOOP, int MODE, int WIN>
__device__ __forceinline__ void scan_item(const InteractArgs &a, Lds<LOOP, WIN> &L, int &nc, const Chunk &ch,
                                          IData &d, bool valid, const float4 &lo, const float4 &hi,
                                          const float4 &cen, Acc &acc)
{
    const float ex = hi.x - lo.x, ey = hi.y - lo.y, ez = hi.z - lo.z;
    const float halfdiag = 0.5f * sqrtf(fmaxf(ex * ex + ey * ey + ez * ez, 0.f));
    float hjm = 0.f;  // largest support of the surviving j-tiles so far
    const int lane = threadIdx.x & 63;
    int nj, jt0 = 0;
    if (MODE == 0) {
        nj = (ch.jn + 63) >> 6;
    } else {
        jt0 = a.jt_off[ch.cell];
        nj = a.jt_off[ch.cell + 1] - jt0;
    }
    const float hmi = lo.w;
    for (int base = 0; base < nj; base += 64) {
        // 1. lane-parallel cull of up to 64 j-tiles on their stored boxes
        TileInfo ti{0, 0, 0.f, 0.f, 0.f};
        bool ok = false;
        const int q = base + lane;
        if (q < nj) {
            float4 blo, bhi;
            if (MODE == 0) {
                const int64_t bt = (int64_t)ch.jchunk0 - a.chunk_base + q;
                blo = a.bounds[2 * bt];
                bhi = a.bounds[2 * bt + 1];
                ti.js0 = ch.jslot0 - a.slot_base + 64 * (int64_t)q;
                ti.jn = min(64, ch.jn - 64 * q);
            } else {
                const JTile e = a.jt[jt0 + q];
                const Nbr nb = a.nbr[e.nbr];
                const Chunk tj = a.items_chunks[e.tile];
                blo = a.bounds[2 * (int64_t)e.tile];
                bhi = a.bounds[2 * (int64_t)e.tile + 1];
                ti.js0 = tj.slot0;
                ti.jn = tj.n;
                ti.tx = nb.dx;
                ti.ty = nb.dy;
                ti.tz = nb.dz;
            }
            const float gx = fmaxf(fmaxf(blo.x + ti.tx - hi.x, lo.x - (bhi.x + ti.tx)), 0.f);
            const float gy = fmaxf(fmaxf(blo.y + ti.ty - hi.y, lo.y - (bhi.y + ti.ty)), 0.f);
            const float gz = fmaxf(fmaxf(blo.z + ti.tz - hi.z, lo.z - (bhi.z + ti.tz)), 0.f);
            const float reach = LOOP == 2 ? fmaxf(hmi, blo.w) : hmi;
            ok = fmaf(gz, gz, fmaf(gy, gy, gx * gx)) < reach * reach * 1.0001f;
        }
        uint64_t m = __ballot(ok);
        if (m == 0) continue;
        if constexpr (LOOP == 2) {
            // candidates of these tiles reach at most max(i-tile support, their tile's support)
            float hj = 0.f;
            if (ok) hj = MODE == 0 ? a.bounds[2 * ((int64_t)ch.jchunk0 - a.chunk_base + q)].w
                                   : a.bounds[2 * (int64_t)a.jt[jt0 + q].tile].w;
            hjm = fmaxf(hjm, wmax(hj));
            d.rj = halfdiag + 1.001f * fmaxf(hmi, hjm);
        }
        // 2. stage surviving tiles, the next tile's records loaded ahead
        int cur = __builtin_ctzll(m);
        m &= m - 1;
        TileInfo ct = bcast(ti, cur);
        JRec<LOOP> cr;
        load_j<LOOP>(a, ct.js0 + lane, lane < ct.jn, cr);
        for (;;) {
            const bool more = m != 0;
            TileInfo nt = ct;
            JRec<LOOP> nr;
            if (more) {
                const int nx = __builtin_ctzll(m);
                m &= m - 1;
                nt = bcast(ti, nx);
                load_j<LOOP>(a, nt.js0 + lane, lane < nt.jn, nr);
            }
            stage_tile<LOOP, WIN>(a, L, nc, ct, cr, d, valid, lo, hi, cen, acc);
            if (!more) break;
            ct = nt;
            cr = nr;
        }
    }
}

template <int LOOP, int MODE, int WIN>
__global__ __launch_bounds__(256) void k_interact(InteractArgs a)
{
    __shared__ Lds<LOOP, WIN> lds[4];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    Lds<LOOP, WIN> &L = lds[wv];
    const int64_t wave_id = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + wv));
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    int64_t iter = 0;
    for (;;) {
        int64_t item;
        if (MODE == 0) {
            item = iter == 0 ? wave_id : a.nitems;
        } else if (a.use_queue) {
            int v = 0;
            if (lane == 0) v = atomicAdd(a.queue, 1);
            item = __builtin_amdgcn_readfirstlane(v);
        } else {
            item = wave_id + iter * nwaves;
        }
        ++iter;
        if (item >= a.nitems) break;
        Chunk ch;
        int64_t islot;
        if (MODE == 0) {
            ch = a.items_chunks[a.chunk_base + item];
            islot = ch.slot0 - a.slot_base + lane;
        } else {
            ch = a.items_chunks[a.items[item]];
            islot = ch.slot0 + lane;
        }
        const bool valid = lane < ch.n;
        IData d;
        load_i<LOOP>(a, islot, valid, d);
        const float inf = __builtin_huge_valf();
        float4 lo, hi;
        lo.x = wmin(valid ? d.x : inf);
        lo.y = wmin(valid ? d.y : inf);
        lo.z = wmin(valid ? d.z : inf);
        lo.w = wmax(valid ? d.H : 0.f);
        hi.x = wmax(valid ? d.x : -inf);
        hi.y = wmax(valid ? d.y : -inf);
        hi.z = wmax(valid ? d.z : -inf);
        hi.w = 0.f;
        // i positions relative to the tile centre; phase-1 constants
        float4 cen;
        cen.x = 0.5f * (lo.x + hi.x);
        cen.y = 0.5f * (lo.y + hi.y);
        cen.z = 0.5f * (lo.z + hi.z);
        cen.w = 0.f;
        {
            const float ex = hi.x - lo.x, ey = hi.y - lo.y, ez = hi.z - lo.z;
            const float halfdiag = valid ? 0.5f * sqrtf(ex * ex + ey * ey + ez * ez) : 0.f;
            d.x -= cen.x;
            d.y -= cen.y;
            d.z -= cen.z;
            d.ri = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
            d.xi2 = fmaf(d.z, d.z, fmaf(d.y, d.y, d.x * d.x));
            d.rj = halfdiag + 1.001f * lo.w;
            d.nx2 = -2.0f * d.x;
            d.ny2 = -2.0f * d.y;
            d.nz2 = -2.0f * d.z;
            d.t0 = (d.xi2 - test_delta(d.ri, d.rj)) - d.H2;
        }
        Acc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0};
        int nc = 0;
        scan_item<LOOP, MODE, WIN>(a, L, nc, ch, d, valid, lo, hi, cen, acc);
        if (nc > 0) flush<LOOP, WIN>(a, L, nc, d, valid, acc);
        if (valid) write_out<LOOP>(a, d, acc);
    }
}

__global__ void k_reset_queue(int32_t *q) { *q = 0; }

template <int LOOP, int MODE, int WIN>
static void launch_one(const InteractArgs &a, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_interact<LOOP, MODE, WIN>), dim3(grid), dim3(256), 0, st, a);
}

template <int LOOP, int MODE>
static sph_status launch_win(const InteractArgs &a, int win, unsigned grid, hipStream_t st)
{
    switch (win) {
    case 64: launch_one<LOOP, MODE, 64>(a, grid, st); break;
    case 128: launch_one<LOOP, MODE, 128>(a, grid, st); break;
    case 256: launch_one<LOOP, MODE, 256>(a, grid, st); break;
    case 512:
        if constexpr (LOOP == 2) return fail(SPH_E_ARG, "force window is at most 256");
        else launch_one<LOOP, MODE, 512>(a, grid, st);
        break;
    default: return fail(SPH_E_ARG, "bad window");
    }
    SPH_CHECK_LAUNCH("interaction launch");
    return SPH_OK;
}

sph_status launch_interact(const sph_plan *p, int loop, bool cells, int32_t t0, int32_t t1, const void *pack,
                           const sph_params *prm, const sph_tuning *tn, void *res, int32_t *counts, void *ws,
                           hipStream_t st)
{
    InteractArgs a{};
    a.pack = (const char *)pack;
    a.res = (float *)res;
    a.counts = counts;
    a.gam = prm->gamma_ad;
    a.beta = prm->beta_visc;
    a.eps = prm->balsara_eps;
    int win;
    unsigned grid;
    if (!cells) {
        const int64_t ns = p->slot_off[t1] - p->slot_off[t0];
        a.P = round_slots(ns);
        a.items_chunks = p->d_chunks;
        a.chunk_base = p->chunk_off[t0];
        a.slot_base = p->slot_off[t0];
        a.nitems = p->chunk_off[t1] - p->chunk_off[t0];
        a.bounds = (const float4 *)(a.pack + a.P * 4 * kPackFloats[loop]);
        if (a.nitems == 0) return SPH_OK;
        grid = (unsigned)((a.nitems + 3) / 4);
        win = loop == 0 ? 128 : (loop == 1 ? 128 : 64);
        if (p->max_cell > 64) win = loop == 2 ? 128 : 256;
    } else {
        a.P = round_slots(p->n);
        a.items_chunks = p->d_tiles;
        a.items = p->d_items;
        a.nitems = p->ntile;
        a.cellr = p->d_cellr;
        a.nbr = p->d_nbr;
        a.nbr_off = p->d_nbr_off;
        a.jt_off = p->d_jt_off;
        a.jt = p->d_jt;
        a.bounds = (const float4 *)(a.pack + a.P * 4 * kPackFloats[loop]);
        a.queue = (int32_t *)ws;
        a.use_queue = tn->queue;
        if (a.nitems == 0) return SPH_OK;
        grid = (unsigned)std::min<int64_t>((int64_t)tn->blocks_per_cu * p->num_cu, (a.nitems + 3) / 4);
        win = tn->window[loop];
        if (a.use_queue) {
            hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, st, a.queue);
            SPH_CHECK_LAUNCH("queue reset launch");
        }
    }
    if (loop == 0) return cells ? launch_win<0, 1>(a, win, grid, st) : launch_win<0, 0>(a, win, grid, st);
    if (loop == 1) return cells ? launch_win<1, 1>(a, win, grid, st) : launch_win<1, 0>(a, win, grid, st);
    return cells ? launch_win<2, 1>(a, win, grid, st) : launch_win<2, 0>(a, win, grid, st);
}

}  // namespace sph
