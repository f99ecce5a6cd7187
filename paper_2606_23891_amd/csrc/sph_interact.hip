// Density, gradient and force interaction loops (paper Sec. 2.1: per reference
// particle, a weighted sum over the neighbours inside its support radius).
//
// Mapping on gfx950.  One wave64 owns an i-tile: up to 64 consecutive packed
// particles of one cell, one per lane.  It walks the j-tiles of the partner
// cell(s) in three steps:
//   1. tile cull -- a j-tile whose bounding box (written by the pack kernel)
//      lies beyond the i-tile's reach is skipped whole;
//   2. stage -- lane k loads j-particle k of a surviving tile, drops it when
//      it is beyond reach of the i-tile's box, and the survivors are compacted
//      (ballot + mbcnt) into an LDS candidate window together with the
//      per-particle quantities the pair term needs (sound speed, A = P/(Omega
//      rho^2), Balsara-limited viscosity, ...), computed once per candidate;
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
template <int LOOP, int WIN>
struct Lds;

template <int WIN>
struct Lds<0, WIN> {
    float4 c0[WIN];  // x y z m
    int32_t jslot[WIN];
    uint32_t mask[WIN / 32][64];
};
template <int WIN>
struct Lds<1, WIN> {
    float4 c0[WIN];  // x y z m
    float4 c1[WIN];  // vx vy vz c
    float2 c2[WIN];  // u m/rho
    int32_t jslot[WIN];
    uint32_t mask[WIN / 32][64];
};
template <int WIN>
struct Lds<2, WIN> {
    float4 c0[WIN];  // x y z H^2
    float4 c1[WIN];  // vx vy vz m
    float4 c2[WIN];  // H 1/H A c
    float4 c3[WIN];  // K5 alpha~ alpha_d rho
    float c4[WIN];   // u
    int32_t jslot[WIN];
    uint32_t mask[WIN / 32][64];
};

struct IData {
    float x, y, z, H, H2, invH;
    float vx, vy, vz, u, c;
    float K5, A, at, ad, rho;
    int32_t slot;
};

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

// stage candidate j (pack slot js, translated by (tx,ty,tz)) at LDS index k
template <int LOOP, int WIN>
__device__ __forceinline__ void stage_j(const InteractArgs &a, Lds<LOOP, WIN> &L, int k, int64_t js,
                                        const float4 &p0, float tx, float ty, float tz)
{
    const float g = a.gam;
    const float x = p0.x + tx, y = p0.y + ty, z = p0.z + tz;
    L.jslot[k] = (int32_t)js;
    if constexpr (LOOP == 0) {
        const float m = ((const float *)(a.pack + a.P * 16))[js];
        L.c0[k] = make_float4(x, y, z, m);
    } else if constexpr (LOOP == 1) {
        const float4 p1 = ((const float4 *)(a.pack + a.P * 16))[js];
        const float2 p2 = ((const float2 *)(a.pack + a.P * 32))[js];
        L.c0[k] = make_float4(x, y, z, p1.w);
        L.c1[k] = make_float4(p1.x, p1.y, p1.z, sqrtf(g * (g - 1.0f) * p2.x));
        L.c2[k] = make_float2(p2.x, p1.w / p2.y);
    } else {
        const float4 p1 = ((const float4 *)(a.pack + a.P * 16))[js];
        const float4 p2 = ((const float4 *)(a.pack + a.P * 32))[js];
        const float4 p3 = ((const float4 *)(a.pack + a.P * 48))[js];
        const float ad = ((const float *)(a.pack + a.P * 64))[js];
        const float h = p0.w, u = p2.x, rho = p2.y, rdh = p2.z, D = p2.w;
        const float H = kGammaK * h, ih = 1.0f / H;
        const float A = (g - 1.0f) * u / (rho + h * rdh * (1.0f / 3.0f));
        const float c = sqrtf(g * (g - 1.0f) * u);
        const float irho = 1.0f / rho;
        const float div = fabsf(D * irho);
        const float curl = sqrtf(p3.x * p3.x + p3.y * p3.y + p3.z * p3.z) * irho;
        const float at = p3.w * div / (div + curl + a.eps * c / h);
        L.c0[k] = make_float4(x, y, z, H * H);
        L.c1[k] = p1;
        L.c2[k] = make_float4(H, ih, A, c);
        L.c3[k] = make_float4(kC3 * ih * ih * ih * ih * ih, at, ad, rho);
        L.c4[k] = u;
    }
}

template <int LOOP>
__device__ __forceinline__ bool hit(const IData &d, const float4 &c, float &r2)
{
    const float dx = d.x - c.x, dy = d.y - c.y, dz = d.z - c.z;
    r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if constexpr (LOOP == 2) return r2 < fmaxf(d.H2, c.w);
    else return r2 < d.H2;
}

template <int LOOP, int WIN>
__device__ __forceinline__ void pair(const InteractArgs &a, const Lds<LOOP, WIN> &L, int k, const IData &d,
                                     Acc &acc)
{
    const float4 c0 = L.c0[k];
    const float rx = d.x - c0.x, ry = d.y - c0.y, rz = d.z - c0.z;
    const float r2 = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
    if constexpr (LOOP == 0) {
        const float r = fast_sqrt(r2);
        const float q = r * d.invH;
        float w, dw;
        spline_w_dw(q, w, dw);
        acc.s0 = fmaf(c0.w, w, acc.s0);                      // sum m w
        acc.s1 = fmaf(c0.w, fmaf(q, dw, 3.0f * w), acc.s1);  // sum m (3w + q w')
        acc.s2 += w;                                         // sum w
        acc.n++;
    } else {
        if (L.jslot[k] == d.slot) return;  // j != i
        const float4 c1 = L.c1[k];
        const float vx = d.vx - c1.x, vy = d.vy - c1.y, vz = d.vz - c1.z;
        const float invr = r2 > 0.f ? fast_rsq(r2) : 0.f;
        const float r = r2 * invr;
        const float dot = fmaf(vz, rz, fmaf(vy, ry, vx * rx));
        const float mu = fminf(dot * invr, 0.0f);
        if constexpr (LOOP == 1) {
            const float2 c2 = L.c2[k];
            const float f = spline_f(r * d.invH, d.H * invr);    // w'/q
            const float mf = c0.w * f;
            acc.s0 = fmaf(mf, dot, acc.s0);                                   // D
            acc.s1 = fmaf(mf, fmaf(vy, rz, -vz * ry), acc.s1);                // R
            acc.s2 = fmaf(mf, fmaf(vz, rx, -vx * rz), acc.s2);
            acc.s3 = fmaf(mf, fmaf(vx, ry, -vy * rx), acc.s3);
            acc.s4 = fmaf(c2.y * (d.u - c2.x), f, acc.s4);                    // L / 2
            acc.s5 = fmaxf(acc.s5, d.c + c1.w - a.beta * mu);                 // V
            acc.n++;
        } else {
            const float4 c2 = L.c2[k];  // H 1/H A c
            const float4 c3 = L.c3[k];  // K5 at ad rho
            const float uj = L.c4[k];
            const float fi = r2 < d.H2 ? d.K5 * spline_f(r * d.invH, d.H * invr) : 0.0f;
            const float fj = r2 < c0.w ? c3.x * spline_f(r * c2.y, c2.x * invr) : 0.0f;
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
    const int nw = (nc + 31) >> 5;
    for (int w = 0; w < nw; ++w) {
        uint32_t m = 0;
        const int kb = 32 * w;
        const int kn = min(32, nc - kb);
        if (kn == 32) {
#pragma unroll 8
            for (int b = 0; b < 32; ++b) {
                float r2;
                m |= (hit<LOOP>(d, L.c0[kb + b], r2) ? 1u : 0u) << b;
            }
        } else {
            for (int b = 0; b < kn; ++b) {
                float r2;
                m |= (hit<LOOP>(d, L.c0[kb + b], r2) ? 1u : 0u) << b;
            }
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
            const int b = __builtin_ctz(cur);
            cur &= cur - 1;
            pair<LOOP, WIN>(a, L, 32 * w + b, d, acc);
        }
    }
    wave_sync();
}

// gather the candidates of one j range (slots [js0, js0 + jn), bounds of its
// 64-slot tiles at bnd, translation t) into the window, flushing when full
template <int LOOP, int WIN>
__device__ __forceinline__ void scan_range(const InteractArgs &a, Lds<LOOP, WIN> &L, int &nc, int64_t js0,
                                           int jn, const float4 *bnd, float tx, float ty, float tz,
                                           const IData &d, bool valid, const float4 &lo, const float4 &hi,
                                           Acc &acc)
{
    const int lane = threadIdx.x & 63;
    const int ntile = (jn + 63) >> 6;
    const float hmi = lo.w;  // largest support of the i-tile
    for (int t = 0; t < ntile; ++t) {
        // 1. tile cull on the j-tile's stored box
        const float4 blo = bnd[2 * t], bhi = bnd[2 * t + 1];
        const float gx = fmaxf(fmaxf(blo.x + tx - hi.x, lo.x - (bhi.x + tx)), 0.f);
        const float gy = fmaxf(fmaxf(blo.y + ty - hi.y, lo.y - (bhi.y + ty)), 0.f);
        const float gz = fmaxf(fmaxf(blo.z + tz - hi.z, lo.z - (bhi.z + tz)), 0.f);
        const float reach_t = LOOP == 2 ? fmaxf(hmi, blo.w) : hmi;
        if (fmaf(gz, gz, fmaf(gy, gy, gx * gx)) >= reach_t * reach_t * 1.0001f) continue;
        // 2. stage the j particles of the tile that reach the i box
        const int jk = 64 * t + lane;
        const bool jv = jk < jn;
        const int64_t js = js0 + jk;
        float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f);
        bool keep = false;
        if (jv) {
            p0 = ((const float4 *)a.pack)[js];
            const float x = p0.x + tx, y = p0.y + ty, z = p0.z + tz;
            const float ex = fmaxf(fmaxf(lo.x - x, x - hi.x), 0.f);
            const float ey = fmaxf(fmaxf(lo.y - y, y - hi.y), 0.f);
            const float ez = fmaxf(fmaxf(lo.z - z, z - hi.z), 0.f);
            const float reach = LOOP == 2 ? fmaxf(hmi, kGammaK * p0.w) : hmi;
            keep = fmaf(ez, ez, fmaf(ey, ey, ex * ex)) < reach * reach * 1.0001f;
        }
        const uint64_t bal = __ballot(keep);
        const int cnt = __popcll(bal);
        if (cnt == 0) continue;
        if (nc + cnt > WIN) {
            flush<LOOP, WIN>(a, L, nc, d, valid, acc);
            nc = 0;
        }
        if (keep) {
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            stage_j<LOOP, WIN>(a, L, nc + rank, js, p0, tx, ty, tz);
        }
        nc += cnt;
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
        Acc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0};
        int nc = 0;
        if (MODE == 0) {
            scan_range<LOOP, WIN>(a, L, nc, ch.jslot0 - a.slot_base, ch.jn,
                                  a.bounds + 2 * (ch.jchunk0 - a.chunk_base), 0.f, 0.f, 0.f, d, valid, lo, hi,
                                  acc);
        } else {
            const int e0 = a.nbr_off[ch.cell], e1 = a.nbr_off[ch.cell + 1];
            for (int e = e0; e < e1; ++e) {
                const Nbr nb = a.nbr[e];
                const CellRange cr = a.cellr[nb.cell];
                scan_range<LOOP, WIN>(a, L, nc, cr.first, cr.count, a.bounds + 2 * cr.tile0, nb.dx, nb.dy, nb.dz,
                                      d, valid, lo, hi, acc);
            }
        }
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
