// Density, gradient and force interaction loops (paper Sec. 2.1: per reference
// particle, a weighted sum over the neighbours inside its support radius).
//
// Mapping on gfx950.  One wave64 owns an i-tile: up to 64 consecutive packed
// particles of one cell, one per lane.  It walks the j-tiles of the partner
// cell(s) in three steps:
//   1. tile cull -- lane k tests j-tile k of the item's j-tile list against
//      the i-tile's box (tile boxes are written by the pack kernel), so one
//      ballot culls 64 tiles with one round trip to memory;
//   2. stage -- for each surviving tile lane k holds j-particle k (the records
//      of a batch of tiles are loaded together), drops it when it is beyond
//      reach of the i-tile's box, and the survivors are compacted (ballot +
//      mbcnt) into an LDS candidate window together with the per-particle
//      quantities the pair term needs (sound speed, A = P/(Omega rho^2),
//      Balsara-limited viscosity, ...);
//   3. when the window is full (or the tile list ends) every lane's particle is
//      tested against every candidate -- the expanded distance test is a small
//      dense product, done on the matrix cores (test_words_mfma) -- and the
//      hits are recorded as bits; then each lane walks only its own set bits
//      and evaluates the pair term on the VALU, reading the candidate record
//      from LDS.
// Sums stay in registers: no atomics, a fixed order per lane, so results are
// deterministic.  The pair terms themselves are FP32 VALU work: a sum of
// per-pair nonlinear terms is not a contraction.  Each kernel comes in two
// variants: with pair counts (exact support and j != i tests before every
// term) and without (the timed one; see pair()).
//
// Two work sources share the code:
//   per-task (MODE 0): an item is one 64-slot chunk of one side of a task; the
//     partner is the other side (the same side for a self task); results are
//     the task's partial sums per slot, reduced later by unpack;
//   batched (MODE 1): an item is one tile of one cell, pulled from device work
//     queues (one queue in descending-cost order, or one per XCD over a
//     spatially contiguous share); the partners are all neighbour
//     cells of the cell, each translated into its frame; results are final.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sph_internal.hpp"

namespace sph {

// compile-time loop: fn(integral_constant<int, I>) for I in [I0, N)
template <int I, int N, class Fn>
__device__ __forceinline__ void unroll(Fn &&fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        unroll<I + 1, N>(fn);
    }
}

// compile-time loop threading a value: s = fn(integral_constant<int, I>, s)
template <int I, int N, class S, class Fn>
__device__ __forceinline__ S unroll_fold(S s, Fn &&fn)
{
    if constexpr (I < N) return unroll_fold<I + 1, N>(fn(std::integral_constant<int, I>{}, s), fn);
    else return s;
}

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
    const int32_t *items_x;     // MODE 1: tile order of the per-XCD shares
    const CellRange *cellr;
    const Nbr *nbr;
    const int32_t *nbr_off;
    const int32_t *jt_off;      // MODE 1: per cell j-tile list
    const JTile *jt;
    int32_t *queue;
    const float *q;             // MODE 1, gradient and force: derived planes
    int32_t use_queue;          // 0 static stride, 1 one queue, 2 per-XCD shares
    int32_t xoff[kQueues], xlen[kQueues];  // use_queue 2: shares of items

    float gam, beta, eps;
};

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

// cubic spline pieces in q = r / H, from t = 1 - q and s = 1/2 - q, each
// clamped at 0: w = 2 t^3 - 8 s^3 and w' = 24 s^2 - 6 t^2.  The inner piece
// (q < 1/2) is the outer one minus 8 s^3, a cubic that vanishes with its slope
// at q = 1/2, so one branch-free form covers the support and gives exactly 0
// beyond it.
__device__ __forceinline__ void spline_w_dw(float q, float &w, float &dw)
{
    const float t = fmaxf(1.0f - q, 0.0f), s = fmaxf(t - 0.5f, 0.0f);
    const float t2 = t * t, s2 = s * s;
    w = fmaf(2.0f * t2, t, -8.0f * s2 * s);
    dw = fmaf(24.0f, s2, -6.0f * t2);
}
// w'(q)/q from r, 1/r, 1/H and -6H: 18 q - 12 = 6 - 18 t for t > 1/2, else
// -6 t^2 H / r, with t = 1 - r/H clamped at 0 (the spline is C1 at t = 1/2,
// so either side may take the boundary; beyond the support the factor is 0)
__device__ __forceinline__ float spline_f(float r, float invr, float ih, float m6H)
{
    const float t = fmaxf(fmaf(-r, ih, 1.0f), 0.0f);
    return t > 0.5f ? fmaf(-18.0f, t, 6.0f) : m6H * t * t * invr;
}

// ---------------------------------------------------------------------------
// per-loop data: i registers, LDS candidate window, pair terms
// ---------------------------------------------------------------------------
// LDS candidate window of one wave.  ph holds, per candidate, the position
// relative to the i-tile centre and -|x|^2 (the phase-1 test reads only ph,
// plus 1/H for the force loop's mixed-support test); the other planes feed the
// pair term.  Every plane of the gradient and force windows has a 16-byte
// stride, so one address serves all reads of a candidate.  The gradient
// window carries the candidate's pack slot in a spare component.  The force
// window packs its 16 floats into four planes -- 64 bytes per candidate, so a
// 128-candidate window and its masks take 10 KB and sixteen waves fit a CU --
// and recomputes -|x|^2 (from x y z), nkB (= -3 kD) and H^2 (from 1/H) where
// they are needed; its counting variant adds a slot array.
template <int LOOP, int WIN, bool CNT>
struct Lds;

template <int WIN, bool CNT>
struct Lds<0, WIN, CNT> {
    float4 ph[WIN];  // x y z m
    uint32_t mask[WIN / 32][64];
};
template <int WIN, bool CNT>
struct Lds<1, WIN, CNT> {
    float4 ph[WIN];  // x y z -|x|^2
    float4 c1[WIN];  // vx vy vz m
    float4 c2[WIN];  // u m/rho c slot(bits)
    uint32_t mask[WIN / 32][64];
};
template <int WIN>
struct LdsForce {
    float4 ph[WIN];  // x y z vx
    float4 c1[WIN];  // vy vz m 1/H
    float4 c2[WIN];  // kA kD A2 c
    float4 c3[WIN];  // atq adh rh u
    uint32_t mask[WIN / 32][64];
};
template <int WIN>
struct Lds<2, WIN, false> : LdsForce<WIN> {
};
template <int WIN>
struct Lds<2, WIN, true> : LdsForce<WIN> {
    int32_t jslot[WIN];
};

struct IData {
    float x, y, z, H, H2, invH;    // position relative to the i-tile centre
    float vx, vy, vz, u, c;
    float kA, nkB, kD, A2, atq, adh, rh;  // force: see derive_force; gradient: kA = -6H
    float nx2, ny2, nz2;            // -2 x, -2 y, -2 z (phase-1 test)
    float t0;                       // |x|^2 - delta - H^2 (density, gradient) or |x|^2 - delta (force)
    float ri, xi2;                  // |x| and |x|^2
    float rj;                       // bound on |x_j| of staged candidates (tile centre frame)
    float hmin;                     // smallest support of the i-tile (uniform)
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

// the spline constants of derive_force from K and h: {kA, nkB, kD, H}
__device__ __forceinline__ float4 spline_consts(float K, float h)
{
    const float H = kGammaK * h;
    return make_float4(-3.0f * K * H, -9.0f * K, 3.0f * K, H);
}

// half the spline factor of one side (constants of derive_force): t = 1 - r/H
// clamped at 0, so beyond the support the factor is exactly zero
__device__ __forceinline__ float half_factor(float r, float invr, float ih, float kA, float nkB, float kD)
{
    const float t = fmaxf(fmaf(-r, ih, 1.0f), 0.0f);
    return t > 0.5f ? fmaf(nkB, t, kD) : kA * t * t * invr;
}

// derived planes of the batched form: float4 planes at q and q + 4P (force);
// one float4 plane (gradient)
template <int LOOP, bool PREP>
__device__ __forceinline__ void load_i(const InteractArgs &a, int64_t slot, bool valid, IData &d)
{
    d.slot = (int32_t)slot;
    if (!valid) {
        d.x = d.y = d.z = 0.f;
        d.H = 0.f;
        d.H2 = -1.f;
        d.invH = 0.f;
        d.vx = d.vy = d.vz = d.u = d.c = 0.f;
        d.kA = d.nkB = d.kD = d.A2 = d.atq = d.adh = d.rh = 0.f;
        return;
    }
    const float4 p0 = ((const float4 *)a.pack)[slot];
    d.x = p0.x;
    d.y = p0.y;
    d.z = p0.z;
    const float g = a.gam;
    if constexpr (LOOP == 2) {
        ForceDerived f;
        if constexpr (PREP) {
            f.q0 = ((const float4 *)a.q)[slot];
            f.q1 = ((const float4 *)(a.q + 4 * a.P))[slot];
        } else {
            const float4 p2 = ((const float4 *)(a.pack + a.P * 32))[slot];
            const float4 p3 = ((const float4 *)(a.pack + a.P * 48))[slot];
            const float ad = ((const float *)(a.pack + a.P * 64))[slot];
            f = derive_force(p0, p2, p3, ad, g, a.eps);
        }
        const float4 k = spline_consts(f.q0.y, p0.w);
        d.H = k.w;
        d.H2 = d.H * d.H;
        d.invH = f.q0.x;
        d.kA = k.x;
        d.nkB = k.y;
        d.kD = k.z;
        d.A2 = f.q0.z;
        d.c = f.q0.w;
        d.atq = f.q1.x;
        d.adh = f.q1.y;
        d.rh = f.q1.z;
        d.u = f.q1.w;
    } else {
        d.H = kGammaK * p0.w;
        d.H2 = d.H * d.H;
        d.invH = 1.0f / d.H;
        d.kA = -6.0f * d.H;
    }
    if constexpr (LOOP >= 1) {
        const float4 p1 = ((const float4 *)(a.pack + a.P * 16))[slot];
        d.vx = p1.x;
        d.vy = p1.y;
        d.vz = p1.z;
        if constexpr (LOOP == 1) {
            float4 q;
            if constexpr (PREP) q = ((const float4 *)a.q)[slot];
            else q = derive_gradient(p1, ((const float2 *)(a.pack + a.P * 32))[slot], g);
            d.u = q.x;
            d.c = q.z;
        }
    }
}

// the record of one j particle, held in registers between its load and its
// staging: packed fields, plus the derived planes in the batched form
template <int LOOP, bool PREP>
struct JRec;
template <bool PREP>
struct JRec<0, PREP> {
    float4 p0;
    float m;
};
template <>
struct JRec<1, false> {
    float4 p0, p1;
    float2 p2;
};
template <>
struct JRec<1, true> {
    float4 p0, p1, q0;
};
template <>
struct JRec<2, false> {
    float4 p0, p1, p2, p3;
    float ad;
};
template <>
struct JRec<2, true> {
    float4 p0, p1, q0, q1;
};

// loads of one j record; js is always a slot inside the buffer (the caller
// clamps lanes beyond the tile to its first slot)
template <int LOOP, bool PREP>
__device__ __forceinline__ void load_j(const InteractArgs &a, int64_t js, JRec<LOOP, PREP> &r)
{
    r.p0 = ((const float4 *)a.pack)[js];
    if constexpr (LOOP == 0) {
        r.m = ((const float *)(a.pack + a.P * 16))[js];
    } else {
        r.p1 = ((const float4 *)(a.pack + a.P * 16))[js];
        if constexpr (LOOP == 1 && PREP) {
            r.q0 = ((const float4 *)a.q)[js];
        } else if constexpr (LOOP == 1) {
            r.p2 = ((const float2 *)(a.pack + a.P * 32))[js];
        } else if constexpr (PREP) {
            r.q0 = ((const float4 *)a.q)[js];
            r.q1 = ((const float4 *)(a.q + 4 * a.P))[js];
        } else {
            r.p2 = ((const float4 *)(a.pack + a.P * 32))[js];
            r.p3 = ((const float4 *)(a.pack + a.P * 48))[js];
            r.ad = ((const float *)(a.pack + a.P * 64))[js];
        }
    }
}

// stage candidate j (record r, pack slot js, translated by (tx,ty,tz) and
// shifted to the i-tile centre (cx,cy,cz)) at LDS index k
template <int LOOP, bool PREP, int WIN, bool CNT>
__device__ __forceinline__ void stage_j(const InteractArgs &a, Lds<LOOP, WIN, CNT> &L, int k, int64_t js,
                                        const JRec<LOOP, PREP> &r, float tx, float ty, float tz, float cx,
                                        float cy, float cz)
{
    const float x = (r.p0.x + tx) - cx, y = (r.p0.y + ty) - cy, z = (r.p0.z + tz) - cz;
    if constexpr (LOOP == 0) {
        L.ph[k] = make_float4(x, y, z, r.m);
    } else if constexpr (LOOP == 1) {
        L.ph[k] = make_float4(x, y, z, -fmaf(z, z, fmaf(y, y, x * x)));
        L.c1[k] = make_float4(r.p1.x, r.p1.y, r.p1.z, r.p1.w);
        float4 q;
        if constexpr (PREP) q = r.q0;
        else q = derive_gradient(r.p1, r.p2, a.gam);
        L.c2[k] = make_float4(q.x, q.y, q.z, __int_as_float((int32_t)js));  // slot: j != i test
    } else {
        ForceDerived f;
        if constexpr (PREP) {
            f.q0 = r.q0;
            f.q1 = r.q1;
        } else {
            f = derive_force(r.p0, r.p2, r.p3, r.ad, a.gam, a.eps);
        }
        const float4 sc = spline_consts(f.q0.y, r.p0.w);
        L.ph[k] = make_float4(x, y, z, r.p1.x);
        L.c1[k] = make_float4(r.p1.y, r.p1.z, r.p1.w, f.q0.x);
        L.c2[k] = make_float4(sc.x, sc.z, f.q0.z, f.q0.w);
        L.c3[k] = f.q1;
        if constexpr (CNT) L.jslot[k] = (int32_t)js;
    }
}

// Phase-1 test of candidate k on the VALU, as a sign: the result is negative
// when |x_i - x_j|^2 < H^2 + delta_i, evaluated as |x_i|^2 - delta_i - H^2 +
// |x_j|^2 - 2 x_i.x_j with delta_i covering the rounding of these operations, so
// the hits are a superset of the exact test.  PERCAND (force loop, mixed
// supports): H^2 is max(H_i^2, H_j^2) with the candidate's own H_j^2; otherwise
// t0 already holds the support term.
template <int LOOP, int WIN, bool CNT, bool PERCAND>
__device__ __forceinline__ float test_sign(const Lds<LOOP, WIN, CNT> &L, int k, const IData &d)
{
    const float4 q = L.ph[k];
    // -|x_j|^2: stored by the density and gradient windows, rebuilt for force
    const float nq2 = LOOP == 2 ? -fmaf(q.z, q.z, fmaf(q.y, q.y, q.x * q.x)) : q.w;
    float t;
    if constexpr (PERCAND) {
        static_assert(LOOP == 2, "per-candidate supports are the force loop's");
        const float ih = L.c1[k].w;
        t = (d.t0 - fmaxf(d.H2, __builtin_amdgcn_rcpf(ih * ih))) - nq2;
    } else {
        t = d.t0 - nq2;
    }
    return fmaf(d.nx2, q.x, fmaf(d.ny2, q.y, fmaf(d.nz2, q.z, t)));
}

// phase 1 over the nw words of a window on the VALU: one 32-bit mask per word
// and lane, candidate kb + b at bit b
template <int LOOP, int WIN, bool CNT, bool PERCAND>
__device__ __forceinline__ void test_words(Lds<LOOP, WIN, CNT> &L, int nc, int nw, const IData &dd, bool valid)
{
    const int lane = threadIdx.x & 63;
    for (int w = 0; w < nw; ++w) {
        uint32_t m = 0;
        const int kb = 32 * w;
        const int kn = __builtin_amdgcn_readfirstlane(min(32, nc - kb));
        // shift each candidate's sign bit in from the top candidate down
        if (kn == 32) {
#pragma unroll 8
            for (int b = 31; b >= 0; --b)
                m = __builtin_amdgcn_alignbit(m, __float_as_uint(test_sign<LOOP, WIN, CNT, PERCAND>(L, kb + b, dd)), 31);
        } else {
            for (int b = kn - 1; b >= 0; --b)
                m = __builtin_amdgcn_alignbit(m, __float_as_uint(test_sign<LOOP, WIN, CNT, PERCAND>(L, kb + b, dd)), 31);
        }
        L.mask[w][lane] = valid ? m : 0u;
    }
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// sign bits of the 16 results of one 32x32 product, result r at bit r
__device__ __forceinline__ uint32_t sign_bits(const f32x16 &d)
{
    uint32_t m = 0;
#pragma unroll
    for (int r = 15; r >= 0; --r) m = __builtin_amdgcn_alignbit(m, __float_as_uint(d[r]), 31);
    return m;
}

// Phase 1 on the matrix cores.  The expanded test of every candidate j against
// every lane's particle i is one entry of a 32 x 64 product with K = 6:
//   (x_j, y_j, z_j, -|x_j|^2, 1, 0) . (-2 x_i, -2 y_i, -2 z_i, -1, t0_i, 0),
// three v_mfma_f32_32x32x2f32 per half of the wave's particles (A row i = a
// candidate, B column = a particle; lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32]; result r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4 of
// column l % 32).  Row i reads window slot b(i) = 16 ((i / 4) % 2) + 4 (i / 8)
// + i % 4, so that after one permlane32 swap of the two halves' sign masks every
// lane holds its own particle's bits with candidate kb + b at bit b, as the
// VALU test leaves them.  The products are accumulated in FP32 with no more
// roundings than the VALU form, which the margin delta covers.
// DUAL (force loop, mixed supports): a second product shares the first four
// columns and takes -H_j^2 of each candidate in its sixth column (against a 1
// in the particle's) with t1 = |x_i|^2 - delta in the fifth; a candidate is a
// hit when either product is negative, r^2 < H_i^2 or r^2 < H_j^2 (t0 then
// holds t1 - H_i^2).
template <int LOOP, int WIN, bool CNT, bool DUAL = false>
__device__ __forceinline__ void test_words_mfma(Lds<LOOP, WIN, CNT> &L, int nc, int nw, const IData &dd, bool valid,
                                                float t1 = 0.f)
{
    const int lane = threadIdx.x & 63;
    // B operands of the particle halves 0-31 ([0]) and 32-63 ([1])
    const auto bxy = __builtin_amdgcn_permlane32_swap(__float_as_uint(dd.nx2), __float_as_uint(dd.ny2), false, false);
    const auto bzw = __builtin_amdgcn_permlane32_swap(__float_as_uint(dd.nz2), __float_as_uint(-1.0f), false, false);
    const auto bt = __builtin_amdgcn_permlane32_swap(__float_as_uint(dd.t0), 0u, false, false);
    const auto bt1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(t1), __float_as_uint(1.0f), false, false);
    const float one = lane < 32 ? 1.0f : 0.0f;
    const int i = lane & 31;
    const int slot = 16 * ((i >> 2) & 1) + 4 * (i >> 3) + (i & 3);
    const int comp = lane >> 5;  // x (z) in the lower half, y (w) in the upper
    for (int w = 0; w < nw; ++w) {
        const int kb = 32 * w;
        float axy, azw;
        if constexpr (LOOP != 1) {
            const float4 v = L.ph[kb + slot];  // x y z vx / m: -|x|^2 rebuilt
            axy = comp ? v.y : v.x;
            azw = comp ? -fmaf(v.z, v.z, fmaf(v.y, v.y, v.x * v.x)) : v.z;
        } else {
            const float *q = (const float *)&L.ph[kb + slot];
            axy = q[comp];
            azw = q[2 + comp];
        }
        // sixth column of the second product: -H_j^2 of the row's candidate
        float hj = one;
        if constexpr (DUAL) {
            if (comp) {
                const float ih = L.c1[kb + slot].w;
                hj = -__builtin_amdgcn_rcpf(ih * ih);
            }
        }
        // one half at a time: 16 accumulator registers live, not 32 (the
        // second product is recomputed rather than kept beside the first)
        f32x16 d = __builtin_amdgcn_mfma_f32_32x32x2f32(axy, __uint_as_float(bxy[0]), f32x16{}, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x2f32(azw, __uint_as_float(bzw[0]), d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x2f32(one, __uint_as_float(bt[0]), d, 0, 0, 0);
        uint32_t m0 = sign_bits(d);
        if constexpr (DUAL) {
            __builtin_amdgcn_sched_barrier(0);
            d = __builtin_amdgcn_mfma_f32_32x32x2f32(axy, __uint_as_float(bxy[0]), f32x16{}, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_32x32x2f32(azw, __uint_as_float(bzw[0]), d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_32x32x2f32(hj, __uint_as_float(bt1[0]), d, 0, 0, 0);
            m0 |= sign_bits(d);
        }
        __builtin_amdgcn_sched_barrier(0);
        d = __builtin_amdgcn_mfma_f32_32x32x2f32(axy, __uint_as_float(bxy[1]), f32x16{}, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x2f32(azw, __uint_as_float(bzw[1]), d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_32x32x2f32(one, __uint_as_float(bt[1]), d, 0, 0, 0);
        uint32_t m1 = sign_bits(d);
        if constexpr (DUAL) {
            __builtin_amdgcn_sched_barrier(0);
            d = __builtin_amdgcn_mfma_f32_32x32x2f32(axy, __uint_as_float(bxy[1]), f32x16{}, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_32x32x2f32(azw, __uint_as_float(bzw[1]), d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_32x32x2f32(hj, __uint_as_float(bt1[1]), d, 0, 0, 0);
            m1 |= sign_bits(d);
        }
        const auto h = __builtin_amdgcn_permlane32_swap(m0, m1, false, false);
        uint32_t m = h[0] | (h[1] << 16);
        const int kn = __builtin_amdgcn_readfirstlane(min(32, nc - kb));
        if (kn < 32) m &= (1u << kn) - 1u;  // slots beyond the window's count
        L.mask[w][lane] = valid ? m : 0u;
    }
}

// One staged candidate as phase 2 holds it in registers: its position in the
// i-tile frame and what the pair term reads of it.
template <int LOOP>
struct Cand;
template <>
struct Cand<0> {
    float x, y, z, m;
};
template <>
struct Cand<1> {
    float x, y, z;
    int32_t js;
    float4 c1, c2;  // v m | u m/rho c -
};
template <>
struct Cand<2> {
    float x, y, z, vx;
    int32_t js;
    float4 c1, c2, c3;  // vy vz m 1/H | kA kD A2 c | atq adh rh u
};

template <int LOOP, int WIN, bool CNT>
__device__ __forceinline__ Cand<LOOP> cand_load(const Lds<LOOP, WIN, CNT> &L, int k)
{
    Cand<LOOP> c;
    // byte offsets by shifts (the planes' strides are 16 and 4 bytes)
    const uint32_t o4 = (uint32_t)k << 2;
    const float4 p = *(const float4 *)((const char *)L.ph + (o4 << 2));
    c.x = p.x;
    c.y = p.y;
    c.z = p.z;
    if constexpr (LOOP == 0) {
        c.m = p.w;
    } else {
        c.c1 = L.c1[k];
        c.c2 = L.c2[k];
        if constexpr (LOOP == 1) {
            c.js = __float_as_int(c.c2.w);
        } else {
            c.vx = p.w;
            c.c3 = L.c3[k];
            if constexpr (CNT) c.js = L.jslot[k];
        }
    }
    return c;
}

// the pair term of lane's particle i with candidate c.  The counting variant
// (CNT) applies the exact support test and the j != i test before anything
// else and counts the pair.  Without counts most of these tests are not
// needed: beyond a support the clamped spline gives w = w' = 0 exactly, so such
// a candidate adds zeros, and for j = i (r = 0) every gradient and force term
// carries a factor r, v_ij or u_i - u_j that is zero; only the gradient loop's
// signal-velocity maximum still needs both tests.
template <int LOOP, bool CNT>
__device__ __forceinline__ void pair(const InteractArgs &a, const Cand<LOOP> &c, const IData &d, Acc &acc)
{
    const float rx = d.x - c.x, ry = d.y - c.y, rz = d.z - c.z;
    const float r2 = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
    if constexpr (LOOP == 0) {
        if constexpr (CNT) {
            if (!(r2 < d.H2)) return;  // the exact criterion
        }
        const float mj = c.m;
        const float r = fast_sqrt(r2);
        const float q = r * d.invH;
        float w, dw;
        spline_w_dw(q, w, dw);
        acc.s0 = fmaf(mj, w, acc.s0);                      // sum m w
        acc.s1 = fmaf(mj, fmaf(q, dw, 3.0f * w), acc.s1);  // sum m (3w + q w')
        acc.s2 += w;                                       // sum w
        if constexpr (CNT) acc.n++;
    } else {
        if constexpr (CNT) {
            if (c.js == d.slot) return;  // j != i
            if constexpr (LOOP == 1) {
                if (!(r2 < d.H2)) return;
            } else {
                if (!(r2 < fmaxf(d.H2, __builtin_amdgcn_rcpf(c.c1.w * c.c1.w)))) return;
            }
        }
        const float4 c1 = c.c1;
        float vx, vy, vz;
        if constexpr (LOOP == 1) {
            vx = d.vx - c1.x;
            vy = d.vy - c1.y;
            vz = d.vz - c1.z;
        } else {
            vx = d.vx - c.vx;
            vy = d.vy - c1.x;
            vz = d.vz - c1.y;
        }
        // r = 0 (j = i, or coincident particles) gives a finite 1/r and r = 0;
        // the added 2^-126 is below half an ulp of any r^2 above 2^-100
        const float invr = fast_rsq(r2 + 0x1p-126f);
        const float r = r2 * invr;
        const float dot = fmaf(vz, rz, fmaf(vy, ry, vx * rx));
        const float mu = fminf(dot * invr, 0.0f);
        if constexpr (LOOP == 1) {
            const float4 c2 = c.c2;  // u m/rho c slot
            const float f = spline_f(r, invr, d.invH, d.kA);    // w'/q
            const float mf = c1.w * f;
            acc.s0 = fmaf(mf, dot, acc.s0);                                   // D
            acc.s1 = fmaf(mf, fmaf(vy, rz, -vz * ry), acc.s1);                // R
            acc.s2 = fmaf(mf, fmaf(vz, rx, -vx * rz), acc.s2);
            acc.s3 = fmaf(mf, fmaf(vx, ry, -vy * rx), acc.s3);
            acc.s4 = fmaf(c2.y * (d.u - c2.x), f, acc.s4);                    // L / 2
            const float vs = d.c + c2.z - a.beta * mu;
            if constexpr (CNT) {
                if (vs > acc.s5) acc.s5 = vs;                                 // V
                acc.n++;
            } else {
                if (c.js != d.slot && r2 < d.H2 && vs > acc.s5) acc.s5 = vs;
            }
        } else {
            const float mj = c1.z, ihj = c1.w;
            const float4 c2 = c.c2;  // kA kD A2 c
            const float4 c3 = c.c3;  // atq adh rh u
            // fi, fj: halves of w'(q)/q K of i and j, so fb is their average
            float fi, fj;
            if constexpr (CNT) {
                fi = r2 < d.H2 ? half_factor(r, invr, d.invH, d.kA, d.nkB, d.kD) : 0.0f;
                fj = r2 < __builtin_amdgcn_rcpf(ihj * ihj) ? half_factor(r, invr, ihj, c2.x, -3.0f * c2.y, c2.y)
                                                           : 0.0f;
            } else {
                fi = half_factor(r, invr, d.invH, d.kA, d.nkB, d.kD);
                fj = half_factor(r, invr, ihj, c2.x, -3.0f * c2.y, c2.y);
            }
            const float fb = fi + fj;
            const float vsig = d.c + c2.w - a.beta * mu;
            const float g = fast_rcp(d.rh + c3.z) * fb;                // fb / rho_ij
            const float pf = (d.atq + c3.x) * vsig * mu * g;           // Pi_ij fb
            const float ai = d.A2 * fi, aj = c2.z * fj;                // A_i w_i, A_j w_j
            const float ms = mj * ((ai + aj) + pf);
            acc.s0 = fmaf(-ms, rx, acc.s0);
            acc.s1 = fmaf(-ms, ry, acc.s1);
            acc.s2 = fmaf(-ms, rz, acc.s2);
            const float cond = (d.adh + c3.y) * fabsf(dot) * (d.u - c3.w) * g;
            acc.s3 = fmaf(mj, fmaf(dot, fmaf(0.5f, pf, ai), cond), acc.s3);
            if constexpr (CNT) acc.n++;
        }
    }
}

template <int LOOP, bool CNT>
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
    if constexpr (CNT) a.counts[s] = acc.n;
}

// hits of the same mask word a lane takes per trip of the walk: the trip's
// bookkeeping (word advance, lowest set bit, exit test) is shared by two pair
// terms (density 2.86 -> 2.68 ms, gradient 3.76 -> 3.56, force 4.13 -> 4.01 at
// 256^3; three or four per trip measure the same)
template <int LOOP>
constexpr int kHitsPerTrip = 2;

// test every staged candidate against every lane (phase 1: one bit per lane
// and candidate, in LDS), then let each lane walk its own hits (phase 2)
template <int LOOP, int WIN, bool CNT, bool DUAL>
__device__ __forceinline__ void flush(const InteractArgs &a, Lds<LOOP, WIN, CNT> &L, int nc, float hw, const IData &d,
                                      bool valid, Acc &acc)
{
    const int lane = threadIdx.x & 63;
    wave_sync();
    nc = __builtin_amdgcn_readfirstlane(nc);
    const int nw = (nc + 31) >> 5;
    IData dd = d;
    if constexpr (LOOP == 2) {
        // the force loop's support is max(H_i, H_j): when no lane's support is
        // much below the window's largest Hw, max(H_i, Hw) costs nothing in
        // extra hits and saves a per-candidate maximum; otherwise (mixed
        // scales) the test takes each candidate's own H_j, on the VALU or
        // (DUAL) as a second matrix-core product -- the kernel variant for
        // plans whose cells differ in width, where such windows are common
        // (its extra registers would make the other variant spill)
        dd.t0 = dd.xi2 - test_delta(dd.ri, dd.rj);
        if (hw <= 1.02f * dd.hmin) {
            dd.t0 -= fmaxf(dd.H2, hw * hw);
            test_words_mfma<LOOP, WIN, CNT>(L, nc, nw, dd, valid);
        } else if constexpr (DUAL) {
            const float t1 = dd.t0;
            dd.t0 -= dd.H2;
            test_words_mfma<LOOP, WIN, CNT, true>(L, nc, nw, dd, valid, t1);
        } else {
            test_words<LOOP, WIN, CNT, true>(L, nc, nw, dd, valid);
        }
    } else {
        test_words_mfma<LOOP, WIN, CNT>(L, nc, nw, dd, valid);
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
            const int b = __builtin_ctz(cur);  // lowest slot first
            cur &= cur - 1u;
            pair<LOOP, CNT>(a, cand_load<LOOP, WIN, CNT>(L, 32 * w + b), d, acc);
            // the lane's next hits of the same word, in slot order (a lane's
            // sum keeps the order of its hits)
            unroll<1, kHitsPerTrip<LOOP>>([&](auto) {
                if (cur != 0) {
                    const int b2 = __builtin_ctz(cur);
                    cur &= cur - 1u;
                    pair<LOOP, CNT>(a, cand_load<LOOP, WIN, CNT>(L, 32 * w + b2), d, acc);
                }
            });
        }
    }
    wave_sync();
}

// one j-tile as seen by one lane during the cull: slots, translation, box
struct TileInfo {
    int64_t js0;
    int32_t jn;
    float tx, ty, tz;
    float hm;  // largest support in the tile
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
    o.hm = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t.hm), l));
    return o;
}

// does lane's particle of tile t reach the i-tile box (lo, hi)?
template <int LOOP, class R>
__device__ __forceinline__ bool tile_keep(const TileInfo &t, const R &r, const float4 &lo,
                                          const float4 &hi)
{
    const int lane = threadIdx.x & 63;
    if (lane >= t.jn) return false;
    const float x = r.p0.x + t.tx, y = r.p0.y + t.ty, z = r.p0.z + t.tz;
    const float ex = fmaxf(fmaxf(lo.x - x, x - hi.x), 0.f);
    const float ey = fmaxf(fmaxf(lo.y - y, y - hi.y), 0.f);
    const float ez = fmaxf(fmaxf(lo.z - z, z - hi.z), 0.f);
    const float reach = LOOP == 2 ? fmaxf(lo.w, kGammaK * r.p0.w) : lo.w;
    return fmaf(ez, ez, fmaf(ey, ey, ex * ex)) < reach * reach * 1.0001f;
}

// stage the kept particles of a batch of B loaded tiles, in tile order,
// flushing the window whenever the next tile's survivors do not fit (one
// flush call site, so the batch stays in registers)
template <int LOOP, bool PREP, int WIN, int B, bool CNT, bool DUAL>
__device__ __forceinline__ void stage_batch(const InteractArgs &a, Lds<LOOP, WIN, CNT> &L, int &nc, float &hw,
                                            const TileInfo (&tb)[B], const JRec<LOOP, PREP> (&rb)[B], const IData &d,
                                            bool valid, const float4 &lo, const float4 &hi, const float4 &cen,
                                            Acc &acc)
{
    const int lane = threadIdx.x & 63;
    bool keep[B];
    uint64_t bal[B];
    unroll<0, B>([&](auto I) {
        constexpr int b = decltype(I)::value;
        keep[b] = tile_keep<LOOP>(tb[b], rb[b], lo, hi);
        bal[b] = __ballot(keep[b]);
    });
    // staging state threaded through the unrolled tiles: first tile not yet
    // staged, whether it did not fit, and the window count
    struct St {
        int b0, stop, nc;
        float hw;  // largest support of the staged tiles (force)
    };
    St st{0, 0, nc, hw};
    for (;;) {
        st.stop = 0;
        st = unroll_fold<0, B>(st, [&](auto I, St s) {
            constexpr int b = decltype(I)::value;
            if (b >= s.b0 && !s.stop) {
                const int cnt = __popcll(bal[b]);
                if (s.nc + cnt > WIN) {
                    s.stop = 1;
                } else {
                    if (keep[b]) {
                        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[b] >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)bal[b], 0u));
                        stage_j<LOOP, PREP, WIN, CNT>(a, L, s.nc + rank, tb[b].js0 + lane, rb[b], tb[b].tx, tb[b].ty,
                                                 tb[b].tz, cen.x, cen.y, cen.z);
                    }
                    s.nc = __builtin_amdgcn_readfirstlane(s.nc + cnt);
                    if (cnt > 0) s.hw = fmaxf(s.hw, tb[b].hm);
                    s.b0 = b + 1;
                }
            }
            return s;
        });
        if (!__builtin_amdgcn_readfirstlane(st.stop)) break;
        flush<LOOP, WIN, CNT, DUAL>(a, L, st.nc, st.hw, d, valid, acc);
        st.nc = 0;
        st.hw = 0.f;
    }
    nc = st.nc;
    hw = st.hw;
}

// j tiles whose records are loaded together before any of them is staged:
// one memory round trip per batch instead of per tile
template <int LOOP>
constexpr int kJBatch = LOOP == 0 ? 4 : 2;

// gather the candidates of one item's j-tile list (nj tiles) into the window
template <int LOOP, int MODE, int WIN, bool CNT, bool DUAL>
__device__ __forceinline__ void scan_item(const InteractArgs &a, Lds<LOOP, WIN, CNT> &L, int &nc, float &hw,
                                          const Chunk &ch,
                                          IData &d, bool valid, const float4 &lo, const float4 &hi,
                                          const float4 &cen, float halfdiag, Acc &acc)
{
    constexpr int B = kJBatch<LOOP>;
    constexpr bool PREP = MODE == 1 && LOOP >= 1;
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
        TileInfo ti{0, 0, 0.f, 0.f, 0.f, 0.f};
        bool ok = false;
        float hj = 0.f;
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
                blo = a.bounds[2 * (int64_t)e.tile];
                bhi = a.bounds[2 * (int64_t)e.tile + 1];
                ti.js0 = e.slot0;
                ti.jn = e.n;
                ti.tx = e.tx;
                ti.ty = e.ty;
                ti.tz = e.tz;
            }
            const float gx = fmaxf(fmaxf(blo.x + ti.tx - hi.x, lo.x - (bhi.x + ti.tx)), 0.f);
            const float gy = fmaxf(fmaxf(blo.y + ti.ty - hi.y, lo.y - (bhi.y + ti.ty)), 0.f);
            const float gz = fmaxf(fmaxf(blo.z + ti.tz - hi.z, lo.z - (bhi.z + ti.tz)), 0.f);
            const float reach = LOOP == 2 ? fmaxf(hmi, blo.w) : hmi;
            ok = fmaf(gz, gz, fmaf(gy, gy, gx * gx)) < reach * reach * 1.0001f;
            hj = blo.w;
            ti.hm = blo.w;
        }
        uint64_t m = __ballot(ok);
        if (m == 0) continue;
        if constexpr (LOOP == 2) {
            // candidates of these tiles reach at most max(i-tile support, their tile's support)
            hjm = fmaxf(hjm, wave_max_u(ok ? hj : 0.f));
            d.rj = halfdiag + 1.001f * fmaxf(hmi, hjm);
        }
        // 2. stage the surviving tiles, B tiles' records in flight at a time
        while (m != 0) {
            TileInfo tb[B];
            JRec<LOOP, PREP> rb[B];
            unroll<0, B>([&](auto I) {
                constexpr int b = decltype(I)::value;
                if (m != 0) {
                    const int idx = __builtin_ctzll(m);
                    m &= m - 1;
                    tb[b] = bcast(ti, idx);
                } else {
                    tb[b] = TileInfo{0, 0, 0.f, 0.f, 0.f, 0.f};  // slot 0 is inside every buffer
                }
                load_j<LOOP, PREP>(a, tb[b].js0 + (lane < tb[b].jn ? lane : 0), rb[b]);
            });
            stage_batch<LOOP, PREP, WIN, B, CNT, DUAL>(a, L, nc, hw, tb, rb, d, valid, lo, hi, cen, acc);
        }
    }
}

// resident waves per SIMD the register allocation must allow
template <int LOOP>
constexpr int kMinWaves = LOOP == 0 ? 5 : 4;

// One wave per workgroup: the waves share nothing, and one-wave workgroups
// let the CU pack as many LDS windows as fit (a wave's window is its only
// LDS), instead of rounding down to whole four-window groups.
template <int LOOP, int MODE, int WIN, bool CNT, bool DUAL>
__device__ __forceinline__ void interact_waves(const InteractArgs &a)
{
    __shared__ Lds<LOOP, WIN, CNT> L;
    const int lane = threadIdx.x & 63;
    const int64_t wave_id = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
    const int64_t nwaves = (int64_t)gridDim.x;
    const int qmode = MODE == 1 ? a.use_queue : 0;
    // the next item is claimed while the current one runs (lane 0's atomic
    // result stays in a register until the loop head needs it)
    const int xhome = (int)(blockIdx.x % kQueues);
    int xr = xhome;  // share being drained (qmode 2)
    int qv = 0;
    if (qmode == 1 && lane == 0) qv = atomicAdd(a.queue, 1);
    if (qmode == 2 && lane == 0) qv = atomicAdd(a.queue + kQueueStride * xr, 1);
    int64_t iter = 0;
    for (;;) {
        int64_t item;
        if (MODE == 0) {
            item = iter == 0 ? wave_id : a.nitems;
        } else if (qmode == 1) {
            item = __builtin_amdgcn_readfirstlane(qv);
        } else if (qmode == 2) {
            const int v = __builtin_amdgcn_readfirstlane(qv);
            if (v >= a.xlen[xr]) {
                // this share is drained: move on to the next one, until all are
                xr = xr + 1 == kQueues ? 0 : xr + 1;
                if (xr == xhome) break;
                if (lane == 0) qv = atomicAdd(a.queue + kQueueStride * xr, 1);
                continue;
            }
            item = a.xoff[xr] + v;
        } else {
            item = wave_id + iter * nwaves;
        }
        ++iter;
        if (item >= a.nitems) break;
        if (qmode == 1 && lane == 0) qv = atomicAdd(a.queue, 1);
        if (qmode == 2 && lane == 0) qv = atomicAdd(a.queue + kQueueStride * xr, 1);
        Chunk ch;
        int64_t islot, bi;
        if (MODE == 0) {
            ch = a.items_chunks[a.chunk_base + item];
            islot = ch.slot0 - a.slot_base + lane;
            bi = item;
        } else {
            bi = qmode == 2 ? a.items_x[item] : a.items[item];
            ch = a.items_chunks[bi];
            islot = ch.slot0 + lane;
        }
        // the i-tile's box and largest support, as the pack kernel recorded them
        const float4 lo = a.bounds[2 * bi];
        const float4 hi = a.bounds[2 * bi + 1];
        const bool valid = lane < ch.n;
        IData d;
        load_i<LOOP, MODE == 1 && LOOP >= 1>(a, islot, valid, d);
        // i positions relative to the tile centre; phase-1 constants
        float4 cen;
        cen.x = 0.5f * (lo.x + hi.x);
        cen.y = 0.5f * (lo.y + hi.y);
        cen.z = 0.5f * (lo.z + hi.z);
        cen.w = 0.f;
        const float ex = hi.x - lo.x, ey = hi.y - lo.y, ez = hi.z - lo.z;
        const float halfdiag = 0.5f * sqrtf(fmaxf(ex * ex + ey * ey + ez * ez, 0.f));
        d.x -= cen.x;
        d.y -= cen.y;
        d.z -= cen.z;
        d.ri = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
        d.xi2 = fmaf(d.z, d.z, fmaf(d.y, d.y, d.x * d.x));
        d.rj = halfdiag + 1.001f * lo.w;
        if constexpr (LOOP == 2) d.hmin = wave_min_u(valid ? d.H : __builtin_huge_valf());
        d.nx2 = -2.0f * d.x;
        d.ny2 = -2.0f * d.y;
        d.nz2 = -2.0f * d.z;
        d.t0 = (d.xi2 - test_delta(d.ri, d.rj)) - d.H2;
        Acc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0};
        int nc = 0;
        float hw = 0.f;
        scan_item<LOOP, MODE, WIN, CNT, DUAL>(a, L, nc, hw, ch, d, valid, lo, hi, cen, halfdiag, acc);
        if (nc > 0) flush<LOOP, WIN, CNT, DUAL>(a, L, nc, hw, d, valid, acc);
        if (valid) write_out<LOOP, CNT>(a, d, acc);
    }
}

template <int LOOP, int MODE, int WIN, bool CNT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kMinWaves<LOOP>))) void k_interact(
    InteractArgs a)
{
    interact_waves<LOOP, MODE, WIN, CNT, false>(a);
}

// the force loop for plans whose cells differ in width: mixed supports tested
// as two matrix-core products; three waves per SIMD leave it the registers of
// the second product without spills (as fast as four waves with spills)
template <int MODE, int WIN, bool CNT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_interact_mixed(
    InteractArgs a)
{
    interact_waves<2, MODE, WIN, CNT, true>(a);
}

__global__ void k_reset_queue(int32_t *q)
{
    if (threadIdx.x < kQueues) q[kQueueStride * threadIdx.x] = 0;
}

struct PrepArgs {
    const char *pack;
    int64_t P, n;
    float *q;
    float gam, eps;
};

// the derived planes of the batched form, one thread per particle
template <int LOOP>
__global__ __launch_bounds__(256) void k_prep(PrepArgs a)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= a.n) return;
    const float4 p1 = ((const float4 *)(a.pack + a.P * 16))[s];
    if constexpr (LOOP == 1) {
        ((float4 *)a.q)[s] = derive_gradient(p1, ((const float2 *)(a.pack + a.P * 32))[s], a.gam);
    } else {
        const float4 p0 = ((const float4 *)a.pack)[s];
        const float4 p2 = ((const float4 *)(a.pack + a.P * 32))[s];
        const float4 p3 = ((const float4 *)(a.pack + a.P * 48))[s];
        const float ad = ((const float *)(a.pack + a.P * 64))[s];
        const ForceDerived f = derive_force(p0, p2, p3, ad, a.gam, a.eps);
        ((float4 *)a.q)[s] = f.q0;
        ((float4 *)(a.q + 4 * a.P))[s] = f.q1;
    }
}

// the counting variant runs only when the caller asks for pair counts
template <int LOOP, int MODE, int WIN>
static void launch_one(const InteractArgs &a, unsigned grid, hipStream_t st, bool mixed)
{
    if constexpr (LOOP == 2) {
        if (mixed) {
            if (a.counts) hipLaunchKernelGGL((k_interact_mixed<MODE, WIN, true>), dim3(grid), dim3(64), 0, st, a);
            else hipLaunchKernelGGL((k_interact_mixed<MODE, WIN, false>), dim3(grid), dim3(64), 0, st, a);
            return;
        }
    }
    if (a.counts) hipLaunchKernelGGL((k_interact<LOOP, MODE, WIN, true>), dim3(grid), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_interact<LOOP, MODE, WIN, false>), dim3(grid), dim3(64), 0, st, a);
}

template <int LOOP, int MODE>
static sph_status launch_win(const InteractArgs &a, int win, unsigned grid, hipStream_t st, bool mixed)
{
    switch (win) {
    case 128: launch_one<LOOP, MODE, 128>(a, grid, st, mixed); break;
    case 256: launch_one<LOOP, MODE, 256>(a, grid, st, mixed); break;
    case 512:
        if constexpr (LOOP == 2) return fail(SPH_E_ARG, "force window is at most 256");
        else launch_one<LOOP, MODE, 512>(a, grid, st, false);
        break;
    default: return fail(SPH_E_ARG, "bad window");
    }
    SPH_CHECK_LAUNCH("interaction launch");
    return SPH_OK;
}

sph_status launch_interact(const sph_plan *p, int loop, bool cells, int32_t t0, int32_t t1, const void *pack,
                           const sph_params *prm, const sph_tuning *tn, void *res, int32_t *counts, void *ws,
                           hipStream_t st, const int32_t *items, int64_t nitems, bool prepped)
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
        grid = (unsigned)a.nitems;
        win = 128;
        if (p->max_cell > 64 && loop < 2) win = 256;
    } else {
        a.P = round_slots(p->n);
        a.items_chunks = p->d_tiles;
        a.items = p->d_items;
        a.items_x = p->d_items_x;
        for (int q = 0; q < kQueues; ++q) {
            a.xoff[q] = p->xoff[q];
            a.xlen[q] = p->xlen[q];
        }
        a.nitems = p->ntile;
        a.cellr = p->d_cellr;
        a.nbr = p->d_nbr;
        a.nbr_off = p->d_nbr_off;
        a.jt_off = p->d_jt_off;
        a.jt = p->d_jt;
        a.bounds = (const float4 *)(a.pack + a.P * 4 * kPackFloats[loop]);
        a.queue = (int32_t *)ws;
        a.use_queue = tn->queue;
        if (items) {
            // a subset of the tiles in plan order: eight contiguous shares of
            // equal length, one per XCD queue, as for the full list
            a.items = items;
            a.items_x = items;
            a.nitems = nitems;
            for (int q = 0; q < kQueues; ++q) {
                a.xoff[q] = (int32_t)(nitems * q / kQueues);
                a.xlen[q] = (int32_t)(nitems * (q + 1) / kQueues) - a.xoff[q];
            }
            a.use_queue = 2;
        }
        if (a.nitems == 0) return SPH_OK;
        // blocks_per_cu counts groups of four waves; a loop may set its own
        const int bpc = tn->blocks_per_loop[loop] > 0 ? tn->blocks_per_loop[loop] : tn->blocks_per_cu;
        grid = (unsigned)std::min<int64_t>((int64_t)bpc * 4 * p->num_cu, a.nitems);
        win = tn->window[loop];
        if (a.use_queue) {
            hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, a.queue);
            SPH_CHECK_LAUNCH("queue reset launch");
        }
        if (loop >= 1 && prepped) {
            a.q = (float *)((char *)ws + kQueueBytes);  // written by the step's pack
        } else if (loop >= 1) {
            PrepArgs pa{a.pack, a.P, p->n, (float *)((char *)ws + kQueueBytes), a.gam, a.eps};
            a.q = pa.q;
            const unsigned pg = (unsigned)((p->n + 255) / 256);
            if (loop == 1) hipLaunchKernelGGL(k_prep<1>, dim3(pg), dim3(256), 0, st, pa);
            else hipLaunchKernelGGL(k_prep<2>, dim3(pg), dim3(256), 0, st, pa);
            SPH_CHECK_LAUNCH("derived-plane launch");
        }
    }
    if (loop == 0) return cells ? launch_win<0, 1>(a, win, grid, st, false) : launch_win<0, 0>(a, win, grid, st, false);
    if (loop == 1) return cells ? launch_win<1, 1>(a, win, grid, st, false) : launch_win<1, 0>(a, win, grid, st, false);
    return cells ? launch_win<2, 1>(a, win, grid, st, p->mixed_widths) : launch_win<2, 0>(a, win, grid, st, p->mixed_widths);
}

}  // namespace sph
