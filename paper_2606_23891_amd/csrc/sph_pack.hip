// Pack and unpack kernels (paper Sec. 2.3, Table 1).
//
// One wave64 handles one chunk of up to 64 consecutive particles of one cell
// (one side of a task, or a tile of the batched form).  Lanes walk
// consecutive particles, so every field load of a substruct is a coalesced
// strided access whose stride is the substruct's record size: an AoS record
// drags its whole cache lines, a split substruct only the fields the loop
// needs -- the paper's point, now at HBM instead of host memory.
// Layout, loop and field offsets are template parameters, so each load folds
// to base + p * stride + constant.
//
// Pack: positions become float32 offsets from the task origin, computed in
// float64 and rounded once; every other field is copied bit for bit.  The
// wave also emits its chunk's bounding box and largest support radius, used
// by the interaction kernels to skip far tiles.
// Unpack: per-task results are added (float32, fixed slot order) into the
// store; the signal velocity keeps the larger value.
//
// Also here, as the other kernels that read or write the store directly: the
// loop-fission passes of pack and unpack (Sec. 3.3), the whole-store layout
// conversion, the smoothing-length Newton step with its tile compaction, and
// the kick, drift and time-step kernels of the time integration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "sph_internal.hpp"

namespace sph {

template <int I, int N, class Fn>
__device__ __forceinline__ void static_for(Fn &&fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1, N>(fn);
    }
}

template <int L, int F, int C>
__device__ __forceinline__ char *field_ptr(const StoreArg &s, int64_t p)
{
    constexpr int sb = kLayouts[L].sub[F][C];
    constexpr int off = kLayouts[L].off[F][C];
    constexpr int stride = kLayouts[L].sub_bytes[sb];
    char *base = (char *)__builtin_assume_aligned(s.sub[sb], 256);
    return base + p * stride + off;
}

template <int L, int F, int C, typename T>
__device__ __forceinline__ T ld(const StoreArg &s, int64_t p)
{
    return *reinterpret_cast<const T *>(field_ptr<L, F, C>(s, p));
}

template <int L, int F, int C, typename T>
__device__ __forceinline__ void st(const StoreArg &s, int64_t p, T v)
{
    *reinterpret_cast<T *>(field_ptr<L, F, C>(s, p)) = v;
    if constexpr (F == FX) {
        // replicated positions: every copy holds the same bits
        static_for<0, kLayouts[L].nxrep>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            constexpr int sb = kLayouts[L].xrep_sub[r];
            char *base = (char *)__builtin_assume_aligned(s.sub[sb], 256);
            *reinterpret_cast<T *>(base + p * kLayouts[L].sub_bytes[sb] + kLayouts[L].xrep_off[r] + 8 * C) = v;
        });
    }
}

struct PackArgs {
    StoreArg store;
    const Chunk *chunks;
    const sph_cell *cells;
    const sph_task *tasks;
    int64_t chunk_base;
    int64_t nchunk;
    int64_t slot_base;
    int64_t P;      // slots per plane
    char *buf;
    float4 *bounds; // 2 per chunk
    // staged step (batched form): earlier loops' outputs and the derived planes
    const float *step_res;  // kStepPlanes planes of P floats
    float *derived;         // gradient: 1 float4 plane; force: 2 float4 planes
    float gam, eps;
};

// fields each loop's pack reads (paper Table 1)
constexpr bool kPackReads[3][NFIELD] = {
    // X  V  A  M  H  U  UDT RHO RDH WC DIV ROT LAP VSIG AV AD TB ID COLD
    {1, 0, 0, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {1, 1, 0, 1, 1, 1, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {1, 1, 0, 1, 1, 1, 0, 1, 1, 0, 1, 1, 0, 0, 1, 1, 0, 0, 0}};

// byte span [lo, hi) of substruct S's record that loop LOOP's pack reads
// (lo > hi when it reads nothing there), and the widest load that the record
// stride and the span's start allow (records are 256-byte aligned arrays)
constexpr int span_lo(int L, int LOOP, int S)
{
    int lo = 1 << 30;
    for (int f = 0; f < NFIELD; ++f)
        if (kPackReads[LOOP][f])
            for (int c = 0; c < kNComp[f]; ++c)
                if (kLayouts[L].sub[f][c] == S && kLayouts[L].off[f][c] < lo) lo = kLayouts[L].off[f][c];
    return lo;
}
constexpr int span_hi(int L, int LOOP, int S)
{
    int hi = -1;
    for (int f = 0; f < NFIELD; ++f)
        if (kPackReads[LOOP][f])
            for (int c = 0; c < kNComp[f]; ++c)
                if (kLayouts[L].sub[f][c] == S && kLayouts[L].off[f][c] + kCompBytes[f] > hi)
                    hi = kLayouts[L].off[f][c] + kCompBytes[f];
    return hi;
}
constexpr int load_width(int record, int lo)
{
    return (record % 16 == 0 && lo % 16 == 0) ? 16 : (record % 8 == 0 && lo % 8 == 0) ? 8 : 4;
}

// ---------------------------------------------------------------------------
// outputs of a staged step (see the write-back below)
// ---------------------------------------------------------------------------
// the output of each step result plane, and the loop producing it
constexpr int kStepOutF[kStepPlanes] = {FRHO, FRHODH, FWCOUNT, FDIV, FROT, FROT, FROT, FLAP, FVSIG, FA, FA, FA, FUDT};
constexpr int kStepOutC[kStepPlanes] = {0, 0, 0, 0, 0, 1, 2, 0, 0, 0, 1, 2, 0};
constexpr int kStepOutLoop[kStepPlanes] = {0, 0, 0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2};
constexpr int kStepVsig = 8;

// the value an output holds once unpacked from a per-particle result: +0 + r,
// the signal velocity the larger of +0 and r (the batched unpack's reduction)
__device__ __forceinline__ float settle(float r, bool vmax)
{
    return vmax ? ((r > 0.0f) ? r : 0.0f) : 0.0f + r;
}

// does loop LOOP's pack load the whole record of substruct S (its span, widened
// to the load width, covers the record)?
constexpr bool full_load(int L, int LOOP, int S)
{
    const int lo = span_lo(L, LOOP, S), hi = span_hi(L, LOOP, S);
    if (lo != 0 || hi <= 0) return false;
    const int R = kLayouts[L].sub_bytes[S];
    const int G = load_width(R, 0);
    return (hi + G - 1) / G * G == R;
}
// who stores step output q into the store: the first later pack that loads
// its substruct whole (it writes the record back with the outputs it holds),
// else the write-back at the end of the step (3)
constexpr int step_writer(int L, int q)
{
    const int S = kLayouts[L].sub[kStepOutF[q]][kStepOutC[q]];
    for (int lp = kStepOutLoop[q] + 1; lp <= 2; ++lp)
        if (full_load(L, lp, S)) return lp;
    return 3;
}
constexpr bool pack_writes_sub(int L, int LOOP, int S)
{
    for (int q = 0; q < kStepPlanes; ++q)
        if (step_writer(L, q) == LOOP && kLayouts[L].sub[kStepOutF[q]][kStepOutC[q]] == S) return true;
    return false;
}

// the values a pack reads, by field
struct PackVals {
    double x[3];
    float m, h, v[3], u, rho, rdh, div, rot[3], av, ad;
    template <int F, int C>
    __device__ __forceinline__ void set(const uint32_t *w)
    {
        if constexpr (F == FX) {
            const uint64_t b = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
            x[C] = __longlong_as_double((long long)b);
        } else {
            const float f = __uint_as_float(w[0]);
            if constexpr (F == FMASS) m = f;
            else if constexpr (F == FH) h = f;
            else if constexpr (F == FV) v[C] = f;
            else if constexpr (F == FU) u = f;
            else if constexpr (F == FRHO) rho = f;
            else if constexpr (F == FRHODH) rdh = f;
            else if constexpr (F == FDIV) div = f;
            else if constexpr (F == FROT) rot[C] = f;
            else if constexpr (F == FAV) av = f;
            else if constexpr (F == FAD) ad = f;
        }
    }
};

// Read the span of substruct S with the widest aligned loads, then take every
// field the loop reads out of the loaded words: one pass over each record
// instead of one narrow load per field (the bytes are the same, the requests
// a fraction)
// STEP (staged step): a substruct this pack loads whole and that holds
// outputs of earlier loops of the step gets those outputs, settled from the
// step's result planes (P floats each), written into the loaded record, which
// is stored back whole; the fields are then taken from the patched record.
template <int L, int LOOP, int S, bool STEP = false>
__device__ __forceinline__ void load_sub(const StoreArg &st, int64_t p, PackVals &v, const float *res = nullptr,
                                         int64_t P = 0)
{
    constexpr int lo = span_lo(L, LOOP, S), hi = span_hi(L, LOOP, S);
    if constexpr (lo < hi) {
        constexpr int R = kLayouts[L].sub_bytes[S];
        constexpr int G = load_width(R, lo);
        constexpr int NB = (hi - lo + G - 1) / G * G;  // lo + NB <= R: R and lo are multiples of G
        uint32_t w[NB / 4];
        const char *base = (const char *)__builtin_assume_aligned(st.sub[S], 256) + p * R + lo;
        static_for<0, NB / G>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if constexpr (G == 16) {
                const uint4 q = *(const uint4 *)(base + 16 * k);
                w[4 * k] = q.x;
                w[4 * k + 1] = q.y;
                w[4 * k + 2] = q.z;
                w[4 * k + 3] = q.w;
            } else if constexpr (G == 8) {
                const uint2 q = *(const uint2 *)(base + 8 * k);
                w[2 * k] = q.x;
                w[2 * k + 1] = q.y;
            } else {
                w[k] = *(const uint32_t *)(base + 4 * k);
            }
        });
        if constexpr (STEP && pack_writes_sub(L, LOOP, S)) {
            static_for<0, kStepPlanes>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int F = kStepOutF[q], C = kStepOutC[q];
                if constexpr (kStepOutLoop[q] < LOOP && kLayouts[L].sub[F][C] == S)
                    w[kLayouts[L].off[F][C] / 4] = __float_as_uint(settle(res[q * P + p], q == kStepVsig));
            });
            char *wb = (char *)__builtin_assume_aligned(st.sub[S], 256) + p * R;
            static_for<0, NB / G>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                if constexpr (G == 16)
                    *(uint4 *)(wb + 16 * k) = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
                else if constexpr (G == 8)
                    *(uint2 *)(wb + 8 * k) = make_uint2(w[2 * k], w[2 * k + 1]);
                else
                    *(uint32_t *)(wb + 4 * k) = w[k];
            });
        }
        static_for<0, NFIELD>([&](auto fc) {
            constexpr int F = decltype(fc)::value;
            if constexpr (kPackReads[LOOP][F]) {
                static_for<0, kNComp[F]>([&](auto cc) {
                    constexpr int C = decltype(cc)::value;
                    if constexpr (kLayouts[L].sub[F][C] == S) v.template set<F, C>(w + (kLayouts[L].off[F][C] - lo) / 4);
                });
            }
        });
    }
}

// STEP: the pack of a staged step (batched form only): the fields earlier
// loops of the step produce are taken, settled, from the step's result planes
// rather than from the store (which receives them at the step's end), and the
// derived planes of the gradient / force pair terms are written beside the
// packed record
template <int L, int LOOP, bool STEP = false>
__global__ __launch_bounds__(512) void k_pack(PackArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = __builtin_amdgcn_readfirstlane((int)((int64_t)blockIdx.x * (blockDim.x >> 6) +
                                                           (threadIdx.x >> 6)));
    if (c >= a.nchunk) return;
    const Chunk ch = a.chunks[a.chunk_base + c];
    const sph_cell &oc = a.cells[ch.cell];
    double o0 = oc.loc[0], o1 = oc.loc[1], o2 = oc.loc[2];
    if (ch.side) {
        const sph_task &t = a.tasks[ch.task];
        o0 = o0 - t.shift[0];
        o1 = o1 - t.shift[1];
        o2 = o2 - t.shift[2];
    }
    const bool valid = lane < ch.n;
    const int64_t p = ch.part0 + lane;
    const int64_t slot = ch.slot0 - a.slot_base + lane;
    const int64_t P = a.P;
    float dx = 0.f, dy = 0.f, dz = 0.f, hh = 0.f;
    if (valid) {
        PackVals v;
        static_for<0, kLayouts[L].nsub>([&](auto sc) {
            load_sub<L, LOOP, decltype(sc)::value, STEP>(a.store, p, v, a.step_res, P);
        });
        if constexpr (STEP && LOOP >= 1) {
            const float *r = a.step_res;
            v.rho = settle(r[p], false);
            if constexpr (LOOP == 2) {
                v.rdh = settle(r[P + p], false);
                v.div = settle(r[3 * P + p], false);
                v.rot[0] = settle(r[4 * P + p], false);
                v.rot[1] = settle(r[5 * P + p], false);
                v.rot[2] = settle(r[6 * P + p], false);
            }
        }
        dx = (float)(v.x[0] - o0);
        dy = (float)(v.x[1] - o1);
        dz = (float)(v.x[2] - o2);
        hh = v.h;
        float4 *pl0 = (float4 *)a.buf;
        pl0[slot] = make_float4(dx, dy, dz, hh);
        if constexpr (LOOP == 0) {
            float *pl1 = (float *)(a.buf + P * 16);
            pl1[slot] = v.m;
        } else {
            float4 *pl1 = (float4 *)(a.buf + P * 16);
            pl1[slot] = make_float4(v.v[0], v.v[1], v.v[2], v.m);
            if constexpr (LOOP == 1) {
                float2 *pl2 = (float2 *)(a.buf + P * 32);
                pl2[slot] = make_float2(v.u, v.rho);
            } else {
                float4 *pl2 = (float4 *)(a.buf + P * 32);
                pl2[slot] = make_float4(v.u, v.rho, v.rdh, v.div);
                float4 *pl3 = (float4 *)(a.buf + P * 48);
                pl3[slot] = make_float4(v.rot[0], v.rot[1], v.rot[2], v.av);
                float *pl4 = (float *)(a.buf + P * 64);
                pl4[slot] = v.ad;
            }
        }
        if constexpr (STEP && LOOP == 1) {
            ((float4 *)a.derived)[slot] = derive_gradient(make_float4(v.v[0], v.v[1], v.v[2], v.m),
                                                          make_float2(v.u, v.rho), a.gam);
        } else if constexpr (STEP && LOOP == 2) {
            const ForceDerived f = derive_force(make_float4(dx, dy, dz, hh), make_float4(v.u, v.rho, v.rdh, v.div),
                                                make_float4(v.rot[0], v.rot[1], v.rot[2], v.av), v.ad, a.gam,
                                                a.eps);
            ((float4 *)a.derived)[slot] = f.q0;
            ((float4 *)(a.derived + 4 * P))[slot] = f.q1;
        }
    }
    // chunk bounds by DPP reductions (VALU, no LDS round trips)
    const float inf = __builtin_huge_valf();
    const float lx = wave_min_u(valid ? dx : inf), ly = wave_min_u(valid ? dy : inf), lz = wave_min_u(valid ? dz : inf);
    const float hx = wave_max_u(valid ? dx : -inf), hy = wave_max_u(valid ? dy : -inf), hz = wave_max_u(valid ? dz : -inf);
    const float hm = wave_max_u(valid ? kGammaK * hh : 0.f);
    if (lane == 0) {
        a.bounds[2 * c] = make_float4(lx, ly, lz, hm);
        a.bounds[2 * c + 1] = make_float4(hx, hy, hz, 0.f);
    }
}

// ---------------------------------------------------------------------------
// loop fission (Sec. 3.3): a pack split into passes, each its own launch over
// the same chunks, converting only the members of its mask
// ---------------------------------------------------------------------------
// members of the force record in plane order; density and gradient pack the
// subsets kItemsOf[loop]
constexpr int kNItem = 17;
constexpr int kItemF[kNItem] = {FX, FX, FX, FH, FV, FV, FV, FMASS, FU, FRHO, FRHODH, FDIV, FROT, FROT, FROT, FAV, FAD};
constexpr int kItemC[kNItem] = {0, 1, 2, 0, 0, 1, 2, 0, 0, 0, 0, 0, 0, 1, 2, 0, 0};
constexpr uint32_t kItemsOf[3] = {0x8Fu, 0x3FFu, 0x1FFFFu};
// the member stored in word w of plane q of a loop's record (-1: none)
constexpr int kPlaneItem[3][5][4] = {{{0, 1, 2, 3}, {7, -1, -1, -1}},
                                     {{0, 1, 2, 3}, {4, 5, 6, 7}, {8, 9, -1, -1}},
                                     {{0, 1, 2, 3}, {4, 5, 6, 7}, {8, 9, 10, 11}, {12, 13, 14, 15}, {16, -1, -1, -1}}};

constexpr uint32_t plane_mask(int loop, int q)
{
    uint32_t m = 0;
    for (int w = 0; w < 4; ++w)
        if (kPlaneItem[loop][q][w] >= 0) m |= 1u << kPlaneItem[loop][q][w];
    return m;
}

// One pass of a fissioned pack: as k_pack, restricted to the members in
// `mask` (uniform, so every test below is a scalar branch).  A plane whose
// members all belong to the pass is stored whole, otherwise member by member;
// the pass holding a position component writes that component's chunk bounds,
// the pass holding h the largest support radius.
template <int L, int LOOP>
__global__ __launch_bounds__(512) void k_pack_pass(PackArgs a, uint32_t mask)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = __builtin_amdgcn_readfirstlane((int)((int64_t)blockIdx.x * (blockDim.x >> 6) +
                                                           (threadIdx.x >> 6)));
    if (c >= a.nchunk) return;
    const Chunk ch = a.chunks[a.chunk_base + c];
    const sph_cell &oc = a.cells[ch.cell];
    double o[3] = {oc.loc[0], oc.loc[1], oc.loc[2]};
    if (ch.side) {
        const sph_task &t = a.tasks[ch.task];
        o[0] = o[0] - t.shift[0];
        o[1] = o[1] - t.shift[1];
        o[2] = o[2] - t.shift[2];
    }
    const bool valid = lane < ch.n;
    const int64_t p = ch.part0 + lane;
    const int64_t slot = ch.slot0 - a.slot_base + lane;
    float val[kNItem] = {};
    if (valid) {
        static_for<0, kNItem>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr int F = kItemF[k], C = kItemC[k];
            if constexpr ((kItemsOf[LOOP] >> k) & 1u) {
                if ((mask >> k) & 1u) {
                    if constexpr (F == FX) val[k] = (float)(ld<L, FX, C, double>(a.store, p) - o[C]);
                    else val[k] = ld<L, F, C, float>(a.store, p);
                }
            }
        });
        int64_t plane_off = 0;
        static_for<0, kPackPlanes[LOOP]>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int nf = kPlaneFloats[LOOP][q];
            constexpr uint32_t pm = plane_mask(LOOP, q);
            float *pl = (float *)(a.buf + plane_off) + slot * nf;
            if ((mask & pm) == pm) {
                if constexpr (nf == 4)
                    *(float4 *)pl = make_float4(val[kPlaneItem[LOOP][q][0]], val[kPlaneItem[LOOP][q][1]],
                                                val[kPlaneItem[LOOP][q][2]], val[kPlaneItem[LOOP][q][3]]);
                else if constexpr (nf == 2)
                    *(float2 *)pl = make_float2(val[kPlaneItem[LOOP][q][0]], val[kPlaneItem[LOOP][q][1]]);
                else
                    *pl = val[kPlaneItem[LOOP][q][0]];
            } else if (mask & pm) {
                static_for<0, nf>([&](auto wc) {
                    constexpr int w = decltype(wc)::value;
                    if ((mask >> kPlaneItem[LOOP][q][w]) & 1u) pl[w] = val[kPlaneItem[LOOP][q][w]];
                });
            }
            plane_off += a.P * 4 * nf;
        });
    }
    float *lo = (float *)&a.bounds[2 * c], *hi = (float *)&a.bounds[2 * c + 1];
    const float inf = __builtin_huge_valf();
    static_for<0, 3>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if ((mask >> k) & 1u) {
            const float l = wave_min_u(valid ? val[k] : inf), h = wave_max_u(valid ? val[k] : -inf);
            if (lane == 0) {
                lo[k] = l;
                hi[k] = h;
            }
        }
    });
    if ((mask >> 3) & 1u) {
        const float hm = wave_max_u(valid ? kGammaK * val[3] : 0.f);
        if (lane == 0) {
            lo[3] = hm;
            hi[3] = 0.f;
        }
    }
}

// loop outputs: (field, component) per result plane
constexpr int kOutF[3][6] = {{FRHO, FRHODH, FWCOUNT}, {FDIV, FROT, FROT, FROT, FLAP, FVSIG}, {FA, FA, FA, FUDT}};
constexpr int kOutC[3][6] = {{0, 0, 0}, {0, 0, 1, 2, 0, 0}, {0, 1, 2, 0}};

// the reduction of one result into one output value
template <int LOOP, int K>
__device__ __forceinline__ float reduce_one(float cur, float r)
{
    if constexpr (LOOP == 1 && K == 5) return (r > cur) ? r : cur;  // signal velocity: maximum
    else return cur + r;
}

struct UnpackArgs {
    StoreArg store;
    const Chunk *chunks;
    int64_t chunk_base;
    int64_t nchunk;
    int64_t slot_base;
    int64_t P;
    const float *res;
    const int64_t *csr_off;
    const int64_t *csr;
    int64_t slot_lo, slot_hi;  // absolute slots of the range (CSR path)
    int64_t n;
    uint32_t mask;             // result planes of a fissioned pass (MASKED kernels)
};

// One chunk per wave.  CELLS: per-particle results, out = +0 (+) r; else one
// task's partials added into the current value (slots of one task touch
// distinct particles, so lanes never collide).  MASKED: one pass of a
// fissioned unpack, writing only the result planes in a.mask.
template <int L, int LOOP, bool CELLS, bool MASKED>
__global__ __launch_bounds__(512) void k_unpack_chunks(UnpackArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = __builtin_amdgcn_readfirstlane((int)((int64_t)blockIdx.x * (blockDim.x >> 6) +
                                                           (threadIdx.x >> 6)));
    if (c >= a.nchunk) return;
    const Chunk ch = a.chunks[a.chunk_base + c];
    if (lane >= ch.n) return;
    const int64_t p = ch.part0 + lane;
    const int64_t slot = ch.slot0 - a.slot_base + lane;
    // every load before the first store: loads and stores retire through one
    // in-order counter, so a load behind a store would wait for it (one
    // memory round trip per output instead of one in all)
    float r[kResPlanes[LOOP]], cur[kResPlanes[LOOP]];
    static_for<0, kResPlanes[LOOP]>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int F = kOutF[LOOP][k], C = kOutC[LOOP][k];
        r[k] = 0.0f;
        cur[k] = 0.0f;
        if constexpr (MASKED)
            if (!((a.mask >> k) & 1u)) return;
        r[k] = a.res[k * a.P + slot];
        if constexpr (!CELLS) cur[k] = ld<L, F, C, float>(a.store, p);
    });
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, kResPlanes[LOOP]>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int F = kOutF[LOOP][k], C = kOutC[LOOP][k];
        if constexpr (MASKED)
            if (!((a.mask >> k) & 1u)) return;
        st<L, F, C, float>(a.store, p, reduce_one<LOOP, k>(cur[k], r[k]));
    });
}

// Several tasks: one thread per particle walks its slots in ascending order.
template <int L, int LOOP>
__global__ __launch_bounds__(256) void k_unpack_csr(UnpackArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    int64_t b = a.csr_off[p];
    const int64_t e = a.csr_off[p + 1];
    while (b < e && a.csr[b] < a.slot_lo) ++b;
    if (b == e || a.csr[b] >= a.slot_hi) return;
    // every output's current value and every partial read before the first
    // store (a load behind a store waits for it); each output still takes its
    // partials in ascending slot order
    float cur[kResPlanes[LOOP]];
    static_for<0, kResPlanes[LOOP]>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        cur[k] = ld<L, kOutF[LOOP][k], kOutC[LOOP][k], float>(a.store, p);
    });
    for (int64_t q = b; q < e && a.csr[q] < a.slot_hi; ++q) {
        const int64_t s = a.csr[q] - a.slot_lo;
        static_for<0, kResPlanes[LOOP]>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            cur[k] = reduce_one<LOOP, k>(cur[k], a.res[k * a.P + s]);
        });
    }
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, kResPlanes[LOOP]>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        st<L, kOutF[LOOP][k], kOutC[LOOP][k], float>(a.store, p, cur[k]);
    });
}

// ---------------------------------------------------------------------------
// staged step: one write-back of every output at the end of the step
// ---------------------------------------------------------------------------
// does byte b of substruct S of layout L hold an output the write-back
// stores (one that no pack of the step has written already)?
constexpr bool out_byte(int L, int S, int b)
{
    for (int q = 0; q < kStepPlanes; ++q) {
        const int f = kStepOutF[q], c = kStepOutC[q];
        if (step_writer(L, q) == 3 && kLayouts[L].sub[f][c] == S && b >= kLayouts[L].off[f][c] &&
            b < kLayouts[L].off[f][c] + 4)
            return true;
    }
    return false;
}
constexpr int out_bytes_in(int L, int S, int lo, int len)
{
    int k = 0;
    for (int b = lo; b < lo + len; ++b) k += out_byte(L, S, b) ? 1 : 0;
    return k;
}

// One wave per tile, one lane per particle.  Each substruct that holds an
// output is written in whole records when the record is at most 64 bytes
// (so consecutive lanes cover whole 32-byte sectors), otherwise in the
// aligned chunks that hold outputs; a chunk that also holds other members or
// padding is read first and merged, so those bytes keep their bits.
template <int L>
__global__ __launch_bounds__(512) void k_writeback(UnpackArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = __builtin_amdgcn_readfirstlane((int)((int64_t)blockIdx.x * (blockDim.x >> 6) +
                                                           (threadIdx.x >> 6)));
    if (c >= a.nchunk) return;
    const Chunk ch = a.chunks[c];
    if (lane >= ch.n) return;
    const int64_t p = ch.part0 + lane;
    static_for<0, kLayouts[L].nsub>([&](auto sc) {
        constexpr int S = decltype(sc)::value;
        constexpr int R = kLayouts[L].sub_bytes[S];
        if constexpr (out_bytes_in(L, S, 0, R) > 0) {
            constexpr int G = load_width(R, 0);
            constexpr bool whole = R <= 64;
            char *base = (char *)__builtin_assume_aligned(a.store.sub[S], 256) + p * R;
            uint32_t w[R / 4];
            static_for<0, R / G>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                constexpr int no = out_bytes_in(L, S, k * G, G);
                if constexpr ((whole || no > 0) && no < G) {
                    if constexpr (G == 16) {
                        const uint4 q = *(const uint4 *)(base + 16 * k);
                        w[4 * k] = q.x;
                        w[4 * k + 1] = q.y;
                        w[4 * k + 2] = q.z;
                        w[4 * k + 3] = q.w;
                    } else if constexpr (G == 8) {
                        const uint2 q = *(const uint2 *)(base + 8 * k);
                        w[2 * k] = q.x;
                        w[2 * k + 1] = q.y;
                    } else {
                        w[k] = *(const uint32_t *)(base + 4 * k);
                    }
                }
            });
            static_for<0, kStepPlanes>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int F = kStepOutF[q], C = kStepOutC[q];
                if constexpr (step_writer(L, q) == 3 && kLayouts[L].sub[F][C] == S)
                    w[kLayouts[L].off[F][C] / 4] = __float_as_uint(settle(a.res[q * a.P + p], q == kStepVsig));
            });
            static_for<0, R / G>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                if constexpr (whole || out_bytes_in(L, S, k * G, G) > 0) {
                    if constexpr (G == 16)
                        *(uint4 *)(base + 16 * k) = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
                    else if constexpr (G == 8)
                        *(uint2 *)(base + 8 * k) = make_uint2(w[2 * k], w[2 * k + 1]);
                    else
                        *(uint32_t *)(base + 4 * k) = w[k];
                }
            });
        }
    });
}

template <int L>
static sph_status writeback_l(const UnpackArgs &a, int waves, hipStream_t st)
{
    const unsigned grid = (unsigned)((a.nchunk + waves - 1) / waves);
    hipLaunchKernelGGL((k_writeback<L>), dim3(grid), dim3(64 * waves), 0, st, a);
    SPH_CHECK_LAUNCH("write-back launch");
    return SPH_OK;
}

template <int L>
static sph_status pack_step_l(int loop, const PackArgs &a, int waves, hipStream_t st)
{
    const unsigned grid = (unsigned)((a.nchunk + waves - 1) / waves);
    const dim3 blk(64 * waves);
    if (loop == 0) hipLaunchKernelGGL((k_pack<L, 0, true>), dim3(grid), blk, 0, st, a);
    else if (loop == 1) hipLaunchKernelGGL((k_pack<L, 1, true>), dim3(grid), blk, 0, st, a);
    else hipLaunchKernelGGL((k_pack<L, 2, true>), dim3(grid), blk, 0, st, a);
    SPH_CHECK_LAUNCH("step pack launch");
    return SPH_OK;
}

// the fission groups of a layout's pack (unpack) members under a schedule
template <int L>
static int passes_l(int loop, int schedule, bool unpack, uint32_t *masks)
{
    const int nmem = unpack ? kResPlanes[loop] : kNItem;
    int key[kNItem];
    int ng = 0;
    for (int k = 0; k < nmem; ++k) {
        if (!unpack && !((kItemsOf[loop] >> k) & 1u)) continue;
        const int F = unpack ? kOutF[loop][k] : kItemF[k];
        const int C = unpack ? kOutC[loop][k] : kItemC[k];
        const int sub = kLayouts[L].sub[F][C], bytes = kCompBytes[F];
        const int kk = schedule == 1 ? sub : schedule == 2 ? F : schedule == 3 ? bytes : schedule == 4 ? sub * 16 + bytes : 0;
        int g = 0;
        while (g < ng && key[g] != kk) ++g;
        if (g == ng) {
            key[ng] = kk;
            masks[ng++] = 0;
        }
        masks[g] |= 1u << k;
    }
    return ng;
}

int fission_passes(int layout, int loop, int schedule, bool unpack, uint32_t *masks)
{
    switch (layout) {
    case 0: return passes_l<0>(loop, schedule, unpack, masks);
    case 1: return passes_l<1>(loop, schedule, unpack, masks);
    case 2: return passes_l<2>(loop, schedule, unpack, masks);
    case 3: return passes_l<3>(loop, schedule, unpack, masks);
    case 4: return passes_l<4>(loop, schedule, unpack, masks);
    case 5: return passes_l<5>(loop, schedule, unpack, masks);
    case 6: return passes_l<6>(loop, schedule, unpack, masks);
    case 7: return passes_l<7>(loop, schedule, unpack, masks);
    case 8: return passes_l<8>(loop, schedule, unpack, masks);
    case 9: return passes_l<9>(loop, schedule, unpack, masks);
    default: return 0;
    }
}

template <int L>
static sph_status pack_l(const sph_plan *p, int loop, const PackArgs &a, int waves, int schedule, hipStream_t st)
{
    const unsigned grid = (unsigned)((a.nchunk + waves - 1) / waves);
    const dim3 blk(64 * waves);
    if (schedule == 0) {
        if (loop == 0) hipLaunchKernelGGL((k_pack<L, 0>), dim3(grid), blk, 0, st, a);
        else if (loop == 1) hipLaunchKernelGGL((k_pack<L, 1>), dim3(grid), blk, 0, st, a);
        else hipLaunchKernelGGL((k_pack<L, 2>), dim3(grid), blk, 0, st, a);
    } else {
        uint32_t masks[kNItem];
        const int np = passes_l<L>(loop, schedule, false, masks);
        for (int q = 0; q < np; ++q) {
            if (loop == 0) hipLaunchKernelGGL((k_pack_pass<L, 0>), dim3(grid), blk, 0, st, a, masks[q]);
            else if (loop == 1) hipLaunchKernelGGL((k_pack_pass<L, 1>), dim3(grid), blk, 0, st, a, masks[q]);
            else hipLaunchKernelGGL((k_pack_pass<L, 2>), dim3(grid), blk, 0, st, a, masks[q]);
        }
    }
    (void)p;
    SPH_CHECK_LAUNCH("pack launch");
    return SPH_OK;
}

template <int L, int LOOP>
static void unpack_ll(const UnpackArgs &a, bool cells, bool csr, int waves, int schedule, hipStream_t st)
{
    if (csr) {
        hipLaunchKernelGGL((k_unpack_csr<L, LOOP>), dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
        return;
    }
    const unsigned grid = (unsigned)((a.nchunk + waves - 1) / waves);
    if (!cells) {
        hipLaunchKernelGGL((k_unpack_chunks<L, LOOP, false, false>), dim3(grid), dim3(64 * waves), 0, st, a);
    } else if (schedule == 0) {
        hipLaunchKernelGGL((k_unpack_chunks<L, LOOP, true, false>), dim3(grid), dim3(64 * waves), 0, st, a);
    } else {
        uint32_t masks[kNItem];
        const int np = passes_l<L>(LOOP, schedule, true, masks);
        UnpackArgs b = a;
        for (int q = 0; q < np; ++q) {
            b.mask = masks[q];
            hipLaunchKernelGGL((k_unpack_chunks<L, LOOP, true, true>), dim3(grid), dim3(64 * waves), 0, st, b);
        }
    }
}

template <int L>
static sph_status unpack_l(int loop, const UnpackArgs &a, bool cells, bool csr, int waves, int schedule,
                           hipStream_t st)
{
    if (loop == 0) unpack_ll<L, 0>(a, cells, csr, waves, schedule, st);
    else if (loop == 1) unpack_ll<L, 1>(a, cells, csr, waves, schedule, st);
    else unpack_ll<L, 2>(a, cells, csr, waves, schedule, st);
    SPH_CHECK_LAUNCH("unpack launch");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// layout conversion: every member of every particle from one layout's store
// into another's (a store that changes its decomposition between phases)
// ---------------------------------------------------------------------------
// a particle's members as 32-bit words: 8-byte components take two, the
// 1-byte time bin one (low byte)
constexpr int comp_words(int f) { return kCompBytes[f] == 8 ? 2 : 1; }
constexpr int word_of(int f, int c)
{
    int w = 0;
    for (int g = 0; g < f; ++g) w += kNComp[g] * comp_words(g);
    return w + c * comp_words(f);
}
constexpr int kParticleWords = word_of(NFIELD - 1, 0) + kNComp[NFIELD - 1] * comp_words(NFIELD - 1);
static_assert(kParticleWords == 40, "member words");

// Read substruct S of layout L whole (records of 1 byte: one byte load) and
// take out its members.
template <int L, int S>
__device__ __forceinline__ void read_record(const StoreArg &st, int64_t p, uint32_t *v)
{
    constexpr int R = kLayouts[L].sub_bytes[S];
    const char *base = (const char *)__builtin_assume_aligned(st.sub[S], 256) + p * R;
    if constexpr (R == 1) {
        // the only 1-byte record is a lone 1-byte member
        static_for<0, NFIELD>([&](auto fc) {
            constexpr int F = decltype(fc)::value;
            static_for<0, kNComp[F]>([&](auto cc) {
                constexpr int C = decltype(cc)::value;
                if constexpr (has_member(kLayouts[L], F, C, S)) v[word_of(F, C)] = *(const uint8_t *)base;
            });
        });
    } else {
        constexpr int G = load_width(R, 0);
        uint32_t w[R / 4];
        static_for<0, R / G>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if constexpr (G == 16) {
                const uint4 q = *(const uint4 *)(base + 16 * k);
                w[4 * k] = q.x;
                w[4 * k + 1] = q.y;
                w[4 * k + 2] = q.z;
                w[4 * k + 3] = q.w;
            } else if constexpr (G == 8) {
                const uint2 q = *(const uint2 *)(base + 8 * k);
                w[2 * k] = q.x;
                w[2 * k + 1] = q.y;
            } else {
                w[k] = *(const uint32_t *)(base + 4 * k);
            }
        });
        static_for<0, NFIELD>([&](auto fc) {
            constexpr int F = decltype(fc)::value;
            static_for<0, kNComp[F]>([&](auto cc) {
                constexpr int C = decltype(cc)::value;
                if constexpr (has_member(kLayouts[L], F, C, S)) {
                    constexpr int off = member_off(kLayouts[L], F, C, S), k = word_of(F, C);
                    if constexpr (kCompBytes[F] == 8) {
                        v[k] = w[off / 4];
                        v[k + 1] = w[off / 4 + 1];
                    } else if constexpr (kCompBytes[F] == 4) {
                        v[k] = w[off / 4];
                    } else {
                        v[k] = (w[off / 4] >> (8 * (off % 4))) & 0xFFu;
                    }
                }
            });
        });
    }
}

// Assemble substruct S of layout L from the member words (padding bytes
// zero) and write the record whole.
template <int L, int S>
__device__ __forceinline__ void write_record(const StoreArg &st, int64_t p, const uint32_t *v)
{
    constexpr int R = kLayouts[L].sub_bytes[S];
    char *base = (char *)__builtin_assume_aligned(st.sub[S], 256) + p * R;
    if constexpr (R == 1) {
        static_for<0, NFIELD>([&](auto fc) {
            constexpr int F = decltype(fc)::value;
            static_for<0, kNComp[F]>([&](auto cc) {
                constexpr int C = decltype(cc)::value;
                if constexpr (has_member(kLayouts[L], F, C, S)) *(uint8_t *)base = (uint8_t)v[word_of(F, C)];
            });
        });
    } else {
        constexpr int G = load_width(R, 0);
        uint32_t w[R / 4];
        static_for<0, R / 4>([&](auto kc) { w[decltype(kc)::value] = 0u; });
        static_for<0, NFIELD>([&](auto fc) {
            constexpr int F = decltype(fc)::value;
            static_for<0, kNComp[F]>([&](auto cc) {
                constexpr int C = decltype(cc)::value;
                if constexpr (has_member(kLayouts[L], F, C, S)) {
                    constexpr int off = member_off(kLayouts[L], F, C, S), k = word_of(F, C);
                    if constexpr (kCompBytes[F] == 8) {
                        w[off / 4] = v[k];
                        w[off / 4 + 1] = v[k + 1];
                    } else if constexpr (kCompBytes[F] == 4) {
                        w[off / 4] = v[k];
                    } else {
                        w[off / 4] |= (v[k] & 0xFFu) << (8 * (off % 4));
                    }
                }
            });
        });
        static_for<0, R / G>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if constexpr (G == 16)
                *(uint4 *)(base + 16 * k) = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
            else if constexpr (G == 8)
                *(uint2 *)(base + 8 * k) = make_uint2(w[2 * k], w[2 * k + 1]);
            else
                *(uint32_t *)(base + 4 * k) = w[k];
        });
    }
}

// one thread per particle: every source record read once, every destination
// record written once
template <int LS, int LD>
__global__ __launch_bounds__(256) void k_convert(StoreArg src, StoreArg dst, int64_t n)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t v[kParticleWords];
    static_for<0, kLayouts[LS].nsub>([&](auto sc) { read_record<LS, decltype(sc)::value>(src, p, v); });
    static_for<0, kLayouts[LD].nsub>([&](auto sc) { write_record<LD, decltype(sc)::value>(dst, p, v); });
}

template <int LS, int LD>
static sph_status convert_ll(const StoreArg &src, const StoreArg &dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL((k_convert<LS, LD>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    SPH_CHECK_LAUNCH("convert launch");
    return SPH_OK;
}

template <int LS>
static sph_status convert_l(int ld, const StoreArg &src, const StoreArg &dst, int64_t n, hipStream_t st)
{
    switch (ld) {
    case 0: return convert_ll<LS, 0>(src, dst, n, st);
    case 1: return convert_ll<LS, 1>(src, dst, n, st);
    case 2: return convert_ll<LS, 2>(src, dst, n, st);
    case 3: return convert_ll<LS, 3>(src, dst, n, st);
    case 4: return convert_ll<LS, 4>(src, dst, n, st);
    case 5: return convert_ll<LS, 5>(src, dst, n, st);
    case 6: return convert_ll<LS, 6>(src, dst, n, st);
    case 7: return convert_ll<LS, 7>(src, dst, n, st);
    case 8: return convert_ll<LS, 8>(src, dst, n, st);
    case 9: return convert_ll<LS, 9>(src, dst, n, st);
    default: return fail(SPH_E_LAYOUT, "unknown layout");
    }
}

// ---------------------------------------------------------------------------
// smoothing-length iteration: Newton steps on rho(h) h^3 = m eta^3 between
// density passes (the per-particle update between the density and gradient
// loops)
// ---------------------------------------------------------------------------
struct HIterArgs {
    StoreArg store;
    const Chunk *tiles;
    const double *reach;  // per cell: the support its tasks cover
    int64_t ntile;
    float eta3;        // eta^3
    float tol;         // converged when |dh| <= tol h
    int32_t *flags;    // per tile: the tile's particles moved by this step
};

// One wave per tile.  With f(h) = rho h^3 - m eta^3 and f' = h^3 rho' + 3 h^2
// rho, the Newton step is dh = -h (rho - n) / (3 rho + h rho'), n = m eta^3 /
// h^3 the density at which h would be consistent; where the denominator is
// not positive the step is the fixed-point one, h eta-scaled to the current
// density.  A particle whose step is within tol h keeps its h (and with it the
// density just computed); any other takes h + dh limited to [h/2, 2h].  Every
// h, moved or not, is then held to a support no wider than its cell's reach
// (the distance within which the cell's tasks cover every other cell).
template <int L>
__global__ __launch_bounds__(256) void k_h_newton(HIterArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = __builtin_amdgcn_readfirstlane((int)((int64_t)blockIdx.x * (blockDim.x >> 6) +
                                                           (threadIdx.x >> 6)));
    if (c >= a.ntile) return;
    const Chunk ch = a.tiles[c];
    bool moved = false;
    if (lane < ch.n) {
        const int64_t p = ch.part0 + lane;
        const float h = ld<L, FH, 0, float>(a.store, p);
        const float m = ld<L, FMASS, 0, float>(a.store, p);
        const float rho = ld<L, FRHO, 0, float>(a.store, p);
        const float drho = ld<L, FRHODH, 0, float>(a.store, p);
        const float n = m * a.eta3 / (h * h * h);
        const float den = 3.0f * rho + h * drho;
        const float dh = den > 0.0f ? -h * (rho - n) / den : h * (cbrtf(n / rho) - 1.0f);
        float hn = h;
        if (!(fabsf(dh) <= a.tol * h)) hn = fminf(fmaxf(h + dh, 0.5f * h), 2.0f * h);
        hn = fminf(hn, (float)(a.reach[ch.cell] / (double)kGammaK));
        if (hn != h) {
            st<L, FH, 0, float>(a.store, p, hn);
            moved = true;
        }
    }
    const uint64_t bal = __ballot(moved);
    if (lane == 0) a.flags[c] = (int32_t)__popcll(bal);
}

// the tiles flagged by the last step as a work list in ascending tile order
// (the plan's spatial order), by an ordered compaction: per-block counts of
// flagged tiles and of moved particles, one block's scan of them, then every
// block writes its flagged tiles at its offset (no atomics: a same-address
// atomic per tile serialises in L2)
__device__ __forceinline__ int32_t wave_sum_i(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(256) void k_flag_counts(const int32_t *flags, int64_t ntile, int32_t *blk,
                                                     int32_t *blk_moved)
{
    __shared__ int32_t ws[4], wm[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t mv = t < ntile ? flags[t] : 0;
    const uint64_t bal = __ballot(mv != 0);
    const int32_t sm = wave_sum_i(mv);
    if (lane == 0) {
        ws[wv] = (int32_t)__popcll(bal);
        wm[wv] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        blk[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
        blk_moved[blockIdx.x] = wm[0] + wm[1] + wm[2] + wm[3];
    }
}

// exclusive scan of nblk tile counts in place by one block of 256 threads,
// 256 counts per round with the running total carried; count[0] = moved
// particles (sum of blk_moved), count[1] = flagged tiles
__global__ __launch_bounds__(256) void k_scan_counts(int32_t *blk, const int32_t *blk_moved, int64_t nblk,
                                                     int32_t *count)
{
    __shared__ int32_t sh[256];
    __shared__ int32_t wm[4];
    int32_t carry = 0, moved = 0;
    for (int64_t b0 = 0; b0 < nblk; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int32_t v = i < nblk ? blk[i] : 0;
        const int32_t mvs = wave_sum_i(i < nblk ? blk_moved[i] : 0);
        if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mvs;
        sh[threadIdx.x] = v;
        __syncthreads();
        moved += wm[0] + wm[1] + wm[2] + wm[3];
        for (int off = 1; off < 256; off <<= 1) {
            const int32_t add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nblk) blk[i] = carry + sh[threadIdx.x] - v;
        carry += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        count[0] = moved;
        count[1] = carry;
    }
}

__global__ __launch_bounds__(256) void k_flag_scatter(const int32_t *flags, int64_t ntile, const int32_t *blk,
                                                      int32_t *items)
{
    __shared__ int32_t ws[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = t < ntile && flags[t] != 0;
    const uint64_t bal = __ballot(f);
    if (lane == 0) ws[wv] = (int32_t)__popcll(bal);
    __syncthreads();
    int32_t off = blk[blockIdx.x];
    for (int k = 0; k < wv; ++k) off += ws[k];
    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (f) items[off + rank] = (int32_t)t;
}

template <int L>
static sph_status h_newton_l(const HIterArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_h_newton<L>), dim3((unsigned)((a.ntile + 3) / 4)), dim3(256), 0, st, a);
    SPH_CHECK_LAUNCH("smoothing-length step launch");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// time integration around the loops: kick, drift and the CFL time step
// (float32 and float64 operations exactly as written, no contraction)
// ---------------------------------------------------------------------------
struct KickArgs {
    StoreArg store;
    int64_t n;
    float dt;
};

// v += a dt and u += u_dt dt, each a float32 product rounded, then a sum.
// Every load is issued before the first store: loads and stores complete
// through one in-order counter, so a load placed after a store would wait for
// that store too, and the particle would take one memory round trip per field
// instead of one in all.
template <int L>
__global__ __launch_bounds__(256) void k_kick(KickArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    float v[3], acc[3];
    static_for<0, 3>([&](auto cc) {
        constexpr int C = decltype(cc)::value;
        v[C] = ld<L, FV, C, float>(a.store, p);
        acc[C] = ld<L, FA, C, float>(a.store, p);
    });
    const float u = ld<L, FU, 0, float>(a.store, p), udt = ld<L, FUDT, 0, float>(a.store, p);
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, 3>([&](auto cc) {
        constexpr int C = decltype(cc)::value;
        st<L, FV, C, float>(a.store, p, v[C] + acc[C] * a.dt);
    });
    st<L, FU, 0, float>(a.store, p, u + udt * a.dt);
}

struct DriftArgs {
    StoreArg store;
    const Chunk *tiles;
    const sph_cell *cells;
    int64_t ntile;
    double dt;
    double *blk_out;  // per block: largest distance of a particle outside its cell
    float *blk_h;     // per block: largest h
    float kick_dt;    // KICK: the kick before the drift (v, u += a, u_dt times this)
    int kick;
};

__device__ __forceinline__ double wave_max_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max_f(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_min_f(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}

// x += v dt in float64 (v widened exactly), one wave per tile, the waves
// striding over the tiles (a bounded grid keeps the per-block partials few);
// the distance by which the drifted particle lies outside its cell's cube, in
// float64.  KICK: the half kick of a kick-drift-kick step first, in the same
// pass (the same operations as k_kick, then the drift with the kicked v).
template <int L, bool KICK>
__global__ __launch_bounds__(256) void k_drift(DriftArgs a)
{
    __shared__ double so[4];
    __shared__ float sh[4];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double out = 0.0;
    float hm = 0.0f;
    for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv; c < a.ntile;
         c += (int64_t)gridDim.x * (blockDim.x >> 6)) {
        const Chunk ch = a.tiles[c];
        if (lane < ch.n) {
            const int64_t p = ch.part0 + lane;
            const sph_cell cl = a.cells[ch.cell];
            // every load before the first store (one memory round trip per
            // tile, as in k_kick)
            float v[3], acc[3], u = 0.0f, udt = 0.0f;
            double x[3];
            static_for<0, 3>([&](auto cc) {
                constexpr int C = decltype(cc)::value;
                v[C] = ld<L, FV, C, float>(a.store, p);
                if constexpr (KICK) acc[C] = ld<L, FA, C, float>(a.store, p);
                x[C] = ld<L, FX, C, double>(a.store, p);
            });
            if constexpr (KICK) {
                u = ld<L, FU, 0, float>(a.store, p);
                udt = ld<L, FUDT, 0, float>(a.store, p);
            }
            hm = fmaxf(hm, ld<L, FH, 0, float>(a.store, p));
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (KICK) st<L, FU, 0, float>(a.store, p, u + udt * a.kick_dt);
            double e2 = 0.0;
            static_for<0, 3>([&](auto cc) {
                constexpr int C = decltype(cc)::value;
                if constexpr (KICK) {
                    v[C] = v[C] + acc[C] * a.kick_dt;
                    st<L, FV, C, float>(a.store, p, v[C]);
                }
                const double xn = x[C] + (double)v[C] * a.dt;
                st<L, FX, C, double>(a.store, p, xn);
                const double e = fmax(fmax(cl.loc[C] - xn, xn - (cl.loc[C] + cl.width)), 0.0);
                e2 = e2 + e * e;
            });
            out = fmax(out, sqrt(e2));
        }
    }
    out = wave_max_d(out);
    hm = wave_max_f(hm);
    if (lane == 0) {
        so[wv] = out;
        sh[wv] = hm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.blk_out[blockIdx.x] = fmax(fmax(so[0], so[1]), fmax(so[2], so[3]));
        a.blk_h[blockIdx.x] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
    }
}

// per block: the smallest cfl (gamma_K h) / v_sig over particles with v_sig > 0
struct CflArgs {
    StoreArg store;
    int64_t n;
    float cfl;
    float *blk_dt;
};

template <int L>
__global__ __launch_bounds__(256) void k_cfl(CflArgs a)
{
    __shared__ float sm[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float dt = __builtin_huge_valf();
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += (int64_t)gridDim.x * blockDim.x) {
        const float vs = ld<L, FVSIG, 0, float>(a.store, p);
        if (vs > 0.0f) dt = fminf(dt, (a.cfl * (kGammaK * ld<L, FH, 0, float>(a.store, p))) / vs);
    }
    dt = wave_min_f(dt);
    if (lane == 0) sm[wv] = dt;
    __syncthreads();
    if (threadIdx.x == 0) a.blk_dt[blockIdx.x] = fminf(fminf(sm[0], sm[1]), fminf(sm[2], sm[3]));
}

// one block folds the per-block partials: out[0] = max of d, out[1] = max of
// f (as float bits in a double slot), or the min of f when MIN
template <bool MIN>
__global__ __launch_bounds__(256) void k_fold(const double *d, const float *f, int64_t nblk, double *out)
{
    __shared__ double sd[4];
    __shared__ float sf[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double md = 0.0;
    float mf = MIN ? __builtin_huge_valf() : 0.0f;
    for (int64_t i = threadIdx.x; i < nblk; i += blockDim.x) {
        if (d) md = fmax(md, d[i]);
        mf = MIN ? fminf(mf, f[i]) : fmaxf(mf, f[i]);
    }
    md = wave_max_d(md);
    mf = MIN ? wave_min_f(mf) : wave_max_f(mf);
    if (lane == 0) {
        sd[wv] = md;
        sf[wv] = mf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = fmax(fmax(sd[0], sd[1]), fmax(sd[2], sd[3]));
        out[1] = MIN ? (double)fminf(fminf(sf[0], sf[1]), fminf(sf[2], sf[3]))
                     : (double)fmaxf(fmaxf(sf[0], sf[1]), fmaxf(sf[2], sf[3]));
    }
}

template <int L>
static sph_status kick_l(const KickArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_kick<L>), dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
    SPH_CHECK_LAUNCH("kick launch");
    return SPH_OK;
}

// blocks of the reductions' first stage (grid-stride beyond)
constexpr int64_t kFoldBlocks = 2048;

template <int L>
static sph_status drift_l(const DriftArgs &a, hipStream_t st)
{
    const dim3 grid((unsigned)std::min<int64_t>((a.ntile + 3) / 4, kFoldBlocks));
    if (a.kick) hipLaunchKernelGGL((k_drift<L, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_drift<L, false>), grid, dim3(256), 0, st, a);
    SPH_CHECK_LAUNCH("drift launch");
    return SPH_OK;
}

template <int L>
static sph_status cfl_l(const CflArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_cfl<L>), dim3((unsigned)std::min<int64_t>((a.n + 255) / 256, kFoldBlocks)), dim3(256), 0,
                       st, a);
    SPH_CHECK_LAUNCH("time-step launch");
    return SPH_OK;
}

#define SPH_BY_LAYOUT(layout, fn, ...)                                              \
    switch (layout) {                                                               \
    case 0: return fn<0>(__VA_ARGS__); case 1: return fn<1>(__VA_ARGS__);            \
    case 2: return fn<2>(__VA_ARGS__); case 3: return fn<3>(__VA_ARGS__);            \
    case 4: return fn<4>(__VA_ARGS__); case 5: return fn<5>(__VA_ARGS__);            \
    case 6: return fn<6>(__VA_ARGS__); case 7: return fn<7>(__VA_ARGS__);            \
    case 8: return fn<8>(__VA_ARGS__); case 9: return fn<9>(__VA_ARGS__);            \
    default: return fail(SPH_E_LAYOUT, "unknown layout");                           \
    }

sph_status launch_pack(const sph_plan *p, int loop, const sph_store *s, bool cells, int32_t t0, int32_t t1,
                       void *buf, int waves, hipStream_t st, int schedule)
{
    PackArgs a{};
    a.store = store_arg(s);
    a.cells = p->d_cells;
    a.tasks = p->d_tasks;
    a.buf = (char *)buf;
    int64_t nslot;
    if (cells) {
        a.chunks = p->d_tiles;
        a.chunk_base = 0;
        a.nchunk = p->ntile;
        a.slot_base = 0;
        nslot = p->n;
    } else {
        a.chunks = p->d_chunks;
        a.chunk_base = p->chunk_off[t0];
        a.nchunk = p->chunk_off[t1] - p->chunk_off[t0];
        a.slot_base = p->slot_off[t0];
        nslot = p->slot_off[t1] - p->slot_off[t0];
    }
    a.P = round_slots(nslot);
    a.bounds = (float4 *)(a.buf + a.P * 4 * kPackFloats[loop]);
    if (a.nchunk == 0) return SPH_OK;
    SPH_BY_LAYOUT(s->layout, pack_l, p, loop, a, waves, schedule, st);
}

template <int L>
static void writers_l(int32_t *w)
{
    for (int q = 0; q < kStepPlanes; ++q) w[q] = step_writer(L, q);
}

sph_status step_writers(int layout, int32_t *w)
{
    switch (layout) {
    case 0: writers_l<0>(w); break;
    case 1: writers_l<1>(w); break;
    case 2: writers_l<2>(w); break;
    case 3: writers_l<3>(w); break;
    case 4: writers_l<4>(w); break;
    case 5: writers_l<5>(w); break;
    case 6: writers_l<6>(w); break;
    case 7: writers_l<7>(w); break;
    case 8: writers_l<8>(w); break;
    case 9: writers_l<9>(w); break;
    default: return fail(SPH_E_LAYOUT, "unknown layout");
    }
    return SPH_OK;
}

sph_status launch_pack_step(const sph_plan *p, int loop, const sph_store *s, const float *res, void *buf,
                            float *derived, const sph_params *prm, int waves, hipStream_t st)
{
    PackArgs a{};
    a.store = store_arg(s);
    a.cells = p->d_cells;
    a.tasks = p->d_tasks;
    a.buf = (char *)buf;
    a.chunks = p->d_tiles;
    a.chunk_base = 0;
    a.nchunk = p->ntile;
    a.slot_base = 0;
    a.P = round_slots(p->n);
    a.bounds = (float4 *)(a.buf + a.P * 4 * kPackFloats[loop]);
    a.step_res = res;
    a.derived = derived;
    a.gam = prm->gamma_ad;
    a.eps = prm->balsara_eps;
    if (a.nchunk == 0) return SPH_OK;
    SPH_BY_LAYOUT(s->layout, pack_step_l, loop, a, waves, st);
}

sph_status launch_writeback(const sph_plan *p, const sph_store *s, const float *res, int waves, hipStream_t st)
{
    UnpackArgs a{};
    a.store = store_arg(s);
    a.chunks = p->d_tiles;
    a.nchunk = p->ntile;
    a.P = round_slots(p->n);
    a.res = res;
    a.n = p->n;
    if (a.nchunk == 0) return SPH_OK;
    SPH_BY_LAYOUT(s->layout, writeback_l, a, waves, st);
}

sph_status launch_pack_tiles(const sph_plan *p, int loop, const sph_store *s, int32_t tile0, int32_t tile1,
                             void *buf, int waves, hipStream_t st, int schedule)
{
    PackArgs a{};
    a.store = store_arg(s);
    a.cells = p->d_cells;
    a.tasks = p->d_tasks;
    a.buf = (char *)buf;
    a.chunks = p->d_tiles;
    a.chunk_base = tile0;
    a.nchunk = tile1 - tile0;
    a.slot_base = 0;
    a.P = round_slots(p->n);
    // chunk c of the launch is tile tile0 + c: its bounds sit at that tile's place
    a.bounds = (float4 *)(a.buf + a.P * 4 * kPackFloats[loop]) + 2 * (int64_t)tile0;
    if (a.nchunk <= 0) return SPH_OK;
    SPH_BY_LAYOUT(s->layout, pack_l, p, loop, a, waves, schedule, st);
}

sph_status launch_unpack_tiles(const sph_plan *p, int loop, const void *res, int32_t tile0, int32_t tile1,
                               const sph_store *s, int waves, hipStream_t st, int schedule)
{
    UnpackArgs a{};
    a.store = store_arg(s);
    a.res = (const float *)res;
    a.n = p->n;
    a.chunks = p->d_tiles;
    a.chunk_base = tile0;
    a.nchunk = tile1 - tile0;
    a.P = round_slots(p->n);
    if (a.nchunk <= 0) return SPH_OK;
    SPH_BY_LAYOUT(s->layout, unpack_l, loop, a, true, false, waves, schedule, st);
}

sph_status launch_unpack(sph_plan *p, int loop, const void *res, bool cells, int32_t t0, int32_t t1,
                         const sph_store *s, int waves, hipStream_t st, int schedule)
{
    UnpackArgs a{};
    a.store = store_arg(s);
    a.res = (const float *)res;
    a.n = p->n;
    bool csr = false;
    if (cells) {
        a.chunks = p->d_tiles;
        a.nchunk = p->ntile;
        a.P = round_slots(p->n);
    } else {
        a.chunks = p->d_chunks;
        a.chunk_base = p->chunk_off[t0];
        a.nchunk = p->chunk_off[t1] - p->chunk_off[t0];
        a.slot_base = p->slot_off[t0];
        a.P = round_slots(p->slot_off[t1] - p->slot_off[t0]);
        if (t1 - t0 > 1) {
            csr = true;
            a.csr_off = p->d_csr_off;
            a.csr = p->d_csr;
            a.slot_lo = p->slot_off[t0];
            a.slot_hi = p->slot_off[t1];
        }
    }
    if (a.nchunk == 0) return SPH_OK;
    SPH_BY_LAYOUT(s->layout, unpack_l, loop, a, cells, csr, waves, schedule, st);
}

sph_status launch_convert(const sph_store *src, const sph_store *dst, hipStream_t st)
{
    if (src->n == 0) return SPH_OK;
    const StoreArg a = store_arg(src), b = store_arg(dst);
    SPH_BY_LAYOUT(src->layout, convert_l, dst->layout, a, b, src->n, st);
}

sph_status launch_h_newton(const sph_plan *p, const sph_store *s, float eta, float tol, int32_t *flags,
                           hipStream_t st)
{
    HIterArgs a{};
    a.store = store_arg(s);
    a.tiles = p->d_tiles;
    a.reach = p->d_reach;
    a.ntile = p->ntile;
    a.eta3 = eta * eta * eta;
    a.tol = tol;
    a.flags = flags;
    if (a.ntile == 0) return SPH_OK;
    SPH_BY_LAYOUT(s->layout, h_newton_l, a, st);
}

sph_status launch_flagged_tiles(const sph_plan *p, const int32_t *flags, int32_t *items, int32_t *blk,
                                int32_t *count, hipStream_t st)
{
    if (p->ntile == 0) return SPH_OK;
    const int64_t nblk = ((int64_t)p->ntile + 255) / 256;
    int32_t *blk_moved = blk + nblk;
    hipLaunchKernelGGL(k_flag_counts, dim3((unsigned)nblk), dim3(256), 0, st, flags, (int64_t)p->ntile, blk,
                       blk_moved);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(256), 0, st, blk, (const int32_t *)blk_moved, nblk, count);
    hipLaunchKernelGGL(k_flag_scatter, dim3((unsigned)nblk), dim3(256), 0, st, flags, (int64_t)p->ntile, blk, items);
    SPH_CHECK_LAUNCH("tile list launch");
    return SPH_OK;
}

static size_t fold_blocks(const sph_plan *p)
{
    return (size_t)std::min<int64_t>(std::max<int64_t>((p->ntile + 3) / 4, (p->n + 255) / 256), kFoldBlocks);
}

size_t integrate_ws_bytes(const sph_plan *p)
{
    const size_t nb = fold_blocks(p);
    return (nb * 8 + 255) / 256 * 256 + (nb * 4 + 255) / 256 * 256 + 256;
}

sph_status launch_kick(const sph_store *s, float dt, hipStream_t st)
{
    KickArgs a{store_arg(s), s->n, dt};
    if (a.n == 0) return SPH_OK;
    SPH_BY_LAYOUT(s->layout, kick_l, a, st);
}

sph_status launch_drift(const sph_plan *p, const sph_store *s, double dt, void *ws, hipStream_t st, bool kick,
                        float kick_dt)
{
    const size_t nb = fold_blocks(p);
    DriftArgs a{};
    a.kick = kick ? 1 : 0;
    a.kick_dt = kick_dt;
    a.store = store_arg(s);
    a.tiles = p->d_tiles;
    a.cells = p->d_cells;
    a.ntile = p->ntile;
    a.dt = dt;
    a.blk_out = (double *)ws;
    a.blk_h = (float *)((char *)ws + (nb * 8 + 255) / 256 * 256);
    double *out = (double *)((char *)a.blk_h + (nb * 4 + 255) / 256 * 256);
    if (a.ntile == 0) return SPH_OK;
    const int64_t nblk = std::min<int64_t>((a.ntile + 3) / 4, kFoldBlocks);
    sph_status r;
    switch (s->layout) {
    case 0: r = drift_l<0>(a, st); break;
    case 1: r = drift_l<1>(a, st); break;
    case 2: r = drift_l<2>(a, st); break;
    case 3: r = drift_l<3>(a, st); break;
    case 4: r = drift_l<4>(a, st); break;
    case 5: r = drift_l<5>(a, st); break;
    case 6: r = drift_l<6>(a, st); break;
    case 7: r = drift_l<7>(a, st); break;
    case 8: r = drift_l<8>(a, st); break;
    case 9: r = drift_l<9>(a, st); break;
    default: return fail(SPH_E_LAYOUT, "unknown layout");
    }
    if (r) return r;
    hipLaunchKernelGGL(k_fold<false>, dim3(1), dim3(256), 0, st, (const double *)a.blk_out, (const float *)a.blk_h,
                       nblk, out);
    SPH_CHECK_LAUNCH("fold launch");
    return SPH_OK;
}

sph_status launch_cfl(const sph_plan *p, const sph_store *s, float cfl, void *ws, hipStream_t st)
{
    const size_t nb = fold_blocks(p);
    CflArgs a{store_arg(s), s->n, cfl, (float *)((char *)ws + (nb * 8 + 255) / 256 * 256)};
    double *out = (double *)((char *)a.blk_dt + (nb * 4 + 255) / 256 * 256);
    if (a.n == 0) return SPH_OK;
    const int64_t nblk = std::min<int64_t>((a.n + 255) / 256, kFoldBlocks);
    sph_status r;
    switch (s->layout) {
    case 0: r = cfl_l<0>(a, st); break;
    case 1: r = cfl_l<1>(a, st); break;
    case 2: r = cfl_l<2>(a, st); break;
    case 3: r = cfl_l<3>(a, st); break;
    case 4: r = cfl_l<4>(a, st); break;
    case 5: r = cfl_l<5>(a, st); break;
    case 6: r = cfl_l<6>(a, st); break;
    case 7: r = cfl_l<7>(a, st); break;
    case 8: r = cfl_l<8>(a, st); break;
    case 9: r = cfl_l<9>(a, st); break;
    default: return fail(SPH_E_LAYOUT, "unknown layout");
    }
    if (r) return r;
    hipLaunchKernelGGL(k_fold<true>, dim3(1), dim3(256), 0, st, (const double *)nullptr, (const float *)a.blk_dt,
                       nblk, out);
    SPH_CHECK_LAUNCH("fold launch");
    return SPH_OK;
}

}  // namespace sph
