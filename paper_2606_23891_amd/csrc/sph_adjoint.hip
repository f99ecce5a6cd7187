// Hand-written adjoint of L = sum_i |a_i|^2 through the density and force
// loops (the differentiable form of the interaction loops of Sec. 2.1).
//
// Inputs are per-particle arrays in store order; the artificial-viscosity
// switch alpha~ and alpha_d, h and u are constants.  The backward pass never
// stores pair terms: it re-evaluates them, and it recomputes the density of
// the current positions instead of taking it from the forward pass.
//
// Pair form used for the force adjoint.  With r = x_k - x_j, v = v_k - v_j,
//   a_k = - sum_j m_j S_kj r,   S = A_k F_k(r) + A_j F_j(r) + Pi(mu) Fbar(r),
// and S symmetric in (k, j), the contribution of the pair {k, j} to dL is
//   Phi = S (r . w),   w = m_k abar_j - m_j abar_k,
// so every particle gathers dPhi/dr, dPhi/dv, dPhi/dm_k, dPhi/drho_k and
// dPhi/drho_dh_k over its own neighbours -- no atomics, no scatter.
// The density adjoint then gathers, for the pair {k, j},
//   m_j (rhobar_k W'(r,h_k) + rhodhbar_k W_h'(r,h_k)) rhat
// + m_k (rhobar_j W'(r,h_j) + rhodhbar_j W_h'(r,h_j)) rhat  into xbar_k and
//   rhobar_j W(r,h_j) + rhodhbar_j W_h(r,h_j)                 into mbar_k.
//
// Mapping: one wave per tile (up to 64 particles of one cell, one per lane),
// optionally split over several waves that take disjoint ranges of the cell's
// neighbour entries (a small set fills the chip that way; the partial sums are
// added in a fixed order by a second kernel).  The wave walks the particles of
// its neighbour cells 64 at a time, one per lane, keeps those within reach of
// the tile's box and compacts them (ballot + prefix count) into an LDS window
// with what the pair term needs of them, computed once per staged candidate.
// When the window is full every lane tests its particle against every
// candidate (one bit per candidate), then walks only its own hits, lowest
// first, so each particle's pair terms are summed in the order of the walk.
// Arithmetic is float64 throughout, with separations taken from the float64
// positions; the stored inputs v, m, h, u, alpha~, alpha_d are float32.  a is a sum of pair terms that nearly
// cancel on a near-uniform particle set, and so are the gradient components
// that are small against their kind's rms: float32 pair arithmetic (and the
// float32 rounding of a position offset alone, about 1e-7 of a pair
// separation) leaves those components a few 1e-4 off, where float64 keeps
// them to rounding.  MI355X runs float64 vector arithmetic at the rate of
// unpacked float32.
#include <hip/hip_runtime.h>

#include "sph_internal.hpp"

namespace sph {

constexpr double kGammaK64 = 1.8257418583505537115;  // sqrt(10/3)
constexpr double kC3_64 = 2.5464790894703253723;     // 8 / pi

struct AdjArgs {
    int64_t n, P;  // particles, workspace plane stride
    const Chunk *tiles;
    int32_t ntile;
    const CellRange *cellr;
    const Nbr *nbr;
    const int32_t *nbr_off;
    const sph_cell *cells;
    // per particle (workspace)
    float2 *hm;      // h m
    float4 *v;       // vx vy vz (w unused)
    float4 *ua;      // u alpha~ alpha_d (w unused)
    double *rho64;   // rho, rho_dh of the current positions
    double gam, beta;
};

// cubic spline w(q), w'(q), w''(q) for q < 1
__device__ __forceinline__ void spl64(double q, double &w, double &dw, double &d2w)
{
    if (q < 0.5) {
        w = 1.0 - 6.0 * q * q + 6.0 * q * q * q;
        dw = -12.0 * q + 18.0 * q * q;
        d2w = -12.0 + 36.0 * q;
    } else {
        const double t = q < 1.0 ? 1.0 - q : 0.0;
        w = 2.0 * t * t * t;
        dw = -6.0 * t * t;
        d2w = 12.0 * t;
    }
}

// F = (1/r) dW/dr = C3 H^-5 w'(q)/q and dF/dr = C3 H^-6 (q w'' - w')/q^2, both 0
// beyond H; from r, 1/r (0 at r = 0, where only the inner piece is reached),
// H and 1/H, with 1/q = H/r, so no division
__device__ __forceinline__ void kern_F64(double r, double ir, double H, double iH, double &F, double &Fp)
{
    if (!(r < H)) {
        F = 0.0;
        Fp = 0.0;
        return;
    }
    const double q = r * iH, iH2 = iH * iH;
    const double K5 = kC3_64 * iH2 * iH2 * iH;
    if (q < 0.5) {
        F = K5 * (-12.0 + 18.0 * q);
        Fp = K5 * iH * 18.0;
    } else {
        const double t = 1.0 - q;
        F = K5 * (-6.0 * t * t * H * ir);
        Fp = K5 * 6.0 * t * (1.0 + q) * H * ir * ir;
    }
}

// per-particle quantities of the force loop, from the workspace's float64
// density of the same positions
struct Q64 {
    double H, iH, A, Aom, c, rho, om, u, at, ad;  // om = rho + h rho_dh / 3, Aom = A / om
};

__device__ __forceinline__ Q64 q64(const AdjArgs &a, int64_t i)
{
    Q64 p;
    const double h = a.hm[i].x;
    const float4 ua = a.ua[i];
    const double g = a.gam;
    p.H = kGammaK64 * h;
    p.iH = 1.0 / p.H;
    p.rho = a.rho64[2 * i];
    p.om = p.rho + h * a.rho64[2 * i + 1] / 3.0;
    p.u = ua.x;
    p.A = (g - 1.0) * p.u / p.om;
    p.Aom = p.A / p.om;
    p.c = sqrt(g * (g - 1.0) * p.u);
    p.at = ua.y;
    p.ad = ua.z;
    return p;
}

// ---------------------------------------------------------------------------
// pair kinds and candidate windows
// ---------------------------------------------------------------------------
// Kinds: 0 density, 1 force, 2 force adjoint, 3 density adjoint.  A staged
// candidate takes NF doubles: its position translated into the tile's frame,
// then its support gamma h_j (its mass for the density), then what the pair
// term reads of it.  WIN candidates per window, NACC sums per particle, WAVES
// resident waves per SIMD the register allocation must allow.  MIXED kinds
// interact within max(H_i, H_j), the density within H_i.
template <int KIND>
struct AdjKind;
template <>
struct AdjKind<0> {
    static constexpr int NF = 4, WIN = 128, NACC = 2, WAVES = 6;
    static constexpr bool MIXED = false;
};
template <>
struct AdjKind<1> {  // x y | z H | A c | rho u | at ad | m vx | vy vz | j 1/H
    static constexpr int NF = 16, WIN = 64, NACC = 4, WAVES = 4;
    static constexpr bool MIXED = true;
};
template <>
struct AdjKind<2> {  // x y | z H | A c | rho at | m vx | vy vz | abx aby | abz j | 1/H -
    static constexpr int NF = 18, WIN = 64, NACC = 9, WAVES = 3;
    static constexpr bool MIXED = true;
};
template <>
struct AdjKind<3> {  // x y | z H | m rhobar | rhodhbar 1/H
    static constexpr int NF = 8, WIN = 128, NACC = 4, WAVES = 4;
    static constexpr bool MIXED = true;
};

constexpr int kAdjMaxSplit = 4, kAdjMaxAcc = 9;

// arrays of one pass
struct AdjIO {
    const double *x;
    const double *abar;              // force adjoint: dL/da
    const double *rbar, *dbar;       // density adjoint: dL/drho, dL/drho_dh
    double *o0, *o1, *o2, *o3, *o4;  // outputs, per kind (see adj_finish)
    double *part;                    // split > 1: partial sums [split][NACC][P]
    int32_t split;
};

// the lane's particle
struct IAdj {
    double x, y, z, H, H2, iH;
    Q64 P;
    double vx, vy, vz, abx, aby, abz, hk, mk, rbk, dbk;
};

template <int KIND>
__device__ __forceinline__ void adj_load_i(const AdjArgs &a, const AdjIO &io, int64_t k, IAdj &I)
{
    I.x = io.x[3 * k];
    I.y = io.x[3 * k + 1];
    I.z = io.x[3 * k + 2];
    const float2 hm = a.hm[k];
    I.H = kGammaK64 * (double)hm.x;
    I.H2 = I.H * I.H;
    I.iH = 1.0 / I.H;
    I.hk = hm.x;
    I.mk = hm.y;
    if constexpr (KIND == 1 || KIND == 2) {
        I.P = q64(a, k);
        const float4 v = a.v[k];
        I.vx = v.x;
        I.vy = v.y;
        I.vz = v.z;
    }
    if constexpr (KIND == 2) {
        I.abx = io.abar[3 * k];
        I.aby = io.abar[3 * k + 1];
        I.abz = io.abar[3 * k + 2];
    }
    if constexpr (KIND == 3) {
        I.rbk = io.rbar[k];
        I.dbk = io.dbar[k];
    }
}

// the staged record of candidate j at position (xj, yj, zj) in the tile's frame
template <int KIND>
__device__ __forceinline__ void adj_stage(const AdjArgs &a, const AdjIO &io, int64_t j, double xj, double yj,
                                          double zj, double Hj, double2 *r)
{
    const double mj = a.hm[j].y;
    r[0] = make_double2(xj, yj);
    r[1] = make_double2(zj, KIND == 0 ? mj : Hj);
    if constexpr (KIND == 1 || KIND == 2) {
        const Q64 Q = q64(a, j);
        const float4 v = a.v[j];
        r[2] = make_double2(Q.A, Q.c);
        if constexpr (KIND == 1) {
            r[3] = make_double2(Q.rho, Q.u);
            r[4] = make_double2(Q.at, Q.ad);
            r[5] = make_double2(mj, (double)v.x);
            r[6] = make_double2((double)v.y, (double)v.z);
            r[7] = make_double2((double)j, Q.iH);
        } else {
            r[3] = make_double2(Q.rho, Q.at);
            r[4] = make_double2(mj, (double)v.x);
            r[5] = make_double2((double)v.y, (double)v.z);
            r[6] = make_double2(io.abar[3 * j], io.abar[3 * j + 1]);
            r[7] = make_double2(io.abar[3 * j + 2], (double)j);
            r[8] = make_double2(Q.iH, 0.0);
        }
    }
    if constexpr (KIND == 3) {
        r[2] = make_double2(mj, io.rbar[j]);
        r[3] = make_double2(io.dbar[j], 1.0 / Hj);
    }
}

// separation of the lane's particle from a staged candidate
__device__ __forceinline__ double adj_r2(const IAdj &I, const double2 *r, double &rx, double &ry, double &rz)
{
    const double2 p0 = r[0], p1 = r[1];
    rx = I.x - p0.x;
    ry = I.y - p0.y;
    rz = I.z - p1.x;
    return rx * rx + ry * ry + rz * rz;
}

// the pair term of the lane's particle k with a staged candidate that passed
// the support test, added to the sums s
template <int KIND>
__device__ __forceinline__ void adj_pair(const AdjArgs &a, const IAdj &I, int64_t k, const double2 *rec, double *s)
{
    double rx, ry, rz;
    const double r2 = adj_r2(I, rec, rx, ry, rz);
    if constexpr (KIND == 0) {
        const double q = sqrt(r2) * I.iH;
        double w, dw, d2w;
        spl64(q, w, dw, d2w);
        const double mj = rec[1].y;
        s[0] += mj * w;
        s[1] += mj * (3.0 * w + q * dw);
    } else if constexpr (KIND == 1) {
        const double2 c2 = rec[2], c3 = rec[3], c4 = rec[4], c5 = rec[5], c6 = rec[6], c7 = rec[7];
        if (c7.x == (double)k) return;  // j == k
        const Q64 &P = I.P;
        const double QH = rec[1].y, QA = c2.x, Qc = c2.y, Qrho = c3.x, Qu = c3.y, Qat = c4.x, Qad = c4.y;
        const double mj = c5.x;
        const double r = sqrt(r2);
        const double ir = r > 0.0 ? 1.0 / r : 0.0;
        double Fk, Fkp, Fj, Fjp;
        kern_F64(r, ir, P.H, P.iH, Fk, Fkp);
        kern_F64(r, ir, QH, c7.y, Fj, Fjp);
        const double Fb = 0.5 * (Fk + Fj);
        const double vx = I.vx - c5.y, vy = I.vy - c6.x, vz = I.vz - c6.y;
        const double dot = vx * rx + vy * ry + vz * rz;
        const double mu = dot < 0.0 ? dot * ir : 0.0;
        const double irb = 2.0 / (P.rho + Qrho);  // 1 / rho_ij
        const double Pi = -0.5 * 0.5 * (P.at + Qat) * (P.c + Qc - a.beta * mu) * mu * irb;
        const double S = P.A * Fk + QA * Fj + Pi * Fb;
        s[0] -= mj * S * rx;
        s[1] -= mj * S * ry;
        s[2] -= mj * S * rz;
        s[3] += mj * (P.A * Fk * dot + 0.5 * Pi * Fb * dot + 0.5 * (P.ad + Qad) * fabs(dot) * (P.u - Qu) * Fb * irb);
    } else if constexpr (KIND == 2) {
        const double2 c2 = rec[2], c3 = rec[3], c4 = rec[4], c5 = rec[5], c6 = rec[6], c7 = rec[7];
        if (c7.y == (double)k) return;  // j == k
        const Q64 &P = I.P;
        const double QH = rec[1].y, QA = c2.x, Qc = c2.y, Qrho = c3.x, Qat = c3.y;
        const double mj = c4.x;
        const double r = sqrt(r2);
        const double ir = r > 0.0 ? 1.0 / r : 0.0;
        const double ex = rx * ir, ey = ry * ir, ez = rz * ir;
        double Fk, Fkp, Fj, Fjp;
        kern_F64(r, ir, P.H, P.iH, Fk, Fkp);
        kern_F64(r, ir, QH, rec[8].x, Fj, Fjp);
        const double Fb = 0.5 * (Fk + Fj), Fbp = 0.5 * (Fkp + Fjp);
        const double vx = I.vx - c4.y, vy = I.vy - c5.x, vz = I.vz - c5.y;
        const double dot = vx * rx + vy * ry + vz * rz;
        const bool appr = r > 0.0 && dot < 0.0;
        const double mu = appr ? dot * ir : 0.0;
        const double irb = 2.0 / (P.rho + Qrho);  // 1 / rho_ij
        const double al = 0.5 * (P.at + Qat);
        const double Pi = -0.5 * al * (P.c + Qc - a.beta * mu) * mu * irb;
        const double dPi = -0.5 * (al * irb) * (P.c + Qc - 2.0 * a.beta * mu);  // dPi/dmu
        const double S = P.A * Fk + QA * Fj + Pi * Fb;
        const double abjx = c6.x, abjy = c6.y, abjz = c7.x;
        const double wx = I.mk * abjx - mj * I.abx, wy = I.mk * abjy - mj * I.aby, wz = I.mk * abjz - mj * I.abz;
        const double rw = rx * wx + ry * wy + rz * wz;
        // grad_r S = (A_k F_k' + A_j F_j' + Pi Fbar') rhat + Fbar dPi/dmu grad_r mu
        const double sr = P.A * Fkp + QA * Fjp + Pi * Fbp;
        double mx = 0, my = 0, mz = 0;  // grad_r mu
        if (appr) {
            mx = (vx - mu * ex) * ir;
            my = (vy - mu * ey) * ir;
            mz = (vz - mu * ez) * ir;
        }
        const double cP = Fb * dPi;
        s[0] += S * wx + rw * (sr * ex + cP * mx);
        s[1] += S * wy + rw * (sr * ey + cP * my);
        s[2] += S * wz + rw * (sr * ez + cP * mz);
        if (appr) {  // grad_v mu = rhat
            s[3] += rw * cP * ex;
            s[4] += rw * cP * ey;
            s[5] += rw * cP * ez;
        }
        s[6] += S * (rx * abjx + ry * abjy + rz * abjz);
        s[7] += rw * (Fk * -P.Aom - 0.5 * Fb * Pi * irb);
        s[8] += rw * Fk * (-(I.hk / 3.0) * P.Aom);
    } else {
        const double Hk = I.H, Hj = rec[1].y;
        const double2 c2 = rec[2];
        const double mj = c2.x;
        const double r = sqrt(r2);
        const double ir = r > 0.0 ? 1.0 / r : 0.0;
        double g = 0.0;  // radial derivative collected over both directions
        if (r < Hk) {    // rho_k's term m_j W(r, h_k)
            const double iH = I.iH, q = r * iH;
            double w, dw, d2w;
            spl64(q, w, dw, d2w);
            const double iH4 = iH * iH * iH * iH;
            const double Wr = kC3_64 * iH4 * dw;                                       // dW/dr
            const double Whr = -kGammaK64 * kC3_64 * iH4 * iH * (4.0 * dw + q * d2w);  // d(dW/dh)/dr
            g += mj * (I.rbk * Wr + I.dbk * Whr);
        }
        if (r < Hj) {  // rho_j's term m_k W(r, h_j)
            const double iH = rec[3].y, q = r * iH;
            double w, dw, d2w;
            spl64(q, w, dw, d2w);
            const double iH3 = iH * iH * iH, iH4 = iH3 * iH;
            const double rbj = c2.y, dbj = rec[3].x;
            g += I.mk * (rbj * kC3_64 * iH4 * dw + dbj * (-kGammaK64 * kC3_64 * iH4 * iH * (4.0 * dw + q * d2w)));
            s[3] += rbj * kC3_64 * iH3 * w + dbj * (-kGammaK64 * kC3_64 * iH4 * (3.0 * w + q * dw));
        }
        s[0] += g * rx * ir;
        s[1] += g * ry * ir;
        s[2] += g * rz * ir;
    }
}

// particle k's sums into the outputs of its kind
template <int KIND>
__device__ __forceinline__ void adj_finish(const AdjArgs &a, const AdjIO &io, int64_t k, const double *s)
{
    if constexpr (KIND == 0) {  // rho, rho_dh into the workspace and, when given, o0, o1
        const double H = kGammaK64 * (double)a.hm[k].x;
        const double C = kC3_64 / (H * H * H);
        const double r0 = C * s[0], r1 = -kGammaK64 * C / H * s[1];
        a.rho64[2 * k] = r0;
        a.rho64[2 * k + 1] = r1;
        if (io.o0) {
            io.o0[k] = r0;
            io.o1[k] = r1;
        }
    } else if constexpr (KIND == 1) {  // a (o0), u_dt (o1)
        io.o0[3 * k] = s[0];
        io.o0[3 * k + 1] = s[1];
        io.o0[3 * k + 2] = s[2];
        io.o1[k] = s[3];
    } else if constexpr (KIND == 2) {  // x_bar, v_bar, m_bar, rho_bar, rhodh_bar (written)
        io.o0[3 * k] = s[0];
        io.o0[3 * k + 1] = s[1];
        io.o0[3 * k + 2] = s[2];
        io.o1[3 * k] = s[3];
        io.o1[3 * k + 1] = s[4];
        io.o1[3 * k + 2] = s[5];
        io.o2[k] = s[6];
        io.o3[k] = s[7];
        io.o4[k] = s[8];
    } else {  // x_bar (o0), m_bar (o1), accumulated
        io.o0[3 * k] += s[0];
        io.o0[3 * k + 1] += s[1];
        io.o0[3 * k + 2] += s[2];
        io.o1[k] += s[3];
    }
}

// wave-scope ordering of LDS traffic between lanes of one wave
__device__ __forceinline__ void adj_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a value every lane holds, moved to scalar registers
__device__ __forceinline__ double uniform64(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double wave_min64(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return uniform64(v);
}

__device__ __forceinline__ double wave_max64(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return uniform64(v);
}

// test the nc staged candidates against every lane's particle (one bit per
// candidate), then let each lane walk its own hits, lowest first
template <int KIND>
__device__ __forceinline__ void adj_flush(const AdjArgs &a, const IAdj &I, int64_t k, bool valid,
                                          const double2 (*L)[AdjKind<KIND>::NF / 2], int nc, double *s)
{
    using K = AdjKind<KIND>;
    constexpr int NW = K::WIN / 64;
    adj_wave_sync();
    uint64_t m[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        m[w] = 0;
        const int n = nc - 64 * w < 64 ? nc - 64 * w : 64;
#pragma unroll 2
        for (int c = 0; c < n; ++c) {
            double rx, ry, rz;
            const double r2 = adj_r2(I, L[64 * w + c], rx, ry, rz);
            bool hit;
            if constexpr (K::MIXED) {
                const double Hj = L[64 * w + c][1].y;
                const double Hm = I.H > Hj ? I.H : Hj;
                hit = r2 < Hm * Hm;
            } else {
                hit = r2 < I.H2;
            }
            m[w] |= (uint64_t)hit << c;
        }
        if (!valid) m[w] = 0;
    }
    uint64_t cur = m[0];
    int base = 0;
    for (;;) {
        if constexpr (NW == 2) {
            if (cur == 0 && base == 0) {
                cur = m[1];
                base = 64;
            }
        }
        const bool act = cur != 0;
        if (__ballot(act) == 0) break;
        if (act) {
            const int c = __builtin_ctzll(cur);
            cur &= cur - 1;
            adj_pair<KIND>(a, I, k, L[base + c], s);
            if (cur != 0) {  // a second hit of the same word shares the trip
                const int c2 = __builtin_ctzll(cur);
                cur &= cur - 1;
                adj_pair<KIND>(a, I, k, L[base + c2], s);
            }
        }
    }
    adj_wave_sync();
}

// One wave per (tile, share of the cell's neighbour entries).  All 64 lanes
// stay active to the end (ballots and shuffles); lanes beyond the tile hold a
// copy of its first particle and record no hits.
template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(AdjKind<KIND>::WAVES))) void k_adj_pairs(
    AdjArgs a, AdjIO io)
{
    using K = AdjKind<KIND>;
    constexpr int NF2 = K::NF / 2;
    __shared__ double2 L[K::WIN][NF2];
    const int lane = threadIdx.x;
    const int S = io.split;
    const int b = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
    const int t = b / S, g = b - t * S;
    const Chunk tl = a.tiles[t];
    const bool valid = lane < tl.n;
    const int64_t k = tl.part0 + (valid ? lane : 0);
    IAdj I;
    adj_load_i<KIND>(a, io, k, I);
    // the tile's box and largest support
    const double inf = __builtin_huge_val();
    const double lox = wave_min64(valid ? I.x : inf), hix = wave_max64(valid ? I.x : -inf);
    const double loy = wave_min64(valid ? I.y : inf), hiy = wave_max64(valid ? I.y : -inf);
    const double loz = wave_min64(valid ? I.z : inf), hiz = wave_max64(valid ? I.z : -inf);
    const double Hmax = wave_max64(valid ? I.H : 0.0);
    const int cell = tl.cell;
    const double clx = a.cells[cell].loc[0], cly = a.cells[cell].loc[1], clz = a.cells[cell].loc[2];
    const int e0 = a.nbr_off[cell], ne = a.nbr_off[cell + 1] - e0;
    const int eb = e0 + (int)((int64_t)g * ne / S), ee = e0 + (int)((int64_t)(g + 1) * ne / S);
    double s[K::NACC];
#pragma unroll
    for (int v = 0; v < K::NACC; ++v) s[v] = 0.0;
    int nc = 0;
    for (int e = eb; e < ee; ++e) {
        const Nbr nb = a.nbr[e];
        const sph_cell &cj = a.cells[nb.cell];
        const CellRange cr = a.cellr[nb.cell];
        // translation = loc(cj) + shift - loc(ck)
        const double sx = ((double)nb.dx - cj.loc[0]) + clx;
        const double sy = ((double)nb.dy - cj.loc[1]) + cly;
        const double sz = ((double)nb.dz - cj.loc[2]) + clz;
        for (int q0 = 0; q0 < cr.count; q0 += 64) {
            const bool inb = q0 + lane < cr.count;
            const int64_t j = cr.first + q0 + (inb ? lane : 0);
            const double xj = io.x[3 * j] + sx, yj = io.x[3 * j + 1] + sy, zj = io.x[3 * j + 2] + sz;
            const double Hj = kGammaK64 * (double)a.hm[j].x;
            // distance to the tile's box; the margin keeps every candidate
            // some lane's support test could accept
            const double bx = fmax(fmax(lox - xj, xj - hix), 0.0);
            const double by = fmax(fmax(loy - yj, yj - hiy), 0.0);
            const double bz = fmax(fmax(loz - zj, zj - hiz), 0.0);
            const double R = K::MIXED ? fmax(Hmax, Hj) : Hmax;
            const bool keep = inb && bx * bx + by * by + bz * bz < R * R * (1.0 + 1e-9);
            const uint64_t bal = __ballot(keep);
            const int cnt = __popcll(bal);
            if (cnt == 0) continue;
            if (nc + cnt > K::WIN) {
                adj_flush<KIND>(a, I, k, valid, L, nc, s);
                nc = 0;
            }
            if (keep) adj_stage<KIND>(a, io, j, xj, yj, zj, Hj, L[nc + __popcll(bal & ((1ull << lane) - 1ull))]);
            nc += cnt;
        }
    }
    if (nc > 0) adj_flush<KIND>(a, I, k, valid, L, nc, s);
    if (!valid) return;
    if (S == 1) {
        adj_finish<KIND>(a, io, k, s);
    } else {
#pragma unroll
        for (int v = 0; v < K::NACC; ++v) io.part[((int64_t)g * K::NACC + v) * a.P + k] = s[v];
    }
}

// the shares' partial sums of every particle, added in share order
template <int KIND>
__global__ __launch_bounds__(256) void k_adj_combine(AdjArgs a, AdjIO io)
{
    using K = AdjKind<KIND>;
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double s[K::NACC];
#pragma unroll
    for (int v = 0; v < K::NACC; ++v) s[v] = io.part[v * a.P + k];
    for (int g = 1; g < io.split; ++g) {
#pragma unroll
        for (int v = 0; v < K::NACC; ++v) s[v] += io.part[((int64_t)g * K::NACC + v) * a.P + k];
    }
    adj_finish<KIND>(a, io, k, s);
}

__global__ void k_adj_prep(AdjArgs a, const float *v, const float *m, const float *h, const float *u,
                           const float *at, const float *ad)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    a.hm[k] = make_float2(h[k], m[k]);
    a.v[k] = make_float4(v[3 * k], v[3 * k + 1], v[3 * k + 2], 0.f);
    a.ua[k] = make_float4(u[k], at[k], ad[k], 0.f);
}

// h and m only (the density adjoint reads nothing else)
__global__ void k_adj_prep_hm(AdjArgs a, const float *m, const float *h)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    a.hm[k] = make_float2(h[k], m[k]);
}

// waves per tile: enough shares of the neighbour entries that the launch
// holds about sixteen waves per compute unit
static int adj_split(const sph_plan *p)
{
    if (p->ntile <= 0) return 1;
    const int64_t s = (int64_t)16 * p->num_cu / p->ntile;
    return (int)(s < 1 ? 1 : s > kAdjMaxSplit ? kAdjMaxSplit : s);
}

static size_t adj_ws_bytes(const sph_plan *p)
{
    const int64_t P = round_slots(p->n);
    const int S = adj_split(p);
    return (size_t)P * 64 + (S > 1 ? (size_t)P * S * kAdjMaxAcc * sizeof(double) : 0);
}

static sph_status adj_setup(const sph_plan *p, void *ws, size_t ws_bytes, AdjArgs &a, AdjIO &io)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    if (!p->batched_ok) return fail(SPH_E_UNSUPPORTED, "cells do not tile the store in order");
    const size_t need = adj_ws_bytes(p);
    if (!ws || ((uintptr_t)ws & 255u)) return fail(SPH_E_ARG, "workspace null or misaligned");
    if (ws_bytes < need) return fail(SPH_E_CAPACITY, "adjoint workspace needs " + std::to_string(need) + " bytes");
    a.n = p->n;
    a.P = round_slots(p->n);
    a.tiles = p->d_tiles;
    a.ntile = p->ntile;
    a.cellr = p->d_cellr;
    a.nbr = p->d_nbr;
    a.nbr_off = p->d_nbr_off;
    a.cells = p->d_cells;
    a.v = (float4 *)ws;
    a.ua = a.v + a.P;
    a.rho64 = (double *)(a.ua + a.P);
    a.hm = (float2 *)(a.rho64 + 2 * a.P);
    io = AdjIO{};
    io.split = adj_split(p);
    io.part = (double *)((char *)ws + (size_t)a.P * 64);
    return SPH_OK;
}

template <int KIND>
static void adj_launch(const AdjArgs &a, const AdjIO &io, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_pairs<KIND>, dim3((unsigned)((int64_t)a.ntile * io.split)), dim3(64), 0, st, a, io);
    if (io.split > 1)
        hipLaunchKernelGGL(k_adj_combine<KIND>, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a, io);
}

static dim3 adj_flat(const AdjArgs &a) { return dim3((unsigned)((a.n + 255) / 256)); }

}  // namespace sph

using namespace sph;

extern "C" {

sph_status sph_adjoint_ws_bytes(const sph_plan *p, size_t *bytes)
{
    if (!p || !bytes) return fail(SPH_E_ARG, "null argument");
    *bytes = adj_ws_bytes(p);
    return SPH_OK;
}

sph_status sph_adjoint_forward(const sph_plan *p, const double *x, const float *v, const float *m, const float *h,
                               const float *u, const float *atilde, const float *alpha_d, const sph_params *prm,
                               double *rho, double *rho_dh, double *acc, double *u_dt, void *ws, size_t ws_bytes,
                               void *stream)
{
    AdjArgs a{};
    AdjIO io{};
    sph_status s = adj_setup(p, ws, ws_bytes, a, io);
    if (s) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (p->n == 0) return SPH_OK;
    if (!x || !v || !m || !h || !u || !atilde || !alpha_d || !rho || !rho_dh || !acc || !u_dt)
        return fail(SPH_E_ARG, "null array");
    a.gam = prm->gamma_ad;
    a.beta = prm->beta_visc;
    hipStream_t st = (hipStream_t)stream;
    io.x = x;
    hipLaunchKernelGGL(k_adj_prep, adj_flat(a), dim3(256), 0, st, a, v, m, h, u, atilde, alpha_d);
    io.o0 = rho;
    io.o1 = rho_dh;
    adj_launch<0>(a, io, st);
    io.o0 = acc;
    io.o1 = u_dt;
    adj_launch<1>(a, io, st);
    SPH_CHECK_LAUNCH("adjoint forward launch");
    return SPH_OK;
}

sph_status sph_force_adjoint(const sph_plan *p, const double *x, const float *v, const float *m, const float *h,
                             const float *u, const float *atilde, const float *alpha_d, const sph_params *prm,
                             const double *a_bar, double *x_bar, double *v_bar, double *m_bar, double *rho_bar,
                             double *rhodh_bar, void *ws, size_t ws_bytes, void *stream)
{
    AdjArgs a{};
    AdjIO io{};
    sph_status s = adj_setup(p, ws, ws_bytes, a, io);
    if (s) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (p->n == 0) return SPH_OK;
    if (!x || !v || !m || !h || !u || !atilde || !alpha_d || !a_bar || !x_bar || !v_bar || !m_bar || !rho_bar ||
        !rhodh_bar)
        return fail(SPH_E_ARG, "null array");
    a.gam = prm->gamma_ad;
    a.beta = prm->beta_visc;
    hipStream_t st = (hipStream_t)stream;
    io.x = x;
    hipLaunchKernelGGL(k_adj_prep, adj_flat(a), dim3(256), 0, st, a, v, m, h, u, atilde, alpha_d);
    // density of the current positions, recomputed rather than kept from the forward pass
    adj_launch<0>(a, io, st);
    io.abar = a_bar;
    io.o0 = x_bar;
    io.o1 = v_bar;
    io.o2 = m_bar;
    io.o3 = rho_bar;
    io.o4 = rhodh_bar;
    adj_launch<2>(a, io, st);
    SPH_CHECK_LAUNCH("force adjoint launch");
    return SPH_OK;
}

sph_status sph_density_adjoint(const sph_plan *p, const double *x, const float *m, const float *h,
                               const double *rho_bar, const double *rhodh_bar, double *x_bar, double *m_bar,
                               void *ws, size_t ws_bytes, void *stream)
{
    AdjArgs a{};
    AdjIO io{};
    sph_status s = adj_setup(p, ws, ws_bytes, a, io);
    if (s) return s;
    if (p->n == 0) return SPH_OK;
    if (!x || !m || !h || !rho_bar || !rhodh_bar || !x_bar || !m_bar) return fail(SPH_E_ARG, "null array");
    hipStream_t st = (hipStream_t)stream;
    io.x = x;
    io.rbar = rho_bar;
    io.dbar = rhodh_bar;
    io.o0 = x_bar;
    io.o1 = m_bar;
    hipLaunchKernelGGL(k_adj_prep_hm, adj_flat(a), dim3(256), 0, st, a, m, h);
    adj_launch<3>(a, io, st);
    SPH_CHECK_LAUNCH("density adjoint launch");
    return SPH_OK;
}
}
