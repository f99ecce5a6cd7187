// Hand-written adjoint of L = sum_i |a_i|^2 through the density and force
// loops (the differentiable form of the interaction loops of Sec. 2.1).
//
// Inputs are per-particle arrays in store order; the artificial-viscosity
// switch alpha~ and alpha_d, h and u are constants.  The backward pass never
// stores pair terms: it re-evaluates them.
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
// Mapping: one thread per particle k, walking the particles of its cell's
// neighbour cells (the plan's cell tasks).  The forward pass that produces
// rho, rho_dh and a evaluates in FP64 from the float64 positions: a is a sum
// of pair terms that nearly cancel on a near-uniform particle set, and every
// gradient is proportional to abar = dL/da = 2a, so FP32 rounding of a (up to a
// few 1e-3 of |a| for such particles) would set the accuracy of the whole
// gradient.  MI355X runs FP64 vector arithmetic at the rate of unpacked FP32.
// The hand-written backward kernels run in FP32 on positions packed once to
// float32 offsets from each particle's own cell corner.
#include <hip/hip_runtime.h>

#include "sph_internal.hpp"

namespace sph {

struct AdjArgs {
    int64_t n;
    const Chunk *tiles;
    int32_t ntile;
    const CellRange *cellr;
    const Nbr *nbr;
    const int32_t *nbr_off;
    const sph_cell *cells;
    // packed per particle (workspace)
    float4 *pos;  // dx dy dz (cell frame) h
    float4 *vm;   // vx vy vz m
    float4 *ua;      // u alpha~ alpha_d (unused)
    double *rho64;   // forward rho, rho_dh in float64
    float gam, beta;
};

__device__ __forceinline__ void spl(float q, float &w, float &dw, float &d2w)
{
    const float t = fmaxf(1.0f - q, 0.0f);
    if (q < 0.5f) {
        w = 1.0f - 6.0f * q * q + 6.0f * q * q * q;
        dw = -12.0f * q + 18.0f * q * q;
        d2w = -12.0f + 36.0f * q;
    } else {
        w = 2.0f * t * t * t;
        dw = -6.0f * t * t;
        d2w = 12.0f * t;
    }
}

// F = (1/r) dW/dr = C3 H^-5 w'(q)/q and dF/dr = C3 H^-6 (q w'' - w')/q^2, both 0 beyond H
__device__ __forceinline__ void kern_F(float r, float H, float &F, float &Fp)
{
    if (!(r < H)) {
        F = 0.f;
        Fp = 0.f;
        return;
    }
    const float iH = 1.0f / H, q = r * iH;
    const float K5 = kC3 * iH * iH * iH * iH * iH;
    if (q < 0.5f) {
        F = K5 * (-12.0f + 18.0f * q);
        Fp = K5 * iH * 18.0f;
    } else {
        const float t = 1.0f - q;
        F = K5 * (-6.0f * t * t / q);
        Fp = K5 * iH * 6.0f * t * (1.0f + q) / (q * q);
    }
}

// FP64 pieces of the forward pass
__device__ __forceinline__ void spl64(double q, double &w, double &dw)
{
    if (q < 0.5) {
        w = 1.0 - 6.0 * q * q + 6.0 * q * q * q;
        dw = -12.0 * q + 18.0 * q * q;
    } else {
        const double t = q < 1.0 ? 1.0 - q : 0.0;
        w = 2.0 * t * t * t;
        dw = -6.0 * t * t;
    }
}

__device__ __forceinline__ double kern_F64(double r, double H)
{
    if (!(r < H)) return 0.0;
    const double q = r / H, H2 = H * H;
    const double K5 = (8.0 / 3.14159265358979323846) / (H2 * H2 * H);
    if (q < 0.5) return K5 * (-12.0 + 18.0 * q);
    const double t = 1.0 - q;
    return K5 * (-6.0 * t * t / q);
}

// walk every neighbour-cell particle j of particle k with float64 separations
// x_k - x_j + shift, the shift recovered from the entry's translation
template <class Fn>
__device__ __forceinline__ void for_neighbours64(const AdjArgs &a, int32_t cell, int64_t k, const double *x, Fn &&fn)
{
    const double xk = x[3 * k], yk = x[3 * k + 1], zk = x[3 * k + 2];
    const sph_cell &ck = a.cells[cell];
    const int e0 = a.nbr_off[cell], e1 = a.nbr_off[cell + 1];
    for (int e = e0; e < e1; ++e) {
        const Nbr nb = a.nbr[e];
        const sph_cell &cj = a.cells[nb.cell];
        const CellRange cr = a.cellr[nb.cell];
        // translation = loc(cj) + shift - loc(ck)
        const double sx = ((double)nb.dx - cj.loc[0]) + ck.loc[0];
        const double sy = ((double)nb.dy - cj.loc[1]) + ck.loc[1];
        const double sz = ((double)nb.dz - cj.loc[2]) + ck.loc[2];
        for (int q = 0; q < cr.count; ++q) {
            const int64_t j = cr.first + q;
            fn(j, xk - (x[3 * j] + sx), yk - (x[3 * j + 1] + sy), zk - (x[3 * j + 2] + sz));
        }
    }
}

// walk every neighbour-cell particle j of particle k; fn(j, rx, ry, rz)
template <class Fn>
__device__ __forceinline__ void for_neighbours(const AdjArgs &a, int32_t cell, float4 pk, Fn &&fn)
{
    const int e0 = a.nbr_off[cell], e1 = a.nbr_off[cell + 1];
    for (int e = e0; e < e1; ++e) {
        const Nbr nb = a.nbr[e];
        const CellRange cr = a.cellr[nb.cell];
        for (int q = 0; q < cr.count; ++q) {
            const int64_t j = cr.first + q;
            const float4 pj = a.pos[j];
            const float rx = pk.x - (pj.x + nb.dx), ry = pk.y - (pj.y + nb.dy), rz = pk.z - (pj.z + nb.dz);
            fn(j, rx, ry, rz);
        }
    }
}

// one thread per tile lane: particle index and its cell
__device__ __forceinline__ bool my_particle(const AdjArgs &a, int64_t &k, int32_t &cell)
{
    const int64_t t = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= a.ntile) return false;
    const Chunk tl = a.tiles[t];
    const int lane = threadIdx.x & 63;
    if (lane >= tl.n) return false;
    k = tl.part0 + lane;
    cell = tl.cell;
    return true;
}

__global__ void k_adj_prep(AdjArgs a, const double *x, const float *v, const float *m, const float *h,
                           const float *u, const float *at, const float *ad)
{
    int64_t k;
    int32_t c;
    if (!my_particle(a, k, c)) return;
    const sph_cell &cl = a.cells[c];
    a.pos[k] = make_float4((float)(x[3 * k] - cl.loc[0]), (float)(x[3 * k + 1] - cl.loc[1]),
                           (float)(x[3 * k + 2] - cl.loc[2]), h[k]);
    a.vm[k] = make_float4(v[3 * k], v[3 * k + 1], v[3 * k + 2], m[k]);
    a.ua[k] = make_float4(u[k], at[k], ad[k], 0.f);
}

// positions and masses only (the density adjoint reads nothing else)
__global__ void k_adj_prep_xm(AdjArgs a, const double *x, const float *m, const float *h)
{
    int64_t k;
    int32_t c;
    if (!my_particle(a, k, c)) return;
    const sph_cell &cl = a.cells[c];
    a.pos[k] = make_float4((float)(x[3 * k] - cl.loc[0]), (float)(x[3 * k + 1] - cl.loc[1]),
                           (float)(x[3 * k + 2] - cl.loc[2]), h[k]);
    a.vm[k] = make_float4(0.f, 0.f, 0.f, m[k]);
}

__global__ void k_adj_density(AdjArgs a, const double *x, float *rho, float *rho_dh, double *rho64)
{
    int64_t k;
    int32_t c;
    if (!my_particle(a, k, c)) return;
    const double H = 1.8257418583505537 * (double)a.pos[k].w, H2 = H * H;
    double s0 = 0.0, s1 = 0.0;
    for_neighbours64(a, c, k, x, [&](int64_t j, double rx, double ry, double rz) {
        const double r2 = rx * rx + ry * ry + rz * rz;
        if (!(r2 < H2)) return;
        const double q = sqrt(r2) / H;
        double w, dw;
        spl64(q, w, dw);
        const double mj = a.vm[j].w;
        s0 += mj * w;
        s1 += mj * (3.0 * w + q * dw);
    });
    const double C = (8.0 / 3.14159265358979323846) / (H2 * H);
    const double r0 = C * s0, r1 = -1.8257418583505537 * C / H * s1;
    rho[k] = (float)r0;
    rho_dh[k] = (float)r1;
    rho64[2 * k] = r0;
    rho64[2 * k + 1] = r1;
}

struct PairQ {  // per-particle quantities of the force loop
    float H, A, c, rho, u, at, ad, om;  // om = rho + h rho_dh / 3
};

__device__ __forceinline__ PairQ pq(const AdjArgs &a, int64_t k, const float *rho, const float *rho_dh)
{
    PairQ p;
    const float h = a.pos[k].w;
    const float4 ua = a.ua[k];
    p.H = kGammaK * h;
    p.rho = rho[k];
    p.om = p.rho + h * rho_dh[k] * (1.0f / 3.0f);
    p.u = ua.x;
    p.A = (a.gam - 1.0f) * p.u / p.om;
    p.c = sqrtf(a.gam * (a.gam - 1.0f) * p.u);
    p.at = ua.y;
    p.ad = ua.z;
    return p;
}

__global__ void k_adj_force(AdjArgs a, const double *x, const double *rho64, float *acc, float *udt)
{
    int64_t k;
    int32_t c;
    if (!my_particle(a, k, c)) return;
    const double g = a.gam, beta = a.beta;
    auto q64 = [&](int64_t i, double &H, double &A, double &cs, double &rh, double &u, double &at, double &ad) {
        const double h = a.pos[i].w;
        const float4 ua = a.ua[i];
        H = 1.8257418583505537 * h;
        rh = rho64[2 * i];
        u = ua.x;
        A = (g - 1.0) * u / (rh + h * rho64[2 * i + 1] / 3.0);
        cs = sqrt(g * (g - 1.0) * u);
        at = ua.y;
        ad = ua.z;
    };
    double Hk, Ak, ck, rk, uk, atk, adk;
    q64(k, Hk, Ak, ck, rk, uk, atk, adk);
    const float4 vk = a.vm[k];
    double ax = 0.0, ay = 0.0, az = 0.0, du = 0.0;
    for_neighbours64(a, c, k, x, [&](int64_t j, double rx, double ry, double rz) {
        if (j == k) return;
        const double Hj0 = 1.8257418583505537 * (double)a.pos[j].w;
        const double r2 = rx * rx + ry * ry + rz * rz;
        const double Hm = Hk > Hj0 ? Hk : Hj0;
        if (!(r2 < Hm * Hm)) return;
        double Hj, Aj, cj, rj, uj, atj, adj;
        q64(j, Hj, Aj, cj, rj, uj, atj, adj);
        const float4 vj = a.vm[j];
        const double r = sqrt(r2);
        const double Fk = kern_F64(r, Hk), Fj = kern_F64(r, Hj), Fb = 0.5 * (Fk + Fj);
        const double vx = (double)vk.x - vj.x, vy = (double)vk.y - vj.y, vz = (double)vk.z - vj.z;
        const double dot = vx * rx + vy * ry + vz * rz;
        const double mu = (r > 0.0 && dot < 0.0) ? dot / r : 0.0;
        const double rb = 0.5 * (rk + rj);
        const double Pi = -0.5 * 0.5 * (atk + atj) * (ck + cj - beta * mu) * mu / rb;
        const double S = Ak * Fk + Aj * Fj + Pi * Fb;
        const double mj = vj.w;
        ax -= mj * S * rx;
        ay -= mj * S * ry;
        az -= mj * S * rz;
        du += mj * (Ak * Fk * dot + 0.5 * Pi * Fb * dot + 0.5 * (adk + adj) * fabs(dot) * (uk - uj) * Fb / rb);
    });
    acc[3 * k] = (float)ax;
    acc[3 * k + 1] = (float)ay;
    acc[3 * k + 2] = (float)az;
    udt[k] = (float)du;
}

__global__ void k_force_adjoint(AdjArgs a, const float *rho, const float *rho_dh, const float *abar, float *xbar,
                                float *vbar, float *mbar, float *rhobar, float *rhodhbar)
{
    int64_t k;
    int32_t c;
    if (!my_particle(a, k, c)) return;
    const float4 pk = a.pos[k];
    const float4 vk = a.vm[k];
    const PairQ P = pq(a, k, rho, rho_dh);
    const float abx = abar[3 * k], aby = abar[3 * k + 1], abz = abar[3 * k + 2];
    const float hk = pk.w;
    float gx = 0.f, gy = 0.f, gz = 0.f, hx = 0.f, hy = 0.f, hz = 0.f, gm = 0.f, grho = 0.f, gdh = 0.f;
    for_neighbours(a, c, pk, [&](int64_t j, float rx, float ry, float rz) {
        if (j == k) return;
        const float Hj = kGammaK * a.pos[j].w;
        const float r2 = rx * rx + ry * ry + rz * rz;
        const float Hm = fmaxf(P.H, Hj);
        if (!(r2 < Hm * Hm)) return;
        const PairQ Q = pq(a, j, rho, rho_dh);
        const float4 vj = a.vm[j];
        const float mk = vk.w, mj = vj.w;
        const float r = sqrtf(r2);
        const float ir = r > 0.f ? 1.0f / r : 0.f;
        const float ex = rx * ir, ey = ry * ir, ez = rz * ir;
        float Fk, Fkp, Fj, Fjp;
        kern_F(r, P.H, Fk, Fkp);
        kern_F(r, Q.H, Fj, Fjp);
        const float Fb = 0.5f * (Fk + Fj), Fbp = 0.5f * (Fkp + Fjp);
        const float vx = vk.x - vj.x, vy = vk.y - vj.y, vz = vk.z - vj.z;
        const float dot = vx * rx + vy * ry + vz * rz;
        const bool appr = r > 0.f && dot < 0.f;
        const float mu = appr ? dot * ir : 0.f;
        const float rb = 0.5f * (P.rho + Q.rho);
        const float al = 0.5f * (P.at + Q.at);
        const float vs = P.c + Q.c - a.beta * mu;
        const float Pi = -0.5f * al * vs * mu / rb;
        const float dPi = -0.5f * (al / rb) * (P.c + Q.c - 2.0f * a.beta * mu);  // dPi/dmu
        const float S = P.A * Fk + Q.A * Fj + Pi * Fb;
        const float4 abj4 = make_float4(abar[3 * j], abar[3 * j + 1], abar[3 * j + 2], 0.f);
        const float wx = mk * abj4.x - mj * abx, wy = mk * abj4.y - mj * aby, wz = mk * abj4.z - mj * abz;
        const float rw = rx * wx + ry * wy + rz * wz;
        // grad_r S = (A_k F_k' + A_j F_j' + Pi Fbar') rhat + Fbar dPi/dmu grad_r mu
        const float sr = P.A * Fkp + Q.A * Fjp + Pi * Fbp;
        float mx = 0.f, my = 0.f, mz = 0.f;  // grad_r mu
        if (appr) {
            mx = (vx - mu * ex) * ir;
            my = (vy - mu * ey) * ir;
            mz = (vz - mu * ez) * ir;
        }
        const float cP = Fb * dPi;
        gx += S * wx + rw * (sr * ex + cP * mx);
        gy += S * wy + rw * (sr * ey + cP * my);
        gz += S * wz + rw * (sr * ez + cP * mz);
        if (appr) {  // grad_v mu = rhat
            hx += rw * cP * ex;
            hy += rw * cP * ey;
            hz += rw * cP * ez;
        }
        gm += S * (rx * abj4.x + ry * abj4.y + rz * abj4.z);
        const float dA_drho = -P.A / P.om;
        const float dA_ddh = -P.A * (hk * (1.0f / 3.0f)) / P.om;
        grho += rw * (Fk * dA_drho - Fb * Pi / (2.0f * rb));
        gdh += rw * Fk * dA_ddh;
    });
    xbar[3 * k] = gx;
    xbar[3 * k + 1] = gy;
    xbar[3 * k + 2] = gz;
    vbar[3 * k] = hx;
    vbar[3 * k + 1] = hy;
    vbar[3 * k + 2] = hz;
    mbar[k] = gm;
    rhobar[k] = grho;
    rhodhbar[k] = gdh;
}

__global__ void k_density_adjoint(AdjArgs a, const float *rhobar, const float *rhodhbar, float *xbar, float *mbar)
{
    int64_t k;
    int32_t c;
    if (!my_particle(a, k, c)) return;
    const float4 pk = a.pos[k];
    const float Hk = kGammaK * pk.w;
    const float mk = a.vm[k].w;
    const float rbk = rhobar[k], dbk = rhodhbar[k];
    float gx = 0.f, gy = 0.f, gz = 0.f, gm = 0.f;
    for_neighbours(a, c, pk, [&](int64_t j, float rx, float ry, float rz) {
        const float Hj = kGammaK * a.pos[j].w;
        const float r2 = rx * rx + ry * ry + rz * rz;
        const float Hm = fmaxf(Hk, Hj);
        if (!(r2 < Hm * Hm)) return;
        const float r = sqrtf(r2);
        const float ir = r > 0.f ? 1.0f / r : 0.f;
        const float mj = a.vm[j].w;
        float g = 0.f;  // radial derivative collected over both directions
        if (r < Hk) {  // rho_k's term m_j W(r, h_k)
            const float iH = 1.0f / Hk, q = r * iH;
            float w, dw, d2w;
            spl(q, w, dw, d2w);
            const float iH4 = iH * iH * iH * iH;
            const float Wr = kC3 * iH4 * dw;                                   // dW/dr
            const float Whr = -kGammaK * kC3 * iH4 * iH * (4.0f * dw + q * d2w);  // d(dW/dh)/dr
            g += mj * (rbk * Wr + dbk * Whr);
        }
        if (r < Hj) {  // rho_j's term m_k W(r, h_j)
            const float iH = 1.0f / Hj, q = r * iH;
            float w, dw, d2w;
            spl(q, w, dw, d2w);
            const float iH3 = iH * iH * iH, iH4 = iH3 * iH;
            const float rbj = rhobar[j], dbj = rhodhbar[j];
            g += mk * (rbj * kC3 * iH4 * dw + dbj * (-kGammaK * kC3 * iH4 * iH * (4.0f * dw + q * d2w)));
            gm += rbj * kC3 * iH3 * w + dbj * (-kGammaK * kC3 * iH4 * (3.0f * w + q * dw));
        }
        gx += g * rx * ir;
        gy += g * ry * ir;
        gz += g * rz * ir;
    });
    xbar[3 * k] += gx;
    xbar[3 * k + 1] += gy;
    xbar[3 * k + 2] += gz;
    mbar[k] += gm;
}

static sph_status adj_setup(const sph_plan *p, void *ws, size_t ws_bytes, AdjArgs &a)
{
    if (!p) return fail(SPH_E_ARG, "plan is null");
    if (!p->batched_ok) return fail(SPH_E_UNSUPPORTED, "cells do not tile the store in order");
    const size_t need = (size_t)round_slots(p->n) * 64;
    if (!ws || ((uintptr_t)ws & 255u)) return fail(SPH_E_ARG, "workspace null or misaligned");
    if (ws_bytes < need) return fail(SPH_E_CAPACITY, "adjoint workspace needs " + std::to_string(need) + " bytes");
    a.n = p->n;
    a.tiles = p->d_tiles;
    a.ntile = p->ntile;
    a.cellr = p->d_cellr;
    a.nbr = p->d_nbr;
    a.nbr_off = p->d_nbr_off;
    a.cells = p->d_cells;
    const int64_t P = round_slots(p->n);
    a.pos = (float4 *)ws;
    a.vm = a.pos + P;
    a.ua = a.vm + P;
    a.rho64 = (double *)(a.ua + P);
    return SPH_OK;
}

static dim3 adj_grid(const AdjArgs &a) { return dim3((unsigned)((a.ntile + 3) / 4)); }

}  // namespace sph

using namespace sph;

extern "C" {

sph_status sph_adjoint_ws_bytes(const sph_plan *p, size_t *bytes)
{
    if (!p || !bytes) return fail(SPH_E_ARG, "null argument");
    *bytes = (size_t)round_slots(p->n) * 64;
    return SPH_OK;
}

sph_status sph_adjoint_forward(const sph_plan *p, const double *x, const float *v, const float *m, const float *h,
                               const float *u, const float *atilde, const float *alpha_d, const sph_params *prm,
                               float *rho, float *rho_dh, float *acc, float *u_dt, void *ws, size_t ws_bytes,
                               void *stream)
{
    AdjArgs a{};
    sph_status s = adj_setup(p, ws, ws_bytes, a);
    if (s) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (p->n == 0) return SPH_OK;
    if (!x || !v || !m || !h || !u || !atilde || !alpha_d || !rho || !rho_dh || !acc || !u_dt)
        return fail(SPH_E_ARG, "null array");
    a.gam = prm->gamma_ad;
    a.beta = prm->beta_visc;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_adj_prep, adj_grid(a), dim3(256), 0, st, a, x, v, m, h, u, atilde, alpha_d);
    hipLaunchKernelGGL(k_adj_density, adj_grid(a), dim3(256), 0, st, a, x, rho, rho_dh, a.rho64);
    hipLaunchKernelGGL(k_adj_force, adj_grid(a), dim3(256), 0, st, a, x, (const double *)a.rho64, acc, u_dt);
    SPH_CHECK_LAUNCH("adjoint forward launch");
    return SPH_OK;
}

sph_status sph_force_adjoint(const sph_plan *p, const double *x, const float *v, const float *m, const float *h,
                             const float *u, const float *atilde, const float *alpha_d, const float *rho,
                             const float *rho_dh, const sph_params *prm, const float *a_bar, float *x_bar,
                             float *v_bar, float *m_bar, float *rho_bar, float *rhodh_bar, void *ws,
                             size_t ws_bytes, void *stream)
{
    AdjArgs a{};
    sph_status s = adj_setup(p, ws, ws_bytes, a);
    if (s) return s;
    if (!prm) return fail(SPH_E_ARG, "params is null");
    if (p->n == 0) return SPH_OK;
    if (!x || !v || !m || !h || !u || !atilde || !alpha_d || !rho || !rho_dh || !a_bar || !x_bar || !v_bar ||
        !m_bar || !rho_bar || !rhodh_bar)
        return fail(SPH_E_ARG, "null array");
    a.gam = prm->gamma_ad;
    a.beta = prm->beta_visc;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_adj_prep, adj_grid(a), dim3(256), 0, st, a, x, v, m, h, u, atilde, alpha_d);
    hipLaunchKernelGGL(k_force_adjoint, adj_grid(a), dim3(256), 0, st, a, rho, rho_dh, a_bar, x_bar, v_bar, m_bar,
                       rho_bar, rhodh_bar);
    SPH_CHECK_LAUNCH("force adjoint launch");
    return SPH_OK;
}

sph_status sph_density_adjoint(const sph_plan *p, const double *x, const float *m, const float *h,
                               const float *rho_bar, const float *rhodh_bar, float *x_bar, float *m_bar, void *ws,
                               size_t ws_bytes, void *stream)
{
    AdjArgs a{};
    sph_status s = adj_setup(p, ws, ws_bytes, a);
    if (s) return s;
    if (p->n == 0) return SPH_OK;
    if (!x || !m || !h || !rho_bar || !rhodh_bar || !x_bar || !m_bar) return fail(SPH_E_ARG, "null array");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_adj_prep_xm, adj_grid(a), dim3(256), 0, st, a, x, m, h);
    hipLaunchKernelGGL(k_density_adjoint, adj_grid(a), dim3(256), 0, st, a, rho_bar, rhodh_bar, x_bar, m_bar);
    SPH_CHECK_LAUNCH("density adjoint launch");
    return SPH_OK;
}
}
