/*
 * CPU oracle for the SPH pack / interact / unpack path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke entry and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * Everything here is the plain definition, evaluated slowly and obviously:
 *   - interaction loops are O(N^2) brute force over all particles with the
 *     minimum-image convention in the periodic unit box, in FP64; an optional
 *     uniform grid only skips particles beyond a given reach (it hands the
 *     loop the same j in the same ascending order, minus ones that cannot
 *     interact), so its results are those of the brute force bit for bit;
 *   - pack / unpack walk tasks, cells and particles in order, one field at a
 *     time, through the oracle's own particle-layout tables.
 *
 * Paper anchors (the paper gives no SPH equations, see the design notes for
 * the readings used):
 *   - interaction-loop pattern: weighted sums over neighbours inside a support
 *     radius H that varies per particle (Sec. 2.1);
 *   - which attributes each loop packs and unpacks: Table 1;
 *   - packing copies only the needed attributes and pre-processes them, e.g.
 *     the periodic coordinate shift; unpacking performs the reductions into the
 *     particles (Sec. 2.3);
 *   - particle layouts AoS / random-order / sAoS (pack-gradient, pack-force,
 *     pack-shared, and their type-split variants) / SoA (Sec. 3.1).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Kernel: 3-D cubic spline with compact support H = gamma_k h.              */
/* W(r,h) = (8/pi) H^-3 w(q), q = r/H,                                       */
/*   w = 1 - 6q^2 + 6q^3 (q < 1/2), 2(1-q)^3 (1/2 <= q < 1), 0 otherwise.    */
/* ------------------------------------------------------------------------ */
static const double OR_PI = 3.141592653589793238462643383279502884;
static const double OR_GAMMA_K = 1.8257418583505537115232326093360; /* sqrt(10/3) */

double or_gamma_k(void) { return OR_GAMMA_K; }

double or_w(double q)
{
    if (q < 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q < 1.0) return 2.0 * (1.0 - q) * (1.0 - q) * (1.0 - q);
    return 0.0;
}

double or_dw(double q) /* dw/dq */
{
    if (q < 0.5) return -12.0 * q + 18.0 * q * q;
    if (q < 1.0) return -6.0 * (1.0 - q) * (1.0 - q);
    return 0.0;
}

double or_W(double r, double h)
{
    double H = OR_GAMMA_K * h;
    return 8.0 / OR_PI / (H * H * H) * or_w(r / H);
}

/* dW/dh at fixed r: -gamma_k (8/pi) H^-4 (3 w + q w'). */
double or_dWdh(double r, double h)
{
    double H = OR_GAMMA_K * h, q = r / H;
    return -OR_GAMMA_K * 8.0 / OR_PI / (H * H * H * H) * (3.0 * or_w(q) + q * or_dw(q));
}

/* Gradient factor F with grad_i W(r_ij, h) = F * r_ij, i.e. (1/r) dW/dr. */
double or_F(double r, double h)
{
    double H = OR_GAMMA_K * h, q = r / H;
    if (q >= 1.0) return 0.0;
    double wq = (q < 0.5) ? (-12.0 + 18.0 * q) : (-6.0 * (1.0 - q) * (1.0 - q) / q);
    return 8.0 / OR_PI / (H * H * H * H * H) * wq;
}

/* Derivatives used only by the error scale (first-order condition bound). */
double or_dWdr(double r, double h) /* dW/dr = (8/pi) H^-4 w'(q) */
{
    double H = OR_GAMMA_K * h;
    return 8.0 / OR_PI / (H * H * H * H) * or_dw(r / H);
}

static double or_d2w(double q)
{
    if (q < 0.5) return -12.0 + 36.0 * q;
    if (q < 1.0) return 12.0 * (1.0 - q);
    return 0.0;
}

double or_d2Wdhdr(double r, double h) /* d/dr of dW/dh = -gamma_k (8/pi) H^-5 (4 w' + q w'') */
{
    double H = OR_GAMMA_K * h, q = r / H;
    return -OR_GAMMA_K * 8.0 / OR_PI / (H * H * H * H * H) * (4.0 * or_dw(q) + q * or_d2w(q));
}

double or_dFdr(double r, double h) /* dF/dr with F = (8/pi) H^-5 w'(q)/q */
{
    double H = OR_GAMMA_K * h, q = r / H;
    if (q >= 1.0) return 0.0;
    double fp = (q < 0.5) ? 18.0 : 6.0 * (1.0 - q) * (1.0 + q) / (q * q);
    return 8.0 / OR_PI / (H * H * H * H * H * H) * fp;
}

/* minimum-image separation in the periodic unit box; x in [0,1) */
static inline double mi(double d)
{
    if (d > 0.5) return d - 1.0;
    if (d < -0.5) return d + 1.0;
    return d;
}


/* ------------------------------------------------------------------------ */
/* Optional candidate grid.  Cells of width >= reach over the unit box; the  */
/* candidates of particle i are the particles of the 27 cells around its    */
/* own, sorted ascending, so a loop visits them in the brute-force order.   */
/* Every j within reach of i (minimum image) is among them.  With fewer     */
/* than 3 cells per side there is no grid (NULL): the loops then visit all  */
/* j.                                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t G;
    int64_t *start; /* G^3 + 1 offsets into idx */
    int64_t *idx;   /* particle indices grouped by cell, ascending in a cell */
    int64_t maxc;   /* most particles in one cell */
} or_grid;

static int64_t grid_axis(double xv, int64_t G)
{
    double w = xv - floor(xv);
    int64_t c = (int64_t)(w * (double)G);
    return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

void *or_grid_build(int64_t n, const double *x, double reach)
{
    if (!(reach > 0.0)) return NULL;
    int64_t G = (int64_t)floor(1.0 / reach);
    if (G < 3) return NULL;
    if (G > 1024) G = 1024;
    or_grid *g = (or_grid *)calloc(1, sizeof(or_grid));
    int64_t nc = G * G * G;
    g->G = G;
    g->start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    g->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        cell[i] = (grid_axis(x[3 * i + 2], G) * G + grid_axis(x[3 * i + 1], G)) * G + grid_axis(x[3 * i], G);
        g->start[cell[i] + 1]++;
    }
    g->maxc = 0;
    for (int64_t c = 0; c < nc; c++) {
        if (g->start[c + 1] > g->maxc) g->maxc = g->start[c + 1];
        g->start[c + 1] += g->start[c];
    }
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)nc);
    for (int64_t i = 0; i < n; i++) g->idx[fill[cell[i]]++] = i; /* ascending within a cell */
    free(fill);
    free(cell);
    return g;
}

void or_grid_free(void *p)
{
    or_grid *g = (or_grid *)p;
    if (!g) return;
    free(g->start);
    free(g->idx);
    free(g);
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t u = *(const int64_t *)a, v = *(const int64_t *)b;
    return (u > v) - (u < v);
}

/* candidates of particle i into buf (room for 27 maxc); returns the count */
static int64_t grid_cands(const or_grid *g, const double *x, int64_t i, int64_t *buf)
{
    const int64_t G = g->G;
    const int64_t cx = grid_axis(x[3 * i], G), cy = grid_axis(x[3 * i + 1], G), cz = grid_axis(x[3 * i + 2], G);
    int64_t nb = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                int64_t c = (((cz + dz + G) % G) * G + (cy + dy + G) % G) * G + (cx + dx + G) % G;
                for (int64_t t = g->start[c]; t < g->start[c + 1]; t++) buf[nb++] = g->idx[t];
            }
    qsort(buf, (size_t)nb, sizeof(int64_t), cmp_i64);
    return nb;
}

static int64_t *cand_buffer(const or_grid *g)
{
    return g ? (int64_t *)malloc(sizeof(int64_t) * (size_t)(27 * g->maxc + 1)) : NULL;
}

/* ------------------------------------------------------------------------ */
/* Reach of every cell (the reading of Sec. 2.2's "neighbours lie in cells   */
/* that share a task"): the smallest distance, minimum image in the unit     */
/* box, between the cell's cube and the cube of any non-empty cell with no   */
/* task joining the two; at most 1/2.  Brute force over all cell pairs.      */
/* ------------------------------------------------------------------------ */
void or_cell_reach(int32_t ncell, const double *loc, const double *width, const int32_t *count,
                   int32_t ntask, const int32_t *ci, const int32_t *cj, double *reach)
{
    /* the cells each cell shares a task with, as lists */
    int64_t *off = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    for (int32_t t = 0; t < ntask; t++) { off[ci[t] + 1]++; off[cj[t] + 1]++; }
    for (int32_t c = 0; c < ncell; c++) off[c + 1] += off[c];
    int32_t *lst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(off[ncell] > 0 ? off[ncell] : 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    for (int32_t c = 0; c < ncell; c++) pos[c] = off[c];
    for (int32_t t = 0; t < ntask; t++) { lst[pos[ci[t]]++] = cj[t]; lst[pos[cj[t]]++] = ci[t]; }
#pragma omp parallel
    {
        unsigned char *partner = (unsigned char *)calloc((size_t)(ncell > 0 ? ncell : 1), 1);
#pragma omp for schedule(dynamic, 64)
        for (int32_t c = 0; c < ncell; c++) {
            for (int64_t e = off[c]; e < off[c + 1]; e++) partner[lst[e]] = 1;
            double best = 0.5;
            for (int32_t d = 0; d < ncell; d++) {
                if (d == c || partner[d] || count[d] == 0) continue;
                double g2 = 0.0;
                for (int k = 0; k < 3; k++) {
                    double a = loc[3 * c + k] + 0.5 * width[c];
                    double b = loc[3 * d + k] + 0.5 * width[d];
                    double sep = mi(b - a);
                    double g = fabs(sep) - 0.5 * (width[c] + width[d]);
                    if (g > 0.0) g2 += g * g;
                }
                double gap = sqrt(g2);
                if (gap < best) best = gap;
            }
            reach[c] = best;
            for (int64_t e = off[c]; e < off[c + 1]; e++) partner[lst[e]] = 0;
        }
        free(partner);
    }
    free(pos);
    free(lst);
    free(off);
}

/* ------------------------------------------------------------------------ */
/* Density loop: over all j including i with r < H_i                         */
/*   rho_i = sum m_j W(r, h_i);  rho_dh_i = sum m_j dW/dh(r, h_i);            */
/*   wcount_i = sum W(r, h_i).                                               */
/* Error scales returned beside every sum (for the parity tolerance):        */
/*   S: arithmetic scale, per term the sum of |elementary products|;          */
/*   P: position scale, per term a bound on |d term / d r_ij| times           */
/*      (epsx_i + epsx_j), the resolution of the packed positions (optional); */
/*   band: pairs within 1e-6 H + epsx_i + epsx_j of the support edge.         */
/* ------------------------------------------------------------------------ */
void or_density(int64_t n, const double *x, const float *m, const float *h,
                int64_t nrow, const int64_t *rows,
                const double *epsx, double *rho, double *rho_dh, double *wcount, double *S, double *P,
                int32_t *cnt, int32_t *band, const void *grid)
{
    int64_t nr = rows ? nrow : n;
    const or_grid *g = (const or_grid *)grid;
#pragma omp parallel
    {
    int64_t *cand = cand_buffer(g);
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nr; k++) {
        int64_t i = rows ? rows[k] : k;
        double H = OR_GAMMA_K * (double)h[i];
        double sr = 0, sd = 0, sw = 0, s0 = 0, s1 = 0, s2 = 0, q0 = 0, q1 = 0, q2 = 0;
        int32_t c = 0, b = 0;
        int64_t nc = g ? grid_cands(g, x, i, cand) : n;
        for (int64_t t = 0; t < nc; t++) {
            int64_t j = g ? cand[t] : t;
            double dx = mi(x[3 * i] - x[3 * j]);
            double dy = mi(x[3 * i + 1] - x[3 * j + 1]);
            double dz = mi(x[3 * i + 2] - x[3 * j + 2]);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double ep = epsx ? epsx[i] + epsx[j] : 0.0;
            if (fabs(r - H) < 1e-6 * H + ep) b++;
            if (!(r < H)) continue;
            double W = or_W(r, h[i]);
            double Wh = or_dWdh(r, h[i]);
            double mj = m[j];
            sr += mj * W;
            sd += mj * Wh;
            sw += W;
            double Wr = fabs(or_dWdr(r, h[i]));
            s0 += mj * W;
            s1 += fabs(mj * Wh);
            s2 += W;
            q0 += mj * Wr * ep;
            q1 += mj * fabs(or_d2Wdhdr(r, h[i])) * ep;
            q2 += Wr * ep;
            c++;
        }
        rho[k] = sr; rho_dh[k] = sd; wcount[k] = sw;
        if (S) { S[3 * k] = s0; S[3 * k + 1] = s1; S[3 * k + 2] = s2; }
        if (P) { P[3 * k] = q0; P[3 * k + 1] = q1; P[3 * k + 2] = q2; }
        if (cnt) cnt[k] = c;
        if (band) band[k] = b;
    }
    free(cand);
    }
}

/* per-particle quantities every consumer derives from the stored ones */
static double sound_speed(double gam, double u) { return sqrt(gam * (gam - 1.0) * u); }

/* ------------------------------------------------------------------------ */
/* Gradient loop: over j != i with r < H_i                                   */
/*   D_i = sum m_j v_ij . grad_i W_ij            (div v_i  = -D_i / rho_i)    */
/*   R_i = sum m_j v_ij x grad_i W_ij            (curl v_i =  R_i / rho_i)    */
/*   L_i = sum 2 (m_j/rho_j) (u_i - u_j) F_ij    (Brookshaw Laplacian of u)  */
/*   V_i = max(0, max_j [c_i + c_j - beta min(0, v_ij . rhat_ij)])           */
/* ------------------------------------------------------------------------ */
void or_gradient(int64_t n, const double *x, const float *v, const float *m, const float *h,
                 const float *u, const double *rhoj, double gam, double beta,
                 int64_t nrow, const int64_t *rows, const double *epsx,
                 double *D, double *R, double *L, double *V, double *S, double *P, int32_t *cnt,
                 int32_t *band, const void *grid)
{
    int64_t nr = rows ? nrow : n;
    const or_grid *g = (const or_grid *)grid;
#pragma omp parallel
    {
    int64_t *cand = cand_buffer(g);
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nr; k++) {
        int64_t i = rows ? rows[k] : k;
        double H = OR_GAMMA_K * (double)h[i];
        double ci = sound_speed(gam, u[i]);
        double d = 0, r0 = 0, r1 = 0, r2 = 0, l = 0, vmax = 0;
        double ad = 0, ar0 = 0, ar1 = 0, ar2 = 0, al = 0;
        double pd = 0, pr0 = 0, pr1 = 0, pr2 = 0, pl = 0;
        int32_t c = 0, b = 0;
        int64_t nc = g ? grid_cands(g, x, i, cand) : n;
        for (int64_t t = 0; t < nc; t++) {
            int64_t j = g ? cand[t] : t;
            if (j == i) continue;
            double rx = mi(x[3 * i] - x[3 * j]);
            double ry = mi(x[3 * i + 1] - x[3 * j + 1]);
            double rz = mi(x[3 * i + 2] - x[3 * j + 2]);
            double r = sqrt(rx * rx + ry * ry + rz * rz);
            double ep = epsx ? epsx[i] + epsx[j] : 0.0;
            if (fabs(r - H) < 1e-6 * H + ep) b++;
            if (!(r < H)) continue;
            double F = or_F(r, h[i]);
            double gx = F * rx, gy = F * ry, gz = F * rz; /* grad_i W(r_ij, h_i) */
            double vx = (double)v[3 * i] - v[3 * j];
            double vy = (double)v[3 * i + 1] - v[3 * j + 1];
            double vz = (double)v[3 * i + 2] - v[3 * j + 2];
            double mj = m[j];
            double td = mj * (vx * gx + vy * gy + vz * gz);
            double t0 = mj * (vy * gz - vz * gy);
            double t1 = mj * (vz * gx - vx * gz);
            double t2 = mj * (vx * gy - vy * gx);
            double tl = 2.0 * (mj / rhoj[j]) * ((double)u[i] - (double)u[j]) * F;
            d += td; r0 += t0; r1 += t1; r2 += t2; l += tl;
            /* scales: componentwise products; gradient-norm bounds times ep */
            double aF = fabs(F), aFp = fabs(or_dFdr(r, h[i]));
            double vn = sqrt(vx * vx + vy * vy + vz * vz);
            double vrr = fabs(vx * rx + vy * ry + vz * rz);
            ad += mj * aF * (fabs(vx * rx) + fabs(vy * ry) + fabs(vz * rz));
            ar0 += mj * aF * (fabs(vy * rz) + fabs(vz * ry));
            ar1 += mj * aF * (fabs(vz * rx) + fabs(vx * rz));
            ar2 += mj * aF * (fabs(vx * ry) + fabs(vy * rx));
            al += fabs(tl);
            pd += mj * (aFp * vrr + aF * vn) * ep;
            pr0 += mj * (aFp * fabs(vy * rz - vz * ry) + aF * vn) * ep;
            pr1 += mj * (aFp * fabs(vz * rx - vx * rz) + aF * vn) * ep;
            pr2 += mj * (aFp * fabs(vx * ry - vy * rx) + aF * vn) * ep;
            pl += 2.0 * (mj / rhoj[j]) * fabs((double)u[i] - (double)u[j]) * aFp * ep;
            double vr = (r > 0) ? (vx * rx + vy * ry + vz * rz) / r : 0.0;
            double mu = vr < 0 ? vr : 0.0;
            double sig = ci + sound_speed(gam, u[j]) - beta * mu;
            if (sig > vmax) vmax = sig;
            c++;
        }
        D[k] = d; R[3 * k] = r0; R[3 * k + 1] = r1; R[3 * k + 2] = r2; L[k] = l; V[k] = vmax;
        if (S) { S[5 * k] = ad; S[5 * k + 1] = ar0; S[5 * k + 2] = ar1; S[5 * k + 3] = ar2; S[5 * k + 4] = al; }
        if (P) { P[5 * k] = pd; P[5 * k + 1] = pr0; P[5 * k + 2] = pr1; P[5 * k + 3] = pr2; P[5 * k + 4] = pl; }
        if (cnt) cnt[k] = c;
        if (band) band[k] = b;
    }
    free(cand);
    }
}

/* ------------------------------------------------------------------------ */
/* Force loop: over j != i with r < max(H_i, H_j)                            */
/* per particle:  Omega = 1 + h rho_dh / (3 rho),  P = (gamma-1) rho u,       */
/*                A = P / (Omega rho^2),  c = sqrt(gamma (gamma-1) u),         */
/*                B = |div v| / (|div v| + |curl v| + eps c / h),              */
/*                alpha~ = alpha_v B                                          */
/* per pair:      G_i = grad_i W(r_ij,h_i) (0 beyond H_i), G_j likewise,       */
/*                Gbar = (G_i + G_j)/2, mu = min(0, v_ij . rhat),              */
/*                v_sig = c_i + c_j - beta mu, rhobar = (rho_i + rho_j)/2,     */
/*                Pi = -(1/2) (alpha~_i + alpha~_j)/2 v_sig mu / rhobar        */
/* a_i     = -sum m_j [A_i G_i + A_j G_j + Pi Gbar]                           */
/* du_i/dt =  sum m_j [A_i v_ij.G_i + Pi/2 v_ij.Gbar                          */
/*                     + (alpha_d,i + alpha_d,j)/2 |v_ij.rhat| (u_i - u_j)     */
/*                       (rhat . Gbar) / rhobar]                              */
/* ------------------------------------------------------------------------ */
typedef struct { double A, c, at, rho, u, ad, H; } or_pp;

static or_pp per_particle(int64_t i, const float *h, const float *u, const double *rho,
                          const double *rho_dh, const double *D, const double *R,
                          const float *alpha_v, const float *alpha_d, const double *atilde,
                          double gam, double eps)
{
    or_pp p;
    double hh = h[i], rr = rho[i];
    double omega = 1.0 + hh * rho_dh[i] / (3.0 * rr);
    double P = (gam - 1.0) * rr * u[i];
    p.A = P / (omega * rr * rr);
    p.c = sound_speed(gam, u[i]);
    if (atilde) {
        p.at = atilde[i];
    } else {
        double div = -D[i] / rr;
        double curl = sqrt(R[3 * i] * R[3 * i] + R[3 * i + 1] * R[3 * i + 1] + R[3 * i + 2] * R[3 * i + 2]) / rr;
        double B = fabs(div) / (fabs(div) + curl + eps * p.c / hh);
        p.at = (double)alpha_v[i] * B;
    }
    p.rho = rr;
    p.u = u[i];
    p.ad = alpha_d[i];
    p.H = OR_GAMMA_K * hh;
    return p;
}

void or_balsara(int64_t n, const float *h, const float *u, const double *rho, const double *D,
                const double *R, const float *alpha_v, double gam, double eps, double *atilde)
{
    for (int64_t i = 0; i < n; i++) {
        double c = sound_speed(gam, u[i]);
        double div = -D[i] / rho[i];
        double curl = sqrt(R[3 * i] * R[3 * i] + R[3 * i + 1] * R[3 * i + 1] + R[3 * i + 2] * R[3 * i + 2]) / rho[i];
        atilde[i] = (double)alpha_v[i] * fabs(div) / (fabs(div) + curl + eps * c / h[i]);
    }
}

/* atilde may be NULL (then computed from D, R); otherwise it is used as given. */
void or_force(int64_t n, const double *x, const float *v, const float *m, const float *h,
              const float *u, const double *rho, const double *rho_dh, const double *D,
              const double *R, const float *alpha_v, const float *alpha_d, const double *atilde,
              double gam, double beta, double eps, int64_t nrow, const int64_t *rows, const double *epsx,
              double *acc, double *udt, double *S, double *P, int32_t *cnt, int32_t *band,
              const void *grid)
{
    const or_grid *g = (const or_grid *)grid;
    int64_t nr = rows ? nrow : n;
    or_pp *pp = (or_pp *)malloc(sizeof(or_pp) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; j++)
        pp[j] = per_particle(j, h, u, rho, rho_dh, D, R, alpha_v, alpha_d, atilde, gam, eps);
#pragma omp parallel
    {
    int64_t *cand = cand_buffer(g);
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < nr; k++) {
        int64_t i = rows ? rows[k] : k;
        or_pp pi = pp[i];
        double a0 = 0, a1 = 0, a2 = 0, du = 0;
        double s0 = 0, s1 = 0, s2 = 0, sd = 0, q0 = 0, q1 = 0, q2 = 0, qd = 0;
        int32_t c = 0, b = 0;
        int64_t nc = g ? grid_cands(g, x, i, cand) : n;
        for (int64_t t = 0; t < nc; t++) {
            int64_t j = g ? cand[t] : t;
            if (j == i) continue;
            or_pp pj = pp[j];
            double rx = mi(x[3 * i] - x[3 * j]);
            double ry = mi(x[3 * i + 1] - x[3 * j + 1]);
            double rz = mi(x[3 * i + 2] - x[3 * j + 2]);
            double r = sqrt(rx * rx + ry * ry + rz * rz);
            double Hmax = pi.H > pj.H ? pi.H : pj.H;
            double ep = epsx ? epsx[i] + epsx[j] : 0.0;
            if (fabs(r - Hmax) < 1e-6 * Hmax + ep) b++;
            if (!(r < Hmax)) continue;
            double Fi = (r < pi.H) ? or_F(r, h[i]) : 0.0;
            double Fj = (r < pj.H) ? or_F(r, h[j]) : 0.0;
            double Fbar = 0.5 * (Fi + Fj);
            double vx = (double)v[3 * i] - v[3 * j];
            double vy = (double)v[3 * i + 1] - v[3 * j + 1];
            double vz = (double)v[3 * i + 2] - v[3 * j + 2];
            double ex = 0, ey = 0, ez = 0; /* rhat, 0 at r = 0 */
            if (r > 0) { ex = rx / r; ey = ry / r; ez = rz / r; }
            double vr = vx * ex + vy * ey + vz * ez;
            double mu = vr < 0 ? vr : 0.0;
            double vsig = pi.c + pj.c - beta * mu;
            double rhobar = 0.5 * (pi.rho + pj.rho);
            double aij = 0.5 * (pi.at + pj.at);
            double Pi = -0.5 * aij * vsig * mu / rhobar;
            double mj = m[j];
            /* G vectors */
            double Gix = Fi * rx, Giy = Fi * ry, Giz = Fi * rz;
            double Gjx = Fj * rx, Gjy = Fj * ry, Gjz = Fj * rz;
            double Gbx = Fbar * rx, Gby = Fbar * ry, Gbz = Fbar * rz;
            double p0x = -mj * pi.A * Gix, p1x = -mj * pj.A * Gjx, p2x = -mj * Pi * Gbx;
            double p0y = -mj * pi.A * Giy, p1y = -mj * pj.A * Gjy, p2y = -mj * Pi * Gby;
            double p0z = -mj * pi.A * Giz, p1z = -mj * pj.A * Gjz, p2z = -mj * Pi * Gbz;
            a0 += p0x + p1x + p2x; a1 += p0y + p1y + p2y; a2 += p0z + p1z + p2z;
            double e0 = mj * pi.A * (vx * Gix + vy * Giy + vz * Giz);
            double e1 = mj * 0.5 * Pi * (vx * Gbx + vy * Gby + vz * Gbz);
            double e2 = mj * 0.5 * (pi.ad + pj.ad) * fabs(vr) * (pi.u - pj.u) *
                        (ex * Gbx + ey * Gby + ez * Gbz) / rhobar;
            du += e0 + e1 + e2;
            /* scales: |elementary products|; gradient-norm bounds times ep */
            double Fip = (r < pi.H) ? fabs(or_dFdr(r, h[i])) : 0.0;
            double Fjp = (r < pj.H) ? fabs(or_dFdr(r, h[j])) : 0.0;
            double X = fabs(pi.A * Fi) + fabs(pj.A * Fj) + fabs(Pi * Fbar);
            double Xp = fabs(pi.A) * Fip + fabs(pj.A) * Fjp + fabs(Pi) * 0.5 * (Fip + Fjp);
            double vn = sqrt(vx * vx + vy * vy + vz * vz);
            double dPi = 0.5 * aij * (pi.c + pj.c + 2.0 * beta * fabs(mu)) / rhobar; /* |dPi/dmu| */
            double gs = Xp + (r > 0 ? fabs(Fbar) * dPi * vn / r : 0.0);             /* |grad s| */
            s0 += mj * X * fabs(rx);
            s1 += mj * X * fabs(ry);
            s2 += mj * X * fabs(rz);
            q0 += mj * (gs * fabs(rx) + X) * ep;
            q1 += mj * (gs * fabs(ry) + X) * ep;
            q2 += mj * (gs * fabs(rz) + X) * ep;
            double cvr = fabs(vx * rx) + fabs(vy * ry) + fabs(vz * rz), dvr = fabs(vx * rx + vy * ry + vz * rz);
            double Fbp = 0.5 * (Fip + Fjp), adb = 0.5 * (pi.ad + pj.ad), du_ = fabs(pi.u - pj.u);
            sd += mj * fabs(pi.A * Fi) * cvr + 0.5 * mj * fabs(Pi * Fbar) * cvr +
                  mj * adb * du_ / rhobar * fabs(Fbar) * cvr;
            qd += (mj * fabs(pi.A) * (Fip * dvr + fabs(Fi) * vn) +
                   0.5 * mj * (fabs(Pi) * (Fbp * dvr + fabs(Fbar) * vn) + (r > 0 ? fabs(Fbar) * dvr * dPi * vn / r : 0.0)) +
                   mj * adb * du_ / rhobar * (Fbp * dvr + fabs(Fbar) * vn)) * ep;
            c++;
        }
        acc[3 * k] = a0; acc[3 * k + 1] = a1; acc[3 * k + 2] = a2; udt[k] = du;
        if (S) { S[4 * k] = s0; S[4 * k + 1] = s1; S[4 * k + 2] = s2; S[4 * k + 3] = sd; }
        if (P) { P[4 * k] = q0; P[4 * k + 1] = q1; P[4 * k + 2] = q2; P[4 * k + 3] = qd; }
        if (cnt) cnt[k] = c;
        if (band) band[k] = b;
    }
    free(cand);
    }
    free(pp);
}

/* ======================================================================== */
/* Particle layouts (Sec. 3.1), the oracle's own tables.                    */
/* A layout is a list of substructs; each substruct is a list of members     */
/* placed in order at their natural alignment, the record padded to 8 bytes. */
/* SoA is one array per scalar component.  A layout may list x again in      */
/* later substructs (Sec. 5, data replication): the first copy is the one    */
/* read, and writing x writes every copy.                                    */
/* ======================================================================== */
enum { F_X, F_V, F_A, F_MASS, F_H, F_U, F_UDT, F_RHO, F_RHODH, F_WCOUNT, F_DIV, F_ROT,
       F_LAP, F_VSIG, F_AV, F_AD, F_TBIN, F_ID, F_COLD, NF };
/* components and bytes per component of each field */
static const int f_ncomp[NF] = {3, 3, 3, 1, 1, 1, 1, 1, 1, 1, 1, 3, 1, 1, 1, 1, 1, 1, 5};
static const int f_csize[NF] = {8, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 1, 8, 8};

enum { L_AOS, L_AOS_RANDOM, L_SAOS_GRAD, L_SAOS_FORCE, L_SAOS_SHARED, L_SAOS_GRAD_TYPE,
       L_SAOS_FORCE_TYPE, L_SAOS_SHARED_TYPE, L_SOA, L_SAOS_SHARED_REPL, NL };

#define END (-1)
#define NEXT (-2)
/* member lists: substructs separated by NEXT, terminated by END */
static const int lay_aos[] = {F_X, F_V, F_A, F_MASS, F_H, F_U, F_UDT, F_RHO, F_RHODH, F_WCOUNT,
                              F_DIV, F_ROT, F_LAP, F_VSIG, F_AV, F_AD, F_TBIN, F_ID, F_COLD, END};
/* members of the AoS record in the order of a fixed shuffle (numpy PCG64 seed 0) */
static const int lay_rand[] = {F_A, F_DIV, F_MASS, F_AV, F_X, F_LAP, F_H, F_COLD, F_RHO, F_U,
                               F_ID, F_TBIN, F_RHODH, F_ROT, F_UDT, F_VSIG, F_WCOUNT, F_V, F_AD, END};
static const int lay_grad[] = {F_X, F_V, F_MASS, F_H, F_U, F_RHO, NEXT,
                               F_RHODH, F_DIV, F_ROT, F_AV, F_AD, NEXT,
                               F_A, F_UDT, F_WCOUNT, F_LAP, F_VSIG, NEXT,
                               F_TBIN, F_ID, F_COLD, END};
static const int lay_force[] = {F_X, F_V, F_MASS, F_H, F_U, F_RHO, F_RHODH, F_DIV, F_ROT, F_AV, F_AD, NEXT,
                                F_A, F_UDT, F_WCOUNT, F_LAP, F_VSIG, NEXT,
                                F_TBIN, F_ID, F_COLD, END};
static const int lay_shared[] = {F_X, F_MASS, F_H, NEXT,
                                 F_V, F_U, F_RHO, NEXT,
                                 F_RHODH, F_DIV, F_ROT, F_AV, F_AD, NEXT,
                                 F_A, F_UDT, F_WCOUNT, F_LAP, F_VSIG, NEXT,
                                 F_TBIN, F_ID, F_COLD, END};
static const int lay_grad_t[] = {F_X, NEXT, F_V, F_MASS, F_H, F_U, F_RHO, NEXT,
                                 F_RHODH, F_DIV, F_ROT, F_AV, F_AD, NEXT,
                                 F_A, F_UDT, F_WCOUNT, F_LAP, F_VSIG, NEXT,
                                 F_TBIN, F_ID, NEXT, F_COLD, END};
static const int lay_force_t[] = {F_X, NEXT, F_V, F_MASS, F_H, F_U, F_RHO, F_RHODH, F_DIV, F_ROT, F_AV, F_AD, NEXT,
                                  F_A, F_UDT, F_WCOUNT, F_LAP, F_VSIG, NEXT,
                                  F_TBIN, F_ID, NEXT, F_COLD, END};
static const int lay_shared_t[] = {F_X, NEXT, F_MASS, F_H, NEXT,
                                   F_V, F_U, F_RHO, NEXT,
                                   F_RHODH, F_DIV, F_ROT, F_AV, F_AD, NEXT,
                                   F_A, F_UDT, F_WCOUNT, F_LAP, F_VSIG, NEXT,
                                   F_TBIN, F_ID, NEXT, F_COLD, END};
/* pack-shared with the position in every substruct a loop packs from */
static const int lay_shared_repl[] = {F_X, F_MASS, F_H, NEXT,
                                      F_X, F_V, F_U, F_RHO, NEXT,
                                      F_X, F_RHODH, F_DIV, F_ROT, F_AV, F_AD, NEXT,
                                      F_A, F_UDT, F_WCOUNT, F_LAP, F_VSIG, NEXT,
                                      F_TBIN, F_ID, F_COLD, END};
static const int *const lay_lists[NL] = {lay_aos, lay_rand, lay_grad, lay_force, lay_shared,
                                         lay_grad_t, lay_force_t, lay_shared_t, NULL, lay_shared_repl};

typedef struct {
    int nsub;
    size_t sub_bytes[32];
    int sub_of[NF][5];     /* per field component: the copy that is read */
    size_t off_of[NF][5];
    int nxcopy;            /* further copies of x */
    int xcopy_sub[4];
    size_t xcopy_off[4];   /* offset of x[0]; x[c] 8 bytes further */
} or_layout;

static int build_layout(int L, or_layout *o)
{
    memset(o, 0, sizeof(*o));
    if (L < 0 || L >= NL) return -1;
    if (L == L_SOA) {
        int s = 0;
        for (int f = 0; f < NF; f++) {
            if (f == F_COLD) { /* the cold block stays one 40-byte element */
                for (int c = 0; c < 5; c++) { o->sub_of[f][c] = s; o->off_of[f][c] = 8 * c; }
                o->sub_bytes[s++] = 40;
                continue;
            }
            for (int c = 0; c < f_ncomp[f]; c++) {
                o->sub_of[f][c] = s;
                o->off_of[f][c] = 0;
                o->sub_bytes[s++] = f_csize[f];
            }
        }
        o->nsub = s;
        return 0;
    }
    const int *lst = lay_lists[L];
    int s = 0, seen_x = 0;
    size_t off = 0;
    for (int k = 0;; k++) {
        int f = lst[k];
        if (f == NEXT || f == END) {
            o->sub_bytes[s] = (off + 7) / 8 * 8;
            s++;
            off = 0;
            if (f == END) break;
            continue;
        }
        size_t align = f_csize[f] < 8 ? (size_t)f_csize[f] : 8;
        off = (off + align - 1) / align * align;
        if (f == F_X && seen_x) { /* a further copy of the position */
            o->xcopy_sub[o->nxcopy] = s;
            o->xcopy_off[o->nxcopy] = off;
            o->nxcopy++;
        } else {
            for (int c = 0; c < f_ncomp[f]; c++) {
                o->sub_of[f][c] = s;
                o->off_of[f][c] = off + (size_t)c * f_csize[f];
            }
            if (f == F_X) seen_x = 1;
        }
        off += (size_t)f_ncomp[f] * f_csize[f];
    }
    o->nsub = s;
    return 0;
}

int or_layout_info(int L, int *nsub, size_t *sub_bytes)
{
    or_layout o;
    if (build_layout(L, &o)) return -1;
    *nsub = o.nsub;
    for (int s = 0; s < o.nsub; s++) sub_bytes[s] = o.sub_bytes[s];
    return 0;
}

int or_x_copies(int L, int *count, int *sub, size_t *off)
{
    or_layout o;
    if (build_layout(L, &o)) return -1;
    *count = o.nxcopy;
    for (int r = 0; r < o.nxcopy; r++) { sub[r] = o.xcopy_sub[r]; off[r] = o.xcopy_off[r]; }
    return 0;
}

int or_field_location(int L, int f, int comp, int *sub, size_t *off, size_t *stride)
{
    or_layout o;
    if (build_layout(L, &o) || f < 0 || f >= NF || comp < 0 || comp >= f_ncomp[f]) return -1;
    *sub = o.sub_of[f][comp];
    *off = o.off_of[f][comp];
    *stride = o.sub_bytes[*sub];
    return 0;
}

static inline unsigned char *loc_ptr(const or_layout *o, void *const *subs, int f, int c, int64_t p)
{
    int s = o->sub_of[f][c];
    return (unsigned char *)subs[s] + (size_t)p * o->sub_bytes[s] + o->off_of[f][c];
}

/* copy a dense [n][ncomp] array of the field's type into / out of the store */
int or_store_put(int L, int64_t n, void *const *subs, int f, const void *src)
{
    or_layout o;
    if (build_layout(L, &o) || f < 0 || f >= NF) return -1;
    const unsigned char *s = (const unsigned char *)src;
    size_t cs = f_csize[f];
    for (int64_t p = 0; p < n; p++)
        for (int c = 0; c < f_ncomp[f]; c++) {
            memcpy(loc_ptr(&o, subs, f, c, p), s + ((size_t)p * f_ncomp[f] + c) * cs, cs);
            if (f == F_X)
                for (int r = 0; r < o.nxcopy; r++)
                    memcpy((unsigned char *)subs[o.xcopy_sub[r]] + (size_t)p * o.sub_bytes[o.xcopy_sub[r]] +
                               o.xcopy_off[r] + 8 * (size_t)c,
                           s + ((size_t)p * f_ncomp[f] + c) * cs, cs);
        }
    return 0;
}

int or_store_get(int L, int64_t n, void *const *subs, int f, void *dst)
{
    or_layout o;
    if (build_layout(L, &o) || f < 0 || f >= NF) return -1;
    unsigned char *d = (unsigned char *)dst;
    size_t cs = f_csize[f];
    for (int64_t p = 0; p < n; p++)
        for (int c = 0; c < f_ncomp[f]; c++)
            memcpy(d + ((size_t)p * f_ncomp[f] + c) * cs, loc_ptr(&o, subs, f, c, p), cs);
    return 0;
}

/* ======================================================================== */
/* Pack / unpack (Sec. 2.3, Table 1).                                        */
/* Packed record per slot, by loop, as planes (plane k of a buffer holding   */
/* P slots starts at P times the bytes of the planes before it):             */
/*   density : [dx dy dz h] [m]                                              */
/*   gradient: [dx dy dz h] [vx vy vz m] [u rho]                             */
/*   force   : [dx dy dz h] [vx vy vz m] [u rho rho_dh D] [R0 R1 R2 alpha_v]  */
/*             [alpha_d]                                                     */
/* dx = (float)(x - o) with o = loc(ci) for ci's particles and               */
/* o = loc(ci) - shift for cj's, both in FP64 then rounded to nearest.       */
/* Results per slot, one float plane each:                                   */
/*   density [rho rho_dh wcount]; gradient [D R0 R1 R2 L V];                  */
/*   force [a0 a1 a2 u_dt].                                                  */
/* ======================================================================== */
typedef struct { double loc[3]; double width; int64_t first; int32_t count; int32_t pad; } or_cell;
typedef struct { int32_t ci, cj; int32_t pad[2]; double shift[3]; } or_task;

static const int pk_nplane[3] = {2, 3, 5};
static const int pk_plane_floats[3][5] = {{4, 1}, {4, 4, 2}, {4, 4, 4, 4, 1}};
static const int res_nplane[3] = {3, 6, 4};

int64_t or_round_slots(int64_t nslot) { return (nslot + 63) / 64 * 64; }

static int64_t task_slots(const or_cell *cells, const or_task *t)
{
    return t->ci == t->cj ? cells[t->ci].count : (int64_t)cells[t->ci].count + cells[t->cj].count;
}

int64_t or_range_slots(const or_cell *cells, const or_task *tasks, int32_t t0, int32_t t1)
{
    int64_t s = 0;
    for (int32_t t = t0; t < t1; t++) s += task_slots(cells, &tasks[t]);
    return s;
}

static float getf(const or_layout *o, void *const *subs, int f, int c, int64_t p)
{
    float v;
    memcpy(&v, loc_ptr(o, subs, f, c, p), 4);
    return v;
}

/* write one slot's packed record */
static void pack_slot(const or_layout *o, void *const *subs, int loop, int64_t p, const double org[3],
                      unsigned char *buf, int64_t P, int64_t slot)
{
    float rec[5][4];
    for (int d = 0; d < 3; d++) {
        double xd;
        memcpy(&xd, loc_ptr(o, subs, F_X, d, p), 8);
        rec[0][d] = (float)(xd - org[d]);
    }
    rec[0][3] = getf(o, subs, F_H, 0, p);
    if (loop == 0) {
        rec[1][0] = getf(o, subs, F_MASS, 0, p);
    } else {
        for (int d = 0; d < 3; d++) rec[1][d] = getf(o, subs, F_V, d, p);
        rec[1][3] = getf(o, subs, F_MASS, 0, p);
        rec[2][0] = getf(o, subs, F_U, 0, p);
        rec[2][1] = getf(o, subs, F_RHO, 0, p);
        if (loop == 2) {
            rec[2][2] = getf(o, subs, F_RHODH, 0, p);
            rec[2][3] = getf(o, subs, F_DIV, 0, p);
            for (int d = 0; d < 3; d++) rec[3][d] = getf(o, subs, F_ROT, d, p);
            rec[3][3] = getf(o, subs, F_AV, 0, p);
            rec[4][0] = getf(o, subs, F_AD, 0, p);
        }
    }
    size_t base = 0;
    for (int k = 0; k < pk_nplane[loop]; k++) {
        size_t pb = 4 * (size_t)pk_plane_floats[loop][k];
        memcpy(buf + base + (size_t)slot * pb, rec[k], pb);
        base += (size_t)P * pb;
    }
}

/* slots of tasks [t0, t1): task order, ci's particles then cj's, store order */
int or_pack(int L, int loop, int64_t n, void *const *subs, const or_cell *cells, const or_task *tasks,
            int32_t t0, int32_t t1, void *buf)
{
    or_layout o;
    if (build_layout(L, &o) || loop < 0 || loop > 2) return -1;
    (void)n;
    int64_t P = or_round_slots(or_range_slots(cells, tasks, t0, t1));
    int64_t slot = 0;
    for (int32_t t = t0; t < t1; t++) {
        const or_task *tk = &tasks[t];
        const or_cell *ci = &cells[tk->ci];
        double org[3];
        for (int d = 0; d < 3; d++) org[d] = ci->loc[d];
        for (int32_t k = 0; k < ci->count; k++)
            pack_slot(&o, subs, loop, ci->first + k, org, (unsigned char *)buf, P, slot++);
        if (tk->ci != tk->cj) {
            const or_cell *cj = &cells[tk->cj];
            for (int d = 0; d < 3; d++) org[d] = ci->loc[d] - tk->shift[d];
            for (int32_t k = 0; k < cj->count; k++)
                pack_slot(&o, subs, loop, cj->first + k, org, (unsigned char *)buf, P, slot++);
        }
    }
    return 0;
}

/* one slot per particle in store order, relative to the particle's own cell */
int or_pack_cells(int L, int loop, int64_t n, void *const *subs, const or_cell *cells, int32_t ncell,
                  void *buf)
{
    or_layout o;
    if (build_layout(L, &o) || loop < 0 || loop > 2) return -1;
    int64_t P = or_round_slots(n);
    for (int32_t c = 0; c < ncell; c++)
        for (int32_t k = 0; k < cells[c].count; k++)
            pack_slot(&o, subs, loop, cells[c].first + k, cells[c].loc, (unsigned char *)buf, P,
                      cells[c].first + k);
    return 0;
}

static const int res_field[3][6] = {{F_RHO, F_RHODH, F_WCOUNT}, {F_DIV, F_ROT, F_ROT, F_ROT, F_LAP, F_VSIG},
                                    {F_A, F_A, F_A, F_UDT}};
static const int res_comp[3][6] = {{0, 0, 0}, {0, 0, 1, 2, 0, 0}, {0, 1, 2, 0}};

/* the loop's outputs set to +0.0f */
int or_zero_outputs(int L, int loop, int64_t n, void *const *subs)
{
    or_layout o;
    if (build_layout(L, &o) || loop < 0 || loop > 2) return -1;
    float z = 0.0f;
    for (int64_t p = 0; p < n; p++)
        for (int k = 0; k < res_nplane[loop]; k++)
            memcpy(loc_ptr(&o, subs, res_field[loop][k], res_comp[loop][k], p), &z, 4);
    return 0;
}

/* reduce: sums in FP32 in slot order; the signal velocity V takes the larger */
static void reduce_slot(const or_layout *o, void *const *subs, int loop, int64_t p, const float *res,
                        int64_t P, int64_t slot)
{
    for (int k = 0; k < res_nplane[loop]; k++) {
        float r = res[(size_t)k * P + slot];
        unsigned char *dst = loc_ptr(o, subs, res_field[loop][k], res_comp[loop][k], p);
        float cur;
        memcpy(&cur, dst, 4);
        if (loop == 1 && k == 5)
            cur = (r > cur) ? r : cur;
        else
            cur = cur + r;
        memcpy(dst, &cur, 4);
    }
}

int or_unpack(int L, int loop, int64_t n, void *const *subs, const or_cell *cells, const or_task *tasks,
              int32_t t0, int32_t t1, const void *res)
{
    or_layout o;
    if (build_layout(L, &o) || loop < 0 || loop > 2) return -1;
    (void)n;
    int64_t P = or_round_slots(or_range_slots(cells, tasks, t0, t1));
    int64_t slot = 0;
    for (int32_t t = t0; t < t1; t++) {
        const or_task *tk = &tasks[t];
        const or_cell *ci = &cells[tk->ci];
        for (int32_t k = 0; k < ci->count; k++)
            reduce_slot(&o, subs, loop, ci->first + k, (const float *)res, P, slot++);
        if (tk->ci != tk->cj) {
            const or_cell *cj = &cells[tk->cj];
            for (int32_t k = 0; k < cj->count; k++)
                reduce_slot(&o, subs, loop, cj->first + k, (const float *)res, P, slot++);
        }
    }
    return 0;
}

/* per-particle results (slot = particle): zero the outputs, then one reduction each */
int or_unpack_cells(int L, int loop, int64_t n, void *const *subs, const void *res)
{
    or_layout o;
    if (build_layout(L, &o) || loop < 0 || loop > 2) return -1;
    or_zero_outputs(L, loop, n, subs);
    int64_t P = or_round_slots(n);
    for (int64_t p = 0; p < n; p++) reduce_slot(&o, subs, loop, p, (const float *)res, P, p);
    return 0;
}
