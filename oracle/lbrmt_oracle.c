/*
 * lbrmt_oracle.c -- TEST INFRASTRUCTURE ONLY (see lbrmt_oracle.h).
 *
 * Plain FP64 CPU implementation of the LBRMT time step (Alg. 1 of Sun &
 * Rycroft), written for clarity, not speed: every step is a separate loop over
 * the whole grid, in the order of Alg. 1, with the formulas in the paper's own
 * notation.  OpenMP only splits independent per-node loops; nothing is fused,
 * blocked or reordered.  Built with -ffp-contract=off.
 */
#define _GNU_SOURCE
#include "lbrmt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocity set and weights: Table "d2q9" (Sec. 2.2) */
#define NQ 9
static const int CX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[NQ] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2, Sec. 2.2 */
static const double PI = 3.14159265358979323846;

struct orc_sim {
    orc_params p;
    int nsolid;
    orc_solid body;
    int nxp, nyp;           /* padded extents                              */
    int ox, oy;             /* padding offset: 2 on walled axes, 0 periodic */
    long N, NP;
    /* lattice Boltzmann state (interior nodes) */
    double* f;              /* f_i^n, [q][N] */
    double* fhat;           /* post-collision populations */
    double* fnew;
    double* rho;            /* rho^n */
    double* ux;             /* u^n (with half force of Fx, Fy) */
    double* uy;
    double* Fx;             /* force density of the last step */
    double* Fy;
    /* reference map state (padded grid) at step n */
    double *X, *Y, *phi;
    unsigned char* set;
    /* new values being built during a step */
    double *X1, *Y1, *phi1;
    unsigned char* set1;
    int* layer;             /* 0 solid, l = 1..L layer, -1 none */
    int have_new;           /* advect/extrapolate done, relabel pending */
    /* half-edge blended solid stress: x-edges and y-edges, (xx, xy, yy) */
    double *ex, *ey;
    long step;
    long cnt[ORC_CNT_N];
};

/* ------------------------------------------------------------------ */
/* pointwise definitions                                              */
/* ------------------------------------------------------------------ */

void orc_d2q9(int32_t* cx, int32_t* cy, double* w)
{
    for (int q = 0; q < NQ; q++) {
        cx[q] = CX[q];
        cy[q] = CY[q];
        w[q] = WQ[q];
    }
}

/* smoothed Heaviside H_eps(phi), Eq. (2_3_heaviside) */
double orc_heaviside(double phi, double eps)
{
    if (phi <= -eps) return 0.0;
    if (phi >= eps) return 1.0;
    return 0.5 * (1.0 + phi / eps + sin(PI * phi / eps) / PI);
}

/* equilibrium with the smooth flux correction, Eq. (2_3_feq_sfc):
 * the second-order expansion of Eq. (2_2_feq_taylor) for every direction,
 * then w_i*drho moved from each moving direction onto f_0. */
void orc_feq_sfc(double rho, double ux, double uy, double drho, double* feq)
{
    double vv = ux * ux + uy * uy;
    for (int i = 0; i < NQ; i++) {
        double vc = ux * CX[i] + uy * CY[i];
        feq[i] = WQ[i] * rho * (1.0 + vc / CS2 + (vc * vc - CS2 * vv) / (2.0 * CS2 * CS2));
    }
    double moved = 0.0;
    for (int i = 1; i < NQ; i++) moved += WQ[i] * drho;
    feq[0] += moved;
    for (int i = 1; i < NQ; i++) feq[i] -= WQ[i] * drho;
}

/* Guo forcing term, Eq. (2_2_Fi) with F a force per unit volume */
void orc_guo(double ux, double uy, double fx, double fy, double* fi)
{
    for (int i = 0; i < NQ; i++) {
        double cv = CX[i] * ux + CY[i] * uy;
        double ax = (CX[i] - ux) / CS2 + cv * CX[i] / (CS2 * CS2);
        double ay = (CY[i] - uy) / CS2 + cv * CY[i] / (CS2 * CS2);
        fi[i] = WQ[i] * (ax * fx + ay * fy);
    }
}

/* plane-strain neo-Hookean deviatoric stress, Eqs. (3_3_refmap_deformation)
 * and (3_3_solid_stress): F = J^{-1}, tau = G (F F^T - (tr(F F^T) + 1) I / 3) */
int orc_solid_stress(const double* J, double G, double detJ_min, double* tau)
{
    double det = J[0] * J[3] - J[1] * J[2];
    if (!(det > detJ_min)) {
        tau[0] = tau[1] = tau[2] = 0.0;
        return 0;
    }
    double F00 = J[3] / det, F01 = -J[1] / det;
    double F10 = -J[2] / det, F11 = J[0] / det;
    double Bxx = F00 * F00 + F01 * F01;
    double Bxy = F00 * F10 + F01 * F11;
    double Byy = F10 * F10 + F11 * F11;
    double tr = Bxx + Byy;
    tau[0] = G * (Bxx - (tr + 1.0) / 3.0);
    tau[1] = G * Bxy;
    tau[2] = G * (Byy - (tr + 1.0) / 3.0);
    return 1;
}

/* layers of the extrapolation zone (Sec. 3.2): layer 1 = non-solid nodes
 * 4-adjacent to the solid; layer l = unmarked nodes 4-adjacent to layer l-1. */
void orc_layers_mask(int32_t nx, int32_t ny, const uint8_t* solid, int32_t L, int32_t* out)
{
    for (long k = 0; k < (long)nx * ny; k++) out[k] = solid[k] ? 0 : -1;
    for (int l = 1; l <= L; l++) {
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long k = (long)j * nx + i;
                if (out[k] != -1) continue;
                int hit = 0;
                if (i > 0 && out[k - 1] == l - 1) hit = 1;
                if (i < nx - 1 && out[k + 1] == l - 1) hit = 1;
                if (j > 0 && out[k - nx] == l - 1) hit = 1;
                if (j < ny - 1 && out[k + nx] == l - 1) hit = 1;
                if (hit) out[k] = l;
            }
    }
}

/* ------------------------------------------------------------------ */
/* grid helpers                                                       */
/* ------------------------------------------------------------------ */

static int wrapi(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* index of reference-map node (i, j) on the padded grid, or -1 if outside */
static long pidx(const orc_sim* s, int i, int j)
{
    if (s->p.periodic_x) i = wrapi(i, s->p.nx);
    else if (i < -2 || i > s->p.nx + 1) return -1;
    if (s->p.periodic_y) j = wrapi(j, s->p.ny);
    else if (j < -2 || j > s->p.ny + 1) return -1;
    return (long)(j + s->oy) * s->nxp + (i + s->ox);
}

static int is_interior(const orc_sim* s, int i, int j)
{
    return i >= 0 && i < s->p.nx && j >= 0 && j < s->p.ny;
}

/* position of node index i along an axis; on a periodic axis the nearest
 * image to the body centre is used, so a reference map stays continuous */
static double node_x(const orc_sim* s, int i)
{
    double x = i + 0.5;
    if (s->p.periodic_x && s->nsolid) {
        double L = s->p.nx, d = x - s->body.cx;
        d -= L * floor(d / L + 0.5);
        x = s->body.cx + d;
    }
    return x;
}
static double node_y(const orc_sim* s, int j)
{
    double y = j + 0.5;
    if (s->p.periodic_y && s->nsolid) {
        double L = s->p.ny, d = y - s->body.cy;
        d -= L * floor(d / L + 0.5);
        y = s->body.cy + d;
    }
    return y;
}

/* Reference level set phi0(X) of a solid (Alg. 1 init and relabel).  Disc:
 * |X - c| - R.  Ellipse (semi-axes a = R and b, a axis at angle theta): the
 * paper gives no formula; we take |X - c| (1 - 1/q) with q the ellipse's
 * normalised radius sqrt((x'/a)^2 + (y'/b)^2) in the body frame, which is
 * zero exactly on the ellipse, negative inside, and equal to the disc's
 * |X - c| - R when a = b.  At the centre itself it is -min(a, b). */
double orc_phi0(const orc_solid* body, double X, double Y)
{
    double dx = X - body->cx, dy = Y - body->cy;
    double d = sqrt(dx * dx + dy * dy);
    if (body->shape != 1) return d - body->R;
    if (d == 0.0) return -(body->R < body->b ? body->R : body->b);
    double c = cos(body->theta), sn = sin(body->theta);
    double xp = c * dx + sn * dy, yp = -sn * dx + c * dy;
    double q = sqrt((xp / body->R) * (xp / body->R) + (yp / body->b) * (yp / body->b));
    return d * (1.0 - 1.0 / q);
}

static double phi0(const orc_sim* s, double X, double Y) { return orc_phi0(&s->body, X, Y); }

/* loop bounds of the reference-map domain along an axis */
static int dom_lo(int periodic) { return periodic ? 0 : -2; }
static int dom_hi(int periodic, int n) { return periodic ? n - 1 : n + 1; }

static int solid_node(const orc_sim* s, int i, int j)
{
    long k = pidx(s, i, j);
    if (k < 0 || !is_interior(s, i, j)) return 0;
    return s->set[k] && s->phi[k] < 0.0;
}

/* ------------------------------------------------------------------ */
/* lifecycle                                                          */
/* ------------------------------------------------------------------ */

orc_sim* orc_create(const orc_params* p, const orc_solid* solids, int32_t nsolid)
{
    if (!p || p->nx < 4 || p->ny < 4 || nsolid < 0 || nsolid > 1) return NULL;
    if (nsolid && (solids[0].shape < 0 || solids[0].shape > 1 || !(solids[0].R > 0.0) ||
                   (solids[0].shape == 1 && !(solids[0].b > 0.0))))
        return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->p = *p;
    s->nsolid = nsolid;
    if (nsolid) s->body = solids[0];
    s->ox = p->periodic_x ? 0 : 2;
    s->oy = p->periodic_y ? 0 : 2;
    s->nxp = p->nx + 2 * s->ox;
    s->nyp = p->ny + 2 * s->oy;
    s->N = (long)p->nx * p->ny;
    s->NP = (long)s->nxp * s->nyp;
    s->f = (double*)calloc(NQ * s->N, sizeof(double));
    s->fhat = (double*)calloc(NQ * s->N, sizeof(double));
    s->fnew = (double*)calloc(NQ * s->N, sizeof(double));
    s->rho = (double*)calloc(s->N, sizeof(double));
    s->ux = (double*)calloc(s->N, sizeof(double));
    s->uy = (double*)calloc(s->N, sizeof(double));
    s->Fx = (double*)calloc(s->N, sizeof(double));
    s->Fy = (double*)calloc(s->N, sizeof(double));
    s->X = (double*)calloc(s->NP, sizeof(double));
    s->Y = (double*)calloc(s->NP, sizeof(double));
    s->phi = (double*)calloc(s->NP, sizeof(double));
    s->set = (unsigned char*)calloc(s->NP, 1);
    s->X1 = (double*)calloc(s->NP, sizeof(double));
    s->Y1 = (double*)calloc(s->NP, sizeof(double));
    s->phi1 = (double*)calloc(s->NP, sizeof(double));
    s->set1 = (unsigned char*)calloc(s->NP, 1);
    s->layer = (int*)calloc(s->NP, sizeof(int));
    s->ex = (double*)calloc(3 * (long)(p->nx + 2) * (p->ny + 2), sizeof(double));
    s->ey = (double*)calloc(3 * (long)(p->nx + 2) * (p->ny + 2), sizeof(double));
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->f); free(s->fhat); free(s->fnew);
    free(s->rho); free(s->ux); free(s->uy); free(s->Fx); free(s->Fy);
    free(s->X); free(s->Y); free(s->phi); free(s->set);
    free(s->X1); free(s->Y1); free(s->phi1); free(s->set1);
    free(s->layer); free(s->ex); free(s->ey);
    free(s);
}

/* mark layers 1..L around the current solid set S = {interior, phi < 0} */
static void mark_layers(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny, L = s->p.layers;
    const int i0 = dom_lo(s->p.periodic_x), i1 = dom_hi(s->p.periodic_x, nx);
    const int j0 = dom_lo(s->p.periodic_y), j1 = dom_hi(s->p.periodic_y, ny);
    for (int j = j0; j <= j1; j++)
        for (int i = i0; i <= i1; i++) s->layer[pidx(s, i, j)] = solid_node(s, i, j) ? 0 : -1;
    static const int NB[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int l = 1; l <= L; l++) {
        for (int j = j0; j <= j1; j++)
            for (int i = i0; i <= i1; i++) {
                long k = pidx(s, i, j);
                if (s->layer[k] != -1) continue;
                int hit = 0;
                for (int d = 0; d < 4; d++) {
                    long kn = pidx(s, i + NB[d][0], j + NB[d][1]);
                    if (kn >= 0 && s->layer[kn] == l - 1) hit = 1;
                }
                if (hit) s->layer[k] = l;
            }
    }
}

void orc_init(orc_sim* s, const double* u0)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const int i0 = dom_lo(s->p.periodic_x), i1 = dom_hi(s->p.periodic_x, nx);
    const int j0 = dom_lo(s->p.periodic_y), j1 = dom_hi(s->p.periodic_y, ny);
    memset(s->set, 0, s->NP);
    memset(s->cnt, 0, sizeof(s->cnt));
    s->step = 0;
    s->have_new = 0;
    if (s->nsolid) {
        /* solid set from phi0(x) (Alg. 1: label by phi(xi_0) with xi_0 = x) */
        for (int j = j0; j <= j1; j++)
            for (int i = i0; i <= i1; i++) {
                long k = pidx(s, i, j);
                s->X[k] = node_x(s, i);
                s->Y[k] = node_y(s, j);
                s->phi[k] = phi0(s, s->X[k], s->Y[k]);
                s->set[k] = 1;
            }
        mark_layers(s);
        /* xi_0 = x on the solid and its extrapolation zone (Sec. 3) */
        for (long k = 0; k < s->NP; k++) {
            s->set[k] = s->layer[k] >= 0;
            if (!s->set[k]) {
                s->X[k] = s->Y[k] = NAN;
                s->phi[k] = INFINITY;
            }
        }
    } else {
        for (long k = 0; k < s->NP; k++) {
            s->X[k] = s->Y[k] = NAN;
            s->phi[k] = INFINITY;
        }
    }
    /* global density, Eq. (2_4_smooth_density); velocity v0; f = f^eq */
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            long n = (long)j * nx + i;
            long k = pidx(s, i, j);
            double H = s->set[k] ? orc_heaviside(s->phi[k], s->p.eps) : 1.0;
            double rs = s->nsolid ? s->body.rho_s : s->p.rho_f;
            s->rho[n] = H * s->p.rho_f + (1.0 - H) * rs;
            s->ux[n] = u0 ? u0[n] : 0.0;
            s->uy[n] = u0 ? u0[s->N + n] : 0.0;
            double drho = s->rho[n] - s->p.rho_f; /* Eq. (2_3_drho) with rho = rho_t */
            double feq[NQ];
            orc_feq_sfc(s->rho[n], s->ux[n], s->uy[n], drho, feq);
            for (int q = 0; q < NQ; q++) s->f[q * s->N + n] = feq[q];
            s->Fx[n] = s->Fy[n] = 0.0;
        }
}

/* ------------------------------------------------------------------ */
/* RMT phases                                                         */
/* ------------------------------------------------------------------ */

/* one-sided second-order upwind derivative, Eq. (3_1_eno), along (di, dj);
 * vel > 0 uses the nodes behind, vel < 0 the nodes ahead.  Returns 0 if a
 * stencil node holds no reference map. */
static int upwind(const orc_sim* s, int i, int j, int di, int dj, double vel,
                  double* dX, double* dY)
{
    *dX = *dY = 0.0;
    if (vel == 0.0) return 1;
    int sg = vel > 0.0 ? 1 : -1;
    long k0 = pidx(s, i, j);
    long k1 = pidx(s, i - sg * di, j - sg * dj);
    long k2 = pidx(s, i - 2 * sg * di, j - 2 * sg * dj);
    if (k1 < 0 || k2 < 0 || !s->set[k1] || !s->set[k2]) return 0;
    if (sg > 0) {
        *dX = (3.0 * s->X[k0] - 4.0 * s->X[k1] + s->X[k2]) / 2.0;
        *dY = (3.0 * s->Y[k0] - 4.0 * s->Y[k1] + s->Y[k2]) / 2.0;
    } else {
        *dX = (-3.0 * s->X[k0] + 4.0 * s->X[k1] - s->X[k2]) / 2.0;
        *dY = (-3.0 * s->Y[k0] + 4.0 * s->Y[k1] - s->Y[k2]) / 2.0;
    }
    return 1;
}

/* Sec. 3.1, Eq. (3_1_refmap_adv): xi^{n+1} = xi^n - (u d/dx + v d/dy) xi^n on
 * solid nodes (phi^n < 0, blur zone excluded), forward Euler, dt = 1. */
void orc_phase_advect(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    memset(s->set1, 0, s->NP);
    long miss = 0;
#pragma omp parallel for reduction(+ : miss) schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            if (!solid_node(s, i, j)) continue;
            long k = pidx(s, i, j);
            long n = (long)j * nx + i;
            double u = s->ux[n], v = s->uy[n];
            double dXx, dYx, dXy, dYy;
            int okx = upwind(s, i, j, 1, 0, u, &dXx, &dYx);
            int oky = upwind(s, i, j, 0, 1, v, &dXy, &dYy);
            if (!okx || !oky) {
                miss++;
                s->X1[k] = s->X[k];
                s->Y1[k] = s->Y[k];
            } else {
                s->X1[k] = s->X[k] - (u * dXx + v * dXy);
                s->Y1[k] = s->Y[k] - (u * dYx + v * dYy);
            }
            s->set1[k] = 1;
        }
    s->cnt[ORC_CNT_ADVECT_MISS] += miss;
    s->have_new = 1;
}

static double det3(double a00, double a01, double a02, double a10, double a11, double a12,
                   double a20, double a21, double a22)
{
    return a00 * (a11 * a22 - a12 * a21) - a01 * (a10 * a22 - a12 * a20) +
           a02 * (a10 * a21 - a11 * a20);
}

/* extrapolate one target node t = (i, j) of layer l (Sec. 3.2 steps (i)-(iii)) */
static int extrap_target(orc_sim* s, int i, int j, int l)
{
    long kt = pidx(s, i, j);
    /* approximated outward surface normal of phi^n at the target (l <= 2) */
    int use_n = 0;
    double nxh = 0.0, nyh = 0.0;
    if (l <= 2) {
        long ke = pidx(s, i + 1, j), kw = pidx(s, i - 1, j);
        long kn = pidx(s, i, j + 1), ks = pidx(s, i, j - 1);
        if (ke >= 0 && kw >= 0 && kn >= 0 && ks >= 0 && s->set[ke] && s->set[kw] &&
            s->set[kn] && s->set[ks]) {
            double gx = (s->phi[ke] - s->phi[kw]) / 2.0;
            double gy = (s->phi[kn] - s->phi[ks]) / 2.0;
            double g = sqrt(gx * gx + gy * gy);
            if (g > 0.0) {
                nxh = gx / g;
                nyh = gy / g;
                use_n = 1;
            }
        }
    }
    for (int r = 2; r <= s->p.r_max; r++) {
        /* step (i): count valid nodes in the scan window */
        int count = 0;
        for (int b = -r; b <= r; b++)
            for (int a = -r; a <= r; a++) {
                long k = pidx(s, i + a, j + b);
                if (k < 0) continue;
                int lk = s->layer[k];
                if (lk == 0 || (lk > 0 && lk < l && s->set1[k])) count++;
            }
        if (count < 3) continue;
        /* step (ii): weighted least-squares fit xi = A x + B y + C, in
         * coordinates centred at the target, weights of Eq. (3_2_extrap_weight) */
        double M00 = 0, M01 = 0, M02 = 0, M11 = 0, M12 = 0, M22 = 0;
        double bX0 = 0, bX1 = 0, bX2 = 0, bY0 = 0, bY1 = 0, bY2 = 0;
        for (int b = -r; b <= r; b++)
            for (int a = -r; a <= r; a++) {
                long k = pidx(s, i + a, j + b);
                if (k < 0) continue;
                int lk = s->layer[k];
                if (!(lk == 0 || (lk > 0 && lk < l && s->set1[k]))) continue;
                double w = ldexp(1.0, -(abs(a) + abs(b)));
                if (l <= 2 && use_n) {
                    /* d = x_target - x_valid */
                    double ddx = -(double)a, ddy = -(double)b;
                    double dn = (ddx * nxh + ddy * nyh) / sqrt(ddx * ddx + ddy * ddy);
                    w = dn * w > 0.0 ? dn * w : 0.0;
                }
                double dx = a, dy = b;
                M00 += w * dx * dx; M01 += w * dx * dy; M02 += w * dx;
                M11 += w * dy * dy; M12 += w * dy; M22 += w;
                bX0 += w * dx * s->X1[k]; bX1 += w * dy * s->X1[k]; bX2 += w * s->X1[k];
                bY0 += w * dx * s->Y1[k]; bY1 += w * dy * s->Y1[k]; bY2 += w * s->Y1[k];
            }
        double det = det3(M00, M01, M02, M01, M11, M12, M02, M12, M22);
        if (!(det > s->p.det_rel * M22 * M22 * M22)) continue; /* ill-defined: grow r */
        /* step (iii): the fitted map at the target is its intercept C (Cramer) */
        s->X1[kt] = det3(M00, M01, bX0, M01, M11, bX1, M02, M12, bX2) / det;
        s->Y1[kt] = det3(M00, M01, bY0, M01, M11, bY1, M02, M12, bY2) / det;
        s->set1[kt] = 1;
        return 1;
    }
    return 0;
}

/* Sec. 3.2: layers around S^n, then layer-by-layer LSQ extrapolation.  Valid
 * nodes are solid nodes or already-set nodes of earlier layers only, so the
 * targets of one layer are independent of each other. */
void orc_phase_extrapolate(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const int i0 = dom_lo(s->p.periodic_x), i1 = dom_hi(s->p.periodic_x, nx);
    const int j0 = dom_lo(s->p.periodic_y), j1 = dom_hi(s->p.periodic_y, ny);
    mark_layers(s);
    const int W = i1 - i0 + 1, H = j1 - j0 + 1;
    for (int l = 1; l <= s->p.layers; l++) {
        long fail = 0;
#pragma omp parallel for reduction(+ : fail) schedule(dynamic, 4)
        for (int jj = 0; jj < H; jj++) {
            int j = s->p.reverse_order ? j1 - jj : j0 + jj;
            for (int ii = 0; ii < W; ii++) {
                int i = s->p.reverse_order ? i1 - ii : i0 + ii;
                long k = pidx(s, i, j);
                if (s->layer[k] != l) continue;
                if (!extrap_target(s, i, j, l)) fail++;
            }
        }
        s->cnt[ORC_CNT_EXTRAP_FAIL] += fail;
    }
}

/* Sec. 3.2 end / Alg. 1: recompute phi = phi0(xi^{n+1}) on every node that
 * holds a reference map, then make the new map the current one. */
void orc_phase_relabel(orc_sim* s)
{
    for (long k = 0; k < s->NP; k++) {
        if (s->set1[k]) {
            s->phi1[k] = phi0(s, s->X1[k], s->Y1[k]);
        } else {
            s->X1[k] = s->Y1[k] = NAN;
            s->phi1[k] = INFINITY;
        }
    }
    double* t;
    unsigned char* tc;
    t = s->X; s->X = s->X1; s->X1 = t;
    t = s->Y; s->Y = s->Y1; s->Y1 = t;
    t = s->phi; s->phi = s->phi1; s->phi1 = t;
    tc = s->set; s->set = s->set1; s->set1 = tc;
    s->have_new = 0;
}

/* blended stress (1 - H(phi_e)) tau_s on the half-edge between nodes a and b.
 * dir = 0: x-edge (i-1/2, j) with a = (i-1, j), b = (i, j);
 * dir = 1: y-edge (i, j-1/2) with a = (i, j-1), b = (i, j).
 * Gradients of Eq. (3_3_refmap_jacobian); the tangential one averages the
 * four nodes beside the edge. */
static void edge_stress(orc_sim* s, int i, int j, int dir, double* out, long* miss, long* sing)
{
    out[0] = out[1] = out[2] = 0.0;
    if (!s->nsolid) return;
    int ia = dir == 0 ? i - 1 : i, ja = dir == 0 ? j : j - 1;
    long ka = pidx(s, ia, ja), kb = pidx(s, i, j);
    if (ka < 0 || kb < 0 || !s->set[ka] || !s->set[kb]) return;
    double phie = 0.5 * (s->phi[ka] + s->phi[kb]);
    double lam = 1.0 - orc_heaviside(phie, s->p.eps);
    if (!(lam > 0.0)) return;
    long k1, k2, k3, k4; /* (+t, a), (+t, b) ... side nodes */
    double J[4];
    if (dir == 0) {
        k1 = pidx(s, i, j + 1); k2 = pidx(s, i - 1, j + 1);
        k3 = pidx(s, i, j - 1); k4 = pidx(s, i - 1, j - 1);
    } else {
        k1 = pidx(s, i + 1, j); k2 = pidx(s, i + 1, j - 1);
        k3 = pidx(s, i - 1, j); k4 = pidx(s, i - 1, j - 1);
    }
    if (k1 < 0 || k2 < 0 || k3 < 0 || k4 < 0 || !s->set[k1] || !s->set[k2] || !s->set[k3] ||
        !s->set[k4]) {
        (*miss)++;
        return;
    }
    double nX = s->X[kb] - s->X[ka], nY = s->Y[kb] - s->Y[ka];
    double tX = (s->X[k1] + s->X[k2] - s->X[k3] - s->X[k4]) / 4.0;
    double tY = (s->Y[k1] + s->Y[k2] - s->Y[k3] - s->Y[k4]) / 4.0;
    if (dir == 0) {
        J[0] = nX; J[1] = tX; J[2] = nY; J[3] = tY;
    } else {
        J[0] = tX; J[1] = nX; J[2] = tY; J[3] = nY;
    }
    double tau[3];
    if (!orc_solid_stress(J, s->body.G, s->p.detJ_min, tau)) {
        (*sing)++;
        return;
    }
    out[0] = lam * tau[0];
    out[1] = lam * tau[1];
    out[2] = lam * tau[2];
}

/* half-edge arrays: x-edge (i-1/2, j) and y-edge (i, j-1/2) stored at
 * ((j+1)*(nx+2) + i+1), for i = 0..nx, j = 0..ny */
static long eidx(const orc_sim* s, int i, int j) { return (long)(j + 1) * (s->p.nx + 2) + (i + 1); }

/* all half-edge stresses touching interior nodes */
static void compute_edges(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    long miss = 0, sing = 0;
#pragma omp parallel for reduction(+ : miss, sing) schedule(static)
    for (int j = 0; j <= ny; j++)
        for (int i = 0; i <= nx; i++) {
            if (j < ny) edge_stress(s, i, j, 0, &s->ex[3 * eidx(s, i, j)], &miss, &sing);
            if (i < nx) edge_stress(s, i, j, 1, &s->ey[3 * eidx(s, i, j)], &miss, &sing);
        }
    s->cnt[ORC_CNT_STRESS_MISS] += miss;
    s->cnt[ORC_CNT_DETJ] += sing;
}

/* stresses of the four half-edges around interior node (i, j): L, R, B, T */
static void node_edges(const orc_sim* s, int i, int j, const double** L, const double** R,
                       const double** B, const double** T)
{
    int ir = i + 1, jt = j + 1;
    if (s->p.periodic_x && ir == s->p.nx) ir = 0;
    if (s->p.periodic_y && jt == s->p.ny) jt = 0;
    *L = &s->ex[3 * eidx(s, i, j)];
    *R = &s->ex[3 * eidx(s, ir, j)];
    *B = &s->ey[3 * eidx(s, i, j)];
    *T = &s->ey[3 * eidx(s, i, jt)];
}

/* Eq. (3_3_div_solid_stress) assembled into the force density of
 * Eq. (2_4_F_divs): div[(1-H) tau_s] + (1-H) f_ext,s + H f_ext,f, with the
 * solid's external force in the buoyancy form (rho_s - rho_f) g of Sec. 4.3
 * and f_ext,f a uniform force density on the fluid. */
void orc_phase_force(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    compute_edges(s);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            long n = (long)j * nx + i;
            const double *L, *R, *B, *T;
            node_edges(s, i, j, &L, &R, &B, &T);
            double fx = (R[0] - L[0]) + (T[1] - B[1]);
            double fy = (R[1] - L[1]) + (T[2] - B[2]);
            long k = pidx(s, i, j);
            double H = 1.0;
            if (s->nsolid && s->set[k]) {
                H = orc_heaviside(s->phi[k], s->p.eps);
                fx += (1.0 - H) * (s->body.rho_s - s->p.rho_f) * s->p.gx;
                fy += (1.0 - H) * (s->body.rho_s - s->p.rho_f) * s->p.gy;
            }
            fx += H * s->p.fext_x;
            fy += H * s->p.fext_y;
            s->Fx[n] = fx;
            s->Fy[n] = fy;
        }
}

/* ------------------------------------------------------------------ */
/* LB phases                                                          */
/* ------------------------------------------------------------------ */

/* Sec. 3.4: SFC equilibrium with drho of Eq. (2_3_drho) from phi^{n+1}, BGK
 * collision, Guo forcing with F^n; then Sec. 3.5 walls and streaming. */
void orc_phase_collide_stream(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const long N = s->N;
    const double tau = s->p.tau;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            long n = (long)j * nx + i;
            long k = pidx(s, i, j);
            double drho = 0.0;
            if (s->nsolid && s->set[k])
                drho = (1.0 - orc_heaviside(s->phi[k], s->p.eps)) * (s->body.rho_s - s->p.rho_f);
            double feq[NQ], Fi[NQ];
            orc_feq_sfc(s->rho[n], s->ux[n], s->uy[n], drho, feq);
            orc_guo(s->ux[n], s->uy[n], s->Fx[n], s->Fy[n], Fi);
            for (int q = 0; q < NQ; q++) {
                double fq = s->f[q * N + n];
                s->fhat[q * N + n] = fq - (fq - feq[q]) / tau + (1.0 - 1.0 / (2.0 * tau)) * Fi[q];
            }
        }
    /* streaming; a population leaving through a wall is reflected back into
     * the opposite direction at its own node (halfway bounce-back).  The top
     * buffer row, corners included, moves with the lid velocity u_w, which
     * adds -2 w_i rho_w (c_i . u_w) / c_s^2 with rho_w the node's density. */
    static const int OPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            long n = (long)j * nx + i;
            for (int q = 0; q < NQ; q++) {
                int id = i + CX[q], jd = j + CY[q];
                if (s->p.periodic_x) id = wrapi(id, nx);
                if (s->p.periodic_y) jd = wrapi(jd, ny);
                double fh = s->fhat[q * N + n];
                if (is_interior(s, id, jd)) {
                    s->fnew[q * N + (long)jd * nx + id] = fh;
                } else {
                    double uw = (jd == ny) ? s->p.lid_ux : 0.0;
                    double cu = CX[q] * uw;
                    s->fnew[OPP[q] * N + n] = fh - 2.0 * WQ[q] * s->rho[n] * cu / CS2;
                }
            }
        }
    double* t = s->f;
    s->f = s->fnew;
    s->fnew = t;
}

/* Sec. 3.4 moments: rho = sum f_i, u = (sum c_i f_i)/rho + F/(2 rho) */
void orc_phase_moments(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const long N = s->N;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            long n = (long)j * nx + i;
            const double* f = s->f + n;
            double f0 = f[0], f1 = f[N], f2 = f[2 * N], f3 = f[3 * N], f4 = f[4 * N];
            double f5 = f[5 * N], f6 = f[6 * N], f7 = f[7 * N], f8 = f[8 * N];
            double rho = f0 + f1 + f2 + f3 + f4 + f5 + f6 + f7 + f8;
            s->rho[n] = rho;
            s->ux[n] = (f1 + f5 + f8 - f3 - f6 - f7) / rho + s->Fx[n] / (2.0 * rho);
            s->uy[n] = (f2 + f5 + f6 - f4 - f7 - f8) / rho + s->Fy[n] / (2.0 * rho);
        }
}

/* Alg. 1 main loop */
void orc_step(orc_sim* s, int64_t n)
{
    for (int64_t t = 0; t < n; t++) {
        if (s->nsolid) {
            orc_phase_advect(s);
            orc_phase_extrapolate(s);
            orc_phase_relabel(s);
        }
        orc_phase_force(s);
        orc_phase_collide_stream(s);
        orc_phase_moments(s);
        s->step++;
    }
}

/* ------------------------------------------------------------------ */
/* reads                                                              */
/* ------------------------------------------------------------------ */

int64_t orc_step_count(const orc_sim* s) { return s->step; }

void orc_read_macro(const orc_sim* s, double* rho, double* ux, double* uy)
{
    for (long n = 0; n < s->N; n++) {
        if (rho) rho[n] = s->rho[n];
        if (ux) ux[n] = s->ux[n];
        if (uy) uy[n] = s->uy[n];
    }
}

void orc_read_populations(const orc_sim* s, double* f9)
{
    memcpy(f9, s->f, sizeof(double) * NQ * s->N);
}

void orc_read_force(const orc_sim* s, double* fx, double* fy)
{
    memcpy(fx, s->Fx, sizeof(double) * s->N);
    memcpy(fy, s->Fy, sizeof(double) * s->N);
}

void orc_read_refmap(const orc_sim* s, double* X, double* Y, double* phi)
{
    for (int j = 0; j < s->p.ny; j++)
        for (int i = 0; i < s->p.nx; i++) {
            long n = (long)j * s->p.nx + i, k = pidx(s, i, j);
            int ok = s->set[k];
            if (X) X[n] = ok ? s->X[k] : NAN;
            if (Y) Y[n] = ok ? s->Y[k] : NAN;
            if (phi) phi[n] = ok ? s->phi[k] : NAN;
        }
}

/* the padded layout used by the read/set calls: [(ny+4)][(nx+4)], node (i, j)
 * at ((j+2)*(nx+4) + i+2); on periodic axes the pad cells are left NaN */
static long ext_idx(const orc_sim* s, int i, int j) { return (long)(j + 2) * (s->p.nx + 4) + (i + 2); }

void orc_read_refmap_padded(const orc_sim* s, double* X, double* Y, double* phi)
{
    long NE = (long)(s->p.nx + 4) * (s->p.ny + 4);
    for (long e = 0; e < NE; e++) X[e] = Y[e] = phi[e] = NAN;
    for (int j = -2; j <= s->p.ny + 1; j++)
        for (int i = -2; i <= s->p.nx + 1; i++) {
            if ((s->p.periodic_x && (i < 0 || i >= s->p.nx)) ||
                (s->p.periodic_y && (j < 0 || j >= s->p.ny)))
                continue;
            long k = pidx(s, i, j), e = ext_idx(s, i, j);
            if (s->set[k]) {
                X[e] = s->X[k];
                Y[e] = s->Y[k];
                phi[e] = s->phi[k];
            }
        }
}

void orc_read_layers_padded(const orc_sim* s, int32_t* layer)
{
    long NE = (long)(s->p.nx + 4) * (s->p.ny + 4);
    for (long e = 0; e < NE; e++) layer[e] = -1;
    for (int j = -2; j <= s->p.ny + 1; j++)
        for (int i = -2; i <= s->p.nx + 1; i++) {
            if ((s->p.periodic_x && (i < 0 || i >= s->p.nx)) ||
                (s->p.periodic_y && (j < 0 || j >= s->p.ny)))
                continue;
            layer[ext_idx(s, i, j)] = s->layer[pidx(s, i, j)];
        }
}

void orc_set_refmap_padded(orc_sim* s, const double* X, const double* Y)
{
    for (int j = -2; j <= s->p.ny + 1; j++)
        for (int i = -2; i <= s->p.nx + 1; i++) {
            if ((s->p.periodic_x && (i < 0 || i >= s->p.nx)) ||
                (s->p.periodic_y && (j < 0 || j >= s->p.ny)))
                continue;
            long k = pidx(s, i, j), e = ext_idx(s, i, j);
            if (isnan(X[e])) {
                s->set[k] = 0;
                s->X[k] = s->Y[k] = NAN;
                s->phi[k] = INFINITY;
            } else {
                s->set[k] = 1;
                s->X[k] = X[e];
                s->Y[k] = Y[e];
                s->phi[k] = s->nsolid ? phi0(s, X[e], Y[e]) : INFINITY;
            }
        }
}

void orc_set_populations(orc_sim* s, const double* f9)
{
    memcpy(s->f, f9, sizeof(double) * NQ * s->N);
}

void orc_set_moments(orc_sim* s, const double* rho, const double* ux, const double* uy)
{
    for (long n = 0; n < s->N; n++) {
        if (rho) s->rho[n] = rho[n];
        if (ux) s->ux[n] = ux[n];
        if (uy) s->uy[n] = uy[n];
    }
}

void orc_read_stress(orc_sim* s, double* sxx, double* sxy, double* syy)
{
    compute_edges(s);
    for (int j = 0; j < s->p.ny; j++)
        for (int i = 0; i < s->p.nx; i++) {
            long n = (long)j * s->p.nx + i;
            const double *L, *R, *B, *T;
            node_edges(s, i, j, &L, &R, &B, &T);
            sxx[n] = (L[0] + R[0] + B[0] + T[0]) / 4.0;
            sxy[n] = (L[1] + R[1] + B[1] + T[1]) / 4.0;
            syy[n] = (L[2] + R[2] + B[2] + T[2]) / 4.0;
        }
}

void orc_counters(const orc_sim* s, int64_t* out)
{
    for (int c = 0; c < ORC_CNT_N; c++) out[c] = s->cnt[c];
}

void orc_diag(const orc_sim* s, double* out)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const long N = s->N;
    double mass = 0, px = 0, py = 0, lw = 0, lx = 0, ly = 0, dx = 0, dy = 0, umax = 0;
    double nsol = 0, nband = 0;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            long n = (long)j * nx + i;
            double rho = 0, jx = 0, jy = 0;
            for (int q = 0; q < NQ; q++) {
                double fq = s->f[q * N + n];
                rho += fq;
                jx += CX[q] * fq;
                jy += CY[q] * fq;
            }
            mass += rho;
            px += jx + 0.5 * s->Fx[n];
            py += jy + 0.5 * s->Fy[n];
            double um = sqrt(s->ux[n] * s->ux[n] + s->uy[n] * s->uy[n]);
            if (um > umax) umax = um;
            long k = pidx(s, i, j);
            if (s->nsolid && s->set[k]) {
                nband += 1;
                if (s->phi[k] < 0) nsol += 1;
                double lam = 1.0 - orc_heaviside(s->phi[k], s->p.eps);
                double x = node_x(s, i), y = node_y(s, j);
                lw += lam;
                lx += lam * x;
                ly += lam * y;
                dx += lam * (x - s->X[k]);
                dy += lam * (y - s->Y[k]);
            }
        }
    out[0] = mass;
    out[1] = px;
    out[2] = py;
    out[3] = lw > 0 ? lx / lw : NAN;
    out[4] = lw > 0 ? ly / lw : NAN;
    out[5] = lw > 0 ? dx / lw : NAN;
    out[6] = lw > 0 ? dy / lw : NAN;
    out[7] = umax;
    out[8] = nsol;
    out[9] = nband;
}
