/*
 * lbrmt_oracle.c -- TEST INFRASTRUCTURE ONLY (see lbrmt_oracle.h).
 *
 * Plain FP64 CPU implementation of the LBRMT time step (Alg. 1 of Sun &
 * Rycroft), written for clarity, not speed: every step is a separate loop over
 * the whole grid, in the order of Alg. 1, with the formulas in the paper's own
 * notation.  OpenMP only splits independent per-node loops; nothing is fused,
 * blocked or reordered.  Built with -ffp-contract=off.
 *
 * Several solids (Sec. 3.6): every solid keeps its own reference map, level
 * set and extrapolation zone on the whole padded grid (the role of the
 * paper's per-node list of maps), each advected, extrapolated and relabelled
 * exactly as a single solid is.  They meet only in the stress, force and
 * density of the shared lattice.
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

/* one solid's reference map state on the padded grid */
typedef struct {
    orc_solid body;
    double *X, *Y, *phi;    /* xi^n, phi^n                                 */
    unsigned char* set;     /* node holds a value of this map              */
    double *X1, *Y1, *phi1; /* new values being built during a step        */
    unsigned char* set1;
    int* layer;             /* 0 solid, l = 1..L layer, -1 none            */
} orc_map;

struct orc_sim {
    orc_params p;
    int nsolid;
    orc_map* m;             /* nsolid maps                                 */
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
    int have_new;           /* advect/extrapolate done, relabel pending */
    /* half-edge global solid stress (blend of all solids plus contact):
     * x-edges and y-edges, (xx, xy, yy) */
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

/* position of node index i along an axis, seen by solid m; on a periodic
 * axis the nearest image to the solid's reference centre is used, so its
 * reference map stays continuous across the boundary */
static double node_x(const orc_sim* s, const orc_map* m, int i)
{
    double x = i + 0.5;
    if (s->p.periodic_x) {
        double L = s->p.nx, d = x - m->body.cx;
        d -= L * floor(d / L + 0.5);
        x = m->body.cx + d;
    }
    return x;
}
static double node_y(const orc_sim* s, const orc_map* m, int j)
{
    double y = j + 0.5;
    if (s->p.periodic_y) {
        double L = s->p.ny, d = y - m->body.cy;
        d -= L * floor(d / L + 0.5);
        y = m->body.cy + d;
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

static double phi0(const orc_map* m, double X, double Y) { return orc_phi0(&m->body, X, Y); }

/* loop bounds of the reference-map domain along an axis */
static int dom_lo(int periodic) { return periodic ? 0 : -2; }
static int dom_hi(int periodic, int n) { return periodic ? n - 1 : n + 1; }

static int solid_node(const orc_sim* s, const orc_map* m, int i, int j)
{
    long k = pidx(s, i, j);
    if (k < 0 || !is_interior(s, i, j)) return 0;
    return m->set[k] && m->phi[k] < 0.0;
}

/* solid fraction lambda = 1 - H(phi) of map m at padded index k (0 where the
 * map holds no value) */
static double lambda_at(const orc_sim* s, const orc_map* m, long k)
{
    return m->set[k] ? 1.0 - orc_heaviside(m->phi[k], s->p.eps) : 0.0;
}

/* ------------------------------------------------------------------ */
/* lifecycle                                                          */
/* ------------------------------------------------------------------ */

static int solid_ok(const orc_solid* b)
{
    if (b->shape < 0 || b->shape > 1 || !(b->R > 0.0)) return 0;
    if (b->shape == 1 && !(b->b > 0.0)) return 0;
    return b->rho_s > 0.0 && b->G >= 0.0;
}

orc_sim* orc_create(const orc_params* p, const orc_solid* solids, int32_t nsolid)
{
    if (!p || p->nx < 4 || p->ny < 4 || nsolid < 0 || nsolid > ORC_MAX_SOLIDS) return NULL;
    if (p->lid_rho_mode != 0 && p->lid_rho_mode != 1) return NULL;
    if (nsolid && !solids) return NULL;
    for (int b = 0; b < nsolid; b++)
        if (!solid_ok(&solids[b])) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->p = *p;
    s->nsolid = nsolid;
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
    s->m = (orc_map*)calloc(nsolid > 0 ? nsolid : 1, sizeof(orc_map));
    for (int b = 0; b < nsolid; b++) {
        orc_map* m = &s->m[b];
        m->body = solids[b];
        m->X = (double*)calloc(s->NP, sizeof(double));
        m->Y = (double*)calloc(s->NP, sizeof(double));
        m->phi = (double*)calloc(s->NP, sizeof(double));
        m->set = (unsigned char*)calloc(s->NP, 1);
        m->X1 = (double*)calloc(s->NP, sizeof(double));
        m->Y1 = (double*)calloc(s->NP, sizeof(double));
        m->phi1 = (double*)calloc(s->NP, sizeof(double));
        m->set1 = (unsigned char*)calloc(s->NP, 1);
        m->layer = (int*)calloc(s->NP, sizeof(int));
    }
    s->ex = (double*)calloc(3 * (long)(p->nx + 2) * (p->ny + 2), sizeof(double));
    s->ey = (double*)calloc(3 * (long)(p->nx + 2) * (p->ny + 2), sizeof(double));
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->f); free(s->fhat); free(s->fnew);
    free(s->rho); free(s->ux); free(s->uy); free(s->Fx); free(s->Fy);
    for (int b = 0; b < s->nsolid; b++) {
        orc_map* m = &s->m[b];
        free(m->X); free(m->Y); free(m->phi); free(m->set);
        free(m->X1); free(m->Y1); free(m->phi1); free(m->set1);
        free(m->layer);
    }
    free(s->m);
    free(s->ex); free(s->ey);
    free(s);
}

/* mark layers 1..L around solid m's current solid set S = {interior, phi < 0} */
static void mark_layers(orc_sim* s, orc_map* m)
{
    const int nx = s->p.nx, ny = s->p.ny, L = s->p.layers;
    const int i0 = dom_lo(s->p.periodic_x), i1 = dom_hi(s->p.periodic_x, nx);
    const int j0 = dom_lo(s->p.periodic_y), j1 = dom_hi(s->p.periodic_y, ny);
    for (int j = j0; j <= j1; j++)
        for (int i = i0; i <= i1; i++) m->layer[pidx(s, i, j)] = solid_node(s, m, i, j) ? 0 : -1;
    static const int NB[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int l = 1; l <= L; l++) {
        for (int j = j0; j <= j1; j++)
            for (int i = i0; i <= i1; i++) {
                long k = pidx(s, i, j);
                if (m->layer[k] != -1) continue;
                int hit = 0;
                for (int d = 0; d < 4; d++) {
                    long kn = pidx(s, i + NB[d][0], j + NB[d][1]);
                    if (kn >= 0 && m->layer[kn] == l - 1) hit = 1;
                }
                if (hit) m->layer[k] = l;
            }
    }
}

/* Density of the mixture at padded index k, Eq. (2_4_smooth_density) for
 * one solid; for several, each solid's fraction replaces that much fluid and
 * the fractions are normalised where they sum above one:
 * rho_f + sum_i lambda_i (rho_s,i - rho_f) / max(1, sum_i lambda_i). */
static double mixture_drho(const orc_sim* s, long k)
{
    double lsum = 0.0, acc = 0.0;
    for (int b = 0; b < s->nsolid; b++) {
        const orc_map* m = &s->m[b];
        if (!m->set[k]) continue;
        double lam = 1.0 - orc_heaviside(m->phi[k], s->p.eps);
        lsum += lam;
        acc += lam * (m->body.rho_s - s->p.rho_f);
    }
    return lsum > 1.0 ? acc / lsum : acc;
}

void orc_init(orc_sim* s, const double* u0)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const int i0 = dom_lo(s->p.periodic_x), i1 = dom_hi(s->p.periodic_x, nx);
    const int j0 = dom_lo(s->p.periodic_y), j1 = dom_hi(s->p.periodic_y, ny);
    memset(s->cnt, 0, sizeof(s->cnt));
    s->step = 0;
    s->have_new = 0;
    for (int b = 0; b < s->nsolid; b++) {
        orc_map* m = &s->m[b];
        /* solid set from phi0(x) (Alg. 1: label by phi(xi_0) with xi_0 = x) */
        for (int j = j0; j <= j1; j++)
            for (int i = i0; i <= i1; i++) {
                long k = pidx(s, i, j);
                m->X[k] = node_x(s, m, i);
                m->Y[k] = node_y(s, m, j);
                m->phi[k] = phi0(m, m->X[k], m->Y[k]);
                m->set[k] = 1;
            }
        mark_layers(s, m);
        /* xi_0 = x on the solid and its extrapolation zone (Sec. 3) */
        for (long k = 0; k < s->NP; k++) {
            m->set[k] = m->layer[k] >= 0;
            if (!m->set[k]) {
                m->X[k] = m->Y[k] = NAN;
                m->phi[k] = INFINITY;
            }
        }
    }
    /* global density, Eq. (2_4_smooth_density) (several solids: rho_f plus
     * the mixture term); velocity v0; f = f^eq */
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            long n = (long)j * nx + i;
            long k = pidx(s, i, j);
            double drho; /* Eq. (2_3_drho) with rho = rho_t */
            if (s->nsolid <= 1) {
                const orc_map* m = s->nsolid ? &s->m[0] : NULL;
                double H = (m && m->set[k]) ? orc_heaviside(m->phi[k], s->p.eps) : 1.0;
                double rs = m ? m->body.rho_s : s->p.rho_f;
                s->rho[n] = H * s->p.rho_f + (1.0 - H) * rs;
                drho = s->rho[n] - s->p.rho_f;
            } else {
                drho = mixture_drho(s, k);
                s->rho[n] = s->p.rho_f + drho;
            }
            s->ux[n] = u0 ? u0[n] : 0.0;
            s->uy[n] = u0 ? u0[s->N + n] : 0.0;
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
static int upwind(const orc_sim* s, const orc_map* m, int i, int j, int di, int dj, double vel,
                  double* dX, double* dY)
{
    *dX = *dY = 0.0;
    if (vel == 0.0) return 1;
    int sg = vel > 0.0 ? 1 : -1;
    long k0 = pidx(s, i, j);
    long k1 = pidx(s, i - sg * di, j - sg * dj);
    long k2 = pidx(s, i - 2 * sg * di, j - 2 * sg * dj);
    if (k1 < 0 || k2 < 0 || !m->set[k1] || !m->set[k2]) return 0;
    if (sg > 0) {
        *dX = (3.0 * m->X[k0] - 4.0 * m->X[k1] + m->X[k2]) / 2.0;
        *dY = (3.0 * m->Y[k0] - 4.0 * m->Y[k1] + m->Y[k2]) / 2.0;
    } else {
        *dX = (-3.0 * m->X[k0] + 4.0 * m->X[k1] - m->X[k2]) / 2.0;
        *dY = (-3.0 * m->Y[k0] + 4.0 * m->Y[k1] - m->Y[k2]) / 2.0;
    }
    return 1;
}

/* Sec. 3.1, Eq. (3_1_refmap_adv): xi^{n+1} = xi^n - (u d/dx + v d/dy) xi^n on
 * solid nodes (phi^n < 0, blur zone excluded), forward Euler, dt = 1; every
 * solid's map is advected by the one velocity field. */
void orc_phase_advect(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    long miss = 0;
    for (int b = 0; b < s->nsolid; b++) {
        orc_map* m = &s->m[b];
        memset(m->set1, 0, s->NP);
#pragma omp parallel for reduction(+ : miss) schedule(static)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                if (!solid_node(s, m, i, j)) continue;
                long k = pidx(s, i, j);
                long n = (long)j * nx + i;
                double u = s->ux[n], v = s->uy[n];
                double dXx, dYx, dXy, dYy;
                int okx = upwind(s, m, i, j, 1, 0, u, &dXx, &dYx);
                int oky = upwind(s, m, i, j, 0, 1, v, &dXy, &dYy);
                if (!okx || !oky) {
                    miss++;
                    m->X1[k] = m->X[k];
                    m->Y1[k] = m->Y[k];
                } else {
                    m->X1[k] = m->X[k] - (u * dXx + v * dXy);
                    m->Y1[k] = m->Y[k] - (u * dYx + v * dYy);
                }
                m->set1[k] = 1;
            }
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

/* extrapolate one target node t = (i, j) of layer l of map m (Sec. 3.2
 * steps (i)-(iii)) */
static int extrap_target(orc_sim* s, orc_map* m, int i, int j, int l)
{
    long kt = pidx(s, i, j);
    /* approximated outward surface normal of phi^n at the target (l <= 2) */
    int use_n = 0;
    double nxh = 0.0, nyh = 0.0;
    if (l <= 2) {
        long ke = pidx(s, i + 1, j), kw = pidx(s, i - 1, j);
        long kn = pidx(s, i, j + 1), ks = pidx(s, i, j - 1);
        if (ke >= 0 && kw >= 0 && kn >= 0 && ks >= 0 && m->set[ke] && m->set[kw] &&
            m->set[kn] && m->set[ks]) {
            double gx = (m->phi[ke] - m->phi[kw]) / 2.0;
            double gy = (m->phi[kn] - m->phi[ks]) / 2.0;
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
                int lk = m->layer[k];
                if (lk == 0 || (lk > 0 && lk < l && m->set1[k])) count++;
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
                int lk = m->layer[k];
                if (!(lk == 0 || (lk > 0 && lk < l && m->set1[k]))) continue;
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
                bX0 += w * dx * m->X1[k]; bX1 += w * dy * m->X1[k]; bX2 += w * m->X1[k];
                bY0 += w * dx * m->Y1[k]; bY1 += w * dy * m->Y1[k]; bY2 += w * m->Y1[k];
            }
        double det = det3(M00, M01, M02, M01, M11, M12, M02, M12, M22);
        if (!(det > s->p.det_rel * M22 * M22 * M22)) continue; /* ill-defined: grow r */
        /* step (iii): the fitted map at the target is its intercept C (Cramer) */
        m->X1[kt] = det3(M00, M01, bX0, M01, M11, bX1, M02, M12, bX2) / det;
        m->Y1[kt] = det3(M00, M01, bY0, M01, M11, bY1, M02, M12, bY2) / det;
        m->set1[kt] = 1;
        return 1;
    }
    return 0;
}

/* Sec. 3.2: layers around S^n, then layer-by-layer LSQ extrapolation, for
 * each solid on its own.  Valid nodes are solid nodes or already-set nodes
 * of earlier layers only, so the targets of one layer are independent of
 * each other. */
void orc_phase_extrapolate(orc_sim* s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const int i0 = dom_lo(s->p.periodic_x), i1 = dom_hi(s->p.periodic_x, nx);
    const int j0 = dom_lo(s->p.periodic_y), j1 = dom_hi(s->p.periodic_y, ny);
    const int W = i1 - i0 + 1, H = j1 - j0 + 1;
    for (int bi = 0; bi < s->nsolid; bi++) {
        orc_map* m = &s->m[bi];
        mark_layers(s, m);
        for (int l = 1; l <= s->p.layers; l++) {
            long fail = 0;
#pragma omp parallel for reduction(+ : fail) schedule(dynamic, 4)
            for (int jj = 0; jj < H; jj++) {
                int j = s->p.reverse_order ? j1 - jj : j0 + jj;
                for (int ii = 0; ii < W; ii++) {
                    int i = s->p.reverse_order ? i1 - ii : i0 + ii;
                    long k = pidx(s, i, j);
                    if (m->layer[k] != l) continue;
                    if (!extrap_target(s, m, i, j, l)) fail++;
                }
            }
            s->cnt[ORC_CNT_EXTRAP_FAIL] += fail;
        }
    }
}

/* Sec. 3.2 end / Alg. 1: recompute phi = phi0(xi^{n+1}) on every node that
 * holds a reference map, then make the new map the current one. */
void orc_phase_relabel(orc_sim* s)
{
    for (int b = 0; b < s->nsolid; b++) {
        orc_map* m = &s->m[b];
        for (long k = 0; k < s->NP; k++) {
            if (m->set1[k]) {
                m->phi1[k] = phi0(m, m->X1[k], m->Y1[k]);
            } else {
                m->X1[k] = m->Y1[k] = NAN;
                m->phi1[k] = INFINITY;
            }
        }
        double* t;
        unsigned char* tc;
        t = m->X; m->X = m->X1; m->X1 = t;
        t = m->Y; m->Y = m->Y1; m->Y1 = t;
        t = m->phi; m->phi = m->phi1; m->phi1 = t;
        tc = m->set; m->set = m->set1; m->set1 = tc;
    }
    s->have_new = 0;
}

/* The stencil of a half-edge: dir = 0: x-edge (i-1/2, j) between a = (i-1, j)
 * and b = (i, j); dir = 1: y-edge (i, j-1/2) between a = (i, j-1) and
 * b = (i, j).  k1..k4 are the four nodes beside the edge: (+t, b), (+t, a),
 * (-t, b), (-t, a) along the tangent t.  A derivative at the edge is the
 * difference b - a along the normal and the average of the two side
 * differences along the tangent (the stencil of Eq. (3_3_refmap_jacobian)). */
typedef struct {
    long ka, kb, k1, k2, k3, k4;
    int full; /* all six nodes exist */
} edge_st;

static edge_st edge_stencil(const orc_sim* s, int i, int j, int dir)
{
    edge_st e;
    int ia = dir == 0 ? i - 1 : i, ja = dir == 0 ? j : j - 1;
    e.ka = pidx(s, ia, ja);
    e.kb = pidx(s, i, j);
    if (dir == 0) {
        e.k1 = pidx(s, i, j + 1); e.k2 = pidx(s, i - 1, j + 1);
        e.k3 = pidx(s, i, j - 1); e.k4 = pidx(s, i - 1, j - 1);
    } else {
        e.k1 = pidx(s, i + 1, j); e.k2 = pidx(s, i + 1, j - 1);
        e.k3 = pidx(s, i - 1, j); e.k4 = pidx(s, i - 1, j - 1);
    }
    e.full = e.ka >= 0 && e.kb >= 0 && e.k1 >= 0 && e.k2 >= 0 && e.k3 >= 0 && e.k4 >= 0;
    return e;
}

static int edge_all_set(const edge_st* e, const unsigned char* set)
{
    return e->full && set[e->k1] && set[e->k2] && set[e->k3] && set[e->k4];
}

/* gradient (d/dx, d/dy) at the half-edge of a field whose values on the
 * stencil nodes (a, b, k1, k2, k3, k4) are v[0..5] */
static void edge_grad(const double* v, int dir, double* gx, double* gy)
{
    double gn = v[1] - v[0];
    double gt = (v[2] + v[3] - v[4] - v[5]) / 4.0;
    *gx = dir == 0 ? gn : gt;
    *gy = dir == 0 ? gt : gn;
}

static void edge_values(const edge_st* e, const double* f, double* v)
{
    v[0] = f[e->ka]; v[1] = f[e->kb];
    v[2] = f[e->k1]; v[3] = f[e->k2]; v[4] = f[e->k3]; v[5] = f[e->k4];
}

/* solid m's blended stress lambda_m tau_s,m on a half-edge, with lambda_m =
 * 1 - H(phi_e) at the edge's mean level set; returns lambda_m (0 where the
 * map does not cover both ends of the edge) */
static double solid_edge(const orc_sim* s, const orc_map* m, const edge_st* e, int dir,
                         double* out, long* miss, long* sing)
{
    out[0] = out[1] = out[2] = 0.0;
    if (e->ka < 0 || e->kb < 0 || !m->set[e->ka] || !m->set[e->kb]) return 0.0;
    double phie = 0.5 * (m->phi[e->ka] + m->phi[e->kb]);
    double lam = 1.0 - orc_heaviside(phie, s->p.eps);
    if (!(lam > 0.0)) return 0.0;
    if (!edge_all_set(e, m->set)) {
        (*miss)++;
        return lam;
    }
    double J[4], v[6];
    edge_values(e, m->X, v);
    edge_grad(v, dir, &J[0], &J[1]);
    edge_values(e, m->Y, v);
    edge_grad(v, dir, &J[2], &J[3]);
    double tau[3];
    if (!orc_solid_stress(J, m->body.G, s->p.detJ_min, tau)) {
        (*sing)++;
        return lam;
    }
    out[0] = lam * tau[0];
    out[1] = lam * tau[1];
    out[2] = lam * tau[2];
    return lam;
}

/* contact function of Eq. (3_6_collision_force): (1 - x / eps) / 2 below
 * eps, zero above; not capped for deep overlap */
static double contact_f(double x, double eps) { return x < eps ? 0.5 * (1.0 - x / eps) : 0.0; }

/* Eq. (3_6_collision_stress) for the pair (p, q) on a half-edge, added to
 * out: -eta min(f(phi_p), f(phi_q)) (G_p + G_q) (n n^T - I/2), with the level
 * sets taken at the edge's mean and n the unit gradient of phi_p - phi_q
 * (Eq. (3_6_normal)) on the edge stencil.  Only where both maps cover the
 * whole stencil. */
static void contact_edge(const orc_sim* s, const orc_map* mp, const orc_map* mq,
                         const edge_st* e, int dir, double* out)
{
    if (!edge_all_set(e, mp->set) || !mp->set[e->ka] || !mp->set[e->kb]) return;
    if (!edge_all_set(e, mq->set) || !mq->set[e->ka] || !mq->set[e->kb]) return;
    double fp = contact_f(0.5 * (mp->phi[e->ka] + mp->phi[e->kb]), s->p.eps);
    double fq = contact_f(0.5 * (mq->phi[e->ka] + mq->phi[e->kb]), s->p.eps);
    double fmin = fp < fq ? fp : fq;
    if (!(fmin > 0.0)) return;
    /* phi_p - phi_q on the six stencil nodes */
    double vp[6], vq[6], d[6];
    edge_values(e, mp->phi, vp);
    edge_values(e, mq->phi, vq);
    for (int t = 0; t < 6; t++) d[t] = vp[t] - vq[t];
    double gx, gy;
    edge_grad(d, dir, &gx, &gy);
    double g = sqrt(gx * gx + gy * gy);
    if (!(g > 0.0)) return;
    double nx = gx / g, ny = gy / g;
    double c = -s->p.eta * fmin * (mp->body.G + mq->body.G);
    out[0] += c * (nx * nx - 0.5);
    out[1] += c * (nx * ny);
    out[2] += c * (ny * ny - 0.5);
}

/* Global solid stress on one half-edge (Eq. (3_6_global_stress) without the
 * fluid part, which the lattice carries): sum_m lambda_m tau_s,m, divided by
 * sum_m lambda_m where that exceeds one, plus the contact stress of every
 * pair of solids.  For one solid this is Eq. (2_4_smooth_stress)'s solid
 * term (1 - H) tau_s. */
static void edge_stress(orc_sim* s, int i, int j, int dir, double* out, long* miss, long* sing)
{
    out[0] = out[1] = out[2] = 0.0;
    if (!s->nsolid) return;
    edge_st e = edge_stencil(s, i, j, dir);
    double lsum = 0.0, acc[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < s->nsolid; b++) {
        double t[3];
        double lam = solid_edge(s, &s->m[b], &e, dir, t, miss, sing);
        if (!(lam > 0.0)) continue;
        lsum += lam;
        acc[0] += t[0];
        acc[1] += t[1];
        acc[2] += t[2];
    }
    if (lsum > 1.0) {
        acc[0] /= lsum;
        acc[1] /= lsum;
        acc[2] /= lsum;
    }
    out[0] = acc[0];
    out[1] = acc[1];
    out[2] = acc[2];
    if (s->p.eta != 0.0)
        for (int p = 0; p < s->nsolid; p++)
            for (int q = p + 1; q < s->nsolid; q++)
                contact_edge(s, &s->m[p], &s->m[q], &e, dir, out);
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
 * and f_ext,f a uniform force density on the fluid.  Several solids: the
 * stress is the global one of Eq. (3_6_global_stress) with contact; the
 * buoyancy is sum_m lambda_m (rho_s,m - rho_f) g, normalised like the density
 * where the fractions sum above one; the fluid's share of f_ext,f is
 * 1 - min(1, sum_m lambda_m) (H for one solid). */
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
            double hf = 1.0;
            if (s->nsolid == 1) {
                /* the single-solid form, as written in Eq. (2_4_F_divs) */
                const orc_map* m = &s->m[0];
                if (m->set[k]) {
                    double H = orc_heaviside(m->phi[k], s->p.eps);
                    fx += (1.0 - H) * (m->body.rho_s - s->p.rho_f) * s->p.gx;
                    fy += (1.0 - H) * (m->body.rho_s - s->p.rho_f) * s->p.gy;
                    hf = H;
                }
            } else if (s->nsolid > 1) {
                double lsum = 0.0;
                for (int b = 0; b < s->nsolid; b++) lsum += lambda_at(s, &s->m[b], k);
                double drho = mixture_drho(s, k);
                fx += drho * s->p.gx;
                fy += drho * s->p.gy;
                hf = lsum < 1.0 ? 1.0 - lsum : 0.0;
            }
            fx += hf * s->p.fext_x;
            fy += hf * s->p.fext_y;
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
            double drho = mixture_drho(s, k);
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
     * adds -2 w_i rho_w (c_i . u_w) / c_s^2 with rho_w the node's density
     * (or the fluid density rho_f, lid_rho_mode 1). */
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
                    double rw = s->p.lid_rho_mode ? s->p.rho_f : s->rho[n];
                    s->fnew[OPP[q] * N + n] = fh - 2.0 * WQ[q] * rw * cu / CS2;
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
int32_t orc_nsolid(const orc_sim* s) { return s->nsolid; }

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

void orc_read_refmap_body(const orc_sim* s, int32_t b, double* X, double* Y, double* phi)
{
    const orc_map* m = (b >= 0 && b < s->nsolid) ? &s->m[b] : NULL;
    for (int j = 0; j < s->p.ny; j++)
        for (int i = 0; i < s->p.nx; i++) {
            long n = (long)j * s->p.nx + i, k = pidx(s, i, j);
            int ok = m && m->set[k];
            if (X) X[n] = ok ? m->X[k] : NAN;
            if (Y) Y[n] = ok ? m->Y[k] : NAN;
            if (phi) phi[n] = ok ? m->phi[k] : NAN;
        }
}

void orc_read_refmap(const orc_sim* s, double* X, double* Y, double* phi)
{
    orc_read_refmap_body(s, 0, X, Y, phi);
}

/* the padded layout used by the read/set calls: [(ny+4)][(nx+4)], node (i, j)
 * at ((j+2)*(nx+4) + i+2); on periodic axes the pad cells are left NaN */
static long ext_idx(const orc_sim* s, int i, int j) { return (long)(j + 2) * (s->p.nx + 4) + (i + 2); }

void orc_read_refmap_padded(const orc_sim* s, double* X, double* Y, double* phi)
{
    long NE = (long)(s->p.nx + 4) * (s->p.ny + 4);
    for (long e = 0; e < NE; e++) X[e] = Y[e] = phi[e] = NAN;
    if (!s->nsolid) return;
    const orc_map* m = &s->m[0];
    for (int j = -2; j <= s->p.ny + 1; j++)
        for (int i = -2; i <= s->p.nx + 1; i++) {
            if ((s->p.periodic_x && (i < 0 || i >= s->p.nx)) ||
                (s->p.periodic_y && (j < 0 || j >= s->p.ny)))
                continue;
            long k = pidx(s, i, j), e = ext_idx(s, i, j);
            if (m->set[k]) {
                X[e] = m->X[k];
                Y[e] = m->Y[k];
                phi[e] = m->phi[k];
            }
        }
}

void orc_read_layers_padded(const orc_sim* s, int32_t* layer)
{
    long NE = (long)(s->p.nx + 4) * (s->p.ny + 4);
    for (long e = 0; e < NE; e++) layer[e] = -1;
    if (!s->nsolid) return;
    const orc_map* m = &s->m[0];
    for (int j = -2; j <= s->p.ny + 1; j++)
        for (int i = -2; i <= s->p.nx + 1; i++) {
            if ((s->p.periodic_x && (i < 0 || i >= s->p.nx)) ||
                (s->p.periodic_y && (j < 0 || j >= s->p.ny)))
                continue;
            layer[ext_idx(s, i, j)] = m->layer[pidx(s, i, j)];
        }
}

void orc_set_refmap_padded(orc_sim* s, const double* X, const double* Y)
{
    if (!s->nsolid) return;
    orc_map* m = &s->m[0];
    for (int j = -2; j <= s->p.ny + 1; j++)
        for (int i = -2; i <= s->p.nx + 1; i++) {
            if ((s->p.periodic_x && (i < 0 || i >= s->p.nx)) ||
                (s->p.periodic_y && (j < 0 || j >= s->p.ny)))
                continue;
            long k = pidx(s, i, j), e = ext_idx(s, i, j);
            if (isnan(X[e])) {
                m->set[k] = 0;
                m->X[k] = m->Y[k] = NAN;
                m->phi[k] = INFINITY;
            } else {
                m->set[k] = 1;
                m->X[k] = X[e];
                m->Y[k] = Y[e];
                m->phi[k] = phi0(m, X[e], Y[e]);
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

/* solid fraction moments of map m over interior nodes: sum lambda, sum
 * lambda x, sum lambda y, sum lambda (x - X), sum lambda (y - Y), solid
 * nodes, nodes with a value */
static void body_moments(const orc_sim* s, const orc_map* m, double* acc7)
{
    for (int t = 0; t < 7; t++) acc7[t] = 0.0;
    for (int j = 0; j < s->p.ny; j++)
        for (int i = 0; i < s->p.nx; i++) {
            long k = pidx(s, i, j);
            if (!m->set[k]) continue;
            acc7[6] += 1;
            if (m->phi[k] < 0) acc7[5] += 1;
            double lam = 1.0 - orc_heaviside(m->phi[k], s->p.eps);
            double x = node_x(s, m, i), y = node_y(s, m, j);
            acc7[0] += lam;
            acc7[1] += lam * x;
            acc7[2] += lam * y;
            acc7[3] += lam * (x - m->X[k]);
            acc7[4] += lam * (y - m->Y[k]);
        }
}

void orc_diag_body(const orc_sim* s, int32_t b, double* out)
{
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    if (b >= 0 && b < s->nsolid) body_moments(s, &s->m[b], a);
    double lw = a[0];
    out[0] = lw > 0 ? a[1] / lw : NAN;
    out[1] = lw > 0 ? a[2] / lw : NAN;
    out[2] = lw > 0 ? a[3] / lw : NAN;
    out[3] = lw > 0 ? a[4] / lw : NAN;
    out[4] = a[5];
    out[5] = a[6];
}

void orc_diag(const orc_sim* s, double* out)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const long N = s->N;
    double mass = 0, px = 0, py = 0, umax = 0;
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
        }
    /* the solids' moments, summed over solids (each in its own unwrapped
     * frame) */
    double tot[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < s->nsolid; b++) {
        double a[7];
        body_moments(s, &s->m[b], a);
        for (int t = 0; t < 7; t++) tot[t] += a[t];
    }
    double lw = tot[0];
    out[0] = mass;
    out[1] = px;
    out[2] = py;
    out[3] = lw > 0 ? tot[1] / lw : NAN;
    out[4] = lw > 0 ? tot[2] / lw : NAN;
    out[5] = lw > 0 ? tot[3] / lw : NAN;
    out[6] = lw > 0 ? tot[4] / lw : NAN;
    out[7] = umax;
    out[8] = tot[5];
    out[9] = tot[6];
}
