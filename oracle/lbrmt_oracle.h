/*
 * lbrmt_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of one time step of the lattice
 * Boltzmann reference map technique (LBRMT; Sun & Rycroft, "A fully-integrated
 * lattice Boltzmann method for fluid-structure interaction"), written from the
 * paper to check and time the GPU library.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or table with the GPU library.
 *
 * Conventions (readings of the paper, listed with the others in the design
 * notes):
 *   - interior node (i, j), 0 <= i < nx, 0 <= j < ny, sits at x = (i+1/2, j+1/2);
 *     walls are halfway, at x = 0, nx and y = 0, ny; the top wall is the lid.
 *   - the reference map / level set live on the padded grid i = -2 .. nx+1
 *     (two buffer layers, Sec. 3) along walled axes; along periodic axes the
 *     index wraps and there is no padding.
 *   - all fields returned to the caller are row-major [ny][nx], x fastest.
 */
#ifndef LBRMT_ORACLE_H
#define LBRMT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny;
    int32_t periodic_x, periodic_y;
    double tau;         /* BGK relaxation time, Eq. (2_2_bgk)                */
    double lid_ux;      /* velocity of the top wall (walled y only)          */
    double gx, gy;      /* gravity acting on the solid (buoyancy form)       */
    double fext_x, fext_y; /* external force density on the fluid, f_ext,f */
    double rho_f;       /* fluid density                                     */
    double eps;         /* blur-zone half-width of H_eps, Eq. (2_3_heaviside)*/
    int32_t layers;     /* extrapolation-zone layers (Sec. 4: 11)            */
    int32_t r_max;      /* largest scan-window half-width                    */
    double det_rel;     /* LSQ fit ill-defined if det M <= det_rel*(sum w)^3 */
    double detJ_min;    /* half-edge stress dropped if det(grad xi) <= this  */
    int32_t reverse_order; /* process extrapolation targets in reverse order */
    int32_t lid_rho_mode;  /* moving-lid density: 0 the node's rho, 1 rho_f */
    double eta;         /* contact factor of Eq. (3_6_collision_stress)      */
} orc_params;

/* most solids one simulation may hold */
#define ORC_MAX_SOLIDS 64

typedef struct {
    double cx, cy;      /* centre in the reference configuration             */
    double R;           /* disc radius; the ellipse's semi-axis a            */
    double G;           /* small-strain shear modulus                        */
    double rho_s;       /* solid density                                     */
    int32_t shape;      /* 0 disc, 1 ellipse                                 */
    int32_t reserved;
    double b;           /* ellipse: semi-axis b                              */
    double theta;       /* ellipse: angle of the a axis to the x axis        */
} orc_solid;

/* counters kept by the oracle (index into orc_counters' output) */
enum {
    ORC_CNT_ADVECT_MISS = 0,   /* advection stencil node without a value     */
    ORC_CNT_EXTRAP_FAIL = 1,   /* target left unset after r > r_max          */
    ORC_CNT_STRESS_MISS = 2,   /* half-edge stencil node without a value     */
    ORC_CNT_DETJ = 3,          /* half-edge with det(grad xi) <= detJ_min    */
    ORC_CNT_N = 8
};

typedef struct orc_sim orc_sim;

/* lifecycle (0 <= nsolid <= ORC_MAX_SOLIDS; NULL on a bad parameter) */
orc_sim* orc_create(const orc_params* p, const orc_solid* solids, int32_t nsolid);
void     orc_destroy(orc_sim* s);
/* Alg. 1 initialisation; u0 = NULL or 2*ny*nx (ux plane then uy plane) */
void     orc_init(orc_sim* s, const double* u0);
/* n full time steps of Alg. 1 */
void     orc_step(orc_sim* s, int64_t n);

/* the phases of one step, in the order of Alg. 1 (orc_step calls them) */
void orc_phase_advect(orc_sim* s);        /* reference-map advection        */
void orc_phase_extrapolate(orc_sim* s);   /* layers + LSQ extrapolation     */
void orc_phase_relabel(orc_sim* s);       /* phi = phi0(xi), swap to n+1    */
void orc_phase_force(orc_sim* s);         /* div of blended solid stress    */
void orc_phase_collide_stream(orc_sim* s);/* SFC+Guo collision, walls, stream*/
void orc_phase_moments(orc_sim* s);       /* rho, u with half force         */

/* reads (host arrays, row-major [ny][nx]) */
int64_t orc_step_count(const orc_sim* s);
void orc_read_macro(const orc_sim* s, double* rho, double* ux, double* uy);
void orc_read_populations(const orc_sim* s, double* f9);      /* [9][ny][nx] */
void orc_read_force(const orc_sim* s, double* fx, double* fy); /* last F    */
/* xi and phi of solid b (orc_read_refmap: solid 0) on interior nodes; NaN
 * where the node holds no value of that map */
void orc_read_refmap(const orc_sim* s, double* X, double* Y, double* phi);
void orc_read_refmap_body(const orc_sim* s, int32_t b, double* X, double* Y, double* phi);
int32_t orc_nsolid(const orc_sim* s);
/* padded-grid versions (solid 0): [(ny+4)][(nx+4)], offset 2 in each
 * walled axis */
void orc_read_refmap_padded(const orc_sim* s, double* X, double* Y, double* phi);
void orc_read_layers_padded(const orc_sim* s, int32_t* layer);
/* node average of the four global half-edge solid stresses (xx, xy, yy) */
void orc_read_stress(orc_sim* s, double* sxx, double* sxy, double* syy);
void orc_counters(const orc_sim* s, int64_t* out8);
/* diag: [mass, mom_x, mom_y, centroid_x, centroid_y, disp_x, disp_y,
 *        max|u|, n_solid, n_band]; the solid terms summed over all solids */
void orc_diag(const orc_sim* s, double* out10);
/* one solid: [centroid_x, centroid_y, disp_x, disp_y, n_solid, n_band] */
void orc_diag_body(const orc_sim* s, int32_t b, double* out6);

/* overwrite state (tests): xi/phi of solid 0 on the padded grid, NaN X = no
 * value */
void orc_set_refmap_padded(orc_sim* s, const double* X, const double* Y);
void orc_set_populations(orc_sim* s, const double* f9);
void orc_set_moments(orc_sim* s, const double* rho, const double* ux, const double* uy);

/* pointwise definitions, exported so the tests can pin them */
double orc_heaviside(double phi, double eps);
void   orc_feq_sfc(double rho, double ux, double uy, double drho, double* feq9);
void   orc_guo(double ux, double uy, double fx, double fy, double* fi9);
/* J = [dX/dx, dX/dy, dY/dx, dY/dy]; returns 0 and tau = 0 if det J <= detJ_min */
int    orc_solid_stress(const double* J4, double G, double detJ_min, double* tau3);
double orc_phi0(const orc_solid* body, double X, double Y);
/* layers on an arbitrary nx*ny mask grid (4-adjacency, non-periodic), literal
 * layer-by-layer marking; solid != 0 marks S; out: 0 solid, l, or -1 */
void   orc_layers_mask(int32_t nx, int32_t ny, const uint8_t* solid, int32_t L, int32_t* out);
void   orc_d2q9(int32_t* cx, int32_t* cy, double* w);

#ifdef __cplusplus
}
#endif
#endif
