/*
 * lbrmt.h -- C ABI of the MI355X (gfx950) LBRMT time-step library.
 *
 * The library advances the lattice Boltzmann reference map technique of Sun &
 * Rycroft ("A fully-integrated lattice Boltzmann method for fluid-structure
 * interaction"): a D2Q9 BGK fluid with Guo body forcing (Sec. 2.2), the smooth
 * flux correction across solid/fluid density differences (Sec. 2.3), and
 * neo-Hookean solids tracked by a reference map xi on the same fixed grid
 * (Secs. 2.1, 2.4, 3.1-3.3), one time step of Alg. 1 per iteration.
 *
 * Conventions used by every call:
 *   - lattice units: dx = dt = 1; node (i, j), 0 <= i < nx, 0 <= j < ny, sits at
 *     x = (i + 1/2, j + 1/2); no-slip walls are halfway, at x = 0, nx, y = 0, ny;
 *     the top wall (y = ny) is the lid and moves with (lid_ux, 0).
 *   - every field buffer is row-major [ny][nx], x fastest, float64, DEVICE memory,
 *     interior nodes only; vector fields are separate planes.
 *   - the caller owns the workspace, every input/output buffer and the stream;
 *     the library owns only a small host-side context (freed by lbrmt_destroy)
 *     plus one internal stream and a few events for fork/join inside a step.
 *     It never allocates device memory.
 *   - every call is stream-ordered on the context's stream and asynchronous
 *     unless stated otherwise; the calls that synchronise say so.
 *   - no exception crosses the ABI; every call returns an lbrmt_status.  A
 *     context is not thread-safe; separate contexts are independent.
 */
#ifndef LBRMT_H
#define LBRMT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBRMT_OK = 0,
    LBRMT_EINVAL = 1,      /* null pointer, nx or ny < 8, tau <= 1/2, bad shape,
                              lid_rho_mode not 0 or 1                            */
    LBRMT_EWORKSPACE = 2,  /* workspace too small or misaligned (256 B)          */
    LBRMT_EHIP = 3,        /* a HIP call failed; text via lbrmt_last_error       */
    LBRMT_EUNSTABLE = 4,   /* device health counters report a failure            */
    LBRMT_ECAPACITY = 5,   /* more solids than the context was created for       */
    LBRMT_ESTATE = 6       /* call out of order (e.g. step before init)          */
} lbrmt_status;

/* Storage and arithmetic precision of a context.
 *   LBRMT_FP64: populations f_i and the reference map xi in double.
 *   LBRMT_FP32: populations stored as deviations f_i - w_i rho_f in float with
 *               float lattice arithmetic; xi stored as the displacement xi - x
 *               in float with float stencil arithmetic (advection, fit
 *               right-hand sides, stress).  Double is kept for the level set
 *               phi0(xi) (it decides the solid set), the fit's normal matrix
 *               and well-posedness test, the inversion of grad xi where
 *               det < kappa_J (0.25 by default), the force planes and every
 *               diagnostic reduction.
 * Reads return float64 in both modes (xi, not the displacement). */
typedef enum { LBRMT_FP64 = 0, LBRMT_FP32 = 1 } lbrmt_precision;

/* Grid and fluid parameters (Table "sim_quantities", Secs. 2.2-2.4, 3.5). */
typedef struct {
    int32_t nx, ny;          /* interior nodes                                   */
    int32_t periodic_x;      /* 1: periodic along x (Sec. 3.5), 0: halfway walls */
    int32_t periodic_y;      /* 1: periodic along y, 0: walls with the lid on top*/
    double tau;              /* BGK relaxation time, nu = (tau - 1/2)/3          */
    double lid_ux;           /* top-wall velocity (ignored when periodic_y)      */
    double gx, gy;           /* gravity g; the solid feels (1-H)(rho_s-rho_f) g  */
    double fext_x, fext_y;   /* uniform external force density on the fluid (H-weighted) */
    double rho_f;            /* fluid density (1 in lattice units)               */
    double eps;              /* blur-zone half-width epsilon of H_eps            */
    int32_t layers;          /* extrapolation-zone layers (11)                   */
    int32_t r_max;           /* largest least-squares scan half-width (8)        */
    double det_rel;          /* fit ill-defined if det M <= det_rel (sum w)^3 (1e-8) */
    double detJ_min;         /* half-edge stress dropped if det(grad xi) <= this (1e-12) */
    int32_t precision;       /* lbrmt_precision                                  */
    int32_t body_window;     /* several solids: side of each solid's own window
                                along a periodic axis (0: 128); see below       */
    double eta;              /* contact factor eta of Eq. (3_6_collision_stress)
                                (several solids; 1 in the paper's runs)         */
    double kappa_J;          /* FP32: grad xi is inverted in double where its
                                determinant (the J of Eq. (3_3_refmap_deformation))
                                is below kappa_J; <= 0 selects 0.25            */
    int32_t lid_rho_mode;    /* density rho_w in the moving-lid term of the
                                bounce-back (Sec. 3.5): 0 the node's rho^n
                                (default), 1 the fluid density rho_f            */
    int32_t reserved;
} lbrmt_grid_desc;

/* Several solids (Sec. 3.6).  A context created with max_solids > 1 keeps
 * every solid's reference map, level set and extrapolation zone on a window
 * of its own: along a periodic axis whose length is a multiple of 16 and at
 * least body_window + 36 the window is body_window nodes centred on the
 * solid, elsewhere it is the whole axis.  The solids meet in the global
 * half-edge stress (their blended stresses normalised by the summed solid
 * fraction where it exceeds one, Eq. (3_6_global_stress)), the contact stress
 * of every overlapping pair (Eqs. (3_6_collision_stress) to (3_6_normal), on
 * half-edges), and the density rho_f + sum_i lambda_i (rho_s,i - rho_f) /
 * max(1, sum_i lambda_i).  A body_window window follows its solid: after a
 * step whose zone (the solid's box dilated by `layers`) comes within 4 nodes
 * of the window's border, the window moves so that the box is centred (the
 * maps move with it; no value changes).  A zone that would cross the seam of
 * a whole-axis window (which cannot move) raises LBRMT_H_WINDOW_CLIP:
 * results are wrong from then on, and lbrmt_diag returns EUNSTABLE.  Not
 * available with several solids: the tile-shape options, the autotuners and
 * the adjoint. */

/* One solid (Sec. 3.6 "mat_const"/"object"): a disc (shape 0) of radius a, or
 * an ellipse (shape 1) of semi-axes a and b whose a axis makes the angle theta
 * with the x axis.  The reference level set is the disc's signed distance
 * |X - c| - a, and for the ellipse |X - c| (1 - 1/q) with
 * q = sqrt((x'/a)^2 + (y'/b)^2) in the body frame (negative inside, zero on
 * the boundary, the disc's when a = b).  Other shapes: LBRMT_EINVAL. */
typedef struct {
    int32_t shape;           /* 0: disc, 1: ellipse                              */
    int32_t reserved;
    double cx, cy;           /* centre of the reference (undeformed) shape       */
    double a, b;             /* disc: radius a (b unused); ellipse: semi-axes    */
    double theta;            /* ellipse: angle of the a axis (radians)           */
    double G;                /* small-strain shear modulus                       */
    double rho_s;            /* solid density                                    */
} lbrmt_solid_desc;

/* Device health counters (cumulative since lbrmt_init). */
typedef enum {
    LBRMT_H_ADVECT_MISS = 0, /* advection stencil node without a reference map   */
    LBRMT_H_EXTRAP_FAIL = 1, /* zone node left unset after r > r_max             */
    LBRMT_H_STRESS_MISS = 2, /* half-edge stencil node without a reference map   */
    LBRMT_H_DETJ = 3,        /* half-edge with det(grad xi) <= detJ_min          */
    LBRMT_H_DETJ_SOLID = 4,  /* ... of those, edges with solid fraction > 1/2    */
    LBRMT_H_NONFINITE = 5,   /* nodes whose density is not finite or <= 0        */
    LBRMT_H_WINDOW_CLIP = 6, /* a solid's zone reached its window's border (one
                                solid: also its box moved down > 2 rows in a step) */
    LBRMT_H_LIST_OVERFLOW = 7, /* list entries dropped at capacity (layer lists;
                                  solids met by one force block beyond 32)      */
    LBRMT_H_COUNT = 8
} lbrmt_health_index;

/* lbrmt_diag output: FP64 reductions over interior nodes of the state f^n. */
typedef struct {
    int64_t step;            /* completed steps                                  */
    double mass;             /* sum_nodes sum_i f_i                              */
    double mom_x, mom_y;     /* sum_nodes (sum_i c_i f_i + F/2)                  */
    /* the solid's centroid and mean displacement, weighted by its fraction
     * lambda = 1 - H(phi) (Eq. (2_3_heaviside)); the paper tracks a solid's
     * centroid (Sec. 4.1, Fig. 4_1_ldc) without defining it, this is the
     * smooth (differentiable) reading */
    double centroid_x, centroid_y; /* sum lambda x / sum lambda                  */
    double disp_x, disp_y;   /* sum lambda (x - xi) / sum lambda                 */
    double max_u;            /* max |u|                                          */
    double n_solid;          /* nodes with phi < 0                               */
    double n_band;           /* nodes holding a reference map                    */
    double lambda_sum;       /* sum lambda (the centroid's denominator)          */
    uint32_t health[LBRMT_H_COUNT];
} lbrmt_diag_t;

/* lbrmt_validate output (App. A): derived numbers and warnings. */
typedef struct {
    double nu;               /* (tau - 1/2) / 3                                  */
    double mach_lb;          /* Ma* = |lid| / sqrt(1/3)                           */
    double reynolds;         /* |lid| * nx / nu                                  */
    int32_t tau_ok;          /* 1/2 < tau <= 1                                   */
    int32_t mach_ok;         /* Ma* <= 0.3                                       */
    int32_t solids_inside;   /* every solid's zone fits inside the padded grid  */
    int32_t reserved;
} lbrmt_validation_t;

typedef struct lbrmt_ctx lbrmt_ctx;

/* Status text; never NULL. */
const char* lbrmt_status_string(int status);
/* Text of the last error on this context (empty string if none). */
const char* lbrmt_last_error(const lbrmt_ctx* ctx);

/* Bytes of device workspace a context of this shape needs (host only). */
int lbrmt_workspace_bytes(const lbrmt_grid_desc* desc, int32_t max_solids, size_t* bytes);

/* Create a context on caller workspace d_workspace (device, 256-B aligned, at
 * least lbrmt_workspace_bytes) and caller stream hip_stream (hipStream_t, may
 * be NULL for the null stream).  The context never frees the workspace. */
int lbrmt_create(const lbrmt_grid_desc* desc, int32_t max_solids, void* d_workspace,
                 size_t bytes, void* hip_stream, lbrmt_ctx** out);
void lbrmt_destroy(lbrmt_ctx* ctx);

/* Register solids (before lbrmt_init).  ECAPACITY beyond max_solids, or for
 * a solid too large for its window (2 (extent + layers + 4) > body_window
 * along a windowed axis). */
int lbrmt_add_solids(lbrmt_ctx* ctx, const lbrmt_solid_desc* solids, int32_t n);
/* Most solids one context may hold. */
#define LBRMT_MAX_SOLIDS 4096

/* Alg. 1 initialisation: xi = x on the solid and its extrapolation zone, phi
 * from the reference shape, rho = H rho_f + (1-H) rho_s, v = v0 and f = f^eq
 * of Eq. (2_3_feq_sfc).  d_u0: NULL (fluid at rest) or device float64
 * [2][ny][nx] (ux plane, then uy plane). */
int lbrmt_init(lbrmt_ctx* ctx, const double* d_u0);

/* Advance nsteps time steps of Alg. 1 (asynchronous). */
int lbrmt_step(lbrmt_ctx* ctx, int64_t nsteps);
int64_t lbrmt_step_count(const lbrmt_ctx* ctx);

/* rho^n and u^n (half-force velocity of Eq. (2_2_lbm_moments_force)); any
 * pointer may be NULL. */
int lbrmt_read_macro(lbrmt_ctx* ctx, double* d_rho, double* d_ux, double* d_uy);
/* pre-collision populations f_i^n, [9][ny][nx] */
int lbrmt_read_populations(lbrmt_ctx* ctx, double* d_f9);
/* force density F used by the last step (Eq. (2_4_F_divs)) */
int lbrmt_read_force(lbrmt_ctx* ctx, double* d_fx, double* d_fy);
/* reference map xi = (X, Y) and level set phi = phi0(xi) of solid `solid`
 * on the fixed grid (Sec. 3, Fig. 3_mmap: each solid's own map over its solid
 * nodes and extrapolation zone); NaN where the node holds no map of that
 * solid.  Any pointer may be NULL. */
int lbrmt_read_refmap(lbrmt_ctx* ctx, int32_t solid, double* d_X, double* d_Y, double* d_phi);
/* node average of the four blended half-edge solid stresses (1-H) tau_s
 * (Eqs. (3_3_solid_stress), (2_4_smooth_stress)); xx, xy, yy planes.  With
 * several solids the global half-edge stress of Eq. (3_6_global_stress):
 * the normalised blend plus the contact stress of every pair. */
int lbrmt_read_stress(lbrmt_ctx* ctx, double* d_sxx, double* d_sxy, double* d_syy);

/* Reductions of the current state into host memory (synchronises the stream).
 * Returns EUNSTABLE if a NONFINITE, DETJ_SOLID, EXTRAP_FAIL, LIST_OVERFLOW or
 * WINDOW_CLIP counter is set or the mass is not finite (the output is filled
 * in either case).
 * With several solids the solid terms are summed over all solids. */
int lbrmt_diag(lbrmt_ctx* ctx, lbrmt_diag_t* host_out);
/* The FP64 sums behind lbrmt_diag, stream-ordered and without synchronising
 * the host (so a run can record them every step): d_out (device, 11 doubles)
 * receives {mass, mom_x, mom_y, sum lambda, sum lambda x, sum lambda y,
 * sum lambda (x - xi) x and y components, n_solid, n_band, max |u|}; the
 * centroid and mean displacement of lbrmt_diag_t are the ratios to
 * sum lambda.  Contexts with one solid at most (ESTATE otherwise). */
int lbrmt_diag_sums(lbrmt_ctx* ctx, double* d_out);
/* lbrmt_diag for callers that cannot allocate device memory (code that must
 * not call hipMalloc: under HIP graph capture, tight serving loops, harnesses
 * that forbid it): the same reductions, results and return codes, with their
 * scratch in a static device array that the library holds on each GPU it
 * runs on until the process ends (147 712 bytes: the per-block partial records, the
 * reduced record and 7 doubles per solid).  No device memory is allocated by
 * this call, and the context's workspace is not used for the reductions.
 * EINVAL for a context with more than LBRMT_DIAG_NOALLOC_MAX_SOLIDS solids
 * (text via lbrmt_last_error).  Call with the context's device current.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (from several host threads, or on several streams) race and
 * give wrong results; serialise them.  Synchronises the stream. */
#define LBRMT_DIAG_NOALLOC_MAX_SOLIDS 1024
int lbrmt_diag_noalloc(lbrmt_ctx* ctx, lbrmt_diag_t* host_out);
/* One solid's terms of lbrmt_diag into host memory: centroid_x, centroid_y,
 * disp_x, disp_y (each in the solid's own unwrapped frame), n_solid, n_band. */
int lbrmt_diag_solid(lbrmt_ctx* ctx, int32_t solid, double* host_out6);

/* Checkpoint: an opaque device blob of lbrmt_state_bytes bytes holding the
 * whole step state (with several solids: every solid's maps, window and
 * region, the force-block stamps and lists); load restores it bit for bit
 * into a context of the same shape (grid, precision, solid count and window
 * sizes), whatever that context held before, and returns EINVAL with a
 * message for a blob of another shape.  Save and load synchronise the
 * context's stream; the buffer is the caller's. */
int lbrmt_state_bytes(const lbrmt_ctx* ctx, size_t* bytes);
int lbrmt_save_state(lbrmt_ctx* ctx, void* d_buf);
int lbrmt_load_state(lbrmt_ctx* ctx, const void* d_buf);

/* Failure injection for tests: field 0 sets every population of interior node
 * `index` (= j*nx + i) to `value`. */
int lbrmt_debug_poke(lbrmt_ctx* ctx, int32_t field, int64_t index, double value);

/* Host-only check of App. A constraints (1/2 < tau <= 1, Ma* <= 0.3) and of
 * solid placement; EINVAL for unusable input, OK with flags otherwise. */
int lbrmt_validate(const lbrmt_grid_desc* desc, const lbrmt_solid_desc* solids, int32_t n,
                   lbrmt_validation_t* out);

/* Discrete adjoint: the exact reverse-mode derivative of the step of Alg. 1
 * as the forward kernels compute it (FP64 contexts with one solid, ESTATE
 * otherwise).  The reverse of one step n needs what the forward step
 * used and made: lbrmt_step_snapshot advances the context one step (eager
 * launches) and copies that into a caller device buffer of
 * lbrmt_snapshot_bytes bytes (the state n lattice, F^{n-1}, F^n, xi^n, phi^n,
 * xi^{n+1}, phi^{n+1}, the layer tags and the windows).
 *
 * Adjoint state: a caller device buffer of lbrmt_adjoint_bytes bytes holding
 * dL/df (natural populations), dL/dxi, dL/dphi, dL/dF and the accumulated
 * dL/dG, dL/d(lid speed).  lbrmt_adjoint_zero clears it; lbrmt_adjoint_loss
 * adds the gradient of L_s = (|c - c*|^2 + |d - d*|^2) w of one state s,
 * with c = sum lambda x / sum lambda and d = sum lambda (x - xi) / sum
 * lambda, lambda = 1 - H(phi) (the centroid and mean displacement of
 * lbrmt_diag); coef = {c_x, c_y, d_x, d_y, dL/dc_x, dL/dc_y, dL/dd_x,
 * dL/dd_y} (host), with which = 0 for the snapshot's state n, 1 for its
 * state n + 1.  lbrmt_adjoint_step takes the adjoint of state n + 1 to state
 * n (snapshots are consumed last step first); lbrmt_adjoint_init turns the
 * adjoint of state 0 (after the step of snapshot 0) into dL/du_0 (device
 * float64 [2][ny][nx]) and returns {dL/dG, dL/dU} in host_GU.  Discrete
 * decisions (solid set, layers, scan windows, upwind sides, fallbacks) are
 * those the forward step took. */
int lbrmt_snapshot_bytes(const lbrmt_ctx* ctx, size_t* bytes);
int lbrmt_step_snapshot(lbrmt_ctx* ctx, void* d_snap);
int lbrmt_adjoint_bytes(const lbrmt_ctx* ctx, size_t* bytes);
int lbrmt_adjoint_zero(lbrmt_ctx* ctx, void* d_adj);
int lbrmt_adjoint_loss(lbrmt_ctx* ctx, void* d_adj, const void* d_snap, int32_t which,
                       const double* host_coef8);
int lbrmt_adjoint_step(lbrmt_ctx* ctx, void* d_adj, const void* d_snap);
int lbrmt_adjoint_init(lbrmt_ctx* ctx, void* d_adj, const void* d_snap0, double* d_u0bar,
                       double* host_GU);

/* Average device time (ms) per launch of each step kernel, measured with HIP
 * events on the stream each kernel runs on.  Enabling timing makes lbrmt_step
 * launch eagerly (no graph) and bracket every kernel with events; names:
 * "advect" (advection with the layers of the extrapolation zone), "extrap"
 * (the layer-by-layer fits), "relabel", "force", "lb_bulk" (the whole lattice
 * with overlap off; the tiles away from the solid with overlap on), "lb_band"
 * (the tiles meeting the solid windows, overlap on). */
int lbrmt_set_timing(lbrmt_ctx* ctx, int32_t enable);
int lbrmt_kernel_time(lbrmt_ctx* ctx, const char* name, double* avg_ms, int64_t* launches);

/* Launch options of a context (host only; an option change drops the
 * captured step graph after synchronising the stream):
 *   LBRMT_OPT_OVERLAP     1 (default): the reference-map chain runs on an
 *                         internal stream while the lattice Boltzmann update of
 *                         the tiles away from the solid runs on the caller's,
 *                         then the tiles meeting the solid windows are updated;
 *                         0: one stream, the chain then one full lattice update.
 *   LBRMT_OPT_LB_VARIANT  tile shape of the lattice Boltzmann update, 0 ..
 *                         LBRMT_OPT_LB_VARIANT_COUNT - 1, default 3 for FP64 and
 *                         5 for FP32 (results are bitwise identical across
 *                         variants; only speed differs).
 *   LBRMT_OPT_GRAPH       1 (default): whole blocks of six steps replay one
 *                         captured HIP graph; 0: every kernel is launched
 *                         eagerly (results are bitwise identical).
 *   LBRMT_OPT_BULK_BLOCKS with overlap: the most workgroups the bulk lattice
 *                         update may use (they stride over its tiles), which
 *                         leaves HBM bandwidth to the reference-map chain
 *                         running beside it; 0: one workgroup per tile.
 *                         Results do not depend on it.
 *   LBRMT_OPT_FUSED_FIT   1024, 512 or 256: one solid on walled axes
 *                         with at most 11 layers fits all layers of the
 *                         extrapolation (Sec. 3.2) in one launch of blocks of
 *                         that many threads, each taking a tile of the window
 *                         with the margin its later layers read; tiles whose
 *                         targets need wider scan windows than the margin
 *                         holds are finished by a second, one-block launch.
 *                         0: one launch per layer; 1: 1024 threads with the
 *                         margin check one node tighter, so that the second
 *                         launch finishes most tiles (a check of that
 *                         launch); -1 (default): 512 in FP64 and 1024
 *                         in FP32, or 0 when LBRMT_OPT_BULK_BLOCKS caps
 *                         the bulk update.  With
 *                         overlap and no cap, the bulk lattice update then
 *                         starts when the advection pass has finished, so
 *                         that these blocks are resident before the bulk
 *                         update fills the compute units.  Results are
 *                         bitwise identical.
 *   LBRMT_OPT_HOLD_BULK   -1 (default): with overlap, the one-launch
 *                         extrapolation and an uncapped bulk update, the bulk
 *                         update starts when the advection pass has ended; a
 *                         capped one (LBRMT_OPT_BULK_BLOCKS > 0) starts with
 *                         the step.  1: held, and a cap is refused (EINVAL,
 *                         either order of the two calls: a held and capped
 *                         bulk update once stalled the step for about 0.1 s
 *                         and is not offered).  0: never held.  Results are
 *                         bitwise identical.
 *   LBRMT_OPT_BULK_EARLY  0 .. 1000: when the bulk update is held, of the
 *                         first this many thousandths of its tiles (the first
 *                         rows of the grid) those wholly below the previous
 *                         step's window by more than 2 rows are updated by a
 *                         launch of their own, which starts when the
 *                         previous step's bulk update has ended, beside the
 *                         end of that step's chain and this step's
 *                         advection pass; the held launch takes the other
 *                         tiles.  -1 (default): 300 on grids of 2048 x 2048
 *                         nodes or more, else 0.  Ignored while kernel timing
 *                         is on.  Results are bitwise identical.  (A solid
 *                         box whose lower edge moves down by more than 2
 *                         rows in one step is counted in LBRMT_H_WINDOW_CLIP.)
 * EINVAL for an unknown option or value. */
typedef enum {
    LBRMT_OPT_OVERLAP = 0,
    LBRMT_OPT_LB_VARIANT = 1,
    LBRMT_OPT_LB_VARIANT_COUNT = 2, /* read only */
    LBRMT_OPT_GRAPH = 3,
    LBRMT_OPT_BULK_BLOCKS = 4,
    LBRMT_OPT_FUSED_FIT = 5,
    LBRMT_OPT_HOLD_BULK = 6,
    LBRMT_OPT_BULK_EARLY = 7
} lbrmt_option;
int lbrmt_set_option(lbrmt_ctx* ctx, int32_t option, int64_t value);
int lbrmt_get_option(const lbrmt_ctx* ctx, int32_t option, int64_t* value);

/* band_nodes: nodes the next step's "lb_band" launch updates (the lattice
 * tiles that meet the solid windows of this and the previous step; "lb_bulk"
 * updates the rest); window_nodes: nodes of the current working window of the
 * reference map.  Synchronises the stream. */
int lbrmt_band_nodes(lbrmt_ctx* ctx, int64_t* band_nodes, int64_t* window_nodes);

/* ---------------------------------------------------------------- autotuner
 * Times every lattice tile shape (LBRMT_OPT_LB_VARIANT values: tile width
 * 32-512 x height 1-8 threads, i.e. 1-8 waves per workgroup, 1, 2 or 4 nodes
 * per thread, nontemporal stores or not) on the current state, reps launches
 * each, and selects the fastest (results do not depend on the shape).  The
 * timed launches read the state's lattice and write the other lattice, which
 * the next step overwrites, so the state is unchanged.  The choice is
 * remembered for the process per (nx, ny, precision): contexts created later
 * with the same grid start with it (lbrmt_batch_autotune: per member count,
 * total nodes and precision, for batches).  best_variant / best_ms
 * (nullable): the choice and its time per launch.  Synchronises the stream.
 * ESTATE before init or on a batch member. */
int lbrmt_autotune(lbrmt_ctx* ctx, int32_t reps, int32_t* best_variant, double* best_ms);

/* Chooses LBRMT_OPT_FUSED_FIT between the one-launch extrapolation (1024) and
 * one launch per layer (0) by timing `steps` whole steps with each (rounded
 * up to whole six-step graphs, after about `steps` / 4 + 6 untimed ones); the
 * simulation advances by every step taken,
 * as lbrmt_step would (results do not depend on the choice).  Only a context
 * with one solid on walled axes and at most 11 layers has the choice; any
 * other leaves the option and the state as they are.  best_fused / best_ms
 * (nullable): the choice and its time per step.  Synchronises the stream.
 * ESTATE before init, on a batch member or with several solids; EINVAL for
 * steps < 1. */
int lbrmt_autotune_steps(lbrmt_ctx* ctx, int32_t steps, int32_t* best_fused, double* best_ms);

/* ---------------------------------------------------------------- batches
 * Many independent simulations (members) of any sizes stepped together: each
 * kernel of the step is one launch over all members, so a step costs the same
 * 17 launches whatever the member count, and blocks of six steps replay one
 * HIP graph.  Every member follows exactly the arithmetic of a single context
 * with the same description: results are bitwise identical to stepping each
 * member alone.  All members share the precision and the layer count; each
 * holds zero or one solid.  The batch carves one caller-owned device
 * workspace (member states plus the launch tables) and never allocates. */
typedef struct lbrmt_batch lbrmt_batch;

/* Workspace bytes for members descs[0..n-1].  EINVAL for an invalid
 * description, mixed precisions or mixed layer counts. */
int lbrmt_batch_workspace_bytes(const lbrmt_grid_desc* descs, int32_t n, size_t* bytes);

/* solids[k] is member k's solid when has_solid is NULL or has_solid[k] != 0;
 * solids NULL: no member has a solid.  d_workspace: 256-byte aligned device
 * memory of lbrmt_batch_workspace_bytes bytes; stream: caller's HIP stream
 * (all work of the batch and its members is ordered on it). */
int lbrmt_batch_create(const lbrmt_grid_desc* descs, const lbrmt_solid_desc* solids,
                       const int32_t* has_solid, int32_t n, void* d_workspace, size_t bytes,
                       void* hip_stream, lbrmt_batch** out);
void lbrmt_batch_destroy(lbrmt_batch* batch);
/* Alg. 1 initialisation of every member (fluid at rest). */
int lbrmt_batch_init(lbrmt_batch* batch);
/* nsteps time steps of every member; asynchronous on the stream. */
int lbrmt_batch_step(lbrmt_batch* batch, int64_t nsteps);
int32_t lbrmt_batch_size(const lbrmt_batch* batch);
/* Member k as a context for reads (lbrmt_read_*, lbrmt_diag, lbrmt_save_state,
 * lbrmt_step_count, lbrmt_band_nodes); lbrmt_step, lbrmt_load_state and
 * lbrmt_set_option on it return ESTATE.  Owned by the batch. */
lbrmt_ctx* lbrmt_batch_member(lbrmt_batch* batch, int32_t k);
/* LBRMT_OPT_LB_VARIANT (one tile shape for the whole batch),
 * LBRMT_OPT_GRAPH and LBRMT_OPT_FUSED_FIT (1024: every member's
 * extrapolation layers in one launch, member per grid row, when every member
 * has one solid on walled axes and at most 11 layers; 0, default, or -1: one
 * launch per layer over all members, faster for batches of many members;
 * results are bitwise identical); get also reads
 * LBRMT_OPT_LB_VARIANT_COUNT. */
int lbrmt_batch_set_option(lbrmt_batch* batch, int32_t option, int64_t value);
int lbrmt_batch_get_option(const lbrmt_batch* batch, int32_t option, int64_t* value);
/* lbrmt_autotune for the batched lattice update. */
int lbrmt_batch_autotune(lbrmt_batch* batch, int32_t reps, int32_t* best_variant,
                         double* best_ms);
const char* lbrmt_batch_last_error(const lbrmt_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* LBRMT_H */
