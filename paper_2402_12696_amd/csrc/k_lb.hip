// Lattice Boltzmann kernels of the LBRMT step on gfx950.
//
// Storage: nine structure-of-arrays planes per lattice, row pitch `pitch`, two
// lattices A/B.  A holds the post-collision populations of the previous step
// (a "pull" scheme): a node gathers f_i(x) = fhat_i(x - c_i) from its
// neighbours, or, when x - c_i is a wall, the reflected fhat_opp(i)(x) of its
// own node (halfway bounce-back, Sec. 3.5).  The moving-lid term of the
// reflected population is folded into the stored value when the top-row node
// writes it, using that node's density, so the gather is a plain copy.
//
// One thread per node; a workgroup covers a TX x TY tile.  Workgroup ids are
// remapped so that each XCD (8 on MI355X, round-robin dispatch) walks one
// contiguous slab of tiles and keeps the shared tile-edge cache lines in its
// own L2.
//
// FP64 path: f stored and computed in double.  FP32 path: the deviation
// f_i - w_i rho_f is stored in float and the arithmetic is float, so rho =
// rho_f + sum(df) keeps its small part.
#include "lb_node.h"

namespace lbrmt {

__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int per = nb / 8, rem = nb % 8;
    const int x = b % 8, k = b / 8;
    return x * per + min(x, rem) + k;
}

// Band region of a step: every interior node where the force of this step or
// of the previous one may differ from the uniform fluid force.
__device__ __forceinline__ Rect band_region(const GridP& g, const Rect& a, const Rect& b)
{
    Rect u;
    u.ok = a.ok || b.ok;
    if (!u.ok) return u;
    u.i0 = min(a.ok ? a.i0 : b.i0, b.ok ? b.i0 : a.i0);
    u.i1 = max(a.ok ? a.i1 : b.i1, b.ok ? b.i1 : a.i1);
    u.j0 = min(a.ok ? a.j0 : b.j0, b.ok ? b.j0 : a.j0);
    u.j1 = max(a.ok ? a.j1 : b.j1, b.ok ? b.j1 : a.j1);
    u.i0 = max(u.i0, 0);
    u.j0 = max(u.j0, 0);
    u.i1 = min(u.i1, g.nx - 1);
    u.j1 = min(u.j1, g.ny - 1);
    u.ok = u.i0 <= u.i1 && u.j0 <= u.j1;
    return u;
}

// Update of one tile of LB_TX x (LB_TY * R) nodes: each thread updates R
// nodes of one column, issuing all their gathers before any arithmetic so
// that more loads are in flight per wave.  PART 1 tiles (outside the band
// region) use the uniform fluid force; otherwise the force planes are read
// inside the windows of this and the previous step.
// VP, VC: where the force planes of the previous and of this step are held
// (Rect: a solid's window; StampValid: force-block stamps of several solids)
template <typename S, int PART, int LB_TX, int LB_TY, int R, bool NT, typename VP = Rect,
          typename VC = Rect>
__device__ __forceinline__ void lb_tile(const GridP& g, const S* __restrict__ A, S* __restrict__ B,
                                        const double* __restrict__ fpx,
                                        const double* __restrict__ fpy,
                                        const double* __restrict__ fcx,
                                        const double* __restrict__ fcy,
                                        const double* __restrict__ drho, const VP& wp,
                                        const VC& wc, double fpo_x, double fpo_y,
                                        unsigned* __restrict__ health, int tile_x, int tile_y)
{
    using C = typename Prec<S>::C;
    constexpr int TH = LB_TY * R;  // tile height
    const int tx = threadIdx.x % LB_TX, ty = threadIdx.x / LB_TX;
    const int i = tile_x * LB_TX + tx;
    if (i >= g.nx) return;
    Neigh q[R];
    bool ok[R];
    C f[R][NQ];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int j = tile_y * TH + ty + r * LB_TY;
        // PART 3 leaves the nodes of the current window to the force pass
        ok[r] = j < g.ny && !(PART == 3 && wc.has(i, j));
        q[r] = neigh(g, i, j < g.ny ? j : g.ny - 1);
        if (PART != 3 || ok[r]) gather<S>(g, q[r], A, f[r]);
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (!ok[r]) continue;
        const int j = tile_y * TH + ty + r * LB_TY;
        C Fpx = C(fpo_x), Fpy = C(fpo_y);
        C Fx = C(g.fext_x), Fy = C(g.fext_y), dr = C(0);
        if (PART != 1) {
            if (wp.has(i, j)) {
                Fpx = C(fpx[q[r].n]);
                Fpy = C(fpy[q[r].n]);
            }
            if (PART != 3 && wc.has(i, j)) {
                Fx = C(fcx[q[r].n]);
                Fy = C(fcy[q[r].n]);
                dr = C(drho[q[r].n]);
            }
        }
        lb_finish_node<S, NT>(g, B, q[r], f[r], Fpx, Fpy, Fx, Fy, dr, health);
    }
}

// PART 0: every tile, per-node window tests.  PART 1: tiles outside the band
// region only (uniform force).  PART 2: tiles of the band region only,
// grid-stride.  PART 3: every node outside the current window (whose nodes
// the force pass updates as soon as their force is known): this step's force
// is the uniform one there, the previous step's is read inside its window.
// PART 0 and PART 2 also reduce the force pass's nbox partial boxes of the
// new solid set into ring slot wnext (block 0, before anything else).
template <typename S, int PART, int LB_TX, int LB_TY, int R, bool NT>
__global__ __launch_bounds__(LB_TX* LB_TY) void k_lb(
    GridP g, const S* __restrict__ A, S* __restrict__ B, const double* __restrict__ fpx,
    const double* __restrict__ fpy, const double* __restrict__ fcx, const double* __restrict__ fcy,
    const double* __restrict__ drho, Win* win, int wprev, int wcur, double fpo_x, double fpo_y,
    unsigned* __restrict__ health, const int* __restrict__ boxpart, int nbox, int wnext,
    int tile0, int tile1, int split)
{
    if ((PART == 0 || PART == 2) && nbox > 0 && blockIdx.x == 0) {
        const Win r = reduce_boxes(boxpart, nbox, &win[wnext], nullptr);
        if (threadIdx.x == 0) check_zone(g, r, health);
    }
    constexpr int TH = LB_TY * R;
    const int ntx = (g.nx + LB_TX - 1) / LB_TX;
    const int nty = (g.ny + TH - 1) / TH;
    const Rect wp = window_of(win, wprev, g);
    // PART 3, split 1: the early launch, which may run before this step's
    // window is written, never reads it (its tiles lie below every node it
    // can hold)
    const Rect wc = PART == 3 && split == 1 ? Rect{0, -1, 0, -1, false} : window_of(win, wcur, g);
    // PART 3 split into an early and a held launch: the tile rows wholly
    // below the previous step's window by more than BULK_EARLY_GAP rows (none
    // without one) go to the early launch, up to its range tile0 .. tile1 - 1
    const int far_end = PART == 3 && split != 0 && wp.ok && wp.j0 - BULK_EARLY_GAP > 0
                            ? (wp.j0 - BULK_EARLY_GAP) / TH * ntx : 0;
    const Rect U = band_region(g, wp, wc);
    int t_begin, t_step, t_end;
    int utx0 = 0, uty0 = 0, untx = 1;
    if (PART == 2) {
        if (!U.ok) return;
        utx0 = U.i0 / LB_TX;
        uty0 = U.j0 / TH;
        untx = U.i1 / LB_TX - utx0 + 1;
        const int unty = U.j1 / TH - uty0 + 1;
        t_begin = blockIdx.x;
        t_step = gridDim.x;
        t_end = untx * unty;
    } else {
        // one tile per block, or a capped grid striding over the tiles, of
        // the tiles tile0 .. tile1 - 1 (PART 3; the others take all).  Split
        // 1 (early): the tiles of 0 .. tile1 - 1 before far_end; split 2
        // (held): every tile from min(tile0, far_end) on, striding
        int first = PART == 3 ? tile0 : 0;
        t_end = PART == 3 ? min(tile1, ntx * nty) : ntx * nty;
        if (PART == 3 && split == 1) t_end = min(t_end, far_end);
        if (PART == 3 && split == 2) first = min(tile0, far_end);
        t_begin = first + xcd_remap(blockIdx.x, gridDim.x);
        t_step = gridDim.x;
    }
    for (int t = t_begin; t < t_end; t += t_step) {
        int tile_x, tile_y;
        if (PART == 2) {
            tile_x = utx0 + t % untx;
            tile_y = uty0 + t / untx;
        } else {
            tile_x = t % ntx;
            tile_y = t / ntx;
            if (PART == 1 && U.ok) {
                const int x0 = tile_x * LB_TX, y0 = tile_y * TH;
                if (x0 <= U.i1 && x0 + LB_TX - 1 >= U.i0 && y0 <= U.j1 && y0 + TH - 1 >= U.j0)
                    continue;
            }
            if (PART == 3 && wc.ok) {
                // a tile inside the window (clipped to the interior) is the
                // force pass's
                const int x0 = tile_x * LB_TX, y0 = tile_y * TH;
                const int x1 = min(x0 + LB_TX, g.nx) - 1, y1 = min(y0 + TH, g.ny) - 1;
                if (x0 >= wc.i0 && x1 <= wc.i1 && y0 >= wc.j0 && y1 <= wc.j1) continue;
            }
        }
        lb_tile<S, PART, LB_TX, LB_TY, R, NT>(g, A, B, fpx, fpy, fcx, fcy, drho, wp, wc, fpo_x,
                                              fpo_y, health, tile_x, tile_y);
    }
}

// Batched form over the concatenated tile lists of every member: block b
// takes tile t = xcd_remap(b) of member tile_sim[t].
template <typename S, int LB_TX, int LB_TY, int R, bool NT>
__global__ __launch_bounds__(LB_TX* LB_TY) void kb_lb(const LbArgs* __restrict__ args,
                                                     const int* __restrict__ tile_sim)
{
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const LbArgs& a = args[tile_sim[t]];
    const int local = t - a.tile_base;
    // the member's first tile reduces the force pass's partial boxes
    if (local == 0 && a.nbox > 0) {
        const Win r = reduce_boxes(a.boxpart, a.nbox, &a.winw[a.wnext], nullptr);
        if (threadIdx.x == 0) check_zone(a.g, r, a.health);
    }
    const int ntx = (a.g.nx + LB_TX - 1) / LB_TX;
    const Rect wp = window_of(a.win, a.wprev, a.g);
    const Rect wc = window_of(a.win, a.wcur, a.g);
    lb_tile<S, 0, LB_TX, LB_TY, R, NT>(a.g, (const S*)a.A, (S*)a.B, a.fpx, a.fpy, a.fcx, a.fcy,
                                       a.drho, wp, wc, a.fpo_x, a.fpo_y, a.health, local % ntx,
                                       local / ntx);
}

// Several solids: every tile, force planes where the block stamps say so.
template <typename S, int LB_TX, int LB_TY, int R, bool NT>
__global__ __launch_bounds__(LB_TX* LB_TY) void k_lb_mb(
    GridP g, const S* __restrict__ A, S* __restrict__ B, const double* __restrict__ fpx,
    const double* __restrict__ fpy, const double* __restrict__ fcx, const double* __restrict__ fcy,
    const double* __restrict__ drho, StampValid vp, StampValid vc, double fpo_x, double fpo_y,
    unsigned* __restrict__ health, const long long* __restrict__ dstep)
{
    constexpr int TH = LB_TY * R;
    const int ntx = (g.nx + LB_TX - 1) / LB_TX;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    vp.val = (int)*dstep;
    vc.val = vp.val + 1;
    lb_tile<S, 0, LB_TX, LB_TY, R, NT, StampValid, StampValid>(
        g, A, B, fpx, fpy, fcx, fcy, drho, vp, vc, fpo_x, fpo_y, health, t % ntx, t / ntx);
    (void)TH;
}

// Tile shapes of the lattice Boltzmann update: tx x ty threads (tx * ty / 64
// waves per workgroup), r nodes per thread (rows ty apart), nontemporal
// stores or not; the variant is chosen per context (lbrmt_set_option) by
// measurement (lbrmt_autotune).
struct LbVariant {
    int tx, ty, r;
    bool nt;
};
constexpr LbVariant LB_VARIANTS[] = {
    {64, 4, 1, false}, {128, 2, 1, false}, {256, 1, 1, false}, {64, 4, 1, true},
    {128, 2, 1, true}, {256, 1, 1, true},  {32, 8, 1, false},  {64, 2, 1, false},
    {256, 1, 2, true}, {256, 1, 4, true},  {512, 1, 1, true},  {512, 1, 2, true},
    {128, 2, 2, true}, {256, 1, 2, false},
    // eight waves per workgroup, one or two waves, and eight waves with two
    // nodes per thread
    {64, 8, 1, true},  {128, 4, 1, true},  {256, 2, 1, true},  {128, 1, 1, true},
    {64, 1, 1, true},  {128, 4, 2, true}};
constexpr int N_LB_VARIANTS = sizeof(LB_VARIANTS) / sizeof(LB_VARIANTS[0]);

int lb_variant_count() { return N_LB_VARIANTS; }
void lb_variant_tile(int v, int* tx, int* ty)
{
    *tx = LB_VARIANTS[v].tx;
    *ty = LB_VARIANTS[v].ty * LB_VARIANTS[v].r;
}

// PART 3 takes tiles [frac0, frac1) / 1000 of the grid's tiles (row by row)
template <typename S, int PART, int TX, int TY, int R, bool NT>
static void lb_launch_one(const GridP& g, const void* A, void* B, const double* fpx,
                          const double* fpy, const double* fcx, const double* fcy,
                          const double* drho, Win* win, int wprev, int wcur, double fpo_x,
                          double fpo_y, int max_blocks, unsigned* health, hipStream_t st,
                          const int* boxpart, int nbox, int wnext, int frac0, int frac1,
                          int split)
{
    const int ntiles = ((g.nx + TX - 1) / TX) * ((g.ny + TY * R - 1) / (TY * R));
    int t0 = 0, t1 = ntiles;
    if (PART == 3) {
        t0 = (int)((long long)ntiles * frac0 / 1000);
        t1 = (int)((long long)ntiles * frac1 / 1000);
    }
    // (the held launch also takes the early range's tiles that the early
    // launch leaves, so it runs, striding, even when its own range is empty)
    const bool held = PART == 3 && split == 2;
    if (t1 <= t0 && !held) return;
    int grid = PART == 2 ? (ntiles < 2048 ? ntiles : 2048) : t1 - t0;
    if (held && grid < 256) grid = ntiles < 256 ? ntiles : 256;
    if ((PART == 1 || PART == 3) && max_blocks > 0 && max_blocks < grid) grid = max_blocks;
    k_lb<S, PART, TX, TY, R, NT><<<grid, TX * TY, 0, st>>>(g, (const S*)A, (S*)B, fpx, fpy, fcx,
                                                          fcy, drho, win, wprev, wcur, fpo_x,
                                                          fpo_y, health, boxpart, nbox, wnext,
                                                          t0, t1, split);
}

template <typename S, int PART>
static void lb_launch_variant(int v, const GridP& g, const void* A, void* B, const double* fpx,
                              const double* fpy, const double* fcx, const double* fcy,
                              const double* drho, Win* win, int wprev, int wcur,
                              double fpo_x, double fpo_y, int max_blocks, unsigned* health,
                              hipStream_t st, const int* boxpart, int nbox, int wnext,
                              int frac0, int frac1, int split)
{
#define LBV(TX, TY, R, NT)                                                                       \
    lb_launch_one<S, PART, TX, TY, R, NT>(g, A, B, fpx, fpy, fcx, fcy, drho, win, wprev, wcur, \
                                          fpo_x, fpo_y, max_blocks, health, st, boxpart, nbox,  \
                                          wnext, frac0, frac1, split)
    switch (v) {
    case 1: LBV(128, 2, 1, false); break;
    case 2: LBV(256, 1, 1, false); break;
    case 3: LBV(64, 4, 1, true); break;
    case 4: LBV(128, 2, 1, true); break;
    case 5: LBV(256, 1, 1, true); break;
    case 6: LBV(32, 8, 1, false); break;
    case 7: LBV(64, 2, 1, false); break;
    case 8: LBV(256, 1, 2, true); break;
    case 9: LBV(256, 1, 4, true); break;
    case 10: LBV(512, 1, 1, true); break;
    case 11: LBV(512, 1, 2, true); break;
    case 12: LBV(128, 2, 2, true); break;
    case 13: LBV(256, 1, 2, false); break;
    case 14: LBV(64, 8, 1, true); break;
    case 15: LBV(128, 4, 1, true); break;
    case 16: LBV(256, 2, 1, true); break;
    case 17: LBV(128, 1, 1, true); break;
    case 18: LBV(64, 1, 1, true); break;
    case 19: LBV(128, 4, 2, true); break;
    default: LBV(64, 4, 1, false); break;
    }
#undef LBV
}

hipError_t launch_lb(const GridP& g, int precision, int variant, const void* A, void* B,
                     const double* fpx, const double* fpy, const double* fcx, const double* fcy,
                     const double* drho, Win* win, int wprev, int wcur, double fpo_x,
                     double fpo_y, int part, unsigned* health, hipStream_t st, int max_blocks,
                     const int* boxpart, int nbox, Win* winw, int wnext, int frac0, int frac1,
                     int split)
{
    (void)winw;
#define LBP(S, PARTV)                                                                        \
    lb_launch_variant<S, PARTV>(variant, g, A, B, fpx, fpy, fcx, fcy, drho, win, wprev, wcur, \
                                fpo_x, fpo_y, max_blocks, health, st, boxpart, nbox, wnext,  \
                                frac0, frac1, split)
    if (precision == 0) {
        if (part == 0) LBP(double, 0);
        else if (part == 1) LBP(double, 1);
        else if (part == 2) LBP(double, 2);
        else LBP(double, 3);
    } else {
        if (part == 0) LBP(float, 0);
        else if (part == 1) LBP(float, 1);
        else if (part == 2) LBP(float, 2);
        else LBP(float, 3);
    }
#undef LBP
    return hipGetLastError();
}

template <typename S>
static void lb_batch_variant(int v, const LbArgs* args, const int* tile_sim, int total,
                             hipStream_t st)
{
#define LBB(TX, TY, R, NT) kb_lb<S, TX, TY, R, NT><<<total, TX * TY, 0, st>>>(args, tile_sim)
    switch (v) {
    case 1: LBB(128, 2, 1, false); break;
    case 2: LBB(256, 1, 1, false); break;
    case 3: LBB(64, 4, 1, true); break;
    case 4: LBB(128, 2, 1, true); break;
    case 5: LBB(256, 1, 1, true); break;
    case 6: LBB(32, 8, 1, false); break;
    case 7: LBB(64, 2, 1, false); break;
    case 8: LBB(256, 1, 2, true); break;
    case 9: LBB(256, 1, 4, true); break;
    case 10: LBB(512, 1, 1, true); break;
    case 11: LBB(512, 1, 2, true); break;
    case 12: LBB(128, 2, 2, true); break;
    case 13: LBB(256, 1, 2, false); break;
    case 14: LBB(64, 8, 1, true); break;
    case 15: LBB(128, 4, 1, true); break;
    case 16: LBB(256, 2, 1, true); break;
    case 17: LBB(128, 1, 1, true); break;
    case 18: LBB(64, 1, 1, true); break;
    case 19: LBB(128, 4, 2, true); break;
    default: LBB(64, 4, 1, false); break;
    }
#undef LBB
}

template <typename S, int TX, int TY, int R, bool NT>
static void lb_mb_one(const GridP& g, const void* A, void* B, const double* fpx,
                      const double* fpy, const double* fcx, const double* fcy,
                      const double* drho, StampValid vp, StampValid vc, double fpo_x,
                      double fpo_y, unsigned* health, hipStream_t st, const long long* dstep)
{
    const int ntiles = ((g.nx + TX - 1) / TX) * ((g.ny + TY * R - 1) / (TY * R));
    k_lb_mb<S, TX, TY, R, NT><<<ntiles, TX * TY, 0, st>>>(g, (const S*)A, (S*)B, fpx, fpy, fcx,
                                                         fcy, drho, vp, vc, fpo_x, fpo_y,
                                                         health, dstep);
}

hipError_t launch_lb_mb(const GridP& g, int precision, int variant, const void* A, void* B,
                        const double* fpx, const double* fpy, const double* fcx,
                        const double* fcy, const double* drho, StampValid vp, StampValid vc,
                        double fpo_x, double fpo_y, unsigned* health, hipStream_t st,
                        const long long* dstep)
{
    // the measured single-solid choices: 64 x 4 (FP64), 256 x 1 (FP32), nontemporal stores
    (void)variant;
    if (precision == 0)
        lb_mb_one<double, 64, 4, 1, true>(g, A, B, fpx, fpy, fcx, fcy, drho, vp, vc, fpo_x,
                                          fpo_y, health, st, dstep);
    else
        lb_mb_one<float, 256, 1, 1, true>(g, A, B, fpx, fpy, fcx, fcy, drho, vp, vc, fpo_x,
                                          fpo_y, health, st, dstep);
    return hipGetLastError();
}

hipError_t launch_lb_batch(int precision, int variant, const LbArgs* args, const int* tile_sim,
                           int total_tiles, hipStream_t st)
{
    if (total_tiles <= 0) return hipSuccess;
    if (precision == 0) lb_batch_variant<double>(variant, args, tile_sim, total_tiles, st);
    else lb_batch_variant<float>(variant, args, tile_sim, total_tiles, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------- initialisation

// f^0 = f^eq_SFC(rho_0, v_0, drho_0) in natural (pre-collision) layout
template <typename S>
__global__ void k_init_feq(GridP g, BodyP b, const S* __restrict__ phi0,
                           const Win* __restrict__ win, int wslot, const double* __restrict__ u0,
                           S* __restrict__ T, const double* __restrict__ drho0)
{
    const long long N = (long long)g.nx * g.ny;
    const Rect w = window_of(win, wslot, g);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        double H = 1.0;
        if (b.present && w.has(i, j)) {
            const double ph = (double)phi0[pidx(g, i, j)];
            if (ph < INFINITY) {
                // smoothed Heaviside, Eq. (2_3_heaviside)
                if (ph <= -g.eps) H = 0.0;
                else if (ph >= g.eps) H = 1.0;
                else H = 0.5 * (1.0 + ph / g.eps + sin(M_PI * ph / g.eps) / M_PI);
            }
        }
        const double rs = b.present ? b.rho_s : g.rho_f;
        double rho = H * g.rho_f + (1.0 - H) * rs;  // Eq. (2_4_smooth_density)
        double dr = rho - g.rho_f;                  // Eq. (2_3_drho) with rho = rho_t
        if (drho0) {
            // several solids: rho_f plus the normalised mixture excess
            dr = drho0[(long long)j * g.pitch + i];
            rho = g.rho_f + dr;
        }
        const double ux = u0 ? u0[e] : 0.0, uy = u0 ? u0[N + e] : 0.0;
        const double usq = ux * ux + uy * uy;
        const long long n = (long long)j * g.pitch + i;
        const double cu[NQ] = {0.0, ux, uy, -ux, -uy, ux + uy, uy - ux, -ux - uy, ux - uy};
        const double wq[NQ] = {W0, W1, W1, W1, W1, W2, W2, W2, W2};
        for (int k = 0; k < NQ; k++) {
            double fe = wq[k] * rho * (1.0 + 3.0 * cu[k] + 4.5 * cu[k] * cu[k] - 1.5 * usq);
            fe += k == 0 ? (5.0 / 9.0) * dr : -wq[k] * dr;
            if (Prec<S>::dev) fe -= wq[k] * g.rho_f;
            T[k * g.plane + n] = S(fe);
        }
    }
}

// A such that the pull gather of A reproduces T: A_i(y) = T_i(y + c_i), or
// T_opp(i)(y) where y + c_i lies beyond a wall.
template <typename S>
__global__ void k_inverse_stream(GridP g, const S* __restrict__ T, S* __restrict__ A)
{
    const int CXv[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int CYv[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const int OPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const long long N = (long long)g.nx * g.ny;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        const long long n = (long long)j * g.pitch + i;
        for (int k = 0; k < NQ; k++) {
            int id = i + CXv[k], jd = j + CYv[k];
            if (g.px) id = wrap_axis(id, g.nx);
            if (g.py) jd = wrap_axis(jd, g.ny);
            const bool inside = id >= 0 && id < g.nx && jd >= 0 && jd < g.ny;
            A[k * g.plane + n] = inside ? T[k * g.plane + (long long)jd * g.pitch + id]
                                        : T[OPP[k] * g.plane + n];
        }
    }
}

hipError_t launch_init_populations(const GridP& g, int precision, const BodyP& b,
                                   const void* phi0, const Win* win, int wslot,
                                   const double* u0, void* tmp, void* A, hipStream_t st,
                                   const double* drho0)
{
    const long long N = (long long)g.nx * g.ny;
    const int blocks = (int)((N + 255) / 256 < 8192 ? (N + 255) / 256 : 8192);
    if (precision == 0) {
        k_init_feq<double><<<blocks, 256, 0, st>>>(g, b, (const double*)phi0, win, wslot, u0,
                                                   (double*)tmp, drho0);
        k_inverse_stream<double><<<blocks, 256, 0, st>>>(g, (const double*)tmp, (double*)A);
    } else {
        k_init_feq<float><<<blocks, 256, 0, st>>>(g, b, (const float*)phi0, win, wslot, u0,
                                                  (float*)tmp, drho0);
        k_inverse_stream<float><<<blocks, 256, 0, st>>>(g, (const float*)tmp, (float*)A);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- reads

template <typename S>
__global__ void k_gather_macro(GridP g, const S* __restrict__ A, const double* __restrict__ fpx,
                               const double* __restrict__ fpy, const Win* __restrict__ win,
                               int wprev, double fpo_x, double fpo_y, double* rho_o,
                               double* ux_o, double* uy_o, double* f9, StampValid sv)
{
    const long long N = (long long)g.nx * g.ny;
    const Rect wr = window_of(win, wprev, g);
    const double wq[NQ] = {W0, W1, W1, W1, W1, W2, W2, W2, W2};
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        const Neigh q = neigh(g, i, j);
        double f[NQ];
        {
            typename Prec<S>::C fs[NQ];
            gather<S>(g, q, A, fs);
            for (int k = 0; k < NQ; k++)
                f[k] = Prec<S>::dev ? (double)fs[k] + wq[k] * g.rho_f : (double)fs[k];
        }
        const double rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
        double Fx = fpo_x, Fy = fpo_y;
        if (sv.stamp ? sv.has(i, j) : wr.has(i, j)) {
            Fx = fpx[q.n];
            Fy = fpy[q.n];
        }
        if (rho_o) rho_o[e] = rho;
        if (ux_o) ux_o[e] = (f[1] + f[5] + f[8] - f[3] - f[6] - f[7]) / rho + Fx / (2.0 * rho);
        if (uy_o) uy_o[e] = (f[2] + f[5] + f[6] - f[4] - f[7] - f[8]) / rho + Fy / (2.0 * rho);
        if (f9)
            for (int k = 0; k < NQ; k++) f9[k * N + e] = f[k];
    }
}

hipError_t launch_gather_macro(const GridP& g, int precision, const void* A, const double* fpx,
                               const double* fpy, const Win* win, int wprev, double fpo_x,
                               double fpo_y, double* rho, double* ux, double* uy, double* f9,
                               hipStream_t st, StampValid sv)
{
    const long long N = (long long)g.nx * g.ny;
    const int blocks = (int)((N + 255) / 256 < 8192 ? (N + 255) / 256 : 8192);
    if (precision == 0)
        k_gather_macro<double><<<blocks, 256, 0, st>>>(g, (const double*)A, fpx, fpy, win, wprev,
                                                       fpo_x, fpo_y, rho, ux, uy, f9, sv);
    else
        k_gather_macro<float><<<blocks, 256, 0, st>>>(g, (const float*)A, fpx, fpy, win, wprev,
                                                      fpo_x, fpo_y, rho, ux, uy, f9, sv);
    return hipGetLastError();
}

__global__ void k_read_force(GridP g, const double* __restrict__ fpx, const double* __restrict__ fpy,
                             const Win* __restrict__ win, int wprev, double fpo_x, double fpo_y,
                             double* fx, double* fy, StampValid sv)
{
    const long long N = (long long)g.nx * g.ny;
    const Rect wp = window_of(win, wprev, g);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        const long long n = (long long)j * g.pitch + i;
        const bool in = sv.stamp ? sv.has(i, j) : wp.has(i, j);
        fx[e] = in ? fpx[n] : fpo_x;
        fy[e] = in ? fpy[n] : fpo_y;
    }
}

hipError_t launch_read_force(const GridP& g, const double* fpx, const double* fpy, const Win* win,
                             int wprev, double fpo_x, double fpo_y, double* fx, double* fy,
                             hipStream_t st, StampValid sv)
{
    const long long N = (long long)g.nx * g.ny;
    const int blocks = (int)((N + 255) / 256 < 8192 ? (N + 255) / 256 : 8192);
    k_read_force<<<blocks, 256, 0, st>>>(g, fpx, fpy, win, wprev, fpo_x, fpo_y, fx, fy, sv);
    return hipGetLastError();
}

template <typename S>
__global__ void k_poke(GridP g, S* A, long long node, double value)
{
    const int i = (int)(node % g.nx), j = (int)(node / g.nx);
    const long long n = (long long)j * g.pitch + i;
    if (threadIdx.x < NQ) A[threadIdx.x * g.plane + n] = S(value);
}

hipError_t launch_poke(const GridP& g, int precision, void* A, long long node, double value,
                       hipStream_t st)
{
    if (precision == 0) k_poke<double><<<1, 64, 0, st>>>(g, (double*)A, node, value);
    else k_poke<float><<<1, 64, 0, st>>>(g, (float*)A, node, value);
    return hipGetLastError();
}

}  // namespace lbrmt
