// Internal declarations of the gfx950 LBRMT library: kernel parameter blocks,
// grid helpers and the host-side launchers of every kernel.  Not installed;
// the public ABI is include/lbrmt.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbrmt {

constexpr int NQ = 9;   // D2Q9 (Sec. 2.2, Table "d2q9")
constexpr int PAD = 2;  // buffer layers of the reference-map grid (Sec. 3)

// Tag codes of the reference-map nodes during one step (int8 per node).
constexpr int TAG_NONE = -1;   // no reference map
constexpr int TAG_SOLID = 0;   // phi^n < 0, interior
constexpr int TAG_FAIL = 64;   // OR-ed onto a layer number when the fit failed
constexpr int MAX_LAYERS = 31;

// Launch shapes of the reference-map chain.
constexpr int BOX_BLOCKS = 512;       // initial solid box
// force pass (relabel, stress divergence, the window's lattice update): one
// partial box per block; 1024 blocks striding over the window's 32 x 8 tiles
// (2048^2 FP32 step 0.1072 -> 0.1064 ms against 2048, FP64 the same; 4096
// and 512 slower)
constexpr int RELABEL_BLOCKS = 1024;
constexpr int DT_BLOCKS = 2048;       // distance transform
constexpr int ADV_MIN_WORKERS = 256;  // advection blocks beside the distance transform (one solid)
constexpr int FIT_BLOCKS = 256;       // one extrapolation layer
constexpr int FIT_LANES = 8;          // lanes sharing one extrapolation target
constexpr int LCOUNT_PAD = 32;        // layer counters 128 B apart
constexpr int NSUB = 8;               // sub-lists per layer (distance-transform block mod 8)
constexpr int FF_TILE = 32;           // fused extrapolation: tile side
constexpr int FF_LAYERS = 11;         // fused extrapolation: most layers
constexpr int FF_BLOCKS = 256;        // fused extrapolation: blocks striding over its tile list
constexpr int FF_NO_CUT = 127;        // tile not stopped (cut_layer)
constexpr int FF_REST_THREADS = 256;  // fused extrapolation: the one-block pass
constexpr int FF_NORMALS = 1024;      // fused extrapolation: layer-1/2 normals found up front
constexpr int FF_BATCH_BLOCKS = 64;   // fused extrapolation of a batch: blocks per member

// Several solids: the lattice is cut into force blocks of FB x FB nodes;
// a block holds valid force planes at step n when its stamp equals n + 1.
constexpr int FB_LOG = 4;
constexpr int FB = 1 << FB_LOG;
// advection and distance transform of several solids: blocks per solid (a
// multiple of NSUB); 8 (each block taking about two tiles of a solid's
// window): 4096^2 suspension of 400 solids FP32 step 0.590 -> 0.540 ms
// against 16 (24: 0.546)
constexpr int MB_DT_BLOCKS = 8;
// relabel of several solids: two partial boxes per block, 8 blocks per
// solid (4096^2 suspension of 400 solids: FP32 step 0.6157 -> 0.6120 ms
// against 16, 0.637 at 32; 4 as fast as 8)
constexpr int MB_BAND_BLOCKS = 8;
// one block per solid runs all its layers; 768 threads leave 170 registers a
// lane (1024 would leave 128, and both precisions would spill)
constexpr int MB_FIT_THREADS_F64 = 768;
constexpr int MB_FIT_THREADS_F32 = 768;
// nodes of a several-solid fit block's LDS copy (its window dilated by 2)
constexpr int MB_FIT_LDS_NODES = 8192;
constexpr int MB_MAX_PER_BLOCK = 32;  // solids overlapping one force block
// force combine of several solids: blocks striding over the stamped force
// blocks (4096: suspension FP32 step 0.5416 -> 0.5370 ms against 2048)
constexpr int MB_COMBINE_BLOCKS = 4096;
// a sub-window moves when its solid's zone comes this close to its border
constexpr int MB_RECENTRE_MARGIN = 4;
// the early part of a held bulk update takes tile rows wholly below the
// previous step's window by more than this many rows; a solid box whose
// lower edge moves down by more than this in one step is counted in
// health[6] (the early launch may then have updated nodes of the window)
constexpr int BULK_EARLY_GAP = 2;

// Axis-aligned box of the interior solid nodes of one body (i0 > i1: empty).
// The working window of a step is this box dilated by `layers` nodes.
struct Win {
    int i0, i1, j0, j1;
};

struct GridP {
    int nx, ny;
    int pitch;            // lattice row pitch (elements)
    int pp;               // reference-map row pitch (elements), nx + 4 rounded up
    long long plane;      // lattice plane stride = pitch * ny
    long long pplane;     // reference-map plane stride = pp * (ny + 4)
    int px, py;           // periodic axes
    int layers, r_max;
    double omega;         // 1 / tau
    double cforce;        // 1 - 1 / (2 tau)
    double lid_ux;
    double gx, gy, fext_x, fext_y;
    double rho_f, eps;
    double det_rel, detJ_min;
    int rm32;             // reference map stored in FP32 as displacement xi - x
    // the lattice seen from a reference-map grid.  A solid of a several-solid
    // context keeps its map on a window of its own: along an axis flagged in
    // wx / wy the window is the sub-range [o, o + n) of a periodic lattice
    // axis (window node i is lattice column (i + ox) mod lnx, at position
    // i + ox + 1/2, and the window axis itself is not periodic); along other
    // axes the window is the whole lattice axis (o = 0).
    int ox, oy;
    int wx, wy;
    int lnx, lny;         // lattice extents
    int lpx, lpy;         // lattice periodic axes
    double eta;           // contact factor of Eq. (3_6_collision_stress)
    long long lcap;       // capacity of one layer sub-list (entries)
    // det(grad xi) below which the FP32 reference-map path inverts grad xi
    // in FP64 (near-singular maps, J -> 0 of Eq. (3_3_refmap_deformation))
    double kappa_J;
    int lid_rho_mode;     // moving-lid density: 0 the node's rho, 1 rho_f
};

struct BodyP {
    int present;
    int shape;            // 0 disc of radius R; 1 ellipse of semi-axes R and Rb
    double cx, cy, R, G, rho_s;
    double Rb;            // ellipse semi-axis b
    double ct, st;        // cos, sin of the angle of the R axis (host libm)
};

// Step-invariant pointers of the reference-map state.
struct BandBufs {
    // reference map components, padded grid, double-buffered: xi itself in
    // double (FP64 mode) or the displacement xi - x in float (FP32 mode)
    void* X[2];
    void* Y[2];
    void* phi[2];         // level set (double / float); +inf where no reference map
    int8_t* tag;          // TAG_* or layer number, padded grid
    int8_t* gcol;         // column distance to the solid (distance transform)
    int* lists;           // zone nodes of layer l, sub-list s at lists + (l * NSUB + s) * sub_cap
    int* lcount;          // entries of (l, s) at lcount[(l * NSUB + s) * LCOUNT_PAD]
    int* boxpart;         // per-block partial boxes, RELABEL_BLOCKS x 4
    unsigned* ticket;     // arrival counter of last-block reductions
    Win* win;             // ring of 3 boxes
    unsigned* health;
    // fused extrapolation: per window tile the layer where it stopped
    // (FF_NO_CUT between steps), the stopped tiles and their count
    int8_t* cut_layer;
    int* cut_tiles;
    int* ncut;
    // fused extrapolation: the tiles the zone reaches, listed once each by
    // the distance transform (flag per tile, list, count; cleared each step)
    int* ff_flag;
    int* ff_list;
    int* ff_n;
};

// ---- box reductions (wave64 shuffles + LDS)

__device__ __forceinline__ int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Reduces n partial boxes {i0, i1, j0, j1} (one block; every thread calls it)
// into *dst0 (and *dst1 when not null), and returns it in thread 0; an empty
// result is the empty box.
// SAME_KERNEL: the partials were written by other blocks of the running
// kernel (read through volatile loads after the last-block handshake);
// otherwise by an earlier kernel (plain loads, all issued at once).
template <bool SAME_KERNEL = false>
__device__ inline Win reduce_boxes(const int* part, int n, Win* dst0, Win* dst1)
{
    Win r{};
    __shared__ int sb[4][16];
    int a0 = 0x3fffffff, a1 = -0x3fffffff, a2 = 0x3fffffff, a3 = -0x3fffffff;
    if (SAME_KERNEL) {
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const volatile int* q = part + 4 * k;
            a0 = min(a0, q[0]);
            a1 = max(a1, q[1]);
            a2 = min(a2, q[2]);
            a3 = max(a3, q[3]);
        }
    } else {
        // eight partials per thread in flight at a time
        constexpr int NB = 8;
        const int4* p4 = reinterpret_cast<const int4*>(part);
        for (int k0 = threadIdx.x; k0 < n; k0 += NB * blockDim.x) {
            int4 q[NB];
#pragma unroll
            for (int u = 0; u < NB; u++) {
                const int k = k0 + u * blockDim.x;
                q[u] = p4[k < n ? k : 0];
            }
#pragma unroll
            for (int u = 0; u < NB; u++) {
                if (k0 + u * (int)blockDim.x >= n) continue;
                a0 = min(a0, q[u].x);
                a1 = max(a1, q[u].y);
                a2 = min(a2, q[u].z);
                a3 = max(a3, q[u].w);
            }
        }
    }
    a0 = wave_min(a0);
    a1 = wave_max(a1);
    a2 = wave_min(a2);
    a3 = wave_max(a3);
    const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int nw = (blockDim.x + 63) / 64;
    if (lane == 0) {
        sb[0][wid] = a0;
        sb[1][wid] = a1;
        sb[2][wid] = a2;
        sb[3][wid] = a3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; w++) {
            a0 = min(a0, sb[0][w]);
            a1 = max(a1, sb[1][w]);
            a2 = min(a2, sb[2][w]);
            a3 = max(a3, sb[3][w]);
        }
        r.i0 = a0;
        r.i1 = a1;
        r.j0 = a2;
        r.j1 = a3;
        if (a0 > a1) r.i0 = 0x3fffffff, r.i1 = -0x3fffffff, r.j0 = 0x3fffffff, r.j1 = -0x3fffffff;
        *dst0 = r;
        if (dst1) *dst1 = r;
    }
    __syncthreads();
    return r;  // the box, in thread 0
}

// A zone (box dilated by `layers`) that would cross a periodic seam of a
// whole-axis grid, or leave a solid's sub-window, is not representable by the
// working window: counted in health[6] (called by one thread).
__device__ __forceinline__ void check_zone(const GridP& g, const Win& w, unsigned* health)
{
    if (w.i0 > w.i1) return;
    const int L = g.layers;
    if (((g.px || g.wx) && (w.i0 - L < 0 || w.i1 + L > g.nx - 1)) ||
        ((g.py || g.wy) && (w.j0 - L < 0 || w.j1 + L > g.ny - 1)))
        atomicAdd(&health[6], 1u);
}

// Arguments of the step kernels for one member of a batch (device tables,
// one entry per member; the batched kernels take member blockIdx.y).  Plane
// pointers are untyped: the batch precision picks the kernel instance.
struct AdvectArgs {
    GridP g;
    const void* A;
    const double *fpx, *fpy;
    const void *X, *Y, *phi;
    void *X1, *Y1;
    int8_t* tag;
    const Win* win;
    int wprev, wcur;
    int* lists;
    int* lcount;
    unsigned* health;
    // the fused extrapolation's zone-tile list (null: not built)
    int *ff_flag, *ff_list, *ff_n;
};
struct LayersArgs {
    GridP g;
    const Win* win;
    int wslot;
    int8_t* tag;
    int8_t* gcol;
    int* lists;
    int* lcount;
    unsigned* health;
};
struct FitArgs {
    GridP g;
    const Win* win;
    int wcur, wprev;
    int8_t* tag;
    const int* lists;
    const int* lcount;
    const void* phin;
    void *X1, *Y1;
    unsigned* health;
    // the fused extrapolation's buffers (batches of single-solid members)
    int8_t* cut_layer;
    int *cut_tiles, *ncut, *ff_flag, *ff_list, *ff_n;
};
struct EdgesArgs {
    GridP g;
    BodyP b;
    Win* win;
    int wvalid;
    int* boxpart;
    void *X, *Y;
    const int8_t* tag;
    void* phi;  // written: the relabelled level set
    double *o0, *o1, *o2;
    int* lcount;
    unsigned* health;
};
struct LbArgs {
    GridP g;
    const void* A;
    void* B;
    const double *fpx, *fpy, *fcx, *fcy, *drho;
    const Win* win;
    int wprev, wcur;
    double fpo_x, fpo_y;
    unsigned* health;
    int tile_base;  // first entry of this member in the flattened tile list
    Win* winw;      // the ring, for the reduction of the force pass's boxes
    const int* boxpart;
    int nbox, wnext;
};
struct BatchTables {
    AdvectArgs* adv;
    LayersArgs* lay;
    FitArgs* fit;
    EdgesArgs* edg;
    LbArgs* lb;
    // the table row that block row y of the advection and extrapolation
    // passes takes (null: row y)
    const int* ord = nullptr;
};
// blocks per member of the batched reference-map kernels (the distance
// transform count is a multiple of NSUB and at most DT_BLOCKS, which the list
// capacity assumes; relabel's partial boxes number BATCH_BAND_BLOCKS)
constexpr int BATCH_BAND_BLOCKS = 128;
constexpr int BATCH_DT_BLOCKS = 128;
constexpr int BATCH_FIT_BLOCKS = 32;

// Selection of the ring slots / buffers at state n (n completed steps).
struct StepSlots {
    int cur;      // n % 2   : state buffers (lattice A, xi^n, F^n written this step)
    int nxt;      // (n+1)%2 : lattice B, xi^{n+1}, F^{n-1}
    int wprev;    // (n+2)%3 : box of S^{n-1}; window over which xi^n, phi^n, F^{n-1} are valid
    int wcur;     // n % 3   : box of S^n
    int wnext;    // (n+1)%3 : box of S^{n+1}, built by relabel
};

inline StepSlots slots_for(long long n)
{
    StepSlots s;
    s.cur = (int)(n % 2);
    s.nxt = (int)((n + 1) % 2);
    s.wprev = (int)((n + 2) % 3);
    s.wcur = (int)(n % 3);
    s.wnext = (int)((n + 1) % 3);
    return s;
}

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ int wrap_axis(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Dilated, clipped working window of box b (false if empty).
__device__ __forceinline__ bool dilate_window(const Win& b, const GridP& g, int& i0, int& i1,
                                              int& j0, int& j1)
{
    if (b.i0 > b.i1 || b.j0 > b.j1) return false;
    const int L = g.layers;
    const int lox = g.px ? 0 : -PAD, hix = g.px ? g.nx - 1 : g.nx + PAD - 1;
    const int loy = g.py ? 0 : -PAD, hiy = g.py ? g.ny - 1 : g.ny + PAD - 1;
    i0 = max(b.i0 - L, lox);
    i1 = min(b.i1 + L, hix);
    j0 = max(b.j0 - L, loy);
    j1 = min(b.j1 + L, hiy);
    return i0 <= i1 && j0 <= j1;
}

struct Rect {
    int i0, i1, j0, j1;
    bool ok;
    __device__ __forceinline__ bool has(int i, int j) const
    {
        return ok && i >= i0 && i <= i1 && j >= j0 && j <= j1;
    }
};

__device__ __forceinline__ Rect window_of(const Win* win, int slot, const GridP& g)
{
    Rect r;
    Win b = win[slot];
    r.ok = dilate_window(b, g, r.i0, r.i1, r.j0, r.j1);
    return r;
}

// Wrap periodic axes; false if (i, j) is outside the reference-map domain.
__device__ __forceinline__ bool canon(const GridP& g, int& i, int& j)
{
    if (g.px) i = wrap_axis(i, g.nx);
    else if (i < -PAD || i > g.nx + PAD - 1) return false;
    if (g.py) j = wrap_axis(j, g.ny);
    else if (j < -PAD || j > g.ny + PAD - 1) return false;
    return true;
}

__device__ __forceinline__ long long pidx(const GridP& g, int i, int j)
{
    return (long long)(j + PAD) * g.pp + (i + PAD);
}

// Capacity of one layer sub-list: the distance transform runs DT_BLOCKS
// blocks of 256 threads over a window of at most pplane nodes, and sub-list
// s takes the nodes of blocks b = s mod NSUB, at most pplane / NSUB + one
// grid pass.
__host__ __device__ __forceinline__ long long sub_cap(long long pplane)
{
    return pplane / NSUB + (long long)DT_BLOCKS * 256 / NSUB;
}

// Tighter capacity for a grid of nx x ny interior nodes when the block count
// of every distance transform is a multiple of NSUB: sub-list s then takes
// the tiles t = s mod NSUB of the window, whose DTX x DTY tiles cover at most
// (nx + 4 + DTX - 1) (ny + 4 + DTY - 1) nodes, plus one tile.
__host__ __device__ __forceinline__ long long sub_cap_tiles(int nx, int ny)
{
    const long long cover = (long long)(nx + 4 + 31) * (ny + 4 + 15);
    return cover / NSUB + 32 * 16;
}

// Force-plane validity by block stamps (several solids): same interface as
// Rect.
struct StampValid {
    const int* stamp;
    int val, nbx;
    __device__ __forceinline__ bool has(int i, int j) const
    {
        return stamp[(j >> FB_LOG) * nbx + (i >> FB_LOG)] == val;
    }
};

// One solid of a several-solid context (device table, one entry per solid).
struct MbBody {
    GridP g;              // the solid's window
    BodyP b;
    void *X[2], *Y[2], *phi[2];
    Win* win;
    int* boxpart;
    int4 reg;             // force region of the current step, lattice nodes
                          // [x, x + dx] x [y, y + dy] (x, y wrapped), dx < 0: none:
                          // the nodes with phi < eps and their neighbours
};


// ---- adjoint (k_adjoint.hip; FP64, one solid)

// One forward step n as the adjoint reads it (a snapshot taken right after
// the step): window slot 0 is the ring slot wprev of step n (validity of
// xi^n, phi^n, F^{n-1}), slot 1 the slot wcur (validity of xi^{n+1},
// phi^{n+1}, F^n and the layers).
struct AdjSnap {
    const double* A;             // pull-stored lattice of state n
    const double *fpx, *fpy;     // F^{n-1}
    const double *fcx, *fcy;     // F^n
    const double *X0, *Y0, *P0;  // xi^n, phi^n (padded grid)
    const double *X1, *Y1, *P1;  // xi^{n+1}, phi^{n+1}
    const int8_t* tag;           // solid / layer tags of step n
    const Win* win;              // [0] = wprev, [1] = wcur
    const double* fpo;           // F^{n-1} outside the window (x, y)
};

// Adjoint fields of one reverse step: *1 belong to state n+1 (read), *0 to
// state n (written); fb_in = dL/df^{n+1}, fb_out = dL/df^n (natural
// populations, [9][ny][nx]); Fcbar = dL/dF^n, Fpbar = dL/dF^{n-1}
// ([ny][nx]); acc = {dL/dG, dL/dU_lid}.
struct AdjBufs {
    const double* fb_in;
    double* fb_out;
    double *xbar1, *ybar1, *pbar1;
    double *xbar0, *ybar0, *pbar0;
    double *Fcbar_x, *Fcbar_y;
    double *Fpbar_x, *Fpbar_y;
    double* acc;
};

// loss coefficients of one state: centroid c, mean displacement d, and
// gc = dL/dc / sum lambda, gd = dL/dd / sum lambda
struct LossCoef {
    double c[2], d[2], gc[2], gd[2];
};

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns hipGetLastError().

// lattice Boltzmann (k_lb.hip)
// relabel_only: the force kernel relabels and writes partial boxes only
// (several solids: the forces come from launch_mb_combine); blocks per member
// of the distance transform, one extrapolation layer (0: all layers of a
// member in one block) and the force kernel
hipError_t launch_batch_band(int precision, const BatchTables& t, int nsim, int layers,
                             hipStream_t st, bool relabel_only = false,
                             int dt_blocks = BATCH_DT_BLOCKS, int fit_blocks = BATCH_FIT_BLOCKS,
                             int band_blocks = BATCH_BAND_BLOCKS, bool fused = false);
hipError_t launch_lb_batch(int precision, int variant, const LbArgs* args, const int* tile_sim,
                           int total_tiles, hipStream_t st);
// PART 0 / 2 launches with nbox > 0 also reduce the force pass's partial
// boxes (boxpart) into ring slot wnext of win.  PART 3 updates the tiles
// [frac0, frac1) / 1000 of the grid's tiles (none if that range is empty);
// split 1 (the early launch, frac0 = 0): of those only the tile rows wholly
// below the previous step's window by more than BULK_EARLY_GAP rows, without
// reading this step's window; split 2 (the held launch, frac0 = the early
// launch's frac1): also the tiles of the early range the early launch
// leaves, striding from the first of them.
hipError_t launch_lb(const GridP& g, int precision, int variant, const void* A, void* B,
                     const double* fpx, const double* fpy, const double* fcx, const double* fcy,
                     const double* drho, Win* win, int wprev, int wcur, double fpo_x,
                     double fpo_y, int part, unsigned* health, hipStream_t st,
                     int max_blocks = 0, const int* boxpart = nullptr, int nbox = 0,
                     Win* winw = nullptr, int wnext = 0, int frac0 = 0, int frac1 = 1000,
                     int split = 0);
int lb_variant_count();
void lb_variant_tile(int v, int* tx, int* ty);
// drho0 (several solids): the density excess of every node, instead of the
// single solid's level set
hipError_t launch_init_populations(const GridP& g, int precision, const BodyP& b,
                                   const void* phi0, const Win* win, int wslot,
                                   const double* u0, void* tmp, void* A, hipStream_t st,
                                   const double* drho0 = nullptr);
// sv.stamp != nullptr: the stamps, not the window, tell where F^{n-1} is held
hipError_t launch_gather_macro(const GridP& g, int precision, const void* A, const double* fpx,
                               const double* fpy, const Win* win, int wprev, double fpo_x,
                               double fpo_y, double* rho, double* ux, double* uy, double* f9,
                               hipStream_t st, StampValid sv = StampValid{nullptr, 0, 0});
hipError_t launch_read_force(const GridP& g, const double* fpx, const double* fpy, const Win* win,
                             int wprev, double fpo_x, double fpo_y, double* fx, double* fy,
                             hipStream_t st, StampValid sv = StampValid{nullptr, 0, 0});
// lattice update of a several-solid context: every tile, force planes where
// the stamps say so
// (the stamp values are *dstep for vp and *dstep + 1 for vc)
hipError_t launch_lb_mb(const GridP& g, int precision, int variant, const void* A, void* B,
                        const double* fpx, const double* fpy, const double* fcx,
                        const double* fcy, const double* drho, StampValid vp, StampValid vc,
                        double fpo_x, double fpo_y, unsigned* health, hipStream_t st,
                        const long long* dstep);
hipError_t launch_poke(const GridP& g, int precision, void* A, long long node, double value,
                       hipStream_t st);

// reference map (k_band.hip)
hipError_t launch_win_reset(Win* win, int slot, hipStream_t st);
hipError_t launch_init_solid_box(const GridP& g, const BodyP& b, const BandBufs& bb, int slot0,
                                 int slot1, hipStream_t st);
hipError_t launch_init_tags(const GridP& g, const BodyP& b, const BandBufs& bb, int wslot,
                            hipStream_t st);
hipError_t launch_layers(const GridP& g, const BandBufs& bb, int wslot, hipStream_t st);
// fused_threads 256 / 512 / 1024: all layers in one k_fit_fused launch of
// that block size (walled axes, at most FF_LAYERS layers; else, and for 0,
// one launch per layer); 1: 1024 threads with the fits' reach narrowed by one
// node, so that the one-block pass over stopped tiles takes most of them
hipError_t launch_extrapolate(const GridP& g, const BandBufs& bb, const StepSlots& s,
                              hipStream_t st, int fused_threads);
inline bool fused_fit_ok(const GridP& g) { return !g.px && !g.py && g.layers <= FF_LAYERS; }
__host__ __device__ inline long long fused_tiles(int nx, int ny)
{
    return (long long)((nx + 2 * PAD + FF_TILE - 1) / FF_TILE) *
           ((ny + 2 * PAD + FF_TILE - 1) / FF_TILE);
}
hipError_t launch_init_fill(const GridP& g, const BodyP& b, const BandBufs& bb, int wslot,
                            hipStream_t st);
hipError_t launch_advect_layers(const GridP& g, int precision, const BandBufs& bb,
                                const StepSlots& s, const void* A, const double* fpx,
                                const double* fpy, hipStream_t st, bool fused);
// The lattice Boltzmann update fused into the force pass: for each node of
// the window (interior) the pull update from lattice A into B with this
// step's force, F^{n-1} from (fpx, fpy) inside window slot wprev (else the
// uniform force fpo).
struct LbFuse {
    const void* A;
    void* B;
    const double *fpx, *fpy;
    int wprev;
    double fpo_x, fpo_y;
};
// lf null: relabel and force only (the lattice update of the window follows
// in a lattice kernel).  Either way the new solid box is left as partial
// boxes in bb.boxpart (RELABEL_BLOCKS of them).
hipError_t launch_force(const GridP& g, const BodyP& b, const BandBufs& bb, const StepSlots& s,
                        double* fx, double* fy, double* drho, hipStream_t st,
                        const LbFuse* lf = nullptr);
// the force pass's partial boxes into ring slot wnext, with the zone check
hipError_t launch_reduce_window(const GridP& g, const BandBufs& bb, int wcur, int wnext,
                                hipStream_t st);
hipError_t launch_read_stress(const GridP& g, const BodyP& b, const BandBufs& bb, int buf,
                              int wvalid, double* sxx, double* sxy, double* syy, hipStream_t st);
hipError_t launch_read_refmap(const GridP& g, const BodyP& b, const BandBufs& bb, int buf, int wvalid, double* X,
                              double* Y, double* phi, hipStream_t st);

// several solids (k_band.hip).  mark: per solid, reduce the relabel's partial
// boxes into ring slot wnext, flag a window that comes too close to its
// border, and stamp (value sval) the force blocks of its region of slot wcur,
// listing each newly stamped block once (list / count).
// dstep != nullptr: the stamp value is *dstep + 1 (the device step counter,
// so that replayed graphs stamp with the running step)
hipError_t launch_mb_mark(const GridP& lg, MbBody* bodies, int nb, int wcur, int wnext,
                          int nbox, int* stamp, int sval, int* list, int* count, int nbx,
                          unsigned* health, hipStream_t st, const long long* dstep = nullptr);
// advances the device step counter
hipError_t launch_mb_tick(long long* dstep, hipStream_t st);
// combine: over the listed blocks, the global stress of every half-edge
// (blend of the solids normalised by their summed fraction, plus contact),
// its divergence, buoyancy and the fluid force into fx, fy; the density
// excess into drho.  Zeroes *count_clear (the next step's list counter).
// drho_only: the density excess only (initialisation).
hipError_t launch_mb_combine(const GridP& lg, int precision, const MbBody* bodies, int nb,
                             int buf, int wcur, const int* list, const int* count,
                             int* count_clear, int nbx, double* fx, double* fy, double* drho,
                             bool drho_only, unsigned* health, hipStream_t st);
// node averages of the global half-edge solid stresses of the state whose
// maps are in buffer buf over window slot wslot, into [ny][nx] planes
hipError_t launch_mb_read_stress(const GridP& lg, int precision, const MbBody* bodies, int nb,
                                 int buf, int wslot, int nbx, int nby, double* sxx, double* sxy,
                                 double* syy, unsigned* health, hipStream_t st);
// the chain's per-phase argument tables of a several-solid context (each
// entry holds a copy of its solid's window geometry)
struct MbTabs {
    AdvectArgs* adv[7];
    LayersArgs* lay[7];
    FitArgs* fit[7];
    EdgesArgs* edg[7];
};
// the region boxes and window origins of the solid table dst (and of the
// argument tables) from a saved copy src (device)
hipError_t launch_mb_copy_reg(const MbBody* src, MbBody* dst, int nb, const MbTabs& tabs,
                              hipStream_t st);
// moves the sub-window of every solid whose zone (its boxes in ring slots wa
// and wb, dilated by the layers) comes within MB_RECENTRE_MARGIN nodes of the
// window's border, so that the boxes are centred: the maps of buffer buf
// move within the window (through the other buffer, free between steps),
// the ring boxes shift, and the origin changes in the solid table and the
// argument tables; every node keeps its lattice position and value
hipError_t launch_mb_recentre(int precision, MbBody* bodies, int nb, const MbTabs& tabs, int buf,
                              int wa, int wb, hipStream_t st);
hipError_t launch_mb_read_refmap(const GridP& lg, int precision, const MbBody* bodies, int k,
                                 int buf, int wvalid, double* X, double* Y, double* phi,
                                 hipStream_t st);
// per solid: [sum lambda, sum lambda x, sum lambda y, sum lambda (x - X),
// sum lambda (y - Y), solid nodes, nodes with a map] into out + 7 k
hipError_t launch_mb_diag(int precision, const MbBody* bodies, int nb, int buf, int wvalid,
                          double* out, hipStream_t st);

// adjoint (k_adjoint.hip): one reverse step (lattice, force, relabel, the
// layers from last to first, advection); the loss of one state (which = 0:
// the step's input state, 1: its output); the initial velocity
hipError_t launch_adjoint_step(const GridP& g, const BodyP& b, const AdjSnap& s,
                               const AdjBufs& a, hipStream_t st);
hipError_t launch_adjoint_loss(const GridP& g, const BodyP& b, const AdjSnap& s,
                               const AdjBufs& a, int which, const LossCoef& c, hipStream_t st);
hipError_t launch_adjoint_init(const GridP& g, const BodyP& b, const AdjSnap& s,
                               const AdjBufs& a, double* u0bar, hipStream_t st);
// dst[0] = x, dst[1] = y (device, stream-ordered)
hipError_t launch_set2(double* dst, double x, double y, hipStream_t st);

// reductions (k_diag.hip); partial: scratch of diag_partial_doubles() doubles
int diag_blocks();
size_t diag_partial_doubles();
hipError_t launch_diag(const GridP& g, int precision, const BodyP& b, const void* A,
                       const double* fpx, const double* fpy, const Win* win, int wprev,
                       double fpo_x, double fpo_y, const BandBufs& bb, int buf, double* partial,
                       double* out, hipStream_t st, StampValid sv = StampValid{nullptr, 0, 0});

}  // namespace lbrmt
