// Reference-map ("band") kernels of the LBRMT step on gfx950: advection of xi
// (Sec. 3.1), the extrapolation zone and its layer-by-layer least-squares
// extrapolation (Sec. 3.2), relabel phi = phi0(xi), and the divergence of the
// blended half-edge solid stress fed back as the LB force density (Sec. 3.3,
// Eq. (2_4_F_divs)).
//
// Every kernel works inside one rectangular window per body: the box of the
// interior solid nodes dilated by the number of extrapolation layers, kept in
// a device ring of three boxes (previous, current, next step) so no host round
// trip is needed.  A node outside a window holds no reference map.
//
// One step runs: advect (tags: solid / none) -> two-pass Manhattan distance
// transform (exact layer numbers and one node list per layer) -> one fit
// kernel per layer -> relabel (per-block boxes) -> force (LDS-tiled half
// edges; reduces the boxes).
//
// These kernels take every discrete decision of the method (solid set, layers,
// window growth of the fit, singular Jacobians); this file is compiled without
// floating-point contraction so they are taken in plain IEEE arithmetic.
//
// Storage type T of the reference map: double (FP64 mode) holds xi itself;
// float (FP32 mode) holds the displacement d = xi - x, x the node coordinate,
// so values stay small and stencils add the exact lattice offsets (the upwind
// and central differences of x itself are exactly 1).  The FP32 mode runs the
// stencil arithmetic in float and keeps FP64 for the level set phi0(x + d)
// (it decides the solid set), the normal matrix of the fit and its
// well-posedness test (exact sums of powers of two on a few nodes), and the
// inversion of grad xi where det < kappa_J.
#include "lb_node.h"

namespace lbrmt {

constexpr double PI_D = 3.14159265358979323846;

template <typename C>
__device__ __forceinline__ C heaviside(C phi, C eps)
{
    // Eq. (2_3_heaviside)
    const C pi = C(PI_D);
    if (phi <= -eps) return C(0);
    if (phi >= eps) return C(1);
    return C(0.5) * (C(1) + phi / eps + sin(pi * phi / eps) / pi);
}

// reference shape level set phi0(X) (Sec. 3.1): the disc's signed distance
// |X - c| - R; for an ellipse the radial form |X - c| (1 - 1/q), with q the
// normalised radius sqrt((x'/R)^2 + (y'/Rb)^2) in the body frame, zero on the
// boundary and negative inside (at the centre: minus the smaller semi-axis).
// Built without contraction: the sign taken at initialisation and relabel
// decides node sets, so the arithmetic is the plain sequence of rounded ops.
__device__ __forceinline__ double shape_phi(const BodyP& b, double X, double Y)
{
    const double dx = X - b.cx, dy = Y - b.cy;
    const double d = sqrt(dx * dx + dy * dy);
    if (b.shape != 1) return d - b.R;
    if (d == 0.0) return -(b.R < b.Rb ? b.R : b.Rb);
    const double xp = b.ct * dx + b.st * dy, yp = -b.st * dx + b.ct * dy;
    const double q = sqrt((xp / b.R) * (xp / b.R) + (yp / b.Rb) * (yp / b.Rb));
    return d * (1.0 - 1.0 / q);
}

// coordinate of node index i on an axis; on a periodic axis the image nearest
// to the body centre keeps the reference map continuous
__device__ __forceinline__ double node_coord(int i, int periodic, int n, double c)
{
    double x = i + 0.5;
    if (periodic) {
        const double L = n;
        double d = x - c;
        d -= L * floor(d / L + 0.5);
        x = c + d;
    }
    return x;
}

// position of reference-map node (i, j) of grid g, seen by body b (a solid's
// sub-window starts at lattice column ox; its positions are unwrapped)
__device__ __forceinline__ double pos_x(const GridP& g, const BodyP& b, int i)
{
    return node_coord(i + g.ox, g.px, g.nx, b.cx);
}
__device__ __forceinline__ double pos_y(const GridP& g, const BodyP& b, int j)
{
    return node_coord(j + g.oy, g.py, g.ny, b.cy);
}

// lattice column / row of reference-map node i / j
__device__ __forceinline__ int lat_col(const GridP& g, int i)
{
    return g.wx ? wrap_axis(i + g.ox, g.lnx) : i;
}
__device__ __forceinline__ int lat_row(const GridP& g, int j)
{
    return g.wy ? wrap_axis(j + g.oy, g.lny) : j;
}

// a level-set value computed in double, stored as T with its sign kept (a
// negative value too small for float is stored as the smallest negative float)
template <typename T>
__device__ __forceinline__ T store_phi(double p)
{
    T v = T(p);
    if (p < 0.0 && !(v < T(0))) v = -T(1.401298464324817e-45);
    return v;
}

// clears the layer counters of a step (block 0 of the kernel before the
// distance transform)
__device__ __forceinline__ void clear_lcount(int* lcount)
{
    if (blockIdx.x == 0 && threadIdx.x < (MAX_LAYERS + 1) * NSUB)
        lcount[threadIdx.x * LCOUNT_PAD] = 0;
}

// tags: TAG_NONE, TAG_SOLID, layer l (1..layers), or layer | TAG_FAIL
__device__ __forceinline__ bool tag_valid_before(int t, int l)
{
    // solid, or set by an earlier layer
    return t == TAG_SOLID || (t > 0 && t < l);
}

__device__ __forceinline__ bool tag_set(int t)
{
    return t == TAG_SOLID || (t > 0 && t < TAG_FAIL);
}

// ---------------------------------------------------------------- block helpers

// box of the block's flagged nodes, stored as one partial per block
__device__ void block_box(int i0, int i1, int j0, int j1, int* out4)
{
    __shared__ int sb[4][16];
    i0 = wave_min(i0);
    i1 = wave_max(i1);
    j0 = wave_min(j0);
    j1 = wave_max(j1);
    const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int nw = (blockDim.x + 63) / 64;
    if (lane == 0) {
        sb[0][wid] = i0;
        sb[1][wid] = i1;
        sb[2][wid] = j0;
        sb[3][wid] = j1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; w++) {
            i0 = min(i0, sb[0][w]);
            i1 = max(i1, sb[1][w]);
            j0 = min(j0, sb[2][w]);
            j1 = max(j1, sb[3][w]);
        }
        out4[0] = i0;
        out4[1] = i1;
        out4[2] = j0;
        out4[3] = j1;
    }
    __syncthreads();
}

// reduce n partial boxes into one window slot (called by a whole block)

// true in exactly one block: the last to arrive (all blocks must call it)
__device__ bool last_block(unsigned* ticket)
{
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// ---------------------------------------------------------------- window ring

__global__ void k_win_reset(Win* win, int slot)
{
    if (threadIdx.x == 0) {
        win[slot].i0 = 0x3fffffff;
        win[slot].i1 = -0x3fffffff;
        win[slot].j0 = 0x3fffffff;
        win[slot].j1 = -0x3fffffff;
    }
}

hipError_t launch_win_reset(Win* win, int slot, hipStream_t st)
{
    k_win_reset<<<1, 64, 0, st>>>(win, slot);
    return hipGetLastError();
}

// ---------------------------------------------------------------- initialisation

__device__ __forceinline__ bool init_solid(const GridP& g, const BodyP& b, int i, int j)
{
    if (i < 0 || i >= g.nx || j < 0 || j >= g.ny) return false;
    const double x = pos_x(g, b, i);
    const double y = pos_y(g, b, j);
    return shape_phi(b, x, y) < 0.0;
}

// box of the initial solid set {interior nodes: phi0(x) < 0}
__global__ __launch_bounds__(256) void k_init_solid_box(GridP g, BodyP b, int* boxpart,
                                                        unsigned* ticket, Win* win, int s0, int s1)
{
    const long long N = (long long)g.nx * g.ny;
    int i0 = 0x3fffffff, i1 = -0x3fffffff, j0 = 0x3fffffff, j1 = -0x3fffffff;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N; e += stride) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        if (init_solid(g, b, i, j)) {
            i0 = min(i0, i);
            i1 = max(i1, i);
            j0 = min(j0, j);
            j1 = max(j1, j);
        }
    }
    block_box(i0, i1, j0, j1, boxpart + 4 * blockIdx.x);
    if (last_block(ticket)) {
        reduce_boxes<true>(boxpart, gridDim.x, &win[s0], &win[s1]);
        if (threadIdx.x == 0) *ticket = 0u;
    }
}

hipError_t launch_init_solid_box(const GridP& g, const BodyP& b, const BandBufs& bb, int slot0,
                                 int slot1, hipStream_t st)
{
    k_init_solid_box<<<BOX_BLOCKS, 256, 0, st>>>(g, b, bb.boxpart, bb.ticket, bb.win, slot0,
                                                 slot1);
    return hipGetLastError();
}

// initial tags over the window (solid / none)
__global__ __launch_bounds__(256) void k_init_tags(GridP g, BodyP b, int8_t* tag, const Win* win,
                                                   int wslot, int* lcount)
{
    clear_lcount(lcount);
    const Rect W = window_of(win, wslot, g);
    if (!W.ok) return;
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    const long long total = (long long)w * h;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
        tag[pidx(g, i, j)] = init_solid(g, b, i, j) ? TAG_SOLID : TAG_NONE;
    }
}

hipError_t launch_init_tags(const GridP& g, const BodyP& b, const BandBufs& bb, int wslot,
                            hipStream_t st)
{
    k_init_tags<<<2048, 256, 0, st>>>(g, b, bb.tag, bb.win, wslot, bb.lcount);
    return hipGetLastError();
}

// xi_0 = x on the solid and its extrapolation zone, phi = phi0(x) (Alg. 1 init)
template <typename T>
__global__ void k_init_fill(GridP g, BodyP b, const int8_t* tag, const Win* win, int wslot,
                            T* X, T* Y, T* phi, int* lcount)
{
    constexpr bool DISP = sizeof(T) == 4;
    clear_lcount(lcount);  // for the first step's distance transform
    const Rect W = window_of(win, wslot, g);
    if (!W.ok) return;
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)w * h;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
        const long long k = pidx(g, i, j);
        if (tag[k] != TAG_NONE) {
            const double x = pos_x(g, b, i);
            const double y = pos_y(g, b, j);
            X[k] = DISP ? T(0) : T(x);
            Y[k] = DISP ? T(0) : T(y);
            phi[k] = store_phi<T>(shape_phi(b, x, y));
        } else {
            X[k] = T(NAN);
            Y[k] = T(NAN);
            phi[k] = T(INFINITY);
        }
    }
}

hipError_t launch_init_fill(const GridP& g, const BodyP& b, const BandBufs& bb, int wslot,
                            hipStream_t st)
{
    if (g.rm32)
        k_init_fill<float><<<2048, 256, 0, st>>>(g, b, bb.tag, bb.win, wslot, (float*)bb.X[0],
                                                 (float*)bb.Y[0], (float*)bb.phi[0], bb.lcount);
    else
        k_init_fill<double><<<2048, 256, 0, st>>>(g, b, bb.tag, bb.win, wslot, (double*)bb.X[0],
                                                  (double*)bb.Y[0], (double*)bb.phi[0],
                                                  bb.lcount);
    return hipGetLastError();
}

// ---------------------------------------------------------------- advection

// reference-map node (i, j) of step n: canonical index, or -1 if it holds no
// value (outside the domain or outside the window D where xi^n was written)
__device__ __forceinline__ long long ref_index(const GridP& g, const Rect& D, int i, int j)
{
    if (!canon(g, i, j) || !D.has(i, j)) return -1;
    return pidx(g, i, j);
}

// one-sided second-order upwind derivative of Eq. (3_1_eno) from preloaded
// stencil values (m1, m2: one and two nodes behind; p1, p2: ahead).  For
// displacement storage the derivative of the node coordinate itself, exactly
// 1 along the axis, is added by the caller.
template <typename C>
__device__ __forceinline__ bool upwind_d(C vel, C X0, C Y0, bool okm1, bool okm2, C Xm1, C Ym1,
                                         C Xm2, C Ym2, bool okp1, bool okp2, C Xp1, C Yp1, C Xp2,
                                         C Yp2, C& dX, C& dY)
{
    dX = dY = C(0);
    if (vel == C(0)) return true;
    if (vel > C(0)) {
        if (!okm1 || !okm2) return false;
        dX = (C(3) * X0 - C(4) * Xm1 + Xm2) / C(2);
        dY = (C(3) * Y0 - C(4) * Ym1 + Ym2) / C(2);
    } else {
        if (!okp1 || !okp2) return false;
        dX = (C(-3) * X0 + C(4) * Xp1 - Xp2) / C(2);
        dY = (C(-3) * Y0 + C(4) * Yp1 - Yp2) / C(2);
    }
    return true;
}

// Eq. (3_1_refmap_adv) at one solid node (i, j) of S^n = {interior,
// phi^n < 0}.  Every load (the eight upwind stencil nodes with their level
// sets, the nine populations and the previous force) is issued before any is
// used; addresses of absent nodes are clamped to the node itself.  S is both
// the population and the reference-map storage type (FP64: xi; FP32:
// population deviations and displacement).  LATCHK: every lattice node the
// pull gather reads must lie in D (with the chain beside the bulk update,
// the nodes of D are the ones the previous step's force pass updated); a
// solid node on D's rim is counted as an advection miss and keeps its value.
template <typename S, bool LATCHK = false>
__device__ __forceinline__ void advect_node(const GridP& g, const S* __restrict__ A,
                                            const double* __restrict__ fpx,
                                            const double* __restrict__ fpy,
                                            const S* __restrict__ X, const S* __restrict__ Y,
                                            const S* __restrict__ phi, S* X1, S* Y1,
                                            const Rect& D, int i, int j, unsigned* health)
{
    using C = S;
    constexpr bool DISP = sizeof(S) == 4;
    const long long P = g.plane;
    const long long k = pidx(g, i, j);
    // stencil nodes: x-1, x-2, x+1, x+2, y-1, y-2, y+1, y+2
    const int di[8] = {-1, -2, 1, 2, 0, 0, 0, 0};
    const int dj[8] = {0, 0, 0, 0, -1, -2, 1, 2};
    long long ks[8];
#pragma unroll
    for (int q = 0; q < 8; q++) ks[q] = ref_index(g, D, i + di[q], j + dj[q]);
    // populations of the pull gather (the node is interior), at the node's
    // lattice position (a solid's window may be a sub-range of the lattice)
    const int li = lat_col(g, i), lj = lat_row(g, j);
    const bool bw = !g.lpx && li == 0, be = !g.lpx && li == g.lnx - 1;
    const bool bs = !g.lpy && lj == 0, bn = !g.lpy && lj == g.lny - 1;
    int im = li - 1, ip = li + 1, jm = lj - 1, jp = lj + 1;
    im = im < 0 ? (g.lpx ? g.lnx - 1 : 0) : im;
    ip = ip >= g.lnx ? (g.lpx ? 0 : g.lnx - 1) : ip;
    jm = jm < 0 ? (g.lpy ? g.lny - 1 : 0) : jm;
    jp = jp >= g.lny ? (g.lpy ? 0 : g.lny - 1) : jp;
    bool lat_ok = true;
    if (LATCHK) {
        // D is a rectangle holding (i, j): the four axis neighbours decide
        int iw = i - 1, ie = i + 1, js = j - 1, jn = j + 1;
        if (g.px) {
            iw = wrap_axis(iw, g.nx);
            ie = wrap_axis(ie, g.nx);
        }
        if (g.py) {
            js = wrap_axis(js, g.ny);
            jn = wrap_axis(jn, g.ny);
        }
        lat_ok = (bw || D.has(iw, j)) && (be || D.has(ie, j)) && (bs || D.has(i, js)) &&
                 (bn || D.has(i, jn));
        if (!lat_ok) {
            im = ip = li;
            jm = jp = lj;
        }
    }
    const long long r0 = (long long)lj * g.pitch, rm = (long long)jm * g.pitch,
                    rp = (long long)jp * g.pitch, n = r0 + li;
    // ---- all loads
    const C X0 = X[k], Y0 = Y[k];
    C ps[8], xs[8], ys[8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const long long kq = ks[q] >= 0 ? ks[q] : k;
        ps[q] = phi[kq];
        xs[q] = X[kq];
        ys[q] = Y[kq];
    }
    C f[NQ];
    f[0] = A[n];
    f[1] = bw ? A[3 * P + n] : A[1 * P + r0 + im];
    f[2] = bs ? A[4 * P + n] : A[2 * P + rm + li];
    f[3] = be ? A[1 * P + n] : A[3 * P + r0 + ip];
    f[4] = bn ? A[2 * P + n] : A[4 * P + rp + li];
    f[5] = (bw || bs) ? A[7 * P + n] : A[5 * P + rm + im];
    f[6] = (be || bs) ? A[8 * P + n] : A[6 * P + rm + ip];
    f[7] = (be || bn) ? A[5 * P + n] : A[7 * P + rp + ip];
    f[8] = (bw || bn) ? A[6 * P + n] : A[8 * P + rp + im];
    const C Fx = C(fpx[n]), Fy = C(fpy[n]);
    // ---- arithmetic: half-force velocity of Eq. (2_2_lbm_moments_force); the
    // FP32 mode stores f_i - w_i rho_f (sum w_i = 1, sum w_i c_i = 0)
    const C s9 = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const C rho = DISP ? C(g.rho_f) + s9 : s9;
    const C u = (f[1] + f[5] + f[8] - f[3] - f[6] - f[7]) / rho + Fx / (C(2) * rho);
    const C v = (f[2] + f[5] + f[6] - f[4] - f[7] - f[8]) / rho + Fy / (C(2) * rho);
    bool okq[8];
#pragma unroll
    for (int q = 0; q < 8; q++) okq[q] = ks[q] >= 0 && ps[q] < C(INFINITY);
    C dXx, dYx, dXy, dYy;
    const bool okx = upwind_d<C>(u, X0, Y0, okq[0], okq[1], xs[0], ys[0], xs[1], ys[1], okq[2],
                                 okq[3], xs[2], ys[2], xs[3], ys[3], dXx, dYx);
    const bool oky = upwind_d<C>(v, X0, Y0, okq[4], okq[5], xs[4], ys[4], xs[5], ys[5], okq[6],
                                 okq[7], xs[6], ys[6], xs[7], ys[7], dXy, dYy);
    if (!okx || !oky || !lat_ok) {
        atomicAdd(&health[0], 1u);
        X1[k] = X0;
        Y1[k] = Y0;
    } else if (DISP) {
        // xi = x + d: d(X)/dx = 1 + dXx, d(Y)/dy = 1 + dYy
        X1[k] = X0 - (u * (C(1) + dXx) + v * dXy);
        Y1[k] = Y0 - (u * dYx + v * (C(1) + dYy));
    } else {
        X1[k] = X0 - (u * dXx + v * dXy);
        Y1[k] = Y0 - (u * dYx + v * dYy);
    }
}


// ---------------------------------------------------------------- layers

// Layers of Sec. 3.2: layer 1 = non-solid nodes 4-adjacent to the solid,
// layer l = unmarked nodes 4-adjacent to layer l-1.  Inside a rectangle this
// is the Manhattan distance to the solid set, computed here exactly in two
// separable passes: per column, the distance to the nearest solid node of the
// column (capped at layers + 1); per row, min over |e| of |e| + that distance.
// One block takes a DTX x DTY tile of the window at a time: it stages the
// solid flags of the tile plus a halo of `layers` nodes in LDS, runs both
// passes there, writes the layer numbers and lists the zone nodes of each
// layer (split into NSUB sub-lists by block so that few blocks share a
// counter; the order inside a list does not matter since targets of one layer
// are independent).  The layer counters were cleared by the kernel before.
constexpr int DTX = 32, DTY = 16;
static_assert(DTX == FF_TILE && FF_TILE % DTY == 0, "a distance-transform tile lies in one fused-fit tile");
constexpr int DRW = DTX + 2 * MAX_LAYERS, DRH = DTY + 2 * MAX_LAYERS;

// LC > 0: the layer count as a compile-time constant (scans unrolled);
// LC = 0: the count of the grid.  ADV = false (initialisation): the solid set
// is read from the tags.  ADV = true (a step): the solid set S^n = {interior,
// phi^n < 0, inside the previous window} is read from the level set, the
// tile's solid nodes are tagged and advected (Sec. 3.1) in the same pass, and
// the tags of the window are all written here.
template <int LC, bool ADV, typename S, bool PRE = false, bool LATCHK = false,
          bool SPLIT = false>
__device__ __forceinline__ void dt_tile_body(GridP g, const Win* __restrict__ win, int wslot,
                                             int wprev, int8_t* tag, int* lists, int* lcount,
                                             unsigned* health, const S* __restrict__ A,
                                             const double* __restrict__ fpx,
                                             const double* __restrict__ fpy,
                                             const S* __restrict__ X, const S* __restrict__ Y,
                                             const S* __restrict__ phi, S* X1, S* Y1,
                                             int* ff_flag = nullptr, int* ff_list = nullptr,
                                             int* ff_n = nullptr)
{
    __shared__ int8_t sol[DRH * DRW];   // solid flags of the tile and its halo
    __shared__ int8_t gc[DTY * DRW];    // column distances of the tile rows
    __shared__ int cnt[MAX_LAYERS + 1];
    __shared__ int base[MAX_LAYERS + 1];
    const Rect W = window_of(win, wslot, g);
    if (!W.ok) return;
    const Rect D = window_of(win, wprev, g);
    const int L = LC > 0 ? LC : g.layers;
    const long long cap = g.lcap;
    const int sub = blockIdx.x % NSUB;
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    const int ntx = (w + DTX - 1) / DTX, nty = (h + DTY - 1) / DTY;
    const int rw = DTX + 2 * L, rh = DTY + 2 * L;  // region in use
    const int lane = __lane_id();
    // SPLIT (one solid): when the grid has at least ADV_MIN_WORKERS blocks
    // beyond the tiles, block t < ntile takes tile t without its advection,
    // and the blocks beyond advect the solid nodes of the window, 256 nodes
    // of it (row-major over its interior part) at a time, one per thread:
    // interior tiles no longer advect 512 nodes each while boundary tiles
    // idle.  The solid set is the same (interior, phi^n < 0, inside D), and
    // each node's advection is the same arithmetic, so the bits are too.
    const int ntile = ntx * nty;
    bool adv_here = ADV;
    if (SPLIT && ADV && (int)gridDim.x - ntile >= ADV_MIN_WORKERS) {
        adv_here = false;
        if ((int)blockIdx.x >= ntile) {
            const int i0 = max(W.i0, 0), i1 = min(W.i1, g.nx - 1);
            const int j0 = max(W.j0, 0), j1 = min(W.j1, g.ny - 1);
            if (i0 > i1 || j0 > j1) return;
            const int ww = i1 - i0 + 1;
            const long long nn = (long long)ww * (j1 - j0 + 1);
            const int nwork = gridDim.x - ntile;
            for (long long e = (long long)(blockIdx.x - ntile) * blockDim.x + threadIdx.x; e < nn;
                 e += (long long)nwork * blockDim.x) {
                const int x = i0 + (int)(e % ww), y = j0 + (int)(e / ww);
                if (D.has(x, y) && phi[pidx(g, x, y)] < S(0))
                    advect_node<S, LATCHK>(g, A, fpx, fpy, X, Y, phi, X1, Y1, D, x, y, health);
            }
            return;
        }
    }
    for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
        const int x0 = W.i0 + (t % ntx) * DTX, y0 = W.j0 + (t / ntx) * DTY;
        if (threadIdx.x <= MAX_LAYERS) cnt[threadIdx.x] = 0;
        // solid flags of the region (nodes outside the window hold none).
        // With PRE, FP32 steps with a compile-time layer count issue all of a
        // thread's level-set loads before using any (one solid: advection
        // pass 25.0 -> 23.1 us at 2048^2; with FP64 values the extra
        // registers cost as much, and the several-solid pass at 4096^2 slows
        // from 139 to 154 us)
        constexpr bool PRELOAD = PRE && ADV && LC > 0 && sizeof(S) == 4;
        if (PRELOAD) {
            constexpr int NE = (DTX + 2 * LC) * (DTY + 2 * LC);
            constexpr int NS = (NE + 255) / 256;  // 256 threads per block
            S pv[NS];
            bool inv[NS];
#pragma unroll
            for (int u = 0; u < NS; u++) {
                const int e = threadIdx.x + u * 256;
                const int x = x0 - L + e % rw, y = y0 - L + e / rw;
                inv[u] = e < NE && W.has(x, y) && x >= 0 && x < g.nx && y >= 0 && y < g.ny &&
                         D.has(x, y);
                pv[u] = phi[inv[u] ? pidx(g, x, y) : pidx(g, W.i0, W.j0)];
            }
#pragma unroll
            for (int u = 0; u < NS; u++) {
                const int e = threadIdx.x + u * 256;
                if (e < NE) sol[(e / rw) * DRW + e % rw] = inv[u] && pv[u] < S(0) ? 1 : 0;
            }
        }
        for (int e = threadIdx.x; !PRELOAD && e < rw * rh; e += blockDim.x) {
            const int x = x0 - L + e % rw, y = y0 - L + e / rw;
            bool s = false;
            if (ADV) {
                const bool in = W.has(x, y) && x >= 0 && x < g.nx && y >= 0 && y < g.ny &&
                                D.has(x, y);
                const S p = phi[in ? pidx(g, x, y) : pidx(g, W.i0, W.j0)];
                s = in && p < S(0);
            } else {
                const bool in = W.has(x, y);
                const int8_t tv = tag[in ? pidx(g, x, y) : pidx(g, W.i0, W.j0)];
                s = in && tv == TAG_SOLID;
            }
            sol[(e / rw) * DRW + e % rw] = s ? 1 : 0;
        }
        __syncthreads();
        // column pass over the tile rows, the whole region width
        for (int e = threadIdx.x; e < rw * DTY; e += blockDim.x) {
            const int cx = e % rw, cy = e / rw;
            int best = L + 1;
#pragma unroll
            for (int d = -L; d <= L; d++)
                if (sol[(cy + L + d) * DRW + cx]) best = min(best, abs(d));
            gc[cy * DRW + cx] = (int8_t)best;
        }
        __syncthreads();
        // row pass: DTX x DTY nodes, NPT per thread, row-major in waves; each
        // node's slot in the block's share of its layer list comes from one
        // LDS atomic per wave and layer present
        constexpr int NPT = DTX * DTY / 256;
        int lay[NPT], kk[NPT], slot[NPT];
#pragma unroll
        for (int u = 0; u < NPT; u++) {
            const int e = u * blockDim.x + threadIdx.x;
            const int cx = e % DTX, cy = e / DTX;
            const int x = x0 + cx, y = y0 + cy;
            lay[u] = 0;
            kk[u] = 0;
            slot[u] = 0;
            const bool solid = sol[(cy + L) * DRW + cx + L];
            if (ADV && W.has(x, y) && solid) tag[pidx(g, x, y)] = TAG_SOLID;
            if (W.has(x, y) && !solid) {
                int best = 2 * L + 2;
#pragma unroll
                for (int d = -L; d <= L; d++) best = min(best, abs(d) + gc[cy * DRW + cx + L + d]);
                kk[u] = (int)pidx(g, x, y);
                if (best <= L) lay[u] = best;
                tag[kk[u]] = lay[u] > 0 ? (int8_t)lay[u] : TAG_NONE;
            }
            for (int l = 1; l <= L; l++) {
                const unsigned long long mask = __ballot(lay[u] == l);
                if (mask == 0ull) continue;
                const int leader = __ffsll((long long)mask) - 1;
                int wb = 0;
                if (lane == leader) wb = atomicAdd(&cnt[l], __popcll(mask));
                wb = __shfl(wb, leader);
                if (lay[u] == l) slot[u] = wb + __popcll(mask & ((1ull << lane) - 1ull));
            }
        }
        __syncthreads();
        // one reservation per layer present in the tile
        if (threadIdx.x >= 1 && threadIdx.x <= L && cnt[threadIdx.x] > 0)
            base[threadIdx.x] =
                atomicAdd(&lcount[(threadIdx.x * NSUB + sub) * LCOUNT_PAD], cnt[threadIdx.x]);
        // the fused extrapolation's tile (FF_TILE square, same origin) holding
        // this one is listed once if the zone reaches it
        if (ff_list && threadIdx.x == 0) {
            bool zone = false;
            for (int l = 1; l <= L; l++) zone = zone || cnt[l] > 0;
            if (zone) {
                const int ft = (x0 - W.i0) / FF_TILE +
                               ((y0 - W.j0) / FF_TILE) * ((w + FF_TILE - 1) / FF_TILE);
                if (atomicExch(&ff_flag[ft], 1) == 0) ff_list[atomicAdd(ff_n, 1)] = ft;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NPT; u++) {
            if (lay[u] > 0) {
                const long long at = (long long)base[lay[u]] + slot[u];
                if (at < cap) lists[(lay[u] * NSUB + sub) * cap + at] = kk[u];
                else atomicAdd(&health[7], 1u);  // beyond the sub-list capacity
            }
        }
        if (adv_here) {
            // advection of the tile's solid nodes
            for (int e = threadIdx.x; e < DTX * DTY; e += blockDim.x) {
                const int cx = e % DTX, cy = e / DTX;
                const int x = x0 + cx, y = y0 + cy;
                if (W.has(x, y) && sol[(cy + L) * DRW + cx + L])
                    advect_node<S, LATCHK>(g, A, fpx, fpy, X, Y, phi, X1, Y1, D, x, y, health);
            }
        }
        __syncthreads();
    }
}

// initialisation: layers of the initial solid set (from the tags)
template <int LC>
__global__ __launch_bounds__(256) void k_dt_tile(GridP g, const Win* __restrict__ win, int wslot,
                                                 int8_t* tag, int* lists, int* lcount,
                                                 unsigned* health)
{
    dt_tile_body<LC, false, double>(g, win, wslot, 0, tag, lists, lcount, health, nullptr,
                                    nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

// a step: advection of xi plus the layers of the extrapolation zone
// FP64: five waves per SIMD (96 registers, a few spilled) run the 2048
// blocks in fewer rounds (2048^2 step 0.1626 -> 0.1614 ms); FP32 spills more
// at five and is left as the compiler sizes it
template <int LC, typename S>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 5 : 1, 8))) void k_advect_dt(
    GridP g, const S* __restrict__ A,
                                                   const double* __restrict__ fpx,
                                                   const double* __restrict__ fpy,
                                                   const S* __restrict__ X,
                                                   const S* __restrict__ Y,
                                                   const S* __restrict__ phi, S* X1, S* Y1,
                                                   int8_t* tag, const Win* __restrict__ win,
                                                   int wprev, int wcur, int* lists, int* lcount,
                                                   unsigned* health, int* ff_flag, int* ff_list,
                                                   int* ff_n)
{
    dt_tile_body<LC, true, S, true, true, true>(g, win, wcur, wprev, tag, lists, lcount, health,
                                                A, fpx, fpy, X, Y, phi, X1, Y1, ff_flag, ff_list,
                                                ff_n);
}

// five waves per SIMD: the suspension's 6400 blocks (400 solids) run in
// fewer rounds (FP32 step 0.634 -> 0.619 ms; FP64 0.998 -> 0.994)
template <int LC, typename S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void kb_advect_dt(
    const AdvectArgs* __restrict__ args, const int* __restrict__ ord)
{
    const AdvectArgs& a = args[ord ? ord[blockIdx.y] : blockIdx.y];
    dt_tile_body<LC, true, S>(a.g, a.win, a.wcur, a.wprev, a.tag, a.lists, a.lcount, a.health,
                              (const S*)a.A, a.fpx, a.fpy, (const S*)a.X, (const S*)a.Y,
                              (const S*)a.phi, (S*)a.X1, (S*)a.Y1, a.ff_flag, a.ff_list, a.ff_n);
}

hipError_t launch_advect_layers(const GridP& g, int precision, const BandBufs& bb,
                                const StepSlots& s, const void* A, const double* fpx,
                                const double* fpy, hipStream_t st, bool fused)
{
    int* ffl = fused ? bb.ff_flag : nullptr;
    int* ffs = fused ? bb.ff_list : nullptr;
    int* ffn = fused ? bb.ff_n : nullptr;
#define ADT(LC, S)                                                                                \
    k_advect_dt<LC, S><<<DT_BLOCKS, 256, 0, st>>>(                                              \
        g, (const S*)A, fpx, fpy, (const S*)bb.X[s.cur], (const S*)bb.Y[s.cur],                   \
        (const S*)bb.phi[s.cur], (S*)bb.X[s.nxt], (S*)bb.Y[s.nxt], bb.tag, bb.win, s.wprev,      \
        s.wcur, bb.lists, bb.lcount, bb.health, ffl, ffs, ffn)
    if (precision == 0) {
        if (g.layers == 11) ADT(11, double);
        else ADT(0, double);
    } else {
        if (g.layers == 11) ADT(11, float);
        else ADT(0, float);
    }
#undef ADT
    return hipGetLastError();
}

hipError_t launch_layers(const GridP& g, const BandBufs& bb, int wslot, hipStream_t st)
{
    if (g.layers == 11)
        k_dt_tile<11><<<DT_BLOCKS, 256, 0, st>>>(g, bb.win, wslot, bb.tag, bb.lists, bb.lcount,
                                                 bb.health);
    else
        k_dt_tile<0><<<DT_BLOCKS, 256, 0, st>>>(g, bb.win, wslot, bb.tag, bb.lists, bb.lcount,
                                                bb.health);
    return hipGetLastError();
}

// ---------------------------------------------------------------- extrapolation

__device__ __forceinline__ double det3(double a00, double a01, double a02, double a10,
                                       double a11, double a12, double a20, double a21,
                                       double a22)
{
    return a00 * (a11 * a22 - a12 * a21) - a01 * (a10 * a22 - a12 * a20) +
           a02 * (a10 * a21 - a11 * a20);
}

// Weighted least-squares fit of Sec. 3.2 step (ii) in coordinates centred at
// the target.  The normal matrix and its well-posedness test are kept in
// double (sums of w dx dy with w a power of two, or the normal weight of the
// first two layers); the right-hand sides are accumulated in the storage
// precision C of the reference map.  MT = float is exact where the weights
// are the powers of two alone and r <= FIT_EXACT_R: every term w a b (w =
// 2^-(|a|+|b|) >= 2^-16, |a|, |b| <= 8) is a multiple of 2^-16, and every
// partial sum of them stays below 2^6 in magnitude, so 22 bits hold it: the
// float sums equal the double ones bit for bit, at half the cost.
constexpr int FIT_EXACT_R = 8;
// layers from 3 on weigh by powers of two alone: their sums can run in float
__host__ __device__ __forceinline__ bool float_sums(const GridP& g, int l)
{
    return l >= 3 && g.r_max <= FIT_EXACT_R;
}
template <typename C, typename MT = double>
struct Fit {
    MT M00, M01, M02, M11, M12, M22;
    C bX0, bX1, bX2, bY0, bY1, bY2;
    __device__ __forceinline__ void zero()
    {
        M00 = M01 = M02 = M11 = M12 = M22 = MT(0);
        bX0 = bX1 = bX2 = bY0 = bY1 = bY2 = C(0);
    }
    // one valid node at offset (a, b) from the target, weight of Eq. (3_2_extrap_weight)
    __device__ __forceinline__ void add(int a, int b, bool use_n, double nxh, double nyh, C xv,
                                        C yv)
    {
        double wt = ldexp(1.0, -(abs(a) + abs(b)));
        if (use_n) {
            const double ddx = -(double)a, ddy = -(double)b;  // d = x_target - x_valid
            const double dn = (ddx * nxh + ddy * nyh) / sqrt(ddx * ddx + ddy * ddy);
            wt = dn * wt > 0.0 ? dn * wt : 0.0;
        }
        const MT w = MT(wt), dx = MT(a), dy = MT(b);
        M00 += w * dx * dx;
        M01 += w * dx * dy;
        M02 += w * dx;
        M11 += w * dy * dy;
        M12 += w * dy;
        M22 += w;
        const C wc = C(wt), cx = C(a), cy = C(b);
        bX0 += wc * cx * xv;
        bX1 += wc * cy * xv;
        bX2 += wc * xv;
        bY0 += wc * cx * yv;
        bY1 += wc * cy * yv;
        bY2 += wc * yv;
    }
    // add() for a node that may not be valid (v false: every sum gets a
    // signed zero, which leaves its bits as skipping the node does, since no
    // sum that starts at +0 ever holds -0)
    __device__ __forceinline__ void add_if(bool v, int a, int b, bool use_n, double nxh,
                                           double nyh, C xv, C yv)
    {
        double wt = v ? ldexp(1.0, -(abs(a) + abs(b))) : 0.0;
        if (use_n) {
            const double ddx = -(double)a, ddy = -(double)b;
            // (a valid node is never the target itself, so d2 > 0 for it)
            const double d2 = ddx * ddx + ddy * ddy;
            const double dn = (ddx * nxh + ddy * nyh) / sqrt(d2 > 0.0 ? d2 : 1.0);
            wt = dn * wt > 0.0 ? dn * wt : 0.0;
        }
        const MT w = MT(wt), dx = MT(a), dy = MT(b);
        M00 += w * dx * dx;
        M01 += w * dx * dy;
        M02 += w * dx;
        M11 += w * dy * dy;
        M12 += w * dy;
        M22 += w;
        const C wc = C(wt), cx = C(a), cy = C(b);
        const C xs = v ? xv : C(0), ys = v ? yv : C(0);
        bX0 += wc * cx * xs;
        bX1 += wc * cy * xs;
        bX2 += wc * xs;
        bY0 += wc * cx * ys;
        bY1 += wc * cy * ys;
        bY2 += wc * ys;
    }
    // intercept of the weighted linear fit, if well posed
    __device__ __forceinline__ bool solve(double det_rel, C& x, C& y) const
    {
        const double m00 = M00, m01 = M01, m02 = M02, m11 = M11, m12 = M12, m22 = M22;
        const double det = det3(m00, m01, m02, m01, m11, m12, m02, m12, m22);
        if (!(det > det_rel * m22 * m22 * m22)) return false;
        if (sizeof(C) == 8) {
            x = C(det3(m00, m01, bX0, m01, m11, bX1, m02, m12, bX2) / det);
            y = C(det3(m00, m01, bY0, m01, m11, bY1, m02, m12, bY2) / det);
        } else {
            // Cramer in float: the cofactors of the third column weigh the
            // right-hand sides
            const C c0 = C(m01 * m12 - m11 * m02), c1 = C(m01 * m02 - m00 * m12);
            const C c2 = C(m00 * m11 - m01 * m01), id = C(1.0 / det);
            x = (c0 * bX0 + c1 * bX1 + c2 * bX2) * id;
            y = (c0 * bY0 + c1 * bY1 + c2 * bY2) * id;
        }
        return true;
    }
};

// outward normal of phi^n at a target from its four neighbours (e, w, n, s),
// used by the weights of layers 1 and 2
__device__ __forceinline__ bool normal_from(double pe, double pw, double pn, double ps,
                                            double& nxh, double& nyh)
{
    if (!(pe < INFINITY && pw < INFINITY && pn < INFINITY && ps < INFINITY)) return false;
    const double gx = (pe - pw) / 2.0;
    const double gy = (pn - ps) / 2.0;
    const double gn = sqrt(gx * gx + gy * gy);
    if (!(gn > 0.0)) return false;
    nxh = gx / gn;
    nyh = gy / gn;
    return true;
}

// a lane's partner value by a DPP move within its row (no LDS round trip;
// 64-bit values move as two halves)
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(dpp_move<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    return __hiloint2double(dpp_move<CTRL>(__double2hiint(v)), dpp_move<CTRL>(__double2loint(v)));
}

// sum over the FIT_LANES = 8 lanes of a group (8 aligned lanes, all active
// together): lane i adds lane i ^ 1 (quad_perm 1,0,3,2), then lane i ^ 2
// (quad_perm 2,3,0,1), then the other quad's sum from lane 7 - i (row half
// mirror).  Every lane ends with the same bits, since each addition sees the
// same two operands in either order.
static_assert(FIT_LANES == 8, "group_sum pairs the lanes of an 8-lane group");
template <typename V>
__device__ __forceinline__ V group_sum(V v)
{
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    return v;
}

// Sums of the normal equations over the nodes of the scan window of
// half-width r (side 2r + 1, nodes q = 0 .. side^2 - 1 row by row) that fall
// to this lane: node q goes to lane q mod FIT_LANES; each lane issues the
// loads of PER nodes before adding them.  The offsets (a, b) of node q are
// stepped along instead of divided out.
template <typename T, typename MT>
__device__ __forceinline__ void fit_window(const GridP& g, const Rect& W, int l, int i, int j,
                                           int kt, int r, int sub, bool use_n, double nxh,
                                           double nyh, const int8_t* tag, const T* X1,
                                           const T* Y1, Fit<T, MT>& f, int& count)
{
    constexpr int PER = 4;  // window nodes per lane and pass: 25 of r = 2 in one pass
    const int side = 2 * r + 1, nq = side * side;
    // offsets of this lane's first node
    int a = sub % side - r, b = sub / side - r;
    for (int q0 = sub; q0 < nq; q0 += PER * FIT_LANES) {
        long long kk[PER];
        int tk[PER], aa[PER], bb[PER];
        T xv[PER], yv[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            aa[u] = a;
            bb[u] = b;
            int ci = i + a, cj = j + b;
            kk[u] = (q0 + u * FIT_LANES < nq && canon(g, ci, cj) && W.has(ci, cj))
                        ? pidx(g, ci, cj) : -1;
            // advance by FIT_LANES nodes along the rows
            a += FIT_LANES;
            while (a > r) {
                a -= side;
                b += 1;
            }
        }
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const long long k = kk[u] >= 0 ? kk[u] : kt;
            tk[u] = tag[k];
            xv[u] = X1[k];
            yv[u] = Y1[k];
        }
#pragma unroll
        for (int u = 0; u < PER; u++) {
            if (kk[u] < 0 || !tag_valid_before(tk[u], l)) continue;
            count++;
            f.add(aa[u], bb[u], use_n, nxh, nyh, xv[u], yv[u]);
        }
    }
}

// the group's sums reduced across its lanes, then the intercept, if the
// window held three valid nodes and the fit is well posed
template <typename T, typename MT>
__device__ __forceinline__ bool fit_finish(const GridP& g, Fit<T, MT>& f, int count, T& xo,
                                           T& yo)
{
    count = group_sum(count);
    if (count < 3) return false;
    f.M00 = group_sum(f.M00);
    f.M01 = group_sum(f.M01);
    f.M02 = group_sum(f.M02);
    f.M11 = group_sum(f.M11);
    f.M12 = group_sum(f.M12);
    f.M22 = group_sum(f.M22);
    f.bX0 = group_sum(f.bX0);
    f.bX1 = group_sum(f.bX1);
    f.bX2 = group_sum(f.bX2);
    f.bY0 = group_sum(f.bY0);
    f.bY1 = group_sum(f.bY1);
    f.bY2 = group_sum(f.bY2);
    return f.solve(g.det_rel, xo, yo);
}

// scan window of half-width r = side / 2: reduced normal equations and the
// intercept, if the window holds three valid nodes and the fit is well posed
template <typename T, typename MT>
__device__ __forceinline__ bool fit_at(const GridP& g, const Rect& W, int l, int i, int j, int kt,
                                       int r, int sub, bool use_n, double nxh, double nyh,
                                       const int8_t* tag, const T* X1, const T* Y1, T& xo, T& yo)
{
    int count = 0;
    Fit<T, MT> f;
    f.zero();
    fit_window<T, MT>(g, W, l, i, j, kt, r, sub, use_n, nxh, nyh, tag, X1, Y1, f, count);
    return fit_finish<T, MT>(g, f, count, xo, yo);
}

// fit_window over the block's staged copy of the zone (tags st, values sx,
// sy on a row-major region of rw columns; (li, lj) the target's place in it)
// for the window of half-width 2 (side 5, 25 nodes), the only one the copy is
// searched with: the same nodes in the same lanes and the same order of
// additions as fit_window (lane sub takes nodes sub + 8 u, u = 0 .. 3, below
// 25), every slot added through add_if, so the same bits without a branch
// per node
template <typename T, typename MT>
__device__ __forceinline__ void fit_window_lds_r2(int l, int li, int lj, int sub, bool use_n,
                                                  double nxh, double nyh, const int8_t* st,
                                                  const T* sx, const T* sy, int rw,
                                                  Fit<T, MT>& f, int& count)
{
    constexpr int PER = 4, SIDE = 5, NQ = SIDE * SIDE;
    static_assert(PER * FIT_LANES >= NQ && (PER - 1) * FIT_LANES < NQ,
                  "one pass of PER nodes per lane covers the window");
    const int base = lj * rw + li;
    int tk[PER];
    T xv[PER], yv[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int q = sub + u * FIT_LANES;
        // (a slot past the window reads the target's own place, never used)
        const int k = q < NQ ? base + (q / SIDE - 2) * rw + q % SIDE - 2 : base;
        tk[u] = st[k];
        xv[u] = sx[k];
        yv[u] = sy[k];
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int q = sub + u * FIT_LANES;
        const bool v = q < NQ && tag_valid_before(tk[u], l);
        count += v ? 1 : 0;
        f.add_if(v, q % SIDE - 2, q / SIDE - 2, use_n, nxh, nyh, xv[u], yv[u]);
    }
}

// Fit of one target kt = (i, j) of layer l by the FIT_LANES lanes of a group
// (every lane of the group calls it with the same target): the outward normal
// of phi^n for layers 1 and 2, then scan windows of half-width r = 2 .. r_max
// until one holds three valid nodes and a well-posed fit.  Windows wider than
// rlim are not tried: if the fit needs one, the result is false with cut set.
// outward normal of phi^n at target (i, j) for the weights of layers 1 and 2:
// lanes 0..3 of the group load the four neighbours
template <typename T>
__device__ __forceinline__ bool target_normal(const GridP& g, const Rect& D, int l, int i, int j,
                                              int sub, const T* __restrict__ phin, double& nxh,
                                              double& nyh)
{
    nxh = nyh = 0.0;
    if (l > 2) return false;
    double p = INFINITY;
    if (sub < 4) {
        const int di = sub == 0 ? 1 : sub == 1 ? -1 : 0;
        const int dj = sub == 2 ? 1 : sub == 3 ? -1 : 0;
        const long long kq = ref_index(g, D, i + di, j + dj);
        if (kq >= 0) p = (double)phin[kq];
    }
    const double pe = __shfl(p, 0, FIT_LANES), pw = __shfl(p, 1, FIT_LANES);
    const double pn = __shfl(p, 2, FIT_LANES), ps = __shfl(p, 3, FIT_LANES);
    return normal_from(pe, pw, pn, ps, nxh, nyh);
}

template <typename T, typename MT>
__device__ __forceinline__ bool fit_target(const GridP& g, const Rect& W, const Rect& D, int l,
                                           int kt, int i, int j, int sub, int rlim,
                                           const int8_t* tag, const T* __restrict__ phin,
                                           const T* X1, const T* Y1, T& xo, T& yo, bool& cut)
{
    double nxh, nyh;
    const bool use_n = target_normal<T>(g, D, l, i, j, sub, phin, nxh, nyh);
    cut = false;
    for (int r = 2; r <= g.r_max; r++) {
        if (r > rlim) {
            cut = true;
            return false;
        }
        if (fit_at<T, MT>(g, W, l, i, j, kt, r, sub, use_n, nxh, nyh, tag, X1, Y1, xo, yo))
            return true;
    }
    return false;
}

// fit_target with the scan window read from the block's staged copy of the
// zone ((li, lj): the target's place in it), of half-width 2 only: a target
// whose fit needs a wider window, or whose window of half-width 2 reaches
// beyond the copy (rlim < 2), is not fitted (cut set, unless r_max is 2 and
// the fit has failed for good); k_fit_rest then fits it with the full search,
// which finds the same bits for the window of half-width 2
// (use_n, nxh, nyh: the normal weight of layers 1 and 2, found by the caller
// as target_normal finds it)
template <typename T, typename MT>
__device__ __forceinline__ bool fit_target_lds(const GridP& g, int l, int li, int lj, int sub,
                                               int rlim, const int8_t* st, const T* sx,
                                               const T* sy, int rw, T& xo, T& yo, bool& cut,
                                               bool use_n, double nxh, double nyh)
{
    cut = rlim < 2;
    if (cut) return false;
    int count = 0;
    Fit<T, MT> f;
    f.zero();
    fit_window_lds_r2<T, MT>(l, li, lj, sub, use_n, nxh, nyh, st, sx, sy, rw, f, count);
    if (fit_finish<T, MT>(g, f, count, xo, yo)) return true;
    cut = g.r_max > 2;
    return false;
}

// One layer of Sec. 3.2: every target of the layer list is fitted by a group
// of FIT_LANES lanes that share the scan-window nodes; the sums of the normal
// equations are reduced across the group.  Scan windows grow from r = 2 to
// r_max until they hold three valid nodes and a well-posed fit.  Valid nodes
// come only from earlier layers, so targets of one layer never read each
// other.  With displacement storage the fit of d = xi - x gives the fit of xi
// minus x at the target, since the weighted fit reproduces linear fields.
template <typename T, typename MT>
__device__ __forceinline__ void layer_fit_body(GridP g, const Win* __restrict__ win,
                                                   int wcur, int wprev, int l, int8_t* tag,
                                                   const int* __restrict__ lists,
                                                   const int* __restrict__ lcount,
                                                   const T* __restrict__ phin, T* X1, T* Y1,
                                                   unsigned* health)
{
    // group g takes sub-list g mod NSUB (the sub-lists come from interleaved
    // distance-transform blocks, so they are of similar length); its first
    // list entry is loaded together with the sub-list's count
    const long long cap = g.lcap;
    const int sub = threadIdx.x % FIT_LANES;
    const int grp = (blockIdx.x * blockDim.x + threadIdx.x) / FIT_LANES;
    const int s = grp % NSUB, a0 = grp / NSUB;
    const int astride = gridDim.x * blockDim.x / FIT_LANES / NSUB;
    const int* list = lists + (l * NSUB + s) * cap;
    const int ns = (int)min((long long)lcount[(l * NSUB + s) * LCOUNT_PAD], cap);
    const int kfirst = a0 < cap ? list[a0] : 0;
    const Rect W = window_of(win, wcur, g);
    const Rect D = window_of(win, wprev, g);
    if (a0 >= ns || !W.ok) return;  // whole groups leave together
    // all lanes of a group run the same trip counts, so shuffles see full groups
    for (int at = a0; at < ns; at += astride) {
        const int kt = at == a0 ? kfirst : list[at];
        const int i = kt % g.pp - PAD, j = kt / g.pp - PAD;
        T xo = T(0), yo = T(0);
        bool cut;
        const bool done = fit_target<T, MT>(g, W, D, l, kt, i, j, sub, g.r_max, tag, phin, X1,
                                            Y1, xo, yo, cut);
        if (sub == 0) {
            if (done) {
                X1[kt] = xo;
                Y1[kt] = yo;
            } else {
                tag[kt] = (int8_t)(l | TAG_FAIL);
                atomicAdd(&health[1], 1u);
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_layer_fit(GridP g, const Win* __restrict__ win,
                                                   int wcur, int wprev, int l, int8_t* tag,
                                                   const int* __restrict__ lists,
                                                   const int* __restrict__ lcount,
                                                   const T* __restrict__ phin, T* X1, T* Y1,
                                                   unsigned* health)
{
    if (float_sums(g, l))
        layer_fit_body<T, float>(g, win, wcur, wprev, l, tag, lists, lcount, phin, X1, Y1, health);
    else
        layer_fit_body<T, double>(g, win, wcur, wprev, l, tag, lists, lcount, phin, X1, Y1,
                                  health);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_layer_fit(const FitArgs* __restrict__ args, int l)
{
    const FitArgs& a = args[blockIdx.y];
    if (l > a.g.layers) return;
    if (float_sums(a.g, l))
        layer_fit_body<T, float>(a.g, a.win, a.wcur, a.wprev, l, a.tag, a.lists, a.lcount,
                                 (const T*)a.phin, (T*)a.X1, (T*)a.Y1, a.health);
    else
        layer_fit_body<T, double>(a.g, a.win, a.wcur, a.wprev, l, a.tag, a.lists, a.lcount,
                                  (const T*)a.phin, (T*)a.X1, (T*)a.Y1, a.health);
}

// Every layer of one solid in one block (several solids: a solid's layers
// are short, so one block per solid runs them in order, separated by block
// barriers that make a layer's fitted values visible to the next layer,
// instead of one launch per layer over all solids), on an LDS copy of its
// window dilated by 2 (tags and map values; each fitted value is written to
// the copy as well as to HBM), as the one-launch single-solid kernel does
// for a tile: a scan window of half-width 2 around a target (which lies in
// the window) is read from the copy.  The copy is laid out in unwrapped
// coordinates, each node holding what its periodic image holds, so it is
// kept only while no two of its nodes are images of one node (the copy no
// wider than a period).  A target whose fit needs a wider window takes the
// global path (fit_target, the full search from half-width 2, on the values
// written back so far), and so does every target of a solid whose copy
// would exceed MB_FIT_LDS_NODES nodes or a period.  The same per-target
// arithmetic as layer_fit_body, so the same bits.  Block row y takes table
// row ord[y] (row y when ord is null).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void kb_fit_lds(const FitArgs* __restrict__ args, int layers,
                                                  const int* __restrict__ ord)
{
    __shared__ int8_t st[MB_FIT_LDS_NODES];
    __shared__ T sx[MB_FIT_LDS_NODES], sy[MB_FIT_LDS_NODES];
    __shared__ int s_ns[(MAX_LAYERS + 1) * NSUB];  // sub-list lengths, read once
    // FP32: phi^n of the copy's nodes inside the previous window (+inf
    // elsewhere, as ref_index leaves it), for the normals of layers 1 and 2
    // (in FP64 the copy of phi^n would not fit beside the map values)
    constexpr bool SPHI = sizeof(T) == 4;
    __shared__ T sp[SPHI ? MB_FIT_LDS_NODES : 1];
    constexpr int NG = NT / FIT_LANES;
    const FitArgs& a = args[ord ? ord[blockIdx.y] : blockIdx.y];
    const GridP& g = a.g;
    const Rect W = window_of(a.win, a.wcur, g);
    const Rect D = window_of(a.win, a.wprev, g);
    if (!W.ok) return;
    const int bx0 = W.i0 - 2, by0 = W.j0 - 2;
    const int bw = W.i1 - W.i0 + 5, bh = W.j1 - W.j0 + 5;
    if ((long long)bw * bh > MB_FIT_LDS_NODES || (g.px && bw > g.nx) || (g.py && bh > g.ny)) {
        for (int l = 1; l <= layers; l++) {
            if (float_sums(g, l))
                layer_fit_body<T, float>(g, a.win, a.wcur, a.wprev, l, a.tag, a.lists, a.lcount,
                                         (const T*)a.phin, (T*)a.X1, (T*)a.Y1, a.health);
            else
                layer_fit_body<T, double>(g, a.win, a.wcur, a.wprev, l, a.tag, a.lists,
                                          a.lcount, (const T*)a.phin, (T*)a.X1, (T*)a.Y1,
                                          a.health);
            __syncthreads();
        }
        return;
    }
    T* X1 = (T*)a.X1;
    T* Y1 = (T*)a.Y1;
    const T* phin = (const T*)a.phin;
    const long long cap = g.lcap;
    // the copy: nodes outside the window hold no value (as in fit_window,
    // which wraps a node's periodic axes before the window test); the loads
    // of U nodes per thread are issued before their stores
    constexpr int U = 4;
    const int nn = bw * bh;
    for (int e0 = threadIdx.x; e0 < nn; e0 += U * NT) {
        int8_t tv[U];
        T xv[U], yv[U], pv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int e = e0 + u * NT;
            int x = bx0 + e % bw, y = by0 + e / bw;
            if (g.px) x = wrap_axis(x, g.nx);
            if (g.py) y = wrap_axis(y, g.ny);
            const bool in = e < nn && W.has(x, y);
            const long long k = pidx(g, in ? x : W.i0, in ? y : W.j0);
            tv[u] = in ? a.tag[k] : (int8_t)TAG_NONE;
            xv[u] = in ? X1[k] : T(0);
            yv[u] = in ? Y1[k] : T(0);
            if constexpr (SPHI) {
                const bool ind = e < nn && D.has(x, y);
                pv[u] = ind ? phin[pidx(g, ind ? x : W.i0, ind ? y : W.j0)] : T(INFINITY);
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int e = e0 + u * NT;
            if (e >= nn) break;
            st[e] = tv[u];
            sx[e] = xv[u];
            sy[e] = yv[u];
            if constexpr (SPHI) sp[e] = pv[u];
        }
    }
    for (int q = threadIdx.x; q < (layers + 1) * NSUB; q += NT)
        s_ns[q] = (int)min((long long)a.lcount[q * LCOUNT_PAD], cap);
    __syncthreads();
    // group grp takes sub-list grp mod NSUB, as layer_fit_body does, so the
    // sub-lists of a layer are fitted side by side; the list entry a group
    // fits next is loaded while it fits the current one (the lists are
    // complete before the kernel starts)
    static_assert(NG % NSUB == 0, "whole groups per sub-list");
    constexpr int AS = NG / NSUB;
    const int sub = threadIdx.x % FIT_LANES, grp = threadIdx.x / FIT_LANES;
    const int sl = grp % NSUB, a0 = grp / NSUB;
    int knext = a0 < s_ns[NSUB + sl] ? a.lists[(NSUB + sl) * cap + a0] : 0;
    for (int l = 1; l <= layers; l++) {
        const int* list = a.lists + (l * NSUB + sl) * cap;
        const int ns = s_ns[l * NSUB + sl];
        // every lane of a group runs the same trip counts
        for (int at = a0; at < ns; at += AS) {
            const int kt = knext;
            knext = at + AS < ns ? list[at + AS] : 0;
            const int i = kt % g.pp - PAD, j = kt / g.pp - PAD;
            const int li = i - bx0, lj = j - by0;
            double nxh, nyh;
            bool use_n;
            if constexpr (SPHI) {
                // target_normal with the four neighbours read from the copy
                nxh = nyh = 0.0;
                use_n = false;
                if (l <= 2) {
                    double p = INFINITY;
                    if (sub < 4) {
                        const int di = sub == 0 ? 1 : sub == 1 ? -1 : 0;
                        const int dj = sub == 2 ? 1 : sub == 3 ? -1 : 0;
                        p = (double)sp[(lj + dj) * bw + li + di];
                    }
                    const double pe = __shfl(p, 0, FIT_LANES), pw = __shfl(p, 1, FIT_LANES);
                    const double pn = __shfl(p, 2, FIT_LANES), ps = __shfl(p, 3, FIT_LANES);
                    use_n = normal_from(pe, pw, pn, ps, nxh, nyh);
                }
            } else {
                use_n = target_normal<T>(g, D, l, i, j, sub, phin, nxh, nyh);
            }
            T xo = T(0), yo = T(0);
            bool done, cut;
            int count = 0;
            if (float_sums(g, l)) {
                Fit<T, float> f;
                f.zero();
                fit_window_lds_r2<T, float>(l, li, lj, sub, use_n, nxh, nyh, st, sx, sy, bw,
                                            f, count);
                done = fit_finish<T, float>(g, f, count, xo, yo);
                if (!done && g.r_max > 2)
                    done = fit_target<T, float>(g, W, D, l, kt, i, j, sub, g.r_max, a.tag,
                                                phin, X1, Y1, xo, yo, cut);
            } else {
                Fit<T, double> f;
                f.zero();
                fit_window_lds_r2<T, double>(l, li, lj, sub, use_n, nxh, nyh, st, sx, sy,
                                             bw, f, count);
                done = fit_finish<T, double>(g, f, count, xo, yo);
                if (!done && g.r_max > 2)
                    done = fit_target<T, double>(g, W, D, l, kt, i, j, sub, g.r_max, a.tag,
                                                 phin, X1, Y1, xo, yo, cut);
            }
            if (sub == 0) {
                const int q = lj * bw + li;
                if (done) {
                    sx[q] = xo;
                    sy[q] = yo;
                    X1[kt] = xo;
                    Y1[kt] = yo;
                } else {
                    st[q] = (int8_t)(l | TAG_FAIL);
                    a.tag[kt] = (int8_t)(l | TAG_FAIL);
                    atomicAdd(&a.health[1], 1u);
                }
            }
        }
        if (l < layers) {
            const int n1 = s_ns[(l + 1) * NSUB + sl];
            knext = a0 < n1 ? a.lists[((l + 1) * NSUB + sl) * cap + a0] : 0;
        }
        // the layer's values (copy and global) before the next layer reads them
        __syncthreads();
    }
}

// The tiles k_fit_fused stopped (k_fit_rest, one block): fits, layer by
// layer from the first to the last, every target of the layer lists that
// lies in a stopped tile at or after the layer where that tile stopped (full
// scan windows up to r_max, the per-layer path's fit), then clears that list
// and the list of zone tiles.  With no tile stopped it only clears the lists.
template <typename T, int NT>
__device__ void fit_rest(const GridP& g, const Win* __restrict__ win, int wcur, int wprev,
                         int8_t* tag, const int* __restrict__ lists,
                         const int* __restrict__ lcount, const T* __restrict__ phin, T* X1,
                         T* Y1, unsigned* health, int8_t* cut_layer, const int* cut_tiles,
                         int* ncut, int* ff_flag, const int* ff_list, int* ff_n)
{
    constexpr int NG = NT / FIT_LANES;
    // this thread's first list entry is loaded together with the two counters
    // (the list holds one entry per fused-extrapolation tile of the grid, at
    // least one); the windows are read only when a tile was stopped
    const int a0 = threadIdx.x;
    const int e0 = ff_list[min((long long)a0, fused_tiles(g.nx, g.ny) - 1)];
    const int nt = *ff_n, nc = *ncut;
    const long long cap = g.lcap;
    const int sub = threadIdx.x % FIT_LANES, grp = threadIdx.x / FIT_LANES;
    if (nc > 0) {
        const Rect W = window_of(win, wcur, g);
        const Rect D = window_of(win, wprev, g);
        const int ntx = (W.i1 - W.i0 + FF_TILE) / FF_TILE;
        for (int l = 1; l <= g.layers; l++) {
            for (int s = 0; s < NSUB; s++) {
                const int* list = lists + (l * NSUB + s) * cap;
                const int ns = (int)min((long long)lcount[(l * NSUB + s) * LCOUNT_PAD], cap);
                for (int a = grp; a < ns; a += NG) {
                    const int kt = list[a];
                    const int i = kt % g.pp - PAD, j = kt / g.pp - PAD;
                    const int t = (i - W.i0) / FF_TILE + ((j - W.j0) / FF_TILE) * ntx;
                    if (cut_layer[t] > l) continue;
                    T xo = T(0), yo = T(0);
                    bool cut;
                    const bool done =
                        float_sums(g, l)
                            ? fit_target<T, float>(g, W, D, l, kt, i, j, sub, g.r_max, tag, phin,
                                                   X1, Y1, xo, yo, cut)
                            : fit_target<T, double>(g, W, D, l, kt, i, j, sub, g.r_max, tag,
                                                    phin, X1, Y1, xo, yo, cut);
                    if (sub == 0) {
                        if (done) {
                            X1[kt] = xo;
                            Y1[kt] = yo;
                        } else {
                            tag[kt] = (int8_t)(l | TAG_FAIL);
                            atomicAdd(&health[1], 1u);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    // the lists of the next step start empty
    for (int a = threadIdx.x; a < nt; a += NT) ff_flag[a == a0 ? e0 : ff_list[a]] = 0;
    for (int a = threadIdx.x; a < nc; a += NT) cut_layer[cut_tiles[a]] = FF_NO_CUT;
    __syncthreads();
    if (threadIdx.x == 0) {
        *ncut = 0;
        *ff_n = 0;
    }
}

// All layers of one solid in one launch.  Block b takes FF_TILE x FF_TILE
// tiles of the window from the list the distance transform made of the tiles
// the zone reaches; for layer l it fits every layer-l target within
// M_l = 2 (L - l) nodes of its tile, its own and those of the tiles around
// (recomputed, with the same arithmetic, so the same bits as their own
// blocks find), then a block barrier, then layer l + 1.  The block works on a
// copy in LDS: the tags and the advected solid values of the tile and a
// margin of M_1 + 2 nodes are staged once, and each fitted value (or failure)
// goes into the copy; only the tile's own targets are written back.  The
// level-set normals of the layer-1 and layer-2 targets (the weights of
// Eq. (3_2_extrap_weight)) are found before the layers, all their loads in
// one round; a tile with more such targets than FF_NORMALS is stopped
// before its first layer.  A scan
// window of half-width 2 around a target within M_l of the tile stays within
// M_l + 2 = M_{l-1}, where the copy holds every earlier layer, and layer-1
// windows read solid nodes only, which the copy holds across the margin.  A
// target whose fit needs a wider window than that (fewer than three valid
// nodes in it, or an ill-posed fit) stops the tile at that layer:
// the tile is listed, with the layer, for k_fit_rest, which finishes the
// listed tiles layer by layer; the tile's layers before that one are final.
// reach = 2; reach = 1 stops every tile with a target on the rim of its
// margin at layer 2, and every tile with more than 64 targets in layers 1
// and 2 before its first layer (k_fit_rest then fits most of the zone: a
// check of that launch).  Walled axes only (a window across a periodic seam would
// reach another tile's nodes).
template <typename T, int NT>
__device__ __forceinline__ void fit_fused_body(const GridP& g, const Win* __restrict__ win,
                                               int wcur, int wprev, int8_t* tag,
                                               const T* __restrict__ phin, T* X1, T* Y1,
                                               unsigned* health, int8_t* cut_layer,
                                               int* cut_tiles, int* ncut,
                                               const int* __restrict__ ff_list,
                                               const int* __restrict__ ff_n, int reach)
{
    constexpr int RW = FF_TILE + 4 * (FF_LAYERS - 1) + 4;
    constexpr int NG = NT / FIT_LANES;
    __shared__ int8_t st[RW * RW];  // tags of the tile and its margin
    __shared__ T sx[RW * RW];       // xi (or the displacement): solid nodes, then fitted ones
    __shared__ T sy[RW * RW];
    __shared__ short lst[RW * RW];  // the block's targets, layer by layer (places in the copy)
    __shared__ short cand[RW * RW];  // the same, in staging order
    __shared__ int s_cnt[FF_LAYERS + 1], s_base[FF_LAYERS + 2], s_fill[FF_LAYERS + 1];
    // per layer: a target needed a wider window than the copy holds; targets
    // whose fit failed (own nodes)
    __shared__ int s_cut[FF_LAYERS + 1], s_fail[FF_LAYERS + 1];
    __shared__ int s_n;
    // the level-set normals of the first FF_NORMALS layer-1 and layer-2
    // targets (in list order), found before the layers (flag 1: exists)
    __shared__ double s_nx[FF_NORMALS], s_ny[FF_NORMALS];
    __shared__ int8_t s_nok[FF_NORMALS];
    const int ntile = *ff_n;
    if (blockIdx.x >= ntile) return;
    const Rect W = window_of(win, wcur, g);
    if (!W.ok) return;
    const Rect D = window_of(win, wprev, g);
    const int L = g.layers;
    const int S = 2 * (L - 1) + 2, rw = FF_TILE + 2 * S;  // margin of the copy, its width
    const int ntx = (W.i1 - W.i0 + FF_TILE) / FF_TILE;
    const int sub = threadIdx.x % FIT_LANES, grp = threadIdx.x / FIT_LANES;
    constexpr int NIT = (RW * RW + NT - 1) / NT;  // staged nodes per thread
    // normal slots in use (reach 1, a check of k_fit_rest: few, so that
    // most tiles are stopped before their first layer)
    const int ncap = reach == 1 ? 64 : FF_NORMALS;
    for (int k = blockIdx.x; k < ntile; k += gridDim.x) {
        const int t = ff_list[k];
        const int x0 = W.i0 + (t % ntx) * FF_TILE, y0 = W.j0 + (t / ntx) * FF_TILE;
        __syncthreads();  // the previous tile's shared state is no longer read
        if (threadIdx.x == 0) s_n = 0;
        if (threadIdx.x <= FF_LAYERS) {
            s_cnt[threadIdx.x] = 0;
            s_fill[threadIdx.x] = 0;
            s_cut[threadIdx.x] = 0;
            s_fail[threadIdx.x] = 0;
        }
        __syncthreads();
        // staging in two rounds of loads: every tag of the thread's nodes,
        // then the values of its solid nodes
        int8_t tvs[NIT];
#pragma unroll
        for (int u = 0; u < NIT; u++) {
            const int e = threadIdx.x + u * NT;
            const int x = x0 - S + e % rw, y = y0 - S + e / rw;
            const bool in = e < rw * rw && W.has(x, y);
            const long long kq = pidx(g, in ? x : W.i0, in ? y : W.j0);
            tvs[u] = in ? tag[kq] : (int8_t)TAG_NONE;
        }
        T xs[NIT], ys[NIT];
#pragma unroll
        for (int u = 0; u < NIT; u++) {
            const int e = threadIdx.x + u * NT;
            const int x = x0 - S + e % rw, y = y0 - S + e / rw;
            // the owner of a margin node may have marked it failed already:
            // it is fitted here again, to the same verdict
            if (tvs[u] > 0) tvs[u] = (int8_t)(tvs[u] & (TAG_FAIL - 1));
            const bool solid = e < rw * rw && tvs[u] == TAG_SOLID;
            const long long kq = pidx(g, solid ? x : W.i0, solid ? y : W.j0);
            xs[u] = solid ? X1[kq] : T(0);
            ys[u] = solid ? Y1[kq] : T(0);
        }
#pragma unroll
        for (int u = 0; u < NIT; u++) {
            const int e = threadIdx.x + u * NT;
            if (e >= rw * rw) continue;
            const int x = x0 - S + e % rw, y = y0 - S + e / rw;
            const int tv = tvs[u];
            st[e] = (int8_t)tv;
            if (tv == TAG_SOLID) {
                sx[e] = xs[u];
                sy[e] = ys[u];
            }
            // a layer-l node is this block's target within M_l of the tile
            if (tv >= 1 && tv <= L) {
                const int dx = max(max(x0 - x, x - (x0 + FF_TILE - 1)), 0);
                const int dy = max(max(y0 - y, y - (y0 + FF_TILE - 1)), 0);
                if (max(dx, dy) <= 2 * (L - tv)) {
                    atomicAdd(&s_cnt[tv], 1);
                    cand[atomicAdd(&s_n, 1)] = (short)e;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_base[1] = 0;
            for (int l = 1; l <= L; l++) s_base[l + 1] = s_base[l] + s_cnt[l];
        }
        __syncthreads();
        // the targets sorted by layer (the order within a layer does not
        // matter: a layer's targets do not read each other)
        for (int a = threadIdx.x; a < s_n; a += NT) {
            const int q = cand[a];
            const int l = st[q];
            lst[s_base[l] + atomicAdd(&s_fill[l], 1)] = (short)q;
        }
        __syncthreads();
        // the outward normals of phi^n of the layer-1 and layer-2 targets
        // (weights of Eq. (3_2_extrap_weight)), all loads in one round: the
        // same values and arithmetic as target_normal
        {
            // (none when they do not fit: the tile is stopped below)
            const int n12 = s_base[min(L, 2) + 1] <= ncap ? s_base[min(L, 2) + 1] : 0;
            for (int a = threadIdx.x; a < n12; a += NT) {
                const int q = lst[a];
                const int i = x0 - S + q % rw, j = y0 - S + q / rw;
                const long long ke = ref_index(g, D, i + 1, j), kw = ref_index(g, D, i - 1, j);
                const long long kn = ref_index(g, D, i, j + 1), ks = ref_index(g, D, i, j - 1);
                const long long k0 = pidx(g, i, j);
                const T pe = phin[ke >= 0 ? ke : k0], pw = phin[kw >= 0 ? kw : k0];
                const T pn = phin[kn >= 0 ? kn : k0], ps = phin[ks >= 0 ? ks : k0];
                double nxh = 0.0, nyh = 0.0;
                const bool ok = normal_from(ke >= 0 ? (double)pe : INFINITY,
                                            kw >= 0 ? (double)pw : INFINITY,
                                            kn >= 0 ? (double)pn : INFINITY,
                                            ks >= 0 ? (double)ps : INFINITY, nxh, nyh);
                s_nx[a] = nxh;
                s_ny[a] = nyh;
                s_nok[a] = ok ? 1 : 0;
            }
        }
        __syncthreads();
        // more layer-1 and layer-2 targets than normal slots: the tile is
        // stopped before its first layer (k_fit_rest fits it)
        if (s_base[min(L, 2) + 1] > ncap) {
            if (threadIdx.x == 0) {
                cut_layer[t] = (int8_t)1;
                cut_tiles[atomicAdd(ncut, 1)] = t;
            }
            continue;
        }
        for (int l = 1; l <= L; l++) {
            const int M = 2 * (L - l);
            const int n = s_cnt[l];
            const short* lt = lst + s_base[l];
            // the copy holds layer-(l-1) values within K of the tile (layer
            // 1: solid values across the whole copy); reach < 2 narrows it
            const int K = l == 1 ? S : M + reach;
            for (int a = grp; a < n; a += NG) {
                const int q = lt[a];
                const int li = q % rw, lj = q / rw;
                const int i = x0 - S + li, j = y0 - S + lj;
                const int rlim = min(g.r_max, min(min(li - (S - K), S + FF_TILE - 1 + K - li),
                                                  min(lj - (S - K), S + FF_TILE - 1 + K - lj)));
                // the normal found above (layers 1 and 2)
                const int pos = l <= 2 ? s_base[l] + a : 0;
                const bool use_n = l <= 2 && s_nok[pos] != 0;
                const double nxh = use_n ? s_nx[pos] : 0.0, nyh = use_n ? s_ny[pos] : 0.0;
                T xo = T(0), yo = T(0);
                bool cut;
                const bool done =
                    float_sums(g, l)
                        ? fit_target_lds<T, float>(g, l, li, lj, sub, rlim, st, sx, sy, rw, xo,
                                                   yo, cut, use_n, nxh, nyh)
                        : fit_target_lds<T, double>(g, l, li, lj, sub, rlim, st, sx, sy, rw, xo,
                                                    yo, cut, use_n, nxh, nyh);
                if (sub == 0) {
                    const bool own = i >= x0 && i < x0 + FF_TILE && j >= y0 && j < y0 + FF_TILE;
                    const long long kt = pidx(g, i, j);
                    if (done) {
                        sx[q] = xo;
                        sy[q] = yo;
                        if (own) {
                            X1[kt] = xo;
                            Y1[kt] = yo;
                        }
                    } else if (cut) {
                        s_cut[l] = 1;
                    } else {
                        st[q] = (int8_t)(l | TAG_FAIL);
                        if (own) {
                            tag[kt] = (int8_t)(l | TAG_FAIL);
                            atomicAdd(&s_fail[l], 1);
                        }
                    }
                }
            }
            // one barrier per layer: the decision reads this layer's flags,
            // which the next layer does not write
            __syncthreads();
            const bool stop = s_cut[l] != 0;
            if (threadIdx.x == 0) {
                if (stop) {
                    cut_layer[t] = (int8_t)l;
                    cut_tiles[atomicAdd(ncut, 1)] = t;
                } else if (s_fail[l] > 0) {
                    atomicAdd(&health[1], (unsigned)s_fail[l]);
                }
            }
            if (stop) break;
        }
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_fit_fused(GridP g, const Win* __restrict__ win, int wcur,
                                                  int wprev, int8_t* tag,
                                                  const T* __restrict__ phin, T* X1, T* Y1,
                                                  unsigned* health, int8_t* cut_layer,
                                                  int* cut_tiles, int* ncut,
                                                  const int* __restrict__ ff_list,
                                                  const int* __restrict__ ff_n, int reach)
{
    fit_fused_body<T, NT>(g, win, wcur, wprev, tag, phin, X1, Y1, health, cut_layer, cut_tiles,
                          ncut, ff_list, ff_n, reach);
}

// a batch: member blockIdx.y
template <typename T>
__global__ __launch_bounds__(1024) void kb_fit_fused(const FitArgs* __restrict__ args)
{
    const FitArgs& a = args[blockIdx.y];
    fit_fused_body<T, 1024>(a.g, a.win, a.wcur, a.wprev, a.tag, (const T*)a.phin, (T*)a.X1,
                            (T*)a.Y1, a.health, a.cut_layer, a.cut_tiles, a.ncut, a.ff_list,
                            a.ff_n, 2);
}

template <typename T>
__global__ __launch_bounds__(FF_REST_THREADS) void kb_fit_rest(const FitArgs* __restrict__ args)
{
    const FitArgs& a = args[blockIdx.y];
    fit_rest<T, FF_REST_THREADS>(a.g, a.win, a.wcur, a.wprev, a.tag, a.lists, a.lcount,
                                 (const T*)a.phin,
                                 (T*)a.X1, (T*)a.Y1, a.health, a.cut_layer, a.cut_tiles, a.ncut,
                                 a.ff_flag, a.ff_list, a.ff_n);
}

// fit_rest in a block of FF_REST_THREADS threads, which finds a free slot
// beside the bulk update sooner than one that needs a whole compute unit
template <typename T>
__global__ __launch_bounds__(FF_REST_THREADS) void k_fit_rest(
    GridP g, const Win* __restrict__ win, int wcur, int wprev, int8_t* tag,
    const int* __restrict__ lists, const int* __restrict__ lcount, const T* __restrict__ phin,
    T* X1, T* Y1, unsigned* health, int8_t* cut_layer, const int* cut_tiles, int* ncut,
    int* ff_flag, const int* ff_list, int* ff_n)
{
    fit_rest<T, FF_REST_THREADS>(g, win, wcur, wprev, tag, lists, lcount, phin, X1, Y1, health,
                                 cut_layer, cut_tiles, ncut, ff_flag, ff_list, ff_n);
}

hipError_t launch_extrapolate(const GridP& g, const BandBufs& bb, const StepSlots& s,
                              hipStream_t st, int fused_threads)
{
    if (fused_threads > 0 && fused_fit_ok(g)) {
#define FUSED(T, NT)                                                                              \
    k_fit_fused<T, NT><<<FF_BLOCKS, NT, 0, st>>>(                                                 \
        g, bb.win, s.wcur, s.wprev, bb.tag, (const T*)bb.phi[s.cur], (T*)bb.X[s.nxt],             \
        (T*)bb.Y[s.nxt], bb.health, bb.cut_layer, bb.cut_tiles, bb.ncut, bb.ff_list, bb.ff_n,    \
        fused_threads == 1 ? 1 : 2)
#define FUSED_T(T)                                                                                \
    do {                                                                                          \
        if (fused_threads == 256) FUSED(T, 256);                                                  \
        else if (fused_threads == 512) FUSED(T, 512);                                             \
        else FUSED(T, 1024);                                                                      \
        k_fit_rest<T><<<1, FF_REST_THREADS, 0, st>>>(                                             \
            g, bb.win, s.wcur, s.wprev, bb.tag, bb.lists, bb.lcount, (const T*)bb.phi[s.cur],     \
            (T*)bb.X[s.nxt], (T*)bb.Y[s.nxt], bb.health, bb.cut_layer, bb.cut_tiles, bb.ncut,     \
            bb.ff_flag, bb.ff_list, bb.ff_n);                                                     \
    } while (0)
        if (g.rm32) FUSED_T(float);
        else FUSED_T(double);
#undef FUSED_T
#undef FUSED
        return hipGetLastError();
    }
    for (int l = 1; l <= g.layers; l++)
        if (g.rm32)
            k_layer_fit<float><<<FIT_BLOCKS, 256, 0, st>>>(
                g, bb.win, s.wcur, s.wprev, l, bb.tag, bb.lists, bb.lcount,
                (const float*)bb.phi[s.cur], (float*)bb.X[s.nxt], (float*)bb.Y[s.nxt], bb.health);
        else
            k_layer_fit<double><<<FIT_BLOCKS, 256, 0, st>>>(
                g, bb.win, s.wcur, s.wprev, l, bb.tag, bb.lists, bb.lcount,
                (const double*)bb.phi[s.cur], (double*)bb.X[s.nxt], (double*)bb.Y[s.nxt],
                bb.health);
    return hipGetLastError();
}

// ---------------------------------------------------------------- stress and force

constexpr int FTX = 32, FTY = 8;
constexpr int SX = FTX + 2, SY = FTY + 2;

// F = J^{-1} (Eq. (3_3_refmap_deformation)) and the plane-strain
// neo-Hookean deviatoric stress (Eq. (3_3_solid_stress)) scaled by lam
template <typename C>
__device__ __forceinline__ void tau_of(C J0, C J1, C J2, C J3, C det, C G, C lam, C out[3])
{
    const C F00 = J3 / det, F01 = -J1 / det;
    const C F10 = -J2 / det, F11 = J0 / det;
    const C Bxx = F00 * F00 + F01 * F01;
    const C Bxy = F00 * F10 + F01 * F11;
    const C Byy = F10 * F10 + F11 * F11;
    const C tr = Bxx + Byy;
    out[0] = lam * (G * (Bxx - (tr + C(1)) / C(3)));
    out[1] = lam * (G * Bxy);
    out[2] = lam * (G * (Byy - (tr + C(1)) / C(3)));
}

// Blended stress (1 - H(phi_e)) tau_s of one half-edge from the LDS tile.
// a, bb: the two nodes of the edge (a before bb along the normal direction);
// s1..s4: the side nodes of the tangential difference (s1 + s2 - s3 - s4)/4
// (Eq. (3_3_refmap_jacobian), six-node stencil); dir 0: x-edge, 1: y-edge.
// With displacement storage grad xi = I + grad d; where its determinant is
// below kappa_J the inversion is redone in double.
template <typename C>
__device__ void edge_tau(const GridP& g, const BodyP& b, const C* sX, const C* sY, const C* sP,
                         int a, int bb, int s1, int s2, int s3, int s4, int dir, bool count,
                         unsigned* health, C out[3])
{
    constexpr bool DISP = sizeof(C) == 4;
    out[0] = out[1] = out[2] = C(0);
    const C pa = sP[a], pb = sP[bb];
    if (!(pa < C(INFINITY)) || !(pb < C(INFINITY))) return;
    const C phie = C(0.5) * (pa + pb);
    const C lam = C(1) - heaviside<C>(phie, C(g.eps));
    if (!(lam > C(0))) return;
    if (!(sP[s1] < C(INFINITY)) || !(sP[s2] < C(INFINITY)) || !(sP[s3] < C(INFINITY)) ||
        !(sP[s4] < C(INFINITY))) {
        if (count) atomicAdd(&health[2], 1u);
        return;
    }
    const C nX = sX[bb] - sX[a], nY = sY[bb] - sY[a];
    const C tX = (sX[s1] + sX[s2] - sX[s3] - sX[s4]) / C(4);
    const C tY = (sY[s1] + sY[s2] - sY[s3] - sY[s4]) / C(4);
    C J0, J1, J2, J3;  // [dX/dx, dX/dy; dY/dx, dY/dy]
    if (dir == 0) {
        J0 = nX; J1 = tX; J2 = nY; J3 = tY;
    } else {
        J0 = tX; J1 = nX; J2 = tY; J3 = nY;
    }
    if (DISP) {
        J0 += C(1);
        J3 += C(1);
    }
    const C det = J0 * J3 - J1 * J2;
    if (DISP && !(det >= C(g.kappa_J))) {
        // near-singular (or inverted) grad xi: decide and invert in double
        const double dnX = (double)sX[bb] - (double)sX[a], dnY = (double)sY[bb] - (double)sY[a];
        const double dtX =
            ((double)sX[s1] + (double)sX[s2] - (double)sX[s3] - (double)sX[s4]) / 4.0;
        const double dtY =
            ((double)sY[s1] + (double)sY[s2] - (double)sY[s3] - (double)sY[s4]) / 4.0;
        double K0, K1, K2, K3;
        if (dir == 0) {
            K0 = 1.0 + dnX; K1 = dtX; K2 = dnY; K3 = 1.0 + dtY;
        } else {
            K0 = 1.0 + dtX; K1 = dnX; K2 = dtY; K3 = 1.0 + dnY;
        }
        const double dd = K0 * K3 - K1 * K2;
        if (!(dd > g.detJ_min)) {
            if (count) {
                atomicAdd(&health[3], 1u);
                if (lam > C(0.5)) atomicAdd(&health[4], 1u);
            }
            return;
        }
        double o[3];
        tau_of<double>(K0, K1, K2, K3, dd, b.G, (double)lam, o);
        out[0] = C(o[0]);
        out[1] = C(o[1]);
        out[2] = C(o[2]);
        return;
    }
    if (!(det > C(g.detJ_min))) {
        if (count) {
            atomicAdd(&health[3], 1u);
            if (lam > C(0.5)) atomicAdd(&health[4], 1u);
        }
        return;
    }
    tau_of<C>(J0, J1, J2, J3, det, C(b.G), lam, out);
}

// reference-map node k at (i, j) after the extrapolation of a step: its level
// set phi0(xi) in double (it decides the solid set), or +inf if it holds no map
template <typename C>
__device__ __forceinline__ double relabel_phi(const GridP& g, const BodyP& b, int8_t tv, C xv,
                                              C yv, int i, int j)
{
    if (!tag_set(tv)) return INFINITY;
    double X = (double)xv, Y = (double)yv;
    if (sizeof(C) == 4) {  // displacement storage
        X += pos_x(g, b, i);
        Y += pos_y(g, b, j);
    }
    return shape_phi(b, X, Y);
}

// Shared body of the force kernel (MODE 0) and the stress read (MODE 1) over
// interior tiles of region Rg: stage xi, phi of the tile plus a one-node halo
// in LDS (all loads issued first), compute each half-edge once, then combine
// per node.  MODE 0 also relabels (Alg. 1): phi^{n+1} = phi0(xi^{n+1}) is
// evaluated for every staged node from its tag and map, written for the
// tile's own nodes (with the map cleared where none is held), and for the
// window's nodes outside the interior by a strided pass; each block writes
// the partial box of the new interior solid set it saw, which the next
// lattice update reduces into the next ring slot.  MODE 2 is MODE 0 without
// the stresses (one solid of several: the forces are combined over all
// solids afterwards).  MODE 3 is MODE 0 followed, for each of the tile's own
// nodes, by its lattice Boltzmann update with the force just computed (the
// window's nodes; the lattice update of every other node does not depend on
// the solid's force of this step).
template <int MODE, typename C>
__device__ __forceinline__ void edges_body(GridP g, BodyP b, Win* win, int wvalid,
                                           int* boxpart, int whole_grid, C* X, C* Y,
                                           const C* __restrict__ phi, const int8_t* __restrict__ tag,
                                           C* phi1, double* o0, double* o1, double* o2,
                                           int* lcount, unsigned* health, const LbFuse& lf)
{
    // the force pass ends the reference-map chain of a step: clear the layer
    // counters of the next step's distance transform
    constexpr bool RELABEL = MODE == 0 || MODE == 2 || MODE == 3;
    if (RELABEL) clear_lcount(lcount);
    __shared__ C sX[SY * SX], sY[SY * SX], sP[SY * SX];
    __shared__ C ex[FTY][FTX + 1][3];
    __shared__ C ey[FTY + 1][FTX][3];
    const Rect V = window_of(win, wvalid, g);
    const Rect WP = MODE == 3 ? window_of(win, lf.wprev, g) : Rect{0, -1, 0, -1, false};
    int bi0 = 0x3fffffff, bi1 = -0x3fffffff, bj0 = 0x3fffffff, bj1 = -0x3fffffff;
    // MODE 2: also the box of the nodes with phi < eps (where the solid
    // fraction is positive), partials after the solid box's
    int ei0 = 0x3fffffff, ei1 = -0x3fffffff, ej0 = 0x3fffffff, ej1 = -0x3fffffff;
    Rect Rg;
    if (whole_grid) {
        Rg.i0 = 0; Rg.i1 = g.nx - 1; Rg.j0 = 0; Rg.j1 = g.ny - 1;
        Rg.ok = true;
    } else {
        Rg = V;
        Rg.i0 = max(Rg.i0, 0);
        Rg.j0 = max(Rg.j0, 0);
        Rg.i1 = min(Rg.i1, g.nx - 1);
        Rg.j1 = min(Rg.j1, g.ny - 1);
        Rg.ok = V.ok && Rg.i0 <= Rg.i1 && Rg.j0 <= Rg.j1;
    }
    const int ntx = Rg.ok ? (Rg.i1 - Rg.i0) / FTX + 1 : 0;
    const int nty = Rg.ok ? (Rg.j1 - Rg.j0) / FTY + 1 : 0;
    const int tx = threadIdx.x % FTX, ty = threadIdx.x / FTX;
    for (int t = blockIdx.x; t < ntx * nty; t += gridDim.x) {
        const int i0 = Rg.i0 + (t % ntx) * FTX, j0 = Rg.j0 + (t / ntx) * FTY;
        for (int e = threadIdx.x; e < SX * SY; e += blockDim.x) {
            int ci = i0 - 1 + e % SX, cj = j0 - 1 + e / SX;
            const bool in = b.present && canon(g, ci, cj) && V.has(ci, cj);
            const long long k = in ? pidx(g, ci, cj) : 0;
            const C xv = X[k], yv = Y[k];
            C p;
            if (RELABEL) p = store_phi<C>(relabel_phi<C>(g, b, tag[k], xv, yv, ci, cj));
            else p = phi[k];
            const bool set = in && p < C(INFINITY);
            sX[e] = set ? xv : C(NAN);
            sY[e] = set ? yv : C(NAN);
            sP[e] = set ? p : C(INFINITY);
        }
        __syncthreads();
        const int i = i0 + tx, j = j0 + ty;
        const bool mine = i <= Rg.i1 && j <= Rg.j1;
        if (RELABEL && mine) {
            // relabel output of the tile's own node
            const long long k = pidx(g, i, j);
            const C p = sP[(ty + 1) * SX + tx + 1];
            if (p < C(INFINITY)) {
                phi1[k] = p;
                if (p < C(0)) {
                    bi0 = min(bi0, i);
                    bi1 = max(bi1, i);
                    bj0 = min(bj0, j);
                    bj1 = max(bj1, j);
                }
                if (MODE == 2 && p < C(g.eps)) {
                    ei0 = min(ei0, i);
                    ei1 = max(ei1, i);
                    ej0 = min(ej0, j);
                    ej1 = max(ej1, j);
                }
            } else if (V.has(i, j)) {
                phi1[k] = C(INFINITY);
                X[k] = C(NAN);
                Y[k] = C(NAN);
            }
        }
        if (MODE == 2) {
            __syncthreads();
            continue;
        }
        // health counting: an edge is counted once, by the node on its far
        // side, or by its near node when the far node lies outside the region
        const bool rowin = j <= Rg.j1, colin = i <= Rg.i1;
        constexpr bool FORCE = MODE == 0 || MODE == 3;
        const bool cnt_l = FORCE && (mine || (rowin && i == Rg.i1 + 1));
        const bool cnt_b = FORCE && (mine || (colin && j == Rg.j1 + 1));
        // local index of node (i + di, j + dj)
#define LI(di, dj) ((ty + 1 + (dj)) * SX + (tx + 1 + (di)))
        // x-edge (i - 1/2, j): a = (i-1, j), b = (i, j); side (i, j+1), (i-1, j+1), (i, j-1), (i-1, j-1)
        edge_tau<C>(g, b, sX, sY, sP, LI(-1, 0), LI(0, 0), LI(0, 1), LI(-1, 1), LI(0, -1),
                    LI(-1, -1), 0, cnt_l, health, ex[ty][tx]);
        // y-edge (i, j - 1/2): a = (i, j-1), b = (i, j); side (i+1, j), (i+1, j-1), (i-1, j), (i-1, j-1)
        edge_tau<C>(g, b, sX, sY, sP, LI(0, -1), LI(0, 0), LI(1, 0), LI(1, -1), LI(-1, 0),
                    LI(-1, -1), 1, cnt_b, health, ey[ty][tx]);
        if (tx == FTX - 1) {
            // right x-edge (i + 1/2, j) of the last tile column
            edge_tau<C>(g, b, sX, sY, sP, LI(0, 0), LI(1, 0), LI(1, 1), LI(0, 1), LI(1, -1),
                        LI(0, -1), 0, FORCE && mine && i == Rg.i1, health, ex[ty][tx + 1]);
        }
        if (ty == FTY - 1) {
            // top y-edge (i, j + 1/2) of the last tile row
            edge_tau<C>(g, b, sX, sY, sP, LI(0, 0), LI(0, 1), LI(1, 1), LI(1, 0), LI(-1, 1),
                        LI(-1, 0), 1, FORCE && mine && j == Rg.j1, health, ey[ty + 1][tx]);
        }
#undef LI
        __syncthreads();
        if (mine) {
            const C* L = ex[ty][tx];
            const C* Rr = ex[ty][tx + 1];
            const C* B = ey[ty][tx];
            const C* T = ey[ty + 1][tx];
            const long long n = (long long)j * g.pitch + i;
            if (MODE == 0 || MODE == 3) {
                // Eq. (3_3_div_solid_stress) in Eq. (2_4_F_divs)
                C fx = (Rr[0] - L[0]) + (T[1] - B[1]);
                C fy = (Rr[1] - L[1]) + (T[2] - B[2]);
                const C p = sP[(ty + 1) * SX + tx + 1];
                C H = C(1), dr = C(0);
                if (b.present && p < C(INFINITY)) {
                    H = heaviside<C>(p, C(g.eps));
                    const C drs = C(b.rho_s - g.rho_f);
                    fx += (C(1) - H) * drs * C(g.gx);
                    fy += (C(1) - H) * drs * C(g.gy);
                    dr = (C(1) - H) * drs;  // Eq. (2_3_drho)
                }
                fx += H * C(g.fext_x);
                fy += H * C(g.fext_y);
                o0[n] = (double)fx;
                o1[n] = (double)fy;
                o2[n] = (double)dr;
                if (MODE == 3) {
                    // the node's lattice update (Sec. 3.4, 3.5): F^n as just
                    // stored (in double, read back in C as the lattice
                    // kernels do), F^{n-1} inside the previous window
                    const Neigh q = neigh(g, i, j);
                    C fl[NQ];
                    gather<C>(g, q, (const C*)lf.A, fl);
                    C Fpx = C(lf.fpo_x), Fpy = C(lf.fpo_y);
                    if (WP.has(i, j)) {
                        Fpx = C(lf.fpx[n]);
                        Fpy = C(lf.fpy[n]);
                    }
                    lb_finish_node<C, true>(g, (C*)lf.B, q, fl, Fpx, Fpy, C((double)fx),
                                            C((double)fy), C((double)dr), health);
                }
            } else {
                const long long e = (long long)j * g.nx + i;
                o0[e] = (double)((L[0] + Rr[0] + B[0] + T[0]) / C(4));
                o1[e] = (double)((L[1] + Rr[1] + B[1] + T[1]) / C(4));
                o2[e] = (double)((L[2] + Rr[2] + B[2] + T[2]) / C(4));
            }
        }
        __syncthreads();
    }
    if (RELABEL) {
        // relabel of the window's nodes outside the interior (buffer nodes)
        if (V.ok && b.present) {
            const int w = V.i1 - V.i0 + 1, h = V.j1 - V.j0 + 1;
            for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
                 e < (long long)w * h; e += (long long)gridDim.x * blockDim.x) {
                const int i = V.i0 + (int)(e % w), j = V.j0 + (int)(e / w);
                if (i >= 0 && i < g.nx && j >= 0 && j < g.ny) continue;
                const long long k = pidx(g, i, j);
                const double p = relabel_phi<C>(g, b, tag[k], X[k], Y[k], i, j);
                if (p < INFINITY) {
                    phi1[k] = store_phi<C>(p);
                    if (MODE == 2 && store_phi<C>(p) < C(g.eps)) {
                        ei0 = min(ei0, i);
                        ei1 = max(ei1, i);
                        ej0 = min(ej0, j);
                        ej1 = max(ej1, j);
                    }
                } else {
                    phi1[k] = C(INFINITY);
                    X[k] = C(NAN);
                    Y[k] = C(NAN);
                }
            }
        }
        block_box(bi0, bi1, bj0, bj1, boxpart + 4 * blockIdx.x);
        if (MODE == 2) block_box(ei0, ei1, ej0, ej1, boxpart + 4 * (gridDim.x + blockIdx.x));
    }
}

template <int MODE, typename C>
__global__ __launch_bounds__(256) void k_edges(GridP g, BodyP b, Win* win, int wvalid,
                                               int* boxpart, int whole_grid, C* X, C* Y,
                                               const C* __restrict__ phi,
                                               const int8_t* __restrict__ tag, C* phi1,
                                               double* o0, double* o1, double* o2, int* lcount,
                                               unsigned* health, LbFuse lf)
{
    // beside the bulk lattice update (MODE 3) the force pass is on the
    // critical path: its waves take the issue slots of a SIMD first
    if (MODE == 3) __builtin_amdgcn_s_setprio(3);
    edges_body<MODE, C>(g, b, win, wvalid, boxpart, whole_grid, X, Y, phi, tag, phi1, o0, o1,
                        o2, lcount, health, lf);
}

template <int MODE, typename C>
__global__ __launch_bounds__(256) void kb_force(const EdgesArgs* __restrict__ args,
                                                const int* __restrict__ ord)
{
    const EdgesArgs& a = args[ord ? ord[blockIdx.y] : blockIdx.y];
    edges_body<MODE, C>(a.g, a.b, a.win, a.wvalid, a.boxpart, 0, (C*)a.X, (C*)a.Y, nullptr,
                        a.tag, (C*)a.phi, a.o0, a.o1, a.o2, a.lcount, a.health, LbFuse{});
}

hipError_t launch_force(const GridP& g, const BodyP& b, const BandBufs& bb, const StepSlots& s,
                        double* fx, double* fy, double* drho, hipStream_t st, const LbFuse* lf)
{
#define KE(MODE, C, LF)                                                                       \
    k_edges<MODE, C><<<RELABEL_BLOCKS, 256, 0, st>>>(                                         \
        g, b, bb.win, s.wcur, bb.boxpart, 0, (C*)bb.X[s.nxt], (C*)bb.Y[s.nxt], nullptr, bb.tag, \
        (C*)bb.phi[s.nxt], fx, fy, drho, bb.lcount, bb.health, LF)
    if (lf) {
        if (g.rm32) KE(3, float, *lf);
        else KE(3, double, *lf);
    } else {
        if (g.rm32) KE(0, float, LbFuse{});
        else KE(0, double, LbFuse{});
    }
#undef KE
    return hipGetLastError();
}

// one block: the force pass's partial boxes into ring slot wnext, and the
// zone check of the new window (what the band lattice launch does otherwise)
// (also counts a box whose lower edge moved down by more than
// BULK_EARLY_GAP rows from the current one: the early part of the next
// step's bulk update assumes it does not)
__global__ __launch_bounds__(256) void k_reduce_window(GridP g, const int* __restrict__ boxpart,
                                                       int nbox, Win* win, int wcur, int wnext,
                                                       unsigned* health)
{
    const Win cur = win[wcur];
    const Win r = reduce_boxes(boxpart, nbox, &win[wnext], nullptr);
    if (threadIdx.x == 0) {
        check_zone(g, r, health);
        if (r.i0 <= r.i1 && cur.i0 <= cur.i1 && r.j0 < cur.j0 - BULK_EARLY_GAP)
            atomicAdd(&health[6], 1u);
    }
}

hipError_t launch_reduce_window(const GridP& g, const BandBufs& bb, int wcur, int wnext,
                                hipStream_t st)
{
    k_reduce_window<<<1, 256, 0, st>>>(g, bb.boxpart, RELABEL_BLOCKS, bb.win, wcur, wnext,
                                       bb.health);
    return hipGetLastError();
}

hipError_t launch_read_stress(const GridP& g, const BodyP& b, const BandBufs& bb, int buf,
                              int wvalid, double* sxx, double* sxy, double* syy, hipStream_t st)
{
    if (g.rm32)
        k_edges<1, float><<<2048, 256, 0, st>>>(g, b, bb.win, wvalid, nullptr, 1,
                                                (float*)bb.X[buf], (float*)bb.Y[buf],
                                                (const float*)bb.phi[buf], nullptr, nullptr, sxx,
                                                sxy, syy, nullptr, bb.health, LbFuse{});
    else
        k_edges<1, double><<<2048, 256, 0, st>>>(g, b, bb.win, wvalid, nullptr, 1,
                                                 (double*)bb.X[buf], (double*)bb.Y[buf],
                                                 (const double*)bb.phi[buf], nullptr, nullptr,
                                                 sxx, sxy, syy, nullptr, bb.health, LbFuse{});
    return hipGetLastError();
}

// ---------------------------------------------------------------- reads

template <typename T>
__global__ void k_read_refmap(GridP g, BodyP b, const Win* __restrict__ win, int wvalid,
                              const T* __restrict__ X, const T* __restrict__ Y,
                              const T* __restrict__ phi, double* Xo, double* Yo, double* Po)
{
    constexpr bool DISP = sizeof(T) == 4;
    const Rect V = window_of(win, wvalid, g);
    const long long N = (long long)g.nx * g.ny;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        double xv = NAN, yv = NAN, pv = NAN;
        if (V.has(i, j)) {
            const long long k = pidx(g, i, j);
            if (phi[k] < T(INFINITY)) {
                xv = (double)X[k];
                yv = (double)Y[k];
                pv = (double)phi[k];
                if (DISP) {
                    xv += pos_x(g, b, i);
                    yv += pos_y(g, b, j);
                }
            }
        }
        if (Xo) Xo[e] = xv;
        if (Yo) Yo[e] = yv;
        if (Po) Po[e] = pv;
    }
}

hipError_t launch_read_refmap(const GridP& g, const BodyP& b, const BandBufs& bb, int buf,
                              int wvalid, double* X, double* Y, double* phi, hipStream_t st)
{
    if (g.rm32)
        k_read_refmap<float><<<2048, 256, 0, st>>>(g, b, bb.win, wvalid, (const float*)bb.X[buf],
                                                   (const float*)bb.Y[buf],
                                                   (const float*)bb.phi[buf], X, Y, phi);
    else
        k_read_refmap<double><<<2048, 256, 0, st>>>(g, b, bb.win, wvalid, (const double*)bb.X[buf],
                                                    (const double*)bb.Y[buf],
                                                    (const double*)bb.phi[buf], X, Y, phi);
    return hipGetLastError();
}

// ---------------------------------------------------------------- batched launches

// ---------------------------------------------------------------- several solids
//
// Every solid keeps its reference map on a window of its own (the chain
// kernels above run per solid, blockIdx.y = solid, relabelling only).  The
// lattice is cut into FB x FB force blocks; each step every solid stamps the
// blocks of its working window and lists the newly stamped ones, and one
// kernel over the listed blocks combines all solids into the force planes
// (Sec. 3.6): the global half-edge stress is the solids' blend normalised by
// their summed fraction where it exceeds one, plus the contact stress of
// every pair, Eqs. (3_6_global_stress) to (3_6_normal).

// window index of lattice column c (row r) in solid grid g; along a
// sub-window axis the offset from the window origin, in [-PAD, lnx - PAD)
__device__ __forceinline__ int win_col(const GridP& g, int c)
{
    if (!g.wx) return c;
    const int d = wrap_axis(c - g.ox, g.lnx);
    return d >= g.lnx - PAD ? d - g.lnx : d;
}
__device__ __forceinline__ int win_row(const GridP& g, int r)
{
    if (!g.wy) return r;
    const int d = wrap_axis(r - g.oy, g.lny);
    return d >= g.lny - PAD ? d - g.lny : d;
}

// rectangle V of a solid's window as lattice nodes {x, dx, y, dy}: columns
// x .. x + dx (x wrapped, the range may run over a periodic seam), rows
// likewise; dx < 0 or dy < 0: empty
__device__ int4 mb_region(const GridP& g, const Rect& V)
{
    int4 r = make_int4(0, -1, 0, -1);
    if (!V.ok) return r;
    if (g.wx) {
        r.x = wrap_axis(V.i0 + g.ox, g.lnx);
        r.y = V.i1 - V.i0;
    } else {
        r.x = max(V.i0, 0);
        r.y = min(V.i1, g.nx - 1) - r.x;
    }
    if (g.wy) {
        r.z = wrap_axis(V.j0 + g.oy, g.lny);
        r.w = V.j1 - V.j0;
    } else {
        r.z = max(V.j0, 0);
        r.w = min(V.j1, g.ny - 1) - r.z;
    }
    return r;
}

// do [a, a + la] and [b, b + lb] meet (on a circle of n nodes if periodic)?
__device__ __forceinline__ bool ranges_meet(int a, int la, int b, int lb, int n, int periodic)
{
    if (!periodic) return a <= b + lb && b <= a + la;
    return wrap_axis(b - a, n) <= la || wrap_axis(a - b, n) <= lb;
}

// one block per solid
__global__ __launch_bounds__(256) void k_mb_mark(GridP lg, MbBody* bodies, int wcur, int wnext,
                                                 int nbox, int* stamp, int sval, int* list,
                                                 int* count, int nbx, unsigned* health,
                                                 const long long* dstep)
{
    MbBody& B = bodies[blockIdx.x];
    if (dstep) sval = (int)(*dstep + 1);
    __shared__ Win feps;
    if (nbox > 0) {
        reduce_boxes(B.boxpart, nbox, &B.win[wnext], nullptr);
        reduce_boxes(B.boxpart + 4 * nbox, nbox, &feps, nullptr);
    }
    __shared__ int4 reg;
    if (threadIdx.x == 0) {
        const GridP& g = B.g;
        Rect R;
        if (nbox > 0) {
            check_zone(g, B.win[wnext], health);
            // the force region of this step: the nodes with phi < eps and
            // their neighbours (elsewhere every solid fraction is zero on the
            // node and its edges, and the force is the uniform one), inside
            // the working window
            const Win e = feps;
            const Rect V = window_of(B.win, wcur, g);
            R.i0 = max(e.i0 - 1, V.i0);
            R.i1 = min(e.i1 + 1, V.i1);
            R.j0 = max(e.j0 - 1, V.j0);
            R.j1 = min(e.j1 + 1, V.j1);
            R.ok = V.ok && e.i0 <= e.i1 && R.i0 <= R.i1 && R.j0 <= R.j1;
        } else {
            R = window_of(B.win, wcur, g);
        }
        reg = mb_region(g, R);
        B.reg = reg;
    }
    __syncthreads();
    if (reg.y < 0 || reg.w < 0) return;
    // sample columns x, x + FB, ..., x + dx (and rows alike): every block met
    const int nsx = reg.y / FB + 2, nsy = reg.w / FB + 2;
    for (int e = threadIdx.x; e < nsx * nsy; e += blockDim.x) {
        int gx = reg.x + min((e % nsx) * FB, reg.y), gy = reg.z + min((e / nsx) * FB, reg.w);
        if (lg.px) gx = wrap_axis(gx, lg.nx);
        if (lg.py) gy = wrap_axis(gy, lg.ny);
        const int blk = (gy >> FB_LOG) * nbx + (gx >> FB_LOG);
        if (atomicExch(&stamp[blk], sval) != sval) list[atomicAdd(count, 1)] = blk;
    }
}

hipError_t launch_mb_mark(const GridP& lg, MbBody* bodies, int nb, int wcur, int wnext,
                          int nbox, int* stamp, int sval, int* list, int* count, int nbx,
                          unsigned* health, hipStream_t st, const long long* dstep)
{
    if (nb > 0)
        k_mb_mark<<<nb, 256, 0, st>>>(lg, bodies, wcur, wnext, nbox, stamp, sval, list, count,
                                      nbx, health, dstep);
    return hipGetLastError();
}

__global__ void k_mb_tick(long long* dstep)
{
    if (threadIdx.x == 0) *dstep += 1;
}

hipError_t launch_mb_tick(long long* dstep, hipStream_t st)
{
    k_mb_tick<<<1, 64, 0, st>>>(dstep);
    return hipGetLastError();
}

// xi, phi of solid B on the 3 x 3 nodes around window node (wi, wj), index
// (dj + 1) * 3 + (di + 1); a node without a map holds (NaN, NaN, +inf)
template <typename C>
__device__ __forceinline__ void mb_load3(const MbBody& B, const Rect& V, int buf, int wi, int wj,
                                         C* sX, C* sY, C* sP)
{
    const C* X = (const C*)B.X[buf];
    const C* Y = (const C*)B.Y[buf];
    const C* P = (const C*)B.phi[buf];
#pragma unroll
    for (int e = 0; e < 9; e++) {
        int ci = wi + e % 3 - 1, cj = wj + e / 3 - 1;
        const bool in = canon(B.g, ci, cj) && V.has(ci, cj);
        const long long k = in ? pidx(B.g, ci, cj) : 0;
        const C xv = X[k], yv = Y[k], p = P[k];
        const bool set = in && p < C(INFINITY);
        sX[e] = set ? xv : C(NAN);
        sY[e] = set ? yv : C(NAN);
        sP[e] = set ? p : C(INFINITY);
    }
}

// the half-edges of a node in the 3 x 3 stencil: L, R, B, T as (a, b, s1..s4,
// dir) with a before b along the normal and s1 + s2 - s3 - s4 the tangential
// difference (the stencil of the single-solid force kernel)
__constant__ int MB_EDGE[4][7] = {{3, 4, 7, 6, 1, 0, 0},
                                  {4, 5, 8, 7, 2, 1, 0},
                                  {1, 4, 5, 2, 3, 0, 1},
                                  {4, 7, 8, 5, 6, 3, 1}};

// Eq. (3_6_collision_force)
template <typename C>
__device__ __forceinline__ C contact_f(C x, C eps)
{
    return x < eps ? C(0.5) * (C(1) - x / eps) : C(0);
}

// force density and density excess of lattice node (gi, gj) from the solids
// sl[0 .. ns) (index order) of its block.  mode 0: force and density excess
// (fxo, fyo, drho: lattice planes); 1: density excess only; 2: the node
// average of the four global half-edge solid stresses (blend and contact)
// into fxo, fyo, drho as the xx, xy, yy planes of a read ([ny][nx]), with no
// health counts.
template <typename C>
__device__ void mb_node(const GridP& lg, const MbBody* __restrict__ bodies, const int* sl,
                        int ns, int buf, int wcur, int gi, int gj, double* fxo, double* fyo,
                        double* drho, int mode, unsigned* health)
{
    const bool drho_only = mode == 1;
    C acc[4][3], lse[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        lse[e] = C(0);
        acc[e][0] = acc[e][1] = acc[e][2] = C(0);
    }
    C lsum = C(0), dacc = C(0);
    int nset = 0;
    for (int q = 0; q < ns; q++) {
        const MbBody& B = bodies[sl[q]];
        const GridP& g = B.g;
        const int wi = win_col(g, gi), wj = win_row(g, gj);
        const Rect V = window_of(B.win, wcur, g);
        if (!V.has(wi, wj)) continue;
        C sX[9], sY[9], sP[9];
        mb_load3<C>(B, V, buf, wi, wj, sX, sY, sP);
        if (!(sP[4] < C(INFINITY))) continue;
        nset++;
        const C lam = C(1) - heaviside<C>(sP[4], C(g.eps));
        lsum += lam;
        dacc += lam * C(B.b.rho_s - lg.rho_f);
        if (drho_only) continue;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int a = MB_EDGE[e][0], b = MB_EDGE[e][1];
            if (!(sP[a] < C(INFINITY)) || !(sP[b] < C(INFINITY))) continue;
            const C le = C(1) - heaviside<C>(C(0.5) * (sP[a] + sP[b]), C(g.eps));
            if (!(le > C(0))) continue;
            lse[e] += le;
            C t[3];
            // each edge is counted once: by its far node (the L and B edges)
            edge_tau<C>(g, B.b, sX, sY, sP, a, b, MB_EDGE[e][2], MB_EDGE[e][3], MB_EDGE[e][4],
                        MB_EDGE[e][5], MB_EDGE[e][6], mode == 0 && (e == 0 || e == 2), health,
                        t);
            acc[e][0] += t[0];
            acc[e][1] += t[1];
            acc[e][2] += t[2];
        }
    }
    const long long n = (long long)gj * lg.pitch + gi;
    const C dr = lsum > C(1) ? dacc / lsum : dacc;
    if (mode != 2) drho[n] = (double)dr;
    if (drho_only) return;
#pragma unroll
    for (int e = 0; e < 4; e++)
        if (lse[e] > C(1)) {
            acc[e][0] /= lse[e];
            acc[e][1] /= lse[e];
            acc[e][2] /= lse[e];
        }
    if (nset >= 2 && lg.eta != 0.0) {
        // contact stress of every pair (p, q), p < q, on the node's edges
        for (int p = 0; p < ns; p++) {
            const MbBody& Bp = bodies[sl[p]];
            const int pi = win_col(Bp.g, gi), pj = win_row(Bp.g, gj);
            const Rect Vp = window_of(Bp.win, wcur, Bp.g);
            if (!Vp.has(pi, pj)) continue;
            C pX[9], pY[9], pP[9];
            mb_load3<C>(Bp, Vp, buf, pi, pj, pX, pY, pP);
            if (!(pP[4] < C(INFINITY))) continue;
            for (int q = p + 1; q < ns; q++) {
                const MbBody& Bq = bodies[sl[q]];
                const int qi = win_col(Bq.g, gi), qj = win_row(Bq.g, gj);
                const Rect Vq = window_of(Bq.win, wcur, Bq.g);
                if (!Vq.has(qi, qj)) continue;
                C qX[9], qY[9], qP[9];
                mb_load3<C>(Bq, Vq, buf, qi, qj, qX, qY, qP);
                if (!(qP[4] < C(INFINITY))) continue;
                const C cg = C(-lg.eta);
                const C gsum = C(Bp.b.G + Bq.b.G);
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    bool all = true;
#pragma unroll
                    for (int t = 0; t < 6; t++) {
                        const int v = MB_EDGE[e][t];
                        all = all && pP[v] < C(INFINITY) && qP[v] < C(INFINITY);
                    }
                    if (!all) continue;
                    const int a = MB_EDGE[e][0], b = MB_EDGE[e][1];
                    const C fp = contact_f<C>(C(0.5) * (pP[a] + pP[b]), C(lg.eps));
                    const C fq = contact_f<C>(C(0.5) * (qP[a] + qP[b]), C(lg.eps));
                    const C fmin = fp < fq ? fp : fq;
                    if (!(fmin > C(0))) continue;
                    C d[6];
#pragma unroll
                    for (int t = 0; t < 6; t++) {
                        const int v = MB_EDGE[e][t];
                        d[t] = pP[v] - qP[v];
                    }
                    // Eq. (3_6_normal) on the edge stencil
                    const C gn = d[1] - d[0];
                    const C gt = (d[2] + d[3] - d[4] - d[5]) / C(4);
                    const C gx = MB_EDGE[e][6] == 0 ? gn : gt;
                    const C gy = MB_EDGE[e][6] == 0 ? gt : gn;
                    const C gl = sqrt(gx * gx + gy * gy);
                    if (!(gl > C(0))) continue;
                    const C nx = gx / gl, ny = gy / gl;
                    const C c = cg * fmin * gsum;
                    acc[e][0] += c * (nx * nx - C(0.5));
                    acc[e][1] += c * (nx * ny);
                    acc[e][2] += c * (ny * ny - C(0.5));
                }
            }
        }
    }
    if (mode == 2) {
        const long long r = (long long)gj * lg.nx + gi;
        fxo[r] = (double)((acc[0][0] + acc[1][0] + acc[2][0] + acc[3][0]) / C(4));
        fyo[r] = (double)((acc[0][1] + acc[1][1] + acc[2][1] + acc[3][1]) / C(4));
        drho[r] = (double)((acc[0][2] + acc[1][2] + acc[2][2] + acc[3][2]) / C(4));
        return;
    }
    // Eq. (3_3_div_solid_stress) on the node's four edges, buoyancy of the
    // mixture and the fluid's share of the external force
    C fx = (acc[1][0] - acc[0][0]) + (acc[3][1] - acc[2][1]);
    C fy = (acc[1][1] - acc[0][1]) + (acc[3][2] - acc[2][2]);
    fx += dr * C(lg.gx);
    fy += dr * C(lg.gy);
    const C hf = lsum < C(1) ? C(1) - lsum : C(0);
    fx += hf * C(lg.fext_x);
    fy += hf * C(lg.fext_y);
    fxo[n] = (double)fx;
    fyo[n] = (double)fy;
}

// mode as mb_node; list null: every force block (nblk_all of them)
template <typename C>
__global__ __launch_bounds__(256) void k_mb_combine(GridP lg, const MbBody* __restrict__ bodies,
                                                    int nb, int buf, int wcur,
                                                    const int* __restrict__ list,
                                                    const int* __restrict__ count,
                                                    int* count_clear, int nbx, double* fx,
                                                    double* fy, double* drho, int mode,
                                                    unsigned* health, int nblk_all)
{
    static_assert(FB * FB == 256, "one thread per node of a force block");
    if (blockIdx.x == 0 && threadIdx.x == 0 && count_clear) *count_clear = 0;
    __shared__ int sl[MB_MAX_PER_BLOCK];
    __shared__ int wcnt[4];
    __shared__ int ns;
    const int nblk = list ? *count : nblk_all;
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int t = blockIdx.x; t < nblk; t += gridDim.x) {
        const int blk = list ? list[t] : t;
        const int bx0 = (blk % nbx) * FB, by0 = (blk / nbx) * FB;
        if (threadIdx.x == 0) ns = 0;
        __syncthreads();
        // the solids whose region meets this block, in index order
        for (int base = 0; base < nb; base += blockDim.x) {
            const int k = base + threadIdx.x;
            bool hit = false;
            if (k < nb) {
                const int4 r = bodies[k].reg;
                hit = r.y >= 0 && r.w >= 0 &&
                      ranges_meet(r.x, r.y, bx0, FB - 1, lg.nx, lg.px) &&
                      ranges_meet(r.z, r.w, by0, FB - 1, lg.ny, lg.py);
            }
            const unsigned long long m = __ballot(hit);
            if (lane == 0) wcnt[w] = __popcll(m);
            __syncthreads();
            int off = ns + __popcll(m & ((1ull << lane) - 1ull));
            for (int u = 0; u < w; u++) off += wcnt[u];
            if (hit) {
                if (off < MB_MAX_PER_BLOCK) sl[off] = k;
                else if (mode != 2) atomicAdd(&health[7], 1u);
            }
            __syncthreads();
            if (threadIdx.x == 0) ns = min(ns + wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3],
                                           MB_MAX_PER_BLOCK);
            __syncthreads();
        }
        const int gi = bx0 + threadIdx.x % FB, gj = by0 + threadIdx.x / FB;
        if (gi < lg.nx && gj < lg.ny)
            mb_node<C>(lg, bodies, sl, ns, buf, wcur, gi, gj, fx, fy, drho, mode, health);
        __syncthreads();
    }
}

hipError_t launch_mb_combine(const GridP& lg, int precision, const MbBody* bodies, int nb,
                             int buf, int wcur, const int* list, const int* count,
                             int* count_clear, int nbx, double* fx, double* fy, double* drho,
                             bool drho_only, unsigned* health, hipStream_t st)
{
    if (precision == 0)
        k_mb_combine<double><<<MB_COMBINE_BLOCKS, 256, 0, st>>>(
            lg, bodies, nb, buf, wcur, list, count, count_clear, nbx, fx, fy, drho,
            drho_only ? 1 : 0, health, 0);
    else
        k_mb_combine<float><<<MB_COMBINE_BLOCKS, 256, 0, st>>>(
            lg, bodies, nb, buf, wcur, list, count, count_clear, nbx, fx, fy, drho,
            drho_only ? 1 : 0, health, 0);
    return hipGetLastError();
}

hipError_t launch_mb_read_stress(const GridP& lg, int precision, const MbBody* bodies, int nb,
                                 int buf, int wslot, int nbx, int nby, double* sxx, double* sxy,
                                 double* syy, unsigned* health, hipStream_t st)
{
    if (precision == 0)
        k_mb_combine<double><<<MB_COMBINE_BLOCKS, 256, 0, st>>>(
            lg, bodies, nb, buf, wslot, nullptr, nullptr, nullptr, nbx, sxx, sxy, syy, 2, health,
            nbx * nby);
    else
        k_mb_combine<float><<<MB_COMBINE_BLOCKS, 256, 0, st>>>(
            lg, bodies, nb, buf, wslot, nullptr, nullptr, nullptr, nbx, sxx, sxy, syy, 2, health,
            nbx * nby);
    return hipGetLastError();
}

// a solid's window origin in its table entries
__device__ void mb_set_origin(MbBody& B, const MbTabs& tabs, int k, int ox, int oy)
{
    B.g.ox = ox;
    B.g.oy = oy;
    for (int p = 0; p < 7; p++) {
        tabs.adv[p][k].g.ox = ox;
        tabs.adv[p][k].g.oy = oy;
        tabs.lay[p][k].g.ox = ox;
        tabs.lay[p][k].g.oy = oy;
        tabs.fit[p][k].g.ox = ox;
        tabs.fit[p][k].g.oy = oy;
        tabs.edg[p][k].g.ox = ox;
        tabs.edg[p][k].g.oy = oy;
    }
}

// the region boxes and window origins of the solids from a saved copy of the
// solid table (every other field of a table entry is fixed by the context)
__global__ void k_mb_copy_reg(const MbBody* __restrict__ src, MbBody* dst, int nb, MbTabs tabs)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nb) {
        dst[k].reg = src[k].reg;
        mb_set_origin(dst[k], tabs, k, src[k].g.ox, src[k].g.oy);
    }
}

hipError_t launch_mb_copy_reg(const MbBody* src, MbBody* dst, int nb, const MbTabs& tabs,
                              hipStream_t st)
{
    k_mb_copy_reg<<<(nb + 255) / 256, 256, 0, st>>>(src, dst, nb, tabs);
    return hipGetLastError();
}

// the shift of one sub-window axis: 0 while the zone [lo - L, hi + L] keeps
// MB_RECENTRE_MARGIN nodes from both ends of [0, n), else the move that puts
// the box's middle at the window's middle
__device__ __forceinline__ int recentre_shift(int lo, int hi, int L, int n)
{
    if (lo - L >= MB_RECENTRE_MARGIN && hi + L <= n - 1 - MB_RECENTRE_MARGIN) return 0;
    const int mid2 = lo + hi;  // twice the box's middle
    return (mid2 - (n - 1)) / 2;
}

template <typename T>
__global__ __launch_bounds__(256) void k_mb_recentre(MbBody* bodies, MbTabs tabs, int buf,
                                                     int wa, int wb)
{
    const int k = blockIdx.x;
    MbBody& B = bodies[k];
    __shared__ int s_dx, s_dy;
    if (threadIdx.x == 0) {
        const GridP& g = B.g;
        const Win a = B.win[wa], b = B.win[wb];
        const bool av = a.i0 <= a.i1 && a.j0 <= a.j1, bv = b.i0 <= b.i1 && b.j0 <= b.j1;
        int dx = 0, dy = 0;
        if (av || bv) {
            const int i0 = min(av ? a.i0 : b.i0, bv ? b.i0 : a.i0);
            const int i1 = max(av ? a.i1 : b.i1, bv ? b.i1 : a.i1);
            const int j0 = min(av ? a.j0 : b.j0, bv ? b.j0 : a.j0);
            const int j1 = max(av ? a.j1 : b.j1, bv ? b.j1 : a.j1);
            if (g.wx) dx = recentre_shift(i0, i1, g.layers, g.nx);
            if (g.wy) dy = recentre_shift(j0, j1, g.layers, g.ny);
        }
        s_dx = dx;
        s_dy = dy;
    }
    __syncthreads();
    const int dx = s_dx, dy = s_dy;
    if (dx == 0 && dy == 0) return;
    const GridP& g = B.g;
    T* X = (T*)B.X[buf];
    T* Y = (T*)B.Y[buf];
    T* P = (T*)B.phi[buf];
    T* tX = (T*)B.X[1 - buf];
    T* tY = (T*)B.Y[1 - buf];
    T* tP = (T*)B.phi[1 - buf];
    // padded window (-PAD .. n + PAD - 1 on each axis, row pitch pp): node
    // (i, j) of the moved window is node (i + dx, j + dy) of the old one
    const int wpx = g.nx + 2 * PAD, wpy = g.ny + 2 * PAD;
    const long long N = (long long)g.pp * wpy;
    for (long long e = threadIdx.x; e < N; e += blockDim.x) {
        const int pi = (int)(e % g.pp), pj = (int)(e / g.pp);
        const int si = pi + dx, sj = pj + dy;
        const bool in = pi < wpx && si >= 0 && si < wpx && sj >= 0 && sj < wpy;
        const long long q = in ? (long long)sj * g.pp + si : 0;
        tX[e] = in ? X[q] : T(0);
        tY[e] = in ? Y[q] : T(0);
        tP[e] = in ? P[q] : T(INFINITY);
    }
    __syncthreads();
    for (long long e = threadIdx.x; e < N; e += blockDim.x) {
        X[e] = tX[e];
        Y[e] = tY[e];
        P[e] = tP[e];
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 3; q++) {
            Win& w = B.win[q];
            if (w.i0 > w.i1 || w.j0 > w.j1) continue;
            w.i0 -= dx;
            w.i1 -= dx;
            w.j0 -= dy;
            w.j1 -= dy;
        }
        mb_set_origin(B, tabs, k, g.ox + dx, g.oy + dy);
    }
}

hipError_t launch_mb_recentre(int precision, MbBody* bodies, int nb, const MbTabs& tabs, int buf,
                              int wa, int wb, hipStream_t st)
{
    if (precision == 0) k_mb_recentre<double><<<nb, 256, 0, st>>>(bodies, tabs, buf, wa, wb);
    else k_mb_recentre<float><<<nb, 256, 0, st>>>(bodies, tabs, buf, wa, wb);
    return hipGetLastError();
}

// xi and phi of solid k on the lattice nodes (NaN where it holds no map)
template <typename C>
__global__ void k_mb_read_refmap(GridP lg, const MbBody* __restrict__ bodies, int k, int buf,
                                 int wvalid, double* X, double* Y, double* phi)
{
    const MbBody& B = bodies[k];
    const GridP& g = B.g;
    const Rect V = window_of(B.win, wvalid, g);
    const C* Xs = (const C*)B.X[buf];
    const C* Ys = (const C*)B.Y[buf];
    const C* Ps = (const C*)B.phi[buf];
    const long long N = (long long)lg.nx * lg.ny;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int gi = (int)(e % lg.nx), gj = (int)(e / lg.nx);
        const int i = win_col(g, gi), j = win_row(g, gj);
        double xv = NAN, yv = NAN, pv = NAN;
        if (V.has(i, j) && i >= 0 && i < g.nx && j >= 0 && j < g.ny) {
            const long long kk = pidx(g, i, j);
            const C p = Ps[kk];
            if (p < C(INFINITY)) {
                xv = (double)Xs[kk];
                yv = (double)Ys[kk];
                if (sizeof(C) == 4) {
                    xv += pos_x(g, B.b, i);
                    yv += pos_y(g, B.b, j);
                }
                pv = (double)p;
            }
        }
        if (X) X[e] = xv;
        if (Y) Y[e] = yv;
        if (phi) phi[e] = pv;
    }
}

hipError_t launch_mb_read_refmap(const GridP& lg, int precision, const MbBody* bodies, int k,
                                 int buf, int wvalid, double* X, double* Y, double* phi,
                                 hipStream_t st)
{
    const long long N = (long long)lg.nx * lg.ny;
    const int blocks = (int)((N + 255) / 256 < 4096 ? (N + 255) / 256 : 4096);
    if (precision == 0)
        k_mb_read_refmap<double><<<blocks, 256, 0, st>>>(lg, bodies, k, buf, wvalid, X, Y, phi);
    else
        k_mb_read_refmap<float><<<blocks, 256, 0, st>>>(lg, bodies, k, buf, wvalid, X, Y, phi);
    return hipGetLastError();
}

// one block per solid: its fraction moments over the interior nodes of its
// window, reduced in a fixed order
template <typename C>
__global__ __launch_bounds__(256) void k_mb_diag(const MbBody* __restrict__ bodies, int buf,
                                                 int wvalid, double* out)
{
    const MbBody& B = bodies[blockIdx.x];
    const GridP& g = B.g;
    const Rect V = window_of(B.win, wvalid, g);
    const C* Xs = (const C*)B.X[buf];
    const C* Ys = (const C*)B.Y[buf];
    const C* Ps = (const C*)B.phi[buf];
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    if (V.ok) {
        const int i0 = max(V.i0, 0), i1 = min(V.i1, g.nx - 1);
        const int j0 = max(V.j0, 0), j1 = min(V.j1, g.ny - 1);
        const int w = i1 - i0 + 1, h = j1 - j0 + 1;
        if (w > 0 && h > 0)
            for (int e = threadIdx.x; e < w * h; e += blockDim.x) {
                const int i = i0 + e % w, j = j0 + e / w;
                const long long k = pidx(g, i, j);
                const double p = (double)Ps[k];
                if (!(p < INFINITY)) continue;
                a[6] += 1.0;
                if (p < 0.0) a[5] += 1.0;
                const double lam = 1.0 - heaviside<double>(p, g.eps);
                const double x = pos_x(g, B.b, i), y = pos_y(g, B.b, j);
                double dx, dy;
                if (sizeof(C) == 4) {  // displacement storage: x - xi = -d
                    dx = -(double)Xs[k];
                    dy = -(double)Ys[k];
                } else {
                    dx = x - (double)Xs[k];
                    dy = y - (double)Ys[k];
                }
                a[0] += lam;
                a[1] += lam * x;
                a[2] += lam * y;
                a[3] += lam * dx;
                a[4] += lam * dy;
            }
    }
    __shared__ double red[7][256];
    for (int t = 0; t < 7; t++) red[t][threadIdx.x] = a[t];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int t = 0; t < 7; t++) red[t][threadIdx.x] += red[t][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 7) out[7 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_mb_diag(int precision, const MbBody* bodies, int nb, int buf, int wvalid,
                          double* out, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    if (precision == 0) k_mb_diag<double><<<nb, 256, 0, st>>>(bodies, buf, wvalid, out);
    else k_mb_diag<float><<<nb, 256, 0, st>>>(bodies, buf, wvalid, out);
    return hipGetLastError();
}

hipError_t launch_batch_band(int precision, const BatchTables& t, int nsim, int layers,
                             hipStream_t st, bool relabel_only, int dt_blocks, int fit_blocks,
                             int band_blocks, bool fused)
{
    const dim3 gb(band_blocks, nsim), gd(dt_blocks, nsim), gf(fit_blocks, nsim);
    // fit_blocks == 0: every layer of a member in one block (kb_fit_lds);
    // fused: every layer of a member in one launch over its zone tiles (the
    // members' advection pass lists those tiles)
    const dim3 g1(1, nsim), gz(FF_BATCH_BLOCKS, nsim);
    if (precision == 0) {
        if (layers == 11) kb_advect_dt<11, double><<<gd, 256, 0, st>>>(t.adv, t.ord);
        else kb_advect_dt<0, double><<<gd, 256, 0, st>>>(t.adv, t.ord);
        if (fused) {
            kb_fit_fused<double><<<gz, 1024, 0, st>>>(t.fit);
            kb_fit_rest<double><<<g1, FF_REST_THREADS, 0, st>>>(t.fit);
        } else if (fit_blocks == 0) {
            kb_fit_lds<double, MB_FIT_THREADS_F64><<<g1, MB_FIT_THREADS_F64, 0, st>>>(t.fit, layers,
                                                                                 t.ord);
        } else {
            for (int l = 1; l <= layers; l++) kb_layer_fit<double><<<gf, 256, 0, st>>>(t.fit, l);
        }
        if (relabel_only) kb_force<2, double><<<gb, 256, 0, st>>>(t.edg, t.ord);
        else kb_force<0, double><<<gb, 256, 0, st>>>(t.edg, t.ord);
    } else {
        if (layers == 11) kb_advect_dt<11, float><<<gd, 256, 0, st>>>(t.adv, t.ord);
        else kb_advect_dt<0, float><<<gd, 256, 0, st>>>(t.adv, t.ord);
        if (fused) {
            kb_fit_fused<float><<<gz, 1024, 0, st>>>(t.fit);
            kb_fit_rest<float><<<g1, FF_REST_THREADS, 0, st>>>(t.fit);
        } else if (fit_blocks == 0) {
            kb_fit_lds<float, MB_FIT_THREADS_F32><<<g1, MB_FIT_THREADS_F32, 0, st>>>(t.fit, layers,
                                                                                t.ord);
        } else {
            for (int l = 1; l <= layers; l++) kb_layer_fit<float><<<gf, 256, 0, st>>>(t.fit, l);
        }
        if (relabel_only) kb_force<2, float><<<gb, 256, 0, st>>>(t.edg, t.ord);
        else kb_force<0, float><<<gb, 256, 0, st>>>(t.edg, t.ord);
    }
    return hipGetLastError();
}

}  // namespace lbrmt
