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
// floating-point contraction so they are taken in plain IEEE double arithmetic.
#include "lbrmt_internal.h"

namespace lbrmt {

constexpr double PI_D = 3.14159265358979323846;

__device__ __forceinline__ double heaviside(double phi, double eps)
{
    // Eq. (2_3_heaviside)
    if (phi <= -eps) return 0.0;
    if (phi >= eps) return 1.0;
    return 0.5 * (1.0 + phi / eps + sin(PI_D * phi / eps) / PI_D);
}

// reference shape level set phi0(X): disc |X - c| - R
__device__ __forceinline__ double shape_phi(const BodyP& b, double X, double Y)
{
    const double dx = X - b.cx, dy = Y - b.cy;
    return sqrt(dx * dx + dy * dy) - b.R;
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
__device__ void reduce_boxes(const int* part, int n, Win* dst0, Win* dst1)
{
    __shared__ int sb[4][16];
    int a0 = 0x3fffffff, a1 = -0x3fffffff, a2 = 0x3fffffff, a3 = -0x3fffffff;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const volatile int* q = part + 4 * k;
        a0 = min(a0, q[0]);
        a1 = max(a1, q[1]);
        a2 = min(a2, q[2]);
        a3 = max(a3, q[3]);
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
        Win r;
        r.i0 = a0;
        r.i1 = a1;
        r.j0 = a2;
        r.j1 = a3;
        if (a0 > a1) r.i0 = 0x3fffffff, r.i1 = -0x3fffffff, r.j0 = 0x3fffffff, r.j1 = -0x3fffffff;
        *dst0 = r;
        if (dst1) *dst1 = r;
    }
    __syncthreads();
}

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
    const double x = node_coord(i, g.px, g.nx, b.cx);
    const double y = node_coord(j, g.py, g.ny, b.cy);
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
        reduce_boxes(boxpart, gridDim.x, &win[s0], &win[s1]);
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
                                                   int wslot)
{
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
    k_init_tags<<<2048, 256, 0, st>>>(g, b, bb.tag, bb.win, wslot);
    return hipGetLastError();
}

// xi_0 = x on the solid and its extrapolation zone, phi = phi0(x) (Alg. 1 init)
__global__ void k_init_fill(GridP g, BodyP b, const int8_t* tag, const Win* win, int wslot,
                            double* X, double* Y, double* phi)
{
    const Rect W = window_of(win, wslot, g);
    if (!W.ok) return;
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)w * h;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
        const long long k = pidx(g, i, j);
        if (tag[k] != TAG_NONE) {
            const double x = node_coord(i, g.px, g.nx, b.cx);
            const double y = node_coord(j, g.py, g.ny, b.cy);
            X[k] = x;
            Y[k] = y;
            phi[k] = shape_phi(b, x, y);
        } else {
            X[k] = NAN;
            Y[k] = NAN;
            phi[k] = INFINITY;
        }
    }
}

hipError_t launch_init_fill(const GridP& g, const BodyP& b, const BandBufs& bb, int wslot,
                            hipStream_t st)
{
    k_init_fill<<<2048, 256, 0, st>>>(g, b, bb.tag, bb.win, wslot, bb.X[0], bb.Y[0], bb.phi[0]);
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
// stencil values (m1, m2: one and two nodes behind; p1, p2: ahead)
__device__ __forceinline__ bool upwind_d(double vel, double X0, double Y0, bool okm1, bool okm2,
                                         double Xm1, double Ym1, double Xm2, double Ym2,
                                         bool okp1, bool okp2, double Xp1, double Yp1,
                                         double Xp2, double Yp2, double& dX, double& dY)
{
    dX = dY = 0.0;
    if (vel == 0.0) return true;
    if (vel > 0.0) {
        if (!okm1 || !okm2) return false;
        dX = (3.0 * X0 - 4.0 * Xm1 + Xm2) / 2.0;
        dY = (3.0 * Y0 - 4.0 * Ym1 + Ym2) / 2.0;
    } else {
        if (!okp1 || !okp2) return false;
        dX = (-3.0 * X0 + 4.0 * Xp1 - Xp2) / 2.0;
        dY = (-3.0 * Y0 + 4.0 * Yp1 - Yp2) / 2.0;
    }
    return true;
}

// Eq. (3_1_refmap_adv) on the solid nodes S^n = {interior, phi^n < 0}, plus
// the step's tags (solid / none) over the window and the cleared tile flags.
// Every load of a node (its level set, the eight upwind stencil nodes, the
// nine populations and the previous force) is issued before any is used;
// addresses of absent nodes are clamped to the node itself.
template <typename S>
__global__ __launch_bounds__(256) void k_advect(GridP g, const S* __restrict__ A,
                                                const double* __restrict__ fpx,
                                                const double* __restrict__ fpy,
                                                const double* __restrict__ X,
                                                const double* __restrict__ Y,
                                                const double* __restrict__ phi, double* X1,
                                                double* Y1, int8_t* tag,
                                                const Win* __restrict__ win, int wprev, int wcur,
                                                unsigned* health)
{
    const Rect W = window_of(win, wcur, g);
    if (!W.ok) return;
    const Rect D = window_of(win, wprev, g);
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    const long long total = (long long)w * h;
    const long long P = g.plane;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
        const long long k = pidx(g, i, j);
        const bool interior = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
        // stencil nodes: x-1, x-2, x+1, x+2, y-1, y-2, y+1, y+2
        const int di[8] = {-1, -2, 1, 2, 0, 0, 0, 0};
        const int dj[8] = {0, 0, 0, 0, -1, -2, 1, 2};
        long long ks[8];
#pragma unroll
        for (int q = 0; q < 8; q++) ks[q] = ref_index(g, D, i + di[q], j + dj[q]);
        // populations of the pull gather (clamped to the interior)
        const int ic = min(max(i, 0), g.nx - 1), jc = min(max(j, 0), g.ny - 1);
        const bool bw = !g.px && ic == 0, be = !g.px && ic == g.nx - 1;
        const bool bs = !g.py && jc == 0, bn = !g.py && jc == g.ny - 1;
        int im = ic - 1, ip = ic + 1, jm = jc - 1, jp = jc + 1;
        im = im < 0 ? (g.px ? g.nx - 1 : 0) : im;
        ip = ip >= g.nx ? (g.px ? 0 : g.nx - 1) : ip;
        jm = jm < 0 ? (g.py ? g.ny - 1 : 0) : jm;
        jp = jp >= g.ny ? (g.py ? 0 : g.ny - 1) : jp;
        const long long r0 = (long long)jc * g.pitch, rm = (long long)jm * g.pitch,
                        rp = (long long)jp * g.pitch, n = r0 + ic;
        // ---- all loads
        const double p0 = phi[k], X0 = X[k], Y0 = Y[k];
        double ps[8], xs[8], ys[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const long long kq = ks[q] >= 0 ? ks[q] : k;
            ps[q] = phi[kq];
            xs[q] = X[kq];
            ys[q] = Y[kq];
        }
        double f[NQ];
        f[0] = A[n];
        f[1] = bw ? A[3 * P + n] : A[1 * P + r0 + im];
        f[2] = bs ? A[4 * P + n] : A[2 * P + rm + ic];
        f[3] = be ? A[1 * P + n] : A[3 * P + r0 + ip];
        f[4] = bn ? A[2 * P + n] : A[4 * P + rp + ic];
        f[5] = (bw || bs) ? A[7 * P + n] : A[5 * P + rm + im];
        f[6] = (be || bs) ? A[8 * P + n] : A[6 * P + rm + ip];
        f[7] = (be || bn) ? A[5 * P + n] : A[7 * P + rp + ip];
        f[8] = (bw || bn) ? A[6 * P + n] : A[8 * P + rp + im];
        const double Fx = fpx[n], Fy = fpy[n];
        // ---- decisions and arithmetic
        const bool solid = interior && D.has(i, j) && p0 < 0.0;
        tag[k] = solid ? TAG_SOLID : TAG_NONE;
        if (!solid) continue;
        if (sizeof(S) == 4) {
            const double wq[NQ] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
            for (int q = 0; q < NQ; q++) f[q] += wq[q] * g.rho_f;
        }
        // half-force velocity of Eq. (2_2_lbm_moments_force)
        const double rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
        const double u = (f[1] + f[5] + f[8] - f[3] - f[6] - f[7]) / rho + Fx / (2.0 * rho);
        const double v = (f[2] + f[5] + f[6] - f[4] - f[7] - f[8]) / rho + Fy / (2.0 * rho);
        bool okq[8];
#pragma unroll
        for (int q = 0; q < 8; q++) okq[q] = ks[q] >= 0 && ps[q] < INFINITY;
        double dXx, dYx, dXy, dYy;
        const bool okx = upwind_d(u, X0, Y0, okq[0], okq[1], xs[0], ys[0], xs[1], ys[1], okq[2],
                                  okq[3], xs[2], ys[2], xs[3], ys[3], dXx, dYx);
        const bool oky = upwind_d(v, X0, Y0, okq[4], okq[5], xs[4], ys[4], xs[5], ys[5], okq[6],
                                  okq[7], xs[6], ys[6], xs[7], ys[7], dXy, dYy);
        if (!okx || !oky) {
            atomicAdd(&health[0], 1u);
            X1[k] = X0;
            Y1[k] = Y0;
        } else {
            X1[k] = X0 - (u * dXx + v * dXy);
            Y1[k] = Y0 - (u * dYx + v * dYy);
        }
    }
}

hipError_t launch_advect(const GridP& g, int precision, const BodyP& b, const BandBufs& bb,
                         const StepSlots& s, const void* A, const double* fpx, const double* fpy,
                         double fpo_x, double fpo_y, hipStream_t st)
{
    (void)b;
    (void)fpo_x;
    (void)fpo_y;
    if (precision == 0)
        k_advect<double><<<2048, 256, 0, st>>>(g, (const double*)A, fpx, fpy, bb.X[s.cur],
                                               bb.Y[s.cur], bb.phi[s.cur], bb.X[s.nxt],
                                               bb.Y[s.nxt], bb.tag, bb.win, s.wprev,
                                               s.wcur, bb.health);
    else
        k_advect<float><<<2048, 256, 0, st>>>(g, (const float*)A, fpx, fpy, bb.X[s.cur],
                                              bb.Y[s.cur], bb.phi[s.cur], bb.X[s.nxt],
                                              bb.Y[s.nxt], bb.tag, bb.win, s.wprev,
                                              s.wcur, bb.health);
    return hipGetLastError();
}

// ---------------------------------------------------------------- layers

// Layers of Sec. 3.2: layer 1 = non-solid nodes 4-adjacent to the solid,
// layer l = unmarked nodes 4-adjacent to layer l-1.  Inside a rectangle this
// is the Manhattan distance to the solid set, computed here exactly in two
// separable passes: per column, the distance to the nearest solid node of the
// column (capped at layers + 1); per row, min over |e| of |e| + that distance.
__global__ __launch_bounds__(256) void k_dt_cols(GridP g, const Win* __restrict__ win, int wslot,
                                                 const int8_t* __restrict__ tag, int8_t* gcol,
                                                 int* lcount)
{
    if (blockIdx.x == 0 && threadIdx.x < (MAX_LAYERS + 1) * NSUB)
        lcount[threadIdx.x * LCOUNT_PAD] = 0;
    const Rect W = window_of(win, wslot, g);
    if (!W.ok) return;
    const int L = g.layers;
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)w * h;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
        int best = L + 1;
        for (int d = -L; d <= L; d++) {
            const int jj = j + d;
            const bool in = jj >= W.j0 && jj <= W.j1;
            const int8_t t = tag[pidx(g, i, in ? jj : j)];
            if (in && t == TAG_SOLID) best = min(best, abs(d));
        }
        gcol[pidx(g, i, j)] = (int8_t)best;
    }
}

// Row pass of the distance transform: exact layer numbers (Manhattan distance
// to S^{n+1}, up to the layer count) and the lists of the zone nodes of each
// layer, split into NSUB sub-lists by block so that few blocks share a
// counter.  A block counts its nodes per layer in LDS, reserves room in its
// sub-list with one global atomic per layer present, then writes.  The order
// of a list does not matter since targets of one layer are independent.
__global__ __launch_bounds__(256) void k_dt_rows(GridP g, const Win* __restrict__ win, int wslot,
                                                 int8_t* tag, const int8_t* __restrict__ gcol,
                                                 int* lists, int* lcount, unsigned* health)
{
    __shared__ int cnt[MAX_LAYERS + 1];
    __shared__ int base[MAX_LAYERS + 1];
    const Rect W = window_of(win, wslot, g);
    if (!W.ok) return;
    const int L = g.layers;
    const long long cap = sub_cap(g.pplane);
    const int sub = blockIdx.x % NSUB;
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    const long long total = (long long)w * h, stride = (long long)gridDim.x * blockDim.x;
    const long long iters = (total + stride - 1) / stride;
    const int lane = __lane_id();
    for (long long it = 0; it < iters; it++) {
        if (threadIdx.x <= MAX_LAYERS) cnt[threadIdx.x] = 0;
        __syncthreads();
        const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x + it * stride;
        int lay = 0;
        int k = 0;
        if (e < total) {
            const int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
            k = (int)pidx(g, i, j);
            if (tag[k] != TAG_SOLID) {
                int best = 2 * L + 2;
                for (int d = -L; d <= L; d++) {
                    const int ii = i + d;
                    const bool in = ii >= W.i0 && ii <= W.i1;
                    const int gv = gcol[pidx(g, in ? ii : i, j)];
                    if (in) best = min(best, abs(d) + gv);
                }
                if (best <= L) {
                    tag[k] = (int8_t)best;
                    lay = best;
                }
            }
        }
        // slot inside the block: one LDS atomic per wave and layer present
        int slot = 0;
        for (int l = 1; l <= L; l++) {
            const unsigned long long mask = __ballot(lay == l);
            if (mask == 0ull) continue;
            const int leader = __ffsll((long long)mask) - 1;
            int wb = 0;
            if (lane == leader) wb = atomicAdd(&cnt[l], __popcll(mask));
            wb = __shfl(wb, leader);
            if (lay == l) slot = wb + __popcll(mask & ((1ull << lane) - 1ull));
        }
        __syncthreads();
        if (threadIdx.x >= 1 && threadIdx.x <= L && cnt[threadIdx.x] > 0)
            base[threadIdx.x] =
                atomicAdd(&lcount[(threadIdx.x * NSUB + sub) * LCOUNT_PAD], cnt[threadIdx.x]);
        __syncthreads();
        if (lay > 0) {
            const long long at = (long long)base[lay] + slot;
            if (at < cap) lists[(lay * NSUB + sub) * cap + at] = k;
            else atomicAdd(&health[7], 1u);  // cannot happen: see sub_cap
        }
    }
}

hipError_t launch_layers(const GridP& g, const BandBufs& bb, int wslot, hipStream_t st)
{
    k_dt_cols<<<DT_BLOCKS, 256, 0, st>>>(g, bb.win, wslot, bb.tag, bb.gcol, bb.lcount);
    k_dt_rows<<<DT_BLOCKS, 256, 0, st>>>(g, bb.win, wslot, bb.tag, bb.gcol, bb.lists, bb.lcount,
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

struct Fit {
    double M00, M01, M02, M11, M12, M22, bX0, bX1, bX2, bY0, bY1, bY2;
    __device__ __forceinline__ void zero()
    {
        M00 = M01 = M02 = M11 = M12 = M22 = 0.0;
        bX0 = bX1 = bX2 = bY0 = bY1 = bY2 = 0.0;
    }
    // one valid node at offset (a, b) from the target, weight of Eq. (3_2_extrap_weight)
    __device__ __forceinline__ void add(int a, int b, bool use_n, double nxh, double nyh,
                                        double xv, double yv)
    {
        double wt = ldexp(1.0, -(abs(a) + abs(b)));
        if (use_n) {
            const double ddx = -(double)a, ddy = -(double)b;  // d = x_target - x_valid
            const double dn = (ddx * nxh + ddy * nyh) / sqrt(ddx * ddx + ddy * ddy);
            wt = dn * wt > 0.0 ? dn * wt : 0.0;
        }
        const double dx = a, dy = b;
        M00 += wt * dx * dx;
        M01 += wt * dx * dy;
        M02 += wt * dx;
        M11 += wt * dy * dy;
        M12 += wt * dy;
        M22 += wt;
        bX0 += wt * dx * xv;
        bX1 += wt * dy * xv;
        bX2 += wt * xv;
        bY0 += wt * dx * yv;
        bY1 += wt * dy * yv;
        bY2 += wt * yv;
    }
    // intercept of the weighted linear fit, if well posed
    __device__ __forceinline__ bool solve(double det_rel, double& x, double& y) const
    {
        const double det = det3(M00, M01, M02, M01, M11, M12, M02, M12, M22);
        if (!(det > det_rel * M22 * M22 * M22)) return false;
        x = det3(M00, M01, bX0, M01, M11, bX1, M02, M12, bX2) / det;
        y = det3(M00, M01, bY0, M01, M11, bY1, M02, M12, bY2) / det;
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

// Sec. 3.2 steps (i)-(iii) for target (i, j) of layer l from global memory:
// scan windows of half-width r = r0 .. r_max, count the valid nodes (solid, or
// set in an earlier layer), fit xi = A x + B y + C by weighted least squares in
// coordinates centred at the target and take C.  Nodes are visited row by row.
__device__ bool extrapolate_global(const GridP& g, const Rect& W, const Rect& D, int l, int i,
                                   int j, int r0, const int8_t* tag, const double* phin,
                                   const double* X1, const double* Y1, double& xo, double& yo)
{
    bool use_n = false;
    double nxh = 0.0, nyh = 0.0;
    if (l <= 2) {
        const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
        double pv[4];
        for (int d = 0; d < 4; d++) {
            const long long kq = ref_index(g, D, i + di[d], j + dj[d]);
            pv[d] = kq >= 0 ? phin[kq] : INFINITY;
        }
        use_n = normal_from(pv[0], pv[1], pv[2], pv[3], nxh, nyh);
    }
    for (int r = r0; r <= g.r_max; r++) {
        int count = 0;
        for (int b = -r; b <= r; b++)
            for (int a = -r; a <= r; a++) {
                int ci = i + a, cj = j + b;
                if (!canon(g, ci, cj) || !W.has(ci, cj)) continue;
                if (tag_valid_before(tag[pidx(g, ci, cj)], l)) count++;
            }
        if (count < 3) continue;
        Fit f;
        f.zero();
        for (int b = -r; b <= r; b++)
            for (int a = -r; a <= r; a++) {
                int ci = i + a, cj = j + b;
                if (!canon(g, ci, cj) || !W.has(ci, cj)) continue;
                const long long k = pidx(g, ci, cj);
                if (!tag_valid_before(tag[k], l)) continue;
                f.add(a, b, use_n, nxh, nyh, X1[k], Y1[k]);
            }
        if (f.solve(g.det_rel, xo, yo)) return true;
    }
    return false;
}

// sum over the FIT_LANES lanes of a group; the butterfly gives every lane the
// same bits since each addition sees the same two operands in either order
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int m = FIT_LANES / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, FIT_LANES);
    return v;
}
__device__ __forceinline__ int group_sum(int v)
{
#pragma unroll
    for (int m = FIT_LANES / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, FIT_LANES);
    return v;
}

// Sums of the normal equations over the nodes of the scan window of
// half-width r (side = 2r + 1) that fall to this lane: window node q goes to
// lane q mod FIT_LANES; each lane issues all its loads before adding.
template <int SIDE>
__device__ __forceinline__ void fit_window(const GridP& g, const Rect& W, int l, int i, int j,
                                           int kt, int side, int sub, bool use_n, double nxh,
                                           double nyh, const int8_t* tag, const double* X1,
                                           const double* Y1, Fit& f, int& count)
{
    constexpr int PER = 4;  // window nodes per lane and pass: 25 of r = 2 in one pass
    if (SIDE > 0) side = SIDE;
    const int r = side / 2, nq = side * side;
    for (int q0 = 0; q0 < nq; q0 += PER * FIT_LANES) {
        long long kk[PER];
        int tk[PER], aa[PER], bb[PER];
        double xv[PER], yv[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int q = q0 + sub + u * FIT_LANES;
            aa[u] = q % side - r;
            bb[u] = q / side - r;
            int ci = i + aa[u], cj = j + bb[u];
            kk[u] = (q < nq && canon(g, ci, cj) && W.has(ci, cj)) ? pidx(g, ci, cj) : -1;
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

// One layer of Sec. 3.2: every target of the layer list is fitted by a group
// of FIT_LANES lanes that share the scan-window nodes; the sums of the normal
// equations are reduced across the group.  Scan windows grow from r = 2 to
// r_max until they hold three valid nodes and a well-posed fit.  Valid nodes
// come only from earlier layers, so targets of one layer never read each other.
__global__ __launch_bounds__(256) void k_layer_fit(GridP g, const Win* __restrict__ win,
                                                   int wcur, int wprev, int l, int8_t* tag,
                                                   const int* __restrict__ lists,
                                                   const int* __restrict__ lcount,
                                                   const double* __restrict__ phin, double* X1,
                                                   double* Y1, unsigned* health)
{
    const long long cap = sub_cap(g.pplane);
    int ns[NSUB], n = 0;
#pragma unroll
    for (int s = 0; s < NSUB; s++) {
        ns[s] = (int)min((long long)lcount[(l * NSUB + s) * LCOUNT_PAD], cap);
        n += ns[s];
    }
    const int sub = threadIdx.x % FIT_LANES;
    const int g0 = (blockIdx.x * blockDim.x + threadIdx.x) / FIT_LANES;
    const int gstride = gridDim.x * blockDim.x / FIT_LANES;
    if (g0 >= n) return;  // whole groups leave together
    const Rect W = window_of(win, wcur, g);
    if (!W.ok) return;
    const Rect D = window_of(win, wprev, g);
    // all lanes of a group run the same trip counts, so shuffles see full groups
    for (int t = g0; t < n; t += gstride) {
        // position t of the concatenated sub-lists
        int s = 0, at = t;
#pragma unroll
        for (int u = 0; u < NSUB - 1; u++)
            if (s == u && at >= ns[u]) {
                at -= ns[u];
                s = u + 1;
            }
        const int kt = lists[(l * NSUB + s) * cap + at];
        const int i = kt % g.pp - PAD, j = kt / g.pp - PAD;
        // outward normal of phi^n at the target (layers 1, 2): lanes 0..3
        // load the four neighbours
        double nxh = 0.0, nyh = 0.0;
        bool use_n = false;
        if (l <= 2) {
            double p = INFINITY;
            if (sub < 4) {
                const int di = sub == 0 ? 1 : sub == 1 ? -1 : 0;
                const int dj = sub == 2 ? 1 : sub == 3 ? -1 : 0;
                const long long kq = ref_index(g, D, i + di, j + dj);
                if (kq >= 0) p = phin[kq];
            }
            const double pe = __shfl(p, 0, FIT_LANES), pw = __shfl(p, 1, FIT_LANES);
            const double pn = __shfl(p, 2, FIT_LANES), ps = __shfl(p, 3, FIT_LANES);
            use_n = normal_from(pe, pw, pn, ps, nxh, nyh);
        }
        bool done = false;
        double xo = 0.0, yo = 0.0;
        for (int r = 2; r <= g.r_max && !done; r++) {
            Fit f;
            f.zero();
            int count = 0;
            if (r == 2)
                fit_window<5>(g, W, l, i, j, kt, 5, sub, use_n, nxh, nyh, tag, X1, Y1, f, count);
            else
                fit_window<0>(g, W, l, i, j, kt, 2 * r + 1, sub, use_n, nxh, nyh, tag, X1, Y1, f,
                              count);
            count = group_sum(count);
            if (count < 3) continue;
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
            done = f.solve(g.det_rel, xo, yo);
        }
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

hipError_t launch_extrapolate(const GridP& g, const BandBufs& bb, const StepSlots& s,
                              hipStream_t st)
{
    for (int l = 1; l <= g.layers; l++)
        k_layer_fit<<<FIT_BLOCKS, 256, 0, st>>>(g, bb.win, s.wcur, s.wprev, l, bb.tag,
                                                bb.lists, bb.lcount,
                                                bb.phi[s.cur], bb.X[s.nxt], bb.Y[s.nxt],
                                                bb.health);
    return hipGetLastError();
}

// ---------------------------------------------------------------- relabel

// phi^{n+1} = phi0(xi^{n+1}) on every node holding a reference map (Alg. 1);
// one partial box of the new interior solid set per block (reduced by the
// force kernel into the next ring slot)
__global__ __launch_bounds__(256) void k_relabel(GridP g, BodyP b, const int8_t* __restrict__ tag,
                                                 const Win* __restrict__ win, int wcur,
                                                 double* X1, double* Y1, double* phi1,
                                                 int* boxpart)
{
    const Rect W = window_of(win, wcur, g);
    int i0 = 0x3fffffff, i1 = -0x3fffffff, j0 = 0x3fffffff, j1 = -0x3fffffff;
    if (W.ok) {
        const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
        const long long total = (long long)w * h;
        for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
             e += (long long)gridDim.x * blockDim.x) {
            const int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
            const long long k = pidx(g, i, j);
            const int8_t tv = tag[k];
            const double xv = X1[k], yv = Y1[k];
            if (tag_set(tv)) {
                const double p = shape_phi(b, xv, yv);
                phi1[k] = p;
                if (p < 0.0 && i >= 0 && i < g.nx && j >= 0 && j < g.ny) {
                    i0 = min(i0, i);
                    i1 = max(i1, i);
                    j0 = min(j0, j);
                    j1 = max(j1, j);
                }
            } else {
                phi1[k] = INFINITY;
                X1[k] = NAN;
                Y1[k] = NAN;
            }
        }
    }
    block_box(i0, i1, j0, j1, boxpart + 4 * blockIdx.x);
}

hipError_t launch_relabel(const GridP& g, const BodyP& b, const BandBufs& bb, const StepSlots& s,
                          hipStream_t st)
{
    k_relabel<<<RELABEL_BLOCKS, 256, 0, st>>>(g, b, bb.tag, bb.win, s.wcur, bb.X[s.nxt],
                                              bb.Y[s.nxt], bb.phi[s.nxt], bb.boxpart);
    return hipGetLastError();
}

// ---------------------------------------------------------------- stress and force

constexpr int FTX = 32, FTY = 8;
constexpr int SX = FTX + 2, SY = FTY + 2;

// Blended stress (1 - H(phi_e)) tau_s of one half-edge from the LDS tile.
// a, bb: the two nodes of the edge (a before bb along the normal direction);
// s1..s4: the side nodes of the tangential difference (s1 + s2 - s3 - s4)/4
// (Eq. (3_3_refmap_jacobian), six-node stencil); dir 0: x-edge, 1: y-edge.
__device__ void edge_tau(const GridP& g, const BodyP& b, const double* sX, const double* sY,
                         const double* sP, int a, int bb, int s1, int s2, int s3, int s4, int dir,
                         bool count, unsigned* health, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    const double pa = sP[a], pb = sP[bb];
    if (!(pa < INFINITY) || !(pb < INFINITY)) return;
    const double phie = 0.5 * (pa + pb);
    const double lam = 1.0 - heaviside(phie, g.eps);
    if (!(lam > 0.0)) return;
    if (!(sP[s1] < INFINITY) || !(sP[s2] < INFINITY) || !(sP[s3] < INFINITY) ||
        !(sP[s4] < INFINITY)) {
        if (count) atomicAdd(&health[2], 1u);
        return;
    }
    const double nX = sX[bb] - sX[a], nY = sY[bb] - sY[a];
    const double tX = (sX[s1] + sX[s2] - sX[s3] - sX[s4]) / 4.0;
    const double tY = (sY[s1] + sY[s2] - sY[s3] - sY[s4]) / 4.0;
    double J0, J1, J2, J3;  // [dX/dx, dX/dy; dY/dx, dY/dy]
    if (dir == 0) {
        J0 = nX; J1 = tX; J2 = nY; J3 = tY;
    } else {
        J0 = tX; J1 = nX; J2 = tY; J3 = nY;
    }
    const double det = J0 * J3 - J1 * J2;
    if (!(det > g.detJ_min)) {
        if (count) {
            atomicAdd(&health[3], 1u);
            if (lam > 0.5) atomicAdd(&health[4], 1u);
        }
        return;
    }
    // F = J^{-1} (Eq. (3_3_refmap_deformation)); plane-strain neo-Hookean
    // deviatoric stress (Eq. (3_3_solid_stress))
    const double F00 = J3 / det, F01 = -J1 / det;
    const double F10 = -J2 / det, F11 = J0 / det;
    const double Bxx = F00 * F00 + F01 * F01;
    const double Bxy = F00 * F10 + F01 * F11;
    const double Byy = F10 * F10 + F11 * F11;
    const double tr = Bxx + Byy;
    out[0] = lam * (b.G * (Bxx - (tr + 1.0) / 3.0));
    out[1] = lam * (b.G * Bxy);
    out[2] = lam * (b.G * (Byy - (tr + 1.0) / 3.0));
}

// Shared body of the force kernel (MODE 0) and the stress read (MODE 1) over
// interior tiles of region Rg: stage xi, phi of the tile plus a one-node halo
// in LDS (all loads issued first), compute each half-edge once, then combine
// per node.  In MODE 0, block 0 also reduces relabel's partial boxes into the
// next ring slot.
template <int MODE>
__global__ __launch_bounds__(256) void k_edges(GridP g, BodyP b, Win* win, int wvalid, int wnext,
                                               const int* __restrict__ boxpart, int nbox,
                                               int whole_grid, const double* __restrict__ X,
                                               const double* __restrict__ Y,
                                               const double* __restrict__ phi, double* o0,
                                               double* o1, double* o2, unsigned* health)
{
    __shared__ double sX[SY * SX], sY[SY * SX], sP[SY * SX];
    __shared__ double ex[FTY][FTX + 1][3];
    __shared__ double ey[FTY + 1][FTX][3];
    const Rect V = window_of(win, wvalid, g);
    if (MODE == 0 && blockIdx.x == 0) reduce_boxes(boxpart, nbox, &win[wnext], nullptr);
    Rect Rg;
    if (whole_grid) {
        Rg.i0 = 0; Rg.i1 = g.nx - 1; Rg.j0 = 0; Rg.j1 = g.ny - 1;
        Rg.ok = true;
    } else {
        Rg = V;
        if (!Rg.ok) return;
        Rg.i0 = max(Rg.i0, 0);
        Rg.j0 = max(Rg.j0, 0);
        Rg.i1 = min(Rg.i1, g.nx - 1);
        Rg.j1 = min(Rg.j1, g.ny - 1);
        if (Rg.i0 > Rg.i1 || Rg.j0 > Rg.j1) return;
    }
    const int ntx = (Rg.i1 - Rg.i0) / FTX + 1, nty = (Rg.j1 - Rg.j0) / FTY + 1;
    const int tx = threadIdx.x % FTX, ty = threadIdx.x / FTX;
    for (int t = blockIdx.x; t < ntx * nty; t += gridDim.x) {
        const int i0 = Rg.i0 + (t % ntx) * FTX, j0 = Rg.j0 + (t / ntx) * FTY;
        for (int e = threadIdx.x; e < SX * SY; e += blockDim.x) {
            int ci = i0 - 1 + e % SX, cj = j0 - 1 + e / SX;
            const bool in = b.present && canon(g, ci, cj) && V.has(ci, cj);
            const long long k = in ? pidx(g, ci, cj) : 0;
            const double p = phi[k], xv = X[k], yv = Y[k];
            const bool set = in && p < INFINITY;
            sX[e] = set ? xv : NAN;
            sY[e] = set ? yv : NAN;
            sP[e] = set ? p : INFINITY;
        }
        __syncthreads();
        const int i = i0 + tx, j = j0 + ty;
        const bool mine = i <= Rg.i1 && j <= Rg.j1;
        // health counting: an edge is counted once, by the node on its far
        // side, or by its near node when the far node lies outside the region
        const bool rowin = j <= Rg.j1, colin = i <= Rg.i1;
        const bool cnt_l = MODE == 0 && (mine || (rowin && i == Rg.i1 + 1));
        const bool cnt_b = MODE == 0 && (mine || (colin && j == Rg.j1 + 1));
        // local index of node (i + di, j + dj)
#define LI(di, dj) ((ty + 1 + (dj)) * SX + (tx + 1 + (di)))
        // x-edge (i - 1/2, j): a = (i-1, j), b = (i, j); side (i, j+1), (i-1, j+1), (i, j-1), (i-1, j-1)
        edge_tau(g, b, sX, sY, sP, LI(-1, 0), LI(0, 0), LI(0, 1), LI(-1, 1), LI(0, -1), LI(-1, -1),
                 0, cnt_l, health, ex[ty][tx]);
        // y-edge (i, j - 1/2): a = (i, j-1), b = (i, j); side (i+1, j), (i+1, j-1), (i-1, j), (i-1, j-1)
        edge_tau(g, b, sX, sY, sP, LI(0, -1), LI(0, 0), LI(1, 0), LI(1, -1), LI(-1, 0), LI(-1, -1),
                 1, cnt_b, health, ey[ty][tx]);
        if (tx == FTX - 1) {
            // right x-edge (i + 1/2, j) of the last tile column
            edge_tau(g, b, sX, sY, sP, LI(0, 0), LI(1, 0), LI(1, 1), LI(0, 1), LI(1, -1), LI(0, -1),
                     0, MODE == 0 && mine && i == Rg.i1, health, ex[ty][tx + 1]);
        }
        if (ty == FTY - 1) {
            // top y-edge (i, j + 1/2) of the last tile row
            edge_tau(g, b, sX, sY, sP, LI(0, 0), LI(0, 1), LI(1, 1), LI(1, 0), LI(-1, 1), LI(-1, 0),
                     1, MODE == 0 && mine && j == Rg.j1, health, ey[ty + 1][tx]);
        }
#undef LI
        __syncthreads();
        if (mine) {
            const double* L = ex[ty][tx];
            const double* Rr = ex[ty][tx + 1];
            const double* B = ey[ty][tx];
            const double* T = ey[ty + 1][tx];
            const long long n = (long long)j * g.pitch + i;
            if (MODE == 0) {
                // Eq. (3_3_div_solid_stress) in Eq. (2_4_F_divs)
                double fx = (Rr[0] - L[0]) + (T[1] - B[1]);
                double fy = (Rr[1] - L[1]) + (T[2] - B[2]);
                const double p = sP[(ty + 1) * SX + tx + 1];
                double H = 1.0, dr = 0.0;
                if (b.present && p < INFINITY) {
                    H = heaviside(p, g.eps);
                    fx += (1.0 - H) * (b.rho_s - g.rho_f) * g.gx;
                    fy += (1.0 - H) * (b.rho_s - g.rho_f) * g.gy;
                    dr = (1.0 - H) * (b.rho_s - g.rho_f);  // Eq. (2_3_drho)
                }
                fx += H * g.fext_x;
                fy += H * g.fext_y;
                o0[n] = fx;
                o1[n] = fy;
                o2[n] = dr;
            } else {
                const long long e = (long long)j * g.nx + i;
                o0[e] = (L[0] + Rr[0] + B[0] + T[0]) / 4.0;
                o1[e] = (L[1] + Rr[1] + B[1] + T[1]) / 4.0;
                o2[e] = (L[2] + Rr[2] + B[2] + T[2]) / 4.0;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_force(const GridP& g, const BodyP& b, const BandBufs& bb, const StepSlots& s,
                        double* fx, double* fy, double* drho, hipStream_t st)
{
    k_edges<0><<<2048, 256, 0, st>>>(g, b, bb.win, s.wcur, s.wnext, bb.boxpart, RELABEL_BLOCKS,
                                     0, bb.X[s.nxt], bb.Y[s.nxt], bb.phi[s.nxt], fx, fy, drho,
                                     bb.health);
    return hipGetLastError();
}

hipError_t launch_read_stress(const GridP& g, const BodyP& b, const BandBufs& bb, int buf,
                              int wvalid, double* sxx, double* sxy, double* syy, hipStream_t st)
{
    k_edges<1><<<2048, 256, 0, st>>>(g, b, bb.win, wvalid, 0, nullptr, 0, 1, bb.X[buf],
                                     bb.Y[buf], bb.phi[buf], sxx, sxy, syy, bb.health);
    return hipGetLastError();
}

// ---------------------------------------------------------------- reads

__global__ void k_read_refmap(GridP g, const Win* __restrict__ win, int wvalid,
                              const double* __restrict__ X, const double* __restrict__ Y,
                              const double* __restrict__ phi, double* Xo, double* Yo,
                              double* Po)
{
    const Rect V = window_of(win, wvalid, g);
    const long long N = (long long)g.nx * g.ny;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        double xv = NAN, yv = NAN, pv = NAN;
        if (V.has(i, j)) {
            const long long k = pidx(g, i, j);
            if (phi[k] < INFINITY) {
                xv = X[k];
                yv = Y[k];
                pv = phi[k];
            }
        }
        if (Xo) Xo[e] = xv;
        if (Yo) Yo[e] = yv;
        if (Po) Po[e] = pv;
    }
}

hipError_t launch_read_refmap(const GridP& g, const BandBufs& bb, int buf, int wvalid, double* X,
                              double* Y, double* phi, hipStream_t st)
{
    k_read_refmap<<<2048, 256, 0, st>>>(g, bb.win, wvalid, bb.X[buf], bb.Y[buf], bb.phi[buf], X,
                                        Y, phi);
    return hipGetLastError();
}

}  // namespace lbrmt
