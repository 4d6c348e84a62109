// Discrete adjoint of one coupled step (FP64, one solid): the exact reverse
// of the forward step of k_band.hip and k_lb.hip, with every discrete
// decision (solid set, layers, scan-window size, upwind side, stencil and
// singular-J fallbacks) taken as the forward step took it.  One step n of
// Alg. 1 is, in forward order: moments u^n (with half of F^{n-1}),
// advection of xi on S^n (Eq. (3_1_refmap_adv)), layer-by-layer weighted
// least-squares extrapolation (Sec. 3.2), relabel phi^{n+1} = phi0(xi^{n+1}),
// half-edge stresses and their divergence F^n (Eqs. (3_3_refmap_jacobian) to
// (3_3_div_solid_stress), (2_4_F_divs)), collision with the SFC equilibrium
// and Guo forcing (Eqs. (2_3_feq_sfc), (2_2_Fi)), streaming with bounce-back
// and the moving lid (Sec. 3.5).  The kernels below run them backwards.
//
// Adjoint fields: fbar (natural populations f_i(x), [9][ny][nx]), xbar, ybar
// and pbar (xi and phi on the padded reference-map grid), Fbar (force planes,
// [ny][nx]); scalar adjoints of G and of the lid speed accumulate in acc[0],
// acc[1].  Scatters that several threads share use double atomics.
#include <hip/hip_runtime.h>

#include "lbrmt_internal.h"

namespace lbrmt {

namespace {

constexpr double AW0 = 4.0 / 9.0, AW1 = 1.0 / 9.0, AW2 = 1.0 / 36.0;
__constant__ int ACX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int ACY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ int AOPP[NQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__constant__ double AWQ[NQ] = {AW0, AW1, AW1, AW1, AW1, AW2, AW2, AW2, AW2};

// smoothed Heaviside of Eq. (2_3_heaviside) and its derivative
__device__ __forceinline__ double hv(double p, double eps)
{
    if (p <= -eps) return 0.0;
    if (p >= eps) return 1.0;
    return 0.5 * (1.0 + p / eps + sin(M_PI * p / eps) / M_PI);
}
__device__ __forceinline__ double dhv(double p, double eps)
{
    if (p <= -eps || p >= eps) return 0.0;
    return 0.5 / eps * (1.0 + cos(M_PI * p / eps));
}

// gradient of the reference level set phi0 at reference point (X, Y)
__device__ void grad_phi0(const BodyP& b, double X, double Y, double& gx, double& gy)
{
    const double dx = X - b.cx, dy = Y - b.cy;
    const double d = sqrt(dx * dx + dy * dy);
    gx = gy = 0.0;
    if (!(d > 0.0)) return;
    if (b.shape != 1) {
        gx = dx / d;
        gy = dy / d;
        return;
    }
    // phi0 = d (1 - 1/q), q = |(x'/a, y'/b)| in the body frame
    const double xp = b.ct * dx + b.st * dy, yp = -b.st * dx + b.ct * dy;
    const double ua = xp / (b.R * b.R), ub = yp / (b.Rb * b.Rb);
    const double q = sqrt((xp / b.R) * (xp / b.R) + (yp / b.Rb) * (yp / b.Rb));
    const double dqx = (ua * b.ct - ub * b.st) / q, dqy = (ua * b.st + ub * b.ct) / q;
    gx = dx / d * (1.0 - 1.0 / q) + d * dqx / (q * q);
    gy = dy / d * (1.0 - 1.0 / q) + d * dqy / (q * q);
}

// natural populations f_i(x) of the pull-stored lattice A (bounce-back at walls)
__device__ __forceinline__ void nat_gather(const GridP& g, const double* __restrict__ A, int i,
                                           int j, double f[NQ])
{
    const long long P = g.plane;
    const long long n = (long long)j * g.pitch + i;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        int si = i - ACX[q], sj = j - ACY[q];
        if (g.px) si = wrap_axis(si, g.nx);
        if (g.py) sj = wrap_axis(sj, g.ny);
        const bool in = si >= 0 && si < g.nx && sj >= 0 && sj < g.ny;
        f[q] = in ? A[q * P + (long long)sj * g.pitch + si] : A[AOPP[q] * P + n];
    }
}

__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x + 63) / 64; k++) s += red[k];
    __syncthreads();
    return s;
}

}  // namespace

// ---------------------------------------------------------------- lattice
// Streaming, lid, collision and moments backwards, one node per thread:
// fbar_out = dL/df^n (natural), Fpbar = dL/dF^{n-1} (this part), Fcbar +=
// the Guo part of dL/dF^n, pbar1 += the density-excess part of dL/dphi^{n+1}.
__global__ __launch_bounds__(256) void k_adj_lattice(GridP g, BodyP b, AdjSnap s, AdjBufs a)
{
    const long long N = (long long)g.nx * g.ny;
    const Rect wp = window_of(s.win, 0, g);
    const Rect wc = window_of(s.win, 1, g);
    const double om = g.omega, cf = g.cforce;
    double ubar_lid = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        const long long n = (long long)j * g.pitch + i;
        double f[NQ];
        nat_gather(g, s.A, i, j, f);
        double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            rho += f[q];
            jx += ACX[q] * f[q];
            jy += ACY[q] * f[q];
        }
        const bool inp = wp.has(i, j), inc = wc.has(i, j);
        const double Fpx = inp ? s.fpx[n] : s.fpo[0], Fpy = inp ? s.fpy[n] : s.fpo[1];
        const double Fx = inc ? s.fcx[n] : g.fext_x, Fy = inc ? s.fcy[n] : g.fext_y;
        const double ux = (jx + 0.5 * Fpx) / rho, uy = (jy + 0.5 * Fpy) / rho;
        double p1 = INFINITY;
        if (b.present && inc) p1 = s.P1[pidx(g, i, j)];
        const double drs = b.present ? b.rho_s - g.rho_f : 0.0;
        // adjoint of the post-collision values: where each one streams to
        const bool top = !g.py && j == g.ny - 1;
        double gq[NQ];
        double rhobar = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            int di = i + ACX[q], dj = j + ACY[q];
            if (g.px) di = wrap_axis(di, g.nx);
            if (g.py) dj = wrap_axis(dj, g.ny);
            const bool in = di >= 0 && di < g.nx && dj >= 0 && dj < g.ny;
            gq[q] = in ? a.fb_in[q * N + (long long)dj * g.nx + di] : a.fb_in[AOPP[q] * N + e];
            if (top && (q == 5 || q == 6)) {
                // f_opp(q)(x) = fhat_q(x) -/+ rho U / 6 through the lid (Sec. 3.5)
                const double sg = q == 5 ? -1.0 : 1.0;
                const double fo = a.fb_in[AOPP[q] * N + e];
                if (!g.lid_rho_mode) rhobar += fo * sg * g.lid_ux / 6.0;
                ubar_lid += fo * sg * (g.lid_rho_mode ? g.rho_f : rho) / 6.0;
            }
        }
        // collision: fhat_q = f_q + om (feq_q - f_q) + cf Fi_q
        const double usq = ux * ux + uy * uy, uF = ux * Fx + uy * Fy;
        double uxb = 0.0, uyb = 0.0, drb = 0.0, Fxb = 0.0, Fyb = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const double eb = om * gq[q], Fib = cf * gq[q], w = AWQ[q];
            const double cx = ACX[q], cy = ACY[q];
            const double cu = cx * ux + cy * uy, cF = cx * Fx + cy * Fy;
            if (q == 0) {
                rhobar += eb * w * (1.0 - 1.5 * usq);
                uxb += eb * w * rho * (-3.0 * ux);
                uyb += eb * w * rho * (-3.0 * uy);
                drb += eb * (5.0 / 9.0);
                uxb += Fib * w * (-3.0 * Fx);
                uyb += Fib * w * (-3.0 * Fy);
                Fxb += Fib * w * (-3.0 * ux);
                Fyb += Fib * w * (-3.0 * uy);
            } else {
                rhobar += eb * w * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                uxb += eb * w * rho * (3.0 * cx + 9.0 * cu * cx - 3.0 * ux);
                uyb += eb * w * rho * (3.0 * cy + 9.0 * cu * cy - 3.0 * uy);
                drb += eb * (-w);
                uxb += Fib * w * (-3.0 * Fx + 9.0 * cF * cx);
                uyb += Fib * w * (-3.0 * Fy + 9.0 * cF * cy);
                Fxb += Fib * w * (3.0 * (cx - ux) + 9.0 * cu * cx);
                Fyb += Fib * w * (3.0 * (cy - uy) + 9.0 * cu * cy);
            }
        }
        // u = (j + F^{n-1} / 2) / rho
        const double jxb = uxb / rho, jyb = uyb / rho;
        rhobar += -(uxb * ux + uyb * uy) / rho;
#pragma unroll
        for (int q = 0; q < NQ; q++)
            a.fb_out[q * N + e] = (1.0 - om) * gq[q] + rhobar + ACX[q] * jxb + ACY[q] * jyb;
        a.Fpbar_x[e] = inp ? 0.5 * jxb : 0.0;
        a.Fpbar_y[e] = inp ? 0.5 * jyb : 0.0;
        if (inc) {
            a.Fcbar_x[e] += Fxb;
            a.Fcbar_y[e] += Fyb;
            // density excess (1 - H(phi^{n+1})) (rho_s - rho_f), Eq. (2_3_drho)
            if (p1 < INFINITY) a.pbar1[pidx(g, i, j)] += drb * (-dhv(p1, g.eps)) * drs;
        }
    }
    const double t = block_sum(ubar_lid);
    if (threadIdx.x == 0 && t != 0.0) atomicAdd(&a.acc[1], t);
}

// ---------------------------------------------------------------- force
// Half-edge stresses backwards: edge e (x-edge between a = (i-1, j) and
// b = (i, j), y-edge between a = (i, j-1) and b) enters F(b) with a minus
// sign and F(a) with a plus sign.  dL/d(tau_e) -> lambda_e (phi^{n+1} at a
// and b), J_e (xi^{n+1} at the six stencil nodes) and G.  Also the buoyancy
// and fluid-force terms of F at each interior node.
__device__ void adj_edge(const GridP& g, const BodyP& b, const AdjSnap& s, const AdjBufs& a,
                         const Rect& V, const Rect& wc, int i, int j, int dir, double& Gbar)
{
    const int ia = dir == 0 ? i - 1 : i, ja = dir == 0 ? j : j - 1;
    auto fbar = [&](int x, int y, double& fx, double& fy) {
        fx = fy = 0.0;
        if (g.px) x = wrap_axis(x, g.nx);
        if (g.py) y = wrap_axis(y, g.ny);
        if (x < 0 || x >= g.nx || y < 0 || y >= g.ny || !wc.has(x, y)) return;
        fx = a.Fcbar_x[(long long)y * g.nx + x];
        fy = a.Fcbar_y[(long long)y * g.nx + x];
    };
    double fax, fay, fbx, fby;
    fbar(ia, ja, fax, fay);
    fbar(i, j, fbx, fby);
    // dL/d(tau_xx, tau_xy, tau_yy) of this edge
    double tb0, tb1, tb2;
    if (dir == 0) {
        tb0 = fax - fbx;
        tb1 = fay - fby;
        tb2 = 0.0;
    } else {
        tb0 = 0.0;
        tb1 = fax - fbx;
        tb2 = fay - fby;
    }
    if (tb0 == 0.0 && tb1 == 0.0 && tb2 == 0.0) return;
    // the six stencil nodes a, b, s1..s4 (as in the forward force pass)
    int ci[6], cj[6];
    ci[0] = ia; cj[0] = ja;
    ci[1] = i; cj[1] = j;
    if (dir == 0) {
        ci[2] = i; cj[2] = j + 1;
        ci[3] = i - 1; cj[3] = j + 1;
        ci[4] = i; cj[4] = j - 1;
        ci[5] = i - 1; cj[5] = j - 1;
    } else {
        ci[2] = i + 1; cj[2] = j;
        ci[3] = i + 1; cj[3] = j - 1;
        ci[4] = i - 1; cj[4] = j;
        ci[5] = i - 1; cj[5] = j - 1;
    }
    long long k[6];
    double X[6], Y[6], P[6];
    for (int t = 0; t < 6; t++) {
        int x = ci[t], y = cj[t];
        const bool in = canon(g, x, y) && V.has(x, y);
        k[t] = in ? pidx(g, x, y) : -1;
        P[t] = in ? s.P1[k[t]] : INFINITY;
        X[t] = in ? s.X1[k[t]] : 0.0;
        Y[t] = in ? s.Y1[k[t]] : 0.0;
    }
    if (!(P[0] < INFINITY) || !(P[1] < INFINITY)) return;
    const double pe = 0.5 * (P[0] + P[1]);
    const double lam = 1.0 - hv(pe, g.eps);
    if (!(lam > 0.0)) return;
    for (int t = 2; t < 6; t++)
        if (!(P[t] < INFINITY)) return;
    const double nX = X[1] - X[0], nY = Y[1] - Y[0];
    const double tX = (X[2] + X[3] - X[4] - X[5]) / 4.0;
    const double tY = (Y[2] + Y[3] - Y[4] - Y[5]) / 4.0;
    double J0, J1, J2, J3;
    if (dir == 0) {
        J0 = nX; J1 = tX; J2 = nY; J3 = tY;
    } else {
        J0 = tX; J1 = nX; J2 = tY; J3 = nY;
    }
    const double det = J0 * J3 - J1 * J2;
    if (!(det > g.detJ_min)) return;
    const double F00 = J3 / det, F01 = -J1 / det, F10 = -J2 / det, F11 = J0 / det;
    const double Bxx = F00 * F00 + F01 * F01, Bxy = F00 * F10 + F01 * F11;
    const double Byy = F10 * F10 + F11 * F11, tr = Bxx + Byy;
    // deviatoric parts per unit G, Eq. (3_3_solid_stress)
    const double s0 = Bxx - (tr + 1.0) / 3.0, s1 = Bxy, s2 = Byy - (tr + 1.0) / 3.0;
    const double G = b.G;
    // edge stress = lam G (s0, s1, s2)
    const double lamb = G * (tb0 * s0 + tb1 * s1 + tb2 * s2);
    Gbar += lam * (tb0 * s0 + tb1 * s1 + tb2 * s2);
    const double pb = lamb * (-dhv(pe, g.eps)) * 0.5;
    if (pb != 0.0) {
        atomicAdd(&a.pbar1[k[0]], pb);
        atomicAdd(&a.pbar1[k[1]], pb);
    }
    // B adjoint (tau_s = G (B - (tr B + 1)/3 I))
    const double t0 = lam * G * tb0, t1 = lam * G * tb1, t2 = lam * G * tb2;
    const double Bxxb = t0 * (2.0 / 3.0) - t2 / 3.0, Byyb = t2 * (2.0 / 3.0) - t0 / 3.0;
    const double Bxyb = t1;
    // F adjoint (B = F F^T)
    const double Fb00 = 2.0 * F00 * Bxxb + F10 * Bxyb, Fb01 = 2.0 * F01 * Bxxb + F11 * Bxyb;
    const double Fb10 = F00 * Bxyb + 2.0 * F10 * Byyb, Fb11 = F01 * Bxyb + 2.0 * F11 * Byyb;
    // J adjoint (F = J^{-1}): Jbar = -F^T Fbar F^T
    const double m00 = F00 * Fb00 + F10 * Fb10, m01 = F00 * Fb01 + F10 * Fb11;
    const double m10 = F01 * Fb00 + F11 * Fb10, m11 = F01 * Fb01 + F11 * Fb11;
    const double Jb0 = -(m00 * F00 + m01 * F01), Jb1 = -(m00 * F10 + m01 * F11);
    const double Jb2 = -(m10 * F00 + m11 * F01), Jb3 = -(m10 * F10 + m11 * F11);
    double nXb, tXb, nYb, tYb;
    if (dir == 0) {
        nXb = Jb0; tXb = Jb1; nYb = Jb2; tYb = Jb3;
    } else {
        tXb = Jb0; nXb = Jb1; tYb = Jb2; nYb = Jb3;
    }
    const double cX[6] = {-nXb, nXb, tXb / 4.0, tXb / 4.0, -tXb / 4.0, -tXb / 4.0};
    const double cY[6] = {-nYb, nYb, tYb / 4.0, tYb / 4.0, -tYb / 4.0, -tYb / 4.0};
    for (int t = 0; t < 6; t++) {
        if (cX[t] != 0.0) atomicAdd(&a.xbar1[k[t]], cX[t]);
        if (cY[t] != 0.0) atomicAdd(&a.ybar1[k[t]], cY[t]);
    }
}

__global__ __launch_bounds__(256) void k_adj_force(GridP g, BodyP b, AdjSnap s, AdjBufs a)
{
    const Rect wc = window_of(s.win, 1, g);
    const Rect V = wc;  // the force pass's window: where xi^{n+1}, phi^{n+1} are valid
    double Gbar = 0.0;
    const int ex = g.nx + (g.px ? 0 : 1), ey = g.ny + (g.py ? 0 : 1);
    const long long NE = (long long)ex * ey;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NE;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % ex), j = (int)(e / ex);
        if (b.present) {
            if (j < g.ny) adj_edge(g, b, s, a, V, wc, i, j, 0, Gbar);
            if (i < g.nx) adj_edge(g, b, s, a, V, wc, i, j, 1, Gbar);
        }
        // buoyancy (1 - H)(rho_s - rho_f) g and fluid force H f_ext at node (i, j)
        if (b.present && i < g.nx && j < g.ny && wc.has(i, j)) {
            const long long kk = pidx(g, i, j);
            const double p = s.P1[kk];
            if (p < INFINITY) {
                const long long m = (long long)j * g.nx + i;
                const double fx = a.Fcbar_x[m], fy = a.Fcbar_y[m];
                const double dh = dhv(p, g.eps);
                const double v = (fx * g.gx + fy * g.gy) * (-dh) * (b.rho_s - g.rho_f) +
                                 (fx * g.fext_x + fy * g.fext_y) * dh;
                if (v != 0.0) atomicAdd(&a.pbar1[kk], v);
            }
        }
    }
    const double t = block_sum(Gbar);
    if (threadIdx.x == 0 && t != 0.0) atomicAdd(&a.acc[0], t);
}

// ---------------------------------------------------------------- relabel
// phi^{n+1} = phi0(xi^{n+1}) at every node holding a map: pbar1 -> xbar1,
// then pbar1 is spent (cleared).
__global__ __launch_bounds__(256) void k_adj_relabel(GridP g, BodyP b, AdjSnap s, AdjBufs a)
{
    const Rect V = window_of(s.win, 1, g);
    if (!V.ok) return;
    const int w = V.i1 - V.i0 + 1, h = V.j1 - V.j0 + 1;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)w * h;
         e += (long long)gridDim.x * blockDim.x) {
        int i = V.i0 + (int)(e % w), j = V.j0 + (int)(e / w);
        if (!canon(g, i, j)) continue;
        const long long k = pidx(g, i, j);
        const double pb = a.pbar1[k];
        if (pb == 0.0) continue;
        a.pbar1[k] = 0.0;
        if (!(s.P1[k] < INFINITY)) continue;
        double gx, gy;
        grad_phi0(b, s.X1[k], s.Y1[k], gx, gy);
        a.xbar1[k] += pb * gx;
        a.ybar1[k] += pb * gy;
    }
}

// ---------------------------------------------------------------- extrapolation
// Targets of layer l backwards (one thread per target): the fitted intercept
// c = e3^T M^{-1} b with M = sum w a a^T, b = sum w a xi (a = (dx, dy, 1) in
// target-centred coordinates) sends dL/dc to every valid node k with weight
// w_k (a_k . s), s = M^{-1} e3; with the normal weights of layers 1 and 2 the
// weights themselves depend on phi^n at the target's four neighbours:
// dc/dw_k = (a_k . s)(xi_k - a_k . p), p = M^{-1} b.
__global__ __launch_bounds__(256) void k_adj_fit(GridP g, AdjSnap s, AdjBufs a, int l)
{
    const Rect W = window_of(s.win, 1, g);
    const Rect D = window_of(s.win, 0, g);
    if (!W.ok) return;
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)w * h;
         e += (long long)gridDim.x * blockDim.x) {
        int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
        if (!canon(g, i, j)) continue;
        const long long kt = pidx(g, i, j);
        if (s.tag[kt] != l) continue;  // not this layer, or its fit failed
        const double Xb = a.xbar1[kt], Yb = a.ybar1[kt];
        if (Xb == 0.0 && Yb == 0.0) continue;
        // outward normal of phi^n at the target (layers 1, 2)
        bool use_n = false;
        double nxh = 0.0, nyh = 0.0, gx = 0.0, gy = 0.0, gn = 0.0;
        long long kn[4] = {-1, -1, -1, -1};
        if (l <= 2) {
            const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
            double pv[4];
            bool ok = true;
            for (int q = 0; q < 4; q++) {
                int x = i + di[q], y = j + dj[q];
                kn[q] = (canon(g, x, y) && D.has(x, y)) ? pidx(g, x, y) : -1;
                pv[q] = kn[q] >= 0 ? s.P0[kn[q]] : INFINITY;
                ok = ok && pv[q] < INFINITY;
            }
            if (ok) {
                gx = (pv[0] - pv[1]) / 2.0;
                gy = (pv[2] - pv[3]) / 2.0;
                gn = sqrt(gx * gx + gy * gy);
                if (gn > 0.0) {
                    nxh = gx / gn;
                    nyh = gy / gn;
                    use_n = true;
                }
            }
        }
        for (int r = 2; r <= g.r_max; r++) {
            double M00 = 0, M01 = 0, M02 = 0, M11 = 0, M12 = 0, M22 = 0;
            double bX0 = 0, bX1 = 0, bX2 = 0, bY0 = 0, bY1 = 0, bY2 = 0;
            int count = 0;
            for (int bb = -r; bb <= r; bb++)
                for (int aa = -r; aa <= r; aa++) {
                    int x = i + aa, y = j + bb;
                    if (!canon(g, x, y) || !W.has(x, y)) continue;
                    const long long k = pidx(g, x, y);
                    const int t = s.tag[k];
                    if (!(t == TAG_SOLID || (t > 0 && t < l))) continue;
                    count++;
                    double wt = ldexp(1.0, -(abs(aa) + abs(bb)));
                    if (use_n) {
                        const double ddx = -(double)aa, ddy = -(double)bb;
                        const double dn = (ddx * nxh + ddy * nyh) / sqrt(ddx * ddx + ddy * ddy);
                        wt = dn * wt > 0.0 ? dn * wt : 0.0;
                    }
                    const double dx = aa, dy = bb, xv = s.X1[k], yv = s.Y1[k];
                    M00 += wt * dx * dx; M01 += wt * dx * dy; M02 += wt * dx;
                    M11 += wt * dy * dy; M12 += wt * dy; M22 += wt;
                    bX0 += wt * dx * xv; bX1 += wt * dy * xv; bX2 += wt * xv;
                    bY0 += wt * dx * yv; bY1 += wt * dy * yv; bY2 += wt * yv;
                }
            if (count < 3) continue;
            const double det = M00 * (M11 * M22 - M12 * M12) - M01 * (M01 * M22 - M12 * M02) +
                               M02 * (M01 * M12 - M11 * M02);
            if (!(det > g.det_rel * M22 * M22 * M22)) continue;
            // inverse of the symmetric normal matrix
            const double i00 = (M11 * M22 - M12 * M12) / det, i01 = (M02 * M12 - M01 * M22) / det;
            const double i02 = (M01 * M12 - M11 * M02) / det, i11 = (M00 * M22 - M02 * M02) / det;
            const double i12 = (M01 * M02 - M00 * M12) / det, i22 = (M00 * M11 - M01 * M01) / det;
            // s = M^{-1} e3, plane coefficients p = M^{-1} b
            const double s0 = i02, s1 = i12, s2 = i22;
            const double pX0 = i00 * bX0 + i01 * bX1 + i02 * bX2;
            const double pX1 = i01 * bX0 + i11 * bX1 + i12 * bX2;
            const double pX2 = i02 * bX0 + i12 * bX1 + i22 * bX2;
            const double pY0 = i00 * bY0 + i01 * bY1 + i02 * bY2;
            const double pY1 = i01 * bY0 + i11 * bY1 + i12 * bY2;
            const double pY2 = i02 * bY0 + i12 * bY1 + i22 * bY2;
            double nbx = 0.0, nby = 0.0;  // dL/d(normal)
            for (int bb = -r; bb <= r; bb++)
                for (int aa = -r; aa <= r; aa++) {
                    int x = i + aa, y = j + bb;
                    if (!canon(g, x, y) || !W.has(x, y)) continue;
                    const long long k = pidx(g, x, y);
                    const int t = s.tag[k];
                    if (!(t == TAG_SOLID || (t > 0 && t < l))) continue;
                    const double w0 = ldexp(1.0, -(abs(aa) + abs(bb)));
                    double wt = w0, dn = 0.0, ddx = 0.0, ddy = 0.0, dl = 0.0;
                    if (use_n) {
                        ddx = -(double)aa;
                        ddy = -(double)bb;
                        dl = sqrt(ddx * ddx + ddy * ddy);
                        dn = (ddx * nxh + ddy * nyh) / dl;
                        wt = dn * w0 > 0.0 ? dn * w0 : 0.0;
                    }
                    const double as = s0 * aa + s1 * bb + s2;
                    if (wt != 0.0) {
                        atomicAdd(&a.xbar1[k], Xb * wt * as);
                        atomicAdd(&a.ybar1[k], Yb * wt * as);
                    }
                    if (use_n && dn * w0 > 0.0) {
                        const double rX = s.X1[k] - (pX0 * aa + pX1 * bb + pX2);
                        const double rY = s.Y1[k] - (pY0 * aa + pY1 * bb + pY2);
                        const double wb = as * (Xb * rX + Yb * rY);
                        const double dnb = wb * w0;
                        nbx += dnb * ddx / dl;
                        nby += dnb * ddy / dl;
                    }
                }
            if (use_n && (nbx != 0.0 || nby != 0.0)) {
                // n = g / |g|, g = ((phi_e - phi_w) / 2, (phi_n - phi_s) / 2)
                const double dotp = nbx * nxh + nby * nyh;
                const double gbx = (nbx - dotp * nxh) / gn, gby = (nby - dotp * nyh) / gn;
                atomicAdd(&a.pbar0[kn[0]], gbx / 2.0);
                atomicAdd(&a.pbar0[kn[1]], -gbx / 2.0);
                atomicAdd(&a.pbar0[kn[2]], gby / 2.0);
                atomicAdd(&a.pbar0[kn[3]], -gby / 2.0);
            }
            break;
        }
    }
}

// ---------------------------------------------------------------- advection
// Solid nodes of S^n backwards: xi~ = xi - (u d/dx + v d/dy) xi with the
// upwind side of the forward step.  dL/dxi~ (held in xbar1 at solid nodes) ->
// xbar0 at the node and its stencil nodes, and u^n -> f^n, F^{n-1}.
__global__ __launch_bounds__(256) void k_adj_advect(GridP g, AdjSnap s, AdjBufs a)
{
    const Rect W = window_of(s.win, 1, g);
    const Rect D = window_of(s.win, 0, g);
    if (!W.ok) return;
    const long long N = (long long)g.nx * g.ny;
    const int w = W.i1 - W.i0 + 1, h = W.j1 - W.j0 + 1;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)w * h;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = W.i0 + (int)(e % w), j = W.j0 + (int)(e / w);
        if (i < 0 || i >= g.nx || j < 0 || j >= g.ny) continue;
        const long long k0 = pidx(g, i, j);
        if (s.tag[k0] != TAG_SOLID) continue;
        const double Xb = a.xbar1[k0], Yb = a.ybar1[k0];
        if (Xb == 0.0 && Yb == 0.0) continue;
        // u^n at the node
        double f[NQ];
        nat_gather(g, s.A, i, j, f);
        double rho = 0.0, jx = 0.0, jy = 0.0;
        for (int q = 0; q < NQ; q++) {
            rho += f[q];
            jx += ACX[q] * f[q];
            jy += ACY[q] * f[q];
        }
        const long long n = (long long)j * g.pitch + i;
        const bool inp = D.has(i, j);
        const double Fpx = inp ? s.fpx[n] : s.fpo[0], Fpy = inp ? s.fpy[n] : s.fpo[1];
        const double u = (jx + 0.5 * Fpx) / rho, v = (jy + 0.5 * Fpy) / rho;
        // stencils along x and y, as in the forward step
        auto stencil = [&](int dx, int dy, double vel, long long kk[3], double cf[3], double& dX,
                           double& dY) -> bool {
            kk[0] = k0;
            kk[1] = kk[2] = -1;
            cf[0] = cf[1] = cf[2] = 0.0;
            dX = dY = 0.0;
            if (vel == 0.0) return true;
            const int sg = vel > 0.0 ? 1 : -1;
            for (int t = 1; t <= 2; t++) {
                int x = i - sg * t * dx, y = j - sg * t * dy;
                if (!canon(g, x, y) || !D.has(x, y)) return false;
                kk[t] = pidx(g, x, y);
                if (!(s.P0[kk[t]] < INFINITY)) return false;
            }
            if (sg > 0) {
                cf[0] = 1.5; cf[1] = -2.0; cf[2] = 0.5;
            } else {
                cf[0] = -1.5; cf[1] = 2.0; cf[2] = -0.5;
            }
            for (int t = 0; t < 3; t++) {
                dX += cf[t] * s.X0[kk[t]];
                dY += cf[t] * s.Y0[kk[t]];
            }
            return true;
        };
        long long kx[3], ky[3];
        double cx[3], cy[3], dXx, dYx, dXy, dYy;
        const bool okx = stencil(1, 0, u, kx, cx, dXx, dYx);
        const bool oky = stencil(0, 1, v, ky, cy, dXy, dYy);
        if (!okx || !oky) {
            // the forward step kept xi (missing stencil node)
            atomicAdd(&a.xbar0[k0], Xb);
            atomicAdd(&a.ybar0[k0], Yb);
            continue;
        }
        atomicAdd(&a.xbar0[k0], Xb);
        atomicAdd(&a.ybar0[k0], Yb);
        for (int t = 0; t < 3; t++) {
            if (cx[t] != 0.0) {
                atomicAdd(&a.xbar0[kx[t]], -u * cx[t] * Xb);
                atomicAdd(&a.ybar0[kx[t]], -u * cx[t] * Yb);
            }
            if (cy[t] != 0.0) {
                atomicAdd(&a.xbar0[ky[t]], -v * cy[t] * Xb);
                atomicAdd(&a.ybar0[ky[t]], -v * cy[t] * Yb);
            }
        }
        const double ub = -(dXx * Xb + dYx * Yb), vb = -(dXy * Xb + dYy * Yb);
        // u = (j + F^{n-1} / 2) / rho
        const double jxb = ub / rho, jyb = vb / rho;
        const double rb = -(ub * u + vb * v) / rho;
        const long long m = (long long)j * g.nx + i;
        for (int q = 0; q < NQ; q++) a.fb_out[q * N + m] += rb + ACX[q] * jxb + ACY[q] * jyb;
        if (inp) {
            a.Fpbar_x[m] += 0.5 * jxb;
            a.Fpbar_y[m] += 0.5 * jyb;
        }
    }
}

// ---------------------------------------------------------------- loss
// L_n = (|c - c*|^2 + |d - d*|^2) / T with c = sum lambda x / sum lambda,
// d = sum lambda (x - xi) / sum lambda, lambda = 1 - H(phi): coef = {c_x, c_y,
// d_x, d_y, gc_x, gc_y, gd_x, gd_y} with gc = dL/dc / sum lambda and
// gd = dL/dd / sum lambda.  which = 0: the step's input state (xi^n, phi^n,
// adds to xbar0, pbar0); 1: its output state (xi^{n+1}, phi^{n+1}, adds to
// xbar1, pbar1).
__global__ __launch_bounds__(256) void k_adj_loss(GridP g, BodyP b, AdjSnap s, AdjBufs a,
                                                  int which, LossCoef c)
{
    const Rect V = window_of(s.win, which == 0 ? 0 : 1, g);
    if (!V.ok || !b.present) return;
    const double* X = which == 0 ? s.X0 : s.X1;
    const double* Y = which == 0 ? s.Y0 : s.Y1;
    const double* P = which == 0 ? s.P0 : s.P1;
    double* xb = which == 0 ? a.xbar0 : a.xbar1;
    double* yb = which == 0 ? a.ybar0 : a.ybar1;
    double* pb = which == 0 ? a.pbar0 : a.pbar1;
    const int i0 = max(V.i0, 0), i1 = min(V.i1, g.nx - 1);
    const int j0 = max(V.j0, 0), j1 = min(V.j1, g.ny - 1);
    const int w = i1 - i0 + 1, h = j1 - j0 + 1;
    if (w <= 0 || h <= 0) return;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)w * h;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = i0 + (int)(e % w), j = j0 + (int)(e / w);
        const long long k = pidx(g, i, j);
        const double p = P[k];
        if (!(p < INFINITY)) continue;
        double x = i + 0.5, y = j + 0.5;
        if (g.px) x = b.cx + (x - b.cx) - g.nx * floor((x - b.cx) / g.nx + 0.5);
        if (g.py) y = b.cy + (y - b.cy) - g.ny * floor((y - b.cy) / g.ny + 0.5);
        const double lam = 1.0 - hv(p, g.eps);
        const double dl = c.gc[0] * (x - c.c[0]) + c.gc[1] * (y - c.c[1]) +
                          c.gd[0] * ((x - X[k]) - c.d[0]) + c.gd[1] * ((y - Y[k]) - c.d[1]);
        pb[k] += dl * (-dhv(p, g.eps));
        xb[k] += -c.gd[0] * lam;
        yb[k] += -c.gd[1] * lam;
    }
}

// ---------------------------------------------------------------- initial state
// f^0 = f^eq(rho_0, u_0, drho_0) (natural form): dL/du_0 from dL/df^0.
__global__ __launch_bounds__(256) void k_adj_init(GridP g, BodyP b, AdjSnap s, AdjBufs a,
                                                  double* u0bar)
{
    const long long N = (long long)g.nx * g.ny;
    const Rect D = window_of(s.win, 0, g);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        // rho_0 and u_0 from f^0 itself (its moments are rho_0 and rho_0 u_0)
        double f[NQ];
        nat_gather(g, s.A, i, j, f);
        double rho = 0.0, jx = 0.0, jy = 0.0;
        for (int q = 0; q < NQ; q++) {
            rho += f[q];
            jx += ACX[q] * f[q];
            jy += ACY[q] * f[q];
        }
        (void)D;
        const double ux = jx / rho, uy = jy / rho;
        double bx = 0.0, by = 0.0;
        for (int q = 0; q < NQ; q++) {
            const double cx = ACX[q], cy = ACY[q], cu = cx * ux + cy * uy, fb = a.fb_in[q * N + e];
            bx += fb * AWQ[q] * rho * (3.0 * cx + 9.0 * cu * cx - 3.0 * ux);
            by += fb * AWQ[q] * rho * (3.0 * cy + 9.0 * cu * cy - 3.0 * uy);
        }
        u0bar[e] = bx;
        u0bar[N + e] = by;
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_adjoint_step(const GridP& g, const BodyP& b, const AdjSnap& s,
                               const AdjBufs& a, hipStream_t st)
{
    const long long N = (long long)g.nx * g.ny;
    const int blocks = (int)((N + 255) / 256 < 4096 ? (N + 255) / 256 : 4096);
    k_adj_lattice<<<blocks, 256, 0, st>>>(g, b, s, a);
    k_adj_force<<<blocks, 256, 0, st>>>(g, b, s, a);
    if (b.present) {
        k_adj_relabel<<<blocks, 256, 0, st>>>(g, b, s, a);
        for (int l = g.layers; l >= 1; l--) k_adj_fit<<<blocks, 256, 0, st>>>(g, s, a, l);
        k_adj_advect<<<blocks, 256, 0, st>>>(g, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_loss(const GridP& g, const BodyP& b, const AdjSnap& s,
                               const AdjBufs& a, int which, const LossCoef& c, hipStream_t st)
{
    const long long N = (long long)g.nx * g.ny;
    const int blocks = (int)((N + 255) / 256 < 4096 ? (N + 255) / 256 : 4096);
    k_adj_loss<<<blocks, 256, 0, st>>>(g, b, s, a, which, c);
    return hipGetLastError();
}

hipError_t launch_adjoint_init(const GridP& g, const BodyP& b, const AdjSnap& s,
                               const AdjBufs& a, double* u0bar, hipStream_t st)
{
    const long long N = (long long)g.nx * g.ny;
    const int blocks = (int)((N + 255) / 256 < 4096 ? (N + 255) / 256 : 4096);
    k_adj_init<<<blocks, 256, 0, st>>>(g, b, s, a, u0bar);
    return hipGetLastError();
}

__global__ void k_set2(double* dst, double x, double y)
{
    if (threadIdx.x == 0) {
        dst[0] = x;
        dst[1] = y;
    }
}

hipError_t launch_set2(double* dst, double x, double y, hipStream_t st)
{
    k_set2<<<1, 64, 0, st>>>(dst, x, y);
    return hipGetLastError();
}

}  // namespace lbrmt
