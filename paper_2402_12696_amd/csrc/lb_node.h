// Per-node lattice Boltzmann update of the LBRMT step (Sec. 3.4 collision,
// Sec. 3.5 walls and streaming), shared by the lattice kernels and by the
// force pass, which updates the nodes of the solid's window right after
// computing their force.  The arithmetic is contracted into fused
// multiply-adds within one expression (fp contract "on") in every file that
// includes it, so every kernel rounds a node's update identically.
#pragma once

#include "lbrmt_internal.h"

namespace lbrmt {

template <typename S>
struct Prec;
template <>
struct Prec<double> {
    using C = double;
    static constexpr bool dev = false;
};
template <>
struct Prec<float> {
    using C = float;
    static constexpr bool dev = true;
};

// D2Q9 weights (Table "d2q9")
#define W0 (4.0 / 9.0)
#define W1 (1.0 / 9.0)
#define W2 (1.0 / 36.0)

struct Neigh {
    long long n, rm, r0, rp;  // node index and row offsets of j-1, j, j+1
    int im, ip, i;
    bool bw, be, bs, bn;      // wall beyond the west/east/south/north side
};

__device__ __forceinline__ Neigh neigh(const GridP& g, int i, int j)
{
    Neigh q;
    q.i = i;
    q.bw = !g.px && i == 0;
    q.be = !g.px && i == g.nx - 1;
    q.bs = !g.py && j == 0;
    q.bn = !g.py && j == g.ny - 1;
    int im = i - 1, ip = i + 1, jm = j - 1, jp = j + 1;
    // periodic axes wrap; on walled axes the clamped index is never used for
    // data (the reflected population is taken instead) but keeps every
    // address inside the plane
    im = im < 0 ? (g.px ? g.nx - 1 : 0) : im;
    ip = ip >= g.nx ? (g.px ? 0 : g.nx - 1) : ip;
    jm = jm < 0 ? (g.py ? g.ny - 1 : 0) : jm;
    jp = jp >= g.ny ? (g.py ? 0 : g.ny - 1) : jp;
    q.im = im;
    q.ip = ip;
    q.r0 = (long long)j * g.pitch;
    q.rm = (long long)jm * g.pitch;
    q.rp = (long long)jp * g.pitch;
    q.n = q.r0 + i;
    return q;
}

// gather the nine pre-collision populations f_i^n of one node (stored form)
template <typename S>
__device__ __forceinline__ void gather(const GridP& g, const Neigh& q, const S* __restrict__ A,
                                       typename Prec<S>::C f[NQ])
{
    const long long P = g.plane;
    const long long n = q.n;
    f[0] = A[n];
    f[1] = q.bw ? A[3 * P + n] : A[1 * P + q.r0 + q.im];
    f[2] = q.bs ? A[4 * P + n] : A[2 * P + q.rm + q.i];
    f[3] = q.be ? A[1 * P + n] : A[3 * P + q.r0 + q.ip];
    f[4] = q.bn ? A[2 * P + n] : A[4 * P + q.rp + q.i];
    f[5] = (q.bw || q.bs) ? A[7 * P + n] : A[5 * P + q.rm + q.im];
    f[6] = (q.be || q.bs) ? A[8 * P + n] : A[6 * P + q.rm + q.ip];
    f[7] = (q.be || q.bn) ? A[5 * P + n] : A[7 * P + q.rp + q.ip];
    f[8] = (q.bw || q.bn) ? A[6 * P + n] : A[8 * P + q.rp + q.im];
}

// density and momentum sum_i c_i f_i from the stored form
template <typename C, bool DEV>
__device__ __forceinline__ void moments(const C f[NQ], C rho_f, C& rho, C& drho_n, C& jx, C& jy)
{
#pragma clang fp contract(on)
    C s = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    if (DEV) {
        drho_n = s;
        rho = rho_f + s;
    } else {
        rho = s;
        drho_n = s - rho_f;
    }
    jx = (f[1] + f[5] + f[8]) - (f[3] + f[6] + f[7]);
    jy = (f[2] + f[5] + f[6]) - (f[4] + f[7] + f[8]);
}

// Collision of Sec. 3.4: SFC equilibrium (Eq. (2_3_feq_sfc)), BGK relaxation,
// Guo forcing (Eq. (2_2_Fi), force per unit volume).  f holds the stored form
// (f or f - w rho_f); the same form is returned.
template <typename C, bool DEV>
__device__ __forceinline__ void collide(C f[NQ], C rho, C drho_n, C ux, C uy, C Fx, C Fy,
                                        C dr_sfc, C omega, C cf)
{
#pragma clang fp contract(on)
    const C usq = ux * ux + uy * uy;
    const C uF = ux * Fx + uy * Fy;
    const C base = DEV ? drho_n : rho;  // rho term of w_i rho (1 + ...) in stored form
    const C r15 = C(1.5) * rho * usq;
    // q = 0
    {
        C feq = C(W0) * (base - r15) + C(5.0 / 9.0) * dr_sfc;
        C Fi = C(W0) * (C(-3.0) * uF);
        f[0] = f[0] + omega * (feq - f[0]) + cf * Fi;
    }
#define LB_DIR(Q, WQ, CU, CF)                                                          \
    {                                                                                  \
        const C cu = (CU), cF = (CF);                                                  \
        C feq = C(WQ) * (base + rho * (C(3.0) * cu + C(4.5) * cu * cu) - r15 - dr_sfc); \
        C Fi = C(WQ) * (C(3.0) * (cF - uF) + C(9.0) * cu * cF);                        \
        f[Q] = f[Q] + omega * (feq - f[Q]) + cf * Fi;                                  \
    }
    LB_DIR(1, W1, ux, Fx)
    LB_DIR(2, W1, uy, Fy)
    LB_DIR(3, W1, -ux, -Fx)
    LB_DIR(4, W1, -uy, -Fy)
    LB_DIR(5, W2, ux + uy, Fx + Fy)
    LB_DIR(6, W2, uy - ux, Fy - Fx)
    LB_DIR(7, W2, -ux - uy, -Fx - Fy)
    LB_DIR(8, W2, ux - uy, Fx - Fy)
#undef LB_DIR
}

// The update of one node from its gathered populations f (stored form):
// moments, velocity with the half force F^{n-1} (Fp), SFC + Guo collision
// with F^n (F) and the density excess dr, the moving-lid fold, the health
// count of a non-finite or non-positive density, and the store into B.
template <typename S, bool NT>
__device__ __forceinline__ void lb_finish_node(const GridP& g, S* __restrict__ B, const Neigh& q,
                                               typename Prec<S>::C f[NQ],
                                               typename Prec<S>::C Fpx,
                                               typename Prec<S>::C Fpy,
                                               typename Prec<S>::C Fx, typename Prec<S>::C Fy,
                                               typename Prec<S>::C dr, unsigned* health)
{
#pragma clang fp contract(on)
    using C = typename Prec<S>::C;
    constexpr bool DEV = Prec<S>::dev;
    C rho, dn, jx, jy;
    moments<C, DEV>(f, C(g.rho_f), rho, dn, jx, jy);
    const C inv = C(1) / rho;
    const C ux = (jx + C(0.5) * Fpx) * inv;
    const C uy = (jy + C(0.5) * Fpy) * inv;
    collide<C, DEV>(f, rho, dn, ux, uy, Fx, Fy, dr, C(g.omega), C(g.cforce));
    if (q.bn) {
        // lid: the populations 5 and 6 leave through the moving top wall;
        // store them already reflected-with-momentum, -2 w rho_w (c.u_w)/cs^2
        const C rw = g.lid_rho_mode ? C(g.rho_f) : rho;
        const C m = rw * C(g.lid_ux) * C(1.0 / 6.0);
        f[5] -= m;
        f[6] += m;
    }
    if (!(rho > C(0) && rho < C(1e30))) atomicAdd(&health[5], 1u);
    const long long P = g.plane;
    if (NT) {
#pragma unroll
        for (int k = 0; k < NQ; k++) __builtin_nontemporal_store(S(f[k]), &B[k * P + q.n]);
    } else {
#pragma unroll
        for (int k = 0; k < NQ; k++) B[k * P + q.n] = S(f[k]);
    }
}

}  // namespace lbrmt
