// FP64 diagnostics of the LBRMT state on gfx950: mass, momentum, solid
// centroid and mean displacement (lambda = 1 - H(phi) weighted), max |u| and
// node counts.  Two passes: every workgroup reduces its nodes with 64-lane
// wavefront shuffles plus LDS into one partial record, then one workgroup sums
// the partials in block order, so the result does not depend on scheduling.
#include "lbrmt_internal.h"

namespace lbrmt {

constexpr int DIAG_BLOCKS = 1024;
constexpr int DIAG_FIELDS = 11;  // mass, px, py, lw, lx, ly, dx, dy, nsol, nband, umax

int diag_blocks() { return DIAG_BLOCKS; }
size_t diag_partial_doubles() { return (size_t)DIAG_BLOCKS * DIAG_FIELDS; }

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_maxd(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

template <typename S>
__global__ __launch_bounds__(256) void k_diag_partial(GridP g, BodyP b, const S* __restrict__ A,
                                                      const double* __restrict__ fpx,
                                                      const double* __restrict__ fpy,
                                                      const Win* __restrict__ win, int wprev,
                                                      double fpo_x, double fpo_y,
                                                      const S* __restrict__ X,
                                                      const S* __restrict__ Y,
                                                      const S* __restrict__ phi,
                                                      double* partial, StampValid sv)
{
    const long long N = (long long)g.nx * g.ny;
    const Rect D = window_of(win, wprev, g);
    const long long P = g.plane;
    const double wq[NQ] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                           1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
    double acc[DIAG_FIELDS] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.nx), j = (int)(e / g.nx);
        const bool bw = !g.px && i == 0, be = !g.px && i == g.nx - 1;
        const bool bs = !g.py && j == 0, bn = !g.py && j == g.ny - 1;
        int im = i - 1, ip = i + 1, jm = j - 1, jp = j + 1;
        im = im < 0 ? (g.px ? g.nx - 1 : 0) : im;
        ip = ip >= g.nx ? (g.px ? 0 : g.nx - 1) : ip;
        jm = jm < 0 ? (g.py ? g.ny - 1 : 0) : jm;
        jp = jp >= g.ny ? (g.py ? 0 : g.ny - 1) : jp;
        const long long r0 = (long long)j * g.pitch, rm = (long long)jm * g.pitch,
                        rp = (long long)jp * g.pitch, n = r0 + i;
        double f[NQ];
        f[0] = A[n];
        f[1] = bw ? A[3 * P + n] : A[1 * P + r0 + im];
        f[2] = bs ? A[4 * P + n] : A[2 * P + rm + i];
        f[3] = be ? A[1 * P + n] : A[3 * P + r0 + ip];
        f[4] = bn ? A[2 * P + n] : A[4 * P + rp + i];
        f[5] = (bw || bs) ? A[7 * P + n] : A[5 * P + rm + im];
        f[6] = (be || bs) ? A[8 * P + n] : A[6 * P + rm + ip];
        f[7] = (be || bn) ? A[5 * P + n] : A[7 * P + rp + ip];
        f[8] = (bw || bn) ? A[6 * P + n] : A[8 * P + rp + im];
        if (sizeof(S) == 4)
            for (int k = 0; k < NQ; k++) f[k] += wq[k] * g.rho_f;
        double Fx = fpo_x, Fy = fpo_y;
        if (sv.stamp ? sv.has(i, j) : D.has(i, j)) {
            Fx = fpx[n];
            Fy = fpy[n];
        }
        const double rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
        const double jx = f[1] + f[5] + f[8] - f[3] - f[6] - f[7];
        const double jy = f[2] + f[5] + f[6] - f[4] - f[7] - f[8];
        acc[0] += rho;
        acc[1] += jx + 0.5 * Fx;
        acc[2] += jy + 0.5 * Fy;
        const double ux = jx / rho + Fx / (2.0 * rho), uy = jy / rho + Fy / (2.0 * rho);
        acc[10] = fmax(acc[10], sqrt(ux * ux + uy * uy));
        if (b.present && D.has(i, j)) {
            const long long k = pidx(g, i, j);
            const double p = (double)phi[k];
            if (p < INFINITY) {
                acc[9] += 1.0;
                if (p < 0.0) acc[8] += 1.0;
                double H;
                if (p <= -g.eps) H = 0.0;
                else if (p >= g.eps) H = 1.0;
                else H = 0.5 * (1.0 + p / g.eps + sin(M_PI * p / g.eps) / M_PI);
                const double lam = 1.0 - H;
                double x = i + 0.5, y = j + 0.5;
                if (g.px) {
                    double d = x - b.cx;
                    d -= g.nx * floor(d / g.nx + 0.5);
                    x = b.cx + d;
                }
                if (g.py) {
                    double d = y - b.cy;
                    d -= g.ny * floor(d / g.ny + 0.5);
                    y = b.cy + d;
                }
                acc[3] += lam;
                acc[4] += lam * x;
                acc[5] += lam * y;
                // x - xi; the FP32 mode stores the displacement xi - x itself
                const double dx = sizeof(S) == 4 ? -(double)X[k] : x - (double)X[k];
                const double dy = sizeof(S) == 4 ? -(double)Y[k] : y - (double)Y[k];
                acc[6] += lam * dx;
                acc[7] += lam * dy;
            }
        }
    }
    __shared__ double red[DIAG_FIELDS][4];
    const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int c = 0; c < DIAG_FIELDS; c++) {
        const double v = c == 10 ? wave_maxd(acc[c]) : wave_sum(acc[c]);
        if (lane == 0) red[c][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < DIAG_FIELDS) {
        const int c = threadIdx.x;
        double v = red[c][0];
        for (int w = 1; w < (int)(blockDim.x / 64); w++)
            v = c == 10 ? fmax(v, red[c][w]) : v + red[c][w];
        partial[(long long)blockIdx.x * DIAG_FIELDS + c] = v;
    }
}

// one wave per field: lane l adds partials l, l + 64, ... in order, then a
// fixed butterfly combines the lanes, so the result is deterministic
__global__ __launch_bounds__(DIAG_FIELDS * 64) void k_diag_final(const double* __restrict__ partial,
                                                                 int nblocks, double* out)
{
    const int c = threadIdx.x / 64, lane = threadIdx.x % 64;
    double v = 0.0;
    for (int k = lane; k < nblocks; k += 64) {
        const double x = partial[(long long)k * DIAG_FIELDS + c];
        v = c == 10 ? fmax(v, x) : v + x;
    }
    v = c == 10 ? wave_maxd(v) : wave_sum(v);
    if (lane == 0) out[c] = v;
}

hipError_t launch_diag(const GridP& g, int precision, const BodyP& b, const void* A,
                       const double* fpx, const double* fpy, const Win* win, int wprev,
                       double fpo_x, double fpo_y, const BandBufs& bb, int buf, double* partial,
                       double* out, hipStream_t st, StampValid sv)
{
    if (precision == 0)
        k_diag_partial<double><<<DIAG_BLOCKS, 256, 0, st>>>(g, b, (const double*)A, fpx, fpy, win,
                                                            wprev, fpo_x, fpo_y,
                                                            (const double*)bb.X[buf],
                                                            (const double*)bb.Y[buf],
                                                            (const double*)bb.phi[buf], partial,
                                                            sv);
    else
        k_diag_partial<float><<<DIAG_BLOCKS, 256, 0, st>>>(g, b, (const float*)A, fpx, fpy, win,
                                                           wprev, fpo_x, fpo_y,
                                                           (const float*)bb.X[buf],
                                                           (const float*)bb.Y[buf],
                                                           (const float*)bb.phi[buf], partial,
                                                           sv);
    k_diag_final<<<1, DIAG_FIELDS * 64, 0, st>>>(partial, DIAG_BLOCKS, out);
    return hipGetLastError();
}

}  // namespace lbrmt
