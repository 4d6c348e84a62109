"""Seeded synthetic workloads of the LBRMT time step.

This module only states inputs -- grid sizes, parameters, solid placements and
seeded random fields -- in the keyword form that both the GPU binding
(``paper_2402_12696_amd.Sim``) and the CPU oracle accept.  It holds none of the
method's arithmetic.  Lattice units throughout (dx = dt = rho_f = 1); node (i, j)
sits at x = (i + 1/2, j + 1/2).

The paper's own scenes (a soft disc in a lid-driven cavity, Sec. 4.1; settling,
Sec. 4.3) are the templates; no external data set is used.
"""
import numpy as np

_DEFAULTS = dict(
    periodic_x=False, periodic_y=False, lid_ux=0.0, gravity=(0.0, 0.0), fext=(0.0, 0.0),
    rho_f=1.0, eps=1.5, layers=11, r_max=8, det_rel=1e-8, detJ_min=1e-12, eta=1.0, solid=None,
    kappa_J=0.25, lid_rho_mode=0,
)


def make(**kw):
    cfg = dict(_DEFAULTS)
    cfg.update(kw)
    return cfg


def cavity_disc_64():
    """64x64 lid-driven cavity, tau 0.8, lid 0.1, disc R 12 at (32, 40), G 0.01,
    density ratio 1, blur half-width 1.5; fluid at rest, rho 1; 1000 steps."""
    return make(nx=64, ny=64, tau=0.8, lid_ux=0.1,
                solid=dict(cx=32.0, cy=40.0, R=12.0, G=0.01, rho_s=1.0), steps=1000,
                name="cavity_disc_64")


def cavity_disc_2048():
    """2048x2048 lid-driven cavity, tau 0.6, lid 0.05, disc R 0.15 L at
    (0.5 L, 0.6 L), G 0.005, density ratio 1; 20000 steps."""
    L = 2048
    return make(nx=L, ny=L, tau=0.6, lid_ux=0.05,
                solid=dict(cx=0.5 * L, cy=0.6 * L, R=0.15 * L, G=0.005, rho_s=1.0),
                steps=20000, name="cavity_disc_2048")


def cavity_disc_256():
    """256x256 cavity, tau 0.7, lid 0.08, disc R 40 at (128, 153.6), G 0.01."""
    return make(nx=256, ny=256, tau=0.7, lid_ux=0.08,
                solid=dict(cx=128.0, cy=153.6, R=40.0, G=0.01, rho_s=1.0), steps=3000,
                name="cavity_disc_256")


def settling_disc(nx=64, ny=192, rho_s=1.25, g=1e-5):
    """Sec. 4.3 template: a disc of radius 0.2 L in a closed L x 3L box under
    gravity along -y, density contrast rho_s / rho_f != 1."""
    return make(nx=nx, ny=ny, tau=1.0, gravity=(0.0, -g),
                solid=dict(cx=0.5 * nx, cy=0.5 * ny, R=0.2 * nx, G=0.1, rho_s=rho_s),
                name="settling_disc")


def gaussian_velocity(nx, ny, std, seed):
    """i.i.d. Gaussian initial velocity, shape (2, ny, nx) (ux plane, uy plane)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=(2, ny, nx))


def cellular_velocity(nx, ny, amp, cells, seed):
    """Divergence-free cellular flow of shape (2, ny, nx): stream function
    psi = amp / k * sin(k x + a) * sin(k y + b), k = 2 pi cells / max(nx, ny),
    phases a, b from numpy default_rng(seed); u = dpsi/dy, v = -dpsi/dx, so
    |u| <= amp.  A solid placed in it is sheared and carried from the first
    step."""
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(0.0, 2.0 * np.pi, size=2)
    k = 2.0 * np.pi * cells / max(nx, ny)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    X, Y = np.meshgrid(x, y)
    u = np.zeros((2, ny, nx))
    u[0] = amp * np.sin(k * X + a) * np.cos(k * Y + b)
    u[1] = -amp * np.cos(k * X + a) * np.sin(k * Y + b)
    return u


def uniform_velocity(nx, ny, ux, uy):
    u = np.zeros((2, ny, nx))
    u[0] = ux
    u[1] = uy
    return u


def taylor_green_velocity(n, u0):
    """Taylor-Green vortex on an n x n periodic box, wavenumber 2 pi / n."""
    k = 2.0 * np.pi / n
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x)
    u = np.zeros((2, n, n))
    u[0] = -u0 * np.cos(k * X) * np.sin(k * Y)
    u[1] = u0 * np.sin(k * X) * np.cos(k * Y)
    return u


def cavity_ensemble(n=96, seed=4):
    """Ensemble of independent cavity-disc simulations of uneven sizes (the
    batched workload): for each member in order, side L drawn uniformly from
    {96, 128, ..., 768}, tau ~ U[0.55, 1.0], lid ~ U[0.02, 0.1],
    R ~ U[0.1, 0.25] L, log10 G ~ U[-3, log10 0.03]; disc at (0.5 L, 0.6 L),
    density ratio 1; numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    sides = np.arange(96, 769, 32)
    out = []
    for k in range(n):
        L = int(rng.choice(sides))
        tau = float(rng.uniform(0.55, 1.0))
        U = float(rng.uniform(0.02, 0.1))
        R = float(rng.uniform(0.1, 0.25)) * L
        G = float(10.0 ** rng.uniform(-3.0, np.log10(0.03)))
        out.append(make(nx=L, ny=L, tau=tau, lid_ux=U,
                        solid=dict(cx=0.5 * L, cy=0.6 * L, R=R, G=G, rho_s=1.0),
                        name=f"ensemble_{seed}_{k}"))
    return out


def suspension(n=4096, nbody=400, seed=240212696, tau=0.7, g=1e-6, eps=1.5, eta=1.0,
               a_range=(12.0, 24.0), gap=3.0, max_draws=100000):
    """Many soft bodies in a periodic box under gravity (the paper's mixing
    scenes of Sec. 4.5 at a synthetic scale): an n x n periodic box, tau,
    gravity g along -y acting on the density contrast.  For each body in order
    (numpy default_rng(seed)): semi-major axis a ~ U[a_range], aspect ~ U[1, 2]
    (b = a / aspect; an ellipse, a disc when b = a), angle ~ U[0, pi),
    log10 G ~ U[-3, -2], rho_s ~ U[1.2, 2.0]; then the centre ~ U[0, n)^2,
    drawn again until its minimum-image distance to every earlier centre is at
    least a_i + a_j + 2 eps + gap."""
    rng = np.random.default_rng(seed)
    bodies = []
    for k in range(nbody):
        a = float(rng.uniform(*a_range))
        b = a / float(rng.uniform(1.0, 2.0))
        th = float(rng.uniform(0.0, np.pi))
        G = float(10.0 ** rng.uniform(-3.0, -2.0))
        rs = float(rng.uniform(1.2, 2.0))
        for _ in range(max_draws):
            c = rng.uniform(0.0, n, size=2)
            ok = True
            for o in bodies:
                d = np.abs(c - np.array([o["cx"], o["cy"]]))
                d = np.minimum(d, n - d)
                if np.hypot(*d) < a + o["R"] + 2 * eps + gap:
                    ok = False
                    break
            if ok:
                break
        else:
            raise ValueError("could not place every body")
        bodies.append(dict(cx=float(c[0]), cy=float(c[1]), R=a, G=G, rho_s=rs,
                           shape="ellipse", b=b, theta=th))
    return make(nx=n, ny=n, tau=tau, periodic_x=True, periodic_y=True, gravity=(0.0, -g),
                eps=eps, eta=eta, solids=bodies, name=f"suspension_{n}_{nbody}")
