"""The paper's own benchmark setups run on the GPU path (loose physical
checks, not parity).

Soft disc in a lid-driven cavity (Sec. 4.1): L x L cavity, tau = 1, Re = 100,
disc of radius 0.2 L centred at (0.6 L, 0.5 L), G = 0.1 at L = 200, density
ratio 1.  Other sizes keep Re and tau, so the lid speed scales as U = Re nu / L
and time as L^2 (T = 20000 steps at L = 80, 1 280 000 at L = 640); the shear
modulus keeps G / (rho_f U^2) of the L = 200 case: G = 0.1 (U / U_200)^2.
The paper reports the solid's volume change at the same physical time (9.2 %
decrease at L = 80 down to 0.3 % at L = 640) and a spatial convergence rate
near 1.4 against the L = 640 run.

Volume of the solid: sum over nodes of lambda = 1 - H_eps(phi) (lattice
units, one node per unit area), from the level set the library returns.
Convergence: the centroid (sum lambda x / sum lambda) at the final time, in
units of L, against the finest grid run.

``python tests/paper_setups.py [L ...]`` runs the cavity at the given sizes
(default 160, 320, 640; about five minutes on one GPU) and prints the table.
At L = 80 this scaling gives G = 0.625, stiffer than the explicit stress
update tolerates (the run blows up within 20000 steps).
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import workloads  # noqa: E402

TAU, RE, G200, L200 = 1.0, 100.0, 0.1, 200


def cavity_setup(L):
    nu = (TAU - 0.5) / 3.0
    U = RE * nu / L
    U200 = RE * nu / L200
    G = G200 * (U / U200) ** 2
    T = int(round(20000 * (L / 80.0) ** 2))
    cfg = workloads.make(nx=L, ny=L, tau=TAU, lid_ux=U,
                         solid=dict(cx=0.6 * L, cy=0.5 * L, R=0.2 * L, G=G, rho_s=1.0),
                         name=f"zhao_cavity_{L}")
    return cfg, T


def _lambda(phi, eps):
    lam = np.zeros_like(phi)
    ok = np.isfinite(phi)
    p = phi[ok]
    H = np.where(p <= -eps, 0.0, np.where(p >= eps, 1.0,
                 0.5 * (1.0 + p / eps + np.sin(np.pi * p / eps) / np.pi)))
    lam[ok] = 1.0 - H
    return lam


def solid_measures(sim, L, eps=1.5):
    _, _, phi = [t.cpu().numpy() for t in sim.refmap()]
    lam = _lambda(phi, eps)
    y, x = np.mgrid[0:L, 0:L] + 0.5
    area = lam.sum()
    return area, (lam * x).sum() / area / L, (lam * y).sum() / area / L


def run_cavity(L, precision="f64", progress=False):
    from paper_2402_12696_amd import Sim
    cfg, T = cavity_setup(L)
    sim = Sim(device="cuda:0", precision=precision, **cfg).init()
    a0, _, _ = solid_measures(sim, L)
    t0 = time.perf_counter()
    chunk = 60000
    for done in range(0, T, chunk):
        sim.step(min(chunk, T - done))
        if progress and done + chunk < T:
            sim.torch.cuda.synchronize()
            print(f"  L={L} step {done + chunk}", flush=True)
    a1, cx, cy = solid_measures(sim, L)
    health = sim.diag(raise_unstable=False)["health"]
    dt = time.perf_counter() - t0
    _, ux, uy = [t.cpu().numpy() for t in sim.macro()]
    lam = _lambda(sim.refmap()[2].cpu().numpy(), 1.5)
    sim.close()
    U = cfg["lid_ux"]
    return dict(L=L, steps=T, volume_change=a1 / a0 - 1.0, cx=cx, cy=cy, seconds=dt,
                health_ok=all(v == 0 for v in health.values()), u=np.stack([ux, uy]) / U,
                lam=lam)


def restrict(field, k):
    """Cell average of a node-centred field onto a grid k times coarser."""
    *lead, ny, nx = field.shape
    return field.reshape(*lead, ny // k, k, nx // k, k).mean(axis=(-3, -1))


def convergence(rows, key):
    """Relative RMS error of a field against the finest run (restricted onto
    each coarser grid) and the observed orders between successive grids."""
    ref = rows[-1]
    errs = []
    for r in rows[:-1]:
        k = ref["L"] // r["L"]
        fr = restrict(ref[key], k)
        errs.append(np.sqrt(np.mean((r[key] - fr) ** 2)) / np.sqrt(np.mean(fr ** 2)))
    Ls = [r["L"] for r in rows[:-1]]
    rates = [np.log(errs[k] / errs[k + 1]) / np.log(Ls[k + 1] / Ls[k])
             for k in range(len(errs) - 1)]
    return errs, rates


def run_settling(nx=100, ny=300, rho_s=1.25, g=1e-5, steps=20000):
    from paper_2402_12696_amd import Sim
    cfg = workloads.settling_disc(nx=nx, ny=ny, rho_s=rho_s, g=g)
    sim = Sim(device="cuda:0", **cfg).init()
    d0 = sim.diag()
    sim.step(steps)
    d1 = sim.diag(raise_unstable=False)
    sim.close()
    return d0, d1


if __name__ == "__main__":
    sizes = [int(a) for a in sys.argv[1:]] or [160, 320, 640]
    rows = []
    for L in sizes:
        r = run_cavity(L, progress=True)
        rows.append(r)
        print(f"L={L:4d} steps={r['steps']:8d} volume change {100 * r['volume_change']:+.2f} % "
              f"centroid ({r['cx']:.4f}, {r['cy']:.4f}) L  health ok {r['health_ok']}  "
              f"{r['seconds']:.1f} s", flush=True)
    if len(rows) >= 3:
        for key, what in (("u", "velocity / U"), ("lam", "solid fraction")):
            errs, rates = convergence(rows, key)
            print(f"{what}: relative RMS error vs L={rows[-1]['L']}:",
                  [f"{e:.3e}" for e in errs], "orders:", [f"{q:.2f}" for q in rates],
                  flush=True)
        ref = rows[-1]
        print("centroid distance to the finest (units of L):",
              [f"{np.hypot(r['cx'] - ref['cx'], r['cy'] - ref['cy']):.2e}" for r in rows[:-1]],
              flush=True)
    d0, d1 = run_settling()
    print(f"settling 100x300 rho_s 1.25: centroid y {d0['centroid_y']:.2f} -> "
          f"{d1['centroid_y']:.2f}, mass change {d1['mass'] / d0['mass'] - 1:.2e}", flush=True)
