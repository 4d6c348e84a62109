"""Gradients of a trajectory loss through the coupled LBRMT step (FP64, one
solid), by the library's discrete adjoint with sqrt(T) checkpoints.

The loss follows the solid's centroid c^n = sum lambda x / sum lambda and mean
displacement d^n = sum lambda (x - xi) / sum lambda (lambda = 1 - H(phi)) over
states n = 1 .. T against a target trajectory:

    L = (1/T) sum_n |c^n - c*^n|^2 + |d^n - d*^n|^2

and its gradient with respect to the shear modulus G, the lid speed U and the
initial velocity field u_0.  Forward: T steps, the state saved every K steps
(K = round(sqrt(T)) by default).  Backward: for each segment, last first, the
saved state is restored and the segment replayed one step at a time with
lbrmt_step_snapshot (K snapshot buffers), then the adjoint runs back through
the segment's snapshots.  All arithmetic is in the library's kernels; this
module only schedules the calls and evaluates the scalar loss from lbrmt_diag.
"""
import math

import numpy as np

from . import lbrmt as B


def _solid_cfg(cfg, G, U):
    out = dict(cfg)
    out["lid_ux"] = float(U)
    s = dict(out["solid"])
    s["G"] = float(G)
    out["solid"] = s
    return out


class Trajectory:
    """A forward run that keeps what the backward pass needs."""

    def __init__(self, cfg, G, U, u0, T, target, every=None, device="cuda:0"):
        import torch
        from . import Sim
        self.torch = torch
        self.T = int(T)
        self.K = int(every or max(1, round(math.sqrt(self.T))))
        self.sim = Sim(device=device, precision="f64", **_solid_cfg(cfg, G, U))
        self.sim.set_option(B.LBRMT_OPT_GRAPH, 0)
        self.sim.init(u0)
        self.target = np.asarray(target, dtype=np.float64).reshape(self.T, 4)
        self.ckpt = {}
        self.stats = np.zeros((self.T + 1, 5))  # c_x, c_y, d_x, d_y, sum lambda
        for n in range(self.T):
            if n % self.K == 0:
                self.ckpt[n] = self.sim.save_state()
            self.sim.step(1)
            d = self.sim.diag(raise_unstable=False)
            self.stats[n + 1] = (d["centroid_x"], d["centroid_y"], d["disp_x"], d["disp_y"],
                                 d["lambda_sum"])
        # health counters of the run (fallbacks the adjoint follows as taken)
        self.health = {k: v for k, v in d["health"].items() if v} if self.T else {}
        e = self.stats[1:, :4] - self.target
        self.loss = float(np.sum(e * e) / self.T)

    def coef(self, n):
        """Loss coefficients of state n (1 <= n <= T) for lbrmt_adjoint_loss."""
        c = self.stats[n, :2]
        d = self.stats[n, 2:4]
        lam = self.stats[n, 4]
        t = self.target[n - 1]
        gc = 2.0 * (c - t[:2]) / self.T / lam
        gd = 2.0 * (d - t[2:]) / self.T / lam
        return [c[0], c[1], d[0], d[1], gc[0], gc[1], gd[0], gd[1]]

    def backward(self):
        """(dL/dG, dL/dU, dL/du_0 as a [2, ny, nx] tensor)."""
        torch = self.torch
        sim, ctx = self.sim, self.sim.ctx
        sb = B.lbrmt_snapshot_bytes(ctx)
        snaps = [torch.empty(sb, dtype=torch.uint8, device=sim.device) for _ in range(self.K)]
        adj = torch.empty(B.lbrmt_adjoint_bytes(ctx), dtype=torch.uint8, device=sim.device)
        B.lbrmt_adjoint_zero(ctx, adj)
        starts = sorted(self.ckpt)
        for s0 in reversed(starts):
            s1 = min(s0 + self.K, self.T)
            sim.load_state(self.ckpt[s0])
            for n in range(s0, s1):
                B.lbrmt_step_snapshot(ctx, snaps[n - s0])
            if s1 == self.T:
                B.lbrmt_adjoint_loss(ctx, adj, snaps[s1 - 1 - s0], 1, self.coef(self.T))
            for n in reversed(range(s0, s1)):
                if n >= 1:
                    B.lbrmt_adjoint_loss(ctx, adj, snaps[n - s0], 0, self.coef(n))
                B.lbrmt_adjoint_step(ctx, adj, snaps[n - s0])
        u0bar = torch.empty(2, sim.ny, sim.nx, dtype=torch.float64, device=sim.device)
        gG, gU = B.lbrmt_adjoint_init(ctx, adj, snaps[0], u0bar)
        torch.cuda.synchronize(sim.device)
        return gG, gU, u0bar

    def close(self):
        self.sim.close()


def trajectory(cfg, G, U, T, u0=None, device="cuda:0"):
    """c^n, d^n (n = 1 .. T) of a forward run, as a [T, 4] array."""
    from . import Sim
    sim = Sim(device=device, precision="f64", **_solid_cfg(cfg, G, U)).init(u0)
    out = np.zeros((T, 4))
    for n in range(T):
        sim.step(1)
        d = sim.diag(raise_unstable=False)
        out[n] = (d["centroid_x"], d["centroid_y"], d["disp_x"], d["disp_y"])
    sim.close()
    return out


def make_function():
    """torch.autograd.Function: loss(G, U, u0) for a fixed configuration, T and
    target; its backward runs the adjoint."""
    import torch

    class LBRMTTrajectoryLoss(torch.autograd.Function):
        @staticmethod
        def forward(fctx, G, U, u0, cfg, T, target, every):
            tr = Trajectory(cfg, float(G), float(U), u0.detach().cpu().numpy(), T, target, every,
                            device=u0.device)
            fctx.tr = tr
            return torch.tensor(tr.loss, dtype=torch.float64, device=u0.device)

        @staticmethod
        def backward(fctx, gL):
            tr = fctx.tr
            gG, gU, gu0 = tr.backward()
            tr.close()
            s = gL.to(torch.float64)
            dev = gu0.device
            return (s * torch.tensor(gG, dtype=torch.float64, device=dev),
                    s * torch.tensor(gU, dtype=torch.float64, device=dev),
                    s * gu0, None, None, None, None)

    return LBRMTTrajectoryLoss
