"""Gradients of a trajectory loss through the coupled LBRMT step (FP64, one
solid), by the library's discrete adjoint with sqrt(T) checkpoints.

The loss follows the solid's centroid c^n = sum lambda x / sum lambda and mean
displacement d^n = sum lambda (x - xi) / sum lambda (lambda = 1 - H(phi)) over
states n = 1 .. T against a target trajectory:

    L = (1/T) sum_n |c^n - c*^n|^2 + |d^n - d*^n|^2

and its gradient with respect to the shear modulus G, the lid speed U and the
initial velocity field u_0.  Forward: T steps (replaying the library's
captured step graphs), the state saved every K steps (K = round(sqrt(T)) by
default) and the sums behind c^n and d^n recorded on the device after every
step (lbrmt_diag_sums), read back once at the end.  Backward: for each
segment, last first, the saved state is restored and the segment replayed
one step at a time with lbrmt_step_snapshot (K snapshot buffers), then the
adjoint runs back through the segment's snapshots.  All arithmetic of the
step and its adjoint is in the library's kernels; this module schedules the
calls and evaluates the scalar loss from the recorded sums.
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
        self.sim.init(u0)
        self.target = np.asarray(target, dtype=np.float64).reshape(self.T, 4)
        self.ckpt = {}
        sums = torch.empty((self.T + 1, 11), dtype=torch.float64, device=self.sim.device)
        for n in range(self.T):
            if n % self.K == 0:
                self.ckpt[n] = self.sim.save_state()
            self.sim.step(1)
            B.lbrmt_diag_sums(self.sim.ctx, sums[n + 1])
        s = sums.cpu().numpy()
        # the solid-set and map sizes after each step (discrete decisions of
        # the run; two runs that differ here took different branches)
        self.counts = s[1:, 8:10].copy()
        lam = s[:, 3]
        with np.errstate(invalid="ignore", divide="ignore"):
            # lambda-weighted centroid (c_x, c_y) and mean displacement
            # (d_x, d_y) of the solid, and the weight sum lambda
            self.stats = np.stack([s[:, 4] / lam, s[:, 5] / lam, s[:, 6] / lam, s[:, 7] / lam,
                                   lam], axis=1)
        # health counters of the run (fallbacks the adjoint follows as taken)
        d = self.sim.diag(raise_unstable=False)
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
        self.ckpt = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trajectory(cfg, G, U, T, u0=None, device="cuda:0"):
    """c^n, d^n (n = 1 .. T) of a forward run, as a [T, 4] array."""
    import torch
    from . import Sim
    sim = Sim(device=device, precision="f64", **_solid_cfg(cfg, G, U)).init(u0)
    sums = torch.empty((T, 11), dtype=torch.float64, device=sim.device)
    for n in range(T):
        sim.step(1)
        B.lbrmt_diag_sums(sim.ctx, sums[n])
    s = sums.cpu().numpy()
    sim.close()
    lam = s[:, 3:4]
    return s[:, 4:8] / lam


def make_function():
    """torch.autograd.Function: loss(G, U, u0) for a fixed configuration, T and
    target; its backward runs the adjoint."""
    import torch

    class LBRMTTrajectoryLoss(torch.autograd.Function):
        @staticmethod
        def forward(fctx, G, U, u0, cfg, T, target, every):
            tr = Trajectory(cfg, float(G), float(U), u0.detach().cpu().numpy(), T, target, every,
                            device=u0.device)
            loss = torch.tensor(tr.loss, dtype=torch.float64, device=u0.device)
            if any(fctx.needs_input_grad[:3]):
                fctx.tr = tr
            else:
                tr.close()  # no backward will follow: release the run now
            return loss

        @staticmethod
        def backward(fctx, gL):
            tr = fctx.tr
            gG, gU, gu0 = tr.backward()
            tr.close()
            fctx.tr = None
            s = gL.to(torch.float64)
            dev = gu0.device
            need = fctx.needs_input_grad
            return (s * torch.tensor(gG, dtype=torch.float64, device=dev) if need[0] else None,
                    s * torch.tensor(gU, dtype=torch.float64, device=dev) if need[1] else None,
                    s * gu0 if need[2] else None, None, None, None, None)

    return LBRMTTrajectoryLoss
