"""torch.autograd binding of the adjoint: trajectory losses as differentiable
functions of the initial state and the pair tables.

``trajectory_loss`` runs ``nsteps`` timesteps of a fresh system in the
library (``mdpd_forward_record``, checkpoints every ``every`` steps) and
returns the three loss terms (mean fluid many-body density, virial pressure,
mean fluid x-velocity) of the final state or their mean over the steps.  Its
backward is ``mdpd_backward`` with the upstream gradient as the loss weights,
so one reverse pass yields the gradient with respect to x0, v0, A, B and
gamma.  The forward pass and the reverse pass both run in the HIP kernels;
this module only moves arguments.
"""
import numpy as np
import torch

from ._native import FP64, System, make_params


def _host(t):
    return t.detach().to("cpu", torch.float64).numpy() if torch.is_tensor(t) else np.asarray(t, np.float64)


class TrajectoryLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, A, B, gamma, spec):
        kw = dict(spec["params"])
        params = make_params(A=_host(A), B=_host(B), gamma=_host(gamma), **kw)
        dev = x0.device
        if dev.type == "cuda":
            sys_ = System(params=params, x=x0.detach(), v=v0.detach(), types=spec["types"].to(dev),
                          frozen=spec["frozen"].to(dev))
        else:
            sys_ = System(params=params, x=_host(x0), v=_host(v0), types=spec["types"].cpu().numpy(),
                          frozen=spec["frozen"].cpu().numpy())
        loss = sys_.forward_record(spec["nsteps"], every=spec["every"], average=spec["average"])
        ctx.sys = sys_
        ctx.dev = dev
        ctx.vdev = v0.device
        ctx.tdev = [t.device if torch.is_tensor(t) else torch.device("cpu") for t in (A, B, gamma)]
        ctx.tshape = tuple(np.atleast_2d(_host(A)).shape)
        return torch.as_tensor(loss, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, gl):
        w = gl.detach().to("cpu", torch.float64).numpy()
        g = ctx.sys.backward(w, device=ctx.dev if ctx.dev.type == "cuda" else None)
        dx0, dv0 = g["dx0"], g["dv0"]
        if not torch.is_tensor(dx0):
            dx0 = torch.from_numpy(dx0)
            dv0 = torch.from_numpy(dv0)
        tab = [torch.as_tensor(g[k].reshape(ctx.tshape), dtype=torch.float64, device=d)
               for k, d in zip(("dA", "dB", "dgamma"), ctx.tdev)]
        return (dx0.to(ctx.dev), dv0.to(ctx.vdev), *tab, None)


def trajectory_loss(x0, v0, A, B, gamma, types, frozen, box, nsteps, every=10, average=True, rc=1.0,
                    rd=0.75, kT=1.0, dt=0.01, mass=1.0, g=(0.0, 0.0, 0.0), seed=0, precision=FP64,
                    wall_model=0, phi_c=0.5):
    """Loss terms (mean fluid density, pressure, mean fluid x-velocity) of a
    trajectory of nsteps from (x0, v0); differentiable in x0, v0, A, B, gamma
    (T x T float64 tensors).  Frozen particles stay put; with wall_model = 1
    the bounce-back corrector's events of the trajectory are held fixed."""
    spec = {
        "params": dict(box=box, rc=rc, rd=rd, kT=kT, dt=dt, mass=mass, g=g, seed=seed, precision=precision,
                       wall_model=wall_model, phi_c=phi_c),
        "types": torch.as_tensor(types, dtype=torch.int32),
        "frozen": torch.as_tensor(frozen, dtype=torch.uint8),
        "nsteps": int(nsteps),
        "every": int(every),
        "average": bool(average),
    }
    return TrajectoryLoss.apply(x0, v0, A, B, gamma, spec)
