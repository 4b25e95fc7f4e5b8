"""End-to-end inverse design: Adam on the Eq. 5 loss (Demonstrations, Fig. 5).

Each iteration is one fused forward + loss + backward of the library
(rw_forward_backward), followed by rw_adam_step on three parameter groups:
* the DOE phase map;
* the amplitude map (or the second phase map of a two-phase DOE), clamped to
  `amp_bounds` unless that is None;
* the normalised lens parameters.

Everything stays on the device.  The state (parameters, Adam moments, step
count) is a dict of tensors that `save` writes and `Design.resume` reads back
with torch's weights-only loader.
"""
import torch

from .rw import adam_step

GROUPS = ("phase", "amp", "lens")


class Design:
    def __init__(self, plan, lens, phase, amp, target, lr=(1e-2, 1e-2, 1e-2),
                 amp_bounds=(0.0, 1.0), betas=(0.9, 0.999), eps=1e-8):
        """plan: a Plan with a backward workspace; lens, phase, amp: initial values
        (float32 device tensors, copied); target: the Eq. 5 targets [L, F, Q, Q];
        lr: learning rates of (phase, amp, lens)."""
        self.plan = plan
        self.target = target
        self.lr = dict(zip(GROUPS, lr))
        self.amp_bounds = amp_bounds
        self.betas = betas
        self.eps = eps
        self.t = 0
        self.p = {"phase": phase.detach().clone().contiguous(),
                  "amp": amp.detach().clone().contiguous(),
                  "lens": lens.detach().clone().contiguous()}
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.g = {k: torch.empty_like(v) for k, v in self.p.items()}
        dev = phase.device
        self.psf = torch.empty((plan.L, plan.F, plan.Q, plan.Q), dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)

    def step(self):
        """One iteration: the loss and gradients at the current parameters, then
        the Adam update.  Returns the loss tensor of those parameters."""
        self.plan.step(self.p["lens"], self.p["phase"], self.p["amp"], self.target,
                       psf_out=self.psf, loss_out=self.loss, d_phase=self.g["phase"],
                       d_amp=self.g["amp"],
                       d_lens=self.g["lens"] if self.p["lens"].numel() else None)
        self.t += 1
        b1, b2 = self.betas
        for k in GROUPS:
            if self.p[k].numel() == 0:
                continue
            bounds = self.amp_bounds if k == "amp" else None
            adam_step(self.p[k], self.g[k], self.m[k], self.v[k], self.t, self.lr[k], b1, b2,
                      self.eps, bounds)
        return self.loss

    def run(self, steps, callback=None):
        """`steps` iterations; callback(design, loss_value) after each (it may
        synchronise).  Returns the list of losses."""
        out = []
        for _ in range(steps):
            loss = float(self.step().item())
            out.append(loss)
            if callback is not None:
                callback(self, loss)
        return out

    def state_dict(self):
        d = {"t": torch.tensor(self.t)}
        for k in GROUPS:
            d[f"p_{k}"] = self.p[k]
            d[f"m_{k}"] = self.m[k]
            d[f"v_{k}"] = self.v[k]
        return d

    def load_state_dict(self, d):
        self.t = int(d["t"])
        for k in GROUPS:
            self.p[k].copy_(d[f"p_{k}"])
            self.m[k].copy_(d[f"m_{k}"])
            self.v[k].copy_(d[f"v_{k}"])

    def save(self, path):
        torch.save({k: v.detach().cpu() for k, v in self.state_dict().items()}, path)

    @classmethod
    def resume(cls, path, plan, target, **kw):
        """A Design restored from `save`'s file (loaded with weights_only=True)."""
        d = torch.load(path, map_location="cpu", weights_only=True)
        dev = target.device
        des = cls(plan, d["p_lens"].to(dev), d["p_phase"].to(dev), d["p_amp"].to(dev), target,
                  **kw)
        des.load_state_dict({k: v.to(dev) for k, v in d.items()})
        return des
