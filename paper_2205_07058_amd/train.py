"""GPU training of an SVLF scene with the library's own kernels.

One step = svlf_train_step (traversal, gather, decoder, Eq. 3, MSE + L1 loss
and the hand-written backward) followed by svlf_adam_step on the features
(refreshing their BF16 copy in the same pass; dense, or lazy over the feature
rows the batch touched) and on the decoder parameters.
The paper trains with Adam at learning rate 1e-3 (section 4.5).
"""

from __future__ import annotations

import torch

from . import svlf


class Trainer:
    def __init__(self, scene: "svlf.DeviceScene", params: torch.Tensor, widths, K,
                 precision="bf16", tau_mode="voxel", lr_features=1e-3, lr_params=1e-3,
                 lambda_depth=0.1, betas=(0.9, 0.999), eps=1e-8, feature_optimizer="adam",
                 viewdir=False):
        self.scene = scene
        self.params = params
        self.widths = tuple(widths)
        self.opts = svlf.make_opts(K, tau_mode, precision, svlf.FLAG_VIEWDIR if viewdir else 0)
        self.precision = precision
        self.lr_f, self.lr_p = lr_features, lr_params
        self.lam = lambda_depth
        self.b1, self.b2 = betas
        self.eps = eps
        if feature_optimizer not in ("adam", "lazy_adam"):
            raise ValueError("feature_optimizer must be 'adam' or 'lazy_adam'")
        self.feature_optimizer = feature_optimizer
        f = scene.features
        self.gF = torch.zeros_like(f)
        self.mF = torch.zeros_like(f)
        self.vF = torch.zeros_like(f)
        self.gp = torch.zeros_like(params)
        self.mp = torch.zeros_like(params)
        self.vp = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=f.device)
        self.t = 0
        self.ws = svlf.Workspace()
        if precision == "bf16" and scene.features_bf16 is None:
            scene.refresh_bf16()

    def forward_backward(self, ray_o, ray_d, t_rgb, t_depth, out_rgb=None, out_depth=None):
        """Loss and gradients of one batch (gradients accumulate into the
        zeroed gradient buffers)."""
        n = ray_o.shape[0]
        svlf.train_step([self.scene], [n], self.params, self.widths, self.opts, ray_o, ray_d,
                        t_rgb, t_depth, self.lam, 1.0 / max(n, 1), [self.gF], self.gp,
                        out_rgb=out_rgb, out_depth=out_depth, loss_out=self.loss,
                        workspace=self.ws)
        return self.loss

    def optimizer_step(self):
        self.t += 1
        bf = self.scene.features_bf16 if self.precision == "bf16" else None
        upd = svlf.lazy_adam_step if self.feature_optimizer == "lazy_adam" else svlf.adam_step
        upd(self.scene.features, self.gF, self.mF, self.vF, self.lr_f, self.b1, self.b2,
            self.eps, self.t, bf16_out=bf, zero_grad=True)
        svlf.adam_step(self.params, self.gp, self.mp, self.vp, self.lr_p, self.b1, self.b2,
                       self.eps, self.t, zero_grad=True)

    def step(self, ray_o, ray_d, t_rgb, t_depth):
        loss = self.forward_backward(ray_o, ray_d, t_rgb, t_depth)
        self.optimizer_step()
        return loss

    def render(self, ray_o, ray_d):
        n = ray_o.shape[0]
        return svlf.render([self.scene], [n], self.params, self.widths, self.opts, ray_o, ray_d,
                           workspace=self.ws)

    def state_dict(self):
        return {"features": self.scene.features.clone(), "params": self.params.clone(),
                "mF": self.mF.clone(), "vF": self.vF.clone(), "mp": self.mp.clone(),
                "vp": self.vp.clone(), "t": self.t}

    def load_state_dict(self, sd):
        self.scene.features.copy_(sd["features"])
        self.params.copy_(sd["params"])
        self.mF.copy_(sd["mF"])
        self.vF.copy_(sd["vF"])
        self.mp.copy_(sd["mp"])
        self.vp.copy_(sd["vp"])
        self.t = int(sd["t"])
        if self.precision == "bf16":
            self.scene.refresh_bf16()
