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
                 viewdir=False, deterministic=False):
        self.scene = scene
        self.params = params
        self.widths = tuple(widths)
        flags = (svlf.FLAG_VIEWDIR if viewdir else 0) | (svlf.FLAG_DETERMINISTIC if deterministic else 0)
        self.opts = svlf.make_opts(K, tau_mode, precision, flags)
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


class LfTrainer:
    """The paper's staged training of the light-field function (section 4.4):

    stage 1 "surface": Eq. 4 on the voxel holding each ray's target surface
             point (colour, within-voxel depth eta, and the opacity term);
    stage 2 "volume":  Eq. 4 with the composited colour, lambda_tau = 0, the
             colour embeddings Z_C and the colour decoder frozen (neither
             updated nor given gradients; gradients still pass through them
             to eta);
    stage 3 "finetune": as stage 2 with everything trained at the lower
             learning rate.

    Adam runs separately on the density side (the Z_T block of the feature
    table and the density decoder's parameters, a prefix of each array) and
    on the colour side, each with its own step count, so that a frozen side
    keeps its parameters and moments unchanged."""

    STAGES = ("surface", "volume", "finetune")

    def __init__(self, scene: "svlf.DeviceScene", params: torch.Tensor, K, precision="bf16",
                 tau_mode="direct", lambda_eta=1.0, lambda_tau=0.1, lr=1e-3, lr_finetune=2e-4,
                 betas=(0.9, 0.999), eps=1e-8, viewdir=False):
        self.scene = scene
        self.params = params
        self.opts = svlf.make_opts(K, tau_mode, precision, svlf.FLAG_VIEWDIR if viewdir else 0)
        self.precision = precision
        self.lam_eta, self.lam_tau = lambda_eta, lambda_tau
        self.lr, self.lr_ft = lr, lr_finetune
        self.b1, self.b2 = betas
        self.eps = eps
        nv = scene.octree.n_vertices
        self.nf_T = nv * svlf.LF_DECODERS[0]          # Z_T block of the feature array
        opts32 = svlf.make_opts(K, tau_mode, "fp32", self.opts.flags)
        n_all = svlf.lf_param_count(opts32)
        ct, cc, h, nht, nhc = svlf.LF_DECODERS
        widths_t = (2 * ct + 6,) + (h,) * nht + (2,)
        self.np_T = sum(a * b + b for a, b in zip(widths_t[:-1], widths_t[1:]))
        assert params.numel() == n_all
        f = scene.features
        self.gF, self.mF, self.vF = torch.zeros_like(f), torch.zeros_like(f), torch.zeros_like(f)
        self.gp, self.mp, self.vp = (torch.zeros_like(params), torch.zeros_like(params),
                                     torch.zeros_like(params))
        self.loss = torch.zeros(1, dtype=torch.float32, device=f.device)
        self.t = {"density": 0, "color": 0}
        self.ws = svlf.Workspace()
        if precision == "bf16" and scene.features_bf16 is None:
            scene.refresh_bf16()

    def _adam(self, side, lr):
        self.t[side] += 1
        t = self.t[side]
        fs = slice(0, self.nf_T) if side == "density" else slice(self.nf_T, None)
        ps = slice(0, self.np_T) if side == "density" else slice(self.np_T, None)
        bf = self.scene.features_bf16[fs] if self.precision == "bf16" else None
        svlf.adam_step(self.scene.features[fs], self.gF[fs], self.mF[fs], self.vF[fs], lr, self.b1,
                       self.b2, self.eps, t, bf16_out=bf, zero_grad=True)
        svlf.adam_step(self.params[ps], self.gp[ps], self.mp[ps], self.vp[ps], lr, self.b1, self.b2,
                       self.eps, t, zero_grad=True)

    def step(self, stage, ray_o, ray_d, t_rgb, t_depth):
        if stage not in self.STAGES:
            raise ValueError(f"stage must be one of {self.STAGES}")
        n = ray_o.shape[0]
        frozen = stage == "volume"
        loss = svlf.make_lf_loss("surface" if stage == "surface" else "volume", self.lam_eta,
                                 self.lam_tau if stage == "surface" else 0.0, 1.0 / max(n, 1),
                                 freeze_color=frozen)
        svlf.lf_train_stage([self.scene], [n], self.params, self.opts, ray_o, ray_d, t_rgb, t_depth,
                            loss, [self.gF], self.gp, loss_out=self.loss, workspace=self.ws)
        lr = self.lr_ft if stage == "finetune" else self.lr
        self._adam("density", lr)
        if not frozen:
            self._adam("color", lr)
        return self.loss

    def render(self, ray_o, ray_d):
        n = ray_o.shape[0]
        return svlf.lf_render([self.scene], [n], self.params, self.opts, ray_o, ray_d,
                              workspace=self.ws)
