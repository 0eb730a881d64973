"""The hierarchy optimisation of Sec. 5.1 as a loop over the library's calls.

After generation, the paper optimises the interior nodes of a hierarchy
against the training images, with the leaves unchanged: each iteration takes
a random training view and a random target granularity tau in a range, cuts
the hierarchy at that tau (with the interpolation of Sec. 4.2 between a cut
node and its parent), renders and back-propagates through the interpolation
to the nodes (the absolute-value opacity activation and the zero gradient at
the 0.99 clamp of Sec. 7.3 are the library's).  Here an iteration takes a
batch of distinct training views, each with its own tau, drawn log-uniform
over the range (uniform in log tau); the loss is the L1 image distance and
the optimiser Adam on the interior nodes.

Every step runs in the library: ``hgs_render`` (cut, interpolation and
splatting of the batch), ``hgs_l1_loss`` (loss and cotangent) and
``hgs_backward_adam_step`` (the backward with the Adam update applied in its
gradient gather; ``fused=False`` takes ``hgs_render_backward`` into gradient
arrays and ``hgs_adam_step`` instead, with the same result; bit for bit in
the backward's deterministic mode).
This module only draws the views and passes pointers; nothing of a step is
computed in Python.
"""
from __future__ import annotations

import math

import numpy as np

from . import hgs

# Per-group learning rates: scale and opacity are stored activated (metres,
# |o|), so their steps are smaller than 3D Gaussian Splatting's rates for the
# pre-activation values.
DEFAULT_LR = dict(mean=1e-3, scale=5e-4, rot=1e-3, opacity=5e-3, sh=2.5e-3)


def log_uniform_tau(rng: np.random.Generator, n: int, tau_min: float, tau_max: float) -> np.ndarray:
    """n target granularities drawn uniformly in log tau over [tau_min, tau_max]."""
    if not (0.0 < tau_min <= tau_max):
        raise ValueError("need 0 < tau_min <= tau_max")
    u = rng.random(n)
    return np.exp(math.log(tau_min) + u * (math.log(tau_max) - math.log(tau_min)))


class HierarchyOptimizer:
    """Optimises the interior nodes of the hierarchy uploaded to ``renderer``.

    params: dict of the bound parameter tensors (``hgs.params_to_device``,
    then ``renderer.bind``); they are updated in place.  train_views: the
    training cameras (``synth.View``-like); targets: one float32 [H, W, 3]
    CUDA tensor per training view.  Each step draws ``batch`` distinct
    training views (all of them when there are fewer), gives each a tau
    drawn log-uniform over ``tau_range`` and takes one Adam step (fused
    into the backward unless ``fused`` is False).
    """

    def __init__(self, renderer: hgs.Renderer, params: dict, train_views, targets, lr=None,
                 tau_range=(3.0, 15.0), batch: int = 32, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-15, seed: int = 0, fused: bool = True):
        import torch
        if len(train_views) != len(targets) or not train_views:
            raise ValueError("one target image per training view, at least one view")
        for v, t in zip(train_views, targets):
            if not (t.is_cuda and t.dtype == torch.float32 and tuple(t.shape) == (v.height, v.width, 3)):
                raise ValueError("targets must be float32 CUDA tensors of the views' [H, W, 3]")
        self.r = renderer
        self.params = params
        self.views = list(train_views)
        self.targets = [t.contiguous() for t in targets]
        self.lr = dict(DEFAULT_LR) if lr is None else lr
        self.tau_range = (float(tau_range[0]), float(tau_range[1]))
        self.batch = int(batch)
        self.beta1, self.beta2, self.eps = beta1, beta2, eps
        self.rng = np.random.default_rng(seed)
        self.m, self.v = renderer.adam_moments(params)  # one row per interior node
        self.fused = bool(fused)
        self.grads = None if self.fused else {k: torch.zeros_like(t) for k, t in params.items()}
        self.t = 0  # Adam's step count
        self._imgs = {}
        self._dl = {}
        self.loss = torch.zeros((), dtype=torch.float64, device=params["mean"].device)

    def sample(self):
        """The next batch: (indices of the training views, their views with
        the drawn tau)."""
        n = min(self.batch, len(self.views))
        idx = self.rng.choice(len(self.views), size=n, replace=False)
        taus = log_uniform_tau(self.rng, n, *self.tau_range)
        return idx, [self.views[i].replace(tau=float(tau)) for i, tau in zip(idx, taus)]

    def _buffers(self, views, store):
        import torch
        out = []
        count = {}
        for v in views:
            key = (v.height, v.width)
            k = count.get(key, 0)
            count[key] = k + 1
            lst = store.setdefault(key, [])
            if len(lst) <= k:
                lst.append(torch.empty((v.height, v.width, 3), dtype=torch.float32, device=self.loss.device))
            out.append(lst[k])
        return out

    def step(self, idx=None, views=None):
        """One iteration on the batch (idx, views) (default: ``sample()``).
        Returns the batch's loss as a float64 CUDA scalar (not synchronised)
        and the batch."""
        if views is None:
            idx, views = self.sample()
        imgs = self._buffers(views, self._imgs)
        dL = self._buffers(views, self._dl)
        self.r.render(views, out=imgs)
        loss = self.loss.clone()
        self.r.l1_loss([self.targets[i] for i in idx], dL, loss)
        self.t += 1
        if self.fused:
            self.r.backward_adam_step(dL, self.params, self.m, self.v, self.lr, self.t, self.beta1, self.beta2,
                                      self.eps)
        else:
            self.r.backward(dL, self.grads)
            self.r.adam_step(self.params, self.grads, self.m, self.v, self.lr, self.t, self.beta1, self.beta2,
                             self.eps)
        return loss, (idx, views)
