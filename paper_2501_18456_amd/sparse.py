"""Sparse models by element decimation (edDCA, Sec. 2.4 of the paper).

Starting from a trained fully connected model and its chains, alternate

  1. graph update: remove the `drate` fraction of active coupling elements
     with the smallest symmetric Kullback-Leibler distance between the model
     and the model without the element (bmdca_decimate);
  2. parameter updates on the fixed graph (bmdca_train_step_masked), `gsteps`
     at a time, until the Pearson coefficient of Eq. (6) reaches `target`;

until the density (active elements / L (L-1) q^2 / 2) reaches `density`.
Every step runs in the HIP library; this module sequences the calls and reads
back the Pearson value and the active count once per round.
"""
from __future__ import annotations

import math

import torch

from . import _lib as B
from . import api


def decimation(h, J, chains, f1, f2, lr: float, sweeps: int, seed: int, drate: float = 0.01,
               density: float = 0.02, target: float = 0.95, gsteps: int = 10,
               max_epochs: int = 10000, prec="bf16x2", sampler="auto", mask=None,
               epoch0: int = 0):
    """Decimates in place (h, J, chains, mask).  Returns (mask, history of
    (epoch, active elements, Pearson), epochs used)."""
    L, q = api._model(h, J)
    N = chains.shape[0]
    dev = chains.device
    if mask is None:
        mask = api.full_mask(L, q, dev)
        J.mul_(mask.to(J.dtype))
    n_total = L * (L - 1) // 2 * q * q
    n_target = math.ceil(density * n_total)
    ws_t = api.workspace(B.WS_TRAIN_STEP, N, L, q, api._prec(prec) | api._sampler(sampler), dev)
    ws_d = api.workspace(B.WS_DECIMATE, N, L, q, 0, dev)
    pearson = torch.empty(1, dtype=torch.float64, device=dev)
    n_act_d = torch.empty(1, dtype=torch.int64, device=dev)
    epoch = epoch0
    n_act = int((torch.triu(mask, 1) != 0).sum().item())
    history = []
    while True:
        r = -1.0
        while epoch - epoch0 < max_epochs:
            for _ in range(gsteps):
                api.train_step_masked(h, J, mask, chains, f1, f2, lr, sweeps, seed, epoch, prec,
                                      ws_t, pearson, sampler=sampler)
                epoch += 1
            r = float(pearson.item())
            if r >= target:
                break
        history.append((epoch, n_act, r))
        if n_act <= n_target or epoch - epoch0 >= max_epochs:
            return mask, history, epoch - epoch0
        api.decimate(J, mask, chains, q, drate, density, ws_d, n_active=n_act_d)
        n_act = int(n_act_d.item())
