"""Sparse models (Sec. 2.2 of the paper, options in Sec. 3.1 and 3.2): element decimation (edDCA) and
element activation (eaDCA).

edDCA starts from a trained fully connected model and its chains and
alternates

  1. graph update: remove the `drate` fraction of active coupling elements
     with the smallest symmetric Kullback-Leibler distance between the model
     and the model without the element (bmdca_decimate);
  2. parameter updates on the fixed graph (bmdca_train_step_masked), `gsteps`
     at a time, until the Pearson coefficient of Eq. (6) reaches `target`;

until the density (active elements / L (L-1) q^2 / 2) reaches `density`.

eaDCA starts from an empty graph (a profile model) and alternates

  1. graph update: activate the elements whose model pairwise marginal is
     farthest from the data's, as many as the `factivate` fraction of the
     inactive ones (bmdca_activate);
  2. `gsteps` parameter updates on the fixed graph;

until the Pearson coefficient reaches `target`.

Every step runs in the HIP library; these functions sequence the calls and
read back the Pearson value and the active count once per round.
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
    n_act_d = api.mask_apply(J, mask, q)  # couplings off the graph are 0
    n_total = L * (L - 1) // 2 * q * q
    n_target = math.ceil(density * n_total)
    ws_t = api.workspace(B.WS_TRAIN_STEP, N, L, q, api._prec(prec) | api._sampler(sampler), dev)
    ws_d = api.workspace(B.WS_DECIMATE, N, L, q, 0, dev)
    pearson = torch.empty(1, dtype=torch.float64, device=dev)
    epoch = epoch0
    n_act = int(n_act_d.item())
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


def activation(h, J, chains, f1, f2, lr: float, sweeps: int, seed: int, factivate: float = 0.001,
               target: float = 0.95, gsteps: int = 10, max_epochs: int = 10000, prec="bf16x2",
               sampler="auto", mask=None, epoch0: int = 0):
    """eaDCA in place on (h, J, chains, mask); without a mask the graph starts
    empty (J is zero off the graph).  Returns (mask, history of (epoch, active
    elements, Pearson), epochs used)."""
    L, q = api._model(h, J)
    N = chains.shape[0]
    dev = chains.device
    if mask is None:
        mask = api.mask_init(L, q, full=False, device=dev)
    api.mask_apply(J, mask, q)  # couplings off the graph are 0
    ws_t = api.workspace(B.WS_TRAIN_STEP, N, L, q, api._prec(prec) | api._sampler(sampler), dev)
    ws_a = api.workspace(B.WS_DECIMATE, N, L, q, 0, dev)
    pearson = torch.empty(1, dtype=torch.float64, device=dev)
    n_act_d = torch.empty(1, dtype=torch.int64, device=dev)
    epoch = epoch0
    history = []
    while epoch - epoch0 < max_epochs:
        api.activate(mask, chains, f2, q, factivate, ws_a, n_active=n_act_d)
        for _ in range(gsteps):
            api.train_step_masked(h, J, mask, chains, f1, f2, lr, sweeps, seed, epoch, prec,
                                  ws_t, pearson, sampler=sampler)
            epoch += 1
        r = float(pearson.item())
        history.append((epoch, int(n_act_d.item()), r))
        if r >= target:
            break
    return mask, history, epoch - epoch0
