"""Plain bmDCA training of one model (Secs. 2.1-2.3 of the paper).

From an alignment to a trained Potts model:

  1. sequence weights at identity threshold `theta` (Eq. 7, bmdca_reweight);
  2. one- and two-site frequencies with pseudocount (Eqs. 3, 8-9,
     bmdca_stats);
  3. the profile model as the start, h_i(a) = log f_i(a) and J = 0
     (bmdca_profile_fields), and N persistent chains drawn uniformly;
  4. epochs of `sweeps` Gibbs sweeps, chain statistics and the update of
     Eq. (5) until the Pearson coefficient of Eq. (6) reaches `target`
     (the convergence criterion of Sec. 2.1), or `max_epochs`.

The epoch is one captured graph (bmdca_train_group_graph over one model):
its device control record carries the epoch index, and a one-thread kernel at
the end of the epoch stops the model once the target is reached, so replays
after convergence change nothing.  The host replays `check_every` epochs at a
time and reads the record back between batches.  Every step runs in the HIP
library; this module only sequences the calls.
"""
from __future__ import annotations

import torch

from . import _lib as B
from . import api


def bmdca(msa, q: int, theta: float = 0.8, pseudocount: float = -1.0, chains: int = 10000,
          sweeps: int = 10, lr: float = 0.05, target: float = 0.95, max_epochs: int = 10000,
          seed: int = 0, prec="bf16x2", sampler="auto", check_every: int = 10):
    """Trains a model on `msa` (int8 [M, L] on the GPU). Returns (h float32
    [L, q], J float32 [Lq, Lq], chains int8 [N, L], history of (epoch,
    Pearson) read back every `check_every` epochs, epochs run).  Raises
    DeviceError when a kernel flags a token outside 0..q-1 or a non-finite
    parameter or Pearson value (read with every batch of epochs)."""
    api._dev(msa, torch.int8, "msa", 2)
    M, L = msa.shape
    dev = msa.device
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    _, w, _ = api.reweight(msa, q, theta, dev_err=err)
    f1, f2, _ = api.stats(msa, q, w, pseudocount, prec, dev_err=err)
    h = api.profile_fields(f1, L, q, dev_err=err)
    J = torch.zeros((L * q, L * q), dtype=torch.float32, device=dev)
    _raise_on(err, "pre-processing")
    ch = api.init_chains(chains, L, q, seed, device=dev)
    model = api.TrainModel(h, J, ch, f1, f2, lr, sweeps, seed, prec, sampler=sampler,
                           target_pearson=target, dev_err=err)
    graph = api.TrainGroupGraph([model], lanes=1)
    history = []
    try:
        done = 0
        while done < max_epochs:
            n = min(check_every, max_epochs - done)
            for _ in range(n):
                graph.launch()
            done += n
            rec = api.read_ctl(model.ctl)
            history.append((rec["epoch"], float(model.pearson.item())))
            _raise_on(err, f"epoch {rec['epoch']}")
            if not rec["active"]:
                break
    finally:
        graph.close()
    return h, J, ch, history, api.read_ctl(model.ctl)["epoch"]


class DeviceError(RuntimeError):
    """A kernel raised the device error flag (bits BMDCA_DEVERR_*)."""


def _raise_on(err, where: str) -> None:
    bits = int(err.item())
    if bits:
        names = [n for b, n in ((B.DEVERR_TOKEN, "token outside 0..q-1"),
                                (B.DEVERR_NONFINITE, "non-finite parameter or Pearson value"),
                                (B.DEVERR_INDEX, "index out of range")) if bits & b]
        raise DeviceError(f"{where}: device flag {bits:#x} ({', '.join(names)})")
