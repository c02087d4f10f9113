"""bmdca_energy_noalloc (scratch in the library's static device array, no
workspace argument) against bmdca_energy through the C ABI: the same bits on
two calls in a row, the second with a smaller input; an oversized batch is
refused before anything runs."""
import numpy as np
import pytest
import torch

from paper_2501_18456_amd import _lib as B
from paper_2501_18456_amd import api, synth

pytestmark = pytest.mark.gpu


def _noalloc(h, J, S, E, err):
    L, q = h.shape
    return B.lib().bmdca_energy_noalloc(h.data_ptr(), J.data_ptr(), S.data_ptr(), S.shape[0], L,
                                        q, E.data_ptr(), err.data_ptr(),
                                        torch.cuda.current_stream().cuda_stream)


def test_energy_noalloc_equals_energy():
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    for (L, q, n, seed) in [(300, 21, 20000, 1), (64, 5, 777, 2)]:  # second call smaller
        h, J = synth.planted_dense(L, q, seed=500 + seed, sigma_J=0.1)
        hg, Jg = torch.from_numpy(h).cuda(), torch.from_numpy(J).cuda()
        S = torch.from_numpy(synth.random_sequences(n, L, q, 600 + seed)).cuda()
        ref = api.energy(hg, Jg, S)
        E = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
        assert _noalloc(hg, Jg, S, E, err) == B.OK, B.lib().bmdca_last_error()
        torch.cuda.synchronize()
        assert torch.equal(E, ref), f"L={L} n={n}"
    assert int(err.item()) == 0


def test_energy_noalloc_refuses_batches_beyond_the_scratch():
    L, q = 512, 21
    n = 43649  # one more sequence than the 64 MiB array holds at L = 512
    h = torch.zeros((L, q), dtype=torch.float32, device="cuda")
    J = torch.zeros((L * q, L * q), dtype=torch.float32, device="cuda")
    S = torch.zeros((n, L), dtype=torch.int8, device="cuda")
    E = torch.full((n,), 7.0, dtype=torch.float32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert _noalloc(h, J, S, E, err) == B.EINVAL
    assert b"static" in B.lib().bmdca_last_error()
    torch.cuda.synchronize()
    assert bool((E == 7.0).all())  # nothing ran
    # the largest batch that fits runs
    assert _noalloc(h, J, S[:43648], E[:43648], err) == B.OK
    torch.cuda.synchronize()
    assert bool((E[:43648] == 0.0).all())
