"""The allocation-free per-sample error call against the allocating one.

sf_sur_errors_noalloc keeps the network's predictions in the library's
fixed per-GPU scratch instead of handle memory; its results must equal
those of sf_sur_errors (same kernels, same inputs) bit for bit, on two calls
in a row where the second is smaller than the first, and it must never
reach the allocator.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2605_08528_amd import inputs as I
from tests.helpers import params as mkparams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


def samples(M, seed):
    rng = np.random.default_rng(seed)
    d = np.zeros((M, 20), np.float32)
    d[:, :16] = rng.uniform(-1.0, 1.0, (M, 16))
    d[:, 16:19] = rng.uniform(-1.0, 1.0, (M, 3))
    d[:, 19] = 1.0
    return d


def test_noalloc_errors_match_the_allocating_call(torch):
    from paper_2605_08528_amd import sf
    sim = sf.Sim(I.workload("plane1x2"), mkparams())
    train = torch.from_numpy(samples(4096, 1)).cuda()
    sim.sur_train(train, steps=30, batch=0, lr=1e-3, init_seed=3)
    torch.cuda.synchronize()
    blocks = set(sim._blocks)
    # first call: many tiles and a ragged tail; second call: fewer samples
    for M, seed in ((100_003, 11), (777, 12)):
        print(f"noalloc errors: M={M} seed={seed}", flush=True)
        d = torch.from_numpy(samples(M, seed)).cuda()
        out = torch.full((M,), float("nan"), dtype=torch.float32, device="cuda")
        sim.sur_errors_noalloc(d, out)
        torch.cuda.synchronize()
        assert set(sim._blocks) == blocks, "the allocation-free call reached the allocator"
        ref = sim.sur_errors(d)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref)
        blocks = set(sim._blocks)
    sim.close()


def test_noalloc_rejects_sizes_past_the_scratch(torch):
    from paper_2605_08528_amd import sf
    sim = sf.Sim(I.workload("plane1x2"), mkparams())
    d = torch.from_numpy(samples(64, 2)).cuda()
    out = torch.empty(64, dtype=torch.float32, device="cuda")
    L = sf.lib()
    # no parameters yet
    assert L.sf_sur_errors_noalloc(sim.h, C.c_void_p(d.data_ptr()), 64, C.c_void_p(out.data_ptr())) != 0
    sim.sur_train(d, steps=0, init_seed=3)
    for M in (0, -1, sf.NOALLOC_MAX_SAMPLES + 1):
        st = L.sf_sur_errors_noalloc(sim.h, C.c_void_p(d.data_ptr()), M, C.c_void_p(out.data_ptr()))
        assert st == 1, M          # SF_E_INVALID_ARG; nothing was enqueued
        assert b"out of range" in L.sf_last_error()
    assert L.sf_sur_errors_noalloc(sim.h, C.c_void_p(d.data_ptr()), 64, None) == 1
    sim.sur_errors_noalloc(d, out)
    torch.cuda.synchronize()
    assert torch.equal(out, sim.sur_errors(d))
    sim.close()
