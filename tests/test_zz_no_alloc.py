"""The allocation-free preconditioner apply against the allocating one,
through the C interface: two calls in a row (the second with fewer right-hand
sides on a smaller handle), FP64 and mixed, and the size limit of its static
scratch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2412_19207_amd import binding
from paper_2412_19207_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()


def _noalloc(s, r):
    z = torch.full((s.info.P, r.shape[1]), float("nan"), dtype=torch.float64, device=DEV)
    binding.rann_dd_apply_precond_noalloc(s.handle, r.contiguous().data_ptr(), r.shape[1], z.data_ptr())
    torch.cuda.synchronize()
    return z


@pytest.mark.parametrize("precision,precond", [("fp64", "as"), ("fp64", "ras"), ("mixed", "sas")])
def test_noalloc_apply_matches_allocating_apply(precision, precond):
    _need_gpu()
    rng = np.random.default_rng(31)
    big = binding.Solver(wl.small3d(l=(3, 3, 3)), device=DEV, precision=precision, precond=precond)
    big.pca(1e-10)
    small = binding.Solver(wl.small2d(), device=DEV, precision=precision, precond=precond)
    small.pca(1e-10)
    for s, k in [(big, 17), (small, 3)]:
        r = torch.as_tensor(rng.standard_normal((s.info.P, k)), device=DEV)
        z_ref = s.apply_precond(r)
        z = _noalloc(s, r)
        assert torch.equal(z, z_ref), float((z - z_ref).abs().max())
    big.close()
    small.close()


def test_noalloc_rejects_inputs_beyond_its_scratch():
    _need_gpu()
    s = binding.Solver(wl.small2d(), device=DEV)
    s.pca(1e-10)
    k = 4096
    r = torch.zeros((s.info.P, k), dtype=torch.float64, device=DEV)
    z = torch.zeros_like(r)
    rc = binding.load().rann_dd_apply_precond_noalloc(s.handle, ctypes.c_void_p(r.data_ptr()), k,
                                                      ctypes.c_void_p(z.data_ptr()))
    assert rc == binding.RANN_EINVAL
    assert "scratch" in binding.rann_dd_last_error()
    s.close()
