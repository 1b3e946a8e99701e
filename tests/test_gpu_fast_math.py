"""Accuracy of the FP64 reciprocal and square root the face-once stage
kernels use in place of division and sqrt (hardware estimates refined by
Newton-Raphson and Goldschmidt iterations), against IEEE correctly rounded
1/x and sqrt(x) (numpy) on 10^6 inputs over the ranges the solver meets:
densities, pressures and squared speeds in code units from 1e-12 to 1e8,
the whole normal range, and the floor used for square roots that may be
zero (1e-280)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _ulps(a, b):
    """Distance in units in the last place between positive doubles."""
    ia = a.view(np.int64)
    ib = b.view(np.int64)
    return np.abs(ia - ib)


def test_rcp_and_sqrt_are_within_one_ulp():
    import torch
    from paper_2501_15923_amd import _abi
    rng = np.random.default_rng(11)
    n = 1 << 20
    x = np.concatenate([
        10.0 ** rng.uniform(-12, 8, n // 2),               # solver quantities
        10.0 ** rng.uniform(-300, 300, n // 4),            # the normal range
        rng.uniform(1.0, 2.0, n // 4 - 3),                 # one binade, dense
        [1e-280, 1.0, 4.0]])
    xd = torch.from_numpy(x).cuda()
    rd = torch.empty_like(xd)
    sd = torch.empty_like(xd)
    stream = torch.cuda.current_stream().cuda_stream
    _abi.check(_abi.lib().icr_fast_math(_abi.dptr(xd.data_ptr()), len(x),
                                        _abi.dptr(rd.data_ptr()), _abi.dptr(sd.data_ptr()),
                                        stream))
    rcp = rd.cpu().numpy()
    sq = sd.cpu().numpy()
    ur = _ulps(rcp, 1.0 / x)
    us = _ulps(sq, np.sqrt(x))
    print(f"rcp: max {ur.max()} ulp, {np.count_nonzero(ur)} of {len(x)} not correctly rounded; "
          f"sqrt: max {us.max()} ulp, {np.count_nonzero(us)} not correctly rounded", flush=True)
    assert ur.max() <= 1 and us.max() <= 1
    # nearly all results are the correctly rounded ones
    assert np.count_nonzero(ur) <= 1e-3 * len(x)
    assert np.count_nonzero(us) <= 1e-3 * len(x)
    assert sq[-1] == 2.0 and rcp[-2] == 1.0
