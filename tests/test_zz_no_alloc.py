"""The allocation-free operator apply (rs_apply_dev_noalloc) against rs_apply.

The entry point keeps its intermediates in a fixed per-device array instead of
allocated memory; the array keeps the last call's contents.  Two calls in a
row, the second with a smaller input, must each give what rs_apply gives (the
same kernels: bitwise), and a request beyond the array's size is refused."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from workloads import workload_circle10_8holes, workload_small


def _solver(g, **kw):
    import torch

    assert torch.cuda.is_available()
    from paper_2001_11619_amd import RSSolver

    return RSSolver.from_geometry(g, **kw)


def _noalloc(s, X):
    import torch

    xd = torch.tensor(np.ascontiguousarray(X.T), dtype=torch.float64, device="cuda")
    yd = torch.full_like(xd, np.nan)
    torch.cuda.synchronize()
    s.apply_dev_noalloc(xd, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy().T.copy()


def test_noalloc_apply_matches_rs_apply_twice():
    rng = np.random.Generator(np.random.PCG64(17))
    big = _solver(workload_small(seed=11, n_outer=512, n_holes=3, nodes_per_hole=160, radius=3.0), leaf_size=32)
    small = _solver(workload_small(seed=12, n_outer=192, n_holes=1, nodes_per_hole=96, radius=3.0), leaf_size=32)
    Xb = rng.standard_normal((big.n_system, 5))
    Xs = rng.standard_normal((small.n_system, 2))
    yb = _noalloc(big, Xb)
    ys = _noalloc(small, Xs)            # second call, smaller input, same array
    assert np.array_equal(yb, big.apply(Xb))
    assert np.array_equal(ys, small.apply(Xs))
    # and again on the first context with fewer columns
    assert np.array_equal(_noalloc(big, Xb[:, :1]), big.apply(Xb[:, :1]))


def test_noalloc_apply_rejects_oversized_request():
    from paper_2001_11619_amd import RSError

    import torch

    s = _solver(workload_circle10_8holes())
    X = np.ones((s.n_system, 16))
    xd = torch.tensor(np.ascontiguousarray(X.T), dtype=torch.float64, device="cuda")
    yd = torch.zeros_like(xd)
    with pytest.raises(RSError) as e:
        s.apply_dev_noalloc(xd, yd)
    assert e.value.name == "RS_ERR_ARG"
    torch.cuda.synchronize()
    assert float(yd.abs().max()) == 0.0       # nothing written
    # a size that fits (6 columns) works on the same context
    X6 = np.random.Generator(np.random.PCG64(2)).standard_normal((s.n_system, 6))
    assert np.array_equal(_noalloc(s, X6), s.apply(X6))
