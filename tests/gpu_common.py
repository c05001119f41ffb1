"""Shared helpers of the GPU parity tests (inputs come from the seeded
generators; expected values from the FP64 oracle)."""
import numpy as np
import pytest

from paper_1304_4333_amd import synth


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def make_ctx(X, y, C, prior_sd=5.0):
    import torch
    from paper_1304_4333_amd import sps
    ctx = sps.Context(0)
    Xg = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    yg = torch.from_numpy(np.ascontiguousarray(y, dtype=np.int32)).cuda()
    sps.sps_set_data(ctx, Xg, yg, C)
    sps.sps_set_prior(ctx, 0.0, prior_sd)
    ctx._keep = (Xg, yg)
    return ctx


def dataset(T, k, C, seed, design="gauss"):
    """A small logit data set of the requested shape (random-utility draws)."""
    w = synth.Workload("t", C=C, T=T, k=k, J=1, N=1, prior_sd=5.0, design=design,
                       beta_sd=0.7, n_dummy=min(3, max(0, k - 2)), dummy_p=0.3,
                       data_seed=seed)
    X, y, B = synth.make_data(w)
    return X, y, B


def to_gpu(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def check_nse_bar(z, zl=None, what=""):
    """The end-to-end bar of 3 numerical standard errors: every |z| of the
    monitored moments within 3, with at most one exceedance (multiplicity over
    up to 31 moments with t-distributed z), and the logML's |z| within 3."""
    z = np.abs(np.asarray(z, dtype=float))
    print(f"{what} max |z| {z.max():.2f}, exceedances {int((z > 3).sum())}"
          + ("" if zl is None else f", logML |z| {abs(zl):.2f}"), flush=True)
    assert int((z > 3.0).sum()) <= 1, np.round(z, 2)
    if zl is not None:
        assert abs(zl) <= 3.0
