"""sps_loglik_noalloc (no device allocation in the call) against sps_loglik,
through the C ABI: two calls in a row, the second with a smaller input, in
every precision, for binary and multinomial data.  At these sizes the
scratch does not limit the observation split, so the two entry points run
the same kernels on the same split and must agree bit for bit."""
import numpy as np
import pytest

from gpu_common import dataset, make_ctx, need_gpu, to_gpu
from paper_1304_4333_amd import synth

pytestmark = pytest.mark.gpu

@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("C,k", [(2, 30), (4, 20), (6, 50)])
def test_noalloc_matches_loglik(prec, C, k):
    need_gpu()
    import torch
    from paper_1304_4333_amd import sps
    T = 3000
    X, y, _ = dataset(T, k, C, seed=500 + C)
    d = k * (C - 1)
    ctx = make_ctx(X, y, C)
    # first call: 4096 particles over [7, 2993); second: 500 particles over [100, 900)
    for P, t0, t1, seed in ((4096, 7, 2993, 501), (500, 100, 900, 502)):
        th = to_gpu(synth.make_particles(P, d, scale=0.3 / np.sqrt(k), seed=seed))
        print(f"noalloc C={C} k={k} prec={prec} P={P} [{t0},{t1})", flush=True)
        ref = sps.sps_loglik(ctx, th, t0, t1, prec).cpu().numpy()
        out = torch.full((P,), float("nan"), dtype=torch.float64, device="cuda")
        sps.sps_loglik_noalloc(ctx, th, t0, t1, prec, out)
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref)
