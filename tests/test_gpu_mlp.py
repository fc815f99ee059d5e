"""The latency network's HIP forward, backward and Adam kernels against the
FP64 reference (oracle/mlp.py, itself pinned to finite differences).  FP32
sums over at most 64 terms: relative error well under 1e-4."""
import numpy as np
import pytest

from oracle import mlp as R
from paper_2405_00482_amd import pvfl

from gpu_util import torch

pytestmark = pytest.mark.gpu


def _close(got, want, rtol, what):
    got = np.asarray(got, dtype=np.float64)
    scale = max(1.0, float(np.max(np.abs(want))))
    err = float(np.max(np.abs(got - want))) / scale
    assert err < rtol, f"{what}: max error {err:.3g} relative to {scale:.3g}"


@pytest.mark.parametrize("F,H,B", [(21, 64, 256), (5, 64, 1), (64, 64, 33), (3, 17, 10)])
def test_forward_and_gradient_match_reference(F, H, B):
    t = torch()
    net = pvfl.Mlp(F, H, max_batch=256, seed=F * 100 + H)
    rng = np.random.default_rng(B)
    x = rng.standard_normal((B, F)).astype(np.float32)
    tgt = rng.standard_normal(B).astype(np.float32)
    xd, td = t.from_numpy(x).cuda(), t.from_numpy(tgt).cuda()
    p = net.get_params().cpu().numpy().astype(np.float64)
    assert p.size == R.n_params(F, H)
    y = net.forward(xd)
    t.cuda.synchronize()
    _close(y.cpu().numpy(), R.forward(p, F, H, x), 1e-5, "forward")
    g, loss = net.grad(xd, td)
    t.cuda.synchronize()
    gw, lw = R.grad(p, F, H, x, tgt)
    _close(g.cpu().numpy(), gw, 1e-5, "gradient")
    assert abs(float(loss.item()) - lw) <= 1e-5 * max(1.0, lw)


def test_adam_steps_match_reference():
    t = torch()
    F, H, B = 12, 64, 64
    net = pvfl.Mlp(F, H, max_batch=B, seed=7)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((B, F)).astype(np.float32)
    tgt = rng.standard_normal(B).astype(np.float32)
    xd, td = t.from_numpy(x).cuda(), t.from_numpy(tgt).cuda()
    p = net.get_params().cpu().numpy().astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 4):
        # gradient taken from the device at the device's current parameters,
        # so the comparison isolates the update rule
        g, _ = net.grad(xd, td)
        g = g.cpu().numpy().astype(np.float64)
        net.train_step(xd, td, 1e-3)
        p, m, v = R.adam_step(p, m, v, g, step, 1e-3)
        got = net.get_params().cpu().numpy()
        _close(got, p, 1e-5, f"parameters after Adam step {step}")
        p = got.astype(np.float64)


def test_training_fits_a_smooth_target():
    t = torch()
    F, H, B = 4, 64, 512
    net = pvfl.Mlp(F, H, max_batch=B, seed=1)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (B, F)).astype(np.float32)
    tgt = (x[:, 0] * 2 - x[:, 1] ** 2 + 0.5 * np.abs(x[:, 2])).astype(np.float32)
    xd, td = t.from_numpy(x).cuda(), t.from_numpy(tgt).cuda()
    first = float(net.train_step(xd, td, 3e-3).item())
    for _ in range(1500):
        last = net.train_step(xd, td, 3e-3)
    last = float(last.item())
    assert last < 0.02 * first and last < 5e-3


def test_rejects_oversized_batch():
    t = torch()
    net = pvfl.Mlp(3, 8, max_batch=4)
    x = t.zeros((5, 3), dtype=t.float32, device="cuda")
    with pytest.raises(pvfl.PvflError):
        net.grad(x, t.zeros(5, dtype=t.float32, device="cuda"))
