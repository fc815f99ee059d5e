"""The allocation-free product (pvfl_matmul_ct_pt_noalloc, workspace in the
library's fixed device array) against the allocating entry point
(pvfl_matmul_ct_pt) through the C ABI: bit-equal outputs on two calls in a
row, the second with a smaller product, so the second call runs over what the
first left in the shared array.  Needs an MI355X."""
import numpy as np
import pytest

from paper_2405_00482_amd import pvfl

from gpu_util import context, dev_f64, dev_i64, torch

pytestmark = pytest.mark.gpu


def _inputs(ctx, sk, plan, seed):
    rng = np.random.default_rng(seed)
    info = plan.info
    K = info["pt_limbs"]
    ct = dev_f64(plan.bytes("ct_in") // 8)
    Q2 = 2 * (ctx.L + 1) * ctx.N
    for c in range(info["ct_in"]):
        ctx.encrypt_coeffs(sk, ctx.L, dev_i64(rng.integers(-2 ** 40, 2 ** 40, ctx.N)), seed + c, ct[c * Q2:(c + 1) * Q2])
    pt = dev_f64(plan.bytes("pt") // 8)
    ctx.pt_import(ctx.L, K > ctx.L + 1, dev_i64(rng.integers(-2 ** 40, 2 ** 40, (info["n_pts"], ctx.N))), pt)
    return ct, pt


@pytest.mark.parametrize("name,shapes,lazy", [
    ("C3", [(256, 2048), (64, 512)], True),       # m' = 64 then m' = 4
    ("C4", [(300, 700), (16, 4096)], True),       # three special primes: m' = 64 then m' = 8
    ("C1", [(64, 256), (16, 64)], False),         # per-rotation ModDown: m' = 8 then m' = 1
])
def test_noalloc_matches_allocating_entry_point(name, shapes, lazy):
    ctx = context(name)
    sk = ctx.keygen(5)
    plans = [ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=lazy) for (m, n) in shapes]
    assert plans[1].info["n_pts"] < plans[0].info["n_pts"]          # the second product is the smaller one
    assert plans[1].bytes("workspace") <= plans[0].bytes("workspace")
    for p in plans:
        assert p.bytes("workspace") <= pvfl.noalloc_max_bytes()
    gal = sorted(set(g for p in plans for g in p.galois()))
    keys = ctx.rotkeys(sk, gal, 6)
    for k, p in enumerate(plans):
        ct, pt = _inputs(ctx, sk, p, 100 + k)
        want = dev_f64(p.bytes("ct_out") // 8)
        p.matmul(ct, pt, keys, want)
        got = dev_f64(p.bytes("ct_out") // 8).fill_(float("nan"))
        p.matmul_noalloc(ct, pt, keys, got)
        torch().cuda.synchronize()
        assert torch().equal(got, want), f"call {k} ({shapes[k]}): the allocation-free product differs"


def test_noalloc_refuses_what_does_not_fit():
    ctx = context("C5")
    big = ctx.plan(pvfl.PLAN_HYBRID, 65536, 65536, lazy=True)       # four column blocks at N/2 = 16384
    assert big.bytes("workspace") > pvfl.noalloc_max_bytes()
    t = torch()
    one = t.zeros(1, dtype=t.float64, device="cuda")
    bufs = [dev_f64(big.bytes(w) // 8) if w != "pt" else one for w in ("ct_in", "pt", "ct_out")]
    with pytest.raises(pvfl.PvflError) as e:   # the library's own check, before keys or buffers are read
        pvfl._check(pvfl.lib().pvfl_matmul_ct_pt_noalloc(big.h, pvfl._ptr(bufs[0]), pvfl._ptr(bufs[1]), None,
                                                          pvfl._ptr(bufs[2]), pvfl._stream()))
    assert e.value.status == -2
    row = ctx.plan(pvfl.PLAN_ROW, 4, 8)
    with pytest.raises(pvfl.PvflError) as e:
        pvfl._check(pvfl.lib().pvfl_matmul_ct_pt_noalloc(row.h, pvfl._ptr(one), pvfl._ptr(one), None,
                                                          pvfl._ptr(one), pvfl._stream()))
    assert e.value.status == -7
