"""The batched form (one launch per phase over many products, shared keys,
optional HIP-graph replay) computes exactly what the per-call form computes.
The per-call form is itself bit-exact against the oracle (test_gpu_parity).
Needs an MI355X."""
import numpy as np
import pytest

from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import workloads as W

from gpu_util import context, torch

pytestmark = pytest.mark.gpu


def _setup(name, shapes, seed=0):
    t = torch()
    ctx = context(name)
    sk = ctx.keygen(3)
    plans = [ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True) for (m, n) in shapes]
    gal = sorted(set(g for p in plans for g in p.galois()))
    keys = ctx.rotkeys(sk, gal, 4)
    rng = np.random.default_rng(seed)
    X = [t.from_numpy(rng.standard_normal((m, n))).cuda() for (m, n) in shapes]
    v = [t.from_numpy(rng.uniform(-1, 1, n)).cuda() for (m, n) in shapes]

    def bufs():
        f = dict(dtype=t.float64, device="cuda")
        return ([t.zeros(p.bytes("pt") // 8, **f) for p in plans], [t.zeros(p.bytes("ct_in") // 8, **f) for p in plans],
                [t.zeros(p.bytes("ct_out") // 8, **f) for p in plans], [t.zeros(m, **f) for (m, n) in shapes])
    return ctx, sk, plans, keys, X, v, bufs


def _percall(plans, sk, keys, X, v, bufs, seed):
    pt, ct, out, y = bufs()
    for k, p in enumerate(plans):
        p.encode_pt(X[k], pt[k])
        p.encrypt(sk, v[k], seed + k, ct[k])
        p.matmul(ct[k], pt[k], keys, out[k])
        p.decrypt_decode(sk, out[k], y[k])
    torch().cuda.synchronize()
    return pt, ct, out, y


def _same(a, b, what):
    for k, (x, z) in enumerate(zip(a, b)):
        assert torch().equal(x, z), f"{what} of product {k} differs"


@pytest.mark.parametrize("name,shapes,group,chunk,vec", [
    ("C1", [(16, 256), (100, 37), (64, 64), (8, 2048)], 2, 4, 1),
    ("C1", [(16, 256), (100, 37), (64, 64), (8, 2048)], 4, 64, 2),
    ("C1", [(16, 256), (100, 37), (64, 64), (8, 2048)], 2, 5, 2),     # odd chunk
    ("C3", W.c3_shapes(64)[:6], 4, 16, 2),
    ("C3", W.c3_shapes(64)[:6], 1, 1024, 1),
    ("C3", W.c3_shapes(64)[:6], 4, 7, 1),
    ("C4", [(16, 256), (3, 5), (300, 700)], 2, 32, 2),     # three special primes, two digits
    ("C4", [(16, 256), (3, 5), (300, 700)], 2, 9, 2),
    ("C5", [(16, 4096), (3, 5), (40, 1000)], 2, 32, 1),    # ring 2^15, split transforms
    ("C5", [(16, 4096), (3, 5), (40, 1000)], 2, 3, 2),
])
def test_batch_equals_percall(name, shapes, group, chunk, vec):
    ctx, sk, plans, keys, X, v, bufs = _setup(name, shapes)
    seed = 500
    ref = _percall(plans, sk, keys, X, v, bufs, seed)
    pt, ct, out, y = bufs()
    b = pvfl.Batch(ctx, plans, X=X, v=v, pt=pt, ct=ct, out=out, y=y, keys=keys, group=group, chunk=chunk, vec=vec)
    b.encode()
    b.encrypt(sk, seed)
    b.matmul()
    b.decrypt(sk)
    torch().cuda.synchronize()
    _same(pt, ref[0], "plaintexts")
    _same(ct, ref[1], "ciphertexts")
    _same(out, ref[2], "products")
    _same(y, ref[3], "decoded results")
    for k, (m, n) in enumerate(shapes):
        r = X[k].cpu().numpy() @ v[k].cpu().numpy()
        assert np.linalg.norm(y[k].cpu().numpy() - r) / np.linalg.norm(r) < 2.0 ** -20


def test_batch_graph_replays_match_eager():
    shapes = [(16, 256), (100, 37), (64, 64)]
    ctx, sk, plans, keys, X, v, bufs = _setup("C1", shapes, seed=1)
    pt, ct, out, y = bufs()
    b = pvfl.Batch(ctx, plans, X=X, v=v, pt=pt, ct=ct, out=out, y=y, keys=keys, group=2, chunk=8)
    b.run(sk, 77, graph=False)
    torch().cuda.synchronize()
    eager = [t.clone() for t in out] + [t.clone() for t in y]
    for rep in range(3):
        for t in out + y:
            t.zero_()
        torch().cuda.synchronize()
        b.run(sk, 77, graph=True)
        torch().cuda.synchronize()
        got = list(out) + list(y)
        for a, e in zip(got, eager):
            assert torch().equal(a, e), f"graph replay {rep} differs from the eager batch"
        # eager work between replays
        _ = (X[0] * 2).sum().item()


def test_batch_rejects_bad_plans():
    ctx = context("C1")
    sk = ctx.keygen(3)
    p_eager = ctx.plan(pvfl.PLAN_HYBRID, 16, 64, lazy=False)
    t = torch()
    f = dict(dtype=t.float64, device="cuda")
    bufs = [t.zeros(p_eager.bytes(w) // 8, **f) for w in ("pt", "ct_in", "ct_out")]
    with pytest.raises(pvfl.PvflError) as e:
        pvfl.Batch(ctx, [p_eager], pt=[bufs[0]], ct=[bufs[1]], out=[bufs[2]])
    assert e.value.status == -7
    p = ctx.plan(pvfl.PLAN_HYBRID, 16, 512, lazy=True)
    bufs = [t.zeros(p.bytes(w) // 8, **f) for w in ("pt", "ct_in", "ct_out")]
    with pytest.raises(pvfl.PvflError) as e:   # rotations needed, no keys given
        pvfl.Batch(ctx, [p], pt=[bufs[0]], ct=[bufs[1]], out=[bufs[2]])
    assert e.value.status == -4


def test_batch_without_rotations_needs_no_keys():
    """every product with m' = 1 (no rotation): the batch runs with no key set
    and equals the per-call form"""
    shapes = [(3, 5), (16, 64), (1, 1)]
    t = torch()
    ctx = context("C1")
    sk = ctx.keygen(3)
    plans = [ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True) for (m, n) in shapes]
    assert all(p.info["mprime"] == 1 and not p.galois() for p in plans)
    rng = np.random.default_rng(9)
    f = dict(dtype=t.float64, device="cuda")
    X = [t.from_numpy(rng.standard_normal((m, n))).cuda() for (m, n) in shapes]
    v = [t.from_numpy(rng.uniform(-1, 1, n)).cuda() for (m, n) in shapes]

    def bufs():
        return ([t.zeros(p.bytes("pt") // 8, **f) for p in plans], [t.zeros(p.bytes("ct_in") // 8, **f) for p in plans],
                [t.zeros(p.bytes("ct_out") // 8, **f) for p in plans], [t.zeros(m, **f) for (m, n) in shapes])
    ref = _percall(plans, sk, None, X, v, bufs, 40)
    pt, ct, out, y = bufs()
    b = pvfl.Batch(ctx, plans, X=X, v=v, pt=pt, ct=ct, out=out, y=y, keys=None, group=2, chunk=8, vec=2)
    b.run(sk, 40, graph=False)
    t.cuda.synchronize()
    _same(out, ref[2], "products")
    _same(y, ref[3], "decoded results")
