"""Degenerate and invalid inputs through the C ABI: every one is refused on the
host with its status code before any kernel runs.  Needs an MI355X (a context
needs a device)."""
import numpy as np
import pytest

from paper_2405_00482_amd import pvfl

from gpu_util import context, dev_f64, torch

pytestmark = pytest.mark.gpu

E_INVALID, E_SHAPE, E_LEVEL, E_NOKEY, E_PLAN = -1, -2, -3, -4, -7


def status_of(fn):
    with pytest.raises(pvfl.PvflError) as e:
        fn()
    return e.value.status


def test_empty_and_oversized_shapes_are_refused():
    ctx = context("C1")                              # N/2 = 2048 slots
    assert status_of(lambda: ctx.plan(pvfl.PLAN_HYBRID, 0, 5)) == E_SHAPE
    assert status_of(lambda: ctx.plan(pvfl.PLAN_HYBRID, 5, 0)) == E_SHAPE
    assert status_of(lambda: ctx.plan(pvfl.PLAN_DIAG, 4096, 3)) == E_SHAPE       # DIAG does not partition
    assert status_of(lambda: ctx.plan(pvfl.PLAN_ROW, 3, 4096)) == E_SHAPE
    assert status_of(lambda: ctx.plan(pvfl.PLAN_CTMAT, 16, 64, n_out=0)) == E_SHAPE
    assert status_of(lambda: ctx.plan(pvfl.PLAN_CTMAT, 16, 64, n_out=4, pack=64)) == E_SHAPE
    assert status_of(lambda: ctx.plan(9, 16, 64)) == E_PLAN
    # the largest hybrid shapes partition instead (row and column blocks)
    p = ctx.plan(pvfl.PLAN_HYBRID, 8192, 8192)
    assert (p.info["row_blocks"], p.info["col_blocks"]) == (4, 4)


def test_levels_are_checked():
    ctx = context("C1")                              # two ciphertext primes: levels 0, 1
    assert status_of(lambda: ctx.plan(pvfl.PLAN_HYBRID, 16, 64, level=2)) == E_LEVEL
    assert status_of(lambda: ctx.plan(pvfl.PLAN_ROW, 16, 64)) == E_LEVEL     # ROW rescales twice
    p = ctx.plan(pvfl.PLAN_HYBRID, 16, 64, level=0)
    assert p.info["in_level"] == 0


def test_missing_rotation_key_is_refused():
    t = torch()
    ctx = context("C1")
    sk = ctx.keygen(1)
    p = ctx.plan(pvfl.PLAN_HYBRID, 64, 256, lazy=True)      # m' = 8: seven rotations
    gal = p.galois()
    partial = ctx.rotkeys(sk, gal[:-1], 2)
    ct, pt, out = (dev_f64(p.bytes(w) // 8) for w in ("ct_in", "pt", "ct_out"))
    assert status_of(lambda: p.matmul(ct, pt, partial, out)) == E_NOKEY
    assert status_of(lambda: p.matmul(ct, pt, None, out)) == E_NOKEY
    # a workspace smaller than the plan needs
    small = t.zeros(8, dtype=t.float64, device="cuda")
    full = ctx.rotkeys(sk, gal, 2)
    assert status_of(lambda: p.matmul(ct, pt, full, out, small)) == E_SHAPE


def test_degenerate_arguments_are_refused():
    ctx = context("C1")
    sk = ctx.keygen(1)
    p = ctx.plan(pvfl.PLAN_HYBRID, 16, 64, lazy=True)
    t = dev_f64(p.bytes("ct_out") // 8)
    assert status_of(lambda: p.matmul_sum([], [], None, t)) == E_INVALID
    assert status_of(lambda: p.encode_out(t, 7, t)) == E_INVALID
    assert status_of(lambda: p.out_add_pt(t, t, 2, t)) == E_INVALID
    assert status_of(lambda: pvfl.Batch(ctx, [], pt=[], ct=[], out=[])) == E_INVALID
    other = context("C1")
    with pytest.raises(pvfl.PvflError):
        other.pk_gen(sk, 3)                        # a key of another context


def test_unit_shape_runs():
    """m = n = 1: one diagonal, no rotation key, one output slot"""
    t = torch()
    ctx = context("C1")
    sk = ctx.keygen(1)
    p = ctx.plan(pvfl.PLAN_HYBRID, 1, 1, lazy=True)
    assert p.galois() == [] and p.info["mprime"] == 1
    f64 = dict(dtype=t.float64, device="cuda")
    pt, ct, out = (t.empty(p.bytes(w) // 8, **f64) for w in ("pt", "ct_in", "ct_out"))
    y = t.empty(1, **f64)
    p.encode_pt(t.tensor([[0.75]], **f64), pt)
    p.encrypt(sk, t.tensor([-0.5], **f64), 9, ct)
    p.matmul(ct, pt, None, out)
    p.decrypt_decode(sk, out, y)
    assert abs(float(y.item()) + 0.375) < 1e-6


def test_binding_checks_tensors():
    """dtype, device, contiguity and size of every buffer are checked before
    the call reaches the library"""
    t = torch()
    ctx = context("C1")
    sk = ctx.keygen(1)
    p = ctx.plan(pvfl.PLAN_HYBRID, 64, 256, lazy=True)
    keys = ctx.rotkeys(sk, p.galois(), 2)
    ct, pt, out = (dev_f64(p.bytes(w) // 8) for w in ("ct_in", "pt", "ct_out"))
    assert status_of(lambda: p.matmul(ct.float(), pt, keys, out)) == E_INVALID        # float32
    assert status_of(lambda: p.matmul(ct.cpu(), pt, keys, out)) == E_INVALID          # host memory
    assert status_of(lambda: p.matmul(ct, pt[: pt.numel() // 2], keys, out)) == E_SHAPE
    assert status_of(lambda: p.matmul(ct, pt, keys, out[::2])) == E_INVALID          # not contiguous
    X = t.zeros(64, 256, dtype=t.float64, device="cuda")
    assert status_of(lambda: p.encode_pt(X[:, :100], pt)) == E_SHAPE                  # rows too short
    assert status_of(lambda: p.encode_pt(X[:32], pt)) == E_SHAPE                      # too few rows
    assert status_of(lambda: p.encode_pt(X.t(), pt)) == E_SHAPE                        # column-major
    y = t.zeros(10, dtype=t.float64, device="cuda")
    assert status_of(lambda: p.encrypt(sk, y, 1, ct)) == E_SHAPE                       # shorter than n
    assert status_of(lambda: p.decrypt_decode(sk, out, y)) == E_SHAPE                  # fewer than m results
    assert status_of(lambda: ctx.pt_import(ctx.L, True, t.zeros(2, ctx.N, dtype=t.float64, device="cuda"),
                                           pt)) == E_INVALID                          # coefficients must be int64
