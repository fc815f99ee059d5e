"""Public-key generation and encryption on the GPU through the C ABI: residues
equal the oracle's; the encrypted product of a public-key ciphertext decrypts
within the precision budget where the scale allows it.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import workloads as W

from gpu_util import context, dev_f64, dev_i64, dev_u64, export_ct, first_mismatch, host_u64

pytestmark = pytest.mark.gpu


def assert_same(got, want, what):
    mm = first_mismatch(np.asarray(got, dtype=np.uint64), np.asarray(want, dtype=np.uint64))
    assert mm is None, f"{what}: first mismatch at {mm[0]} gpu={mm[1]} oracle={mm[2]} ({mm[3]} differ)"


@pytest.mark.parametrize("name", ["C1", "C5"])
def test_pk_and_pk_encryption_match_oracle(name):
    prm = O.Params.from_dict(W.params_dict(name))
    ctx = context(name)
    N, L = prm.N, prm.L
    sk = ctx.keygen(21)
    s = O.keygen(prm, 21)
    pk = ctx.pk_gen(sk, 22)
    opk = O.pk_gen(prm, s, 22)
    out = dev_u64(2 * (L + 1) * N)
    pk.export(out)
    got = host_u64(out).reshape(2, L + 1, N)
    assert_same(got[0], opk[0], "pk b")
    assert_same(got[1], opk[1], "pk a")
    m = np.random.default_rng(3).integers(-2 ** 40, 2 ** 40, N)
    for level in (L, 0):
        ct = dev_f64(2 * (level + 1) * N)
        ctx.encrypt_coeffs_pk(pk, level, dev_i64(m), 23, ct)
        g = export_ct(ctx, level, ct)[0]
        w = O.encrypt_pk(prm, opk, m, level, 23)
        assert_same(g[0], w.c0, f"c0 level {level}")
        assert_same(g[1], w.c1, f"c1 level {level}")


def test_pk_rejects_foreign_keys():
    a, b = context("C1"), context("C1")
    sk = a.keygen(1)
    with pytest.raises(pvfl.PvflError):
        b.pk_gen(sk, 2)


@pytest.mark.parametrize("name,bound", [("C3", 2.0 ** -20), ("C1", 2.0 ** -14)])
def test_product_of_pk_ciphertext(name, bound):
    """X^T [[r]] with [[r]] public-key encrypted: within 2^-20 at Delta = 2^40
    (C3); at C1 (Delta = 2^30, N = 2^12) the larger encryption noise costs
    about four bits, as the noise analysis predicts, and the test bounds it"""
    import torch
    ctx = context(name)
    rng = np.random.default_rng(17)
    m, n = (256, 1024) if name == "C3" else (16, 256)
    X = rng.standard_normal((m, n))
    r = rng.uniform(-1, 1, n)
    f64 = dict(dtype=torch.float64, device="cuda")
    plan = ctx.plan(0, m, n, lazy=True)
    sk = ctx.keygen(31)
    pk = ctx.pk_gen(sk, 32)
    keys = ctx.rotkeys(sk, plan.galois(), 33) if plan.galois() else None
    pt = torch.empty(plan.bytes("pt") // 8, **f64)
    plan.encode_pt(torch.from_numpy(X).to(**f64), pt)
    ct = torch.empty(plan.bytes("ct_in") // 8, **f64)
    plan.encrypt_pk(pk, torch.from_numpy(r).to(**f64), 34, ct)
    out = torch.empty(plan.bytes("ct_out") // 8, **f64)
    plan.matmul(ct, pt, keys, out)
    y = torch.empty(m, **f64)
    plan.decrypt_decode(sk, out, y)
    ref = X @ r
    err = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"{name}: public-key path relative error 2^{np.log2(err):.2f}")
    assert err < bound
