"""Helpers for the GPU parity tests: device buffers and residue comparison."""
import numpy as np

from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import workloads as W


def torch():
    import torch as _t
    return _t


def dev_f64(n):
    t = torch()
    return t.zeros(int(n), dtype=t.float64, device="cuda")


def dev_i64(arr):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(arr, dtype=np.int64)).to("cuda")


def dev_u64(n):
    t = torch()
    return t.zeros(int(n), dtype=t.int64, device="cuda")   # holds uint64 bit patterns


def host_u64(t_dev):
    torch().cuda.synchronize()
    return t_dev.cpu().numpy().view(np.uint64)


def context(name):
    return pvfl.Context.from_dict(W.params_dict(name))


def export(ctx, level, with_p, poly, count):
    nl = level + 1 + (ctx.alpha if with_p else 0)
    out = dev_u64(count * nl * ctx.N)
    ctx.export_coeffs(level, with_p, poly, count, out)
    return host_u64(out).reshape(count, nl, ctx.N)


def export_ct(ctx, level, ct, count=1):
    """ciphertexts [count][2][l+1][N] -> uint64 coefficient residues"""
    return export(ctx, level, False, ct, 2 * count).reshape(count, 2, level + 1, ctx.N)


def first_mismatch(got, want):
    d = np.argwhere(got != want)
    if d.size == 0:
        return None
    return tuple(int(x) for x in d[0]), int(got[tuple(d[0])]), int(want[tuple(d[0])]), int(d.shape[0])
