"""Public-key encryption in the oracle, pinned by brute force: decryption
leaves exactly v e + e0 + e1 s on top of m (negacyclic products computed here
with Python integers), within the CBD(21) bound.  CPU only."""
import numpy as np

from oracle import oracle as O
from tests.test_oracle_matmul import tiny


def negacyclic(a, b):
    """schoolbook product in Z[X]/(X^N + 1), Python integers"""
    N = len(a)
    out = [0] * N
    for i in range(N):
        if a[i] == 0:
            continue
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += int(a[i]) * int(b[j])
            else:
                out[k - N] -= int(a[i]) * int(b[j])
    return out


def centred(x, q):
    x = int(x) % q
    return x - q if x > q // 2 else x


def test_pk_decryption_noise_is_v_e_plus_e0_plus_e1_s():
    prm = tiny(5, 3, 1)
    N = prm.N
    s = O.keygen(prm, 3)
    pk = O.pk_gen(prm, s, 4)
    m = np.random.default_rng(1).integers(-2 ** 20, 2 ** 20, N)
    for level in (prm.L, 1):
        ct = O.encrypt_pk(prm, pk, m, level, 5)
        dec = O.decrypt(prm, s, ct)
        # the samples the encryption drew, redrawn from their streams
        v = O.sample_ternary(5, O.stream_pkenc("v"), N)
        e0 = O.sample_cbd21(5, O.stream_pkenc("e0"), N)
        e1 = O.sample_cbd21(5, O.stream_pkenc("e1"), N)
        e = O.sample_cbd21(4, O.stream_pk_e(), N)
        noise = [x + y + z for x, y, z in zip(negacyclic(v, e), e0, negacyclic(e1, s))]
        bound = 21 * N + 21 + 21 * N
        assert max(abs(x) for x in noise) <= bound
        for i, q in enumerate(prm.q[: level + 1]):
            got = [centred(dec[i][k], q) - int(m[k]) for k in range(N)]
            assert got == noise, f"limb {i}"


def test_pk_is_an_rlwe_sample_of_s():
    """b + a s = e exactly, limb by limb"""
    prm = tiny(5, 2, 1)
    s = O.keygen(prm, 8)
    b, a = O.pk_gen(prm, s, 9)
    e = O.sample_cbd21(9, O.stream_pk_e(), prm.N)
    for i, q in enumerate(prm.q):
        sa = negacyclic([int(x) for x in a[i]], [int(x) for x in s])
        assert [centred(int(b[i][k]) + sa[k], q) for k in range(prm.N)] == [int(x) for x in e]
