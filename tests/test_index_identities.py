"""Index identities the GPU transforms rely on, checked exhaustively on the CPU.

* Orbit order: slot t < N/2 holds exponent 5^t mod 2N, at bit-reversed index
  brv((5^t mod 2N - 1) / 2); slot t + N/2 holds -5^t, at the complement.  The
  kernels walk a thread's slots t = tid + w N/16 as 5^tid (5^(N/16))^w with
  32-bit products and a mask (ntt_core.hpp, OrbitWalk), and the encoder maps
  slot j to DFT input (5^j mod 2N - 1) / 4 the same way.
* Padded LDS sets: element u of a set {base + u 2^ls} lies at padded offset
  (u << ls) + ((u << ls) >> 4) from lds_pad(base) for every set base the
  forward and inverse passes use (lds_load_c / lds_store_c).
* Wave locality: every set of those passes, for the thread tid = 64 w + lane,
  lies inside wave w's 1024 elements.
"""
import pytest

MASK32 = (1 << 32) - 1


def brv(x: int, bits: int) -> int:
    return int(format(x, f"0{bits}b")[::-1], 2)


def lds_pad(j: int) -> int:
    return j + (j >> 4)


@pytest.mark.parametrize("log_n", [12, 13, 14])
def test_orbit_walk_matches_the_permutation_table(log_n):
    n = 1 << log_n
    t_threads = n // 16
    mask = 2 * n - 1
    # the table the host builds (capi.cpp): orbit index t -> bit-reversed index
    perm = [0] * n
    e = 1
    for t in range(n // 2):
        eneg = (2 * n - e) % (2 * n)
        perm[t] = brv((e - 1) // 2, log_n)
        perm[t + n // 2] = brv((eneg - 1) // 2, log_n)
        e = e * 5 % (2 * n)
    step = pow(5, t_threads, 2 * n)
    for tid in range(t_threads):
        # OrbitWalk::start: square-and-multiply over the bits of tid, masked
        r, b = 1, 5
        for k in range(log_n - 4):
            if (tid >> k) & 1:
                r = (r * b) & MASK32 & mask
            b = (b * b) & MASK32 & mask
        assert r == pow(5, tid, 2 * n)
        ew = r
        for w in range(8):
            j = brv(ew >> 1, log_n)
            assert perm[tid + w * t_threads] == j
            assert perm[tid + (w + 8) * t_threads] == j ^ (n - 1)
            assert ew * step < (1 << 32)  # the 32-bit product is exact
            ew = (ew * step) & mask


@pytest.mark.parametrize("log_n", [12, 13, 14])
def test_slot_to_dft_position_walk(log_n):
    n = 1 << log_n
    m = n // 2
    t_threads = n // 16
    slot2f = [0] * m
    e = 1
    for j in range(m):
        slot2f[j] = (e - 1) // 4
        e = e * 5 % (2 * n)
    step = pow(5, t_threads, 2 * n)
    seen = set()
    for tid in range(t_threads):
        ew = pow(5, tid, 2 * n)
        for u in range(8):
            f = ew >> 2
            assert f == slot2f[tid + u * t_threads]
            seen.add(f)
            ew = (ew * step) & (2 * n - 1)
    assert seen == set(range(m))  # every DFT input written exactly once


def _forward_sets(log_n, tid):
    """(S, ls, bases) of the forward passes after the register stages."""
    sets = []
    for ls in (log_n - 8, log_n - 12):  # stages 4..7 and 8..11: pass_bases<LOGN, 4>
        c = tid
        sets.append((4, ls, [((c >> ls) << (ls + 4)) | (c & ((1 << ls) - 1))]))
    if log_n > 12:  # stages 12..: sets of 2^S consecutive elements
        s = log_n - 12
        sets.append((s, 0, [16 * tid + (q << s) for q in range(16 >> s)]))
    return sets


@pytest.mark.parametrize("log_n", [12, 13, 14])
def test_padded_set_offsets_and_wave_locality(log_n):
    n = 1 << log_n
    t_threads = n // 16
    covered = {}
    for tid in range(t_threads):
        wave = tid // 64
        # the cross-wave store of the register stages: base tid, span N/16
        for u in range(16):
            ls = log_n - 4
            assert lds_pad(tid + (u << ls)) - lds_pad(tid) == (u << ls) + ((u << ls) >> 4)
        for s, ls, bases in _forward_sets(log_n, tid):
            for base in bases:
                for u in range(1 << s):
                    el = base + (u << ls)
                    assert lds_pad(el) - lds_pad(base) == (u << ls) + ((u << ls) >> 4)
                    assert el // 1024 == wave, (log_n, tid, el)
                    covered.setdefault((s, ls), set()).add(el)
    for key, els in covered.items():  # each pass partitions the limb
        assert els == set(range(n)), key
