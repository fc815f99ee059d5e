"""Write the RNS parameter sets (prime chains) of the five workloads.

Run:  python -m oracle.gen_params   (writes paper_2405_00482_amd/params.json)

Primes are NTT-friendly (q = 1 mod 2N) and below 2^48, which the library's
exact binary64 modular arithmetic requires.  Rule: ciphertext primes are the
largest such primes below 2^40 (C1 uses two of them, as its workload states
"~40-bit"); for the larger rings q_0 and the special primes are the largest
below 2^48 so that two rescales of the row-order plan leave room at level 0
and the key-switching modulus P exceeds every digit modulus.
"""
import json
import os

from . import oracle as O


def primes_below(bits: int, N: int, count: int, exclude=()) -> list:
    out = []
    step = 2 * N
    x = ((1 << bits) - 1) // step * step + 1
    while len(out) < count:
        if x < (1 << bits) and O.is_prime(x) and x not in exclude:
            out.append(x)
        x -= step
    return out


def config(name, logN, n_q40, n_q48, n_p, log2_scale):
    N = 1 << logN
    q48 = primes_below(48, N, n_q48 + n_p)
    q = q48[:n_q48] + primes_below(40, N, n_q40)
    p = q48[n_q48:]
    assert len(set(q + p)) == len(q + p)
    return {"name": name, "logN": logN, "q": q, "p": p, "log2_scale": log2_scale}


def main():
    cfgs = {
        "C1": config("C1", 12, 2, 0, 1, 30.0),
        "C2": config("C2", 13, 2, 1, 1, 40.0),
        "C3": config("C3", 14, 3, 1, 1, 40.0),
        "C4": config("C4", 14, 5, 1, 3, 40.0),
        "C5": config("C5", 15, 7, 1, 2, 40.0),
    }
    # C4 with fewer special primes (more key-switch digits): the plan selector's
    # digit-count variants; same ciphertext primes, special primes a prefix of C4's
    for a in (1, 2):
        v = dict(cfgs["C4"])
        v["name"] = f"C4a{a}"
        v["p"] = cfgs["C4"]["p"][:a]
        cfgs[v["name"]] = v
    # special primes must be ~2^48; for C1 take the largest below 2^48 as well
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2405_00482_amd", "params.json")
    with open(path, "w") as f:
        json.dump(cfgs, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
