"""Host-side logic of plan selection: regret bookkeeping and the analytic
model's per-operation cost fit (no GPU)."""
import numpy as np
import pytest

pytest.importorskip("scipy")
from paper_2405_00482_amd import planner as P


def _rec(cfg, idx, kind, ms, counts, bsgs=0, lazy=1):
    return {"config": cfg, "idx": idx, "m": 4, "n": 4, "ms": ms, "counts": counts, "features": [0.0] * 24,
            "opts": {"kind": kind, "lazy_moddown": lazy, "bsgs": bsgs, "ras_in_ct": 0}}


def test_regret_of_a_choice():
    recs = [_rec("C1", 0, 0, 2.0, [1] * 8), _rec("C1", 0, 1, 1.0, [1] * 8), _rec("C1", 1, 0, 5.0, [1] * 8),
            _rec("C1", 1, 2, 4.0, [1] * 8)]
    # predictions pick the first candidate of shape 0 (regret 1.0) and the best of shape 1
    res = P.regrets(recs, np.array([0.1, 0.2, 9.0, 3.0]))
    assert [s["regret"] for s in res["shapes"]] == [1.0, 0.0]
    assert res["mean"] == 0.5 and res["max"] == 1.0
    fixed = P.fixed_choice_regret(recs, lambda r: r["opts"]["kind"] == 0)
    assert [s["regret"] for s in fixed["shapes"]] == [1.0, 0.25]


def test_analytic_fit_recovers_known_costs():
    rng = np.random.default_rng(0)
    true = np.array([0.01, 0.002, 0.08, 0.03, 0.05, 0.04, 0.001, 0.02])
    recs = []
    for i in range(200):
        c = list(rng.integers(0, 50, size=7)) + [1]
        recs.append(_rec("C2", i, 0, float(np.dot(c, true)), c))
    got = P.fit_analytic(recs)["C2"]
    assert np.allclose(got, true, rtol=1e-8, atol=1e-10)


def test_digit_count_variants_pool_their_candidates():
    # the same seeded shape on C4 and on its one-special-prime variant is one choice
    recs = [_rec("C4", 0, 0, 3.0, [1] * 8), _rec("C4a1", 0, 0, 2.0, [1] * 8), _rec("C3", 0, 0, 1.0, [1] * 8)]
    res = P.regrets(recs, np.array([0.5, 0.9, 0.1]))
    assert len(res["shapes"]) == 2
    c4 = [s for s in res["shapes"] if s["config"] == "C4"][0]
    assert c4["regret"] == 0.5 and c4["best"].startswith("C4a1")


def test_split_holds_out_every_fourth_shape():
    recs = [_rec("C3", i, 0, 1.0, [1] * 8) for i in range(8)]
    train, test = P.split(recs)
    assert sorted(r["idx"] for r in test) == [3, 7] and len(train) == 6
