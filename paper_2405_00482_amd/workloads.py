"""Seeded synthetic inputs for the five workloads (no HE arithmetic here).

The paper measures on SUSY (efficiency) and NUS-WIDE (accuracy), resampled in
size (Sec. 7, Dataset); neither is available here, so seeded synthetic data of
the workloads' shapes and value distributions stand in for them.  Both the
HIP path and the CPU oracle are fed from these generators.

    C1  ring 2^12, X^T (16 x 256) ~ U[-1,1], r (256) ~ U[-1,1]
    C2  ring 2^13, X (1024 x 256) ~ N(0,1) standardised, r (1024) ~ U[-1,1];
        product X^T [[r]] (m = 256 features, n = 1024 batch)
    C3  ring 2^14, 64 products X_k^T [[r_k]], batch ~ logU[512, 4096],
        features ~ logU[32, 2000], X ~ N(0,1), r ~ U[-1,1]
    C4  ring 2^14, [[H]] 256 x 64 ~ U[-1,1] times W 64 x 256 ~ N(0, 0.1^2);
        backward [[delta]] 256 x 256 ~ U[-1,1] times W^T
    C5  ring 2^15, X 4096 x 5000 with Bernoulli(0.1) mask times N(0,1),
        [[R]] 4096 x 128 ~ U[-1,1]; product X^T [[R]]
"""
from __future__ import annotations

import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(_HERE, "params.json")


def params_dict(name: str) -> dict:
    with open(PARAMS_PATH) as f:
        return json.load(f)[name]


def seed_of(name: str) -> int:
    """1000 + the configuration's index (C4a1, C4a2: C4's digit-count variants, seeded as C4)"""
    digits = ""
    for ch in name[1:]:
        if not ch.isdigit():
            break
        digits += ch
    return 1000 + int(digits)


def rng(name: str, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng([seed_of(name), salt])


def c1_inputs():
    g = rng("C1")
    XT = g.uniform(-1.0, 1.0, size=(16, 256))
    r = g.uniform(-1.0, 1.0, size=256)
    return XT, r


def c2_inputs():
    g = rng("C2")
    X = g.standard_normal(size=(1024, 256))
    X = (X - X.mean(axis=0)) / X.std(axis=0)
    r = g.uniform(-1.0, 1.0, size=1024)
    return np.ascontiguousarray(X.T), r


def c3_shapes(count: int = 64):
    g = rng("C3", 1)
    batch = np.exp(g.uniform(np.log(512), np.log(4096), size=count)).astype(np.int64)
    feats = np.exp(g.uniform(np.log(32), np.log(2000), size=count)).astype(np.int64)
    # product k is X_k^T [[r_k]]: m = features, n = batch
    return [(int(f), int(b)) for f, b in zip(feats, batch)]


def c3_inputs(k: int, shape=None):
    m, n = shape if shape is not None else c3_shapes()[k]
    g = rng("C3", 100 + k)
    XT = g.standard_normal(size=(m, n))
    r = g.uniform(-1.0, 1.0, size=n)
    return XT, r


def c4_inputs():
    g = rng("C4")
    H = g.uniform(-1.0, 1.0, size=(256, 64))
    W = g.normal(0.0, 0.1, size=(64, 256))
    delta = g.uniform(-1.0, 1.0, size=(256, 256))
    return H, W, delta


def c5_inputs(cols=None):
    g = rng("C5")
    X = g.standard_normal(size=(4096, 5000)) * (g.uniform(size=(4096, 5000)) < 0.1)
    R = g.uniform(-1.0, 1.0, size=(4096, 128))
    if cols is not None:
        R = R[:, cols]
    return np.ascontiguousarray(X.T), R


# the matrix shapes (m x n) of Table 4, compared at ring degree 2^13
TABLE4_SHAPES = [(512, 64), (512, 256), (512, 1024), (512, 4096), (64, 512), (256, 512), (1024, 512), (4096, 512),
                 (64, 64), (256, 256), (1024, 1024), (4096, 4096)]


def table4_inputs(m: int, n: int):
    """X ~ N(0,1) (m x n, standardised columns) and y ~ U[-1,1] (n), seeded by the shape."""
    g = np.random.default_rng(7000 + 13 * m + n)
    X = g.standard_normal(size=(m, n))
    if m > 1:
        X = (X - X.mean(axis=0)) / X.std(axis=0)
    y = g.uniform(-1.0, 1.0, size=n)
    return np.ascontiguousarray(X), y


def seeds(name: str) -> dict:
    """Seeds of the counter-based generator for keys and encryption noise."""
    s = seed_of(name)
    return {"sk": s * 7919 + 1, "rotkeys": s * 7919 + 2, "enc": s * 7919 + 3}


def planner_shapes(name: str, count: int):
    """Shapes (m, n) for plan-selection data: m ~ logU[1, 2048] rows of X,
    n ~ logU[2, 4096] entries of the encrypted vector (the feature and batch
    ranges of the VFL products, extended down to tiny shapes)."""
    g = rng(name, 7)
    m = np.exp(g.uniform(np.log(1), np.log(2048), size=count)).astype(np.int64)
    n = np.exp(g.uniform(np.log(2), np.log(4096), size=count)).astype(np.int64)
    return [(int(max(1, a)), int(max(2, b))) for a, b in zip(m, n)]


def planner_inputs(name: str, idx: int, shape):
    """X ~ N(0,1) (m x n) and y ~ U[-1,1] (n) for planner shape idx"""
    g = rng(name, 1000 + idx)
    m, n = shape
    return g.standard_normal(size=(m, n)), g.uniform(-1.0, 1.0, size=n)
