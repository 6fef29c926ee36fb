"""The eigenvalue solvers' host-side logic, built with g++ from the library's
plain C++ header and checked on the CPU against the oracle: the flat shift
directions of the NLL (the same subspace: equal projectors in the gauge
metric) and the gauge projection inside the box (the same point)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import solver as S

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2407_19892_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("host") / "host_solve_driver")
    subprocess.run([gxx, "-std=c++17", "-O2", "-I", CSRC, os.path.join(HERE, "host_solve_driver.cpp"), "-o", exe],
                   check=True)
    return exe


def _run(exe, text):
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True, timeout=60)
    return out.stdout.split("\n")


def _random_sets(rng, L):
    """Modalities covering all L axes: 2 to 4 axes each, distinct axis sets."""
    sets, cover = [], set()
    while len(cover) < L or not sets:
        K = int(rng.integers(2, min(4, L) + 1))
        m = tuple(sorted(int(a) for a in rng.choice(L, size=K, replace=False)))
        if m not in sets:
            sets.append(m)
            cover |= set(m)
    return sets


def _projector(F, r):
    if not F:
        return np.zeros((len(r), len(r)))
    return sum(np.outer(c, c) for c in F) @ np.diag(r)


def test_flat_directions_match_the_oracle(driver):
    rng = np.random.default_rng(0)
    cases = []
    for it in range(300):
        L = int(rng.integers(2, 9))
        sets = _random_sets(rng, L)
        ranks = rng.integers(1, 30, L)
        traces = rng.uniform(1.0, 100.0, L)
        if it % 3 == 0:                          # balanced: every null shift flat
            traces = np.full(L, 50.0)
        cases.append((sets, ranks, traces))
    # the COIL-20 shape: 20 (frame, row_i, col_i), balanced and not
    coil = [(0, 1 + 2 * i, 2 + 2 * i) for i in range(20)]
    r41 = np.array([72] + [128] * 40)
    cases.append((coil, r41, np.array([20.0] + [1.0] * 40)))
    cases.append((coil, np.array([10] * 41), rng.uniform(1.0, 5.0, 41)))
    text = ""
    for sets, ranks, traces in cases:
        text += f"F {len(ranks)} {len(sets)} " + " ".join(str(int(x)) for x in ranks) + " " + \
                " ".join(repr(float(x)) for x in traces) + " " + \
                " ".join(f"{len(m)} " + " ".join(str(a) for a in m) for m in sets) + "\n"
    out = _run(driver, text)
    pos = 0
    for sets, ranks, traces in cases:
        d = int(out[pos])
        F_cpp = [np.array([float(x) for x in out[pos + 1 + q].split()]) for q in range(d)]
        pos += 1 + d
        F_ora = S.flat_shift_space(sets, ranks, traces)
        assert d == len(F_ora), (sets, d, len(F_ora))
        r = np.asarray(ranks, dtype=np.float64)
        np.testing.assert_allclose(_projector(F_cpp, r), _projector(F_ora, r), atol=1e-10)


def test_gauge_projection_matches_the_oracle(driver):
    rng = np.random.default_rng(1)
    cases = []
    for it in range(2000):
        L = int(rng.integers(2, 9)) if it % 10 else 41
        q = int(rng.integers(1, L)) if it % 10 else 21
        C = np.linalg.qr(rng.standard_normal((L, q)))[0].T * rng.uniform(0.05, 1.0)
        lam = [10.0 ** rng.uniform(-6, 1, int(rng.integers(1, 6))) for _ in range(L)]
        eps = 10.0 ** rng.uniform(-15, -7, L)
        for l in rng.choice(L, size=int(rng.integers(0, 3)), replace=False):
            lam[l][0] = eps[l]                  # an axis already at its bound
        ts = rng.standard_normal(q) * 10.0 ** rng.uniform(-6, 2)
        cases.append((C, lam, eps, ts))
    text = ""
    for C, lam, eps, ts in cases:
        q, L = C.shape
        text += f"Q {q} {L} " + " ".join(repr(float(x)) for x in C.ravel()) + " " + \
                " ".join(repr(float(x)) for x in eps) + " " + \
                " ".join(repr(float(l.min())) for l in lam) + " " + " ".join(repr(float(x)) for x in ts) + "\n"
    out = _run(driver, text)
    for (C, lam, eps, ts), line in zip(cases, out):
        t_cpp = np.array([float(x) for x in line.split()])
        t_ora = S.nearest_feasible_shift(ts, list(C), lam, list(eps))
        scale = np.max(np.abs(ts)) + np.max(np.abs(t_ora))
        assert np.max(np.abs(t_cpp - t_ora)) <= 1e-11 * scale
