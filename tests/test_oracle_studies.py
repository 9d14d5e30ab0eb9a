"""The oracle studies (single precision, coarse spaces, Krylov recycling) on tiny problems:
they run, every scheme reaches its tolerance, and the schemes that must agree do."""
import numpy as np

import workloads as w
from oracle import coarse_study, recycle_study, single_study

SRC = np.array([[0.37, 0.52, 0.61], [0.61, 0.3, 0.45], [0.25, 0.7, 0.3]])


def test_single_study_runs():
    out = single_study.run("unit cube 3^3", w.unit_cube_problem(3, freq=1.0, parts=(2, 2, 1)))
    for tol in (1e-3, 1e-6):
        assert out[(tol, "fp64")][1] <= tol and out[(tol, "mixed")][1] <= 2 * tol
    # at the paper's tolerance the three schemes take the same iterations
    assert out[(1e-3, "fp64")][0] == out[(1e-3, "mixed")][0] == out[(1e-3, "single")][0]


def test_coarse_study_runs():
    p = w.unit_cube_problem(4, freq=1.0, parts=(2, 2, 1))
    out = coarse_study.run(p, factors=(2,), sources=SRC[:2], label="unit cube 4^3")
    assert len(out) == 3
    assert all(res <= 1e-6 for _, res in out.values())


def test_recycle_study_runs():
    p = w.unit_cube_problem(3, freq=1.5, parts=(2, 2, 1))
    out = recycle_study.run(p, ks=(4,), m=10, sources=SRC, label="unit cube 3^3")
    assert set(out) == {"GMRES(10)", "GCRO-DR(10, 4)", "block FGMRES(10)"}
    assert all(res <= 1e-6 for _, res in out.values())
