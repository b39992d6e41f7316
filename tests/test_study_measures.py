"""The error-assessment measures of Sec. 3 (host code of the study module):
each against its definition evaluated by hand on small inputs."""
import numpy as np
import pytest

from paper_1603_05211_amd import study


def test_project_is_cell_means():
    rng = np.random.default_rng(0)
    Q = rng.normal(size=(2, 8, 8))
    P = study.project(Q, 2)
    for f in range(2):
        for j in range(2):
            for i in range(2):
                assert np.isclose(P[f, j, i], Q[f, 4 * j:4 * j + 4, 4 * i:4 * i + 4].mean())
    Q3 = rng.normal(size=(1, 4, 4, 4))
    assert np.isclose(study.project(Q3, 1)[0, 0, 0, 0], Q3.mean())
    assert np.array_equal(study.project(Q, 8), Q)


def test_l1_error_and_perturbation():
    a = np.zeros((4, 4))
    b = np.full((4, 4), 0.5)
    assert study.l1_error(a, b) == pytest.approx(0.5)          # 16 cells x 0.5 x (1/4)^2
    assert study.l1_error(a, b, -1.0, 1.0) == pytest.approx(2.0)
    assert study.accuracy_perturbation(0.01, 0.012) == pytest.approx(0.2)
    assert study.accuracy_perturbation(0.01, 0.008) == pytest.approx(0.2)


def test_compression_and_overhead():
    assert study.memory_compression([100, 300], 1000) == pytest.approx(0.2)
    assert study.mesh_compression([50, 150], 1000) == pytest.approx(0.1)
    assert study.time_compression(2.0, 8.0) == pytest.approx(0.25)
    # same time per leaf-step: no overhead; twice the time per leaf-step: 100 %
    assert study.overhead(1.0, 100.0, 10.0, 1000.0) == pytest.approx(0.0)
    assert study.overhead(2.0, 100.0, 10.0, 1000.0) == pytest.approx(1.0)
