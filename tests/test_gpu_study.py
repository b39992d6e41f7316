"""A small error-assessment study (Sec. 3) on the GPU: the measures come out
in their ranges and the uniform FV error falls with the grid."""
import math

import pytest

from paper_1603_05211_amd import study

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_small_study():
    res = study.run_study(levels=(3, 4), n0=32, n_ref=512, t_end=0.05, log=say)
    say(study.markdown(res))
    a, b = res["runs"]
    for name in ("MR-FV", "AMR-FV"):
        assert b[name]["l1"] < a[name]["l1"] and b[name]["rate"] > 0.3
    for r in res["runs"]:
        for name in study.ADAPTIVE:
            m = r[name]
            assert 0 < m["mesh_compression"] <= m["memory_compression"] <= 2.0
            assert m["mesh_compression"] <= 1.0
            assert math.isfinite(m["overhead"]) and m["l1"] > 0
            assert m["accuracy_perturbation"] < 1.0


def test_small_study_3d():
    res = study.run_study_3d(levels=(2, 3), n0=16, n_ref=128, t_end=0.05, log=say)
    say(study.markdown(res))
    a, b = res["runs"]
    assert b["MR-FV"]["l1"] < a["MR-FV"]["l1"]
    for r in res["runs"]:
        for name in study.ADAPTIVE_3D:
            m = r[name]
            assert 0 < m["mesh_compression"] <= m["memory_compression"] <= 2.0
            assert m["mesh_compression"] <= 1.0
            assert math.isfinite(m["overhead"]) and m["l1"] > 0
            assert m["accuracy_perturbation"] < 1.0
