"""eu_conserved_totals_static (the totals with the library's static device
scratch, for callers that cannot allocate) against eu_conserved_totals: bit
for bit, on two calls in a row, the second on a smaller input, and a clear
error beyond the static scratch's capacity."""
import math

import numpy as np
import pytest

from gpu_helpers import say
from paper_1603_05211_amd import EU_FP32, EU_FP64, EuError, Solver, inputs

pytestmark = pytest.mark.gpu


def totals_pair(s):
    import torch
    n = s.n_instances * s.nv
    ref = torch.full((n,), math.nan, dtype=torch.float64, device=s.device)
    got = torch.full((n,), math.nan, dtype=torch.float64, device=s.device)
    s.conserved_totals(out_dev=ref, host=False)
    s.conserved_totals_static(got)
    s.stream.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_static_totals_match_two_calls_second_smaller():
    # first call: the 2D five-level adaptive hierarchy (5456 tile slots) in FP32
    say("eu_conserved_totals_static: 2D adaptive, 5 levels, FP32")
    a = Solver(2, n0=32, levels=5, precision=EU_FP32, cfl=0.45, eps=1e-3)
    a.init_quadrant(inputs.quadrant_states(0))
    a.advance(20)
    ref, got = totals_pair(a)
    assert np.all(np.isfinite(ref))
    assert np.array_equal(ref, got), (ref, got)
    # second call, smaller input: a batch of three small FP64 instances (one
    # total per instance and field; fewer partial sums than the first call left)
    say("eu_conserved_totals_static: batch of 3 instances, FP64")
    b = inputs.batch(5, n_instances=3)
    s = Solver(2, sides=[32, 64, 32], precision=EU_FP64)
    s.init_quadrant_batch(b.states)
    s.advance(4)
    ref2, got2 = totals_pair(s)
    assert np.all(np.isfinite(ref2))
    assert np.array_equal(ref2, got2), (ref2, got2)
    # and the host copy of the context's own totals agrees
    assert np.array_equal(s.conserved_totals().ravel(), got2)
    # the first context again, after the smaller call reused the array
    ref3, got3 = totals_pair(a)
    assert np.array_equal(ref3, got3) and np.array_equal(ref3, ref)
    a.close()
    s.close()


def test_static_totals_rejects_beyond_capacity():
    # 4096^2 cells = 262144 tiles x 4 fields: more partial sums than 2^19
    say("eu_conserved_totals_static: 4096^2 uniform grid beyond the static scratch")
    import torch
    s = Solver(2, n0=4096, levels=1, precision=EU_FP32, cfl=0.45)
    s.init_quadrant(inputs.quadrant_states(1))
    out = torch.zeros(s.nv, dtype=torch.float64, device=s.device)
    with pytest.raises(EuError) as e:
        s.conserved_totals_static(out)
    assert e.value.code == 2 and "static scratch" in str(e.value)
    s.close()
