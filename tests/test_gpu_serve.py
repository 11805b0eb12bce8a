"""Served ensemble on the GPU: every model's trajectory is bitwise the same
alone and inside the mix, and admission keeps the resident footprint within
the budget."""
import numpy as np
import pytest

import synth
from gpu_common import require_gpu

pytestmark = pytest.mark.gpu


def _req(rid, r, size, arrival, steps=3):
    from paper_1808_04338_amd import Request

    return Request(rid, synth.served_realisation(r, size), arrival, steps=steps, tag=str(size))


def test_alone_equals_mix_bitwise():
    require_gpu()
    from paper_1808_04338_amd import serve

    a = _req(0, 0, (20, 20, 10), 0.0)
    alone, _ = serve([a], keep_state=True)
    # request 4 has 1,008,010 unknowns: its preconditioner runs kernel by kernel,
    # the small models' from their captured graphs
    big = (60, 60, 70)
    mix = [_req(0, 0, (20, 20, 10), 0.0), _req(1, 1, (40, 40, 10), 0.0),
           _req(2, 2, (20, 20, 10), 0.01), _req(3, 3, (60, 60, 10), 0.02),
           _req(4, 4, big, 0.0, steps=2)]
    res, summ = serve(mix, keep_state=True)
    assert summ["completed"] == 5 and summ["peak_active"] >= 2
    assert res[4].state[0].shape[0] == 2 * 60 * 60 * 70
    for u, v in zip(alone[0].state, res[0].state):
        assert np.array_equal(u, v)
    c_alone, _ = serve([_req(2, 2, (20, 20, 10), 0.0)], keep_state=True)
    for u, v in zip(c_alone[2].state, res[2].state):
        assert np.array_equal(u, v)
    big_alone, _ = serve([_req(4, 4, big, 0.0, steps=2)], keep_state=True)
    for u, v in zip(big_alone[4].state, res[4].state):
        assert np.array_equal(u, v)


def test_admission_by_footprint():
    require_gpu()
    from paper_1808_04338_amd import footprint, serve

    reqs = [_req(i, 10 + i, (20, 20, 10), 0.001 * i, steps=2) for i in range(5)]
    fp = footprint(reqs[0].model, "fp32")
    budget = 2 * fp + fp // 2
    res, summ = serve(reqs, budget_bytes=budget)
    assert summ["completed"] == 5
    assert summ["peak_bytes"] <= budget and summ["peak_active"] <= 2
