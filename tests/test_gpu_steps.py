"""Timestep branches against the oracle: sub-step cuts (by the Newton limit and
by the stagnation exit), the regrowth of the sub-step after an accepted one,
the roll-back of a failed step, and the layered five-spot schedule of the
144k-DOF configuration at a size the oracle's direct-solve Newton runs in
seconds.

Tolerances as in the other timestep parity tests: pressure and p_b 1e-9
relative, S_w 1e-9 absolute, material balance 1e-10 per sub-step."""
import numpy as np
import pytest

import synth
from gpu_common import controls, rel_max, require_gpu
from oracle import newton as onewton
from oracle import physics as oph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _start_at_oracle_state(sim, m):
    """Give the handle the oracle's initial state, bit for bit.  A rate
    injector starts at the mean of the initial pressures, which on these
    hydrostatic models equals a perforated node's pressure: exactly the point
    where the perforation switches between injection and back-flow mobility.
    The two sides sum that mean in different orders, so without this the
    first Newton iterates take different branches of the switch (both valid)
    and a struggling sub-step can then fail on one side only."""
    geo = oph.Geometry(m)
    sim.set_state(*oph.unpack_state(oph.initial_state(m), geo.n))


def _compare(pg, sg, bg, xo, n):
    po, so, bo = oph.unpack_state(xo, n)
    assert rel_max(pg, po) <= 1e-9
    assert np.abs(sg - so).max() <= 1e-9
    if bo.size:
        assert rel_max(bg, bo) <= 1e-9


CUT_MODELS = {"c0": lambda: synth.model_small(), "tiny_grav": lambda: synth.model_tiny(4, 3, 2, seed=3)}

# (model, step length in days, Newton limit, sub-steps): from the model's
# initial state the oracle takes
#   c0, 5 days, 20 iterations, stagnation exit after 5 iterations: one cut by
#     the exit (no updated iterate of the first attempt goes below its first
#     one), then two 2.5-day sub-steps; with the exit off the step converges
#     whole;
#   c0, 2 days, 8 iterations: cuts by the Newton limit to 0.5 days, then the
#     sub-step doubles after the accepted one (0.5, 1.0) and the last one is cut
#     back to what remains (0.5);
#   tiny_grav, 8 days, 8 iterations: the same pattern with 2, 4 and 2 days;
#   c0, 10 days, 8 iterations: four cuts to 0.625 days, doubling to 2.5, a
#     fifth cut by the Newton limit from 5, then 2.5 and the last 3.125 days.
# Every decision has a wide margin: failed attempts end at a CNV of 1e-7 or
# more against the tolerance 1e-10, accepted ones at 1e-12 or less.
CUT_CASES = [("c0", 5.0, 20, 5, 2), ("c0", 2.0, 8, 0, 3), ("tiny_grav", 8.0, 8, 0, 3), ("c0", 10.0, 8, 0, 5)]


@pytest.mark.parametrize("name,days,max_newton,stall,substeps", CUT_CASES)
def test_cut_and_regrowth_match_oracle(name, days, max_newton, stall, substeps):
    from paper_1808_04338_amd import Sim

    m = CUT_MODELS[name]()
    dt = days * synth.DAY
    geo = oph.Geometry(m)
    xo, rep, _ = onewton.timestep(geo, oph.initial_state(m), dt, controls(m), tol=1e-10,
                                  max_newton=max_newton, stall=stall)
    assert len(rep) == substeps
    sim = Sim(m, newton_tol=1e-10, lin_rtol=1e-11, max_newton=max_newton, newton_stall=stall)
    _start_at_oracle_state(sim, m)
    info = sim.timestep(dt)
    pg, sg, bg = sim.get_state()
    sim.close()
    print("device: %d sub-steps, %d cuts, %d Newton; oracle: %d sub-steps, %d Newton"
          % (info["substeps"], info["cuts"], info["newton_iters"], len(rep), sum(r["newton"] for r in rep)))
    assert info["cuts"] >= 1
    assert info["substeps"] == substeps
    assert info["dt"] == pytest.approx(dt, rel=1e-15)
    assert info["mb_oil"] <= 1e-10 and info["mb_water"] <= 1e-10
    assert max(max(r["mb_oil"], r["mb_water"]) for r in rep) <= 1e-10
    _compare(pg, sg, bg, xo, geo.n)


def test_stagnation_exit_off_matches_oracle():
    """With the stagnation exit off (the default on both sides) the 5-day step
    converges whole, as the oracle's does."""
    from paper_1808_04338_amd import Sim

    m = synth.model_small()
    dt = 5.0 * synth.DAY
    geo = oph.Geometry(m)
    xo, rep, _ = onewton.timestep(geo, oph.initial_state(m), dt, controls(m), tol=1e-10)
    assert len(rep) == 1
    sim = Sim(m, newton_tol=1e-10, lin_rtol=1e-11)
    _start_at_oracle_state(sim, m)
    info = sim.timestep(dt)
    pg, sg, bg = sim.get_state()
    sim.close()
    assert info["cuts"] == 0 and info["substeps"] == 1
    _compare(pg, sg, bg, xo, geo.n)


def test_failed_step_rolls_back_and_leaves_the_handle_usable():
    """A step that cannot converge (three Newton iterations allowed, one cut:
    the oracle fails the 30-day step with these limits too) returns
    DP_E_NOCONV with the state of the start of the step, bitwise; the same
    handle then takes a short step (one second, three Newton iterations) to
    the same bits as a fresh handle."""
    from paper_1808_04338_amd import Sim
    from paper_1808_04338_amd._lib import DP_E_NOCONV, DpError

    m = synth.model_small()
    opts = dict(newton_tol=1e-10, lin_rtol=1e-12, max_newton=3, max_cuts=1)
    a = Sim(m, **opts)
    before = a.get_state()
    with pytest.raises(DpError) as e:
        a.timestep(30.0 * synth.DAY)
    assert e.value.code == DP_E_NOCONV
    after = a.get_state()
    for u, v in zip(before, after):
        assert np.array_equal(u, v)
    short = 1.0
    info_a = a.timestep(short)
    b = Sim(m, **opts)
    info_b = b.timestep(short)
    assert info_a["cuts"] == 0 and info_b["cuts"] == 0
    for u, v in zip(a.get_state(), b.get_state()):
        assert np.array_equal(u, v)
    a.close()
    b.close()


def test_setup_failure_rolls_back_and_leaves_the_handle_usable():
    """A workspace error in the middle of an AMG setup (the fail_setup hook:
    the handle's second setup fails with DP_E_NOMEM once its first level's
    launches are queued, i.e. in the second Newton iteration of the step)
    ends the timestep with DP_E_NOMEM and the state of the start of the step,
    bitwise; the same handle then takes the step to the same bits as a fresh
    handle, so controls and work buffers were left usable too.  Forced from
    the host: no kernel fails."""
    from paper_1808_04338_amd import Sim
    from paper_1808_04338_amd._lib import DP_E_NOMEM, DpError

    m = synth.served_realisation(0, (20, 20, 10))
    opts = dict(newton_tol=1e-10, lin_rtol=1e-12)
    a = Sim(m, fail_setup=2, **opts)
    before = a.get_state()
    dt = m["schedule"][0]
    with pytest.raises(DpError) as e:
        a.timestep(dt)
    assert e.value.code == DP_E_NOMEM
    assert "fail_setup" in str(e.value)
    for u, v in zip(before, a.get_state()):
        assert np.array_equal(u, v)
    info_a = a.timestep(dt)
    b = Sim(m, **opts)
    info_b = b.timestep(dt)
    assert info_a["newton_iters"] == info_b["newton_iters"] >= 2
    for u, v in zip(a.get_state(), b.get_state()):
        assert np.array_equal(u, v)
    a.close()
    b.close()


def test_layered_five_spot_schedule_matches_oracle():
    """The 144k-DOF configuration's physics, layered permeability and five-spot
    (four injectors, one producer) with its 5-day steps, at the smallest size
    class of the served ensemble (20x20x10, 16,010 DOF): the first three steps
    against the oracle's direct-solve Newton, at the parity tolerances."""
    from paper_1808_04338_amd import Sim

    m = synth.served_realisation(0, (20, 20, 10))
    steps = 3
    geo = oph.Geometry(m)
    x = oph.initial_state(m)
    ctrl = controls(m)
    sim = Sim(m, newton_tol=1e-10, lin_rtol=1e-11)
    _start_at_oracle_state(sim, m)
    total_cuts = 0
    for k in range(steps):
        dt = m["schedule"][k]
        assert dt == 5.0 * synth.DAY
        info = sim.timestep(dt)
        x, rep, ctrl = onewton.timestep(geo, x, dt, ctrl, tol=1e-10)
        total_cuts += info["cuts"]
        assert info["substeps"] == len(rep)
        assert info["mb_oil"] <= 1e-10 and info["mb_water"] <= 1e-10
        pg, sg, bg = sim.get_state()
        _compare(pg, sg, bg, x, geo.n)
        print("step %d: %d sub-steps, %d Newton" % (k, info["substeps"], info["newton_iters"]))
    sim.close()
