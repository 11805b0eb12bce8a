"""GPU (HIP, through the C ABI) against the CPU oracle, element by element.

Tolerances: assembled residual and Jacobian 1e-12 relative (the arithmetic is
the same up to rounding order); decoupled system, ILU(0) factors, AMG
hierarchy and the preconditioner 1e-10 relative (FP64 with different
summation orders); Newton states after a timestep 1e-9 relative in pressure
and 1e-9 absolute in saturation (the required parity bar).
"""
import numpy as np
import pytest

import synth
from gpu_common import (controls, decoupled_err, oracle_cpr, oracle_system, random_state_pair,
                        rel_max, require_gpu, row_scaled_err, sim_at, sparse_rel)
from oracle import cpr as ocpr
from oracle import newton as onewton
from oracle import physics as oph

pytestmark = pytest.mark.gpu

MODELS = {
    "c0": lambda: synth.model_small(),
    "tiny_grav": lambda: synth.model_tiny(4, 3, 2, seed=3),
    "tiny_nowell": lambda: synth.model_tiny(3, 2, 2, seed=4, wells=False),
    "column": lambda: synth.model_tiny(2, 1, 6, seed=5),
    "ragged": lambda: synth.model_tiny(7, 5, 3, seed=6),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("name", sorted(MODELS))
def test_assembly_matches_oracle(name):
    m = MODELS[name]()
    for seed in (1, 2):
        x, x_old = random_state_pair(m, seed)
        dt = 2.5 * synth.DAY
        geo, R, J = oracle_system(m, x, x_old, dt)
        sim = sim_at(m, x, x_old, dt)
        Jg, Rg = sim.export_system(0)
        assert rel_max(Rg, R) <= 1e-12
        assert row_scaled_err(Jg, J) <= 1e-12
        sim.close()


def test_assembly_medium_model():
    m = synth.model_layered()
    x, x_old = random_state_pair(m, 7)
    dt = 5 * synth.DAY
    geo, R, J = oracle_system(m, x, x_old, dt)
    sim = sim_at(m, x, x_old, dt)
    Jg, Rg = sim.export_system(0)
    assert rel_max(Rg, R) <= 1e-12
    assert sparse_rel(Jg, J) <= 1e-12
    sim.close()


@pytest.mark.parametrize("name", ["c0", "tiny_grav", "ragged"])
def test_decoupling_and_ilu_match_oracle(name):
    m = MODELS[name]()
    x, x_old = random_state_pair(m, 3)
    dt = synth.DAY
    geo, R, J = oracle_system(m, x, x_old, dt)
    sim = sim_at(m, x, x_old, dt)
    sim.setup()
    Ag, bg = sim.export_system(1)
    pc, bh, (indptr, indices, dh) = oracle_cpr(geo, J, R)
    assert decoupled_err(Ag, J, pc.A) <= 1e-12
    assert rel_max(bg, bh) <= 1e-12
    ilu = pc.ilu
    perm, br, bc, vals = sim.export_ilu()
    # matrix nodes first (in any order among themselves: they are mutually
    # uncoupled, so the factors do not depend on it), then the fracture nodes
    # and wells in the oracle's order; blocks are compared by canonical index
    n = geo.n
    assert np.array_equal(np.sort(perm[:n]), np.sort(ilu.perm[:n]))
    assert np.array_equal(perm[n:], ilu.perm[n:])
    pos = ilu.pos
    for e in range(br.shape[0]):
        i, j = pos[br[e]], pos[bc[e]]
        cols, blocks = ilu.rows[i]
        ref = ilu.uinv[i] if i == j else blocks[cols.index(j)]
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(vals[e] - ref).max() <= 1e-10 * scale, (e, i, j)
    v = np.random.default_rng(0).standard_normal(geo.N)
    z = sim.apply_stage(0, v)
    zo = ilu.solve(v)
    for comp in (0, 1):
        assert rel_max(z[comp::2], zo[comp::2]) <= 1e-10
    sim.close()


@pytest.mark.parametrize("name", ["medium", "tall_well", "no_wells"])
def test_amg_hierarchy_matches_oracle(name):
    """Identical C/F splittings at every level (a deterministic rule), P and the
    Galerkin operators to 1e-10: on the 144k-DOF model; on a 6x6x900 model
    whose two wells perforate 900 layers, so that Galerkin rows of every length
    class occur (wavefront tiles, workgroup tiles and rows beyond the LDS tiles,
    which take the global sort path); and on a 40x40x6 model without wells,
    whose level 0 has no well rows for the stencil form of the V-cycle."""
    if name == "medium":
        m = synth.model_layered()
    elif name == "tall_well":
        m = synth.model_tiny(6, 6, 900, seed=6)
    else:
        m = synth.model_tiny(40, 40, 6, seed=8, wells=False)
    x, x_old = random_state_pair(m, 5)
    dt = 5 * synth.DAY
    geo, R, J = oracle_system(m, x, x_old, dt)
    sim = sim_at(m, x, x_old, dt)
    sim.setup()
    pc, bh, _ = oracle_cpr(geo, J, R)
    nl, rows, nnz = sim.amg_info()
    assert nl == len(pc.amg.levels) >= 3
    for lv in range(nl):
        g = sim.export_amg_level(lv)
        o = pc.amg.levels[lv]
        assert g["A"].shape == o["A"].shape
        assert sparse_rel(g["A"], o["A"]) <= 1e-10
        if lv < nl - 1:
            assert np.array_equal(g["cf"], o["state"])
            assert sparse_rel(g["P"], o["P"]) <= 1e-10
            assert g["P"].nnz == o["P"].nnz
    if name == "tall_well":
        assert sim.amg_global_sort_products() >= 1
    # the V-cycle on the reduced pressure system
    rr = np.random.default_rng(2).standard_normal(rows[0])
    e = sim.apply_stage(1, rr)
    eo = pc.amg.vcycle(rr)
    assert rel_max(e, eo) <= 1e-10
    sim.close()


@pytest.mark.parametrize("name", ["c0", "tiny_grav", "medium"])
def test_preconditioner_and_gmres_match_oracle(name):
    m = synth.model_layered() if name == "medium" else MODELS[name]()
    x, x_old = random_state_pair(m, 9)
    dt = synth.DAY
    geo, R, J = oracle_system(m, x, x_old, dt)
    sim = sim_at(m, x, x_old, dt)
    sim.setup()
    pc, bh, _ = oracle_cpr(geo, J, R)
    v = np.random.default_rng(4).standard_normal(geo.N)
    z = sim.apply_precond(v)
    zo = pc.apply(v)
    for comp in (0, 1):
        assert rel_max(z[comp::2], zo[comp::2]) <= 1e-10
    y = sim.apply_matrix(v)
    assert rel_max(y, pc.A @ v) <= 1e-13
    rtol = 1e-8
    its, rel = sim.solve(rtol, 300)
    _, its_o, rel_o = ocpr.gmres(lambda q: pc.A @ q, pc.apply, bh, rtol)
    assert rel <= rtol
    assert abs(its - its_o) <= 1
    sim.close()


@pytest.mark.parametrize("restart", [1, 4, 7])
def test_gmres_short_restarts_match_oracle(restart):
    """GMRES(m) with short cycles, so that several restarts occur: the vector
    left pending at the end of a cycle is dropped and the next cycle starts
    from the true residual.  Iteration counts within 1 of the oracle's GMRES
    with the same restart (48, 32 and 31 iterations there), and the device
    solution's residual recomputed with the oracle's matrix within rtol."""
    m = synth.model_layered()
    x, x_old = random_state_pair(m, 9)
    dt = synth.DAY
    geo, R, J = oracle_system(m, x, x_old, dt)
    sim = sim_at(m, x, x_old, dt, gmres_restart=restart)
    sim.setup()
    pc, bh, _ = oracle_cpr(geo, J, R)
    rtol = 1e-10
    its, rel = sim.solve(rtol, 400)
    _, its_o, rel_o = ocpr.gmres(lambda q: pc.A @ q, pc.apply, bh, rtol, restart=restart, maxit=400)
    assert its > restart  # at least one restart
    assert rel <= rtol
    assert abs(its - its_o) <= 1
    y = sim.get_correction()
    assert np.linalg.norm(bh - pc.A @ y) / np.linalg.norm(bh) <= 1.001 * rtol
    sim.close()


def test_dense_coarse_inverse_selftest():
    from paper_1808_04338_amd.sim import dense_inverse_selftest

    rng = np.random.default_rng(0)
    for n in (1, 31, 32, 33, 100, 300):
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        X = dense_inverse_selftest(A)
        assert np.abs(X @ A - np.eye(n)).max() <= 1e-12 * n


def test_dense_coarse_inverse_with_row_pivoting():
    """Rows shuffled inside every aligned 32-row panel, so that the pivot search
    picks off-diagonal rows and the swaps run (the inverse pivots inside each
    32 x 32 diagonal panel)."""
    from paper_1808_04338_amd.sim import dense_inverse_selftest

    rng = np.random.default_rng(1)
    for n in (32, 64, 100, 300):
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        perm = np.arange(n)
        for b0 in range(0, n, 32):
            perm[b0:b0 + 32] = b0 + rng.permutation(min(32, n - b0))
        Ap = A[perm]
        X = dense_inverse_selftest(Ap)
        assert np.abs(X @ Ap - np.eye(n)).max() <= 1e-12 * n


def test_one_level_hierarchy_is_exact():
    """With the coarse limit above the system size, the pressure stage is an
    exact solve (dense MFMA Gauss-Jordan inverse)."""
    m = synth.model_small()
    x, x_old = random_state_pair(m, 2)
    geo, R, J = oracle_system(m, x, x_old, synth.DAY)
    sim = sim_at(m, x, x_old, synth.DAY, amg_coarse_max=4000)
    sim.setup()
    assert sim.amg_info()[0] == 1
    pc, _, _ = oracle_cpr(geo, J, R, amg_opts=dict(max_coarse=4000))
    rr = np.random.default_rng(1).standard_normal(geo.n + geo.nw)
    e = sim.apply_stage(1, rr)
    assert np.abs(pc.S @ e - rr).max() <= 1e-9 * np.abs(rr).max()
    sim.close()


def _run_both(m, steps, **opts):
    from paper_1808_04338_amd import Sim

    sim = Sim(m, newton_tol=1e-10, lin_rtol=1e-11, **opts)
    geo = oph.Geometry(m)
    x = oph.initial_state(m)
    ctrl = controls(m)
    out = []
    for k in range(steps):
        dt = m["schedule"][k]
        info = sim.timestep(dt)
        x, rep, ctrl = onewton.timestep(geo, x, dt, ctrl, tol=1e-10)
        out.append((sim.get_state(), oph.unpack_state(x, geo.n), info, rep))
    sim.close()
    return out


@pytest.mark.parametrize("name", ["single_cell", "two_cells"])
def test_degenerate_grids_match_oracle(name):
    """The smallest systems the method has: one cell without wells (4
    unknowns; one-level hierarchy of one row, no second ILU colour), relaxing
    to matrix-fracture equilibrium over a long step, and two cells holding one
    injector and one producer."""
    m = synth.model_single_cell() if name == "single_cell" else synth.model_tiny(2, 1, 1, seed=8)
    for (pg, sg, bg), (po, so, bo), info, rep in _run_both(m, 1):
        assert rel_max(pg, po) <= 1e-9
        assert np.abs(sg - so).max() <= 1e-9
        if bo.size:
            assert rel_max(bg, bo) <= 1e-9
    if name == "single_cell":
        # equilibrium: both nodes at one pressure
        assert abs(pg[0] - pg[1]) <= 1e-6 * abs(pg[0])


@pytest.mark.parametrize("name", ["c0", "tiny_grav", "column"])
def test_timesteps_match_oracle(name):
    m = MODELS[name]()
    steps = len(m["schedule"]) if name == "c0" else 3
    for (pg, sg, bg), (po, so, bo), info, rep in _run_both(m, steps):
        assert rel_max(pg, po) <= 1e-9
        assert np.abs(sg - so).max() <= 1e-9
        if bo.size:
            assert rel_max(bg, bo) <= 1e-9
        assert info["mb_oil"] <= 1e-10 and info["mb_water"] <= 1e-10


def test_gpu_1d_closed_form():
    from paper_1808_04338_amd import Sim

    nx = 8
    k = np.exp(np.random.default_rng(5).normal(np.log(100.0), 1.0, nx)) * synth.MD
    m = synth.model_1d(nx=nx, k=k)
    sim = Sim(m, newton_tol=1e-12, lin_rtol=1e-12)
    sim.timestep(m["schedule"][0])
    p, sw, bhp = sim.get_state()
    geo = oph.Geometry(m)
    q = m["wells"][0]["target"]
    pf = p[0::2]
    for i in range(nx - 1):
        assert pf[i] - pf[i + 1] == pytest.approx(q * m["mu_w"] / geo.ft[i], rel=1e-9)
    assert pf[-1] == pytest.approx(m["wells"][1]["target"] + q * m["mu_w"] / geo.perfs[1][1][0], rel=1e-12)
    assert bhp[0] == pytest.approx(pf[0] + q * m["mu_w"] / geo.perfs[0][1][0], rel=1e-12)
    sim.close()


def test_deterministic_and_checkpoint_restore():
    """Two runs are bitwise equal; 2 steps = 1 step, checkpoint, restore, 1 step."""
    from paper_1808_04338_amd import Sim

    m = synth.model_small()
    dt = m["schedule"][0]
    a = Sim(m)
    a.timestep(dt)
    mid = a.get_state()
    a.timestep(dt)
    sa = a.get_state()
    b = Sim(m)
    b.timestep(dt)
    b.timestep(dt)
    sb = b.get_state()
    for u, v in zip(sa, sb):
        assert np.array_equal(u, v)
    c = Sim(m)
    c.set_state(*mid)
    c.timestep(dt)
    for u, v in zip(sa, c.get_state()):
        assert np.array_equal(u, v)
    for s in (a, b, c):
        s.close()


def test_mixed_precision_bound():
    """FP32 preconditioner under FP64 GMRES: the linear residual still meets
    its tolerance in FP64 and the Newton states agree with the FP64 oracle to
    the bound set by the tolerances."""
    from paper_1808_04338_amd import Sim

    m = synth.model_small()
    dt = m["schedule"][0]
    s32 = Sim(m, precision="fp32", newton_tol=1e-10, lin_rtol=1e-10)
    geo = oph.Geometry(m)
    x = oph.initial_state(m)
    ctrl = controls(m)
    for k in range(3):
        info = s32.timestep(dt)
        x, rep, ctrl = onewton.timestep(geo, x, dt, ctrl, tol=1e-10)
        p, sw, bhp = s32.get_state()
        po, so, bo = oph.unpack_state(x, geo.n)
        assert rel_max(p, po) <= 1e-8
        assert np.abs(sw - so).max() <= 1e-8
    # the linear solve itself reaches its tolerance
    s32.mark_old()
    s32.assemble(dt)
    s32.setup()
    its, rel = s32.solve(1e-6, 300)
    assert rel <= 1e-6
    s32.close()


def test_error_paths():
    from paper_1808_04338_amd import Sim
    from paper_1808_04338_amd._lib import DP_E_STATE, DpError

    m = synth.model_small()
    sim = Sim(m)
    with pytest.raises(DpError) as e:
        sim.solve(1e-6, 10)
    assert e.value.code == DP_E_STATE
    sim.assemble(synth.DAY)
    with pytest.raises(DpError) as e:
        sim.export_system(1)
    assert e.value.code == DP_E_STATE
    sim.close()


@pytest.mark.parametrize("choice", [1, 2, 3])
def test_adaptive_forcing_matches_oracle(choice):
    """Eq. (13) forcing terms on one 1-day step of the 1,200-DOF model with a
    multi-level (inexact) AMG.  Every tolerance the device chose equals the
    oracle's forcing_term evaluated on the device's own norms, and the converged
    state equals the oracle's.  (The Newton paths themselves differ: at loose
    tolerances the iterates depend on where GMRES stopped.)"""
    from paper_1808_04338_amd import Sim

    m = synth.model_small()
    dt = 1.0 * synth.DAY
    # enough iterations that neither side cuts the step (sub-steps change the answer)
    sim = Sim(m, precision="fp64", newton_tol=1e-10, forcing=choice, amg_coarse_max=20, max_newton=200)
    info = sim.timestep(dt)
    assert info["cuts"] == 0
    pg, sg, bg = sim.get_state()
    hist = sim.eta_history()
    sim.close()
    assert len(hist) >= 3
    for k, (eta, nb, nr, nd, it) in enumerate(hist):
        if it == 0:
            assert eta == 0.1
            continue
        e_prev, nb_prev, nr_prev = hist[k - 1][0], hist[k - 1][1], hist[k - 1][2]
        want = onewton.forcing_term(choice, e_prev, nb, nb_prev, nr_prev, nd)
        assert abs(eta - want) <= 1e-13 * want
    geo = oph.Geometry(m)
    x, rep, _ = onewton.timestep(geo, oph.initial_state(m), dt, controls(m), tol=1e-10, linear="cpr",
                                 forcing=choice, max_newton=200, cpr_opts=dict(amg_opts=dict(max_coarse=20)))
    assert len(rep) == 1
    po, so, bo = oph.unpack_state(x, geo.n)
    assert rel_max(pg, po) <= 1e-9
    assert np.abs(sg - so).max() <= 1e-9
    assert rel_max(bg, bo) <= 1e-9


@pytest.mark.parametrize("choice", [1, 2])
def test_adaptive_forcing_affine_floor(choice):
    """On an affine residual, b(x^1) - r^0 vanishes and ||b(x^1)|| = ||r^0||, so
    choices 1 and 2 of Eq. (13) give the floor eta_min at the second iteration."""
    from paper_1808_04338_amd import Sim

    m = synth.model_small()
    m["sw0"][:] = 0.9
    m["c_w"] = m["c_o"] = 0.0
    m["gravity"] = 0.0
    sim = Sim(m, precision="fp64", newton_tol=1e-11, mb_tol=1e-12, forcing=choice, amg_coarse_max=20)
    sim.timestep(synth.DAY)
    hist = sim.eta_history()
    sim.close()
    assert hist[0][0] == 0.1 and len(hist) >= 2
    assert hist[1][0] == 1e-8


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_preconditioner_graph_replay_matches_eager(precision):
    """The preconditioner replayed from its HIP graph gives bitwise the same GMRES
    iterates as the eager launches, over two setups (the second one updates the
    captured graph), with the library's own eager work between the replays."""
    m = synth.model_layered()
    x, x_old = random_state_pair(m, 9)
    dt = synth.DAY
    outs = []
    for eager in (1, 2):
        sim = sim_at(m, x, x_old, dt, precision=precision, precond_eager=eager)
        res = []
        for _ in range(2):
            sim.assemble(dt)
            sim.setup()
            its, rel = sim.solve(1e-8, 300, allow_noconv=True)
            res.append((its, sim.get_correction()))
        sim.close()
        outs.append(res)
    for (i1, y1), (i2, y2) in zip(*outs):
        assert i1 == i2
        assert np.array_equal(y1, y2)
