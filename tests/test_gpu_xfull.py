"""Parity at full size: the 60x220x85 channelised model (4,488,010 DOF) in the
configuration bench.py times (FP32 preconditioner, the third Newton iterate of
the first 10-day step, GMRES to 1e-6).

Where the oracle can compute the result at this size it is compared entry by
entry (residual, Jacobian, decoupled system, the solution's true residual);
the oracle's own AMG hierarchy is built at full size and compared level by
level; elsewhere properties that hold at any size are checked (the block
ILU(0) identity (LU)_ij = A_ij on the pattern on sampled rows, the Galerkin
identity A_1 = P^T A_0 P, and the PMIS cover rule).  One more test takes the
first Jacobian of bench.py's default workload, the converged state after the
first step of the run.  The file runs after the other GPU tests (its name sorts
last among them)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from gpu_common import controls, rel_max, sparse_rel
from oracle import cpr as ocpr
from oracle import physics as oph

pytestmark = pytest.mark.gpu

DT = 10.0 * synth.DAY


def _rowmax(A):
    A = abs(A).tocsr()
    out = np.zeros(A.shape[0])
    nz = np.diff(A.indptr) > 0
    if nz.any():
        out[nz] = np.maximum.reduceat(A.data, A.indptr[:-1][nz])
    return out


def _row_err(A, B, scale=None):
    """max over rows of max|A - B| / (row scale), the row scale max|B| unless given."""
    s = _rowmax(B) if scale is None else scale
    d = _rowmax((A - B).tocsr())
    ok = s > 0
    assert np.all(d[~ok] == 0.0)
    return (d[ok] / s[ok]).max()


@pytest.fixture(scope="module")
def full():
    from paper_1808_04338_amd import Sim

    m = synth.model_channelised()
    sim = Sim(m, precision="fp32", lin_rtol=1e-6)
    x_old = oph.initial_state(m)
    sim.mark_old()
    for _ in range(3):
        sim.newton_step(DT, 1e-6)
    p, s, b = sim.get_state()
    x = oph.pack_state(p, s, b)
    sim.assemble(DT)
    sim.setup()
    its, rel = sim.solve(1e-6, 300, allow_noconv=True)
    geo = oph.Geometry(m)
    acc = oph.accumulation(geo, x_old)
    R = oph.residual(geo, x, acc, DT, controls(m))
    J = oph.jacobian(geo, x, DT, controls(m)).tocsr()
    yield dict(m=m, sim=sim, geo=geo, x=x, R=R, J=J, its=its, rel=rel)
    sim.close()


def test_full_assembly(full):
    Jg, Rg = full["sim"].export_system(0)
    assert Jg.shape == full["J"].shape
    assert rel_max(Rg, full["R"]) <= 1e-12
    assert _row_err(Jg, full["J"]) <= 1e-12


@pytest.fixture(scope="module")
def decoupled(full):
    """The oracle's decoupled system D^-1 J, D^-1 (-R) at the full-size state."""
    geo, J, R = full["geo"], full["J"], full["R"]
    indptr, indices, data = oph.to_bsr(geo, J)
    dh, bh = ocpr.decouple(2 * geo.n, indptr, indices, data, -R)
    return oph.bsr_to_csr(indptr, indices, dh), bh


def test_full_decoupling_and_true_residual(full, decoupled):
    geo, J, R = full["geo"], full["J"], full["R"]
    Ag, bg = full["sim"].export_system(1)
    Ah, bh = decoupled
    # first node rows are judged against the magnitudes the Gauss-Jordan step
    # combined: |J_0j| + |a01/a11| |J_1j|
    nb = geo.N // 2
    d = J.diagonal()
    a01 = J.diagonal(1)[0:4 * geo.n:2]  # J[2q, 2q+1] of every node
    f = np.zeros(geo.N)
    f[0:4 * geo.n:2] = np.abs(a01 / d[1:4 * geo.n:2])
    shift = sp.csr_matrix((np.ones(nb), (2 * np.arange(nb), 2 * np.arange(nb) + 1)), shape=J.shape)
    S = abs(J) + sp.diags(f) @ (shift @ abs(J))
    assert _row_err(Ag, Ah, scale=_rowmax(S)) <= 1e-12
    assert rel_max(bg, bh) <= 1e-12
    # the GPU solution's decoupled residual, recomputed by the oracle
    y = full["sim"].get_correction()
    rel = np.linalg.norm(bh - Ah @ y) / np.linalg.norm(bh)
    assert full["rel"] <= 1e-6
    assert rel <= 1.001e-6


@pytest.fixture(scope="module")
def full64(full):
    """An FP64-preconditioner handle at the same old and current state."""
    from paper_1808_04338_amd import Sim

    m, geo = full["m"], full["geo"]
    sim = Sim(m, precision="fp64", lin_rtol=1e-6)
    po, so, bo = oph.unpack_state(oph.initial_state(m), geo.n)
    sim.set_state(po, so, bo)
    sim.mark_old()
    p, s, b = oph.unpack_state(full["x"], geo.n)
    sim.set_state(p, s, b)
    sim.assemble(DT)
    sim.setup()
    yield sim
    sim.close()


def test_full_fp64_form_solves_to_its_tolerance(full, full64, decoupled):
    """The plain FP64 form on the same Jacobian: GMRES reaches 1e-6 and its
    solution's decoupled residual, recomputed by the oracle, is within it."""
    Ah, bh = decoupled
    its, rel = full64.solve(1e-6, 300)
    y = full64.get_correction()
    rel_o = np.linalg.norm(bh - Ah @ y) / np.linalg.norm(bh)
    print("FP64 form: %d GMRES iterations, rel %.3e (oracle %.3e)" % (its, rel, rel_o))
    assert rel <= 1e-6
    assert rel_o <= 1.001e-6


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_block_ilu_identity_on_sampled_rows(full, full64, precision):
    """(LU)_ij = A_ij on the block pattern, on 3000 random block rows plus the
    well rows, in the elimination order, judged against the scale of the terms
    the factorisation summed, (|L||U|)_ij per row (the backward-error bound of a
    triangular factorisation): 1e-5 for the FP32 factors (of the FP32 matrix),
    1e-13 for the FP64 ones."""
    geo = full["geo"]
    sim = full["sim"] if precision == "fp32" else full64
    tol = 1e-5 if precision == "fp32" else 1e-13
    Ag, _ = sim.export_system(1)
    perm, br, bc, vals = sim.export_ilu()
    nb = perm.shape[0]
    pos = np.empty(nb, dtype=np.int64)
    pos[perm] = np.arange(nb)
    pi, pj = pos[br], pos[bc]
    lower = pi > pj
    diag = pi == pj
    upper = pi < pj

    def blocks_to_csr(rows, cols, blk):
        r = (2 * rows[:, None, None] + np.arange(2)[None, :, None]).repeat(2, axis=2)
        c = (2 * cols[:, None, None] + np.arange(2)[None, None, :]).repeat(2, axis=1)
        return sp.csr_matrix((blk.ravel(), (r.ravel(), c.ravel())), shape=(2 * nb, 2 * nb))

    # point matrices in elimination order: L unit lower, U upper with U_ii = inv(stored)
    udiag = np.linalg.inv(vals[diag])
    L = blocks_to_csr(pi[lower], pj[lower], vals[lower]) + sp.identity(2 * nb, format="csr")
    U = blocks_to_csr(pi[upper], pj[upper], vals[upper]) + blocks_to_csr(pi[diag], pj[diag], udiag)
    pp = np.empty(2 * nb, dtype=np.int64)
    pp[0::2] = 2 * pos
    pp[1::2] = 2 * pos + 1
    A = Ag.tocoo()
    Ael = sp.csr_matrix((A.data, (pp[A.row], pp[A.col])), shape=A.shape)
    rng = np.random.default_rng(5)
    brows = np.unique(np.concatenate([rng.choice(nb, 3000, replace=False), np.arange(nb - geo.nw, nb)]))
    prow = np.sort(np.concatenate([2 * brows, 2 * brows + 1]))
    pattern = (abs(L) + abs(U)).tocsr()
    pattern.data[:] = 1.0
    Lr = L[prow]
    LU = (Lr @ U).multiply(pattern[prow]).tocsr()
    scale = _rowmax((abs(Lr) @ abs(U)).multiply(pattern[prow]))
    assert _row_err(LU, Ael[prow], scale=scale) <= tol


@pytest.fixture(scope="module")
def oracle_amg(full):
    """The oracle's AMG hierarchy (NumPy/SciPy) on the full reduced pressure
    system of the full-size state."""
    geo, J, R = full["geo"], full["J"], full["R"]
    indptr, indices, data = oph.to_bsr(geo, J)
    dh, _ = ocpr.decouple(2 * geo.n, indptr, indices, data, -R)
    perm = ocpr.default_ordering(geo)
    App = ocpr.pressure_matrix(indptr, indices, dh)[perm][:, perm].tocsr()
    S, _ = ocpr.reduced_pressure_matrix(App, geo.n)
    return ocpr.AMG(S)


def test_full_amg_hierarchy_matches_oracle(full, oracle_amg):
    """The oracle builds its own AMG hierarchy on the full reduced pressure
    system: identical C/F splittings at every level, P and A_l to 1e-10; plus
    the Galerkin identity A_1 = P^T A_0 P and the PMIS cover rule on the
    device's own level 0."""
    sim = full["sim"]
    amg = oracle_amg
    nl, rows, nnz = sim.amg_info()
    assert nl == len(amg.levels) >= 3
    for lv in range(nl):
        g = sim.export_amg_level(lv)
        o = amg.levels[lv]
        assert g["A"].shape == o["A"].shape
        assert sparse_rel(g["A"], o["A"]) <= 1e-10
        if lv < nl - 1:
            assert np.array_equal(g["cf"], o["state"])
            assert g["P"].nnz == o["P"].nnz
            assert sparse_rel(g["P"], o["P"]) <= 1e-10
    g0 = sim.export_amg_level(0)
    A0, P0, cf = g0["A"].tocsr(), g0["P"].tocsr(), g0["cf"]
    A1 = (P0.T @ A0 @ P0).tocsr()
    assert sparse_rel(sim.export_amg_level(1)["A"], A1) <= 1e-10
    # PMIS cover: every F point that influences another depends strongly on a C point
    sm = ocpr.strength(A0, 0.25)
    r = np.repeat(np.arange(A0.shape[0]), np.diff(A0.indptr))
    c = A0.indices
    nst = np.bincount(c[sm], minlength=A0.shape[0])
    hasc = np.zeros(A0.shape[0], dtype=bool)
    hasc[r[sm & (cf[c] == 1)]] = True
    assert np.all(hasc[(cf == -1) & (nst > 0)])


def test_full_vcycle_matches_oracle(full64, oracle_amg):
    """The FP64 V-cycle at full size against the oracle's, on two random
    right-hand sides, to 1e-10: every level operator kind of the apply runs
    here (level 0 in stencil form, CSR row blocks with 4 and 8 lanes per row
    on levels 1-3, SELL-64 prolongations, the dense coarsest level)."""
    nl, rows, _ = full64.amg_info()
    assert nl == len(oracle_amg.levels)
    rng = np.random.default_rng(12)
    for _ in range(2):
        rr = rng.standard_normal(rows[0])
        e = full64.apply_stage(1, rr)
        eo = oracle_amg.vcycle(rr)
        assert rel_max(e, eo) <= 1e-10


def _residual_err(m, geo, x, acc_old, dt, Rg, R):
    """max over rows of |Rg - R| over the size of the terms the row sums.  At a
    converged state the terms cancel, so the row's own value is no scale for
    rounding.  Node rows: (|M_a(x)| + |M_a^n|)/dt + |the flux, transfer and
    well part|.  Well rows: |R| + rho_ref |target| for rate and oil-rate rows,
    |R| + |target| for BHP rows."""
    n = geo.n
    scale = np.zeros_like(R)
    for a, acc_new in enumerate(oph.accumulation(geo, x)):
        rows = slice(a, 4 * n, 2)
        dm = (acc_new - acc_old[a]) / dt
        scale[rows] = (np.abs(acc_new) + np.abs(acc_old[a])) / dt + np.abs(R[rows] - dm)
    for w, wl in enumerate(m["wells"]):
        r = 4 * n + 2 * w
        rho = {"rate": m["rho_w_ref"], "orate": m["rho_o_ref"]}.get(wl["control"], 1.0)
        scale[r] = abs(R[r]) + rho * abs(wl["target"])
        scale[r + 1] = max(abs(R[r + 1]), 1.0)  # the dummy row
    return (np.abs(Rg - R) / scale).max()


def test_full_run_state_matches_oracle(full):
    """The first Jacobian of bench.py's default workload (the Jacobian set of a
    run): the converged state after the first 10-day step, with the initial
    state as the old time level and the 10-day step length.  Residual and
    Jacobian against the oracle's at 1e-12 of each row's scale (for the
    residual, the size of the terms it sums), and the GPU
    solution's decoupled residual recomputed by the oracle within 1.001e-6."""
    from paper_1808_04338_amd import Sim

    m, geo = full["m"], full["geo"]
    dt = m["schedule"][0]
    run = Sim(m, precision="fp32")
    old = run.get_state()
    run.timestep(dt)
    cur = run.get_state()
    run.close()
    sim = Sim(m, precision="fp32", lin_rtol=1e-6)
    try:
        sim.set_state(*old)
        sim.mark_old()
        sim.set_state(*cur)
        sim.assemble(dt)
        sim.setup()
        its, rel_g = sim.solve(1e-6, 300, allow_noconv=True)
        x_old, x = oph.pack_state(*old), oph.pack_state(*cur)
        acc = oph.accumulation(geo, x_old)
        R = oph.residual(geo, x, acc, dt, controls(m))
        J = oph.jacobian(geo, x, dt, controls(m)).tocsr()
        Jg, Rg = sim.export_system(0)
        assert _residual_err(m, geo, x, acc, dt, Rg, R) <= 1e-12
        assert _row_err(Jg, J) <= 1e-12
        indptr, indices, data = oph.to_bsr(geo, J)
        dh, bh = ocpr.decouple(2 * geo.n, indptr, indices, data, -R)
        Ah = oph.bsr_to_csr(indptr, indices, dh)
        y = sim.get_correction()
        assert rel_g <= 1e-6 and its > 10  # harder than the first-step Jacobian
        assert np.linalg.norm(bh - Ah @ y) / np.linalg.norm(bh) <= 1.001e-6
    finally:
        sim.close()
