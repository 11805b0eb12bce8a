"""GPU parity of the other decoupling operators (Sec. 3.2: alternate block
factorisation, true-IMPES) and of the two-stage CPR-FP composition, against the
oracle's decouple(variant) and CPRFPF(variant).

Tolerances follow the rounding each operator adds.  An entry of the decoupled
matrix is judged against (|Q| |J|) at that entry, |Q| a bound of the 2x2 row
operator: Gauss-Jordan and true-IMPES multiply the second row by
f = a01/a11 (or c01/c11) and add it to the first; ABF multiplies by J_ii^-1,
whose entries carry the determinant's relative rounding error, at most a few
units times kappa = (|a00 a11| + |a01 a10|) / |det a|, so its rows get
1e-12 (1 + kappa).  For true-IMPES, f = c01/c11 is a quotient of two sums
over block column i, and its rounding is bounded by
F = (sum_k |J_ki,01| + |f| sum_k |J_ki,11|) / |c11|, which takes f's place in |Q|.  The preconditioner is compared to 1e-10 as the
FPF one is."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from gpu_common import random_state_pair, rel_max, require_gpu, sim_at, oracle_system
from oracle import cpr as ocpr
from oracle import physics as oph

pytestmark = pytest.mark.gpu

MODELS = {
    "c0": lambda: synth.model_small(),
    "tiny_grav": lambda: synth.model_tiny(4, 3, 2, seed=3),
    "ragged": lambda: synth.model_tiny(7, 5, 3, seed=6),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _abs_q_and_kappa(J, n_node_rows, variant):
    """Block-diagonal |Q| (identity on well rows) and a per-row rounding factor."""
    J = J.tocsr()
    N = J.shape[0]
    nd = n_node_rows // 2
    a00 = J.diagonal()[0:n_node_rows:2]
    a11 = J.diagonal()[1:n_node_rows:2]
    a01 = J.diagonal(1)[0:n_node_rows:2]
    a10 = J.diagonal(-1)[0:n_node_rows:2]
    q = np.zeros((N // 2, 2, 2))
    q[:, 0, 0] = q[:, 1, 1] = 1.0
    kappa = np.zeros(N)
    if variant == "gj":
        q[:nd, 0, 1] = np.abs(a01 / a11)
    elif variant == "ti":
        # block column sums: c01 of node i sums the first rows' entries in
        # column 2i+1, c11 the second rows'
        even = np.zeros(N)
        even[0::2] = 1.0
        odd = 1.0 - even
        c01 = (J.T @ even)[1:n_node_rows:2]
        c11 = (J.T @ odd)[1:n_node_rows:2]
        s01 = (abs(J).T @ even)[1:n_node_rows:2]
        s11 = (abs(J).T @ odd)[1:n_node_rows:2]
        f = np.abs(c01 / c11)
        q[:nd, 0, 1] = (s01 + f * s11) / np.abs(c11)
    else:
        det = a00 * a11 - a01 * a10
        q[:nd] = np.abs(np.stack([np.stack([a11, -a01], -1), np.stack([-a10, a00], -1)], -2) / det[:, None, None])
        k = (np.abs(a00 * a11) + np.abs(a01 * a10)) / np.abs(det)
        kappa[0:n_node_rows:2] = k
        kappa[1:n_node_rows:2] = k
    r = (2 * np.arange(N // 2)[:, None, None] + np.arange(2)[None, :, None]).repeat(2, axis=2)
    cidx = (2 * np.arange(N // 2)[:, None, None] + np.arange(2)[None, None, :]).repeat(2, axis=1)
    Q = sp.csr_matrix((q.ravel(), (r.ravel(), cidx.ravel())), shape=(N, N))
    return Q, kappa


@pytest.mark.parametrize("variant", ["gj", "abf", "ti"])
@pytest.mark.parametrize("name", sorted(MODELS))
def test_decoupled_system_matches_oracle(name, variant):
    m = MODELS[name]()
    x, x_old = random_state_pair(m, 3)
    geo, R, J = oracle_system(m, x, x_old, synth.DAY)
    sim = sim_at(m, x, x_old, synth.DAY, decoupling=variant)
    sim.setup()
    Ag, bg = sim.export_system(1)
    indptr, indices, data = oph.to_bsr(geo, J)
    dh, bh = ocpr.decouple(2 * geo.n, indptr, indices, data, -R, variant=variant)
    Ah = oph.bsr_to_csr(indptr, indices, dh)
    Q, kappa = _abs_q_and_kappa(J, 4 * geo.n, variant)
    scale = (Q @ abs(J.tocsr())).toarray()
    D = np.abs((Ag - Ah).toarray())
    bound = 1e-12 * (1.0 + kappa)[:, None] * scale
    assert np.all(D <= bound)
    # the right-hand side: the oracle's operator applied to the device's own
    # residual (the residual's rounding is judged by the assembly tests)
    _, Rg = sim.export_system(0)
    _, bhg = ocpr.decouple(2 * geo.n, indptr, indices, data, -Rg, variant=variant)
    assert np.all(np.abs(bg - bhg) <= 1e-12 * (1.0 + kappa) * (Q @ np.abs(Rg)))
    if variant == "abf":
        # every node diagonal block is the identity, to the rounding bound of Q J_ii
        for i in range(2 * geo.n):
            sl = slice(2 * i, 2 * i + 2)
            blk = Ag[sl, sl].toarray()
            assert np.all(np.abs(blk - np.eye(2)) <= 1e-12 * (1.0 + kappa[2 * i]) * scale[sl, sl])
    sim.close()


@pytest.mark.parametrize("decoupling,cpr", [("gj", "fp"), ("abf", "fpf"), ("ti", "fpf"), ("abf", "fp"),
                                            ("ti", "fp")])
@pytest.mark.parametrize("name", ["c0", "medium"])
def test_preconditioner_variant_and_gmres_match_oracle(name, decoupling, cpr):
    """On the small model at a random state, and on the 144k-DOF model at its
    first Newton iterate (a random state of that model gives true-IMPES a
    reduced pressure matrix with negative diagonal entries, on which GMRES
    stalls in the oracle as on the device)."""
    if name == "medium":
        m = synth.model_layered()
        x = x_old = oph.initial_state(m)
        dt = 5 * synth.DAY
    else:
        m = MODELS[name]()
        x, x_old = random_state_pair(m, 9)
        dt = synth.DAY
    geo, R, J = oracle_system(m, x, x_old, dt)
    sim = sim_at(m, x, x_old, dt, decoupling=decoupling, cpr_variant=cpr)
    sim.setup()
    indptr, indices, data = oph.to_bsr(geo, J)
    dh, bh = ocpr.decouple(2 * geo.n, indptr, indices, data, -R, variant=decoupling)
    pc = ocpr.CPRFPF(geo, indptr, indices, dh, variant=cpr)
    v = np.random.default_rng(4).standard_normal(geo.N)
    z = sim.apply_precond(v)
    zo = pc.apply(v)
    for comp in (0, 1):
        assert rel_max(z[comp::2], zo[comp::2]) <= 1e-10
    rtol = 1e-8
    its, rel = sim.solve(rtol, 300)
    _, its_o, _ = ocpr.gmres(lambda q: pc.A @ q, pc.apply, bh, rtol)
    assert rel <= rtol
    assert abs(its - its_o) <= 1
    sim.close()


@pytest.mark.parametrize("decoupling,cpr", [("abf", "fpf"), ("ti", "fp")])
def test_newton_step_with_variant_matches_oracle(decoupling, cpr):
    """A whole timestep with another decoupling and composition reaches the same
    state as the oracle's Newton loop (the nonlinear solution does not depend on
    the preconditioner; tight tolerances)."""
    from paper_1808_04338_amd import Sim
    from oracle import newton as onewton

    m = synth.model_small()
    geo = oph.Geometry(m)
    dt = m["schedule"][0]
    sim = Sim(m, newton_tol=1e-10, lin_rtol=1e-11, decoupling=decoupling, cpr_variant=cpr)
    sim.timestep(dt)
    pg, sg, bg = sim.get_state()
    sim.close()
    x, rep, ctrl = onewton.timestep(geo, oph.initial_state(m), dt, [w["control"] for w in m["wells"]],
                                    tol=1e-10)
    po, so, bo = oph.unpack_state(x, geo.n)
    assert rel_max(pg, po) <= 1e-9
    assert np.abs(sg - so).max() <= 1e-9
    assert rel_max(bg, bo) <= 1e-9
