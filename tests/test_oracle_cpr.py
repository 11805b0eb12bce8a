"""Pins of the oracle's decoupling, block ILU(0), AMG, CPR-FPF and GMRES
against textbook characterisations and closed forms (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import cpr
from oracle import physics as ph


def _system(m, seed=3, dt=synth.DAY):
    geo = ph.Geometry(m)
    ctrl = [w["control"] for w in m["wells"]]
    x = ph.pack_state(*synth.random_state(m, seed))
    acc_old = ph.accumulation(geo, ph.initial_state(m))
    R = ph.residual(geo, x, acc_old, dt, ctrl)
    J = ph.jacobian(geo, x, dt, ctrl)
    return geo, J, -R


def test_decoupling_definition():
    geo, J, b = _system(synth.model_small())
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, bh = cpr.decouple(2 * geo.n, indptr, indices, data, b)
    Ah = ph.bsr_to_csr(indptr, indices, dh)
    # the transformed system has the same solution
    y = spla.spsolve(J.tocsc(), b)
    yh = spla.spsolve(Ah.tocsc(), bh)
    assert np.allclose(y, yh, rtol=1e-9, atol=0)
    # the node's own saturation is removed from its first equation
    nb = 2 * geo.n + geo.nw
    rows = np.repeat(np.arange(nb), np.diff(indptr))
    diag = indices == rows
    node = rows < 2 * geo.n
    a01 = np.abs(dh[diag & node][:, 0, 1])
    scale = np.abs(data[diag & node][:, 0, 1]) + np.abs(data[diag & node][:, 1, 1])
    assert np.all(a01 <= 1e-14 * scale)
    # second rows untouched, well rows untouched
    assert np.array_equal(dh[:, 1, :], data[:, 1, :])
    assert np.array_equal(dh[rows >= 2 * geo.n], data[rows >= 2 * geo.n])


def test_bilu0_textbook_characterisation():
    """(L U)_ij = A_ij on every block (i, j) of the pattern."""
    geo, J, b = _system(synth.model_tiny(4, 3, 2, seed=2))
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, _ = cpr.decouple(2 * geo.n, indptr, indices, data, b)
    perm = cpr.default_ordering(geo)
    ilu = cpr.BlockILU0(indptr, indices, dh, perm)
    nb = ilu.nb
    Ld = {}
    Ud = {}
    for i, c, v in ilu.factors():
        (Ld if c < i else Ud)[(i, c)] = v
    for i in range(nb):
        Ld[(i, i)] = np.eye(2)
    # (LU)_ij = sum_k L_ik U_kj
    pos = ilu.pos
    Lrows = {}
    for (i, k), v in Ld.items():
        Lrows.setdefault(i, []).append((k, v))
    for r in range(nb):
        for t in range(indptr[r], indptr[r + 1]):
            i, j = pos[r], pos[indices[t]]
            acc = np.zeros((2, 2))
            for k, lv in Lrows[i]:
                if (k, j) in Ud:
                    acc += lv @ Ud[(k, j)]
            ref = dh[t]
            assert np.allclose(acc, ref, rtol=1e-11, atol=1e-11 * np.abs(dh[indptr[r]:indptr[r + 1]]).max())


def test_bilu0_exact_without_fill():
    """With no wells and the ordering (m_c, f_c) cell by cell along a 1-D
    chain, elimination creates no fill, so ILU(0) is the exact LU."""
    m = synth.model_tiny(6, 1, 1, seed=4, wells=False)
    geo, J, b = _system(m)
    indptr, indices, data = ph.to_bsr(geo, J)
    perm = np.ravel(np.column_stack([2 * np.arange(geo.n) + 1, 2 * np.arange(geo.n)]))
    ilu = cpr.BlockILU0(indptr, indices, data, perm)
    y = ilu.solve(b)
    yref = spla.spsolve(J.tocsc(), b)
    assert np.allclose(y, yref, rtol=1e-11, atol=0)


def test_default_ordering_matrix_nodes_eliminated_exactly():
    """Matrix nodes first: each couples only to its own fracture node, so their
    elimination is exact and the fracture diagonal becomes the Schur complement."""
    geo, J, b = _system(synth.model_small())
    indptr, indices, data = ph.to_bsr(geo, J)
    perm = cpr.default_ordering(geo)
    ilu = cpr.BlockILU0(indptr, indices, data, perm)
    A = {}
    nb = ilu.nb
    for r in range(nb):
        for t in range(indptr[r], indptr[r + 1]):
            A[(r, indices[t])] = data[t]
    red_f = perm[geo.n]          # first red fracture node (canonical index)
    mm = red_f + 1
    schur = A[(red_f, red_f)] - A[(red_f, mm)] @ np.linalg.inv(A[(mm, mm)]) @ A[(mm, red_f)]
    i = ilu.pos[red_f]
    assert np.allclose(np.linalg.inv(ilu.uinv[i]), schur, rtol=1e-12)


def test_bilu0_does_not_depend_on_the_order_of_the_matrix_nodes():
    """The matrix nodes are mutually uncoupled, so listing them in another order
    (still before every fracture node) gives the same L and U blocks and the
    same inverted diagonals, block for block in canonical indices."""
    geo, J, b = _system(synth.model_small())
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, _ = cpr.decouple(2 * geo.n, indptr, indices, data, b)
    perm = cpr.default_ordering(geo)
    other = perm.copy()
    other[:geo.n] = np.random.default_rng(5).permutation(perm[:geo.n])
    assert not np.array_equal(other, perm)
    ilus = [cpr.BlockILU0(indptr, indices, dh, p) for p in (perm, other)]
    blocks = []
    for ilu in ilus:
        d = {(int(ilu.perm[i]), int(ilu.perm[c])): v for i, c, v in ilu.factors()}
        for i in range(ilu.nb):
            d[("inv", int(ilu.perm[i]))] = ilu.uinv[i]
        blocks.append(d)
    assert blocks[0].keys() == blocks[1].keys()
    for key, v in blocks[0].items():
        assert np.array_equal(v, blocks[1][key]), key


def _poisson2d(nx, ny, shift=0.0, rng=None):
    n = nx * ny
    rows, cols, vals = [], [], []
    for j in range(ny):
        for i in range(nx):
            c = i + nx * j
            d = shift
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < nx and 0 <= jj < ny:
                    w = 1.0 if rng is None else float(np.exp(rng.normal()))
                    rows.append(c)
                    cols.append(ii + nx * jj)
                    vals.append(-w)
                    d += w
            rows.append(c)
            cols.append(c)
            vals.append(d)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    # symmetrise weights for the random case
    if rng is not None:
        off = A - sp.diags(A.diagonal())
        off = 0.5 * (off + off.T)
        A = (off + sp.diags(-np.asarray(off.sum(axis=1)).ravel() + shift)).tocsr()
    A.sort_indices()
    return A


def test_lowbias32_is_a_bijection_sample():
    h = cpr.lowbias32(np.arange(1 << 20))
    assert np.unique(h).shape[0] == 1 << 20
    assert h.max() < 2 ** 32


def test_pmis_independence_and_cover():
    A = _poisson2d(20, 20, shift=0.01, rng=np.random.default_rng(1))
    sm = cpr.strength(A, 0.25)
    state = cpr.pmis(A, sm)
    A = A.tocsr()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    # no two C points are strongly connected
    assert not np.any(sm & (state[rows] == 1) & (state[cols] == 1))
    # every F point that influences someone depends strongly on a C point
    nst = np.bincount(cols[sm], minlength=A.shape[0])
    hasc = np.zeros(A.shape[0], dtype=bool)
    hasc[rows[sm & (state[cols] == 1)]] = True
    assert np.all(hasc[(state == -1) & (nst > 0)])


def test_interpolation_1d_laplacian_is_linear():
    """Tridiagonal Laplacian with alternate C points: interpolation is the
    average of the two neighbours (1/2, 1/2)."""
    n = 9
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    sm = cpr.strength(A, 0.25)
    state = np.where(np.arange(n) % 2 == 0, 1, -1)
    P = cpr.interpolation(A, sm, state).toarray()
    for i in range(1, n - 1, 2):
        c = i // 2
        assert P[i, c] == pytest.approx(0.5) and P[i, c + 1] == pytest.approx(0.5)
        assert np.count_nonzero(P[i]) == 2


def test_interpolation_reproduces_constants_on_zero_row_sums():
    A = _poisson2d(16, 16, rng=np.random.default_rng(3))  # pure Neumann: zero row sums
    sm = cpr.strength(A, 0.25)
    state = cpr.pmis(A, sm)
    P = cpr.interpolation(A, sm, state)
    rs = np.asarray(P.sum(axis=1)).ravel()
    has = np.diff(P.tocsr().indptr) > 0
    assert np.allclose(rs[has], 1.0, rtol=1e-12)
    assert np.max(np.diff(P.tocsr().indptr)) <= 3


def test_amg_galerkin_and_exact_coarse():
    geo, J, b = _system(synth.model_small())
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, _ = cpr.decouple(2 * geo.n, indptr, indices, data, b)
    Ap = cpr.pressure_matrix(indptr, indices, dh)
    amg = cpr.AMG(Ap, max_coarse=40)
    assert len(amg.levels) >= 3
    for l in range(len(amg.levels) - 1):
        lv = amg.levels[l]
        Ac = amg.levels[l + 1]["A"].toarray()
        ref = lv["P"].toarray().T @ lv["A"].toarray() @ lv["P"].toarray()
        assert np.allclose(Ac, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    # one-level hierarchy: the V-cycle is an exact solve
    one = cpr.AMG(Ap, max_coarse=10 ** 6)
    assert len(one.levels) == 1
    rhs = np.random.default_rng(0).standard_normal(Ap.shape[0])
    x = one.vcycle(rhs)
    assert np.allclose(Ap @ x, rhs, rtol=1e-9, atol=1e-9 * np.abs(rhs).max())


def test_vcycle_contracts_on_poisson():
    A = _poisson2d(40, 40, shift=1e-3, rng=np.random.default_rng(2))
    amg = cpr.AMG(A, max_coarse=50)
    assert len(amg.levels) >= 3
    rng = np.random.default_rng(5)
    xs = rng.standard_normal(A.shape[0])
    b = A @ xs
    x = np.zeros_like(b)
    e0 = np.linalg.norm(xs)
    for _ in range(8):
        x = x + amg.vcycle(b - A @ x)
    # l1-Jacobi V(1,1): a contraction of about 0.6 per cycle here
    assert np.linalg.norm(xs - x) <= 0.7 ** 8 * e0


def test_gmres_arnoldi_relation_and_orthogonality():
    A = _poisson2d(15, 15, shift=0.1, rng=np.random.default_rng(4)) + sp.diags(np.linspace(0, 1, 225))
    A = A.tocsr()
    b = np.random.default_rng(1).standard_normal(225)
    Dinv = 1.0 / A.diagonal()
    tr = {}
    x, its, rel = cpr.gmres(lambda v: A @ v, lambda v: Dinv * v, b, 1e-14, restart=20, maxit=20, trace=tr)
    V, Z, H = tr["V"], tr["Z"], tr["H"]
    k = Z.shape[0]
    AZ = np.stack([A @ Z[j] for j in range(k)])
    lhs = AZ.T
    rhs = V.T @ H
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * spla.norm(A) * np.sqrt(k)
    # 1e-14 needs the re-orthogonalisation: a single classical Gram-Schmidt
    # pass leaves about 3e-13 on this problem
    assert np.abs(V @ V.T - np.eye(V.shape[0])).max() <= 1e-14


def test_gmres_iterate_minimises_the_residual_over_the_krylov_space():
    """After k < n iterations (no restart) the iterate is x = M^-1 K c with K the
    Krylov basis [r, (A M^-1) r, ..., (A M^-1)^(k-1) r] and c minimising
    |b - A M^-1 K c|, found here by a dense least-squares solve on the explicit
    (column-scaled) basis."""
    rng = np.random.default_rng(11)
    n = 60
    A = (sp.diags(np.linspace(1.0, 4.0, n)) + 0.3 * sp.random(n, n, density=0.1, random_state=5)).tocsr()
    b = rng.standard_normal(n)
    d = 1.0 / A.diagonal()
    for k in (1, 3, 6):
        x, its, rel = cpr.gmres(lambda v: A @ v, lambda v: d * v, b, 1e-15, restart=30, maxit=k)
        assert its == k
        K = np.zeros((n, k))
        v = b.copy()
        for i in range(k):
            K[:, i] = v / np.linalg.norm(v)
            v = A @ (d * K[:, i])
        MK = d[:, None] * K
        c, *_ = np.linalg.lstsq(A @ MK, b, rcond=None)
        xref = MK @ c
        assert np.linalg.norm(x - xref) <= 1e-9 * np.linalg.norm(xref)
        assert abs(rel - np.linalg.norm(b - A @ xref) / np.linalg.norm(b)) <= 1e-9


def test_gmres_finite_termination_diagonal():
    k = 7
    d = np.repeat(np.arange(1.0, k + 1.0), 20)
    A = sp.diags(d).tocsr()
    b = np.random.default_rng(2).standard_normal(d.shape[0])
    x, its, rel = cpr.gmres(lambda v: A @ v, lambda v: v, b, 1e-12, restart=30)
    assert its <= k
    assert rel <= 1e-12


def test_cpr_with_exact_full_stage_converges_in_one_iteration():
    geo, J, b = _system(synth.model_small())
    y, its, rel = cpr.solve(geo, J, b, rtol=1e-10, exact_f=True)
    assert its == 1


def test_cpr_gmres_matches_direct_solve():
    geo, J, b = _system(synth.model_small(), seed=11)
    y, its, rel = cpr.solve(geo, J, b, rtol=1e-12)
    yref = spla.spsolve(J.tocsc(), b)
    assert rel <= 1e-12
    # compare the two components on their own scales
    for comp in (0, 1):
        a, r = y[comp:4 * geo.n:2], yref[comp:4 * geo.n:2]
        assert np.abs(a - r).max() <= 1e-8 * np.abs(r).max()
    assert 1 <= its <= 30


def test_reduced_pressure_solve_is_exact_with_one_level():
    """Eliminating the matrix-node pressures is exact: with a one-level
    hierarchy the pressure stage returns A_p^-1 r."""
    geo, J, b = _system(synth.model_small(), seed=5)
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, _ = cpr.decouple(2 * geo.n, indptr, indices, data, b)
    pc = cpr.CPRFPF(geo, indptr, indices, dh, amg_opts=dict(max_coarse=10 ** 6))
    assert len(pc.amg.levels) == 1
    assert pc.S.shape[0] == geo.n + geo.nw
    rp = np.random.default_rng(3).standard_normal(pc.Ap.shape[0])
    e = pc.pressure_solve(rp)
    ref = spla.spsolve(pc.Ap.tocsc(), rp)
    assert np.allclose(e, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    # the reduced matrix keeps the fracture/well pattern; only its diagonal changed
    n = geo.n
    blk = pc.App[n:, n:].tocsr()
    blk.sort_indices()
    assert np.array_equal(blk.indptr, pc.S.indptr) and np.array_equal(blk.indices, pc.S.indices)
    off = blk.indices != np.repeat(np.arange(blk.shape[0]), np.diff(blk.indptr))
    assert np.array_equal(blk.data[off], pc.S.data[off])


def test_abf_decoupling_makes_node_diagonal_blocks_the_identity():
    geo, J, b = _system(synth.model_small())
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, _ = cpr.decouple(2 * geo.n, indptr, indices, data, b, "abf")
    nb = indptr.shape[0] - 1
    rows = np.repeat(np.arange(nb), np.diff(indptr))
    sel = (indices == rows) & (rows < 2 * geo.n)
    d = dh[sel]
    # the blocks mix units (Pa and saturation): each entry is judged against the
    # magnitudes the product combined, (|a^-1| |a|)_ij
    a = data[sel]
    scale = np.einsum("rij,rjk->rik", np.abs(np.linalg.inv(a)), np.abs(a))
    assert np.max(np.abs(d - np.eye(2)) / scale) <= 1e-12


def test_true_impes_weights_are_the_density_ratio():
    """Fluxes between nodes (faces and matrix-fracture transfer) are
    conservative, so they cancel in a block column sum; what is left in the
    column of a node without a perforation is its accumulation derivative,
    d/dS_w of (V phi (1 - S_w) rho_o, V phi S_w rho_w) / dt, and the true-IMPES
    weight Q01 = -c01/c11 is rho_o(p)/rho_w(p) at that node: the pressure row
    becomes the volume balance R_o/rho_o + R_w/rho_w, scaled by rho_o.  Judged against
    the rounding of the column sums, sum_k |J_ki| / |c_i|."""
    m = synth.model_small()
    geo, J, b = _system(m, seed=4)
    indptr, indices, data = ph.to_bsr(geo, J)
    Q = cpr.decoupling_operator(2 * geo.n, indptr, indices, data, "ti")
    p, _, _ = ph.unpack_state(ph.pack_state(*synth.random_state(m, 4)), geo.n)
    rho_o, _ = ph.density(p, m["rho_o_ref"], m["c_o"], m["p_ref"])
    rho_w, _ = ph.density(p, m["rho_w_ref"], m["c_w"], m["p_ref"])
    nb = indptr.shape[0] - 1
    absum = np.zeros((nb, 2, 2))
    csum = np.zeros((nb, 2, 2))
    np.add.at(absum, indices, np.abs(data))
    np.add.at(csum, indices, data)
    perforated = np.zeros(2 * geo.n, dtype=bool)
    for cells, _ in geo.perfs:
        perforated[2 * cells] = True  # wells perforate fracture nodes
    free = ~perforated
    assert free.sum() > geo.n
    w = Q[:2 * geo.n, 0, 1]
    bound = 1e-13 * (absum[:2 * geo.n, 0, 1] / np.abs(csum[:2 * geo.n, 0, 1])
                     + absum[:2 * geo.n, 1, 1] / np.abs(csum[:2 * geo.n, 1, 1]))
    ratio = rho_o / rho_w
    assert np.all(np.abs(w[free] - ratio[free]) <= bound[free] * ratio[free])
    # at perforated nodes the well terms do not cancel: the weight differs
    assert np.abs(w[perforated] - ratio[perforated]).max() > 1e-6


@pytest.mark.parametrize("variant", ["gj", "abf", "ti"])
def test_decoupled_system_has_the_same_solution(variant):
    """D is invertible: D^-1 J y = D^-1 b has the solution of J y = b."""
    geo, J, b = _system(synth.model_small())
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, bh = cpr.decouple(2 * geo.n, indptr, indices, data, b, variant)
    Ah = ph.bsr_to_csr(indptr, indices, dh)
    y0 = spla.spsolve(J.tocsc(), b)
    y1 = spla.spsolve(Ah.tocsc(), bh)
    # the same D^-1 on both sides: the original solution leaves a rounding-level
    # residual in the decoupled system; the two direct solutions differ by about
    # kappa * eps (the system is badly scaled: Pa against saturation)
    res = Ah @ y0 - bh
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(abs(Ah) @ np.abs(y0) + np.abs(bh))
    assert np.abs(y1 - y0).max() <= 1e-6 * np.abs(y0).max()


def test_cpr_fp_with_exact_full_stage_converges_in_one_iteration():
    """Two-stage CPR-FP: z1 = R^T Mp^-1 R r, z = z1 + F^-1 (r - A z1); with F
    exact the second stage alone solves the system."""
    geo, J, b = _system(synth.model_small())
    y, its, rel = cpr.solve(geo, J, b, rtol=1e-10, exact_f=True, variant="fp")
    assert its == 1 and rel <= 1e-10


@pytest.mark.parametrize("decoupling,variant", [("abf", "fpf"), ("ti", "fpf"), ("gj", "fp"), ("abf", "fp")])
def test_cpr_variants_reach_the_direct_solution(decoupling, variant):
    geo, J, b = _system(synth.model_small())
    y, its, rel = cpr.solve(geo, J, b, rtol=1e-10, decoupling=decoupling, variant=variant)
    y0 = spla.spsolve(J.tocsc(), b)
    assert rel <= 1e-10
    assert np.abs(y - y0).max() <= 1e-6 * np.abs(y0).max()


def test_l1_diag_hand_values():
    """d_i = a_ii + sgn(a_ii) sum_{j != i} |a_ij|, worked by hand on a 3x3
    matrix with a negative diagonal entry and an empty off-diagonal row part:
      row 0: 4 + (|-1| + |2|) = 7
      row 1: -5 - (|-1| + |0.5|) = -6.5
      row 2: 2 + |3| = 5
      row 3: 1 (no off-diagonal entries)."""
    A = sp.csr_matrix(np.array([[4.0, -1.0, 2.0, 0.0],
                                [-1.0, -5.0, 0.5, 0.0],
                                [0.0, 3.0, 2.0, 0.0],
                                [0.0, 0.0, 0.0, 1.0]]))
    assert np.array_equal(cpr.l1_diag(A), np.array([7.0, -6.5, 5.0, 1.0]))


def _dense_cpr_parts(m, seed, amg_opts, variant="fpf"):
    """The decoupled matrix A and the dense matrices of M^-1, F^-1 and the
    pressure stage's M_p (each by applying the oracle to the identity columns)."""
    geo, J, b = _system(m, seed=seed)
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, _ = cpr.decouple(2 * geo.n, indptr, indices, data, b)
    pc = cpr.CPRFPF(geo, indptr, indices, dh, amg_opts=amg_opts, variant=variant)
    A = pc.A.toarray()
    N = A.shape[0]
    eye = np.eye(N)
    Minv = np.column_stack([pc.apply(eye[:, k]) for k in range(N)])
    Finv = np.column_stack([pc.fsolve(eye[:, k]) for k in range(N)])
    npr = N // 2
    Mp = np.column_stack([pc.pressure_solve(np.eye(npr)[:, k]) for k in range(npr)])
    R = np.zeros((npr, N))
    R[np.arange(npr), 2 * np.arange(npr)] = 1.0  # the pressure (first) unknown of every block
    return A, Minv, Finv, Mp, R


def _judge(lhs, rhs, A, Minv):
    """Difference of two error-propagation matrices, each entry against the
    magnitudes a product of the factors can reach: (|M^-1| |A|)_ij + 1."""
    scale = np.abs(Minv) @ np.abs(A) + 1.0
    return np.max(np.abs(lhs - rhs) / scale)


@pytest.mark.parametrize("levels", ["one", "multi"])
def test_cpr_fpf_error_propagation_is_the_stage_product(levels):
    """The multiplicative F-P-F composition has the error propagation
    I - M^-1 A = (I - F^-1 A)(I - R^T M_p R A)(I - F^-1 A), with R the pressure
    pick and M_p the pressure stage (the exact A_p^-1 with a one-level
    hierarchy, where A_p = R A R^T).  A sign or ordering error in the pressure
    stage (z2 = z1 - R^T e, a residual taken at r instead of r - A z1, the
    second F stage at z1) breaks the identity by O(1)."""
    m = synth.model_tiny(3, 2, 2, seed=7)
    opts = dict(max_coarse=10 ** 6) if levels == "one" else dict(max_coarse=4)
    A, Minv, Finv, Mp, R = _dense_cpr_parts(m, 9, opts)
    N = A.shape[0]
    I = np.eye(N)
    if levels == "one":
        Ap = R @ A @ R.T
        assert np.allclose(Mp @ Ap, np.eye(Ap.shape[0]), atol=1e-8)
        Mp = np.linalg.inv(Ap)
    EF = I - Finv @ A
    EP = I - R.T @ Mp @ R @ A
    err = _judge(I - Minv @ A, EF @ EP @ EF, A, Minv)
    assert err <= 1e-9
    # the identity is not vacuous: the stages do not commute and none is exact
    assert _judge(I - Minv @ A, EP @ EF @ EF, A, Minv) > 1e-3
    assert _judge(I - Minv @ A, EF @ EF, A, Minv) > 1e-3


def test_cpr_fp_error_propagation_is_the_stage_product():
    """Two-stage CPR-FP, pressure first: I - M^-1 A = (I - F^-1 A)(I - R^T A_p^-1 R A)
    with a one-level hierarchy; the reversed order does not hold."""
    m = synth.model_tiny(3, 2, 2, seed=7)
    A, Minv, Finv, Mp, R = _dense_cpr_parts(m, 9, dict(max_coarse=10 ** 6), variant="fp")
    I = np.eye(A.shape[0])
    Mp = np.linalg.inv(R @ A @ R.T)
    EF = I - Finv @ A
    EP = I - R.T @ Mp @ R @ A
    assert _judge(I - Minv @ A, EF @ EP, A, Minv) <= 1e-9
    assert _judge(I - Minv @ A, EP @ EF, A, Minv) > 1e-3


def test_gmres_cgs2_matches_a_dense_arnoldi():
    """One cycle of the oracle's GMRES against the plain definition: the
    Krylov basis of A M^-1 from b orthonormalised by a dense QR (Householder,
    numpy), whose R factor is the Hessenberg matrix up to column signs, and
    the iterate x = M^-1 V y with y the dense least-squares minimiser of
    |beta e_1 - H y|."""
    rng = np.random.default_rng(21)
    n = 50
    A = (sp.diags(np.linspace(1.0, 3.0, n)) + 0.2 * sp.random(n, n, density=0.15, random_state=8)).tocsr()
    d = 1.0 / A.diagonal()
    b = rng.standard_normal(n)
    k = 5
    tr = {}
    x, its, rel = cpr.gmres(lambda v: A @ v, lambda v: d * v, b, 1e-15, restart=30, maxit=k, trace=tr)
    assert its == k
    V, H = tr["V"], tr["H"]
    # the dense Arnoldi: K = [b, (A M^-1) b, ...], QR with positive R diagonal
    K = np.zeros((n, k + 1))
    v = b.copy()
    for i in range(k + 1):
        K[:, i] = v
        v = A @ (d * v)
    Q, Rq = np.linalg.qr(K)
    sgn = np.sign(np.diag(Rq))
    Q = Q * sgn
    # the monomial Krylov matrix is ill-conditioned: its QR factor is accurate
    # to about cond(K) eps
    tol = 1e-14 * np.linalg.cond(K)
    assert tol < 1e-6
    assert np.abs(V - Q.T).max() <= tol
    AMV = np.column_stack([A @ (d * V[j]) for j in range(k)])
    Href = Q.T @ AMV
    assert np.abs(H - Href).max() <= tol * np.abs(Href).max()
    beta = np.linalg.norm(b)
    e1 = np.zeros(k + 1)
    e1[0] = beta
    y, *_ = np.linalg.lstsq(Href, e1, rcond=None)
    xref = d * (Q[:, :k] @ y)
    assert np.linalg.norm(x - xref) <= tol * np.linalg.norm(xref)
