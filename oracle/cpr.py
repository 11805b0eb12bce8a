"""Oracle linear solver: decoupled, CPR-FPF-preconditioned GMRES (Sec. 3.2).

Part of the CPU oracle (test infrastructure only; see the package docstring).

Readings of what the paper leaves open:

* Decoupling (Eq. (14)), "modified Gauss-Jordan": in every node block row the
  oil row is replaced by oil - (a01/a11) water, where a = J_ii is the diagonal
  block (one Gauss-Jordan step that removes the node's own saturation from the
  first equation); well rows are left as they are.
* CPR-FPF: full-system stage, pressure stage, full-system stage, applied
  multiplicatively: z1 = F^-1 r; z2 = z1 + R^T M_p^-1 R (r - A z1);
  z = z2 + F^-1 (r - A z2), with F = block ILU(0), R picking the first
  component (pressure, or p_b for wells) of every block, and M_p one V(1,1)
  cycle of classical AMG on A_p = R A R^T.
* Block ILU(0) takes the elimination ordering as an argument.  The ordering
  used throughout is: all matrix nodes, then fracture nodes with i+j+k even,
  then those with i+j+k odd, then wells.
* Pressure stage: the pressure system is taken in the elimination order.  A
  matrix-node pressure couples only to the pressure of its own fracture node,
  so it is eliminated exactly first (a diagonal Schur complement on the
  fracture and well pressures; the matrix pressures are recovered afterwards).
  This is the ideal first coarsening of the pressure system (C = fracture and
  well unknowns, F = matrix nodes).
* Classical AMG on the reduced system: strength theta = 0.25 on
  -a_ij sign(a_ii); PMIS coarsening with weights |S^T_i| + h(i)/2^32,
  h = lowbias32; distance-two ("extended") interpolation written as
  W = -D^-1 (A^s_FC + A^s_FF B^-1 Abar^s_FC), truncated to 3 entries per row
  (row sum kept); Galerkin coarse operators R A P with R = P^T; l1-Jacobi
  smoothing; coarsest level solved exactly.
* GMRES: right-preconditioned, restart 30, classical Gram-Schmidt applied
  twice (CGS2), Givens rotations; the tolerance is on the decoupled residual.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import physics as ph


# --------------------------------------------------------------------------
# Decoupling
# --------------------------------------------------------------------------

DECOUPLINGS = ("gj", "abf", "ti")


def decoupling_operator(n_nodes, indptr, indices, data, variant="gj"):
    """The 2x2 matrix Q_i = D_i^-1 of every block row (Sec. 3.2, Eq. (14)); the
    identity on well rows.

      'gj'  one Gauss-Jordan step with a = J_ii: Q = [[1, -a01/a11], [0, 1]]
            (the reading of the paper's modified Gauss-Jordan decoupling; for
            2x2 blocks it is also the Quasi-IMPES operator, whose weights come
            from the diagonal block);
      'abf' alternate block factorisation: Q = J_ii^-1, so that every diagonal
            block becomes the identity;
      'ti'  true-IMPES: Q = [[1, -c01/c11], [0, 1]] with c_i the sum of block
            column i, sum_k J_ki.  Conservative fluxes cancel in a column sum,
            so c_i holds the accumulation (and well) derivatives of node i.
    """
    nb = indptr.shape[0] - 1
    rows = np.repeat(np.arange(nb), np.diff(indptr))
    diag_pos = np.empty(nb, dtype=np.int64)
    diag_pos[rows[indices == rows]] = np.nonzero(indices == rows)[0]
    a = data[diag_pos]
    Q = np.zeros((nb, 2, 2))
    Q[:, 0, 0] = Q[:, 1, 1] = 1.0
    nd = slice(0, n_nodes)
    if variant == "gj":
        Q[nd, 0, 1] = -a[nd, 0, 1] / a[nd, 1, 1]
    elif variant == "abf":
        Q[nd] = np.linalg.inv(a[nd])
    elif variant == "ti":
        c = np.zeros((nb, 2, 2))
        np.add.at(c, indices, data)
        Q[nd, 0, 1] = -c[nd, 0, 1] / c[nd, 1, 1]
    else:
        raise ValueError("unknown decoupling %r" % (variant,))
    return Q


def decouple(n_nodes, indptr, indices, data, b, variant="gj"):
    """Apply D^-1 to the block matrix (indptr, indices, data) and to b (Eq. (14)):
    every block row i is multiplied by Q_i of decoupling_operator."""
    nb = indptr.shape[0] - 1
    rows = np.repeat(np.arange(nb), np.diff(indptr))
    Q = decoupling_operator(n_nodes, indptr, indices, data, variant)
    out = np.einsum("rij,rjk->rik", Q[rows], data)
    bh = np.einsum("rij,rj->ri", Q, b.reshape(nb, 2)).reshape(-1)
    return out, bh


# --------------------------------------------------------------------------
# Ordering and block ILU(0)
# --------------------------------------------------------------------------

def default_ordering(geo):
    """Matrix nodes, then fracture nodes of even colour, odd colour, then wells."""
    i, j, k = ph.cell_ijk(geo.m)
    c = np.arange(geo.n)
    red = c[(i + j + k) % 2 == 0]
    black = c[(i + j + k) % 2 == 1]
    return np.concatenate([2 * c + 1, 2 * red, 2 * black, 2 * geo.n + np.arange(geo.nw)])


def _inv2(a):
    det = a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0]
    return np.array([[a[1, 1], -a[0, 1]], [-a[1, 0], a[0, 0]]]) / det


class BlockILU0:
    """Block ILU(0) of a 2x2-block matrix in a given elimination ordering.

    Factors L (unit block lower) and U (block upper) on the pattern of A in the
    permuted numbering, so that (L U)_ij = A_ij for every (i, j) of the pattern.
    """

    def __init__(self, indptr, indices, data, perm):
        nb = indptr.shape[0] - 1
        self.nb = nb
        self.perm = np.asarray(perm)
        pos = np.empty(nb, dtype=np.int64)
        pos[self.perm] = np.arange(nb)
        self.pos = pos
        rows = []
        for ii in range(nb):
            r = self.perm[ii]
            cols = pos[indices[indptr[r]:indptr[r + 1]]]
            vals = data[indptr[r]:indptr[r + 1]]
            order = np.argsort(cols)
            rows.append((list(cols[order]), [vals[t].copy() for t in order]))
        uinv = [None] * nb
        for i in range(nb):
            cols, vals = rows[i]
            where = {c: t for t, c in enumerate(cols)}
            for t, kk in enumerate(cols):
                if kk >= i:
                    break
                lik = vals[t] @ uinv[kk]
                vals[t] = lik
                kcols, kvals = rows[kk]
                for s, jj in enumerate(kcols):
                    if jj > kk and jj in where:
                        u = where[jj]
                        vals[u] = vals[u] - lik @ kvals[s]
            uinv[i] = _inv2(vals[where[i]])
        self.rows = rows
        self.uinv = uinv
        # point-wise triangular matrices in the permuted numbering:
        # L (unit lower) and Ut = I + D^-1 U_strict (unit upper), plus D^-1
        lr, lc, lv, ur, uc, uv = [], [], [], [], [], []
        for i in range(nb):
            cols, vals = rows[i]
            for c, v in zip(cols, vals):
                if c < i:
                    blk = v
                    rr, cc, vv = lr, lc, lv
                elif c > i:
                    blk = uinv[i] @ v
                    rr, cc, vv = ur, uc, uv
                else:
                    continue
                for a in range(2):
                    for b in range(2):
                        rr.append(2 * i + a)
                        cc.append(2 * c + b)
                        vv.append(blk[a, b])
        n2 = 2 * nb
        eye = sp.identity(n2, format="csr")
        self.L = (sp.csr_matrix((lv, (lr, lc)), shape=(n2, n2)) + eye).tocsr()
        self.Ut = (sp.csr_matrix((uv, (ur, uc)), shape=(n2, n2)) + eye).tocsr()
        self.Dinv = sp.block_diag(uinv, format="csr")
        self.pidx = np.empty(n2, dtype=np.int64)
        self.pidx[0::2] = 2 * self.perm
        self.pidx[1::2] = 2 * self.perm + 1

    def factors(self):
        """(position, column position, L or U block) lists in permuted numbering."""
        out = []
        for i in range(self.nb):
            cols, vals = self.rows[i]
            for c, v in zip(cols, vals):
                out.append((i, c, v))
        return out

    def solve(self, r):
        rp = r[self.pidx]
        y = spla.spsolve_triangular(self.L, rp, lower=True, unit_diagonal=True)
        z = spla.spsolve_triangular(self.Ut, self.Dinv @ y, lower=False, unit_diagonal=True)
        out = np.empty_like(r)
        out[self.pidx] = z
        return out


# --------------------------------------------------------------------------
# Pressure system
# --------------------------------------------------------------------------

def pressure_matrix(indptr, indices, data):
    """A_p: entry (0,0) of every block, on the same (structural) pattern."""
    nb = indptr.shape[0] - 1
    return sp.csr_matrix((data[:, 0, 0].copy(), indices.copy(), indptr.copy()), shape=(nb, nb))


# --------------------------------------------------------------------------
# Classical AMG
# --------------------------------------------------------------------------

def lowbias32(x):
    """32-bit integer mixing hash 'lowbias32' (C. Wellons): xor-shift 16,
    multiply 0x7feb352d, xor-shift 15, multiply 0x846ca68b, xor-shift 16."""
    x = np.asarray(x, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    m32 = np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x7FEB352D)) & m32
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x846CA68B)) & m32
    x ^= x >> np.uint64(16)
    return x


def _csr_parts(A):
    A = A.tocsr()
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    return A, n, rows, A.indices.astype(np.int64), A.data


def strength(A, theta):
    """Boolean mask over the entries of A: j strongly influences i if
    -a_ij sgn(a_ii) >= theta * max_{k != i} (-a_ik sgn(a_ii)) and that max is > 0."""
    A, n, rows, cols, v = _csr_parts(A)
    diag = A.diagonal()
    sgn = np.where(diag < 0.0, -1.0, 1.0)
    off = cols != rows
    neg = -v * sgn[rows]
    mx = np.full(n, -np.inf)
    np.maximum.at(mx, rows[off], neg[off])
    return off & (mx[rows] > 0.0) & (neg >= theta * mx[rows])


def pmis(A, smask):
    """PMIS C/F splitting.  Returns state per point: 1 = C, -1 = F."""
    A, n, rows, cols, _ = _csr_parts(A)
    srow, scol = rows[smask], cols[smask]  # scol strongly influences srow
    nst = np.bincount(scol, minlength=n)     # |S^T_i|
    w = nst.astype(np.float64) + lowbias32(np.arange(n)).astype(np.float64) / 2.0 ** 32
    state = np.zeros(n, dtype=np.int64)
    state[nst == 0] = -1
    # symmetric neighbourhood
    ga = np.concatenate([srow, scol])
    gb = np.concatenate([scol, srow])
    while np.any(state == 0):
        und = state == 0
        both = und[ga] & und[gb]
        beaten = np.zeros(n, dtype=bool)
        # ga loses if a neighbour has a larger (weight, index)
        lose = both & ((w[gb] > w[ga]) | ((w[gb] == w[ga]) & (gb > ga)))
        beaten[ga[lose]] = True
        newc = und & ~beaten
        state[newc] = 1
        # undecided points that strongly depend on a new C point become F
        dep = newc[scol] & (state[srow] == 0)
        state[srow[dep]] = -1
    return state


def interpolation(A, smask, state, trunc=3):
    """Extended (distance-two) interpolation in matrix-product form, truncated.

    For an F point i with strong C set C_i, strong F set F_i and weak set W_i:
      abar_kj = a_kj if j in C_k and a_kj a_kk < 0 (else 0), beta_k = sum_j abar_kj
      d_i  = a_ii + sum_{n in W_i} a_in + sum_{k in F_i, beta_k = 0} a_ik
      w_ij = -(1/d_i) [ a_ij [j in C_i] + sum_{k in F_i, beta_k != 0} a_ik abar_kj / beta_k ]
    then the ``trunc`` largest |w_ij| are kept (3 by default, as in the AMG
    hierarchy; ties: lower coarse index) and scaled so the row sum is
    unchanged.  C points interpolate by injection.
    """
    A, n, rows, cols, v = _csr_parts(A)
    isC = state == 1
    nc = int(isC.sum())
    cidx = np.full(n, -1, dtype=np.int64)
    cidx[isC] = np.arange(nc)
    diag = A.diagonal()
    off = cols != rows
    fr = ~isC[rows]
    sC = smask & isC[cols] & fr
    sF = smask & ~isC[cols] & fr
    weak = off & ~smask & fr
    abar = np.where(sC & (v * diag[rows] < 0.0), v, 0.0)
    beta = np.zeros(n)
    np.add.at(beta, rows, abar)
    dist = sF & (beta[cols] != 0.0)
    lump = sF & (beta[cols] == 0.0)
    d = diag.copy()
    np.add.at(d, rows[weak], v[weak])
    np.add.at(d, rows[lump], v[lump])
    gsel = sC & (beta[rows] != 0.0)
    G = sp.csr_matrix((abar[gsel] / beta[rows[gsel]], (rows[gsel], cidx[cols[gsel]])), shape=(n, nc))
    Asfc = sp.csr_matrix((v[sC], (rows[sC], cidx[cols[sC]])), shape=(n, nc))
    Asff = sp.csr_matrix((v[dist], (rows[dist], cols[dist])), shape=(n, n))
    Wn = (Asfc + Asff @ G).tocsr()
    Wn.sort_indices()
    pr, pc, pv = [], [], []
    for i in range(n):
        if isC[i]:
            pr.append(i)
            pc.append(cidx[i])
            pv.append(1.0)
            continue
        if d[i] == 0.0:
            continue
        a, b = Wn.indptr[i], Wn.indptr[i + 1]
        wc = Wn.indices[a:b]
        wv = -Wn.data[a:b] / d[i]
        keep = wv != 0.0
        wc, wv = wc[keep], wv[keep]
        if wc.shape[0] > trunc:
            order = np.lexsort((wc, -np.abs(wv)))[:trunc]
            total = wv.sum()
            kept = wv[order].sum()
            scale = total / kept if kept != 0.0 else 1.0
            order = np.sort(order)
            wc, wv = wc[order], wv[order] * scale
        pr.extend([i] * wc.shape[0])
        pc.extend(wc.tolist())
        pv.extend(wv.tolist())
    P = sp.csr_matrix((pv, (pr, pc)), shape=(n, nc))
    return P


def l1_diag(A):
    """d_i = a_ii + sgn(a_ii) sum_{j != i} |a_ij|  (l1-Jacobi)."""
    A, n, rows, cols, v = _csr_parts(A)
    diag = A.diagonal()
    sgn = np.where(diag < 0.0, -1.0, 1.0)
    off = np.abs(np.where(cols != rows, v, 0.0))
    s = np.zeros(n)
    np.add.at(s, rows, off)
    return diag + sgn * s


def reduced_pressure_matrix(App, n):
    """Exact elimination of the first n unknowns of App (matrix-node pressures,
    each coupled only to its own fracture pressure): the Schur complement
    App[n:, n:] - App[n:, :n] D^-1 App[:n, n:] with D = diag(App[:n, :n]).  Only
    the diagonal of App[n:, n:] changes, so its stored pattern is kept."""
    App = App.tocsr()
    D = App[:n, :n].diagonal()
    S = App[n:, n:].tocsr().copy()
    S.sort_indices()
    upd = (App[n:, :n] @ sp.diags(1.0 / D) @ App[:n, n:]).tocsr()
    if upd.nnz:
        rows = np.repeat(np.arange(upd.shape[0]), np.diff(upd.indptr))
        if not np.all(upd.indices == rows):
            raise ValueError("matrix nodes must couple to one fracture node only")
        dpos = np.empty(S.shape[0], dtype=np.int64)
        srows = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
        dmask = S.indices == srows
        dpos[srows[dmask]] = np.nonzero(dmask)[0]
        S.data[dpos[rows]] -= upd.data
    return S, D


class AMG:
    """Classical AMG hierarchy on a pressure matrix."""

    def __init__(self, A, theta=0.25, max_coarse=2000, max_levels=25, trunc=3):
        self.levels = []
        A = A.tocsr()
        while True:
            lvl = {"A": A, "dl1": l1_diag(A)}
            self.levels.append(lvl)
            n = A.shape[0]
            if n <= max_coarse or len(self.levels) >= max_levels:
                break
            sm = strength(A, theta)
            state = pmis(A, sm)
            nc = int((state == 1).sum())
            if nc == 0 or nc >= n:
                break
            P = interpolation(A, sm, state, trunc)
            R = P.T.tocsr()
            lvl.update(P=P, R=R, state=state, S=sm)
            A = (R @ A @ P).tocsr()
            A.sort_indices()
        self.coarse_dense = self.levels[-1]["A"].toarray()

    def vcycle(self, b, lev=0):
        lvl = self.levels[lev]
        if lev == len(self.levels) - 1:
            return np.linalg.solve(self.coarse_dense, b)
        A = lvl["A"]
        x = b / lvl["dl1"]
        r = b - A @ x
        e = self.vcycle(lvl["R"] @ r, lev + 1)
        x = x + lvl["P"] @ e
        x = x + (b - A @ x) / lvl["dl1"]
        return x


# --------------------------------------------------------------------------
# CPR-FPF and GMRES
# --------------------------------------------------------------------------

class CPRFPF:
    """CPR-FPF preconditioner for the decoupled block matrix."""

    def __init__(self, geo, indptr, indices, data, perm=None, amg_opts=None, exact_f=False, variant="fpf"):
        nb = indptr.shape[0] - 1
        if variant not in ("fpf", "fp"):
            raise ValueError("unknown CPR variant %r" % (variant,))
        self.variant = variant
        self.A = ph.bsr_to_csr(indptr, indices, data)
        self.perm = default_ordering(geo) if perm is None else perm
        if exact_f:
            lu = spla.splu(self.A.tocsc())
            self.fsolve = lu.solve
            self.ilu = None
        else:
            self.ilu = BlockILU0(indptr, indices, data, self.perm)
            self.fsolve = self.ilu.solve
        self.Ap = pressure_matrix(indptr, indices, data)
        self.n = geo.n
        self.App = self.Ap[self.perm][:, self.perm].tocsr()
        self.S, self.D = reduced_pressure_matrix(self.App, self.n)
        self.amg = AMG(self.S, **(amg_opts or {}))
        self.nb = nb

    def pressure_solve(self, rp):
        """Approximate A_p^-1 rp: exact matrix-node elimination, one V-cycle on
        the reduced system, back-substitution.  rp in canonical block order."""
        n = self.n
        q = rp[self.perm]
        rm, rf = q[:n], q[n:]
        rr = rf - self.App[n:, :n] @ (rm / self.D)
        ef = self.amg.vcycle(rr)
        em = (rm - self.App[:n, n:] @ ef) / self.D
        e = np.empty_like(rp)
        e[self.perm] = np.concatenate([em, ef])
        return e

    def apply(self, r):
        """'fpf': z1 = F^-1 r; z2 = z1 + R^T Mp^-1 R (r - A z1); z = z2 + F^-1 (r - A z2).
        'fp' (two-stage, pressure first): z1 = R^T Mp^-1 R r; z = z1 + F^-1 (r - A z1)."""
        if self.variant == "fpf":
            z = self.fsolve(r)
            res = r - self.A @ z
        else:
            z = np.zeros_like(r)
            res = r
        e = self.pressure_solve(res[0::2])
        z = z.copy()
        z[0::2] += e
        res = r - self.A @ z
        return z + self.fsolve(res)


def gmres(matvec, precond, b, rtol, restart=30, maxit=300, x0=None, trace=None):
    """Right-preconditioned restarted GMRES (Sec. 3.2; Saad and Schultz's
    GMRES(m)) with classical Gram-Schmidt applied twice (CGS2) and Givens
    rotations.  Returns (x, iterations, relative true residual).

    Iteration j, textbook order:
      z_j = M^-1 v_j;  w = A z_j;
      h1 = V^T w,  w <- w - V h1   (first classical Gram-Schmidt pass);
      h2 = V^T w,  w <- w - V h2   (second pass, the re-orthogonalisation);
      H[:j+1, j] = h1 + h2,  H[j+1, j] = |w|,  v_{j+1} = w / |w|;
    then the rotations of the earlier columns are applied to column j, a new
    rotation zeroes H[j+1, j], and |g_{j+1}| is the residual norm of the
    least-squares iterate.  At the end of a cycle y solves the triangular
    system R y = g and x <- x + Z y (right preconditioning: the iterate is
    x0 + M^-1 V y).  The loop stops when |g_{j+1}| <= rtol |b| (x0 = 0) or
    after maxit iterations; each restart starts from the true residual.

    If ``trace`` is a dict, the first cycle's V, Z and (unrotated) Hessenberg
    matrix are stored in it."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    its = 0
    while beta > rtol * bnorm and its < maxit:
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        Hraw = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            h1 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h1
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            hn = np.linalg.norm(w)
            col = np.zeros(restart + 1)
            col[:j + 1] = h1 + h2
            col[j + 1] = hn
            Hraw[:, j] = col
            if hn > 0.0:
                V[j + 1] = w / hn
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            den = np.hypot(col[j], col[j + 1])
            cs[j] = col[j] / den
            sn[j] = col[j + 1] / den
            col[j] = den
            col[j + 1] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            H[:, j] = col
            its += 1
            k = j + 1
            if hn == 0.0 or abs(g[j + 1]) <= rtol * bnorm or its >= maxit:
                break
        if trace is not None and "V" not in trace:
            trace.update(V=V[:k + 1].copy(), Z=Z[:k].copy(), H=Hraw[:k + 1, :k].copy())
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    return x, its, beta / bnorm


def solve(geo, J, rhs, rtol=1e-6, restart=30, maxit=300, amg_opts=None, exact_f=False, decoupling="gj",
          variant="fpf"):
    """Solve J y = rhs: decouple, build CPR-FPF (or CPR-FP), run GMRES on the
    decoupled system.  Returns (y, iterations, relative decoupled residual)."""
    indptr, indices, data = ph.to_bsr(geo, J)
    dh, bh = decouple(2 * geo.n, indptr, indices, data, rhs, decoupling)
    pc = CPRFPF(geo, indptr, indices, dh, amg_opts=amg_opts, exact_f=exact_f, variant=variant)
    y, its, rel = gmres(lambda v: pc.A @ v, pc.apply, bh, rtol, restart, maxit)
    return y, its, rel
