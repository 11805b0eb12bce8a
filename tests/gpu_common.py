"""Shared helpers of the GPU parity tests: oracle reference systems and
comparisons (the oracle is test infrastructure; the GPU side runs only through
the library's C ABI)."""
import numpy as np

import synth
from oracle import cpr as ocpr
from oracle import physics as oph


def require_gpu():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible MI355X")


def controls(m):
    return [w["control"] for w in m["wells"]]


def oracle_system(m, x, x_old, dt):
    geo = oph.Geometry(m)
    acc = oph.accumulation(geo, x_old)
    ctrl = controls(m)
    return geo, oph.residual(geo, x, acc, dt, ctrl), oph.jacobian(geo, x, dt, ctrl)


def oracle_cpr(geo, J, R, amg_opts=None):
    indptr, indices, data = oph.to_bsr(geo, J)
    dh, bh = ocpr.decouple(2 * geo.n, indptr, indices, data, -R)
    pc = ocpr.CPRFPF(geo, indptr, indices, dh, amg_opts=amg_opts)
    return pc, bh, (indptr, indices, dh)


def sim_at(m, x, x_old, dt, **opts):
    """A handle whose old state is x_old and current state x, assembled and set up."""
    from paper_1808_04338_amd import Sim

    sim = Sim(m, **opts)
    n = m["nx"] * m["ny"] * m["nz"]
    po, so, bo = oph.unpack_state(x_old, n)
    sim.set_state(po, so, bo)
    sim.mark_old()
    p, s, b = oph.unpack_state(x, n)
    sim.set_state(p, s, b)
    sim.assemble(dt)
    return sim


def rel_max(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def sparse_rel(A, B):
    return abs(A - B).max() / max(abs(B).max(), 1e-300)


def row_scaled_err(A, B):
    """max over rows of max|A - B| / max|B| in that row (entries that cancel to
    ~0 on one side are judged against their row's scale)."""
    D = abs(A - B).tocsr()
    Bc = abs(B).tocsr()
    err = 0.0
    for i in range(B.shape[0]):
        s = Bc.data[Bc.indptr[i]:Bc.indptr[i + 1]].max(initial=0.0)
        d = D.data[D.indptr[i]:D.indptr[i + 1]].max(initial=0.0)
        if s > 0:
            err = max(err, d / s)
    return err


def random_state_pair(m, seed):
    x = oph.pack_state(*synth.random_state(m, seed))
    x_old = oph.pack_state(*synth.random_state(m, seed + 1000))
    return x, x_old


def decoupled_err(Ag, J, Ahat):
    """Error of the GPU decoupled matrix against the oracle's, each entry of a
    node's first row judged against the magnitudes the Gauss-Jordan step
    combined, |J_0j| + |f| |J_1j| with f = a01/a11 of the diagonal block; second
    rows and well rows against |J_ij|."""
    J = J.tocsr()
    nd = J.shape[0]
    diag = J.diagonal()
    a01 = np.array([J[2 * i, 2 * i + 1] for i in range(nd // 2)])
    a11 = diag[1::2]
    f = np.where(a11 != 0, np.abs(a01 / np.where(a11 != 0, a11, 1.0)), 0.0)
    D = (Ag - Ahat).tocsr()
    Ja = abs(J).tocsr()
    worst = 0.0
    for r in range(nd):
        cols = D.indices[D.indptr[r]:D.indptr[r + 1]]
        if cols.size == 0:
            continue
        d = np.abs(D.data[D.indptr[r]:D.indptr[r + 1]])
        scale = np.asarray(Ja[r, cols].todense()).ravel()
        if r % 2 == 0:
            scale = scale + f[r // 2] * np.asarray(Ja[r + 1, cols].todense()).ravel()
        worst = max(worst, float(np.max(d / np.maximum(scale, 1e-300))))
    return worst
