"""Pins of the oracle's physics against closed forms, invariants and
derivatives (no GPU)."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import newton as nt
from oracle import physics as ph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ctrl(m):
    return [w["control"] for w in m["wells"]]


def test_paper_constants_golden():
    lbm_ft3 = 0.45359237 / 0.3048 ** 3
    conv = {"lbm/ft3": lbm_ft3, "ft": 0.3048}
    bp = synth.base_physics()
    used = {"water_density": bp["rho_w_ref"], "oil_density": bp["rho_o_ref"],
            "well_radius": synth.model_small()["wells"][0]["rw"], "top_depth": bp["top_depth"]}
    for line in open(os.path.join(GOLDEN, "paper_constants.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, val, unit, si, _, _ = line.split()
        assert abs(float(val) * conv[unit] - float(si)) <= 1e-4 * float(si)
        assert used[name] == pytest.approx(float(si), rel=1e-12)


def test_corey_endpoints_and_midpoint():
    m = synth.base_physics()
    sw = np.array([m["swc"], 1.0 - m["sor"], 0.5 * (1 + m["swc"] - m["sor"]), 0.0, 1.0])
    krw, kro, dkrw, dkro = ph.corey(sw, m)
    assert krw[0] == 0.0 and kro[0] == 1.0
    assert kro[1] == 0.0 and krw[1] == 1.0
    assert krw[2] == pytest.approx(0.25) and kro[2] == pytest.approx(0.25)
    # outside the mobile range: clipped values, zero slope
    assert krw[3] == 0.0 and kro[4] == 0.0 and dkrw[3] == 0.0 and dkro[4] == 0.0
    # slope at the midpoint: n s*^(n-1) / (1 - swc - sor)
    assert dkrw[2] == pytest.approx(2 * 0.5 / 0.6)
    assert dkro[2] == pytest.approx(-2 * 0.5 / 0.6)


def test_density_law():
    m = synth.base_physics()
    rho, drho = ph.density(np.array([m["p_ref"], m["p_ref"] + 1e7]), 1000.0, 1e-9, m["p_ref"])
    assert rho[0] == 1000.0
    assert rho[1] == pytest.approx(1000.0 * np.exp(1e-2), rel=1e-15)
    assert drho[1] == pytest.approx(1e-9 * rho[1], rel=1e-15)


def test_transmissibility_closed_forms():
    m = synth.model_tiny(2, 1, 1, wells=False)
    k = 50 * synth.MD
    m["kx"][:] = k
    geo = ph.Geometry(m)
    assert geo.ft.shape == (1,)
    # equal permeabilities: T = k A / L
    assert geo.ft[0] == pytest.approx(k * m["dy"] * m["dz"] / m["dx"], rel=1e-15)
    # unequal: two half-cell resistances in series
    m["kx"][:] = [10 * synth.MD, 1000 * synth.MD]
    geo = ph.Geometry(m)
    a = m["dy"] * m["dz"]
    res = 0.5 * m["dx"] / (m["kx"][0] * a) + 0.5 * m["dx"] / (m["kx"][1] * a)
    assert geo.ft[0] == pytest.approx(1.0 / res, rel=1e-14)


def test_face_counts():
    m = synth.model_small()
    geo = ph.Geometry(m)
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    assert geo.fc.shape[0] == (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    assert np.all(geo.fc < geo.fd)


def test_peaceman_golden():
    for line in open(os.path.join(GOLDEN, "peaceman.txt")):
        if line.startswith("#") or not line.strip():
            continue
        dx, dy, re = map(float, line.split())
        k = 100 * synth.MD
        assert ph.peaceman_re(dx, dy, k, k) == pytest.approx(re, rel=2e-6)


def test_peaceman_symmetry_and_well_index():
    kx, ky = 300 * synth.MD, 30 * synth.MD
    assert ph.peaceman_re(20.0, 10.0, kx, ky) == pytest.approx(ph.peaceman_re(10.0, 20.0, ky, kx), rel=1e-15)
    m = synth.model_small()
    perfs = ph.well_perforations(m)
    cells, wi = perfs[0]
    c = cells[0]
    k = m["kx"][c]
    re = 0.28 * np.sqrt(2 * 20.0 ** 2) / 2
    assert wi[0] == pytest.approx(2 * np.pi * k * m["dz"] / np.log(re / 0.0762), rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_residual_mass_identity(seed):
    """sum over nodes of R_a = (M_a - M_a^n)/dt - Q_a,wells at any state: the
    fluxes and the transfer cancel pairwise."""
    m = synth.model_tiny(4, 3, 2, seed=seed)
    geo = ph.Geometry(m)
    ctrl = _ctrl(m)
    x = ph.pack_state(*synth.random_state(m, 10 + seed))
    xo = ph.pack_state(*synth.random_state(m, 20 + seed))
    acc_old = ph.accumulation(geo, xo)
    dt = 3.7 * synth.DAY
    R = ph.residual(geo, x, acc_old, dt, ctrl)
    acc = ph.accumulation(geo, x)
    qo = sum(float(np.sum(q[1])) for q in ph.well_rates(geo, x, ctrl))
    qw = sum(float(np.sum(q[2])) for q in ph.well_rates(geo, x, ctrl))
    n = geo.n
    lhs_o = R[0:4 * n:2].sum()
    lhs_w = R[1:4 * n:2].sum()
    rhs_o = (acc[0].sum() - acc_old[0].sum()) / dt - qo
    rhs_w = (acc[1].sum() - acc_old[1].sum()) / dt - qw
    scale = np.abs(R[:4 * n]).sum() + np.abs(acc[0]).sum() / dt
    assert abs(lhs_o - rhs_o) <= 1e-13 * scale
    assert abs(lhs_w - rhs_w) <= 1e-13 * scale


@pytest.mark.parametrize("dims,seed", [((3, 2, 2), 1), ((2, 2, 3), 2), ((4, 1, 2), 3)])
def test_jacobian_complex_step(dims, seed):
    m = synth.model_tiny(*dims, seed=seed)
    geo = ph.Geometry(m)
    ctrl = _ctrl(m)
    x = ph.pack_state(*synth.random_state(m, seed))
    acc_old = ph.accumulation(geo, ph.pack_state(*synth.random_state(m, seed + 100)))
    dt = 2.0 * synth.DAY
    J = ph.jacobian(geo, x, dt, ctrl).toarray()
    h = 1e-30
    Jc = np.empty_like(J)
    for j in range(geo.N):
        xc = x.astype(complex)
        xc[j] += 1j * h
        Jc[:, j] = ph.residual(geo, xc, acc_old, dt, ctrl).imag / h
    scale = np.abs(Jc).max(axis=1, keepdims=True)
    scale[scale == 0] = 1.0
    # compare column-scaled (pressure and saturation columns differ by ~1e7)
    cs = np.abs(Jc).max(axis=0, keepdims=True)
    cs[cs == 0] = 1.0
    assert np.max(np.abs(J - Jc) / cs) <= 1e-10


def test_jacobian_central_differences():
    m = synth.model_tiny(3, 3, 1, seed=7)
    geo = ph.Geometry(m)
    ctrl = _ctrl(m)
    x = ph.pack_state(*synth.random_state(m, 7))
    acc_old = ph.accumulation(geo, x * 0.999)
    dt = synth.DAY
    J = ph.jacobian(geo, x, dt, ctrl).toarray()
    Jf = np.empty_like(J)
    for j in range(geo.N):
        h = 1e-6 * max(abs(x[j]), 1e-3) if x[j] > 1.0 else 1e-7
        e = np.zeros(geo.N)
        e[j] = h
        Jf[:, j] = (ph.residual(geo, x + e, acc_old, dt, ctrl)
                    - ph.residual(geo, x - e, acc_old, dt, ctrl)) / (2 * h)
    cs = np.abs(J).max(axis=0, keepdims=True)
    cs[cs == 0] = 1.0
    assert np.max(np.abs(J - Jf) / cs) <= 1e-6


def test_jacobian_in_block_pattern():
    m = synth.model_small()
    geo = ph.Geometry(m)
    x = ph.pack_state(*synth.random_state(m, 3))
    J = ph.jacobian(geo, x, synth.DAY, _ctrl(m))
    indptr, indices, data = ph.to_bsr(geo, J)
    assert abs(ph.bsr_to_csr(indptr, indices, data) - J).max() == 0.0
    n, nw = geo.n, geo.nw
    nf = geo.fc.shape[0]
    nperf = sum(len(c) for c, _ in geo.perfs)
    assert indices.shape[0] == (2 * n + nw) + 2 * nf + 2 * n + 2 * nperf


@pytest.mark.parametrize("hetero", [False, True])
def test_1d_closed_form(hetero):
    """Incompressible water-only flow between a rate injector and a BHP
    producer: linear (series-resistor) pressure profile after one step."""
    nx = 8
    k = None
    if hetero:
        k = np.exp(np.random.default_rng(5).normal(np.log(100.0), 1.0, nx)) * synth.MD
    m = synth.model_1d(nx=nx, k=k)
    geo, states, reps = nt.run(m, tol=1e-12)
    x = states[-1]
    p, sw, bhp = ph.unpack_state(x, geo.n)
    q = m["wells"][0]["target"]
    mu = m["mu_w"]
    pf = p[0::2]
    for i in range(nx - 1):
        assert pf[i] - pf[i + 1] == pytest.approx(q * mu / geo.ft[i], rel=1e-10)
    wi_prod = geo.perfs[1][1][0]
    wi_inj = geo.perfs[0][1][0]
    assert pf[-1] == pytest.approx(m["wells"][1]["target"] + q * mu / wi_prod, rel=1e-12)
    assert bhp[0] == pytest.approx(pf[0] + q * mu / wi_inj, rel=1e-12)
    assert np.allclose(p[1::2], pf, rtol=1e-12)
    assert np.allclose(sw, 1.0 - m["sor"], atol=1e-13)


def test_single_cell_equilibrium():
    """Matrix and fracture of one closed cell equilibrate at the pressure that
    holds the initial water mass: V (phi_f + phi_m) rho(p*) = M."""
    m = synth.model_single_cell()
    geo = ph.Geometry(m)
    x0 = ph.initial_state(m)
    acc0 = ph.accumulation(geo, x0)
    geo, states, _ = nt.run(m, tol=1e-8)  # floor: one ulp of p times the transfer coefficient
    x = states[-1]
    p = x[0:4:2]
    mtot = acc0[1].sum()
    pstar = m["p_ref"] + np.log(mtot / (m["rho_w_ref"] * geo.vol * (m["phi_f"][0] + m["phi_m"][0]))) / m["c_w"]
    assert p[0] == pytest.approx(pstar, rel=1e-9)
    assert p[1] == pytest.approx(pstar, rel=1e-9)
    acc = ph.accumulation(geo, x)
    assert acc[1].sum() == pytest.approx(mtot, rel=1e-13)


def test_material_balance_small_model():
    geo, states, reports = nt.run(synth.model_small())
    for rep in reports:
        for r in rep:
            assert r["mb_oil"] <= 1e-10 and r["mb_water"] <= 1e-10
    p, sw, _ = ph.unpack_state(states[-1], geo.n)
    assert np.all((sw >= 0) & (sw <= 1))
    assert sw.max() > synth.base_physics()["swc"] + 0.1  # water has entered


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (2, 2, 1), (3, 2, 2), (3, 3, 2)])
def test_dense_vs_sparse_direct(dims):
    m = synth.model_tiny(*dims, seed=sum(dims), wells=dims[0] * dims[1] > 1)
    geo = ph.Geometry(m)
    ctrl = _ctrl(m)
    x = ph.pack_state(*synth.random_state(m, 4))
    acc_old = ph.accumulation(geo, ph.initial_state(m))
    R = ph.residual(geo, x, acc_old, synth.DAY, ctrl)
    J = ph.jacobian(geo, x, synth.DAY, ctrl)
    yd = np.linalg.solve(J.toarray(), -R)
    ys = spla.spsolve(J.tocsc(), -R)
    kappa = np.linalg.cond(J.toarray())
    assert np.linalg.norm(yd - ys) <= 1e-13 * kappa * np.linalg.norm(yd)
