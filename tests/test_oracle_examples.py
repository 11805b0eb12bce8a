"""Pins of the oracle's Example 1 and 2 physics (Sec. 4): rock compressibility,
producers on oil-rate control with a minimum BHP, a well index given as data,
and the printed inputs in field units (no GPU)."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from synth import examples as ex
from oracle import newton as nt
from oracle import physics as ph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# unit factors written out here, independently of the input generator
FT = 0.3048
PSI = 4.4482216152605 / 0.0254 ** 2
MD = 9.869233e-16
BBL = 42 * 231 * 0.0254 ** 3
LBM_FT3 = 0.45359237 / FT ** 3
DAY = 86400.0


def _printed():
    out = {1: {}, 2: {}}
    for line in open(os.path.join(GOLDEN, "paper_examples.txt")):
        if line.startswith("#") or not line.strip():
            continue
        e, name, val, unit, _ = line.split()
        out[int(e)][name] = (float(val), unit)
    return out


@pytest.mark.parametrize("number", [1, 2])
def test_example_inputs_match_the_printed_values(number):
    g = _printed()[number]
    m = synth.paper_example(number)
    assert (m["nx"], m["ny"], m["nz"]) == tuple(int(g[k][0]) for k in ("grid_nx", "grid_ny", "grid_nz"))
    close = lambda a, b: a == pytest.approx(b, rel=1e-12)  # noqa: E731
    assert close(m["dx"], g["dxy"][0] * FT) and close(m["dy"], g["dxy"][0] * FT)
    assert close(m["dz"], g["dz"][0] * FT)
    assert close(m["top_depth"], g["top_depth"][0] * FT)
    assert np.allclose(m["kx"], g["kf"][0] * MD, rtol=1e-12)
    assert np.allclose(m["kz"], g["kf"][0] * MD, rtol=1e-12)
    km = np.mean([g["km_x"][0], g["km_y"][0], g["km_z"][0]]) * MD
    assert np.allclose(m["km"], km, rtol=1e-12)
    assert np.all(m["phi_m"] == g["phi_m"][0]) and np.all(m["phi_f"] == g["phi_f"][0])
    assert close(m["c_r"], g["c_r"][0] / PSI)
    assert close(m["p_ref"], g["p_ref"][0] * PSI)
    assert close(m["rho_o_ref"], g["rho_o"][0] * LBM_FT3 / g["bo_ref"][0])
    assert close(m["rho_w_ref"], g["rho_w"][0] * LBM_FT3)
    assert close(m["mu_o"], g["mu_o"][0] * 1e-3)
    assert close(m["c_o"], g["c_o"][0] / PSI)
    top = slice(0, 2 * m["nx"] * m["ny"])
    assert np.allclose(m["p0"][top][0::2], g["p_f"][0] * PSI, rtol=1e-12)
    assert np.allclose(m["p0"][top][1::2], g["p_m"][0] * PSI, rtol=1e-12)
    assert np.all(m["sw0"][0::2] == g["sw_f"][0]) and np.all(m["sw0"][1::2] == g["sw_m"][0])
    inj, p1, p2 = m["wells"]
    assert close(inj["target"], g["inj_rate"][0] * BBL / DAY)
    assert close(inj["bhp_limit"], g["inj_bhp_max"][0] * PSI)
    # rb cp / (day psi) -> m^3
    assert close(inj["wi"], g["inj_wi"][0] * BBL * 1e-3 / (DAY * PSI))
    for p in (p1, p2):
        assert p["control"] == "orate"
        # rho_o,ref * target is the printed surface oil mass rate
        assert close(m["rho_o_ref"] * p["target"], g["prod_oil_rate"][0] * BBL / DAY * g["rho_o"][0] * LBM_FT3)
        assert close(p["bhp_limit"], g["prod_bhp_min"][0] * PSI)
        assert close(p["rw"], g["rw"][0] * FT)
    assert sum(m["schedule"]) == pytest.approx(g["period"][0] * DAY, rel=1e-12)


def _with(m, **kw):
    m = dict(m)
    m.update(kw)
    return m


@pytest.mark.parametrize("controls", [("rate", "orate", "orate"), ("bhp", "bhp", "orate")])
def test_jacobian_complex_step_with_example_physics(controls):
    """Rock compressibility, oil-rate rows and a given well index in the analytic
    Jacobian, against complex-step derivatives of the residual."""
    m = synth.paper_example(2, grid=(3, 3, 2))
    geo = ph.Geometry(m)
    x = ph.pack_state(*synth.random_state(m, 3, p_lo=3e6, p_hi=6e6))
    acc_old = ph.accumulation(geo, ph.pack_state(*synth.random_state(m, 4, p_lo=3e6, p_hi=6e6)))
    dt = 2.0 * synth.DAY
    ctrl = list(controls)
    J = ph.jacobian(geo, x, dt, ctrl).toarray()
    Jc = np.empty_like(J)
    for j in range(geo.N):
        xc = x.astype(complex)
        xc[j] += 1j * 1e-30
        Jc[:, j] = ph.residual(geo, xc, acc_old, dt, ctrl).imag / 1e-30
    cs = np.abs(Jc).max(axis=0, keepdims=True)
    cs[cs == 0] = 1.0
    assert np.max(np.abs(J - Jc) / cs) <= 1e-10


def _closed(m, keep):
    """The model with only the wells listed in keep, incompressible fluids."""
    wells = [m["wells"][i] for i in keep]
    return _with(m, wells=wells, c_o=0.0, c_w=0.0)


def _one_step(m, dt):
    geo = ph.Geometry(m)
    x0 = ph.initial_state(m)
    acc = ph.accumulation(geo, x0)
    ctrl = [w["control"] for w in m["wells"]]
    x1, ok, its, _ = nt.newton_solve(geo, x0, acc, dt, ctrl, tol=1e-12, mb_tol=1e-13, max_newton=30)
    assert ok
    return geo, x0, x1


def test_rock_compressibility_takes_up_the_injected_volume():
    """A closed reservoir with incompressible fluids and one water injector on
    rate control: the pores must grow by the injected volume, so
    sum_nodes V phi_ref c_r (p^{n+1} - p^n) = Q dt, and the oil volume
    sum V phi(p) (1 - S_w) stays the same (backward Euler is exact for these
    linear relations)."""
    m = _closed(synth.paper_example(2, grid=(4, 3, 2)), [0])
    dt = 2.0 * synth.DAY
    geo, x0, x1 = _one_step(m, dt)
    p0, s0, _ = ph.unpack_state(x0, geo.n)
    p1, s1, _ = ph.unpack_state(x1, geo.n)
    v = geo.vol * geo.phi * m["c_r"]
    q = m["wells"][0]["target"]
    assert np.sum(v * (p1 - p0)) == pytest.approx(q * dt, rel=1e-9)
    phi = lambda p: geo.phi * (1.0 + m["c_r"] * (p - m["p_ref"]))  # noqa: E731
    assert np.sum(geo.vol * phi(p1) * (1 - s1)) == pytest.approx(np.sum(geo.vol * phi(p0) * (1 - s0)),
                                                                 rel=1e-12)


def test_oil_rate_producer_releases_the_target_volume():
    """A closed reservoir with incompressible fluids, immobile water (S_w = 0 =
    S_wc) and one producer on oil-rate control: the pores shrink by the produced
    oil volume, sum V phi_ref c_r (p^n - p^{n+1}) = Q_o dt."""
    m = _closed(synth.paper_example(2, grid=(4, 3, 2)), [1])
    m["sw0"] = np.zeros_like(m["sw0"])
    # 5% of the printed rate: the small closed block cannot sustain more
    m["wells"] = [dict(m["wells"][0], target=0.05 * m["wells"][0]["target"])]
    dt = 1.0 * synth.DAY
    geo, x0, x1 = _one_step(m, dt)
    p0, _, _ = ph.unpack_state(x0, geo.n)
    p1, s1, b1 = ph.unpack_state(x1, geo.n)
    assert np.all(s1 == 0.0)
    assert b1[0] > m["wells"][0]["bhp_limit"]
    v = geo.vol * geo.phi * m["c_r"]
    assert np.sum(v * (p0 - p1)) == pytest.approx(m["wells"][0]["target"] * dt, rel=1e-9)


def test_producer_switches_to_bhp_at_its_minimum():
    """An oil-rate target the reservoir cannot deliver drives p_b below the
    minimum: the step is redone on BHP control, p_b sits at the limit and the
    oil rate falls short of the target."""
    m = synth.paper_example(2, grid=(4, 3, 2))
    m["wells"] = [m["wells"][0], dict(m["wells"][1], target=m["wells"][1]["target"] * 1e3)]
    geo = ph.Geometry(m)
    x, rep, ctrl = nt.timestep(geo, ph.initial_state(m), 1.0 * synth.DAY, ["rate", "orate"], tol=1e-10)
    assert ctrl == ["rate", "bhp"]
    _, _, b = ph.unpack_state(x, geo.n)
    assert b[1] == m["wells"][1]["bhp_limit"]
    qo = float(np.sum(ph.well_rates(geo, x, ctrl)[1][1]))
    assert 0.0 < -qo < m["rho_o_ref"] * m["wells"][1]["target"]


def test_given_well_index_is_the_peaceman_index_route():
    """A well index given as data enters exactly as Eq. (8)'s computed one: an
    isotropic square cell's Peaceman index, 2 pi k dz / ln(r_e/r_w) with
    r_e = 0.14 sqrt(2) dx, written here by hand and given as data, reproduces
    the residual of the computed route."""
    m = synth.model_tiny(3, 3, 2, seed=1)
    k = 150.0 * MD
    for key in ("kx", "ky"):
        m[key] = np.full_like(m[key], k)
    w0 = m["wells"][0]
    wi = 2 * np.pi * k * m["dz"] / np.log(0.14 * np.sqrt(2.0) * m["dx"] / w0["rw"])
    m2 = _with(m, wells=[dict(w0, wi=wi)] + m["wells"][1:])
    x = ph.pack_state(*synth.random_state(m, 2))
    for mm in (m, m2):
        geo = ph.Geometry(mm)
        acc = ph.accumulation(geo, ph.initial_state(mm))
        R = ph.residual(geo, x, acc, synth.DAY, [w["control"] for w in mm["wells"]])
        if mm is m:
            R1 = R
    assert np.max(np.abs(R - R1)) <= 1e-13 * np.max(np.abs(R1))


def test_example_1_runs_800_days_with_consistent_wells():
    """Qualitative self-consistency of the whole Example 1 run (the paper's
    comparison curves are not available): every step conserves mass to 1e-10,
    the injector keeps its rate below its BHP maximum, each producer holds its
    oil rate or sits at its BHP minimum, and the producers see water before the
    end."""
    m = synth.paper_example(1)
    geo = ph.Geometry(m)
    x = ph.initial_state(m)
    ctrl = [w["control"] for w in m["wells"]]
    watercut = []
    for dt in m["schedule"]:
        x, rep, ctrl = nt.timestep(geo, x, dt, ctrl, tol=1e-10)
        for r in rep:
            assert max(r["mb_oil"], r["mb_water"]) <= 1e-10
        _, _, b = ph.unpack_state(x, geo.n)
        rates = ph.well_rates(geo, x, ctrl)
        assert ctrl[0] == "rate" and b[0] <= m["wells"][0]["bhp_limit"]
        assert float(np.sum(rates[0][2])) == pytest.approx(m["rho_w_ref"] * m["wells"][0]["target"], rel=1e-6)
        wc = []
        for w in (1, 2):
            qo = -float(np.sum(rates[w][1]))
            qw = -float(np.sum(rates[w][2]))
            wl = m["wells"][w]
            if ctrl[w] == "orate":
                assert qo == pytest.approx(m["rho_o_ref"] * wl["target"], rel=1e-6)
                assert b[w] >= wl["bhp_limit"]
            else:
                assert b[w] == wl["bhp_limit"] and qo <= m["rho_o_ref"] * wl["target"] * (1 + 1e-8)
            wc.append(qw / (qo + qw))
        watercut.append(wc)
    watercut = np.array(watercut)
    assert watercut[-1].min() > 10 * watercut[0].max()
