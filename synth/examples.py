"""The paper's Examples 1 and 2 (Sec. 4) as model inputs, converted from the
field units the paper prints to SI.

Only unit conversion and layout happen here.  What the paper does not print is
a stated reading, the same for both examples:
  * relative permeability: Corey curves with exponent 2, S_wc = 0, S_or = 0.2,
    end-point values 1, the same in both media (the paper gives no curves);
  * water: compressibility 3e-6 1/psi, viscosity 1 cp, formation volume factor 1
    (the paper gives only the water density);
  * oil: the reference density is the printed density divided by the printed
    formation volume factor at the reference pressure, growing with the printed
    compressibility (rho = rho_ref exp(c (p - p_ref)));
  * the matrix permeability enters only the transfer term, through its
    arithmetic mean over the three directions (Kazemi's shape factor with equal
    fracture spacings); the shape factor is the benchmark models' 0.08 1/m^2;
  * initial pressures are those of the top layer; deeper layers add the oil
    hydrostatic gradient rho_o,ref g dz per layer, in both media;
  * rate targets: the injector's water rate is a surface rate with B_w = 1; a
    producer's maximum oil rate (STB/day) becomes a target in m^3/s at the
    reservoir reference density, target = Q_stb * B_o,ref, so that
    rho_o,ref * target is the printed surface mass rate;
  * cells are 1-based [i j k] in the paper, 0-based here;
  * timesteps: 1, 1, 2, 4, 8, 16 days, then equal steps to the printed period
    (12 days for Example 1's 800 days, 16 days for Example 2's 1600 days).
"""
import numpy as np

from .models import DAY, MD, make_model

FT = 0.3048                      # m
PSI = 6894.757293168361          # Pa (lbf/in^2)
LBM_FT3 = 0.45359237 / FT ** 3   # kg/m^3
BBL = 0.158987294928             # m^3
CP = 1.0e-3                      # Pa s
# well index in rb cp / (day psi) -> m^3
WI_FIELD = BBL * CP / (DAY * PSI)

# The printed values, in the paper's units (Sec. 4, Examples 1 and 2).
PRINTED = {
    1: dict(grid=(10, 10, 1), dxy_ft=102.04, dz_ft=100.0, top_ft=2000.0,
            km_md=(100.0, 100.0, 10.0), kf_md=395.85, phi_m=0.1392, phi_f=0.039585,
            c_r_psi=3.0e-6, p_ref_psi=15.0, rho_o_lbm=58.0, rho_w_lbm=62.4, bo_ref=1.036,
            mu_o_cp=40.0, c_o_psi=1.313e-5, p_m_psi=2000.0, p_f_psi=1980.0, sw_m=0.08, sw_f=0.01,
            inj_cell=(5, 1, 1), inj_rate_bbl=500.0, inj_bhp_max_psi=5.0e4, inj_wi=200.0,
            prod_cells=((1, 10, 1), (10, 10, 1)), prod_oil_stb=300.0, prod_bhp_min_psi=15.0,
            rw_ft=0.25, days=800.0),
    2: dict(grid=(10, 10, 3), dxy_ft=102.0, dz_ft=100.0, top_ft=2000.0,
            km_md=(100.0, 100.0, 100.0), kf_md=395.85, phi_m=0.1392, phi_f=0.039585,
            c_r_psi=3.0e-6, p_ref_psi=15.0, rho_o_lbm=58.0, rho_w_lbm=62.4, bo_ref=1.036,
            mu_o_cp=40.0, c_o_psi=1.313e-5, p_m_psi=800.0, p_f_psi=500.0, sw_m=0.08, sw_f=0.01,
            inj_cell=(5, 5, 1), inj_rate_bbl=200.0, inj_bhp_max_psi=5.0e4, inj_wi=200.0,
            prod_cells=((1, 1, 1), (10, 10, 1)), prod_oil_stb=500.0, prod_bhp_min_psi=15.0,
            rw_ft=0.25, days=1600.0),
}

RAMP_DAYS = (1.0, 1.0, 2.0, 4.0, 8.0, 16.0)
STEP_DAYS = {1: 12.0, 2: 16.0}


def _schedule(days, step):
    """The ramp, then equal steps, then what remains (none for the printed periods)."""
    out, t = [], 0.0
    for d in RAMP_DAYS:
        if t + d > days + 1e-9:
            break
        out.append(d)
        t += d
    while t + step <= days + 1e-9:
        out.append(step)
        t += step
    if days - t > 1e-9:
        out.append(days - t)
    return [d * DAY for d in out]


def paper_example(number, grid=None, days=None):
    """Example 1 or 2 of Sec. 4 as a model dict (SI).  ``grid`` replaces the
    printed grid dimensions (same cell sizes; wells keep their printed cells,
    clamped into the grid, and perforate the top layer only), ``days`` the
    simulated period."""
    e = PRINTED[number]
    nx, ny, nz = e["grid"] if grid is None else grid
    n = nx * ny * nz
    dxy, dz = e["dxy_ft"] * FT, e["dz_ft"] * FT
    rho_o_ref = e["rho_o_lbm"] * LBM_FT3 / e["bo_ref"]
    rho_w_ref = e["rho_w_lbm"] * LBM_FT3
    rw = e["rw_ft"] * FT

    def cell(c):
        i, j, k = c
        return min(i - 1, nx - 1), min(j - 1, ny - 1), min(k - 1, nz - 1)

    wells = []
    i, j, k = cell(e["inj_cell"])
    wells.append(dict(i=i, j=j, k0=k, k1=k, kind="inj", control="rate",
                      target=e["inj_rate_bbl"] * BBL / DAY, bhp_limit=e["inj_bhp_max_psi"] * PSI,
                      rw=rw, skin=0.0, wi=e["inj_wi"] * WI_FIELD))
    for c in e["prod_cells"]:
        i, j, k = cell(c)
        wells.append(dict(i=i, j=j, k0=k, k1=k, kind="prod", control="orate",
                          target=e["prod_oil_stb"] * e["bo_ref"] * BBL / DAY,
                          bhp_limit=e["prod_bhp_min_psi"] * PSI, rw=rw, skin=0.0))
    kf = e["kf_md"] * MD
    km = float(np.mean(e["km_md"])) * MD
    sched = _schedule(e["days"] if days is None else days, STEP_DAYS[number])
    m = make_model(nx, ny, nz, dxy, dxy, dz, kf, kf, kf, km, e["phi_f"], e["phi_m"], wells, sched,
                   p_init=e["p_m_psi"] * PSI,
                   rho_o_ref=rho_o_ref, rho_w_ref=rho_w_ref, p_ref=e["p_ref_psi"] * PSI,
                   c_o=e["c_o_psi"] / PSI, c_w=3.0e-6 / PSI, mu_o=e["mu_o_cp"] * CP, mu_w=1.0 * CP,
                   swc=0.0, sor=0.2, n_w=2.0, n_o=2.0, krw_max=1.0, kro_max=1.0,
                   top_depth=e["top_ft"] * FT, c_r=e["c_r_psi"] / PSI)
    layer = np.arange(n) // (nx * ny)
    hydro = rho_o_ref * m["gravity"] * dz * layer
    p0 = np.empty(2 * n)
    p0[0::2] = e["p_f_psi"] * PSI + hydro
    p0[1::2] = e["p_m_psi"] * PSI + hydro
    m["p0"] = p0
    sw0 = np.empty(2 * n)
    sw0[0::2] = e["sw_f"]
    sw0[1::2] = e["sw_m"]
    m["sw0"] = sw0
    return m
