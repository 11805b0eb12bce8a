"""Seeded model descriptions (data only) for the dual-porosity oil-water runs.

A *model* is a plain dict of numbers and NumPy arrays:

  grid      nx, ny, nz, dx, dy, dz [m], top_depth [m, depth of the top-layer
            centre, z grows downward], gravity [m/s^2]
  fields    kx, ky, kz (fracture) and km (matrix, isotropic) [m^2];
            phi_f, phi_m [fraction of the cell bulk volume]; all of length n,
            cell c = i + nx*(j + ny*k)
  fluids    rho_w_ref, rho_o_ref [kg/m^3] at p_ref [Pa]; c_w, c_o [1/Pa];
            mu_w, mu_o [Pa s]
  rel.perm  swc, sor, n_w, n_o, krw_max, kro_max (Corey)
  transfer  sigma [1/m^2] (shape factor)
  wells     list of dicts: i, j, k0, k1 (vertical perforated column),
            kind ('inj' water injector | 'prod' producer),
            control ('rate' | 'bhp'), target (m^3/s at reference water
            density for rate, Pa for bhp), bhp_limit [Pa], rw [m], skin
  state     p0, sw0 of length 2n in node order (node 2c fracture, 2c+1 matrix)
  schedule  list of timestep lengths [s]

The numbers that the paper's examples and the benchmark configurations do not
fix (reference densities, p_ref, depths, rates, BHPs) are chosen here once and
read by both the oracle and the GPU library.
"""
import numpy as np
from scipy.ndimage import gaussian_filter

MD = 9.869233e-16  # 1 millidarcy in m^2
DAY = 86400.0


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def base_physics():
    """Fluid, rock-fluid and transfer constants shared by every configuration.

    Densities are the paper's Example 1 values (62.4 and 58.0 lbm/ft^3) in SI;
    compressibilities and viscosities are the benchmark configuration's.
    """
    return dict(
        rho_w_ref=999.55, rho_o_ref=929.07, p_ref=30.0e6,
        c_w=4.5e-10, c_o=1.0e-9, mu_w=0.5e-3, mu_o=2.0e-3,
        swc=0.2, sor=0.2, n_w=2.0, n_o=2.0, krw_max=1.0, kro_max=1.0,
        sigma=0.08, gravity=9.80665, top_depth=609.6,
    )


def _well(i, j, k0, k1, kind, control, target, bhp_limit=60.0e6, rw=0.0762, skin=0.0):
    return dict(i=int(i), j=int(j), k0=int(k0), k1=int(k1), kind=kind, control=control,
                target=float(target), bhp_limit=float(bhp_limit), rw=float(rw), skin=float(skin))


def make_model(nx, ny, nz, dx, dy, dz, kx, ky, kz, km, phi_f, phi_m, wells,
               schedule, p_init=30.0e6, sw_init=None, **overrides):
    """Assemble a model dict with S_w = S_wc and a hydrostatic initial pressure:
    p_init in the top layer, rising by rho_o,ref * gravity * dz per layer (the
    same value in the fracture and matrix node of a cell)."""
    m = base_physics()
    m.update(overrides)
    n = nx * ny * nz
    m.update(nx=int(nx), ny=int(ny), nz=int(nz), dx=float(dx), dy=float(dy), dz=float(dz))
    for name, arr in (("kx", kx), ("ky", ky), ("kz", kz), ("km", km),
                      ("phi_f", phi_f), ("phi_m", phi_m)):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(arr, dtype=np.float64), (n,)))
        m[name] = a.copy()
    m["wells"] = list(wells)
    m["schedule"] = [float(t) for t in schedule]
    layer = np.arange(n) // (nx * ny)
    p_cell = float(p_init) + m["rho_o_ref"] * m["gravity"] * float(dz) * layer
    m["p0"] = np.repeat(p_cell, 2)
    m["sw0"] = np.full(2 * n, float(m["swc"] if sw_init is None else sw_init))
    return m


def _porosities(rng, n):
    phi_f = rng.uniform(0.005, 0.02, n)
    phi_m = rng.uniform(0.08, 0.2, n)
    return phi_f, phi_m


def model_small(seed=0):
    """10x10x3, 1200 DOF: i.i.d. lognormal fields, one injector, one BHP producer."""
    nx, ny, nz = 10, 10, 3
    n = nx * ny * nz
    rng = _rng(seed)
    kf = np.exp(rng.normal(np.log(100.0), 1.0, n)) * MD
    km = np.exp(rng.normal(np.log(0.1), 0.5, n)) * MD
    phi_f, phi_m = _porosities(rng, n)
    wells = [
        _well(0, 0, 0, nz - 1, "inj", "rate", 100.0 / DAY),
        _well(nx - 1, ny - 1, 0, nz - 1, "prod", "bhp", 20.0e6),
    ]
    return make_model(nx, ny, nz, 20.0, 20.0, 5.0, kf, kf, kf, km, phi_f, phi_m,
                      wells, [1.0 * DAY] * 10)


def _layered_field(rng, nx, ny, nz):
    """Per layer: white noise smoothed by a Gaussian of 5 cells, re-standardised
    to unit variance, plus a layer shift drawn from N(0, 0.5)."""
    out = np.empty((nz, ny, nx))
    for k in range(nz):
        w = gaussian_filter(rng.standard_normal((ny, nx)), sigma=5.0, mode="reflect")
        w = (w - w.mean()) / max(w.std(), 1e-300)
        out[k] = w
    shift = rng.normal(0.0, 0.5, nz)
    return (out + shift[:, None, None]).reshape(-1)


def _five_spot(nx, ny, nz, rate_each):
    return [
        _well(0, 0, 0, nz - 1, "inj", "rate", rate_each),
        _well(nx - 1, 0, 0, nz - 1, "inj", "rate", rate_each),
        _well(0, ny - 1, 0, nz - 1, "inj", "rate", rate_each),
        _well(nx - 1, ny - 1, 0, nz - 1, "inj", "rate", rate_each),
        _well(nx // 2, ny // 2, 0, nz - 1, "prod", "bhp", 20.0e6),
    ]


def layered_model(nx, ny, nz, seed, rate_each, schedule):
    rng = _rng(seed)
    n = nx * ny * nz
    kf = np.exp(np.log(100.0) + _layered_field(rng, nx, ny, nz)) * MD
    km = np.exp(rng.normal(np.log(0.1), 0.5, n)) * MD
    phi_f, phi_m = _porosities(rng, n)
    return make_model(nx, ny, nz, 20.0, 20.0, 5.0, kf, kf, kf, km, phi_f, phi_m,
                      _five_spot(nx, ny, nz, rate_each), schedule)


def model_layered(seed=1):
    """60x60x10, 144k DOF: layered lognormal field, five-spot (4 injectors, 1 producer)."""
    return layered_model(60, 60, 10, seed, 1000.0 / DAY, [5.0 * DAY] * 30)


def model_channelised(seed=2, nx=60, ny=220, nz=85, steps=20):
    """60x220x85, 4.49M DOF: channelised fracture field (30% channels along y)."""
    rng = _rng(seed)
    n = nx * ny * nz
    g = gaussian_filter(rng.standard_normal((nz, ny, nx)), sigma=(1.0, 20.0, 2.0), mode="reflect")
    g = g.reshape(-1)
    thr = np.percentile(g, 70.0)
    channel = g > thr
    lnk = np.where(channel,
                   rng.normal(np.log(500.0), 1.0, n),
                   rng.normal(np.log(1.0), 1.5, n))
    kx = np.exp(lnk) * MD
    km = np.exp(rng.normal(np.log(0.05), 0.7, n)) * MD
    phi_f, phi_m = _porosities(rng, n)
    wells = [
        _well(nx // 2, ny // 2, 0, nz - 1, "inj", "rate", 20000.0 / DAY),
        _well(0, 0, 0, nz - 1, "prod", "bhp", 20.0e6),
        _well(nx - 1, 0, 0, nz - 1, "prod", "bhp", 20.0e6),
        _well(0, ny - 1, 0, nz - 1, "prod", "bhp", 20.0e6),
        _well(nx - 1, ny - 1, 0, nz - 1, "prod", "bhp", 20.0e6),
    ]
    m = make_model(nx, ny, nz, 20.0, 20.0, 5.0, kx, kx, 0.1 * kx, km, phi_f, phi_m,
                   wells, [10.0 * DAY] * steps)
    m["channel_fraction"] = float(channel.mean())
    return m


def model_channelised_fp32(seed=2, **kw):
    """Same model as model_channelised (identical seed); the preconditioner runs in FP32."""
    m = model_channelised(seed, **kw)
    m["precond_precision"] = "fp32"
    return m


def served_size_classes():
    return [(20, 20, 10), (40, 40, 10), (60, 60, 10), (100, 100, 20), (60, 220, 85)]


def served_realisation(r, size):
    """Realisation r of the served ensemble: the layered five-spot model of
    model_layered at the given size, with the same injection rate per
    perforated layer (100 m^3/day) and ten 5-day steps."""
    nx, ny, nz = size
    return layered_model(nx, ny, nz, 1000 + r, 100.0 * nz / DAY, [5.0 * DAY] * 10)


def served_stream(count=256, rate=4.0, seed=4, classes=None):
    """Poisson arrivals: returns a list of (arrival_time_s, realisation, size)."""
    rng = _rng(seed)
    classes = served_size_classes() if classes is None else classes
    gaps = rng.exponential(1.0 / rate, count)
    which = rng.integers(0, len(classes), count)
    t = np.cumsum(gaps)
    return [(float(t[r]), r, classes[int(which[r])]) for r in range(count)]


# --------------------------------------------------------------------------
# Small models used by the oracle's pins
# --------------------------------------------------------------------------

def model_1d(nx=8, k=None, q_m3_per_day=50.0, p_bhp=20.0e6, sigma=0.08, dx=20.0):
    """nx x 1 x 1, water-only flow (S_w = 1 - S_or so k_ro = 0), incompressible
    fluids, no gravity: rate injector in cell 0, BHP producer in cell nx-1."""
    if k is None:
        k = np.full(nx, 100.0 * MD)
    k = np.asarray(k, dtype=np.float64)
    km = np.full(nx, 0.1 * MD)
    phi_f = np.full(nx, 0.01)
    phi_m = np.full(nx, 0.1)
    wells = [_well(0, 0, 0, 0, "inj", "rate", q_m3_per_day / DAY, bhp_limit=1e12),
             _well(nx - 1, 0, 0, 0, "prod", "bhp", p_bhp)]
    bp = base_physics()
    return make_model(nx, 1, 1, dx, 20.0, 5.0, k, k, k, km, phi_f, phi_m, wells,
                      [1.0 * DAY], sw_init=1.0 - bp["sor"], c_w=0.0, c_o=0.0,
                      gravity=0.0, sigma=sigma)


def model_single_cell(p_f0=29.0e6, p_m0=31.0e6):
    """One cell, no wells, water only (S_w = 1), fracture and matrix out of equilibrium."""
    m = make_model(1, 1, 1, 20.0, 20.0, 5.0, 100 * MD, 100 * MD, 100 * MD, 0.1 * MD,
                   0.01, 0.15, [], [1.0e12], sw_init=1.0)
    m["p0"] = np.array([p_f0, p_m0])
    return m


def model_tiny(nx, ny, nz, seed=0, wells=True, gravity=True):
    """Small random model for brute-force and derivative checks."""
    rng = _rng(seed)
    n = nx * ny * nz
    kx = np.exp(rng.normal(np.log(100.0), 1.0, n)) * MD
    ky = np.exp(rng.normal(np.log(100.0), 1.0, n)) * MD
    kz = 0.1 * np.exp(rng.normal(np.log(100.0), 1.0, n)) * MD
    km = np.exp(rng.normal(np.log(0.1), 0.5, n)) * MD
    phi_f, phi_m = _porosities(rng, n)
    wl = []
    if wells:
        wl.append(_well(0, 0, 0, nz - 1, "inj", "rate", 20.0 / DAY))
        wl.append(_well(nx - 1, ny - 1, 0, nz - 1, "prod", "bhp", 25.0e6))
    extra = {} if gravity else dict(gravity=0.0)
    return make_model(nx, ny, nz, 20.0, 20.0, 5.0, kx, ky, kz, km, phi_f, phi_m, wl,
                      [1.0 * DAY] * 3, **extra)


def random_state(model, seed, p_lo=24.0e6, p_hi=32.0e6, margin=0.02):
    """A random interior state: node pressures, saturations strictly inside the
    mobile range (away from the Corey kinks) and well pressures."""
    rng = _rng(seed)
    n = model["nx"] * model["ny"] * model["nz"]
    p = rng.uniform(p_lo, p_hi, 2 * n)
    lo = model["swc"] + margin
    hi = 1.0 - model["sor"] - margin
    sw = rng.uniform(lo, hi, 2 * n)
    bhp = np.array([w["target"] if w["control"] == "bhp" else rng.uniform(p_lo, p_hi)
                    for w in model["wells"]], dtype=np.float64)
    return p, sw, bhp
