"""Oracle physics: properties, geometry, residual and analytic Jacobian.

Part of the CPU oracle (test infrastructure only; see the package docstring).

Unknowns and equations (Sec. 3, first paragraph; reading of the unknown count
in Eq. (11)): every cell c = i + nx*(j + ny*k) carries two nodes, the fracture
node 2c and the matrix node 2c+1.  Each node carries (p_o [Pa], S_w); the two
equations of a node are the oil and water mass balances [kg/s].  Every well w
carries its bottom-hole pressure p_b and a dummy unknown (so that all blocks
are 2x2); its first equation is the control equation (rate: the well's net
mass rate, the sum of both phases' perforation rates, minus the target water
mass rate, Eqs. (6)-(7) -- while every perforation injects, the water rate;
oil rate (producers): the oil perforation rates plus the target oil mass rate;
BHP: p_b minus the target) and its second is ``dummy = 0``.

Global unknown index: node q -> (2q, 2q+1) = (p, S_w); well w -> (4n+2w,
4n+2w+1) = (p_b, dummy).  Equation index: node q -> (2q, 2q+1) = (oil, water).

Every function takes NumPy arrays and also works on complex arrays, so that a
complex-step derivative of the residual can check the analytic Jacobian.  All
branch decisions (upwinding, Corey clipping) use real parts.
"""
import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------
# Properties (Eq. (3)-(4); rock-fluid model by reading: Corey curves,
# exponential density law, zero capillary pressure)
# --------------------------------------------------------------------------

def _ipow(x, e):
    """x**e, using repeated products when e is integral (exact for complex x)."""
    if float(e).is_integer():
        return x ** int(e)
    return x ** e


def density(p, rho_ref, c, p_ref):
    """rho(p) = rho_ref * exp(c (p - p_ref)) and its derivative."""
    rho = rho_ref * np.exp(c * (p - p_ref))
    return rho, c * rho


def corey(sw, m):
    """Corey relative permeabilities and their S_w-derivatives.

    s* = clip((S_w - S_wc)/(1 - S_wc - S_or), 0, 1); k_rw = krw_max s*^n_w,
    k_ro = kro_max (1 - s*)^n_o.  The derivative of s* is 1/(1 - S_wc - S_or)
    on the closed interval 0 <= s*_raw <= 1 and 0 outside it.
    """
    delta = 1.0 - m["swc"] - m["sor"]
    raw = (sw - m["swc"]) / delta
    rr = np.real(raw)
    s = np.where(rr < 0.0, 0.0, np.where(rr > 1.0, 1.0, raw))
    ds = np.where((rr >= 0.0) & (rr <= 1.0), 1.0 / delta, 0.0)
    nw, no = m["n_w"], m["n_o"]
    krw = m["krw_max"] * _ipow(s, nw)
    kro = m["kro_max"] * _ipow(1.0 - s, no)
    dkrw = m["krw_max"] * nw * _ipow(s, nw - 1.0) * ds
    dkro = -m["kro_max"] * no * _ipow(1.0 - s, no - 1.0) * ds
    return krw, kro, dkrw, dkro


# --------------------------------------------------------------------------
# Geometry: faces, transmissibilities, transfer coefficient, well index
# --------------------------------------------------------------------------

def cell_ijk(m):
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    c = np.arange(nx * ny * nz)
    return c % nx, (c // nx) % ny, c // (nx * ny)


def depth(m):
    """Cell-centre depth z (positive downward); the top layer centre sits at top_depth."""
    _, _, k = cell_ijk(m)
    return m["top_depth"] + k * m["dz"]


def faces(m):
    """Interior fracture faces (c, d) with c < d, the TPFA transmissibility
    T = 2 A k_c k_d / (L (k_c + k_d)) (harmonic average of the two half-cell
    conductances), and the depth difference z_d - z_c.  Outer faces are no-flow."""
    nx, ny, nz = m["nx"], m["ny"], m["nz"]
    dx, dy, dz = m["dx"], m["dy"], m["dz"]
    c = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    out_c, out_d, out_t, out_dz = [], [], [], []
    for axis, kname, area, length, dzv in ((2, "kx", dy * dz, dx, 0.0),
                                           (1, "ky", dx * dz, dy, 0.0),
                                           (0, "kz", dx * dy, dz, dz)):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[axis] = slice(0, -1)
        sl_hi[axis] = slice(1, None)
        a = c[tuple(sl_lo)].reshape(-1)
        b = c[tuple(sl_hi)].reshape(-1)
        k = m[kname]
        t = 2.0 * area * k[a] * k[b] / (length * (k[a] + k[b]))
        out_c.append(a)
        out_d.append(b)
        out_t.append(t)
        out_dz.append(np.full(a.shape, dzv))
    return (np.concatenate(out_c), np.concatenate(out_d), np.concatenate(out_t),
            np.concatenate(out_dz))


def transfer_coeff(m):
    """Matrix-fracture coefficient omega = sigma * k_m * V (Warren-Root /
    Kazemi form of the shape-factor transfer term, Sec. 2 after Eq. (5))."""
    vol = m["dx"] * m["dy"] * m["dz"]
    return m["sigma"] * m["km"] * vol


def peaceman_re(dx, dy, kx, ky):
    """Peaceman equivalent radius of a vertical well (Eq. (10), the formula
    written with D_x, D_y, k_x, k_y)."""
    ryx = np.sqrt(ky / kx)
    rxy = np.sqrt(kx / ky)
    num = np.sqrt(dx * dx * ryx + dy * dy * rxy)
    den = ryx ** 0.5 + rxy ** 0.5
    return 0.28 * num / den


def well_perforations(m):
    """For every well, the perforated cells and their well indices
    W = 2 pi k_h w_frac / (ln(r_e/r_w) + s) with k_h = sqrt(kx ky) dz and
    w_frac = 1 (Eq. (8) with Eq. (10)), or the well's own index ``wi`` when it
    gives one (the examples of Sec. 4 state an injector's index directly)."""
    out = []
    nx, ny = m["nx"], m["ny"]
    for w in m["wells"]:
        cells = np.array([w["i"] + nx * (w["j"] + ny * k) for k in range(w["k0"], w["k1"] + 1)],
                         dtype=np.int64)
        kx = m["kx"][cells]
        ky = m["ky"][cells]
        re = peaceman_re(m["dx"], m["dy"], kx, ky)
        kh = np.sqrt(kx * ky) * m["dz"]
        wi = 2.0 * np.pi * kh / (np.log(re / w["rw"]) + w["skin"])
        if w.get("wi", 0.0) > 0.0:
            wi = np.full(cells.shape[0], float(w["wi"]))  # a well index given as data
        out.append((cells, wi))
    return out


class Geometry:
    """Precomputed, state-independent geometry of a model."""

    def __init__(self, m):
        self.m = m
        self.n = m["nx"] * m["ny"] * m["nz"]
        self.nw = len(m["wells"])
        self.N = 4 * self.n + 2 * self.nw
        self.vol = m["dx"] * m["dy"] * m["dz"]
        self.z = depth(m)
        self.fc, self.fd, self.ft, self.fdz = faces(m)
        self.tmf = transfer_coeff(m)
        self.perfs = well_perforations(m)
        # node porosity: node 2c fracture, 2c+1 matrix
        self.phi = np.empty(2 * self.n)
        self.phi[0::2] = m["phi_f"]
        self.phi[1::2] = m["phi_m"]


# --------------------------------------------------------------------------
# State helpers
# --------------------------------------------------------------------------

def pack_state(p, sw, bhp):
    n2 = p.shape[0]
    nw = bhp.shape[0]
    x = np.zeros(2 * n2 + 2 * nw, dtype=np.result_type(p, sw, bhp))
    x[0:2 * n2:2] = p
    x[1:2 * n2:2] = sw
    x[2 * n2::2] = bhp
    return x


def unpack_state(x, n):
    return x[0:4 * n:2], x[1:4 * n:2], x[4 * n::2]


def porosity(geo, p):
    """phi(p) = phi_ref (1 + c_r (p - p_ref)) per node, and d phi/dp (rock
    compressibility; the examples of Sec. 4 give c_r, the benchmark models use
    c_r = 0)."""
    c_r = geo.m.get("c_r", 0.0)
    return geo.phi * (1.0 + c_r * (p - geo.m["p_ref"])), geo.phi * c_r


def initial_state(m):
    bhp = np.array([w["target"] if w["control"] == "bhp" else m["p0"].mean()
                    for w in m["wells"]], dtype=np.float64)
    return pack_state(m["p0"].astype(np.float64), m["sw0"].astype(np.float64), bhp)


def accumulation(geo, x):
    """Phase masses per node: M_o = V phi(p) (1 - S_w) rho_o, M_w = V phi(p) S_w
    rho_w (porosity as a fraction of the cell bulk volume)."""
    m = geo.m
    p, sw, _ = unpack_state(x, geo.n)
    rho_o, _ = density(p, m["rho_o_ref"], m["c_o"], m["p_ref"])
    rho_w, _ = density(p, m["rho_w_ref"], m["c_w"], m["p_ref"])
    vphi = geo.vol * porosity(geo, p)[0]
    return vphi * (1.0 - sw) * rho_o, vphi * sw * rho_w


# --------------------------------------------------------------------------
# Residual and Jacobian (Eq. (5) discretised with backward Euler and TPFA)
# --------------------------------------------------------------------------

def _phase_props(m, p, sw):
    rho_o, drho_o = density(p, m["rho_o_ref"], m["c_o"], m["p_ref"])
    rho_w, drho_w = density(p, m["rho_w_ref"], m["c_w"], m["p_ref"])
    krw, kro, dkrw, dkro = corey(sw, m)
    return {
        "o": (rho_o, drho_o, kro, dkro, m["mu_o"]),
        "w": (rho_w, drho_w, krw, dkrw, m["mu_w"]),
    }


def well_rates(geo, x, control):
    """Perforation mass rates into the fracture node (positive = injection).

    Producer, and an injector's perforation in back-flow (p_b < p):
    q_a = rho_a(p) W lambda_a (p_b - p) with the block's phase mobilities (Eq. (6),
    permeability counted once, in W).  Injecting perforation of a water injector
    (p_b >= p): q_w = rho_w(p) W lambda_t (p_b - p), q_o = 0 (reading: water-only
    injection with the block's total mobility; the mobility is taken from the
    upstream side).  Returns a list per well of (cells, q_o, q_w)."""
    m = geo.m
    p, sw, bhp = unpack_state(x, geo.n)
    out = []
    for w, (cells, wi) in enumerate(geo.perfs):
        pf = p[2 * cells]
        s = sw[2 * cells]
        pr = _phase_props(m, pf, s)
        rho_o, _, kro, _, mu_o = pr["o"]
        rho_w, _, krw, _, mu_w = pr["w"]
        dp = bhp[w] - pf
        qo = rho_o * wi * (kro / mu_o) * dp
        qw = rho_w * wi * (krw / mu_w) * dp
        if m["wells"][w]["kind"] == "inj":
            inj = np.real(dp) >= 0.0
            lt = krw / mu_w + kro / mu_o
            qw = np.where(inj, rho_w * wi * lt * dp, qw)
            qo = np.where(inj, 0.0 * qw, qo)
        out.append((cells, qo, qw))
    return out


def residual(geo, x, acc_old, dt, control):
    """R(x) of the backward-Euler dual-porosity system.

    R_a(f_c) = [M_a - M_a^n]/dt - sum_d F_a,cd + q_a,mf - q_a,well
    R_a(m_c) = [M_a - M_a^n]/dt - q_a,mf
    F_a,cd   = T_cd (k_ra rho_a/mu_a)_up (Phi_a,d - Phi_a,c) is the flow into c
               from d, Phi_a = p - rho_bar_a g z, rho_bar the average of the
               two cells' densities; upstream = d if Phi_d > Phi_c else c
               (ties go to the lower cell index).
    q_a,mf   = omega (k_ra rho_a/mu_a)_up (p_f - p_m), flowing fracture ->
               matrix; upstream = f if p_f >= p_m else m.

    ``control[w]`` is 'rate', 'orate' or 'bhp' for each well.
    """
    m = geo.m
    n = geo.n
    p, sw, bhp = unpack_state(x, n)
    dtype = np.result_type(x, np.float64)
    R = np.zeros(geo.N, dtype=dtype)
    acc_o, acc_w = accumulation(geo, x)
    Ro = (acc_o - acc_old[0]) / dt
    Rw = (acc_w - acc_old[1]) / dt
    pr = _phase_props(m, p, sw)
    g = m["gravity"]
    fc, fd = 2 * geo.fc, 2 * geo.fd
    for ph, Rph in (("o", Ro), ("w", Rw)):
        rho, _, kr, _, mu = pr[ph]
        mob = kr * rho / mu
        rbar = 0.5 * (rho[fc] + rho[fd])
        dphi = (p[fd] - p[fc]) - rbar * g * geo.fdz
        up = np.where(np.real(dphi) > 0.0, fd, fc)
        F = geo.ft * mob[up] * dphi
        np.add.at(Rph, fc, -F)
        np.add.at(Rph, fd, F)
        # matrix-fracture transfer
        f = 2 * np.arange(n)
        mm = f + 1
        upm = np.where(np.real(p[f]) >= np.real(p[mm]), f, mm)
        q = geo.tmf * mob[upm] * (p[f] - p[mm])
        Rph[f] += q
        Rph[mm] -= q
    for w, (cells, qo, qw) in enumerate(well_rates(geo, x, control)):
        np.add.at(Ro, 2 * cells, -qo)
        np.add.at(Rw, 2 * cells, -qw)
        wl = m["wells"][w]
        if control[w] == "rate":
            R[4 * n + 2 * w] = np.sum(qo + qw) - m["rho_w_ref"] * wl["target"]
        elif control[w] == "orate":
            R[4 * n + 2 * w] = np.sum(qo) + m["rho_o_ref"] * wl["target"]
        else:
            target = wl["target"] if wl["control"] == "bhp" else wl["bhp_limit"]
            R[4 * n + 2 * w] = bhp[w] - target
        R[4 * n + 2 * w + 1] = x[4 * n + 2 * w + 1]
    R[0:4 * n:2] = Ro
    R[1:4 * n:2] = Rw
    return R


def jacobian(geo, x, dt, control):
    """Analytic dR/dx as a SciPy CSR matrix (duplicates summed)."""
    m = geo.m
    n = geo.n
    p, sw, bhp = unpack_state(x, n)
    rows, cols, vals = [], [], []

    def add(r, c, v):
        r = np.atleast_1d(r)
        rows.append(np.broadcast_to(r, np.broadcast(r, c, v).shape).ravel())
        cols.append(np.broadcast_to(c, np.broadcast(r, c, v).shape).ravel())
        vals.append(np.broadcast_to(v, np.broadcast(r, c, v).shape).ravel().astype(np.float64))

    pr = _phase_props(m, p, sw)
    nodes = np.arange(2 * n)
    phi, dphi_dp = porosity(geo, p)
    vphi = geo.vol * phi
    vdphi = geo.vol * dphi_dp
    rho_o, drho_o = pr["o"][0], pr["o"][1]
    rho_w, drho_w = pr["w"][0], pr["w"][1]
    # accumulation
    add(2 * nodes, 2 * nodes, (1.0 - sw) * (vphi * drho_o + vdphi * rho_o) / dt)
    add(2 * nodes, 2 * nodes + 1, -vphi * rho_o / dt)
    add(2 * nodes + 1, 2 * nodes, sw * (vphi * drho_w + vdphi * rho_w) / dt)
    add(2 * nodes + 1, 2 * nodes + 1, vphi * rho_w / dt)
    g = m["gravity"]
    fc, fd = 2 * geo.fc, 2 * geo.fd
    f = 2 * np.arange(n)
    mm = f + 1
    for eq, ph in ((0, "o"), (1, "w")):
        rho, drho, kr, dkr, mu = pr[ph]
        mob = kr * rho / mu
        dmob_p = kr * drho / mu
        dmob_s = dkr * rho / mu
        rbar = 0.5 * (rho[fc] + rho[fd])
        dphi = (p[fd] - p[fc]) - rbar * g * geo.fdz
        up = np.where(dphi > 0.0, fd, fc)
        T = geo.ft
        dphi_dpc = -1.0 - 0.5 * drho[fc] * g * geo.fdz
        dphi_dpd = 1.0 - 0.5 * drho[fd] * g * geo.fdz
        # F = T mob_up dphi ; R_c -= F ; R_d += F
        dF_dpc = T * mob[up] * dphi_dpc
        dF_dpd = T * mob[up] * dphi_dpd
        dF_dpup = T * dmob_p[up] * dphi
        dF_dsup = T * dmob_s[up] * dphi
        for sign, r in ((-1.0, fc), (1.0, fd)):
            add(2 * r + eq, 2 * fc, sign * dF_dpc)
            add(2 * r + eq, 2 * fd, sign * dF_dpd)
            add(2 * r + eq, 2 * up, sign * dF_dpup)
            add(2 * r + eq, 2 * up + 1, sign * dF_dsup)
        # transfer q = tmf mob_up (p_f - p_m); R_f += q ; R_m -= q
        upm = np.where(p[f] >= p[mm], f, mm)
        dpm = p[f] - p[mm]
        dq_dpf = geo.tmf * mob[upm]
        dq_dpm = -geo.tmf * mob[upm]
        dq_dpup = geo.tmf * dmob_p[upm] * dpm
        dq_dsup = geo.tmf * dmob_s[upm] * dpm
        for sign, r in ((1.0, f), (-1.0, mm)):
            add(2 * r + eq, 2 * f, sign * dq_dpf)
            add(2 * r + eq, 2 * mm, sign * dq_dpm)
            add(2 * r + eq, 2 * upm, sign * dq_dpup)
            add(2 * r + eq, 2 * upm + 1, sign * dq_dsup)
    for w, (cells, wi) in enumerate(geo.perfs):
        wl = m["wells"][w]
        node = 2 * cells
        pf = p[node]
        s = sw[node]
        prw = _phase_props(m, pf, s)
        dp = bhp[w] - pf
        rw_idx = 4 * n + 2 * w
        comps = []
        for eq, ph in ((0, "o"), (1, "w")):
            rho, drho, kr, dkr, mu = prw[ph]
            lam = kr / mu
            comps.append([eq, rho * wi * lam * dp,
                          wi * lam * (drho * dp - rho),
                          rho * wi * (dkr / mu) * dp,
                          rho * wi * lam])
        if wl["kind"] == "inj":
            inj = dp >= 0.0
            rho, drho, krw, dkrw, mu_w = prw["w"]
            _, _, kro, dkro, mu_o = prw["o"]
            lt = krw / mu_w + kro / mu_o
            dlt = dkrw / mu_w + dkro / mu_o
            inj_w = (rho * wi * lt * dp, wi * lt * (drho * dp - rho), rho * wi * dlt * dp, rho * wi * lt)
            for t in range(4):
                comps[1][1 + t] = np.where(inj, inj_w[t], comps[1][1 + t])
                comps[0][1 + t] = np.where(inj, 0.0, comps[0][1 + t])
        for eq, q, dq_dp, dq_ds, dq_db in comps:
            add(2 * node + eq, 2 * node, -dq_dp)
            add(2 * node + eq, 2 * node + 1, -dq_ds)
            add(2 * node + eq, rw_idx, -dq_db)
            if control[w] == "rate" or (control[w] == "orate" and eq == 0):
                add(rw_idx, 2 * node, dq_dp)
                add(rw_idx, 2 * node + 1, dq_ds)
                add(rw_idx, rw_idx, np.sum(dq_db))
        if control[w] == "bhp":
            add(rw_idx, rw_idx, 1.0)
        add(rw_idx + 1, rw_idx + 1, 1.0)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    return sp.csr_matrix((v, (r, c)), shape=(geo.N, geo.N))


# --------------------------------------------------------------------------
# Structural 2x2 block pattern
# --------------------------------------------------------------------------

def block_pattern(geo):
    """The fixed 2x2-block sparsity pattern (block rows = nodes then wells):
    diagonal; fracture-fracture across every interior face (both directions);
    fracture-matrix of each cell (both directions); fracture-well at every
    perforation (both directions).  There is no matrix-matrix coupling."""
    n = geo.n
    nb = 2 * n + geo.nw
    r = [np.arange(nb)]
    c = [np.arange(nb)]
    r += [2 * geo.fc, 2 * geo.fd]
    c += [2 * geo.fd, 2 * geo.fc]
    f = 2 * np.arange(n)
    r += [f, f + 1]
    c += [f + 1, f]
    for w, (cells, _) in enumerate(geo.perfs):
        wb = 2 * n + w
        r += [2 * cells, np.full(cells.shape, wb)]
        c += [np.full(cells.shape, wb), 2 * cells]
    r = np.concatenate(r)
    c = np.concatenate(c)
    key = np.unique(r.astype(np.int64) * nb + c)
    br = key // nb
    bc = key % nb
    indptr = np.zeros(nb + 1, dtype=np.int64)
    np.add.at(indptr, br + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, bc.astype(np.int64)


def to_bsr(geo, J):
    """Values of the point matrix J on the structural block pattern, as
    (indptr, indices, data[nnzb, 2, 2]).  Every entry of J must lie in the pattern."""
    indptr, indices = block_pattern(geo)
    nb = indptr.shape[0] - 1
    rows = np.repeat(np.arange(nb), np.diff(indptr))
    keys = rows * nb + indices
    Jc = J.tocoo()
    ek = (Jc.row // 2).astype(np.int64) * nb + (Jc.col // 2)
    pos = np.searchsorted(keys, ek)
    pos_ok = np.minimum(pos, keys.shape[0] - 1)
    if not np.all(keys[pos_ok] == ek):
        raise ValueError("Jacobian entry outside the block pattern")
    data = np.zeros((indices.shape[0], 2, 2))
    np.add.at(data, (pos, Jc.row % 2, Jc.col % 2), Jc.data)
    return indptr, indices, data


def bsr_to_csr(indptr, indices, data):
    nb = indptr.shape[0] - 1
    return sp.bsr_matrix((data, indices, indptr), shape=(2 * nb, 2 * nb)).tocsr()
