"""Oracle nonlinear solver: Newton's method with a direct sparse solve, the
timestep loop and the material-balance report.

Part of the CPU oracle (test infrastructure only; see the package docstring).

Algorithm 1 (inexact Newton): the linear system J y = -R is solved by SuperLU
(``linear='lu'``) or by the oracle's own decoupled CPR-FPF GMRES
(``linear='cpr'``) to the relative tolerance eta_l of Eq. (12).  eta_l is fixed
(``forcing=0``, eta_l = ``eta``) or one of the three adaptive choices of
Eq. (13) (``forcing=1, 2, 3``, see ``forcing_term``).

Readings (the paper does not state them): the update chops the saturation
change of each node to at most 0.2 per iteration, stops it at the
relative-permeability end points it would cross, and clamps S_w to [0, 1];
BHP-controlled wells have p_b pinned to the target after every update;
convergence is the scaled max-norm (CNV) together with the material-balance
measure (MB) below; at most ``max_newton``
iterations, then the step is cut in half (at most ``max_cuts`` times).  The
sub-step also fails early when ``stall`` iterations in a row have not lowered
the smallest CNV its updated iterates have reached (a stagnating or
oscillating Newton iteration; off unless ``stall`` > 0).  After a
converged step a rate injector whose p_b exceeds its limit switches to BHP
control at the limit and the step is repeated (at most once per step).
"""
import warnings

import numpy as np
import scipy.sparse.linalg as spla

from . import physics as ph

SAT_CHOP = 0.2


def scaled_residual_norm(geo, R, dt, control):
    """max over rows of |R| scaled to a dimensionless size.

    Node rows: |R_a| dt / (rho_a,ref phi V) (a pore-volume fraction per step).
    Rate rows: |R| / (rho_w,ref max(|Q|, 1e-6 m^3/s)); oil-rate rows the same
    with rho_o,ref.  BHP rows: |R| / target.  (Reference porosity throughout.)
    """
    m = geo.m
    n = geo.n
    vphi = geo.vol * geo.phi
    so = np.abs(R[0:4 * n:2]) * dt / (m["rho_o_ref"] * vphi)
    sw = np.abs(R[1:4 * n:2]) * dt / (m["rho_w_ref"] * vphi)
    worst = max(so.max(initial=0.0), sw.max(initial=0.0))
    for w, wl in enumerate(m["wells"]):
        r = abs(R[4 * n + 2 * w])
        if control[w] == "rate":
            worst = max(worst, r / (m["rho_w_ref"] * max(abs(wl["target"]), 1e-6)))
        elif control[w] == "orate":
            worst = max(worst, r / (m["rho_o_ref"] * max(abs(wl["target"]), 1e-6)))
        else:
            target = wl["target"] if wl["control"] == "bhp" else wl["bhp_limit"]
            worst = max(worst, r / max(abs(target), 1.0))
    return worst


def material_balance_norm(geo, R, dt):
    """max over phases of |sum over nodes of R_a| dt / sum over nodes (rho_a,ref phi V)."""
    m = geo.m
    n = geo.n
    pv = np.sum(geo.vol * geo.phi)
    mo = abs(np.sum(R[0:4 * n:2])) * dt / (m["rho_o_ref"] * pv)
    mw = abs(np.sum(R[1:4 * n:2])) * dt / (m["rho_w_ref"] * pv)
    return max(mo, mw)


def apply_update(geo, x, dx, control):
    """x + dx with the saturation chop, the end-point stops and the clamp, and
    BHP pinning.  A saturation change is limited to +-0.2; an update that
    crosses S_wc from above stops at S_wc and one that crosses 1 - S_or from
    below stops at 1 - S_or (the kinks of the relative permeabilities); the
    result is clamped to [0, 1]."""
    n = geo.n
    m = geo.m
    y = x + dx
    s0 = x[1:4 * n:2]
    s1 = s0 + np.clip(dx[1:4 * n:2], -SAT_CHOP, SAT_CHOP)
    lo, hi = m["swc"], 1.0 - m["sor"]
    s1 = np.where((s0 > lo) & (s1 < lo), lo, s1)
    s1 = np.where((s0 < hi) & (s1 > hi), hi, s1)
    y[1:4 * n:2] = np.clip(s1, 0.0, 1.0)
    for w, wl in enumerate(m["wells"]):
        if control[w] == "bhp":
            y[4 * n + 2 * w] = wl["target"] if wl["control"] == "bhp" else wl["bhp_limit"]
        y[4 * n + 2 * w + 1] = 0.0
    return y


GOLDEN = (1.0 + 5.0 ** 0.5) / 2.0


def forcing_term(choice, eta_prev, nb, nb_prev, nr_prev, nd, gamma=0.9, beta=2.0, eta_max=0.9,
                 eta_min=1e-8):
    """Adaptive forcing term eta_l of Eq. (13) for l >= 1.

    nb = ||b(x^l)||, nb_prev = ||b(x^{l-1})||, nr_prev = ||r^{l-1}|| with
    r^{l-1} = b(x^{l-1}) - J(x^{l-1}) y^{l-1} the linear residual of the previous
    iteration, nd = ||b(x^l) - r^{l-1}|| (2-norms of the undecoupled Newton
    right-hand side b = -R).  Choice 1: nd / nb_prev; choice 2: |nb - nr_prev| /
    nb_prev (the absolute value the printed formula lacks, by reading); choice
    3: gamma (nb / nb_prev)^beta.  Safeguards (by reading, Eisenstat and
    Walker's): choices 1-2 take max(eta, eta_prev^phi) when eta_prev^phi > 0.1,
    phi the golden ratio; choice 3 takes max(eta, gamma eta_prev^beta) when that
    exceeds 0.1; finally eta is clamped to [eta_min, eta_max]."""
    if choice == 1:
        eta = nd / nb_prev
        guard = eta_prev ** GOLDEN
    elif choice == 2:
        eta = abs(nb - nr_prev) / nb_prev
        guard = eta_prev ** GOLDEN
    elif choice == 3:
        eta = gamma * (nb / nb_prev) ** beta
        guard = gamma * eta_prev ** beta
    else:
        raise ValueError("forcing choice must be 1, 2 or 3")
    if guard > 0.1:
        eta = max(eta, guard)
    return min(max(eta, eta_min), eta_max)


def newton_solve(geo, x0, acc_old, dt, control, tol=1e-10, max_newton=20,
                 linear="lu", eta=1e-10, cpr_opts=None, mb_tol=1e-7, forcing=0, eta0=0.1,
                 forcing_opts=None, stall=0):
    """Newton iterations from x0.  Converged when the scaled max-norm (CNV) is at
    most tol and the material-balance measure at most mb_tol.  Not converged
    after max_newton iterations, or when ``stall`` iterations in a row have not
    gone below the smallest CNV of the earlier updated iterates (iterations
    1..l-1; iteration 0 is the start state, the previous step's solution).  With forcing 1-3
    the first linear tolerance is eta0 and the later ones follow Eq. (13).
    Returns (x, converged, iterations, info); info["eta"] lists the tolerances."""
    x = x0.copy()
    info = {"res": [], "lin_iters": [], "eta": []}
    prev = None  # (eta, ||b||, ||r||, r) of the previous iteration
    best, best_it = np.inf, 0  # smallest CNV so far and the iteration that reached it
    for it in range(max_newton + 1):
        R = ph.residual(geo, x, acc_old, dt, control)
        nrm = scaled_residual_norm(geo, R, dt, control)
        info["res"].append(nrm)
        if not np.isfinite(nrm):
            return x, False, it, info
        if nrm <= tol and material_balance_norm(geo, R, dt) <= mb_tol:
            return x, True, it, info
        if it == max_newton:
            break
        if it >= 1:  # only iterates produced by an update count (x0 solved the previous step)
            if nrm < best:
                best, best_it = nrm, it
            elif stall > 0 and it - best_it >= stall:
                return x, False, it, info
        J = ph.jacobian(geo, x, dt, control)
        b = -R
        if forcing:
            nb = float(np.linalg.norm(b))
            if prev is None:
                eta = eta0
            else:
                e_prev, nb_prev, nr_prev, r_prev = prev
                nd = float(np.linalg.norm(b - r_prev))
                eta = forcing_term(forcing, e_prev, nb, nb_prev, nr_prev, nd, **(forcing_opts or {}))
        info["eta"].append(eta)
        # a singular or numerically failed linear stage counts as a failed iteration
        try:
            if linear == "lu":
                with np.errstate(all="ignore"), warnings.catch_warnings():
                    warnings.simplefilter("ignore", spla.MatrixRankWarning)
                    dx = spla.spsolve(J.tocsc(), -R)
                info["lin_iters"].append(1)
            else:
                from . import cpr
                dx, its, _ = cpr.solve(geo, J, -R, rtol=eta, **(cpr_opts or {}))
                info["lin_iters"].append(its)
        except np.linalg.LinAlgError:
            return x, False, it, info
        if not np.all(np.isfinite(dx)):
            return x, False, it, info
        if forcing:
            r = b - J @ dx
            prev = (eta, nb, float(np.linalg.norm(r)), r)
        x = apply_update(geo, x, dx, control)
    return x, False, max_newton, info


def well_totals(geo, x, control):
    """Total well mass rates (oil, water), positive into the reservoir."""
    qo = qw = 0.0
    for _, q_o, q_w in ph.well_rates(geo, x, control):
        qo += float(np.sum(q_o))
        qw += float(np.sum(q_w))
    return qo, qw


def _rel(err, mass):
    return abs(err) / mass if mass > 0.0 else abs(err)


def timestep(geo, x, dt, control, max_cuts=8, **newton_kw):
    """Advance by dt (possibly in several cut sub-steps).  A failed sub-step is
    retried at half length; after an accepted one the length doubles again
    (never beyond what remains of dt).

    Returns (x_new, report) where report lists every accepted sub-step with its
    material balance |M^{n+1} - M^n - dt Q(x^{n+1})| / M^{n+1} per phase."""
    report = []
    remaining = dt
    cuts = 0
    h = dt
    control = list(control)
    while remaining > 0.0:
        h = min(h, remaining)
        acc_old = ph.accumulation(geo, x)
        switched = False
        while True:
            xn, ok, its, info = newton_solve(geo, x, acc_old, h, control, **newton_kw)
            if not ok:
                break
            # BHP limits of rate-controlled wells (an injector's maximum, a
            # producer's minimum): switch once and redo
            redo = False
            if not switched:
                _, _, bhp = ph.unpack_state(xn, geo.n)
                for w, wl in enumerate(geo.m["wells"]):
                    over = control[w] == "rate" and wl["kind"] == "inj" and bhp[w] > wl["bhp_limit"]
                    under = control[w] == "orate" and wl["kind"] == "prod" and bhp[w] < wl["bhp_limit"]
                    if over or under:
                        control[w] = "bhp"
                        redo = True
            if redo:
                switched = True
                continue
            break
        if not ok:
            cuts += 1
            if cuts > max_cuts:
                raise RuntimeError("timestep failed after %d cuts" % max_cuts)
            h *= 0.5
            continue
        acc_new = ph.accumulation(geo, xn)
        qo, qw = well_totals(geo, xn, control)
        mo_old, mw_old = float(np.sum(acc_old[0])), float(np.sum(acc_old[1]))
        mo_new, mw_new = float(np.sum(acc_new[0])), float(np.sum(acc_new[1]))
        report.append(dict(dt=h, newton=its, lin_iters=info["lin_iters"],
                           res=info["res"], eta=info["eta"],
                           mb_oil=_rel(mo_new - mo_old - h * qo, mo_new),
                           mb_water=_rel(mw_new - mw_old - h * qw, mw_new),
                           control=list(control)))
        x = xn
        remaining -= h
        h *= 2.0  # after an accepted sub-step the next may be twice as long
    return x, report, control


def run(model, steps=None, **kw):
    """Run the model's schedule; returns (states after each step, reports)."""
    geo = ph.Geometry(model)
    x = ph.initial_state(model)
    control = [w["control"] for w in model["wells"]]
    states, reports = [], []
    sched = model["schedule"] if steps is None else model["schedule"][:steps]
    for dt in sched:
        x, rep, control = timestep(geo, x, dt, control, **kw)
        states.append(x.copy())
        reports.append(rep)
    return geo, states, reports
