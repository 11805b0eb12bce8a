// Device-side rock/fluid properties and the flux terms of the dual-porosity
// oil-water system (paper Sec. 2, Eqs. (3)-(7)).  Phase index 0 = oil, 1 = water.
#pragma once

#include "common.h"

namespace dp {

struct Phys {
    double rho_ref[2], c[2], mu[2];
    double p_ref, swc, sor, n_w, n_o, krw_max, kro_max, g, dz;
    double c_r;  // rock compressibility: phi(p) = phi_ref (1 + c_r (p - p_ref))
};

// Per-node properties: densities rho = rho_ref exp(c (p - p_ref)), Corey relative
// permeabilities, phase mass mobilities k_r rho / mu and their derivatives.
struct Props {
    double rho[2], drho[2];
    double kr[2], dkr[2];     // d k_r / d S_w
    double mob[2], dmob_p[2], dmob_s[2];
};

__device__ inline double ipow_or_pow(double s, double e) {
    if (e == 2.0) return s * s;
    if (e == 1.0) return s;
    if (e == 3.0) return s * s * s;
    return pow(s, e);
}

__device__ inline Props props(const Phys& P, double p, double sw) {
    Props r;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        r.rho[a] = P.rho_ref[a] * exp(P.c[a] * (p - P.p_ref));
        r.drho[a] = P.c[a] * r.rho[a];
    }
    // s* = clip((S_w - S_wc)/(1 - S_wc - S_or), 0, 1); slope on the closed interval
    double delta = 1.0 - P.swc - P.sor;
    double raw = (sw - P.swc) / delta;
    double s = raw < 0.0 ? 0.0 : (raw > 1.0 ? 1.0 : raw);
    double ds = (raw >= 0.0 && raw <= 1.0) ? 1.0 / delta : 0.0;
    double so = 1.0 - s;
    r.kr[1] = P.krw_max * ipow_or_pow(s, P.n_w);
    r.kr[0] = P.kro_max * ipow_or_pow(so, P.n_o);
    r.dkr[1] = P.krw_max * P.n_w * ipow_or_pow(s, P.n_w - 1.0) * ds;
    r.dkr[0] = -P.kro_max * P.n_o * ipow_or_pow(so, P.n_o - 1.0) * ds;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        r.mob[a] = r.kr[a] * r.rho[a] / P.mu[a];
        r.dmob_p[a] = r.kr[a] * r.drho[a] / P.mu[a];
        r.dmob_s[a] = r.dkr[a] * r.rho[a] / P.mu[a];
    }
    return r;
}

// Two-point flux across one fracture face, oriented from the lower-index cell
// "lo" to the higher-index cell "hi": F_a = T (k_ra rho_a/mu_a)_up (Phi_hi - Phi_lo)
// is the mass rate into lo from hi.  Phi_a = p - rho_bar_a g z with rho_bar the
// mean of the two densities; upstream = hi if Phi_hi > Phi_lo, else lo.
// dzf = z_hi - z_lo.  Both cells evaluate this with identical operands, so the
// two sides of a face see bitwise-equal fluxes.
struct FaceFlux {
    double F[2];
    double dplo[2], dphi[2], dslo[2], dshi[2];
};

__device__ inline FaceFlux face_flux(const Phys& P, double T, double dzf, double plo,
                                     const Props& lo, double phi, const Props& hi) {
    FaceFlux f;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        double rbar = 0.5 * (lo.rho[a] + hi.rho[a]);
        double dpot = (phi - plo) - rbar * P.g * dzf;
        bool up_hi = dpot > 0.0;
        double mob = up_hi ? hi.mob[a] : lo.mob[a];
        double tm = T * mob;
        f.F[a] = tm * dpot;
        double dd_lo = -1.0 - 0.5 * lo.drho[a] * P.g * dzf;
        double dd_hi = 1.0 - 0.5 * hi.drho[a] * P.g * dzf;
        f.dplo[a] = tm * dd_lo + (up_hi ? 0.0 : T * lo.dmob_p[a] * dpot);
        f.dphi[a] = tm * dd_hi + (up_hi ? T * hi.dmob_p[a] * dpot : 0.0);
        f.dslo[a] = up_hi ? 0.0 : T * lo.dmob_s[a] * dpot;
        f.dshi[a] = up_hi ? T * hi.dmob_s[a] * dpot : 0.0;
    }
    return f;
}

// Matrix-fracture transfer q_a = omega (k_ra rho_a/mu_a)_up (p_f - p_m), the rate
// from the fracture node into the matrix node; upstream = f if p_f >= p_m.
struct Transfer {
    double q[2];
    double dpf[2], dpm[2], dsf[2], dsm[2];
};

__device__ inline Transfer transfer(double tmf, double pf, const Props& f, double pm,
                                    const Props& m) {
    Transfer t;
    bool up_f = pf >= pm;
    double dp = pf - pm;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        double mob = up_f ? f.mob[a] : m.mob[a];
        double tm = tmf * mob;
        t.q[a] = tm * dp;
        double dup_p = tmf * (up_f ? f.dmob_p[a] : m.dmob_p[a]) * dp;
        double dup_s = tmf * (up_f ? f.dmob_s[a] : m.dmob_s[a]) * dp;
        t.dpf[a] = tm + (up_f ? dup_p : 0.0);
        t.dpm[a] = -tm + (up_f ? 0.0 : dup_p);
        t.dsf[a] = up_f ? dup_s : 0.0;
        t.dsm[a] = up_f ? 0.0 : dup_s;
    }
    return t;
}

// Perforation mass rate into the fracture node (Eq. (6)), mobility from the
// upstream side: an injecting perforation of a water injector (p_b >= p) gives
// q_w = rho_w W lambda_t (p_b - p), q_o = 0; a producer, or an injector's
// perforation in back-flow, gives q_a = rho_a W lambda_a (p_b - p).
struct Perf {
    double q[2];
    double dp[2], ds[2], db[2];
};

__device__ inline Perf perf_rate(const Phys& P, int kind, double wi, double pb, double p,
                                 const Props& pr) {
    Perf r;
    double dpb = pb - p;
    if (kind == DP_WELL_INJ && dpb >= 0.0) {
        double lt = pr.kr[1] / P.mu[1] + pr.kr[0] / P.mu[0];
        double dlt = pr.dkr[1] / P.mu[1] + pr.dkr[0] / P.mu[0];
        double rho = pr.rho[1];
        r.q[0] = 0.0;
        r.dp[0] = r.ds[0] = r.db[0] = 0.0;
        r.q[1] = rho * wi * lt * dpb;
        r.dp[1] = wi * lt * (pr.drho[1] * dpb - rho);
        r.ds[1] = rho * wi * dlt * dpb;
        r.db[1] = rho * wi * lt;
    } else {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            double lam = pr.kr[a] / P.mu[a];
            double rho = pr.rho[a];
            r.q[a] = rho * wi * lam * dpb;
            r.dp[a] = wi * lam * (pr.drho[a] * dpb - rho);
            r.ds[a] = rho * wi * (pr.dkr[a] / P.mu[a]) * dpb;
            r.db[a] = rho * wi * lam;
        }
    }
    return r;
}

}  // namespace dp
