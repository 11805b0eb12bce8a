// Residual and Jacobian assembly of the dual-porosity system, geometry
// precomputation, accumulation, the scaled residual norm and the Newton update.
//
// One thread per node row (matrix rows, then fracture rows) and one block per
// well row.  Every thread writes only its own row: no atomics, deterministic.
#include "kernels.h"
#include "physics.h"

namespace dp {

// ---------------------------------------------------------------------------
// Geometry (state independent), computed once at create
// ---------------------------------------------------------------------------
struct GeoIn {
    const double *kx, *ky, *kz, *km, *phi_f, *phi_m;
    double dx, dy, dz, top_depth, sigma;
    int nx, ny, n;
};

// Transmissibility of each fracture slot (harmonic two-point form
// T = 2 A k_lo k_hi / (L (k_lo + k_hi))), transfer coefficient sigma km V,
// pore volumes V phi and depths.  The input fields are in grid-cell order
// (cell[q] is the cell of node pair q); the outputs are indexed by q.
__global__ void geometry_kernel(GeoIn g, const int* __restrict__ fcol, const int* __restrict__ cell,
                                const unsigned char* __restrict__ fmask, int n, double* tface,
                                double* tmf, double* pvf, double* pvm, double* depth) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int c = cell[q];
    double vol = g.dx * g.dy * g.dz;
    int k = c / (g.nx * g.ny);
    for (int s = 0; s < 6; ++s) {
        double t = 0.0;
        if (fmask[q] & (1u << s)) {
            int d = cell[fcol[s * n + q] - n];
            int lo = (s & 1) ? c : d;
            int hi = (s & 1) ? d : c;
            const double* kk = s < 2 ? g.kx : (s < 4 ? g.ky : g.kz);
            double area = s < 2 ? g.dy * g.dz : (s < 4 ? g.dx * g.dz : g.dx * g.dy);
            double len = s < 2 ? g.dx : (s < 4 ? g.dy : g.dz);
            t = 2.0 * area * kk[lo] * kk[hi] / (len * (kk[lo] + kk[hi]));
        }
        tface[s * n + q] = t;
    }
    tmf[q] = g.sigma * g.km[c] * vol;
    pvf[q] = vol * g.phi_f[c];
    pvm[q] = vol * g.phi_m[c];
    depth[q] = g.top_depth + k * g.dz;
}

// Peaceman well index of every perforation: W = 2 pi sqrt(kx ky) dz / (ln(r_e/r_w) + s),
// or the well's own index where it gives one (perf_wi > 0).
__global__ void well_index_kernel(const double* __restrict__ kx, const double* __restrict__ ky,
                                  const int* __restrict__ perf_cell, const double* __restrict__ perf_rw,
                                  const double* __restrict__ perf_skin,
                                  const double* __restrict__ perf_wi, int nperf, double dx,
                                  double dy, double dz, double* wi) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nperf) return;
    if (perf_wi[p] > 0.0) {
        wi[p] = perf_wi[p];
        return;
    }
    int c = perf_cell[p];
    double ryx = sqrt(ky[c] / kx[c]);
    double rxy = sqrt(kx[c] / ky[c]);
    double num = sqrt(dx * dx * ryx + dy * dy * rxy);
    double den = sqrt(ryx) + sqrt(rxy);
    double re = 0.28 * num / den;
    double kh = sqrt(kx[c] * ky[c]) * dz;
    wi[p] = 2.0 * M_PI * kh / (log(re / perf_rw[p]) + perf_skin[p]);
}

void launch_geometry(dp_sim* s, const double* kx, const double* ky, const double* kz,
                     const double* km, const double* phi_f, const double* phi_m,
                     const int* perf_cell, const double* perf_rw, const double* perf_skin,
                     const double* perf_wi) {
    Topo& t = s->topo;
    GeoIn g{kx, ky, kz, km, phi_f, phi_m, s->desc.dx, s->desc.dy, s->desc.dz,
            s->desc.top_depth, s->desc.sigma, t.nx, t.ny, t.n};
    geometry_kernel<<<ceil_div(t.n, 256), 256, 0, s->stream>>>(g, t.fcol, t.cell, t.fmask, t.n,
                                                               t.tface, t.tmf, t.pvf, t.pvm, t.depth);
    DP_LAUNCH_CHECK();
    if (t.nperf > 0) {
        well_index_kernel<<<ceil_div(t.nperf, 256), 256, 0, s->stream>>>(
            kx, ky, perf_cell, perf_rw, perf_skin, perf_wi, t.nperf, s->desc.dx, s->desc.dy, s->desc.dz,
            t.wi);
        DP_LAUNCH_CHECK();
    }
}

Phys make_phys(const dp_sim* s) {
    Phys P;
    P.rho_ref[0] = s->rho_o_ref;
    P.rho_ref[1] = s->rho_w_ref;
    P.c[0] = s->c_o;
    P.c[1] = s->c_w;
    P.mu[0] = s->mu_o;
    P.mu[1] = s->mu_w;
    P.p_ref = s->p_ref;
    P.swc = s->swc;
    P.sor = s->sor;
    P.n_w = s->n_w;
    P.n_o = s->n_o;
    P.krw_max = s->krw_max;
    P.kro_max = s->kro_max;
    P.g = s->gravity;
    P.dz = s->dz;
    P.c_r = s->c_r;
    return P;
}

// ---------------------------------------------------------------------------
// Accumulation M = V phi(p) (S rho) per node, at the start of a step
// ---------------------------------------------------------------------------
__global__ void accumulation_kernel(Phys P, const d2* __restrict__ x, const double* __restrict__ pvf,
                                    const double* __restrict__ pvm, int n, d2* acc) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= 2 * n) return;
    double pv = r < n ? pvm[r] : pvf[r - n];
    d2 v = x[r];
    double rho_o = P.rho_ref[0] * exp(P.c[0] * (v.x - P.p_ref));
    double rho_w = P.rho_ref[1] * exp(P.c[1] * (v.x - P.p_ref));
    double pvp = pv * (1.0 + P.c_r * (v.x - P.p_ref));
    acc[r] = mk2(pvp * (1.0 - v.y) * rho_o, pvp * v.y * rho_w);
}

void launch_accumulation(dp_sim* s, const d2* x, d2* acc) {
    Topo& t = s->topo;
    accumulation_kernel<<<ceil_div(2 * t.n, 256), 256, 0, s->stream>>>(make_phys(s), x, t.pvf, t.pvm,
                                                                       t.n, acc);
    DP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Assembly
// ---------------------------------------------------------------------------
struct AsmArgs {
    Phys P;
    double dt;
    const d2* x;
    const d2* acc_old;
    const int* fcol;
    const unsigned char* fmask;
    const int* fperf;
    const int* perf_q;
    const int* perf_well;
    const int* well_ptr;
    const int* well_kind;
    const int* well_ctrl;
    const double* well_target;
    const double* tface;
    const double* tmf;
    const double* pvf;
    const double* pvm;
    const double* wi;
    int n, nw;
    BMat<double> J;
    d2* R;
};

// Accumulation terms of one node row: residual (M - M^n)/dt and diagonal block,
// pv = V phi_ref and the pore volume V phi(p) = pv (1 + c_r (p - p_ref)).
__device__ inline void accum_row(const Phys& P, double pv, double dt, double p, double s,
                                 const Props& pr, d2 old, double R[2], double D[2][2]) {
    double pvp = pv * (1.0 + P.c_r * (p - P.p_ref));
    double dpv = pv * P.c_r;
    double mo = pvp * (1.0 - s) * pr.rho[0];
    double mw = pvp * s * pr.rho[1];
    R[0] = (mo - old.x) / dt;
    R[1] = (mw - old.y) / dt;
    D[0][0] = (1.0 - s) * (pvp * pr.drho[0] + dpv * pr.rho[0]) / dt;
    D[0][1] = -pvp * pr.rho[0] / dt;
    D[1][0] = s * (pvp * pr.drho[1] + dpv * pr.rho[1]) / dt;
    D[1][1] = pvp * pr.rho[1] / dt;
}

// Matrix row c: accumulation minus the transfer from its fracture node n + c.
__device__ void assemble_matrix_row(const AsmArgs& a, int c) {
    const Phys& P = a.P;
    int n = a.n;
    int fpos = n + c;
    d2 xm = a.x[c];
    d2 xf = a.x[fpos];
    Props pm = props(P, xm.x, xm.y);
    Props pf = props(P, xf.x, xf.y);
    double R[2], D[2][2];
    accum_row(P, a.pvm[c], a.dt, xm.x, xm.y, pm, a.acc_old[c], R, D);
    Transfer t = transfer(a.tmf[c], xf.x, pf, xm.x, pm);
    double O[2][2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        R[e] -= t.q[e];
        D[e][0] -= t.dpm[e];
        D[e][1] -= t.dsm[e];
        O[e][0] = -t.dpf[e];
        O[e][1] = -t.dsf[e];
    }
    a.R[c] = mk2(R[0], R[1]);
    a.J.d0[c] = mk2(D[0][0], D[0][1]);
    a.J.d1[c] = mk2(D[1][0], D[1][1]);
    a.J.m0[c] = mk2(O[0][0], O[0][1]);
    a.J.m1[c] = mk2(O[1][0], O[1][1]);
}

// Fracture row q: accumulation, the six faces, the transfer to the matrix node
// and the perforation term.
__device__ void assemble_fracture_row(const AsmArgs& a, int q) {
    const Phys& P = a.P;
    int n = a.n;
    int c = q;  // its matrix node
    int pos = n + q;
    d2 xf = a.x[pos];
    Props pf = props(P, xf.x, xf.y);
    double R[2], D[2][2];
    accum_row(P, a.pvf[c], a.dt, xf.x, xf.y, pf, a.acc_old[pos], R, D);
    unsigned mask = a.fmask[q];
#pragma unroll 1
    for (int s = 0; s < 6; ++s) {
        double O[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        if (mask & (1u << s)) {
            int dpos = a.fcol[s * n + q];
            d2 xd = a.x[dpos];
            Props pd = props(P, xd.x, xd.y);
            double T = a.tface[s * n + q];
            double dzf = (s >= 4) ? P.dz : 0.0;
            bool c_is_lo = (s & 1) != 0;  // + slots point at the higher index
            FaceFlux f = c_is_lo ? face_flux(P, T, dzf, xf.x, pf, xd.x, pd)
                                 : face_flux(P, T, dzf, xd.x, pd, xf.x, pf);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (c_is_lo) {  // R_lo -= F
                    R[e] -= f.F[e];
                    D[e][0] -= f.dplo[e];
                    D[e][1] -= f.dslo[e];
                    O[e][0] = -f.dphi[e];
                    O[e][1] = -f.dshi[e];
                } else {  // R_hi += F
                    R[e] += f.F[e];
                    D[e][0] += f.dphi[e];
                    D[e][1] += f.dshi[e];
                    O[e][0] = f.dplo[e];
                    O[e][1] = f.dslo[e];
                }
            }
        }
        a.J.f0[s * n + q] = mk2(O[0][0], O[0][1]);
        a.J.f1[s * n + q] = mk2(O[1][0], O[1][1]);
    }
    {
        d2 xm = a.x[c];
        Props pm = props(P, xm.x, xm.y);
        Transfer t = transfer(a.tmf[c], xf.x, pf, xm.x, pm);
        double O[2][2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            R[e] += t.q[e];
            D[e][0] += t.dpf[e];
            D[e][1] += t.dsf[e];
            O[e][0] = t.dpm[e];
            O[e][1] = t.dsm[e];
        }
        a.J.f0[6 * n + q] = mk2(O[0][0], O[0][1]);
        a.J.f1[6 * n + q] = mk2(O[1][0], O[1][1]);
    }
    int p = a.fperf[q];
    if (p >= 0) {
        int w = a.perf_well[p];
        double pb = a.x[2 * n + w].x;
        Perf r = perf_rate(P, a.well_kind[w], a.wi[p], pb, xf.x, pf);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            R[e] -= r.q[e];
            D[e][0] -= r.dp[e];
            D[e][1] -= r.ds[e];
        }
        a.J.fw0[p] = mk2(-r.db[0], 0.0);
        a.J.fw1[p] = mk2(-r.db[1], 0.0);
    }
    a.R[pos] = mk2(R[0], R[1]);
    a.J.d0[pos] = mk2(D[0][0], D[0][1]);
    a.J.d1[pos] = mk2(D[1][0], D[1][1]);
}

// Well row w (one block): rate control sum_p (q_o,p + q_w,p) - rho_w,ref Q = 0
// (the net mass rate; the water rate while every perforation injects), oil-rate
// control sum_p q_o,p + rho_o,ref Q = 0 (a producer's oil mass rate), or BHP
// control p_b - target = 0; second row: dummy = 0.  The perforation sum is
// reduced in a fixed order.
__device__ void assemble_well_row(const AsmArgs& a, int w) {
    __shared__ double sh_q[256 / WAVE], sh_db[256 / WAVE];
    const Phys& P = a.P;
    int n = a.n;
    const int ctrl = a.well_ctrl[w];
    const bool rate = ctrl == DP_CTRL_RATE, orate = ctrl == DP_CTRL_ORATE;
    d2 xw = a.x[2 * n + w];
    double q = 0.0, db = 0.0;
    for (int p = a.well_ptr[w] + threadIdx.x; p < a.well_ptr[w + 1]; p += blockDim.x) {
        int pos = n + a.perf_q[p];
        d2 xf = a.x[pos];
        Props pf = props(P, xf.x, xf.y);
        Perf r = perf_rate(P, a.well_kind[w], a.wi[p], xw.x, xf.x, pf);
        if (orate) {
            q += r.q[0];
            db += r.db[0];
            a.J.wf0[p] = mk2(r.dp[0], r.ds[0]);
        } else if (rate) {
            q += r.q[0] + r.q[1];
            db += r.db[0] + r.db[1];
            a.J.wf0[p] = mk2(r.dp[0] + r.dp[1], r.ds[0] + r.ds[1]);
        } else {
            a.J.wf0[p] = mk2(0.0, 0.0);
        }
        a.J.wf1[p] = mk2(0.0, 0.0);
    }
    q = wave_sum(q);
    db = wave_sum(db);
    int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    if (lane == 0) {
        sh_q[wv] = q;
        sh_db[wv] = db;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double qs = 0.0, dbs = 0.0;
        for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) {
            qs += sh_q[i];
            dbs += sh_db[i];
        }
        int pos = 2 * n + w;
        double r0, d00;
        if (rate) {
            r0 = qs - P.rho_ref[1] * a.well_target[w];
            d00 = dbs;
        } else if (orate) {
            r0 = qs + P.rho_ref[0] * a.well_target[w];
            d00 = dbs;
        } else {
            r0 = xw.x - a.well_target[w];
            d00 = 1.0;
        }
        a.R[pos] = mk2(r0, xw.y);
        a.J.d0[pos] = mk2(d00, 0.0);
        a.J.d1[pos] = mk2(0.0, 1.0);
    }
}

__global__ void __launch_bounds__(256) assemble_kernel(AsmArgs a, int blocks_m, int blocks_f) {
    int b = blockIdx.x;
    if (b < blocks_m) {
        int c = b * blockDim.x + threadIdx.x;
        if (c < a.n) assemble_matrix_row(a, c);
    } else if (b < blocks_m + blocks_f) {
        int q = (b - blocks_m) * blockDim.x + threadIdx.x;
        if (q < a.n) assemble_fracture_row(a, q);
    } else {
        assemble_well_row(a, b - blocks_m - blocks_f);
    }
}

void launch_assemble(dp_sim* s, double dt) {
    Topo& t = s->topo;
    AsmArgs a;
    a.P = make_phys(s);
    a.dt = dt;
    a.x = s->x;
    a.acc_old = s->acc_old;
    a.fcol = t.fcol;
    a.fmask = t.fmask;
    a.fperf = t.fperf;
    a.perf_q = t.perf_q;
    a.perf_well = t.perf_well;
    a.well_ptr = t.well_ptr;
    a.well_kind = t.well_kind;
    a.well_ctrl = t.well_ctrl;
    a.well_target = t.well_target;
    a.tface = t.tface;
    a.tmf = t.tmf;
    a.pvf = t.pvf;
    a.pvm = t.pvm;
    a.wi = t.wi;
    a.n = t.n;
    a.nw = t.nw;
    a.J = s->J;
    a.R = s->res;
    int bm = ceil_div(t.n, 256);
    assemble_kernel<<<2 * bm + t.nw, 256, 0, s->stream>>>(a, bm, bm);
    DP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Convergence measures of the residual:
//   CNV = max over node rows of |R_a| dt / (rho_a,ref V phi), control rows |R| *
//         well_scale (NaN counts as +inf)
//   sums over node rows of R_o and R_w (for the material-balance measure)
// Block partials (grid-stride loop, fixed order), then one block combines them
// in block order in a second kernel (the kernel boundary orders the partials).
// ---------------------------------------------------------------------------
constexpr int RN_BLOCKS = 1024;

__global__ void resnorm_kernel(const d2* __restrict__ R, const double* __restrict__ pvf,
                               const double* __restrict__ pvm, const double* __restrict__ well_scale, int n, int nw, double dt,
                               double rho_o, double rho_w, double* part) {
    __shared__ double sh[3][256 / WAVE];
    double v = 0.0, so = 0.0, sw = 0.0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < 2 * n + nw; r += gridDim.x * blockDim.x) {
        if (r < 2 * n) {
            double pv = r < n ? pvm[r] : pvf[r - n];
            d2 x = R[r];
            double a = fabs(x.x) * dt / (rho_o * pv);
            double b = fabs(x.y) * dt / (rho_w * pv);
            double c = fmax(a, b);
            if (!(a == a) || !(b == b)) c = INFINITY;
            v = fmax(v, c);
            so += x.x;
            sw += x.y;
        } else {
            double a = fabs(R[r].x) * well_scale[r - 2 * n];
            v = fmax(v, (a == a) ? a : INFINITY);
        }
    }
    v = wave_max(v);
    so = wave_sum(so);
    sw = wave_sum(sw);
    if (threadIdx.x % WAVE == 0) {
        sh[0][threadIdx.x / WAVE] = v;
        sh[1][threadIdx.x / WAVE] = so;
        sh[2][threadIdx.x / WAVE] = sw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, a = 0.0, b = 0.0;
        for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) {
            m = fmax(m, sh[0][i]);
            a += sh[1][i];
            b += sh[2][i];
        }
        part[3 * (int64_t)blockIdx.x] = m;
        part[3 * (int64_t)blockIdx.x + 1] = a;
        part[3 * (int64_t)blockIdx.x + 2] = b;
    }
}

__global__ void resnorm_final(const double* __restrict__ part, int nblk, double* out) {
    __shared__ double sh[3][256 / WAVE];
    double m = 0.0, a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        m = fmax(m, part[3 * (int64_t)i]);
        a += part[3 * (int64_t)i + 1];
        b += part[3 * (int64_t)i + 2];
    }
    m = wave_max(m);
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x % WAVE == 0) {
        sh[0][threadIdx.x / WAVE] = m;
        sh[1][threadIdx.x / WAVE] = a;
        sh[2][threadIdx.x / WAVE] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = 0.0, aa = 0.0, bb = 0.0;
        for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) {
            mm = fmax(mm, sh[0][i]);
            aa += sh[1][i];
            bb += sh[2][i];
        }
        out[0] = mm;
        out[1] = aa;
        out[2] = bb;
    }
}

ResNorm residual_norm(dp_sim* s, double dt) {
    Topo& t = s->topo;
    int nblk = std::min(ceil_div(2 * t.n + t.nw, 256), RN_BLOCKS);
    if (3 * nblk > 32 * s->red_blocks) fail(DP_E_INVALID, "reduction buffer too small");
    resnorm_kernel<<<nblk, 256, 0, s->stream>>>(s->res, t.pvf, t.pvm, t.well_scale, t.n,
                                                t.nw, dt, s->rho_o_ref, s->rho_w_ref, s->red_part);
    resnorm_final<<<1, 256, 0, s->stream>>>(s->red_part, nblk, s->red_out);
    DP_LAUNCH_CHECK();
    DP_HIP(hipMemcpyAsync(s->hpin, s->red_out, 3 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    DP_HIP(hipStreamSynchronize(s->stream));
    for (int i = 0; i < 3; ++i) s->red_host[i] = s->hpin[i];
    ResNorm r;
    r.cnv = s->red_host[0];
    double pv = s->pore_volume > 0 ? s->pore_volume : 1.0;
    double mo = fabs(s->red_host[1]) * dt / (s->rho_o_ref * pv);
    double mw = fabs(s->red_host[2]) * dt / (s->rho_w_ref * pv);
    r.mb = fmax(mo, mw);
    if (!(mo == mo) || !(mw == mw)) r.mb = INFINITY;
    return r;
}

// ---------------------------------------------------------------------------
// Newton update: x += dx; the saturation change is chopped to +-0.2, stopped at
// the relative-permeability end point it would cross from inside the mobile
// range (S_wc from above, 1 - S_or from below), and S is clamped to [0,1]; BHP
// wells pinned to their target; dummy unknowns kept at 0.
// ---------------------------------------------------------------------------
__global__ void newton_update_kernel(d2* x, const d2* __restrict__ dx, int n, int nw,
                                     const int* __restrict__ well_ctrl,
                                     const double* __restrict__ well_target, double lo, double hi) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < 2 * n) {
        d2 v = x[r];
        d2 d = dx[r];
        double ds = fmin(fmax(d.y, -0.2), 0.2);
        double s = v.y + ds;
        if (v.y > lo && s < lo) s = lo;
        if (v.y < hi && s > hi) s = hi;
        s = fmin(fmax(s, 0.0), 1.0);
        x[r] = mk2(v.x + d.x, s);
    } else if (r < 2 * n + nw) {
        int w = r - 2 * n;
        double pb = well_ctrl[w] == DP_CTRL_BHP ? well_target[w] : x[r].x + dx[r].x;
        x[r] = mk2(pb, 0.0);
    }
}

void launch_newton_update(dp_sim* s) {
    Topo& t = s->topo;
    newton_update_kernel<<<ceil_div(t.nb, 256), 256, 0, s->stream>>>(
        s->x, s->dx, t.n, t.nw, t.well_ctrl, t.well_target, s->swc, 1.0 - s->sor);
    DP_LAUNCH_CHECK();
}

}  // namespace dp
