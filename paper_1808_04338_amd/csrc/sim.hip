// C ABI of the simulator: handle creation, topology and workspace layout,
// the Newton / timestep drivers, GMRES, state I/O and the inspection hooks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "kernels.h"
#include "physics.h"

using namespace dp;

namespace dp {

// Galerkin products per level-0 pressure nonzero that the setup scratch is
// sized for: the worst case trunc^2 with at most four interpolation entries.
constexpr double RAP_EXPANSION = 16.0;
constexpr int MAX_RED_BLOCKS_ALL = 2048;

static void fill_defaults(dp_sim_desc& d) {
    if (d.gmres_restart <= 0) d.gmres_restart = 30;
    if (d.lin_maxit <= 0) d.lin_maxit = 300;
    if (d.lin_rtol <= 0) d.lin_rtol = 1e-6;
    if (d.amg_coarse_max <= 0) d.amg_coarse_max = 2000;
    if (d.amg_max_levels <= 0) d.amg_max_levels = 25;
    if (d.amg_theta <= 0) d.amg_theta = 0.25;
    if (d.amg_trunc <= 0) d.amg_trunc = 3;
    if (d.newton_tol <= 0) d.newton_tol = 1e-3;
    if (d.mb_tol <= 0) d.mb_tol = 1e-7;
    if (d.forcing_eta0 <= 0) d.forcing_eta0 = 0.1;
    if (d.forcing_gamma <= 0) d.forcing_gamma = 0.9;
    if (d.forcing_beta <= 0) d.forcing_beta = 2.0;
    if (d.forcing_eta_min <= 0) d.forcing_eta_min = 1e-8;
    if (d.forcing_eta_max <= 0) d.forcing_eta_max = 0.9;
    if (d.max_newton <= 0) d.max_newton = 20;
    if (d.max_cuts <= 0) d.max_cuts = 8;
}

static void validate(const dp_sim_desc& d) {
    if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0) fail(DP_E_INVALID, "grid dimensions must be positive");
    if ((int64_t)d.nx * d.ny * d.nz > (int64_t)1 << 28) fail(DP_E_INVALID, "grid too large");
    if (!(d.dx > 0 && d.dy > 0 && d.dz > 0)) fail(DP_E_INVALID, "cell sizes must be positive");
    if (!d.kx || !d.ky || !d.kz || !d.km || !d.phi_f || !d.phi_m) fail(DP_E_INVALID, "null field array");
    if (d.nwells < 0 || (d.nwells > 0 && !d.wells)) fail(DP_E_INVALID, "bad well list");
    if (d.gmres_restart > 30) fail(DP_E_INVALID, "gmres_restart must be <= 30");
    if (d.amg_trunc > 8) fail(DP_E_INVALID, "amg_trunc must be <= 8");
    if (d.amg_coarse_max > 4096) fail(DP_E_INVALID, "amg_coarse_max must be <= 4096");
    if (!(d.swc >= 0 && d.sor >= 0 && d.swc + d.sor < 1)) fail(DP_E_INVALID, "bad Corey end points");
    if (d.precond_precision != DP_FP64 && d.precond_precision != DP_FP32)
        fail(DP_E_INVALID, "precond_precision must be DP_FP64 or DP_FP32");
    if (d.forcing < 0 || d.forcing > 3) fail(DP_E_INVALID, "forcing must be 0, 1, 2 or 3");
    if (d.precond_eager < 0 || d.precond_eager > 2) fail(DP_E_INVALID, "precond_eager must be 0, 1 or 2");
    if (d.decoupling < DP_DEC_GJ || d.decoupling > DP_DEC_TI) fail(DP_E_INVALID, "bad decoupling");
    if (!std::isfinite(d.c_r)) fail(DP_E_INVALID, "rock compressibility must be finite");
    if (d.cpr_variant != DP_CPR_FPF && d.cpr_variant != DP_CPR_FP) fail(DP_E_INVALID, "bad cpr_variant");
    if (d.forcing && !(d.forcing_beta > 1.0 && d.forcing_beta <= 2.0 && d.forcing_gamma <= 1.0 &&
                       d.forcing_eta_min <= d.forcing_eta_max && d.forcing_eta_max < 1.0))
        fail(DP_E_INVALID, "forcing parameters out of range");
    for (int w = 0; w < d.nwells; ++w) {
        const dp_well& wl = d.wells[w];
        if (wl.i < 0 || wl.i >= d.nx || wl.j < 0 || wl.j >= d.ny || wl.k0 < 0 || wl.k1 >= d.nz ||
            wl.k0 > wl.k1)
            fail(DP_E_INVALID, "well " + std::to_string(w) + " outside the grid");
        if (wl.kind != DP_WELL_INJ && wl.kind != DP_WELL_PROD) fail(DP_E_INVALID, "bad well kind");
        if (wl.control != DP_CTRL_RATE && wl.control != DP_CTRL_BHP && wl.control != DP_CTRL_ORATE)
            fail(DP_E_INVALID, "bad well control");
        if (wl.kind == DP_WELL_PROD && wl.control == DP_CTRL_RATE)
            fail(DP_E_INVALID, "rate control is supported for injectors only");
        if (wl.kind == DP_WELL_INJ && wl.control == DP_CTRL_ORATE)
            fail(DP_E_INVALID, "oil-rate control is supported for producers only");
        if (!(wl.rw > 0)) fail(DP_E_INVALID, "well radius must be positive");
        if (!(wl.wi >= 0) || !std::isfinite(wl.wi)) fail(DP_E_INVALID, "well index must be >= 0 and finite");
    }
}

// Host-side topology: elimination order, neighbour slots, perforations and the
// level-0 pressure pattern with its source codes.
struct HostTopo {
    int n, nw, nb, nred, nperf;
    std::vector<int> fcell, frow, fcol, fperf, perf_q, perf_well, perf_cell, well_ptr;
    std::vector<unsigned char> fmask;
    std::vector<double> perf_rw, perf_skin, perf_wi;
    std::vector<int> ap_rowptr, ap_col, ap_src;
    int64_t nfaces2 = 0;  // sum over fracture rows of present slots
};

static void build_topology(const dp_sim_desc& d, HostTopo& h) {
    int nx = d.nx, ny = d.ny, nz = d.nz;
    int n = nx * ny * nz;
    h.n = n;
    h.nw = d.nwells;
    h.nb = 2 * n + h.nw;
    h.fcell.resize(n);
    h.frow.resize(n);
    int q = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int c = 0; c < n; ++c) {
            int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
            if (((i + j + k) & 1) == pass) {
                h.fcell[q] = c;
                h.frow[c] = q;
                ++q;
            }
        }
    h.nred = 0;
    for (int c = 0; c < n; ++c) {
        int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        if (((i + j + k) & 1) == 0) ++h.nred;
    }
    h.fcol.assign((size_t)6 * n, 0);
    h.fmask.assign(n, 0);
    for (int qq = 0; qq < n; ++qq) {
        int c = h.fcell[qq];
        int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        int nbr[6] = {i > 0 ? c - 1 : -1,           i < nx - 1 ? c + 1 : -1,
                      j > 0 ? c - nx : -1,          j < ny - 1 ? c + nx : -1,
                      k > 0 ? c - nx * ny : -1,     k < nz - 1 ? c + nx * ny : -1};
        for (int s = 0; s < 6; ++s) {
            if (nbr[s] >= 0) {
                h.fcol[(size_t)s * n + qq] = n + h.frow[nbr[s]];
                h.fmask[qq] |= (unsigned char)(1u << s);
                ++h.nfaces2;
            } else {
                h.fcol[(size_t)s * n + qq] = n + qq;
            }
        }
    }
    h.fperf.assign(n, -1);
    h.well_ptr.assign(h.nw + 1, 0);
    for (int w = 0; w < h.nw; ++w) {
        const dp_well& wl = d.wells[w];
        for (int k = wl.k0; k <= wl.k1; ++k) {
            int c = wl.i + nx * (wl.j + ny * k);
            int qq = h.frow[c];
            if (h.fperf[qq] >= 0) fail(DP_E_INVALID, "two perforations in one cell");
            h.fperf[qq] = (int)h.perf_q.size();
            h.perf_q.push_back(qq);
            h.perf_well.push_back(w);
            h.perf_cell.push_back(c);
            h.perf_rw.push_back(wl.rw);
            h.perf_skin.push_back(wl.skin);
            h.perf_wi.push_back(wl.wi);
        }
        h.well_ptr[w + 1] = (int)h.perf_q.size();
    }
    h.nperf = (int)h.perf_q.size();
    // level-0 pressure pattern of the reduced system (matrix-node pressures
    // eliminated): rows = fracture rows q, then wells n + w; sorted columns
    h.ap_rowptr.assign(n + h.nw + 1, 0);
    std::vector<std::pair<int, int>> row;
    for (int r = 0; r < n + h.nw; ++r) {
        row.clear();
        if (r < n) {
            int qq = r;
            for (int s = 0; s < 6; ++s)
                if (h.fmask[qq] & (1u << s)) row.push_back({h.fcol[(size_t)s * n + qq] - n, s});
            row.push_back({qq, 7});
            if (h.fperf[qq] >= 0) row.push_back({n + h.perf_well[h.fperf[qq]], 8});
        } else {
            int w = r - n;
            for (int p = h.well_ptr[w]; p < h.well_ptr[w + 1]; ++p) row.push_back({h.perf_q[p], p});
            row.push_back({r, -1});
        }
        std::sort(row.begin(), row.end());
        for (auto& e : row) {
            h.ap_col.push_back(e.first);
            h.ap_src.push_back(e.second);
        }
        h.ap_rowptr[r + 1] = (int)h.ap_col.size();
    }
}

template <class T>
static void alloc_bmat(Arena& a, BMat<T>& M, int n, int nb, int nperf, const char* what) {
    M.d0 = a.get<V2<T>>(nb, what);
    M.d1 = a.get<V2<T>>(nb, what);
    M.f0 = a.get<V2<T>>((int64_t)7 * n, what);
    M.f1 = a.get<V2<T>>((int64_t)7 * n, what);
    M.m0 = a.get<V2<T>>(n, what);
    M.m1 = a.get<V2<T>>(n, what);
    M.fw0 = a.get<V2<T>>(nperf, what);
    M.fw1 = a.get<V2<T>>(nperf, what);
    M.wf0 = a.get<V2<T>>(nperf, what);
    M.wf1 = a.get<V2<T>>(nperf, what);
}

template <class T>
static void alloc_ilu(Arena& a, ILUF<T>& F, int n, int nb, int nperf) {
    F.ui0 = a.get<V2<T>>(nb, "ilu");
    F.ui1 = a.get<V2<T>>(nb, "ilu");
    F.l0 = a.get<V2<T>>((int64_t)7 * n, "ilu");
    F.l1 = a.get<V2<T>>((int64_t)7 * n, "ilu");
    F.ubw0 = a.get<V2<T>>(nperf, "ilu");
    F.ubw1 = a.get<V2<T>>(nperf, "ilu");
    F.lw0 = a.get<V2<T>>(nperf, "ilu");
    F.lw1 = a.get<V2<T>>(nperf, "ilu");
}

struct Layout {
    size_t persistent = 0, hier = 0, scratch = 0;
};

// Lays out every persistent array of the handle in 'a' (or only counts bytes
// when a.counting).  Returns the sizes of the AMG hierarchy and scratch regions.
static Layout layout(dp_sim* s, Arena& a, const HostTopo& h) {
    int n = h.n, nb = h.nb, nperf = h.nperf, nw = h.nw;
    Topo& t = s->topo;
    t.fcol = a.get<int>((int64_t)6 * n, "topology");
    t.fmask = a.get<unsigned char>(n, "topology");
    t.cell = a.get<int>(n, "topology");
    t.fperf = a.get<int>(n, "topology");
    t.perf_q = a.get<int>(nperf, "topology");
    t.perf_well = a.get<int>(nperf, "topology");
    t.well_ptr = a.get<int>(nw + 1, "topology");
    t.well_kind = a.get<int>(nw, "wells");
    t.well_ctrl = a.get<int>(nw, "wells");
    t.well_target = a.get<double>(nw, "wells");
    t.well_scale = a.get<double>(nw, "wells");
    t.tface = a.get<double>((int64_t)6 * n, "geometry");
    t.tmf = a.get<double>(n, "geometry");
    t.pvf = a.get<double>(n, "geometry");
    t.pvm = a.get<double>(n, "geometry");
    t.depth = a.get<double>(n, "geometry");
    t.wi = a.get<double>(nperf, "geometry");
    s->x = a.get<d2>(nb, "state");
    s->x_save = a.get<d2>(nb, "state");
    s->x_sub = a.get<d2>(nb, "state");
    s->acc_old = a.get<d2>(2 * (int64_t)n, "state");
    s->res = a.get<d2>(nb, "residual");
    s->rhs = a.get<d2>(nb, "rhs");
    s->dx = a.get<d2>(nb, "correction");
    if (s->desc.forcing) {
        s->ft = a.get<d2>(nb, "forcing terms");
        s->fu = a.get<d2>(nb, "forcing terms");
    }
    alloc_bmat(a, s->J, n, nb, nperf, "jacobian");
    alloc_bmat(a, s->A, n, nb, nperf, "decoupled matrix");
    size_t es = s->fp32 ? 4 : 8;
    if (s->fp32) {
        alloc_bmat(a, s->A32, n, nb, nperf, "decoupled matrix fp32");
        alloc_ilu(a, s->ilu32, n, nb, nperf);
    } else {
        alloc_ilu(a, s->ilu64, n, nb, nperf);
    }
    int64_t nnz0 = (int64_t)h.ap_col.size();
    s->Ap0.n = n + nw;
    s->Ap0.ncols = n + nw;
    s->Ap0.nnz = nnz0;
    s->Ap0.rowptr = a.get<int>(n + nw + 1, "pressure pattern");
    s->Ap0.col = a.get<int>(nnz0, "pressure pattern");
    s->Ap0.val = a.get<double>(nnz0, "pressure pattern");
    s->ap_src = a.get<int>(nnz0, "pressure pattern");
    s->pr = a.take(es * 2 * nb, "precond vectors");
    s->pz = a.take(es * 2 * nb, "precond vectors");
    s->pt = a.take(es * 2 * nb, "precond vectors");
    s->pz2 = a.take(es * 2 * nb, "precond vectors");
    s->rpm = a.take(es * (n > 0 ? n : 1), "precond vectors");
    s->st0 = a.take(es * 8 * (n > 0 ? n : 1), "level-0 stencil");
    int m = s->restart;
    s->V = a.get<double>((int64_t)(m + 1) * 2 * nb, "krylov basis");
    s->Z = a.get<double>((int64_t)m * 2 * nb, "krylov basis");
    s->w = a.get<double>((int64_t)2 * nb, "krylov work");
    s->red_blocks = std::max(MAX_RED_BLOCKS_ALL, ceil_div(2 * (int64_t)n + nw, 256));
    s->red_part = a.get<double>((int64_t)s->red_blocks * 32, "reductions");
    s->red_out = a.get<double>(256, "reductions");
    Layout L;
    L.persistent = a.top;
    int64_t cm = s->desc.amg_coarse_max;
    L.hier = (size_t)(4.0 * nnz0 * (12 + 1.5 * (4 + es)) + 2.0 * nb * (4 + 9 * es + 12 * 8) +
                      (double)cm * cm * es + (1 << 20));
    double expn = RAP_EXPANSION * nnz0;
    // per expanded product: keys and values twice (sort double buffer) + row key
    L.scratch = (size_t)(expn * 36.0 + expn / 8.0 + nnz0 * 24.0 +
                         8.0 * ((double)cm + 32) * ((double)cm + 32) + 64.0 * nb + (4 << 20));
    return L;
}

static void make_phys_scalars(dp_sim* s) {
    const dp_sim_desc& d = s->desc;
    s->rho_w_ref = d.rho_w_ref;
    s->rho_o_ref = d.rho_o_ref;
    s->p_ref = d.p_ref;
    s->c_w = d.c_w;
    s->c_o = d.c_o;
    s->c_r = d.c_r;
    s->mu_w = d.mu_w;
    s->mu_o = d.mu_o;
    s->swc = d.swc;
    s->sor = d.sor;
    s->n_w = d.n_w;
    s->n_o = d.n_o;
    s->krw_max = d.krw_max;
    s->kro_max = d.kro_max;
    s->gravity = d.gravity;
    s->dz = d.dz;
}

static size_t total_bytes(const Layout& L) { return L.persistent + 256 + L.hier + 256 + L.scratch + 256; }

// ---------------------------------------------------------------------------
// well control arrays (device) from the host control state
// ---------------------------------------------------------------------------
static std::vector<int> host_ctrl(dp_sim* s) {
    std::vector<int> c(s->topo.nw);
    DP_HIP(hipMemcpyAsync(c.data(), s->topo.well_ctrl, sizeof(int) * c.size(), hipMemcpyDeviceToHost,
                          s->stream));
    DP_HIP(hipStreamSynchronize(s->stream));
    return c;
}

static void set_controls(dp_sim* s, const std::vector<int>& ctrl) {
    int nw = s->topo.nw;
    if (nw == 0) return;
    std::vector<int> kind(nw);
    std::vector<double> target(nw), scale(nw);
    for (int w = 0; w < nw; ++w) {
        const dp_well& wl = s->wells[w];
        kind[w] = wl.kind;
        if (ctrl[w] == DP_CTRL_RATE) {
            target[w] = wl.target;
            scale[w] = 1.0 / (s->rho_w_ref * std::max(std::fabs(wl.target), 1e-6));
        } else if (ctrl[w] == DP_CTRL_ORATE) {
            target[w] = wl.target;
            scale[w] = 1.0 / (s->rho_o_ref * std::max(std::fabs(wl.target), 1e-6));
        } else {
            target[w] = wl.control == DP_CTRL_BHP ? wl.target : wl.bhp_limit;
            scale[w] = 1.0 / std::max(std::fabs(target[w]), 1.0);
        }
    }
    DP_HIP(hipMemcpyAsync(s->topo.well_kind, kind.data(), sizeof(int) * nw, hipMemcpyHostToDevice, s->stream));
    DP_HIP(hipMemcpyAsync(s->topo.well_ctrl, ctrl.data(), sizeof(int) * nw, hipMemcpyHostToDevice, s->stream));
    DP_HIP(hipMemcpyAsync(s->topo.well_target, target.data(), sizeof(double) * nw, hipMemcpyHostToDevice,
                          s->stream));
    DP_HIP(hipMemcpyAsync(s->topo.well_scale, scale.data(), sizeof(double) * nw, hipMemcpyHostToDevice,
                          s->stream));
    DP_HIP(hipStreamSynchronize(s->stream));
}

// canonical block index of each elimination position
static int canon_of_pos(const dp_sim* s, int pos) {
    const Topo& t = s->topo;
    if (pos < t.n) return 2 * t.h_fcell[pos] + 1;
    if (pos < 2 * t.n) return 2 * t.h_fcell[pos - t.n];
    return pos;
}

static void to_positions(const dp_sim* s, const double* canon, std::vector<d2>& out) {
    int nb = s->topo.nb;
    out.resize(nb);
    for (int pos = 0; pos < nb; ++pos) {
        int b = canon_of_pos(s, pos);
        out[pos] = mk2(canon[2 * b], canon[2 * b + 1]);
    }
}

static void from_positions(const dp_sim* s, const std::vector<d2>& in, double* canon) {
    int nb = s->topo.nb;
    for (int pos = 0; pos < nb; ++pos) {
        int b = canon_of_pos(s, pos);
        canon[2 * b] = in[pos].x;
        canon[2 * b + 1] = in[pos].y;
    }
}

template <class T>
static std::vector<T> dl(dp_sim* s, const T* p, size_t n) {
    std::vector<T> h(n);
    if (n) DP_HIP(hipMemcpyAsync(h.data(), p, sizeof(T) * n, hipMemcpyDeviceToHost, s->stream));
    DP_HIP(hipStreamSynchronize(s->stream));
    return h;
}

// ---------------------------------------------------------------------------
// Timing helpers
// ---------------------------------------------------------------------------
struct PhaseScope {
    dp_sim* s;
    int ph;
    PhaseScope(dp_sim* s_, int ph_) : s(s_), ph(ph_) {
        if (s->timing) DP_HIP(hipEventRecord(s->pev[ph][0], s->stream));
    }
    ~PhaseScope() {
        if (!s->timing) return;
        if (hipEventRecord(s->pev[ph][1], s->stream) != hipSuccess) return;
        if (hipEventSynchronize(s->pev[ph][1]) != hipSuccess) return;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s->pev[ph][0], s->pev[ph][1]) == hipSuccess) {
            s->phase[ph].total_ms += ms;
            s->phase[ph].count += 1;
        }
    }
};

// ---------------------------------------------------------------------------
// GMRES(m), right-preconditioned with CPR-FPF, classical Gram-Schmidt with one
// re-orthogonalisation pass, Givens rotations on the host.  Solves A y = b with
// b = s->rhs into s->dx from y = 0.  Two passes over the basis per iteration:
// the re-orthogonalisation correction and the normalisation of w' are applied
// in the next iteration's first pass (which reads the basis anyway), the norm
// of the corrected vector comes from the Pythagorean relation, and the
// preconditioner takes w' / |w'|; the Hessenberg columns are CGS2's and
// A Z = V H holds for the stored Z.  One host synchronisation per iteration.
// ---------------------------------------------------------------------------
static int gmres(dp_sim* s, double rtol, int maxit, int* iters, double* rel_res) {
    int nb = s->topo.nb;
    int64_t len = 2 * (int64_t)nb;
    int m = s->restart;
    double* b = (double*)s->rhs;
    double* x = (double*)s->dx;
    double* r = s->w;
    double* hb = s->red_out;  // [0,32) h, [32,64) a and |w'|^2, [96] norms
    vec_zero(s, x, len);
    norm2(s, b, len, hb + 96);
    DP_HIP(hipMemcpyAsync(s->hpin, hb + 96, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    DP_HIP(hipStreamSynchronize(s->stream));
    double hn2 = s->hpin[0];
    double bnorm = std::sqrt(hn2);
    *iters = 0;
    if (!(bnorm > 0)) {
        *rel_res = 0.0;
        return bnorm == 0.0 ? DP_OK : DP_E_NUMERIC;
    }
    double beta = bnorm;
    const double* rvec = b;
    int its = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    while (beta > rtol * bnorm && its < maxit) {
        vec_scale_to(s, rvec, 1.0 / beta, s->V, len);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        double scale = 1.0;      // the preconditioner's input is the slot's vector times this
        double inv_alpha = 1.0;  // 1 / |w'' | of the vector pending in slot j
        for (int j = 0; j < m; ++j) {
            // slot j holds v_j (j = 0) or the previous iteration's w', still to be
            // corrected and normalised; the preconditioner takes w' / |w'|
            double* vj = s->V + (int64_t)j * len;
            double* zj = s->Z + (int64_t)j * len;
            {
                PhaseScope ps(s, 4);
                cpr_apply(s, vj, zj, scale);
            }
            {
                PhaseScope ps(s, 3);
                KtScope ks(&s->kt[0], s->stream);
                bspmv<double>(s, (const d2*)zj, (d2*)r);
                ks.bytes(kernel_bytes(s, 0));
            }
            {
                // the two passes over the basis, timed as one launch; bytes: the
                // vectors read and written (j = 0: v_0 and w twice, u written;
                // else v_0..v_j and w, v_j written, then v_0..v_j and w, u written)
                KtScope ks(&s->kt[4], s->stream);
                // h = V^T w over v_0..v_j; for j > 0 the same pass first forms
                // v_j = (w' - V a) / alpha in place from the previous a (at hb + 32)
                if (j == 0) dot_multi(s, s->V, len, 1, r, len, hb);
                else gs_finish_dot(s, s->V, len, j, hb + 32, inv_alpha, r, len, hb);
                // w' = w - V h into slot j + 1, a = V^T w' and |w'|^2 (at hb + 32)
                gs_update_dot_norm(s, s->V, len, j + 1, hb, r, s->V + (int64_t)(j + 1) * len, len, hb + 32);
                ks.bytes(8.0 * (double)len * (j == 0 ? 5.0 : 2.0 * j + 6.0));
            }
            DP_HIP(hipMemcpyAsync(s->hpin, hb, sizeof(double) * 64, hipMemcpyDeviceToHost, s->stream));
            DP_HIP(hipStreamSynchronize(s->stream));
            const double* hbuf = s->hpin;
            // column j: CGS2's coefficients h + a, and |w' - V a| by the
            // Pythagorean relation (V orthonormal)
            double n2 = hbuf[32 + j + 1], aa = 0.0;
            std::vector<double> col(m + 1, 0.0);
            for (int i = 0; i <= j; ++i) {
                col[i] = hbuf[i] + hbuf[32 + i];
                aa += hbuf[32 + i] * hbuf[32 + i];
            }
            if (!std::isfinite(n2) || !std::isfinite(aa)) {
                *iters = its;
                *rel_res = NAN;
                return DP_E_NUMERIC;
            }
            double d = n2 - aa;
            double hn = d > 0.0 ? std::sqrt(d) : 0.0;
            col[j + 1] = hn;
            for (int i = 0; i < j; ++i) {
                double tt = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = tt;
            }
            double den = std::hypot(col[j], col[j + 1]);
            cs[j] = den != 0.0 ? col[j] / den : 1.0;
            sn[j] = den != 0.0 ? col[j + 1] / den : 0.0;
            col[j] = den;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            for (int i = 0; i <= m; ++i) H[(size_t)i * m + j] = col[i];
            ++its;
            k = j + 1;
            if (hn == 0.0 || std::fabs(g[j + 1]) <= rtol * bnorm || its >= maxit) break;
            inv_alpha = 1.0 / hn;
            scale = 1.0 / std::sqrt(n2);
        }
        for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int l = i + 1; l < k; ++l) acc -= H[(size_t)i * m + l] * y[l];
            y[i] = H[(size_t)i * m + i] != 0.0 ? acc / H[(size_t)i * m + i] : 0.0;
        }
        combine(s, s->Z, len, k, y.data(), x, len);
        bresidual<double>(s, (const d2*)b, (const d2*)x, (d2*)r);
        norm2(s, r, len, hb + 96);
        DP_HIP(hipMemcpyAsync(s->hpin, hb + 96, sizeof(double), hipMemcpyDeviceToHost, s->stream));
        DP_HIP(hipStreamSynchronize(s->stream));
        hn2 = s->hpin[0];
        beta = std::sqrt(hn2);
        rvec = r;
        if (!std::isfinite(beta)) {
            *iters = its;
            *rel_res = NAN;
            return DP_E_NUMERIC;
        }
    }
    *iters = its;
    *rel_res = beta / bnorm;
    return beta <= rtol * bnorm ? DP_OK : DP_E_NOCONV;
}

// ---------------------------------------------------------------------------
// Mass balance sums: [M_o^n, M_w^n, M_o, M_w, Q_o, Q_w].  Block partials over a
// fixed grid (grid-stride, fixed order), then one block adds them in block
// order in a second kernel, so the sums do not depend on timing.
// ---------------------------------------------------------------------------
constexpr int MS_BLOCKS = 512;

__global__ void mass_sums_kernel(Phys P, const d2* __restrict__ x, const d2* __restrict__ acc_old,
                                 const double* __restrict__ pvf, const double* __restrict__ pvm,
                                 const int* __restrict__ perf_q,
                                 const int* __restrict__ perf_well, const int* __restrict__ well_kind,
                                 const double* __restrict__ wi, int n, int nperf, double* part) {
    __shared__ double sh[6][256 / WAVE];
    double v[6] = {0, 0, 0, 0, 0, 0};
    const int stride = gridDim.x * blockDim.x;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < 2 * n; r += stride) {
        d2 o = acc_old[r];
        v[0] += o.x;
        v[1] += o.y;
        double pv = r < n ? pvm[r] : pvf[r - n];
        d2 xx = x[r];
        double rho_o = P.rho_ref[0] * exp(P.c[0] * (xx.x - P.p_ref));
        double rho_w = P.rho_ref[1] * exp(P.c[1] * (xx.x - P.p_ref));
        double pvp = pv * (1.0 + P.c_r * (xx.x - P.p_ref));
        v[2] += pvp * (1.0 - xx.y) * rho_o;
        v[3] += pvp * xx.y * rho_w;
    }
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nperf; p += stride) {
        int pos = n + perf_q[p];
        d2 xf = x[pos];
        Props pr = props(P, xf.x, xf.y);
        int w = perf_well[p];
        Perf rr = perf_rate(P, well_kind[w], wi[p], x[2 * n + w].x, xf.x, pr);
        v[4] += rr.q[0];
        v[5] += rr.q[1];
    }
    for (int k = 0; k < 6; ++k) {
        double t = wave_sum(v[k]);
        if (threadIdx.x % WAVE == 0) sh[k][threadIdx.x / WAVE] = t;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double t = 0;
        for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) t += sh[threadIdx.x][i];
        part[6 * (int64_t)blockIdx.x + threadIdx.x] = t;
    }
}

__global__ void mass_sums_final(const double* __restrict__ part, int nblk, double* out) {
    // six lanes of the first wave each add one quantity over the blocks in order
    if (threadIdx.x < 6) {
        double t = 0;
        for (int b = 0; b < nblk; ++b) t += part[6 * (int64_t)b + threadIdx.x];
        out[threadIdx.x] = t;
    }
}

static void mass_sums(dp_sim* s, double out[6]) {
    Topo& t = s->topo;
    int nblk = (int)std::min<int64_t>(MS_BLOCKS, std::max<int64_t>(1, ceil_div(2 * (int64_t)t.n, 256)));
    mass_sums_kernel<<<nblk, 256, 0, s->stream>>>(make_phys(s), s->x, s->acc_old, t.pvf, t.pvm, t.perf_q,
                                                  t.perf_well, t.well_kind, t.wi, t.n, t.nperf, s->red_part);
    DP_LAUNCH_CHECK();
    mass_sums_final<<<1, 64, 0, s->stream>>>(s->red_part, nblk, s->red_out + 128);
    DP_LAUNCH_CHECK();
    DP_HIP(hipMemcpyAsync(s->hpin, s->red_out + 128, sizeof(double) * 6, hipMemcpyDeviceToHost, s->stream));
    DP_HIP(hipStreamSynchronize(s->stream));
    for (int i = 0; i < 6; ++i) out[i] = s->hpin[i];
}

static void copy_state(dp_sim* s, const d2* from, d2* to) {
    DP_HIP(hipMemcpyAsync(to, from, sizeof(d2) * s->topo.nb, hipMemcpyDeviceToDevice, s->stream));
}

static void mark_old(dp_sim* s) { launch_accumulation(s, s->x, s->acc_old); }

static ResNorm assemble(dp_sim* s, double dt) {
    PhaseScope ps(s, 0);
    launch_assemble(s, dt);
    s->dt_assembled = dt;
    s->stage = 1;
    return residual_norm(s, dt);
}

static bool converged(const dp_sim* s, const ResNorm& r) {
    return r.cnv <= s->desc.newton_tol && r.mb <= s->desc.mb_tol;
}

static bool finite(const ResNorm& r) { return std::isfinite(r.cnv) && std::isfinite(r.mb); }

static void setup(dp_sim* s) {
    if (s->stage < 1) fail(DP_E_STATE, "cpr_fpf_setup before assemble_residual_jacobian");
    PhaseScope ps(s, 1);
    cpr_setup(s);
    DP_HIP(hipStreamSynchronize(s->stream));
    s->stage = 2;
}

static int solve(dp_sim* s, double rtol, int maxit, int* its, double* rel) {
    if (s->stage < 2) fail(DP_E_STATE, "krylov_solve before cpr_fpf_setup");
    PhaseScope ps(s, 2);
    return gmres(s, rtol, maxit, its, rel);
}

// Adaptive forcing term eta_l of Eq. (13) for l >= 1 (the readings are stated
// with the descriptor's forcing fields).
static double forcing_term(const dp_sim_desc& d, double eta_prev, double nb, double nb_prev,
                           double nr_prev, double nd) {
    const double phi = 0.5 * (1.0 + std::sqrt(5.0));
    double eta, guard;
    if (d.forcing == 1) {
        eta = nd / nb_prev;
        guard = std::pow(eta_prev, phi);
    } else if (d.forcing == 2) {
        eta = std::fabs(nb - nr_prev) / nb_prev;
        guard = std::pow(eta_prev, phi);
    } else {
        eta = d.forcing_gamma * std::pow(nb / nb_prev, d.forcing_beta);
        guard = d.forcing_gamma * std::pow(eta_prev, d.forcing_beta);
    }
    if (guard > 0.1) eta = std::max(eta, guard);
    return std::min(std::max(eta, d.forcing_eta_min), d.forcing_eta_max);
}

// 2-norm of a device vector of 2 nb doubles (synchronises).
static double dev_norm(dp_sim* s, const double* x) {
    int64_t len = 2 * (int64_t)s->topo.nb;
    double* out = s->red_out + 128;
    norm2(s, x, len, out);
    double h = 0;
    DP_HIP(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    DP_HIP(hipStreamSynchronize(s->stream));
    return std::sqrt(h);
}

// One sub-step of length h from the current state; returns true on convergence.
static bool newton_loop(dp_sim* s, double h, int* newton_its, int* lin_its, double* res_out) {
    const dp_sim_desc& d = s->desc;
    int64_t len = 2 * (int64_t)s->topo.nb;
    // previous iteration's eta, ||b||, ||r|| (b = -R; r = b - J y, stored negated in ft)
    bool have_prev = false;
    double eta_prev = 0, nb_prev = 0, nr_prev = 0;
    // stagnation exit: the smallest CNV of this sub-step's updated iterates and the
    // iteration that reached it
    double best = INFINITY;
    int best_it = 0;
    for (int it = 0; it <= d.max_newton; ++it) {
        ResNorm nrm = assemble(s, h);
        *res_out = nrm.cnv;
        if (!finite(nrm)) return false;
        if (converged(s, nrm)) return true;
        if (it == d.max_newton) break;
        // the residual of the start state (iteration 0) belongs to the previous step's
        // solution; the exit judges only the iterates Newton has produced
        if (it >= 1) {
            if (nrm.cnv < best) {
                best = nrm.cnv;
                best_it = it;
            } else if (d.newton_stall > 0 && it - best_it >= d.newton_stall) {
                return false;
            }
        }
        double eta = d.lin_rtol, nb = 0, nd = 0;
        if (d.forcing) {
            nb = dev_norm(s, (const double*)s->res);
            if (!have_prev) {
                eta = d.forcing_eta0;
            } else {
                // ||b_l - r_{l-1}|| = ||R_l - ft|| with ft = R_{l-1} + J_{l-1} y_{l-1}
                double* dvec = (double*)s->fu;
                vec_copy(s, (const double*)s->res, dvec, len);
                vec_axpy(s, -1.0, (const double*)s->ft, dvec, len);
                nd = dev_norm(s, dvec);
                eta = forcing_term(d, eta_prev, nb, nb_prev, nr_prev, nd);
            }
        }
        // a singular preconditioner (zero pivot) counts as a failed iteration
        try {
            setup(s);
        } catch (const Error& e) {
            if (e.code != DP_E_NUMERIC) throw;
            return false;
        }
        size_t rec = s->eta_hist.size();
        s->eta_hist.insert(s->eta_hist.end(), {eta, nb, 0.0, nd, (double)it});
        int li = 0;
        double rr = 0;
        int st = solve(s, eta, d.lin_maxit, &li, &rr);
        *lin_its += li;
        if (st == DP_E_NUMERIC) return false;
        if (d.forcing) {
            // ft = R + J dx = -(b - J y): the negated linear residual of this iteration
            jspmv(s, (const d2*)s->dx, s->fu);
            vec_copy(s, (const double*)s->res, (double*)s->ft, len);
            vec_axpy(s, 1.0, (const double*)s->fu, (double*)s->ft, len);
            nr_prev = dev_norm(s, (const double*)s->ft);
            s->eta_hist[rec + 2] = nr_prev;
            nb_prev = nb;
            eta_prev = eta;
            have_prev = true;
        }
        launch_newton_update(s);
        ++*newton_its;
    }
    return false;
}

static int timestep_body(dp_sim* s, double dt, dp_step_info* info, const std::vector<int>& ctrl0) {
    const dp_sim_desc& d = s->desc;
    s->eta_hist.clear();
    dp_step_info out{};
    std::vector<int> ctrl = ctrl0;
    // state at the start of the current sub-step (device copy, for retries)
    copy_state(s, s->x, s->x_sub);
    double remaining = dt, h = dt;
    int cuts = 0;
    while (remaining > 0.0) {
        h = std::min(h, remaining);
        mark_old(s);
        bool switched = false, ok = false;
        for (;;) {
            double res = 0;
            ok = newton_loop(s, h, &out.newton_iters, &out.lin_iters, &res);
            out.res_scaled = res;
            if (!ok || switched) break;
            // a rate injector above its BHP maximum, or an oil-rate producer below its
            // BHP minimum, switches to BHP control at that limit
            std::vector<d2> xw = dl(s, s->x + 2 * s->topo.n, s->topo.nw);
            bool redo = false;
            for (int w = 0; w < s->topo.nw; ++w) {
                const dp_well& wl = s->wells[w];
                bool over = ctrl[w] == DP_CTRL_RATE && wl.kind == DP_WELL_INJ && xw[w].x > wl.bhp_limit;
                bool under = ctrl[w] == DP_CTRL_ORATE && wl.kind == DP_WELL_PROD && xw[w].x < wl.bhp_limit;
                if (over || under) {
                    ctrl[w] = DP_CTRL_BHP;
                    redo = true;
                }
            }
            if (!redo) break;
            switched = true;
            set_controls(s, ctrl);
            copy_state(s, s->x_sub, s->x);
        }
        if (!ok) {
            copy_state(s, s->x_sub, s->x);
            ++cuts;
            if (cuts > d.max_cuts) {
                copy_state(s, s->x_save, s->x);
                set_controls(s, ctrl0);
                out.cuts = cuts;
                if (info) *info = out;
                DP_HIP(hipStreamSynchronize(s->stream));
                return DP_E_NOCONV;
            }
            h *= 0.5;
            continue;
        }
        double ms[6];
        mass_sums(s, ms);
        double mbo = std::fabs(ms[2] - ms[0] - h * ms[4]);
        double mbw = std::fabs(ms[3] - ms[1] - h * ms[5]);
        mbo = ms[2] > 0 ? mbo / ms[2] : mbo;
        mbw = ms[3] > 0 ? mbw / ms[3] : mbw;
        out.mb_oil = std::max(out.mb_oil, mbo);
        out.mb_water = std::max(out.mb_water, mbw);
        out.substeps += 1;
        remaining -= h;
        out.dt += h;
        h *= 2.0;  // after an accepted sub-step the next may be twice as long
        copy_state(s, s->x, s->x_sub);
    }
    out.cuts = cuts;
    if (info) *info = out;
    return DP_OK;
}

// A timestep that fails, by non-convergence or by an error thrown anywhere in
// it (a workspace region overflowing in the setup, a failed HIP call), leaves
// the state and the well controls of the start of the step, with no work of
// the step still queued on the stream.
static int do_timestep(dp_sim* s, double dt, dp_step_info* info) {
    std::vector<int> ctrl0 = host_ctrl(s);
    copy_state(s, s->x, s->x_save);
    try {
        return timestep_body(s, dt, info, ctrl0);
    } catch (...) {
        try {
            copy_state(s, s->x_save, s->x);
            set_controls(s, ctrl0);
            DP_HIP(hipStreamSynchronize(s->stream));
        } catch (...) {
            (void)hipStreamSynchronize(s->stream);
        }
        s->stage = 0;
        throw;
    }
}

double kernel_bytes(dp_sim* s, int kernel) {
    const Topo& t = s->topo;
    double n = t.n, nb = t.nb, np = t.nperf;
    double es = s->fp32 ? 4.0 : 8.0;
    double blocks = nb + 7 * n + n + 2 * np;     // stored blocks of the matrix
    double idx = 4.0 * (6 * n + n + 3 * np) + n;  // fcol, fperf, perforations, fmask
    double vec = 16.0 * nb;
    if (kernel == 0) return blocks * 32.0 + idx + 2 * vec;
    if (kernel == 1) {
        // factors: U^-1 diagonals, L blocks (odd rows 7, even rows 1), U blocks taken
        // from the matrix (even rows 6, matrix rows 1), perforation blocks
        double fblocks = nb + 4 * n + 3 * n + n + 2 * np;
        return fblocks * 4 * es + idx + 2 * nb * 2 * es;
    }
    if (kernel == 2) {
        double b = 0;
        for (size_t l = 0; l < s->levels.size(); ++l) {
            const AmgLevel& L = s->levels[l];
            if (l + 1 == s->levels.size()) {
                b += (double)L.n * L.n * es + 2.0 * L.n * es;
                break;
            }
            // two sweeps over A (pre: b, dinv gathered; post: x), P and R once,
            // vectors: b, x, r, t, dinv
            auto opb = [&](const Op& o) {
                if (o.kind == 0) return o.s.nel * (4 + es) + 4.0 * (o.s.nslices + 1);
                return o.nnz * (4 + es) + 4.0 * (o.n + 1) + (o.kind == 2 ? 8.0 * (o.nb + 1) : 0.0);
            };
            b += 2.0 * opb(L.Aop) + opb(L.Pop) + opb(L.Rop);
            b += 8.0 * L.n * es;
        }
        return b;
    }
    if (kernel == 3) {
        // state, old accumulation, geometry read; residual and J written
        return 16.0 * nb + 16.0 * 2 * n + 8.0 * (6 * n + 4 * n + np) + idx + 16.0 * nb +
               blocks * 32.0;
    }
    if (kernel == 5) return 2.0 * 16.0 * nb;  // plain copy of the 2 nb doubles: read + write
    return 0.0;
}

}  // namespace dp

// ===========================================================================
// C ABI
// ===========================================================================
#define ABI_BEGIN try {
#define ABI_END(sim)                                        \
    }                                                       \
    catch (const dp::Error& e) {                            \
        if (sim) (sim)->err = e.what();                     \
        return e.code;                                      \
    }                                                       \
    catch (const std::exception& e) {                       \
        if (sim) (sim)->err = e.what();                     \
        return DP_E_DEVICE;                                 \
    }

static thread_local std::string g_create_error;

extern "C" {

dp_status sim_footprint(const dp_sim_desc* desc, size_t* device_bytes) {
    try {
        if (!desc || !device_bytes) return DP_E_INVALID;
        dp_sim tmp;
        tmp.desc = *desc;
        fill_defaults(tmp.desc);
        validate(tmp.desc);
        tmp.fp32 = tmp.desc.precond_precision == DP_FP32;
        tmp.restart = tmp.desc.gmres_restart;
        HostTopo h;
        build_topology(tmp.desc, h);
        Arena a;
        a.counting = true;
        Layout L = layout(&tmp, a, h);
        *device_bytes = total_bytes(L) + 6 * sizeof(double) * (size_t)h.n + 3 * 8 * (size_t)h.nperf + 4096;
        return DP_OK;
    } catch (const dp::Error& e) {
        g_create_error = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_create_error = e.what();
        return DP_E_INVALID;
    }
}

dp_status sim_create(const dp_sim_desc* desc, const double* p0, const double* sw0, void* d_workspace,
                     size_t workspace_bytes, void* hip_stream, dp_sim** out) {
    if (!desc || !p0 || !sw0 || !out) return DP_E_INVALID;
    *out = nullptr;
    dp_sim* s = new dp_sim();
    try {
        s->desc = *desc;
        fill_defaults(s->desc);
        validate(s->desc);
        if (!d_workspace) fail(DP_E_INVALID, "null workspace");
        if (((uintptr_t)d_workspace) & 255) fail(DP_E_INVALID, "workspace must be 256-byte aligned");
        s->wells.assign(desc->wells, desc->wells + desc->nwells);
        s->desc.wells = nullptr;
        s->desc.kx = s->desc.ky = s->desc.kz = s->desc.km = s->desc.phi_f = s->desc.phi_m = nullptr;
        s->stream = (hipStream_t)hip_stream;
        s->fp32 = s->desc.precond_precision == DP_FP32;
        s->restart = s->desc.gmres_restart;
        make_phys_scalars(s);
        HostTopo h;
        build_topology(*desc, h);
        Topo& t = s->topo;
        t.nx = desc->nx;
        t.ny = desc->ny;
        t.nz = desc->nz;
        t.n = h.n;
        t.nw = h.nw;
        t.nb = h.nb;
        t.nperf = h.nperf;
        t.nred = h.nred;
        t.h_fcol = h.fcol;
        t.h_fcell = h.fcell;
        t.h_fperf = h.fperf;
        t.h_perf_q = h.perf_q;
        t.h_perf_well = h.perf_well;
        t.h_well_ptr = h.well_ptr;
        t.h_fmask = h.fmask;
        s->arena.base = (char*)d_workspace;
        s->arena.cap = workspace_bytes;
        Layout L = layout(s, s->arena, h);
        // per-setup regions
        {
            void* hb = s->arena.take(L.hier, "AMG hierarchy region");
            void* sb = s->arena.take(L.scratch, "AMG setup scratch region");
            s->hier.base = (char*)hb;
            s->hier.cap = L.hier;
            s->scr.base = (char*)sb;
            s->scr.cap = L.scratch;
        }
        // upload topology and inputs
        hipStream_t st = s->stream;
        auto up = [&](void* dst, const void* src, size_t bytes) {
            if (bytes) DP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
        };
        int n = h.n;
        up(t.fcol, h.fcol.data(), sizeof(int) * h.fcol.size());
        up(t.fmask, h.fmask.data(), h.fmask.size());
        up(t.cell, h.fcell.data(), sizeof(int) * n);
        up(t.fperf, h.fperf.data(), sizeof(int) * n);
        up(t.perf_q, h.perf_q.data(), sizeof(int) * h.nperf);
        up(t.perf_well, h.perf_well.data(), sizeof(int) * h.nperf);
        up(t.well_ptr, h.well_ptr.data(), sizeof(int) * (h.nw + 1));
        up(s->Ap0.rowptr, h.ap_rowptr.data(), sizeof(int) * h.ap_rowptr.size());
        up(s->Ap0.col, h.ap_col.data(), sizeof(int) * h.ap_col.size());
        up(s->ap_src, h.ap_src.data(), sizeof(int) * h.ap_src.size());
        // fields: staged in the setup scratch region (free until the first setup)
        Arena& sc = s->scr;
        sc.top = 0;
        double* dk[6];
        const double* hk[6] = {desc->kx, desc->ky, desc->kz, desc->km, desc->phi_f, desc->phi_m};
        for (int i = 0; i < 6; ++i) {
            dk[i] = sc.get<double>(n, "input fields");
            up(dk[i], hk[i], sizeof(double) * n);
        }
        int* pc = sc.get<int>(h.nperf, "perforations");
        double* prw = sc.get<double>(h.nperf, "perforations");
        double* psk = sc.get<double>(h.nperf, "perforations");
        double* pwi = sc.get<double>(h.nperf, "perforations");
        up(pc, h.perf_cell.data(), sizeof(int) * h.nperf);
        up(prw, h.perf_rw.data(), sizeof(double) * h.nperf);
        up(psk, h.perf_skin.data(), sizeof(double) * h.nperf);
        up(pwi, h.perf_wi.data(), sizeof(double) * h.nperf);
        launch_geometry(s, dk[0], dk[1], dk[2], dk[3], dk[4], dk[5], pc, prw, psk, pwi);
        {
            double vol = desc->dx * desc->dy * desc->dz, pv = 0.0;
            for (int c = 0; c < n; ++c) pv += vol * desc->phi_f[c] + vol * desc->phi_m[c];
            s->pore_volume = pv;
        }
        std::vector<int> ctrl(h.nw);
        for (int w = 0; w < h.nw; ++w) ctrl[w] = s->wells[w].control;
        set_controls(s, ctrl);
        // initial state: rate injectors start at the mean initial pressure, BHP wells at target
        double pmean = 0;
        for (int i = 0; i < 2 * n; ++i) pmean += p0[i];
        pmean /= (2.0 * n);
        std::vector<double> canon((size_t)2 * h.nb);
        for (int i = 0; i < 2 * n; ++i) {
            canon[2 * i] = p0[i];
            canon[2 * i + 1] = sw0[i];
        }
        for (int w = 0; w < h.nw; ++w) {
            canon[2 * (2 * n + w)] = s->wells[w].control == DP_CTRL_BHP ? s->wells[w].target : pmean;
            canon[2 * (2 * n + w) + 1] = 0.0;
        }
        std::vector<d2> xs;
        to_positions(s, canon.data(), xs);
        up(s->x, xs.data(), sizeof(d2) * xs.size());
        DP_HIP(hipEventCreate(&s->ev0));
        DP_HIP(hipEventCreate(&s->ev1));
        for (auto& pe : s->pev)
            for (auto& e : pe) DP_HIP(hipEventCreate(&e));
        DP_HIP(hipHostMalloc((void**)&s->hpin, sizeof(double) * 64, hipHostMallocDefault));
        mark_old(s);
        DP_HIP(hipStreamSynchronize(st));
        sc.top = 0;
        *out = s;
        return DP_OK;
    } catch (const dp::Error& e) {
        g_create_error = e.what();
        dp_status c = e.code;
        if (s->hpin) (void)hipHostFree(s->hpin);
        delete s;
        return c;
    } catch (const std::exception& e) {
        g_create_error = e.what();
        if (s->hpin) (void)hipHostFree(s->hpin);
        delete s;
        return DP_E_DEVICE;
    }
}

dp_status sim_destroy(dp_sim* sim) {
    if (!sim) return DP_OK;
    // no kernel of this handle may still write the workspace once the caller frees it
    (void)hipStreamSynchronize(sim->stream);
    if (sim->ev0) (void)hipEventDestroy(sim->ev0);
    if (sim->ev1) (void)hipEventDestroy(sim->ev1);
    for (auto& pe : sim->pev)
        for (auto& e : pe)
            if (e) (void)hipEventDestroy(e);
    for (auto& t : sim->kt)
        for (auto& e : t.ev)
            if (e) (void)hipEventDestroy(e);
    if (sim->pc_exec) (void)hipGraphExecDestroy(sim->pc_exec);
    if (sim->cap_stream) (void)hipStreamDestroy(sim->cap_stream);
    if (sim->hpin) (void)hipHostFree(sim->hpin);
    delete sim;
    return DP_OK;
}

const char* sim_last_error(const dp_sim* sim) {
    if (!sim) return g_create_error.c_str();
    return sim->err.c_str();
}

dp_status sim_mark_old(dp_sim* sim) {
    if (!sim) return DP_E_INVALID;
    ABI_BEGIN
    mark_old(sim);
    DP_HIP(hipStreamSynchronize(sim->stream));
    return DP_OK;
    ABI_END(sim)
}

dp_status assemble_residual_jacobian(dp_sim* sim, double dt, double* res_scaled) {
    if (!sim || !(dt > 0)) return DP_E_INVALID;
    ABI_BEGIN
    ResNorm r = assemble(sim, dt);
    if (res_scaled) *res_scaled = r.cnv;
    return finite(r) ? DP_OK : DP_E_NUMERIC;
    ABI_END(sim)
}

dp_status cpr_fpf_setup(dp_sim* sim) {
    if (!sim) return DP_E_INVALID;
    ABI_BEGIN
    setup(sim);
    return DP_OK;
    ABI_END(sim)
}

dp_status krylov_solve(dp_sim* sim, double rtol, int32_t maxit, int32_t* iters, double* rel_res) {
    if (!sim || !(rtol > 0) || maxit <= 0) return DP_E_INVALID;
    ABI_BEGIN
    int it = 0;
    double rr = 0;
    int st = solve(sim, rtol, maxit, &it, &rr);
    if (iters) *iters = it;
    if (rel_res) *rel_res = rr;
    if (st == DP_E_NOCONV) sim->err = "GMRES reached maxit";
    if (st == DP_E_NUMERIC) sim->err = "GMRES breakdown (non-finite values)";
    return st;
    ABI_END(sim)
}

dp_status newton_update(dp_sim* sim) {
    if (!sim) return DP_E_INVALID;
    ABI_BEGIN
    if (sim->stage < 2) fail(DP_E_STATE, "newton_update before a solve");
    launch_newton_update(sim);
    DP_HIP(hipStreamSynchronize(sim->stream));
    return DP_OK;
    ABI_END(sim)
}

dp_status newton_step(dp_sim* sim, double dt, double eta, dp_newton_info* info) {
    if (!sim || !(dt > 0) || !(eta > 0)) return DP_E_INVALID;
    ABI_BEGIN
    dp_newton_info o{};
    ResNorm nrm = assemble(sim, dt);
    o.res_scaled = nrm.cnv;
    o.mb_scaled = nrm.mb;
    if (!finite(nrm)) {
        if (info) *info = o;
        sim->err = "non-finite residual";
        return DP_E_NUMERIC;
    }
    if (converged(sim, nrm)) {
        o.converged = 1;
        if (info) *info = o;
        return DP_OK;
    }
    setup(sim);
    int it = 0;
    double rr = 0;
    int st = solve(sim, eta, sim->desc.lin_maxit, &it, &rr);
    o.lin_iters = it;
    o.lin_rel_res = rr;
    if (st == DP_E_NUMERIC) {
        if (info) *info = o;
        sim->err = "GMRES breakdown";
        return st;
    }
    launch_newton_update(sim);
    DP_HIP(hipStreamSynchronize(sim->stream));
    if (info) *info = o;
    return DP_OK;
    ABI_END(sim)
}

dp_status timestep(dp_sim* sim, double dt, dp_step_info* info) {
    if (!sim || !(dt > 0)) return DP_E_INVALID;
    ABI_BEGIN
    int st = do_timestep(sim, dt, info);
    if (st == DP_E_NOCONV) sim->err = "timestep failed after the maximum number of cuts";
    return st;
    ABI_END(sim)
}

dp_status batch_timestep(dp_sim** sims, int32_t n, const double* dt, dp_step_info* info,
                         dp_status* status) {
    if (n < 0 || (n > 0 && (!sims || !dt))) return DP_E_INVALID;
    std::vector<dp_status> st(n, DP_OK);
    std::vector<std::thread> th;
    th.reserve(n);
    for (int i = 0; i < n; ++i)
        th.emplace_back([&, i]() { st[i] = timestep(sims[i], dt[i], info ? &info[i] : nullptr); });
    for (auto& t : th) t.join();
    dp_status worst = DP_OK;
    for (int i = 0; i < n; ++i) {
        if (status) status[i] = st[i];
        if (st[i] != DP_OK && worst == DP_OK) worst = st[i];
    }
    return worst;
}

dp_status sim_get_state(dp_sim* sim, double* p, double* sw, double* bhp) {
    if (!sim) return DP_E_INVALID;
    ABI_BEGIN
    std::vector<d2> xs = dl(sim, sim->x, sim->topo.nb);
    std::vector<double> canon((size_t)2 * sim->topo.nb);
    from_positions(sim, xs, canon.data());
    int n = sim->topo.n;
    for (int i = 0; i < 2 * n; ++i) {
        if (p) p[i] = canon[2 * i];
        if (sw) sw[i] = canon[2 * i + 1];
    }
    for (int w = 0; w < sim->topo.nw; ++w)
        if (bhp) bhp[w] = canon[2 * (2 * n + w)];
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_get_correction(dp_sim* sim, double* dx) {
    if (!sim || !dx) return DP_E_INVALID;
    ABI_BEGIN
    if (sim->stage < 2) fail(DP_E_STATE, "no correction before krylov_solve");
    std::vector<d2> xs = dl(sim, sim->dx, sim->topo.nb);
    from_positions(sim, xs, dx);
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_set_state(dp_sim* sim, const double* p, const double* sw, const double* bhp) {
    if (!sim || !p || !sw) return DP_E_INVALID;
    ABI_BEGIN
    int n = sim->topo.n;
    std::vector<d2> cur = dl(sim, sim->x, sim->topo.nb);
    std::vector<double> canon((size_t)2 * sim->topo.nb);
    from_positions(sim, cur, canon.data());
    for (int i = 0; i < 2 * n; ++i) {
        canon[2 * i] = p[i];
        canon[2 * i + 1] = sw[i];
    }
    for (int w = 0; w < sim->topo.nw; ++w)
        if (bhp) canon[2 * (2 * n + w)] = bhp[w];
    std::vector<d2> xs;
    to_positions(sim, canon.data(), xs);
    DP_HIP(hipMemcpyAsync(sim->x, xs.data(), sizeof(d2) * xs.size(), hipMemcpyHostToDevice, sim->stream));
    DP_HIP(hipStreamSynchronize(sim->stream));
    sim->stage = 0;
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_system_size(const dp_sim* sim, int32_t* n_dof, int64_t* nnz) {
    if (!sim) return DP_E_INVALID;
    const Topo& t = sim->topo;
    int64_t nfaces2 = 0;
    for (unsigned char m : t.h_fmask) nfaces2 += __builtin_popcount(m);
    int64_t nnzb = t.nb + nfaces2 + 2 * (int64_t)t.n + 2 * (int64_t)t.nperf;
    if (n_dof) *n_dof = 2 * t.nb;
    if (nnz) *nnz = 4 * nnzb;
    return DP_OK;
}

}  // extern "C"

// Blocks of the current matrix in canonical block coordinates: calls f(brow, bcol, blk) for
// every pattern block; the matrix is read back from device planes.
template <class F>
static void for_each_block(dp_sim* s, const BMat<double>& M, F f) {
    const Topo& t = s->topo;
    int n = t.n, nb = t.nb, np = t.nperf;
    auto d0 = dl(s, M.d0, nb), d1 = dl(s, M.d1, nb);
    auto f0 = dl(s, M.f0, (size_t)7 * n), f1 = dl(s, M.f1, (size_t)7 * n);
    auto m0 = dl(s, M.m0, n), m1 = dl(s, M.m1, n);
    auto fw0 = dl(s, M.fw0, np), fw1 = dl(s, M.fw1, np);
    auto wf0 = dl(s, M.wf0, np), wf1 = dl(s, M.wf1, np);
    for (int pos = 0; pos < nb; ++pos) {
        int br = canon_of_pos(s, pos);
        f(br, br, mkb(d0[pos], d1[pos]));
        if (pos < n) {
            f(br, canon_of_pos(s, n + pos), mkb(m0[pos], m1[pos]));
        } else if (pos < 2 * n) {
            int q = pos - n;
            for (int sl = 0; sl < 6; ++sl)
                if (t.h_fmask[q] & (1u << sl))
                    f(br, canon_of_pos(s, t.h_fcol[(size_t)sl * n + q]), mkb(f0[(size_t)sl * n + q], f1[(size_t)sl * n + q]));
            f(br, canon_of_pos(s, q), mkb(f0[(size_t)6 * n + q], f1[(size_t)6 * n + q]));
            int p = t.h_fperf[q];
            if (p >= 0) f(br, 2 * n + t.h_perf_well[p], mkb(fw0[p], fw1[p]));
        } else {
            int w = pos - 2 * n;
            for (int p = t.h_well_ptr[w]; p < t.h_well_ptr[w + 1]; ++p)
                f(br, canon_of_pos(s, n + t.h_perf_q[p]), mkb(wf0[p], wf1[p]));
        }
    }
}

extern "C" {

dp_status sim_export_system(dp_sim* sim, int32_t which, int32_t* rowptr, int32_t* colind, double* vals,
                            double* rhs) {
    if (!sim || !rowptr || !colind || !vals) return DP_E_INVALID;
    ABI_BEGIN
    if (which == 0 && sim->stage < 1) fail(DP_E_STATE, "nothing assembled");
    if (which == 1 && sim->stage < 2) fail(DP_E_STATE, "no decoupled system before cpr_fpf_setup");
    if (which != 0 && which != 1) fail(DP_E_INVALID, "which must be 0 or 1");
    int nb = sim->topo.nb;
    std::vector<std::vector<std::pair<int, Blk<double>>>> rows(nb);
    for_each_block(sim, which == 0 ? sim->J : sim->A,
                   [&](int br, int bc, const Blk<double>& b) { rows[br].push_back({bc, b}); });
    int64_t e = 0;
    rowptr[0] = 0;
    for (int br = 0; br < nb; ++br) {
        auto& r = rows[br];
        std::sort(r.begin(), r.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        for (int half = 0; half < 2; ++half) {
            for (auto& kv : r) {
                const Blk<double>& b = kv.second;
                colind[e] = 2 * kv.first;
                vals[e] = half == 0 ? b.a00 : b.a10;
                ++e;
                colind[e] = 2 * kv.first + 1;
                vals[e] = half == 0 ? b.a01 : b.a11;
                ++e;
            }
            rowptr[2 * br + half + 1] = (int32_t)e;
        }
    }
    if (rhs) {
        std::vector<d2> v = dl(sim, which == 0 ? sim->res : sim->rhs, nb);
        from_positions(sim, v, rhs);
    }
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_export_ilu(dp_sim* sim, int32_t* perm, int32_t* brow, int32_t* bcol, double* vals) {
    if (!sim || !perm || !brow || !bcol || !vals) return DP_E_INVALID;
    ABI_BEGIN
    if (sim->stage < 2) fail(DP_E_STATE, "no factors before cpr_fpf_setup");
    const Topo& t = sim->topo;
    int n = t.n, nb = t.nb, np = t.nperf;
    for (int pos = 0; pos < nb; ++pos) perm[pos] = canon_of_pos(sim, pos);
    std::vector<Blk<double>> ui(nb), l((size_t)7 * n), ubw(np), lw(np);
    auto get = [&](auto& F) {
        using VT = std::remove_pointer_t<decltype(F.ui0)>;
        auto u0 = dl(sim, F.ui0, nb), u1 = dl(sim, F.ui1, nb);
        auto l0 = dl(sim, F.l0, (size_t)7 * n), l1 = dl(sim, F.l1, (size_t)7 * n);
        auto b0 = dl(sim, F.ubw0, np), b1 = dl(sim, F.ubw1, np);
        auto w0 = dl(sim, F.lw0, np), w1 = dl(sim, F.lw1, np);
        auto cv = [](VT a, VT b) { return Blk<double>{(double)a.x, (double)a.y, (double)b.x, (double)b.y}; };
        for (int i = 0; i < nb; ++i) ui[i] = cv(u0[i], u1[i]);
        for (size_t i = 0; i < l.size(); ++i) l[i] = cv(l0[i], l1[i]);
        for (int i = 0; i < np; ++i) {
            ubw[i] = cv(b0[i], b1[i]);
            lw[i] = cv(w0[i], w1[i]);
        }
    };
    if (sim->fp32) get(sim->ilu32);
    else get(sim->ilu64);
    // U blocks that equal the decoupled matrix's own blocks
    std::vector<Blk<double>> Af((size_t)7 * n), Am(n);
    {
        auto f0 = dl(sim, sim->A.f0, (size_t)7 * n), f1 = dl(sim, sim->A.f1, (size_t)7 * n);
        auto m0 = dl(sim, sim->A.m0, n), m1 = dl(sim, sim->A.m1, n);
        for (size_t i = 0; i < Af.size(); ++i) Af[i] = mkb(f0[i], f1[i]);
        for (int i = 0; i < n; ++i) Am[i] = mkb(m0[i], m1[i]);
    }
    int64_t e = 0;
    auto put = [&](int pr, int pc, const Blk<double>& b) {
        brow[e] = canon_of_pos(sim, pr);
        bcol[e] = canon_of_pos(sim, pc);
        vals[4 * e] = b.a00;
        vals[4 * e + 1] = b.a01;
        vals[4 * e + 2] = b.a10;
        vals[4 * e + 3] = b.a11;
        ++e;
    };
    for (int pos = 0; pos < nb; ++pos) {
        put(pos, pos, ui[pos]);
        if (pos < n) {
            put(pos, n + pos, Am[pos]);
        } else if (pos < 2 * n) {
            int q = pos - n;
            bool red = q < t.nred;
            for (int sl = 0; sl < 6; ++sl)
                if (t.h_fmask[q] & (1u << sl)) put(pos, t.h_fcol[(size_t)sl * n + q], red ? Af[(size_t)sl * n + q] : l[(size_t)sl * n + q]);
            put(pos, q, l[(size_t)6 * n + q]);
            int p = t.h_fperf[q];
            if (p >= 0) put(pos, 2 * n + t.h_perf_well[p], ubw[p]);
        } else {
            int w = pos - 2 * n;
            for (int p = t.h_well_ptr[w]; p < t.h_well_ptr[w + 1]; ++p) put(pos, n + t.h_perf_q[p], lw[p]);
        }
    }
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_amg_info(dp_sim* sim, int32_t* levels, int32_t* rows, int64_t* nnz) {
    if (!sim) return DP_E_INVALID;
    if (sim->stage < 2) {
        sim->err = "no hierarchy before cpr_fpf_setup";
        return DP_E_STATE;
    }
    if (levels) *levels = (int32_t)sim->levels.size();
    for (size_t l = 0; l < sim->levels.size(); ++l) {
        if (rows) rows[l] = sim->levels[l].n;
        if (nnz) nnz[l] = sim->levels[l].A.nnz;
    }
    return DP_OK;
}

dp_status sim_eta_history(dp_sim* sim, double* rec, int32_t cap, int32_t* count) {
    if (!sim || cap < 0 || (cap > 0 && !rec)) return DP_E_INVALID;
    int32_t n = (int32_t)(sim->eta_hist.size() / 5);
    for (int32_t i = 0; i < 5 * n && i < 5 * cap; ++i) rec[i] = sim->eta_hist[i];
    if (count) *count = n;
    return DP_OK;
}

dp_status sim_amg_stats(dp_sim* sim, int64_t* global_sort_products) {
    if (!sim) return DP_E_INVALID;
    if (global_sort_products) *global_sort_products = sim->seg_fallbacks;
    return DP_OK;
}

dp_status sim_export_amg_level(dp_sim* sim, int32_t level, int32_t* cf, int32_t* a_rowptr, int32_t* a_col,
                               double* a_val, int32_t* p_rowptr, int32_t* p_col, double* p_val,
                               int64_t* p_nnz) {
    if (!sim) return DP_E_INVALID;
    ABI_BEGIN
    if (sim->stage < 2) fail(DP_E_STATE, "no hierarchy before cpr_fpf_setup");
    if (level < 0 || level >= (int)sim->levels.size()) fail(DP_E_INVALID, "level out of range");
    AmgLevel& L = sim->levels[level];
    auto cp = [&](auto* dst, auto* src, size_t n) {
        if (dst && src && n) {
            DP_HIP(hipMemcpyAsync(dst, src, sizeof(*src) * n, hipMemcpyDeviceToHost, sim->stream));
        }
    };
    cp(cf, L.cf, (size_t)L.n);
    cp(a_rowptr, L.A.rowptr, (size_t)L.n + 1);
    cp(a_col, L.A.col, (size_t)L.A.nnz);
    cp(a_val, L.A.val, (size_t)L.A.nnz);
    if (p_nnz) *p_nnz = L.cf ? L.P.nnz : 0;
    if (L.cf) {
        cp(p_rowptr, L.P.rowptr, (size_t)L.n + 1);
        cp(p_col, L.P.col, (size_t)L.P.nnz);
        cp(p_val, L.P.val, (size_t)L.P.nnz);
    }
    DP_HIP(hipStreamSynchronize(sim->stream));
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_apply_precond(dp_sim* sim, const double* r, double* z) {
    if (!sim || !r || !z) return DP_E_INVALID;
    ABI_BEGIN
    if (sim->stage < 2) fail(DP_E_STATE, "no preconditioner before cpr_fpf_setup");
    std::vector<d2> rv, zv;
    to_positions(sim, r, rv);
    int nb = sim->topo.nb;
    DP_HIP(hipMemcpyAsync(sim->w, rv.data(), sizeof(d2) * nb, hipMemcpyHostToDevice, sim->stream));
    cpr_apply(sim, sim->w, sim->V);
    zv = dl(sim, (d2*)sim->V, nb);
    from_positions(sim, zv, z);
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_apply_matrix(dp_sim* sim, const double* x, double* y) {
    if (!sim || !x || !y) return DP_E_INVALID;
    ABI_BEGIN
    if (sim->stage < 2) fail(DP_E_STATE, "no decoupled matrix before cpr_fpf_setup");
    std::vector<d2> xv, yv;
    to_positions(sim, x, xv);
    int nb = sim->topo.nb;
    DP_HIP(hipMemcpyAsync(sim->w, xv.data(), sizeof(d2) * nb, hipMemcpyHostToDevice, sim->stream));
    bspmv<double>(sim, (const d2*)sim->w, (d2*)sim->V);
    yv = dl(sim, (d2*)sim->V, nb);
    from_positions(sim, yv, y);
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_apply_stage(dp_sim* sim, int32_t stage, const double* r, double* z) {
    if (!sim || !r || !z || stage < 0 || stage > 1) return DP_E_INVALID;
    ABI_BEGIN
    if (sim->stage < 2) fail(DP_E_STATE, "no preconditioner before cpr_fpf_setup");
    int nb = sim->topo.nb;
    int64_t len = 2 * (int64_t)nb;
    if (stage == 0) {
        std::vector<d2> rv;
        to_positions(sim, r, rv);
        DP_HIP(hipMemcpyAsync(sim->w, rv.data(), sizeof(d2) * nb, hipMemcpyHostToDevice, sim->stream));
        if (sim->fp32) {
            to_f32(sim, sim->w, (float*)sim->pr, len);
            ilu_solve<float>(sim, (const f2*)sim->pr, (f2*)sim->pz);
            to_f64(sim, (const float*)sim->pz, sim->V, len);
        } else {
            ilu_solve<double>(sim, (const d2*)sim->w, (d2*)sim->V);
        }
        std::vector<d2> zv = dl(sim, (d2*)sim->V, nb);
        from_positions(sim, zv, z);
    } else {
        int n0 = sim->levels[0].n;
        DP_HIP(hipMemcpyAsync(sim->w, r, sizeof(double) * n0, hipMemcpyHostToDevice, sim->stream));
        if (sim->fp32) {
            to_f32(sim, sim->w, (float*)sim->levels[0].b, n0);
            float* x = amg_vcycle<float>(sim);
            to_f64(sim, x, sim->V, n0);
        } else {
            DP_HIP(hipMemcpyAsync(sim->levels[0].b, sim->w, sizeof(double) * n0, hipMemcpyDeviceToDevice,
                                  sim->stream));
            double* x = amg_vcycle<double>(sim);
            DP_HIP(hipMemcpyAsync(sim->V, x, sizeof(double) * n0, hipMemcpyDeviceToDevice, sim->stream));
        }
        std::vector<double> zv = dl(sim, sim->V, n0);
        std::copy(zv.begin(), zv.end(), z);
    }
    return DP_OK;
    ABI_END(sim)
}


dp_status sim_bench_kernel(dp_sim* sim, int32_t kernel, int32_t reps, double* avg_ms, double* bytes) {
    if (!sim || kernel < 0 || kernel > 5 || reps <= 0) return DP_E_INVALID;
    ABI_BEGIN
    if (sim->stage < 2) fail(DP_E_STATE, "kernel timing needs cpr_fpf_setup first");
    int64_t len = 2 * (int64_t)sim->topo.nb;
    auto launch = [&]() {
        switch (kernel) {
            case 0:
                bspmv<double>(sim, (const d2*)sim->rhs, (d2*)sim->w);
                break;
            case 1:
                if (sim->fp32) ilu_solve<float>(sim, (const f2*)sim->pr, (f2*)sim->pz);
                else ilu_solve<double>(sim, (const d2*)sim->rhs, (d2*)sim->pz);
                break;
            case 2:
                if (sim->fp32) amg_vcycle<float>(sim);
                else amg_vcycle<double>(sim);
                break;
            case 3:
                launch_assemble(sim, sim->dt_assembled);
                break;
            case 5:
                copy_f64(sim, (const double*)sim->rhs, sim->w, len);
                break;
            default:
                cpr_apply(sim, (const double*)sim->rhs, sim->w);
        }
    };
    if (sim->fp32) to_f32(sim, (const double*)sim->rhs, (float*)sim->pr, len);
    launch();
    DP_HIP(hipEventRecord(sim->ev0, sim->stream));
    for (int r = 0; r < reps; ++r) launch();
    DP_HIP(hipEventRecord(sim->ev1, sim->stream));
    DP_HIP(hipEventSynchronize(sim->ev1));
    float ms = 0.f;
    DP_HIP(hipEventElapsedTime(&ms, sim->ev0, sim->ev1));
    if (avg_ms) *avg_ms = ms / reps;
    if (bytes) *bytes = kernel_bytes(sim, kernel);
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_kernel_timer(dp_sim* sim, int32_t kernel, int32_t on) {
    if (!sim || kernel < 0 || kernel >= KT_N) return DP_E_INVALID;
    ABI_BEGIN
    KernelTimer& t = sim->kt[kernel];
    if (on && t.ev.empty()) {
        t.ev.assign(2 * KT_CAP, nullptr);
        for (auto& e : t.ev) DP_HIP(hipEventCreate(&e));
    }
    DP_HIP(hipStreamSynchronize(sim->stream));
    t.on = on != 0;
    if (on) {
        t.used = 0;
        t.dropped = 0;
        t.bytes = 0;
    }
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_kernel_time(dp_sim* sim, int32_t kernel, double* ms_total, int64_t* launches, double* bytes) {
    if (!sim || kernel < 0 || kernel >= KT_N) return DP_E_INVALID;
    ABI_BEGIN
    KernelTimer& t = sim->kt[kernel];
    DP_HIP(hipStreamSynchronize(sim->stream));
    double tot = 0.0;
    for (int i = 0; i < t.used; ++i) {
        float ms = 0.f;
        DP_HIP(hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]));
        tot += ms;
    }
    if (ms_total) *ms_total = tot;
    if (launches) *launches = t.used;
    if (bytes) *bytes = t.bytes;
    return DP_OK;
    ABI_END(sim)
}

dp_status sim_enable_timing(dp_sim* sim, int32_t on) {
    if (!sim) return DP_E_INVALID;
    sim->timing = on != 0;
    for (auto& p : sim->phase) p = PhaseTimer{};
    return DP_OK;
}

dp_status sim_phase_time(dp_sim* sim, int32_t phase, double* ms_total, int64_t* count) {
    if (!sim || phase < 0 || phase >= 5) return DP_E_INVALID;
    if (ms_total) *ms_total = sim->phase[phase].total_ms;
    if (count) *count = sim->phase[phase].count;
    return DP_OK;
}

}  // extern "C"
