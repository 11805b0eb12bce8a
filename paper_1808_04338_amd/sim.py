"""Python handle around the dpsim C ABI.

Device memory (the workspace) and the HIP stream come from PyTorch; every step
of the computation runs in libdpsim.so.  Host arrays use the canonical node
order of the C ABI: node 2c is the fracture and 2c+1 the matrix node of cell c.
"""
import ctypes as C

import numpy as np
import scipy.sparse as sp

from . import _lib as L

_PREC = {"fp64": L.DP_FP64, "fp32": L.DP_FP32}
_CTRL = {"rate": L.DP_CTRL_RATE, "bhp": L.DP_CTRL_BHP, "orate": L.DP_CTRL_ORATE}


def _dp(a):
    return a.ctypes.data_as(L._dptr)


def _ip(a):
    return a.ctypes.data_as(L._iptr)


def _lp(a):
    return a.ctypes.data_as(L._lptr)


def make_desc(model, precision=None, **opts):
    """Fill a DpSimDesc from a model dict (see synth.models).  Returns the
    struct and the Python objects that must stay alive while it is used."""
    keep = []

    def arr(name):
        a = np.ascontiguousarray(model[name], dtype=np.float64)
        keep.append(a)
        return _dp(a)

    d = L.DpSimDesc()
    d.nx, d.ny, d.nz = model["nx"], model["ny"], model["nz"]
    d.dx, d.dy, d.dz = model["dx"], model["dy"], model["dz"]
    d.top_depth = model["top_depth"]
    d.gravity = model["gravity"]
    d.kx, d.ky, d.kz, d.km = arr("kx"), arr("ky"), arr("kz"), arr("km")
    d.phi_f, d.phi_m = arr("phi_f"), arr("phi_m")
    for k in ("sigma", "rho_w_ref", "rho_o_ref", "p_ref", "c_w", "c_o", "mu_w", "mu_o",
              "swc", "sor", "n_w", "n_o", "krw_max", "kro_max"):
        setattr(d, k, float(model[k]))
    d.c_r = float(model.get("c_r", 0.0))
    wells = (L.DpWell * max(len(model["wells"]), 1))()
    for w, wl in enumerate(model["wells"]):
        wells[w].i, wells[w].j, wells[w].k0, wells[w].k1 = wl["i"], wl["j"], wl["k0"], wl["k1"]
        wells[w].kind = L.DP_WELL_INJ if wl["kind"] == "inj" else L.DP_WELL_PROD
        wells[w].control = _CTRL[wl["control"]]
        wells[w].target = wl["target"]
        wells[w].bhp_limit = wl["bhp_limit"]
        wells[w].rw = wl["rw"]
        wells[w].skin = wl["skin"]
        wells[w].wi = float(wl.get("wi", 0.0))
    keep.append(wells)
    d.nwells = len(model["wells"])
    d.wells = wells
    prec = precision or model.get("precond_precision", "fp64")
    d.precond_precision = _PREC[prec]
    d.gmres_restart = int(opts.get("gmres_restart", 30))
    d.lin_maxit = int(opts.get("lin_maxit", 300))
    d.lin_rtol = float(opts.get("lin_rtol", 1e-6))
    d.amg_coarse_max = int(opts.get("amg_coarse_max", 2000))
    d.amg_max_levels = int(opts.get("amg_max_levels", 25))
    d.amg_theta = float(opts.get("amg_theta", 0.25))
    d.amg_trunc = int(opts.get("amg_trunc", 3))
    d.newton_tol = float(opts.get("newton_tol", 1e-3))
    d.max_newton = int(opts.get("max_newton", 20))
    d.max_cuts = int(opts.get("max_cuts", 8))
    d.mb_tol = float(opts.get("mb_tol", 1e-7))
    d.forcing = int(opts.get("forcing", 0))
    d.forcing_eta0 = float(opts.get("forcing_eta0", 0.1))
    d.forcing_gamma = float(opts.get("forcing_gamma", 0.9))
    d.forcing_beta = float(opts.get("forcing_beta", 2.0))
    d.forcing_eta_min = float(opts.get("forcing_eta_min", 1e-8))
    d.forcing_eta_max = float(opts.get("forcing_eta_max", 0.9))
    d.precond_eager = int(opts.get("precond_eager", 0))
    d.decoupling = {"gj": 0, "abf": 1, "ti": 2}[opts.get("decoupling", "gj")]
    d.cpr_variant = {"fpf": 0, "fp": 1}[opts.get("cpr_variant", "fpf")]
    d.newton_stall = int(opts.get("newton_stall", 0))
    d.fail_setup = int(opts.get("fail_setup", 0))
    return d, keep


def footprint(model, precision=None, **opts):
    """Device bytes a handle for this model needs (no GPU call)."""
    lib = L.load()
    d, keep = make_desc(model, precision, **opts)
    nbytes = C.c_size_t()
    L.check(lib.sim_footprint(C.byref(d), C.byref(nbytes)))
    return nbytes.value


class Sim:
    """One simulator handle on one GPU stream."""

    def __init__(self, model, precision=None, device="cuda:0", stream=None, **opts):
        import torch

        self.lib = L.load()
        self.model = model
        d, keep = make_desc(model, precision, **opts)
        self._keep = keep
        nbytes = C.c_size_t()
        L.check(self.lib.sim_footprint(C.byref(d), C.byref(nbytes)))
        self.footprint = nbytes.value
        self.device = torch.device(device)
        self.workspace = torch.empty(self.footprint + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if self.stream != torch.cuda.current_stream(self.device):
            # the library works on self.stream: the caching allocator must not hand this
            # block to another stream's allocation before that stream's work is done
            self.workspace.record_stream(self.stream)
        p0 = np.ascontiguousarray(model["p0"], dtype=np.float64)
        sw0 = np.ascontiguousarray(model["sw0"], dtype=np.float64)
        h = C.c_void_p()
        L.check(self.lib.sim_create(C.byref(d), _dp(p0), _dp(sw0), C.c_void_p(aligned),
                                    C.c_size_t(self.footprint), C.c_void_p(self.stream.cuda_stream),
                                    C.byref(h)))
        self.h = h
        self.n = model["nx"] * model["ny"] * model["nz"]
        self.nw = len(model["wells"])
        n_dof = C.c_int32()
        nnz = C.c_int64()
        self.lib.sim_system_size(self.h, C.byref(n_dof), C.byref(nnz))
        self.n_dof = n_dof.value
        self.nnz = nnz.value

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, code):
        return L.check(code, self.h)

    # -- hot path --------------------------------------------------------------
    def mark_old(self):
        self._chk(self.lib.sim_mark_old(self.h))

    def assemble(self, dt):
        r = C.c_double()
        self._chk(self.lib.assemble_residual_jacobian(self.h, dt, C.byref(r)))
        return r.value

    def setup(self):
        self._chk(self.lib.cpr_fpf_setup(self.h))

    def solve(self, rtol=1e-6, maxit=300, allow_noconv=False):
        its = C.c_int32()
        rel = C.c_double()
        code = self.lib.krylov_solve(self.h, rtol, maxit, C.byref(its), C.byref(rel))
        if code == L.DP_E_NOCONV and allow_noconv:
            return its.value, rel.value
        self._chk(code)
        return its.value, rel.value

    def newton_update(self):
        self._chk(self.lib.newton_update(self.h))

    def newton_step(self, dt, eta=1e-6):
        info = L.DpNewtonInfo()
        self._chk(self.lib.newton_step(self.h, dt, eta, C.byref(info)))
        return {k: getattr(info, k) for k, _ in L.DpNewtonInfo._fields_}

    def timestep(self, dt):
        info = L.DpStepInfo()
        self._chk(self.lib.timestep(self.h, dt, C.byref(info)))
        return {k: getattr(info, k) for k, _ in L.DpStepInfo._fields_}

    # -- state -----------------------------------------------------------------
    def get_state(self):
        p = np.empty(2 * self.n)
        sw = np.empty(2 * self.n)
        bhp = np.empty(max(self.nw, 1))
        self._chk(self.lib.sim_get_state(self.h, _dp(p), _dp(sw), _dp(bhp)))
        return p, sw, bhp[:self.nw]

    def set_state(self, p, sw, bhp=None):
        p = np.ascontiguousarray(p, dtype=np.float64)
        sw = np.ascontiguousarray(sw, dtype=np.float64)
        b = None
        if bhp is not None and self.nw:
            b = np.ascontiguousarray(bhp, dtype=np.float64)
        self._chk(self.lib.sim_set_state(self.h, _dp(p), _dp(sw), _dp(b) if b is not None else None))

    # -- inspection ------------------------------------------------------------
    def export_system(self, which=0):
        rowptr = np.empty(self.n_dof + 1, dtype=np.int32)
        col = np.empty(self.nnz, dtype=np.int32)
        val = np.empty(self.nnz)
        rhs = np.empty(self.n_dof)
        self._chk(self.lib.sim_export_system(self.h, which, _ip(rowptr), _ip(col), _dp(val), _dp(rhs)))
        return sp.csr_matrix((val, col, rowptr), shape=(self.n_dof, self.n_dof)), rhs

    def export_ilu(self):
        nb = self.n_dof // 2
        nnzb = self.nnz // 4
        perm = np.empty(nb, dtype=np.int32)
        br = np.empty(nnzb, dtype=np.int32)
        bc = np.empty(nnzb, dtype=np.int32)
        vals = np.empty(4 * nnzb)
        self._chk(self.lib.sim_export_ilu(self.h, _ip(perm), _ip(br), _ip(bc), _dp(vals)))
        return perm, br, bc, vals.reshape(-1, 2, 2)

    def amg_info(self):
        nl = C.c_int32()
        rows = np.zeros(64, dtype=np.int32)
        nnz = np.zeros(64, dtype=np.int64)
        self._chk(self.lib.sim_amg_info(self.h, C.byref(nl), _ip(rows), _lp(nnz)))
        return nl.value, rows[:nl.value].copy(), nnz[:nl.value].copy()

    TIMED_KERNELS = ("block_spmv_f64", "block_ilu0_solve", "amg_rowwise_products", "amg_vcycle",
                     "gmres_basis_passes")

    def kernel_timer(self, kernel, on=True):
        """Start (reset) or stop the live timer of kernel 0..4 (TIMED_KERNELS)."""
        self._chk(self.lib.sim_kernel_timer(self.h, int(kernel), 1 if on else 0))

    def kernel_time(self, kernel):
        """(total device ms, timed launches, algorithmic bytes) since the timer started."""
        ms = C.c_double()
        n = C.c_int64()
        b = C.c_double()
        self._chk(self.lib.sim_kernel_time(self.h, int(kernel), C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value

    def get_correction(self):
        """The last Krylov solution y of J y = -R, canonical order."""
        y = np.empty(self.n_dof)
        self._chk(self.lib.sim_get_correction(self.h, _dp(y)))
        return y

    def eta_history(self):
        """Records (eta, ||b||, ||r||, ||b - r_prev||, l) of the last timestep's
        Newton iterations, shape (iterations, 5)."""
        n = C.c_int32()
        self._chk(self.lib.sim_eta_history(self.h, None, 0, C.byref(n)))
        out = np.zeros(5 * max(n.value, 1))
        self._chk(self.lib.sim_eta_history(self.h, _dp(out), n.value, C.byref(n)))
        return out[:5 * n.value].reshape(-1, 5).copy()

    def amg_global_sort_products(self):
        """AMG products (one per level and setup) formed by the global sort path."""
        v = C.c_int64()
        self._chk(self.lib.sim_amg_stats(self.h, C.byref(v)))
        return v.value

    def export_amg_level(self, level):
        nl, rows, nnz = self.amg_info()
        n = int(rows[level])
        cf = np.zeros(n, dtype=np.int32)
        arp = np.empty(n + 1, dtype=np.int32)
        acol = np.empty(int(nnz[level]), dtype=np.int32)
        aval = np.empty(int(nnz[level]))
        pnnz = C.c_int64()
        self._chk(self.lib.sim_export_amg_level(self.h, level, None, None, None, None, None, None, None,
                                                C.byref(pnnz)))
        prp = np.empty(n + 1, dtype=np.int32)
        pcol = np.empty(max(pnnz.value, 1), dtype=np.int32)
        pval = np.empty(max(pnnz.value, 1))
        last = level == nl - 1
        self._chk(self.lib.sim_export_amg_level(self.h, level, None if last else _ip(cf), _ip(arp),
                                                _ip(acol), _dp(aval), None if last else _ip(prp),
                                                None if last else _ip(pcol), None if last else _dp(pval),
                                                C.byref(pnnz)))
        A = sp.csr_matrix((aval, acol, arp), shape=(n, n))
        out = {"A": A}
        if not last:
            nc = int(rows[level + 1])
            out["cf"] = cf
            out["P"] = sp.csr_matrix((pval[:pnnz.value], pcol[:pnnz.value], prp), shape=(n, nc))
        return out

    def apply_precond(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(r)
        self._chk(self.lib.sim_apply_precond(self.h, _dp(r), _dp(z)))
        return z

    def apply_stage(self, stage, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(r)
        self._chk(self.lib.sim_apply_stage(self.h, stage, _dp(r), _dp(z)))
        return z

    def apply_matrix(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        self._chk(self.lib.sim_apply_matrix(self.h, _dp(x), _dp(y)))
        return y

    KERNELS = ["block_spmv_f64", "block_ilu0_solve", "amg_vcycle", "assemble", "cpr_fpf_apply",
               "copy_f64"]

    def bench_kernel(self, kernel, reps=20):
        """(average ms per launch, algorithmic bytes per launch) of a kernel group."""
        ms = C.c_double()
        b = C.c_double()
        self._chk(self.lib.sim_bench_kernel(self.h, kernel, reps, C.byref(ms), C.byref(b)))
        return ms.value, b.value

    def bench_kernels(self, reps=20):
        """All kernel groups; the entry with the largest time per apply first."""
        out = []
        for k, name in enumerate(self.KERNELS):
            ms, b = self.bench_kernel(k, reps)
            out.append(dict(name=name, ms=ms, bytes=b, gbs=(b / (ms * 1e-3) / 1e9) if b else None))
        return out

    def enable_timing(self, on=True):
        self._chk(self.lib.sim_enable_timing(self.h, 1 if on else 0))

    def phase_time(self, phase):
        ms = C.c_double()
        cnt = C.c_int64()
        self._chk(self.lib.sim_phase_time(self.h, phase, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value


def batch_timestep(sims, dts):
    """Advance several handles concurrently (each on its own stream)."""
    lib = L.load()
    n = len(sims)
    arr = (C.c_void_p * n)(*[s.h for s in sims])
    dt = np.ascontiguousarray(dts, dtype=np.float64)
    infos = (L.DpStepInfo * n)()
    st = np.zeros(n, dtype=np.int32)
    lib.batch_timestep(arr, n, _dp(dt), infos, _ip(st))
    out = []
    for i in range(n):
        out.append(dict({k: getattr(infos[i], k) for k, _ in L.DpStepInfo._fields_}, status=int(st[i])))
    return out


def dense_inverse_selftest(a, device="cuda:0"):
    """Invert a dense matrix with the library's coarse-level MFMA Gauss-Jordan."""
    import torch

    lib = L.load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    npad = (n + 31) // 32 * 32
    ws = torch.empty(16 * npad * npad + 65536 + 256, dtype=torch.uint8, device=device)
    base = (ws.data_ptr() + 255) & ~255
    out = np.empty_like(a)
    st = torch.cuda.current_stream(torch.device(device))
    code = lib.dp_selftest_dense_inverse(_dp(a), n, _dp(out), C.c_void_p(base),
                                         C.c_size_t(16 * npad * npad + 65536), C.c_void_p(st.cuda_stream))
    L.check(code)
    return out


def dense_inverse_noalloc(a, device="cuda:0"):
    """The same inverse with the library's static device scratch (no workspace)."""
    import torch

    lib = L.load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    out = np.empty_like(a)
    st = torch.cuda.current_stream(torch.device(device))
    L.check(lib.dp_selftest_dense_inverse_noalloc(_dp(a), n, _dp(out), C.c_void_p(st.cuda_stream)))
    return out
