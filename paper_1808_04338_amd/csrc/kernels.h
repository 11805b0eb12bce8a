// Host-side launchers of the device kernels (one stream per handle).
#pragma once

#include "sim.h"

namespace dp {

struct Phys;
Phys make_phys(const dp_sim* s);

// assemble.hip
void launch_geometry(dp_sim* s, const double* kx, const double* ky, const double* kz,
                     const double* km, const double* phi_f, const double* phi_m,
                     const int* perf_cell, const double* perf_rw, const double* perf_skin,
                     const double* perf_wi);
void launch_accumulation(dp_sim* s, const d2* x, d2* acc);
void launch_assemble(dp_sim* s, double dt);
struct ResNorm {
    double cnv;  // scaled max-norm
    double mb;   // scaled material balance (larger phase)
};
ResNorm residual_norm(dp_sim* s, double dt);
void launch_newton_update(dp_sim* s);

// linalg.hip
void launch_decouple(dp_sim* s);
template <class T> void bspmv(dp_sim* s, const V2<T>* x, V2<T>* y);
void jspmv(dp_sim* s, const d2* x, d2* y);  // y = J x, undecoupled Jacobian
// Algorithmic bytes of one launch of a timed kernel (0 FP64 block SpMV, 1 block
// ILU(0) solve in the preconditioner precision, 2 AMG V-cycle, 3 assembly).
double kernel_bytes(dp_sim* s, int kernel);
void copy_f64(dp_sim* s, const double* x, double* y, int64_t len);
template <class T> void vec_fill_zero(dp_sim* s, T* x, int64_t len);
template <class T> void bresidual(dp_sim* s, const V2<T>* b, const V2<T>* x, V2<T>* y);
template <class T> void bresidual_p(dp_sim* s, const V2<T>* b, const V2<T>* x, T* yp);
template <class T>
void bresidual_prol(dp_sim* s, const V2<T>* b, const V2<T>* x, const T* e, V2<T>* x2, V2<T>* y);
template <class T> void ilu_factor(dp_sim* s);
// z = (LU)^-1 r.  With r64 given, r is formed on the fly as (T)(sc * r64) and
// written to r (then writable) on first use; with zout given, every final z
// entry is also written as zout = (double)(zadd + z).  Both fold the precision
// casts around the FP32 preconditioner into the sweeps.
template <class T>
void ilu_solve(dp_sim* s, const V2<T>* r, V2<T>* z, const d2* r64 = nullptr, double sc = 1.0,
               const V2<T>* zadd = nullptr, d2* zout = nullptr);

// krylov.hip (FP64 vectors of length len doubles)
void vec_copy(dp_sim* s, const double* x, double* y, int64_t len);
void vec_zero(dp_sim* s, double* x, int64_t len);
void vec_scale_to(dp_sim* s, const double* x, double alpha, double* y, int64_t len);
void vec_axpy(dp_sim* s, double alpha, const double* x, double* y, int64_t len);
void to_f32(dp_sim* s, const double* x, float* y, int64_t len, double a = 1.0);  // y = (float)(a x)
void to_f64(dp_sim* s, const float* x, double* y, int64_t len);
void add_to_f64(dp_sim* s, const float* a, const float* b, double* y, int64_t len);
template <class T> void vec_add3(dp_sim* s, const T* a, const T* b, T* y, int64_t len);
// reductions: results land in s->red_out (device) and are copied to s->red_host
// out_i = V_i . w (i < k)
void dot_multi(dp_sim* s, const double* V, int64_t ld, int k, const double* w, int64_t len, double* out);
// u = w - sum_i h_i V_i; out_i = V_i . u (i < k), out_k = u . u
void gs_update_dot_norm(dp_sim* s, const double* V, int64_t ld, int k, const double* h, const double* w,
                        double* u, int64_t len, double* out);
// V_k = (V_k - sum_i a_i V_i) * sc in place; out_i = V_i . w (i <= k)
void gs_finish_dot(dp_sim* s, double* V, int64_t ld, int k, const double* a, double sc, const double* w,
                   int64_t len, double* out);
void norm2(dp_sim* s, const double* x, int64_t len, double* out);
void combine(dp_sim* s, const double* Z, int64_t ld, int k, const double* y, double* x, int64_t len);

// amg.hip
void amg_extract_level0(dp_sim* s);
void amg_setup(dp_sim* s);
template <class T> T* amg_vcycle(dp_sim* s);  // solves levels[0] with b = levels[0].b; returns x
void amg_release(dp_sim* s);

// cpr.hip
void cpr_setup(dp_sim* s);
void cpr_apply(dp_sim* s, const double* r, double* z, double scale = 1.0);  // z = M^-1 (scale r), FP64 [2nb]

}  // namespace dp
