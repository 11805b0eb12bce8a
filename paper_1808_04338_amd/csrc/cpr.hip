// CPR-FPF preconditioner (setup and apply) and the right-preconditioned
// GMRES(m) solve of the decoupled system (Sec. 3.2, Eq. (14)).
//
// Apply, with F = block ILU(0), R = pick the pressure component of every block:
//   z1 = F^-1 r
//   e  = Vcycle(R (r - A z1))            pressure stage
//   z2 = z1 + R^T e,  t = r - A z2        (one fused kernel)
//   z  = z2 + F^-1 t
// In the mixed form every step above runs in FP32 on an FP32 copy of the
// decoupled matrix; GMRES itself stays in FP64.
#include <cmath>
#include <vector>

#include "kernels.h"

namespace dp {

void cpr_setup(dp_sim* s) {
    launch_decouple(s);
    if (s->fp32) ilu_factor<float>(s);
    else ilu_factor<double>(s);
    amg_extract_level0(s);
    amg_setup(s);
}

template <class T>
static void apply_t(dp_sim* s, const V2<T>* r, double* z64) {
    V2<T>* z1 = (V2<T>*)s->pz;
    V2<T>* z2 = (V2<T>*)s->pz2;
    V2<T>* t = (V2<T>*)s->pt;
    int64_t len = 2 * (int64_t)s->topo.nb;
    ilu_solve<T>(s, r, z1);
    bresidual_p<T>(s, r, z1, (T*)s->levels[0].b);
    T* e = amg_vcycle<T>(s);
    bresidual_prol<T>(s, r, z1, e, z2, t);
    ilu_solve<T>(s, t, z1);
    if constexpr (sizeof(T) == sizeof(double)) {
        vec_add3<double>(s, (const double*)z2, (const double*)z1, z64, len);
    } else {
        add_to_f64(s, (const float*)z2, (const float*)z1, z64, len);
    }
}

void cpr_apply(dp_sim* s, const double* r, double* z) {
    if (s->fp32) {
        int64_t len = 2 * (int64_t)s->topo.nb;
        to_f32(s, r, (float*)s->pr, len);
        apply_t<float>(s, (const f2*)s->pr, z);
    } else {
        apply_t<double>(s, (const d2*)r, z);
    }
}

}  // namespace dp
