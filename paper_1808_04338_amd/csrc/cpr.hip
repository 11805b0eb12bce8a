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
    s->pc_graph_ok = false;  // factors and hierarchy changed: recapture before replaying
}

// FPF: z1 = F^-1 r; FP: z1 = 0.  Then the pressure stage, z2 = z1 + R^T e,
// t = r - A z2, z1 = F^-1 t (the caller adds z2 + z1).  Every pointer is fixed between setups, so the whole
// sequence can be captured into a HIP graph when r is the handle's own buffer.
// Folded form (FPF only): r is formed from sc * r64 by the first ILU sweeps and
// the last ones write zout = z2 + z1 in FP64.
template <class T>
static void apply_core(dp_sim* s, const V2<T>* r, const d2* r64 = nullptr, double sc = 1.0,
                       d2* zout = nullptr) {
    V2<T>* z1 = (V2<T>*)s->pz;
    V2<T>* z2 = (V2<T>*)s->pz2;
    V2<T>* t = (V2<T>*)s->pt;
    if (r64 && s->desc.cpr_variant == DP_CPR_FP) fail(DP_E_INVALID, "folded casts need the FPF form");
    // FP starts the pressure stage from z1 = 0 (a fill kernel, not a memset:
    // the sequence may be captured into a graph)
    if (s->desc.cpr_variant == DP_CPR_FP) vec_fill_zero<T>(s, (T*)z1, 2 * (int64_t)s->topo.nb);
    else ilu_solve<T>(s, r, z1, r64, sc);
    bresidual_p<T>(s, r, z1, (T*)s->levels[0].b);
    T* e;
    {
        KtScope ks(s->capturing ? nullptr : &s->kt[3], s->stream);
        e = amg_vcycle<T>(s);
        ks.bytes(kernel_bytes(s, 2));
    }
    bresidual_prol<T>(s, r, z1, e, z2, t);
    ilu_solve<T>(s, t, z1, nullptr, 1.0, zout ? z2 : nullptr, zout);
}

// Capture apply_core on the handle's stream (its input the handle's buffer pr)
// and instantiate it, or update the existing executable graph in place.
// The capture runs on the handle's private stream (the caller's stream may be
// the legacy default stream, which cannot be captured); capturing launches
// nothing, and the graph is then launched on the caller's stream.
static void capture_precond(dp_sim* s) {
    if (!s->cap_stream) DP_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    hipStream_t user = s->stream;
    hipGraph_t g = nullptr;
    DP_HIP(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    s->stream = s->cap_stream;
    s->capturing = true;
    try {
        if (s->fp32) apply_core<float>(s, (const f2*)s->pr);
        else apply_core<double>(s, (const d2*)s->pr);
    } catch (...) {
        s->capturing = false;
        s->stream = user;
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(s->cap_stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        throw;
    }
    s->capturing = false;
    s->stream = user;
    DP_HIP(hipStreamEndCapture(s->cap_stream, &g));
    bool updated = false;
    if (s->pc_exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        updated = hipGraphExecUpdate(s->pc_exec, g, &err_node, &res) == hipSuccess &&
                  res == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(s->pc_exec);
            s->pc_exec = nullptr;
        }
    }
    if (!updated) {
        hipError_t e = hipGraphInstantiate(&s->pc_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            s->pc_exec = nullptr;
            fail(DP_E_DEVICE, std::string("preconditioner graph: ") + hipGetErrorString(e));
        }
    }
    DP_HIP(hipGraphDestroy(g));
    s->pc_graph_ok = true;
}

constexpr int64_t PRECOND_GRAPH_DOF = 1000000;  // auto mode: graphs below this many unknowns

void cpr_apply(dp_sim* s, const double* r, double* z, double scale) {
    int64_t len = 2 * (int64_t)s->topo.nb;
    // graphs pay where launches dominate: small systems (auto), or when forced
    const int mode = s->desc.precond_eager;
    const bool graph = !s->timing && (mode == 2 || (mode == 0 && len < PRECOND_GRAPH_DOF));
    // the core reads the handle's buffer pr, except unscaled eager FP64 (r itself)
    const bool own = s->fp32 || graph || scale != 1.0;
    // eager FP32 CPR-FPF: the casts to and from FP32 run inside the ILU sweeps
    const bool fold = s->fp32 && !graph && s->desc.cpr_variant != DP_CPR_FP;
    if (s->fp32 && !fold) to_f32(s, r, (float*)s->pr, len, scale);
    else if (!s->fp32 && scale != 1.0) vec_scale_to(s, r, scale, (double*)s->pr, len);
    else if (!s->fp32 && graph) copy_f64(s, r, (double*)s->pr, len);
    if (graph) {
        if (!s->pc_graph_ok) capture_precond(s);
        DP_HIP(hipGraphLaunch(s->pc_exec, s->stream));
    } else if (fold) {
        apply_core<float>(s, (const f2*)s->pr, (const d2*)r, scale, (d2*)z);
        return;
    } else if (s->fp32) {
        apply_core<float>(s, (const f2*)s->pr);
    } else {
        apply_core<double>(s, own ? (const d2*)s->pr : (const d2*)r);
    }
    if (s->fp32) add_to_f64(s, (const float*)s->pz2, (const float*)s->pz, z, len);
    else vec_add3<double>(s, (const double*)s->pz2, (const double*)s->pz, z, len);
}

}  // namespace dp
