// The simulator handle and the device data layout.
//
// Internal block order ("elimination order"), used by every device array:
//   positions n .. 2n-1       fracture nodes: first the cells with i+j+k even
//                             (by cell index), then those with i+j+k odd;
//                             fracture row q = position n+q
//   positions 0 .. n-1        matrix nodes, in the same order: the matrix node
//                             of fracture row q's cell sits at position q
//   positions 2n .. 2n+nw-1   wells
// Node pair q (the two nodes of one cell) thus shares index q in every
// per-cell array, and a sweep over the rows of one colour reads them at unit
// stride.  A fracture row q has 7 coupling slots: 0..5 the fracture
// neighbours in -x,+x,-y,+y,-z,+z (slot absent at the boundary: its column
// points at the row itself and its block is zero) and 6 the matrix node q.
// Matrix row q has one coupling: fracture row q.
// Perforation p couples fracture row perf_q[p] and well perf_well[p] in both
// directions.  Blocks are stored as two planes of 2-vectors (row 0, row 1) so
// that kernels that need only the pressure row read half the bytes.
#pragma once

#include <vector>

#include "common.h"

namespace dp {

struct Topo {
    int nx = 0, ny = 0, nz = 0;
    int n = 0, nw = 0, nb = 0, nperf = 0, nred = 0;
    // device
    int* fcol = nullptr;          // [6*n] slot-major: neighbour position
    unsigned char* fmask = nullptr;  // [n] bit s: slot s has a face
    int* cell = nullptr;          // [n] grid cell of node pair q (geometry inputs only)
    int* fperf = nullptr;         // [n] perforation of fracture row q or -1
    int* perf_q = nullptr;        // [nperf]
    int* perf_well = nullptr;     // [nperf]
    int* well_ptr = nullptr;      // [nw+1] perforations of well w
    int* well_kind = nullptr;     // [nw]
    int* well_ctrl = nullptr;     // [nw] current control
    double* well_target = nullptr;  // [nw] rate (m^3/s) or BHP (Pa) of the current control
    double* well_scale = nullptr;   // [nw] 1/scale of the control row in the convergence norm
    double* tface = nullptr;      // [6*n] transmissibility per slot (0 when absent)
    double* tmf = nullptr;        // [n] sigma km V of node pair q
    double* pvf = nullptr;        // [n] V phi_f of node pair q
    double* pvm = nullptr;        // [n] V phi_m of node pair q
    double* depth = nullptr;      // [n] cell-centre depth of node pair q
    double* wi = nullptr;         // [nperf]
    // host mirrors
    std::vector<int> h_fcol, h_fcell, h_fperf, h_perf_q, h_perf_well, h_well_ptr;  // h_fcell: grid cell of q
    std::vector<unsigned char> h_fmask;
};

template <class T>
struct BMat {
    V2<T>*d0 = nullptr, *d1 = nullptr;    // [nb] diagonal blocks
    V2<T>*f0 = nullptr, *f1 = nullptr;    // [7*n] fracture-row slots
    V2<T>*m0 = nullptr, *m1 = nullptr;    // [n] matrix row -> fracture column
    V2<T>*fw0 = nullptr, *fw1 = nullptr;  // [nperf] fracture row -> well column
    V2<T>*wf0 = nullptr, *wf1 = nullptr;  // [nperf] well row -> fracture column
};

template <class T>
struct ILUF {
    V2<T>*ui0 = nullptr, *ui1 = nullptr;    // [nb] inverse of U's diagonal block
    V2<T>*l0 = nullptr, *l1 = nullptr;      // [7*n] L blocks of fracture rows
    V2<T>*ubw0 = nullptr, *ubw1 = nullptr;  // [nperf] U block fracture row -> well column
    V2<T>*lw0 = nullptr, *lw1 = nullptr;    // [nperf] L block well row -> fracture column
};

struct Csr {
    int n = 0, ncols = 0;
    int64_t nnz = 0;
    int* rowptr = nullptr;
    int* col = nullptr;
    double* val = nullptr;
};

// SELL-64: slices of 64 rows stored column-major, width = longest row of the slice.
struct Sell {
    int n = 0, nslices = 0;
    int64_t nel = 0;
    int* sptr = nullptr;  // [nslices+1] element offset of each slice
    int* col = nullptr;   // [nel]
    void* val = nullptr;  // [nel] of the apply precision
};

// An operator of the V-cycle in the apply precision: SELL-64 when its rows are
// short and even, else CSR processed by G lanes per row.
struct Op {
    // 0 SELL-64; 1 CSR with G lanes per row, U entries per lane and pass;
    // 2 CSR in row blocks of bounded entry count (nb blocks described by desc),
    //   L lanes per row in the row sums
    int kind = 0;
    int n = 0, G = 4, U = 1, L = 4, nb = 0;
    int64_t nnz = 0;
    Sell s;
    int* rowptr = nullptr;
    int* col = nullptr;
    void* val = nullptr;
    int2* desc = nullptr;
};

struct AmgLevel {
    int n = 0, nc = 0;
    Csr A;             // FP64 operator (setup)
    Csr P;             // FP64 interpolation n x nc (not on the coarsest level)
    Csr R;             // FP64 restriction P^T
    int* cf = nullptr;  // [n] 1 = C, -1 = F
    Op Aop, Pop, Rop;   // apply copies
    void* dinv = nullptr;  // [n] 1 / l1 diagonal
    void *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr;  // [n] work vectors
};

struct PhaseTimer {
    double total_ms = 0;
    int64_t count = 0;
};

// Live timing of one kernel (or kernel group) inside the normal calls: while
// enabled, every launch is bracketed by a pair of HIP events on the handle's
// stream (up to KT_CAP launches; the events are read when the timer is queried)
// and its algorithmic bytes are added up.
constexpr int KT_CAP = 2048;
constexpr int KT_N = 5;  // 0 FP64 block SpMV, 1 block ILU(0) solve, 2 row-wise AMG products,
                         // 3 AMG V-cycle, 4 GMRES basis passes
struct KernelTimer {
    bool on = false;
    int used = 0;
    int64_t dropped = 0;
    double bytes = 0;
    std::vector<hipEvent_t> ev;  // 2 * KT_CAP
};

struct KtScope {
    KernelTimer* t;
    hipStream_t st;
    int idx = -1;
    KtScope(KernelTimer* t_, hipStream_t st_) : t(t_), st(st_) {
        if (!t || !t->on) return;
        if (t->used >= KT_CAP) {
            ++t->dropped;
            return;
        }
        idx = t->used++;
        DP_HIP(hipEventRecord(t->ev[2 * idx], st));
    }
    void bytes(double b) {
        if (idx >= 0) t->bytes += b;
    }
    ~KtScope() {
        if (idx >= 0) (void)hipEventRecord(t->ev[2 * idx + 1], st);
    }
};

}  // namespace dp

struct dp_sim {
    dp_sim_desc desc{};
    std::vector<dp_well> wells;
    std::string err;
    hipStream_t stream = nullptr;
    dp::Arena arena;      // persistent allocations (whole workspace)
    dp::Arena hier;       // AMG hierarchy, reset by every setup
    dp::Arena scr;        // setup scratch, reset between phases
    bool fp32 = false;
    int restart = 30;
    dp::Topo topo;

    // physics constants (copied from the descriptor)
    double rho_w_ref, rho_o_ref, p_ref, c_w, c_o, c_r, mu_w, mu_o;
    double swc, sor, n_w, n_o, krw_max, kro_max, gravity, dz;
    double pore_volume = 0.0;  // sum over nodes of V phi (material-balance scale)

    // state, [nb] in elimination order: x = (p, S_w) per node, (p_b, dummy) per well
    dp::d2* x = nullptr;
    dp::d2* x_save = nullptr;   // state at the start of the step (rollback)
    dp::d2* x_sub = nullptr;    // state at the start of the current sub-step (retries)
    dp::d2* acc_old = nullptr;  // [2n nodes] (M_o^n, M_w^n)
    dp::d2* res = nullptr;      // R
    dp::d2* rhs = nullptr;      // decoupled right-hand side -D^-1 R
    dp::d2* dx = nullptr;       // Newton correction
    dp::d2* ft = nullptr;       // adaptive forcing: R + J dx of the previous iteration
    dp::d2* fu = nullptr;       // adaptive forcing: work vector
    std::vector<double> eta_hist;  // linear tolerances of the last timestep's Newton iterations
    // preconditioner apply replayed from a HIP graph (captured after each setup)
    hipGraphExec_t pc_exec = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream the capture runs on
    bool pc_graph_ok = false;
    bool capturing = false;  // kernel timers stay out of a capture
    double dt_assembled = 0.0;
    int stage = 0;              // 0 nothing, 1 assembled, 2 setup done

    dp::BMat<double> J, A;       // Jacobian and decoupled matrix
    dp::BMat<float> A32;         // FP32 copy of the decoupled matrix (mixed form)
    dp::ILUF<double> ilu64;
    dp::ILUF<float> ilu32;

    // level-0 pressure matrix (fracture and well pressures after the exact
    // elimination of the matrix-node pressures): fixed structure, source map
    dp::Csr Ap0;
    int* ap_src = nullptr;  // [nnz] source code of each entry

    // AMG hierarchy (rebuilt by every setup)
    std::vector<dp::AmgLevel> levels;
    void* coarse_inv = nullptr;  // dense inverse of the coarsest operator, apply precision
    int coarse_n = 0;

    // preconditioner work vectors (apply precision), [nb] 2-vectors
    void *pr = nullptr, *pz = nullptr, *pt = nullptr, *pz2 = nullptr;
    void* rpm = nullptr;  // [n] matrix-node pressure residuals of the current apply
    void* st0 = nullptr;  // [8n] level-0 pressure operator of fracture row q by slot: faces 0..5, diagonal, well column
    // GMRES (FP64)
    double* V = nullptr;   // [(restart+1) * 2nb]
    double* Z = nullptr;   // [restart * 2nb]
    double* w = nullptr;   // [2nb]
    double* red_part = nullptr;   // per-block partial sums
    double* red_out = nullptr;    // reduction results (device)
    double red_host[256] = {};    // host copy of reduction results
    double* hpin = nullptr;        // [64] pinned host buffer of the small read-backs (GMRES coefficients, norms, sums)
    int red_blocks = 0;
    int64_t seg_fallbacks = 0;  // AMG products that took the global sort path
    int64_t amg_setups = 0;     // AMG setups begun over the handle's lifetime

    // sort / setup scratch (part of the per-setup region)
    size_t scratch_bytes = 0;

    // timing
    bool timing = false;
    dp::PhaseTimer phase[5];
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t pev[5][2] = {};  // per-phase start/stop (phases nest)
    dp::KernelTimer kt[dp::KT_N];
};
