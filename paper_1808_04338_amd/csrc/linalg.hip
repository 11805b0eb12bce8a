// Decoupling, block sparse matrix-vector products and block ILU(0).
//
// Every kernel covers the three row groups of the elimination order in one
// launch: blocks [0, bm) take matrix rows, [bm, bm+bf) fracture rows and the
// last nw blocks one well each.  A thread owns one row and writes only it.
#include "kernels.h"

namespace dp {

// ---------------------------------------------------------------------------
// Decoupling D^-1 J, D^-1 b (Eq. (14)): every block of node row i is multiplied
// by the 2x2 matrix Q = D_i^-1; well rows are copied; b = -R.
//   DP_DEC_GJ   one Gauss-Jordan step with a = J_ii: Q = [[1, -a01/a11], [0, 1]]
//   DP_DEC_ABF  alternate block factorisation: Q = J_ii^-1
//   DP_DEC_TI   true-IMPES: Q = [[1, -c01/c11], [0, 1]], c_i the sum of block column i
//               (gathered from the transposed positions: a face slot s of row q
//               is mirrored by slot s^1 of the neighbour's row)
// ---------------------------------------------------------------------------
struct DecArgs {
    BMat<double> J, A;
    BMat<float> A32;
    bool f32;
    int variant;
    const d2* R;
    d2* b;
    const unsigned char* fmask;
    const int* fcol;
    const int* fperf;
    const int* well_ptr;
    int n, nw;
};

struct Q2 {
    double q00, q01, q10, q11;
};

__device__ inline void dec_pair(const d2* s0, const d2* s1, d2* o0, d2* o1, float2* p0, float2* p1,
                                int64_t i, const Q2& q, bool f32) {
    d2 r0 = s0[i], r1 = s1[i];
    d2 a0 = mk2(q.q00 * r0.x + q.q01 * r1.x, q.q00 * r0.y + q.q01 * r1.y);
    d2 a1 = mk2(q.q10 * r0.x + q.q11 * r1.x, q.q10 * r0.y + q.q11 * r1.y);
    o0[i] = a0;
    o1[i] = a1;
    if (f32) {
        p0[i] = make_float2((float)a0.x, (float)a0.y);
        p1[i] = make_float2((float)a1.x, (float)a1.y);
    }
}

__global__ void __launch_bounds__(256) decouple_kernel(DecArgs a, int bm, int bf) {
    int b = blockIdx.x;
    int n = a.n;
    float2* n0 = nullptr;
    bool f32 = a.f32;
#define F32P(p) (f32 ? (float2*)(p) : n0)
    if (b < bm + bf) {
        int pos = b * blockDim.x + threadIdx.x - (b < bm ? 0 : bm * (int)blockDim.x);
        bool frac = b >= bm;
        if (pos >= n) return;
        int row = frac ? n + pos : pos;
        d2 d0 = a.J.d0[row], d1 = a.J.d1[row];
        const int p = frac ? a.fperf[pos] : -1;
        Q2 q{1.0, 0.0, 0.0, 1.0};
        if (a.variant == DP_DEC_ABF) {
            double det = d0.x * d1.y - d0.y * d1.x;
            q = Q2{d1.y / det, -d0.y / det, -d1.x / det, d0.x / det};
        } else if (a.variant == DP_DEC_TI) {
            // saturation column of the block column sum: J_ii plus every block
            // that couples another row to this node
            double c01 = d0.y, c11 = d1.y;
            if (!frac) {
                int64_t e = (int64_t)6 * n + pos;  // matrix slot of its fracture row
                c01 += a.J.f0[e].y;
                c11 += a.J.f1[e].y;
            } else {
                unsigned mask = a.fmask[pos];
                for (int s = 0; s < 6; ++s) {
                    if (!(mask & (1u << s))) continue;
                    int nq = a.fcol[(int64_t)s * n + pos] - n;
                    int64_t e = (int64_t)(s ^ 1) * n + nq;
                    c01 += a.J.f0[e].y;
                    c11 += a.J.f1[e].y;
                }
                c01 += a.J.m0[pos].y;  // its matrix node
                c11 += a.J.m1[pos].y;
                if (p >= 0) {
                    c01 += a.J.wf0[p].y;
                    c11 += a.J.wf1[p].y;
                }
            }
            q.q01 = -c01 / c11;
        } else {
            q.q01 = -(d0.y / d1.y);
        }
        dec_pair(a.J.d0, a.J.d1, a.A.d0, a.A.d1, F32P(a.A32.d0), F32P(a.A32.d1), row, q, f32);
        d2 r = a.R[row];
        double b0 = -r.x, b1 = -r.y;
        a.b[row] = mk2(q.q00 * b0 + q.q01 * b1, q.q10 * b0 + q.q11 * b1);
        if (!frac) {
            dec_pair(a.J.m0, a.J.m1, a.A.m0, a.A.m1, F32P(a.A32.m0), F32P(a.A32.m1), pos, q, f32);
        } else {
            for (int s = 0; s < 7; ++s)
                dec_pair(a.J.f0, a.J.f1, a.A.f0, a.A.f1, F32P(a.A32.f0), F32P(a.A32.f1),
                         (int64_t)s * n + pos, q, f32);
            if (p >= 0)
                dec_pair(a.J.fw0, a.J.fw1, a.A.fw0, a.A.fw1, F32P(a.A32.fw0), F32P(a.A32.fw1), p, q,
                         f32);
        }
    } else {
        int w = b - bm - bf;
        int row = 2 * n + w;
        const Q2 id{1.0, 0.0, 0.0, 1.0};
        if (threadIdx.x == 0) {
            dec_pair(a.J.d0, a.J.d1, a.A.d0, a.A.d1, F32P(a.A32.d0), F32P(a.A32.d1), row, id, f32);
            d2 r = a.R[row];
            a.b[row] = mk2(-r.x, -r.y);
        }
        for (int p = a.well_ptr[w] + threadIdx.x; p < a.well_ptr[w + 1]; p += blockDim.x)
            dec_pair(a.J.wf0, a.J.wf1, a.A.wf0, a.A.wf1, F32P(a.A32.wf0), F32P(a.A32.wf1), p, id, f32);
    }
#undef F32P
}

void launch_decouple(dp_sim* s) {
    Topo& t = s->topo;
    DecArgs a;
    a.J = s->J;
    a.A = s->A;
    a.A32 = s->A32;
    a.f32 = s->fp32;
    a.variant = s->desc.decoupling;
    a.R = s->res;
    a.b = s->rhs;
    a.fmask = t.fmask;
    a.fcol = t.fcol;
    a.fperf = t.fperf;
    a.well_ptr = t.well_ptr;
    a.n = t.n;
    a.nw = t.nw;
    int bm = ceil_div(t.n, 256);
    decouple_kernel<<<2 * bm + t.nw, 256, 0, s->stream>>>(a, bm, bm);
    DP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Block SpMV.  MODE_Y: y = A x.  MODE_RES: y = b - A x.  MODE_PROL:
// x2 = x + (e, 0), y = b - A x2, x2 written out, where e is the pressure
// correction: e is given on the reduced pressure system (fracture rows, then
// wells) and the matrix-node part is recovered as e_m = (r_m - a_mf e_f)/a_mm.
// MODE_RESP (separate kernel below): the pressure residual restricted to the
// reduced system.
// ---------------------------------------------------------------------------
enum { MODE_Y = 0, MODE_RES = 1, MODE_RESP = 2, MODE_PROL = 3 };

template <class T>
struct SpArgs {
    BMat<T> A;
    const V2<T>* x;
    const V2<T>* b;
    const T* e;     // MODE_PROL: [n + nw] pressure correction on the reduced system
    const T* rpm;   // MODE_PROL: [n] matrix-node pressure residuals
    V2<T>* y;       // MODE_Y/RES/PROL
    T* yp;          // MODE_RESP
    V2<T>* x2;      // MODE_PROL
    const int* fcol;
    const int* fperf;
    const int* perf_q;
    const int* perf_well;
    const int* well_ptr;
    int n, nw;
};

template <class T, int MODE>
__device__ inline V2<T> xval(const SpArgs<T>& a, int pos) {
    V2<T> v = a.x[pos];
    if (MODE == MODE_PROL) {
        if (pos < a.n) {
            T ef = a.e[pos];
            v.x += (a.rpm[pos] - a.A.m0[pos].x * ef) / a.A.d0[pos].x;
        } else {
            v.x += a.e[pos - a.n];
        }
    }
    return v;
}

template <class T, int MODE>
__device__ inline void acc_blk(const V2<T>* p0, const V2<T>* p1, int64_t i, V2<T> v, T& y0, T& y1) {
    V2<T> r0 = p0[i];
    y0 += r0.x * v.x + r0.y * v.y;
    if (MODE != MODE_RESP) {
        V2<T> r1 = p1[i];
        y1 += r1.x * v.x + r1.y * v.y;
    }
}

template <class T, int MODE>
__device__ inline void sp_store(const SpArgs<T>& a, int row, T y0, T y1, V2<T> xself) {
    if (MODE == MODE_Y) {
        a.y[row] = mk2<T>(y0, y1);
    } else if (MODE == MODE_RES) {
        V2<T> bb = a.b[row];
        a.y[row] = mk2<T>(bb.x - y0, bb.y - y1);
    } else if (MODE == MODE_RESP) {
        a.yp[row] = a.b[row].x - y0;
    } else {
        V2<T> bb = a.b[row];
        a.y[row] = mk2<T>(bb.x - y0, bb.y - y1);
        a.x2[row] = xself;
    }
}

template <class T, int MODE>
__global__ void __launch_bounds__(256) spmv_kernel(SpArgs<T> a, int bm, int bf) {
    __shared__ T sh0[256 / WAVE], sh1[256 / WAVE];
    int b = blockIdx.x;
    int n = a.n;
    if (b < bm) {
        int c = xcd_block(b, bm) * blockDim.x + threadIdx.x;
        if (c >= n) return;
        T y0 = 0, y1 = 0;
        V2<T> xs = xval<T, MODE>(a, c);
        acc_blk<T, MODE>(a.A.d0, a.A.d1, c, xs, y0, y1);
        acc_blk<T, MODE>(a.A.m0, a.A.m1, c, xval<T, MODE>(a, n + c), y0, y1);
        sp_store<T, MODE>(a, c, y0, y1, xs);
    } else if (b < bm + bf) {
        int q = xcd_block(b - bm, bf) * blockDim.x + threadIdx.x;
        if (q >= n) return;
        int row = n + q;
        T y0 = 0, y1 = 0;
        V2<T> xs = xval<T, MODE>(a, row);
        acc_blk<T, MODE>(a.A.d0, a.A.d1, row, xs, y0, y1);
#pragma unroll
        for (int s = 0; s < 6; ++s)
            acc_blk<T, MODE>(a.A.f0, a.A.f1, (int64_t)s * n + q, xval<T, MODE>(a, a.fcol[s * n + q]), y0, y1);
        acc_blk<T, MODE>(a.A.f0, a.A.f1, (int64_t)6 * n + q, xval<T, MODE>(a, q), y0, y1);
        int p = a.fperf[q];
        if (p >= 0) acc_blk<T, MODE>(a.A.fw0, a.A.fw1, p, xval<T, MODE>(a, 2 * n + a.perf_well[p]), y0, y1);
        sp_store<T, MODE>(a, row, y0, y1, xs);
    } else {
        int w = b - bm - bf;
        int row = 2 * n + w;
        T y0 = 0, y1 = 0;
        for (int p = a.well_ptr[w] + threadIdx.x; p < a.well_ptr[w + 1]; p += blockDim.x)
            acc_blk<T, MODE>(a.A.wf0, a.A.wf1, p, xval<T, MODE>(a, n + a.perf_q[p]), y0, y1);
        y0 = wave_sum(y0);
        y1 = wave_sum(y1);
        if (threadIdx.x % WAVE == 0) {
            sh0[threadIdx.x / WAVE] = y0;
            sh1[threadIdx.x / WAVE] = y1;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            T s0 = 0, s1 = 0;
            for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) {
                s0 += sh0[i];
                s1 += sh1[i];
            }
            V2<T> xs = xval<T, MODE>(a, row);
            acc_blk<T, MODE>(a.A.d0, a.A.d1, row, xs, s0, s1);
            sp_store<T, MODE>(a, row, s0, s1, xs);
        }
    }
}

// Pressure residual of the reduced system: for fracture row q of cell c,
// r_f = (b - A x)_f,0 and r_m = (b - A x)_m,0 (the two blocks of the matrix
// row recomputed here), rr_q = r_f - a_fm (r_m / a_mm), r_m kept for the
// back-substitution; for well w, rr_{n+w} = (b - A x)_w,0.  Only the pressure
// rows of the blocks are read.
template <class T>
__global__ void __launch_bounds__(256) presid_red_kernel(SpArgs<T> a, int bf, T* rr, T* rpm) {
    __shared__ T sh0[256 / WAVE];
    int b = blockIdx.x;
    int n = a.n;
    if (b < bf) {
        int q = xcd_block(b, bf) * blockDim.x + threadIdx.x;
        if (q >= n) return;
        int row = n + q;
        int c = q;  // the matrix node of fracture row q
        T y0 = 0, dummy = 0;
        acc_blk<T, MODE_RESP>(a.A.d0, a.A.d1, row, a.x[row], y0, dummy);
#pragma unroll
        for (int s = 0; s < 6; ++s)
            acc_blk<T, MODE_RESP>(a.A.f0, a.A.f1, (int64_t)s * n + q, a.x[a.fcol[s * n + q]], y0, dummy);
        V2<T> xm = a.x[c];
        acc_blk<T, MODE_RESP>(a.A.f0, a.A.f1, (int64_t)6 * n + q, xm, y0, dummy);
        int p = a.fperf[q];
        if (p >= 0) acc_blk<T, MODE_RESP>(a.A.fw0, a.A.fw1, p, a.x[2 * n + a.perf_well[p]], y0, dummy);
        T rf = a.b[row].x - y0;
        T ym = 0;
        acc_blk<T, MODE_RESP>(a.A.d0, a.A.d1, c, xm, ym, dummy);
        acc_blk<T, MODE_RESP>(a.A.m0, a.A.m1, c, a.x[row], ym, dummy);
        T rm = a.b[c].x - ym;
        rpm[c] = rm;
        rr[q] = rf - a.A.f0[(int64_t)6 * n + q].x * (rm / a.A.d0[c].x);
    } else {
        int w = b - bf;
        int row = 2 * n + w;
        T y0 = 0, dummy = 0;
        for (int p = a.well_ptr[w] + threadIdx.x; p < a.well_ptr[w + 1]; p += blockDim.x)
            acc_blk<T, MODE_RESP>(a.A.wf0, a.A.wf1, p, a.x[n + a.perf_q[p]], y0, dummy);
        y0 = wave_sum(y0);
        if (threadIdx.x % WAVE == 0) sh0[threadIdx.x / WAVE] = y0;
        __syncthreads();
        if (threadIdx.x == 0) {
            T s0 = 0;
            for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) s0 += sh0[i];
            acc_blk<T, MODE_RESP>(a.A.d0, a.A.d1, row, a.x[row], s0, dummy);
            rr[n + w] = a.b[row].x - s0;
        }
    }
}

template <class T>
static SpArgs<T> sp_args(dp_sim* s, const BMat<T>& A) {
    Topo& t = s->topo;
    SpArgs<T> a{};
    a.A = A;
    a.fcol = t.fcol;
    a.fperf = t.fperf;
    a.perf_q = t.perf_q;
    a.perf_well = t.perf_well;
    a.well_ptr = t.well_ptr;
    a.n = t.n;
    a.nw = t.nw;
    a.rpm = (const T*)s->rpm;
    return a;
}

template <class T, int MODE>
static void sp_launch(dp_sim* s, const SpArgs<T>& a) {
    int bm = ceil_div(s->topo.n, 256);
    spmv_kernel<T, MODE><<<2 * bm + s->topo.nw, 256, 0, s->stream>>>(a, bm, bm);
    DP_LAUNCH_CHECK();
}

template <class T>
const BMat<T>& amat(dp_sim* s);
template <>
const BMat<double>& amat<double>(dp_sim* s) { return s->A; }
template <>
const BMat<float>& amat<float>(dp_sim* s) { return s->A32; }

template <class T>
void bspmv(dp_sim* s, const V2<T>* x, V2<T>* y) {
    SpArgs<T> a = sp_args<T>(s, amat<T>(s));
    a.x = x;
    a.y = y;
    sp_launch<T, MODE_Y>(s, a);
}
template <class T>
void bresidual(dp_sim* s, const V2<T>* b, const V2<T>* x, V2<T>* y) {
    SpArgs<T> a = sp_args<T>(s, amat<T>(s));
    a.x = x;
    a.b = b;
    a.y = y;
    sp_launch<T, MODE_RES>(s, a);
}
template <class T>
void bresidual_p(dp_sim* s, const V2<T>* b, const V2<T>* x, T* rr) {
    SpArgs<T> a = sp_args<T>(s, amat<T>(s));
    a.x = x;
    a.b = b;
    int bf = ceil_div(s->topo.n, 256);
    presid_red_kernel<T><<<bf + s->topo.nw, 256, 0, s->stream>>>(a, bf, rr, (T*)s->rpm);
    DP_LAUNCH_CHECK();
}
template <class T>
void bresidual_prol(dp_sim* s, const V2<T>* b, const V2<T>* x, const T* e, V2<T>* x2, V2<T>* y) {
    SpArgs<T> a = sp_args<T>(s, amat<T>(s));
    a.x = x;
    a.b = b;
    a.e = e;
    a.x2 = x2;
    a.y = y;
    sp_launch<T, MODE_PROL>(s, a);
}

// y = J x with the undecoupled Jacobian (FP64)
void jspmv(dp_sim* s, const d2* x, d2* y) {
    SpArgs<double> a = sp_args<double>(s, s->J);
    a.x = x;
    a.y = y;
    sp_launch<double, MODE_Y>(s, a);
}

template void bspmv<double>(dp_sim*, const d2*, d2*);
template void bspmv<float>(dp_sim*, const f2*, f2*);
template void bresidual<double>(dp_sim*, const d2*, const d2*, d2*);
template void bresidual<float>(dp_sim*, const f2*, const f2*, f2*);
template void bresidual_p<double>(dp_sim*, const d2*, const d2*, double*);
template void bresidual_p<float>(dp_sim*, const f2*, const f2*, float*);
template void bresidual_prol<double>(dp_sim*, const d2*, const d2*, const double*, d2*, d2*);
template void bresidual_prol<float>(dp_sim*, const f2*, const f2*, const float*, f2*, f2*);

// ---------------------------------------------------------------------------
// Block ILU(0) factorisation in the elimination order (matrix nodes, even
// fracture nodes, odd fracture nodes, wells).  The matrix node of a cell couples
// only to its fracture node, so its elimination is exact; even fracture rows
// couple only to odd ones, so their rows see only the matrix-node update; odd
// rows take updates from their matrix node and from every even neighbour; a
// well row takes updates from all its perforated rows, even ones first.
// ---------------------------------------------------------------------------
template <class T>
struct IluArgs {
    BMat<T> A;
    ILUF<T> F;
    const int* fcol;
    const unsigned char* fmask;
    const int* fperf;
    const int* perf_q;
    const int* perf_well;
    const int* well_ptr;
    int n, nw, nred;
};

// even (red) rows: L_rm = A_rm U_mm^-1, U_rr = A_rr - L_rm A_mr
template <class T>
__global__ void ilu_red_kernel(IluArgs<T> a) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nred) return;
    int n = a.n;
    int c = q;  // the matrix node of fracture row q
    Blk<T> um_inv = binv(ldb(a.A.d0, a.A.d1, c));
    stb(a.F.ui0, a.F.ui1, c, um_inv);
    Blk<T> l = bmm(ldb(a.A.f0, a.A.f1, (int64_t)6 * n + q), um_inv);
    stb(a.F.l0, a.F.l1, (int64_t)6 * n + q, l);
    Blk<T> d = bsub(ldb(a.A.d0, a.A.d1, n + q), bmm(l, ldb(a.A.m0, a.A.m1, c)));
    stb(a.F.ui0, a.F.ui1, n + q, binv(d));
    int p = a.fperf[q];
    if (p >= 0) stb(a.F.ubw0, a.F.ubw1, p, ldb(a.A.fw0, a.A.fw1, p));
}

// odd (black) rows
template <class T>
__global__ void ilu_black_kernel(IluArgs<T> a) {
    int q = a.nred + blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n) return;
    int n = a.n;
    int c = q;  // the matrix node of fracture row q
    Blk<T> um_inv = binv(ldb(a.A.d0, a.A.d1, c));
    stb(a.F.ui0, a.F.ui1, c, um_inv);
    Blk<T> l6 = bmm(ldb(a.A.f0, a.A.f1, (int64_t)6 * n + q), um_inv);
    stb(a.F.l0, a.F.l1, (int64_t)6 * n + q, l6);
    Blk<T> d = bsub(ldb(a.A.d0, a.A.d1, n + q), bmm(l6, ldb(a.A.m0, a.A.m1, c)));
    int p = a.fperf[q];
    int w = p >= 0 ? a.perf_well[p] : -1;
    Blk<T> ubw = {0, 0, 0, 0};
    if (p >= 0) ubw = ldb(a.A.fw0, a.A.fw1, p);
    unsigned mask = a.fmask[q];
    for (int s = 0; s < 6; ++s) {
        Blk<T> l = {0, 0, 0, 0};
        if (mask & (1u << s)) {
            int rpos = a.fcol[s * n + q];
            int rq = rpos - n;
            l = bmm(ldb(a.A.f0, a.A.f1, (int64_t)s * n + q), ldb(a.F.ui0, a.F.ui1, rpos));
            // the even row's block pointing back at this row sits in the opposite slot
            d = bsub(d, bmm(l, ldb(a.A.f0, a.A.f1, (int64_t)(s ^ 1) * n + rq)));
            int pr = a.fperf[rq];
            if (w >= 0 && pr >= 0 && a.perf_well[pr] == w) ubw = bsub(ubw, bmm(l, ldb(a.A.fw0, a.A.fw1, pr)));
        }
        stb(a.F.l0, a.F.l1, (int64_t)s * n + q, l);
    }
    stb(a.F.ui0, a.F.ui1, n + q, binv(d));
    if (p >= 0) stb(a.F.ubw0, a.F.ubw1, p, ubw);
}

// well rows: one wavefront per well.  The well row's entries are eliminated in
// elimination order: first every even (red) perforation, l_p = A_wp U_pp^-1,
// which fills the well row at the odd perforations of the same well that
// couple to it; then every odd (black) perforation, whose entry gathers that
// fill (A_wp - sum l_r U_rp over its even neighbours perforated by the same
// well) before l_p = (.) U_pp^-1.  U_ww = A_ww - sum_p l_p U_pw, summed per
// lane and then across the wave in a fixed order.
template <class T>
__global__ void __launch_bounds__(WAVE) ilu_well_kernel(IluArgs<T> a) {
    int w = blockIdx.x;
    int lane = threadIdx.x;
    int n = a.n;
    int p0 = a.well_ptr[w], p1 = a.well_ptr[w + 1];
    Blk<T> acc = {0, 0, 0, 0};
    for (int p = p0 + lane; p < p1; p += WAVE) {
        int q = a.perf_q[p];
        if (q >= a.nred) continue;
        Blk<T> l = bmm(ldb(a.A.wf0, a.A.wf1, p), ldb(a.F.ui0, a.F.ui1, n + q));
        stb(a.F.lw0, a.F.lw1, p, l);
        Blk<T> t = bmm(l, ldb(a.F.ubw0, a.F.ubw1, p));
        acc = badd(acc, t);
    }
    __syncthreads();  // the even perforations' l_p are visible to the whole wave
    for (int p = p0 + lane; p < p1; p += WAVE) {
        int q = a.perf_q[p];
        if (q < a.nred) continue;
        Blk<T> lw = ldb(a.A.wf0, a.A.wf1, p);
        unsigned mask = a.fmask[q];
        for (int s = 0; s < 6; ++s) {
            if (!(mask & (1u << s))) continue;
            int rq = a.fcol[s * n + q] - n;
            int pr = a.fperf[rq];
            if (rq < a.nred && pr >= 0 && a.perf_well[pr] == w) {
                // the even row's block pointing back at this row sits in the opposite slot
                Blk<T> u = ldb(a.A.f0, a.A.f1, (int64_t)(s ^ 1) * n + rq);
                lw = bsub(lw, bmm(ldb(a.F.lw0, a.F.lw1, pr), u));
            }
        }
        Blk<T> l = bmm(lw, ldb(a.F.ui0, a.F.ui1, n + q));
        stb(a.F.lw0, a.F.lw1, p, l);
        acc = badd(acc, bmm(l, ldb(a.F.ubw0, a.F.ubw1, p)));
    }
    acc.a00 = wave_sum(acc.a00);
    acc.a01 = wave_sum(acc.a01);
    acc.a10 = wave_sum(acc.a10);
    acc.a11 = wave_sum(acc.a11);
    if (lane == 0) {
        Blk<T> dw = bsub(ldb(a.A.d0, a.A.d1, 2 * n + w), acc);
        stb(a.F.ui0, a.F.ui1, 2 * n + w, binv(dw));
    }
}

template <class T>
const ILUF<T>& ilu_of(dp_sim* s);
template <>
const ILUF<double>& ilu_of<double>(dp_sim* s) { return s->ilu64; }
template <>
const ILUF<float>& ilu_of<float>(dp_sim* s) { return s->ilu32; }

template <class T>
static IluArgs<T> ilu_args(dp_sim* s) {
    Topo& t = s->topo;
    IluArgs<T> a;
    a.A = amat<T>(s);
    a.F = ilu_of<T>(s);
    a.fcol = t.fcol;
    a.fmask = t.fmask;
    a.fperf = t.fperf;
    a.perf_q = t.perf_q;
    a.perf_well = t.perf_well;
    a.well_ptr = t.well_ptr;
    a.n = t.n;
    a.nw = t.nw;
    a.nred = t.nred;
    return a;
}

template <class T>
void ilu_factor(dp_sim* s) {
    Topo& t = s->topo;
    IluArgs<T> a = ilu_args<T>(s);
    if (t.nred > 0) ilu_red_kernel<T><<<ceil_div(t.nred, 256), 256, 0, s->stream>>>(a);
    DP_LAUNCH_CHECK();
    if (t.n - t.nred > 0) ilu_black_kernel<T><<<ceil_div(t.n - t.nred, 256), 256, 0, s->stream>>>(a);
    DP_LAUNCH_CHECK();
    if (t.nw > 0) ilu_well_kernel<T><<<t.nw, WAVE, 0, s->stream>>>(a);
    DP_LAUNCH_CHECK();
}
template void ilu_factor<double>(dp_sim*);
template void ilu_factor<float>(dp_sim*);

// ---------------------------------------------------------------------------
// Block ILU(0) solve z = (LU)^-1 r.  y and z share the output array.
//   even rows:  y_r = r_r - L_rm r_m
//   odd rows:   y_b = r_b - L_bm r_m - sum_s L_bs y_rs; without a perforation
//               z_b = U_bb^-1 y_b and z_m = U_mm^-1 (r_m - A_mb z_b) at once
//   wells:      y_w = r_w - sum_p L_wp y_p; z_w = U_ww^-1 y_w; then the
//               perforated odd rows and their matrix nodes
//   even rows:  z_r = U_rr^-1 (y_r - sum_s A_rs z_bs - A_rw z_w), then z_m
// ---------------------------------------------------------------------------
template <class T>
struct IluSolveArgs {
    IluArgs<T> f;
    const V2<T>* r;
    V2<T>* z;
    const d2* r64;     // optional FP64 right-hand side, scaled by sc on first read
    double sc;
    const V2<T>* zadd;  // optional: final entries also written as zout = zadd + z
    d2* zout;
};

// First read of r[i]: from r64 (scaled, rounded to T and kept in r for the later
// reads of the same solve and of the caller) or from r itself.
template <class T>
__device__ inline V2<T> ilus_rin(const IluSolveArgs<T>& a, int64_t i) {
    if (a.r64) {
        const d2 v = a.r64[i];
        const V2<T> x = mk2<T>((T)(a.sc * v.x), (T)(a.sc * v.y));
        const_cast<V2<T>*>(a.r)[i] = x;
        return x;
    }
    return a.r[i];
}

// Final z[i]; with zout also the FP64 sum zadd + z, rounded as its FP32 sum.
template <class T>
__device__ inline void ilus_zfin(const IluSolveArgs<T>& a, int64_t i, V2<T> v) {
    a.z[i] = v;
    if (a.zout) {
        const V2<T> u = a.zadd[i];
        a.zout[i] = mk2<double>((double)(u.x + v.x), (double)(u.y + v.y));
    }
}

template <class T>
__global__ void ilus_red_fwd(IluSolveArgs<T> a) {
    int q = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (q >= a.f.nred) return;
    int n = a.f.n;
    int c = q;  // the matrix node of fracture row q
    const V2<T> rm = ilus_rin(a, c);
    V2<T> y = vsub(ilus_rin(a, n + q), bmv(ldb(a.f.F.l0, a.f.F.l1, (int64_t)6 * n + q), rm));
    a.z[n + q] = y;
}

template <class T>
__global__ void ilus_black(IluSolveArgs<T> a) {
    int q = a.f.nred + xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (q >= a.f.n) return;
    int n = a.f.n;
    int c = q;  // the matrix node of fracture row q
    V2<T> rm = ilus_rin(a, c);
    V2<T> y = vsub(ilus_rin(a, n + q), bmv(ldb(a.f.F.l0, a.f.F.l1, (int64_t)6 * n + q), rm));
    unsigned mask = a.f.fmask[q];
#pragma unroll
    for (int s = 0; s < 6; ++s)
        if (mask & (1u << s))
            y = vsub(y, bmv(ldb(a.f.F.l0, a.f.F.l1, (int64_t)s * n + q), a.z[a.f.fcol[s * n + q]]));
    if (a.f.fperf[q] >= 0) {
        a.z[n + q] = y;
        return;
    }
    V2<T> zb = bmv(ldb(a.f.F.ui0, a.f.F.ui1, n + q), y);
    ilus_zfin(a, n + q, zb);
    ilus_zfin(a, c, bmv(ldb(a.f.F.ui0, a.f.F.ui1, c), vsub(rm, bmv(ldb(a.f.A.m0, a.f.A.m1, c), zb))));
}

template <class T>
__global__ void ilus_well(IluSolveArgs<T> a) {
    __shared__ T sh0[256 / WAVE], sh1[256 / WAVE];
    __shared__ V2<T> zw_sh;
    int w = blockIdx.x;
    int n = a.f.n;
    int p0 = a.f.well_ptr[w], p1 = a.f.well_ptr[w + 1];
    T y0 = 0, y1 = 0;
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        V2<T> v = bmv(ldb(a.f.F.lw0, a.f.F.lw1, p), a.z[n + a.f.perf_q[p]]);
        y0 += v.x;
        y1 += v.y;
    }
    y0 = wave_sum(y0);
    y1 = wave_sum(y1);
    if (threadIdx.x % WAVE == 0) {
        sh0[threadIdx.x / WAVE] = y0;
        sh1[threadIdx.x / WAVE] = y1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        T s0 = 0, s1 = 0;
        for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) {
            s0 += sh0[i];
            s1 += sh1[i];
        }
        V2<T> rw = ilus_rin(a, 2 * n + w);
        V2<T> zw = bmv(ldb(a.f.F.ui0, a.f.F.ui1, 2 * n + w), mk2<T>(rw.x - s0, rw.y - s1));
        ilus_zfin(a, 2 * n + w, zw);
        zw_sh = zw;
    }
    __syncthreads();
    V2<T> zw = zw_sh;
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        int q = a.f.perf_q[p];
        if (q < a.f.nred) continue;
        int c = q;  // the matrix node of fracture row q
        V2<T> y = vsub(a.z[n + q], bmv(ldb(a.f.F.ubw0, a.f.F.ubw1, p), zw));
        V2<T> zb = bmv(ldb(a.f.F.ui0, a.f.F.ui1, n + q), y);
        ilus_zfin(a, n + q, zb);
        // r[c] of a black row was formed by the black sweep
        ilus_zfin(a, c, bmv(ldb(a.f.F.ui0, a.f.F.ui1, c), vsub(a.r[c], bmv(ldb(a.f.A.m0, a.f.A.m1, c), zb))));
    }
}

template <class T>
__global__ void ilus_red_bwd(IluSolveArgs<T> a) {
    int q = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (q >= a.f.nred) return;
    int n = a.f.n;
    int c = q;  // the matrix node of fracture row q
    V2<T> y = a.z[n + q];
    unsigned mask = a.f.fmask[q];
#pragma unroll
    for (int s = 0; s < 6; ++s)
        if (mask & (1u << s))
            y = vsub(y, bmv(ldb(a.f.A.f0, a.f.A.f1, (int64_t)s * n + q), a.z[a.f.fcol[s * n + q]]));
    int p = a.f.fperf[q];
    if (p >= 0) y = vsub(y, bmv(ldb(a.f.F.ubw0, a.f.F.ubw1, p), a.z[2 * n + a.f.perf_well[p]]));
    V2<T> zr = bmv(ldb(a.f.F.ui0, a.f.F.ui1, n + q), y);
    ilus_zfin(a, n + q, zr);
    // r[c] of a red row was formed by the forward sweep
    ilus_zfin(a, c, bmv(ldb(a.f.F.ui0, a.f.F.ui1, c), vsub(a.r[c], bmv(ldb(a.f.A.m0, a.f.A.m1, c), zr))));
}

template <class T>
void ilu_solve(dp_sim* s, const V2<T>* r, V2<T>* z, const d2* r64, double sc, const V2<T>* zadd, d2* zout) {
    Topo& t = s->topo;
    if (zout && !zadd) fail(DP_E_INVALID, "ILU solve: the sum output needs its addend");
    IluSolveArgs<T> a{ilu_args<T>(s), r, z, r64, sc, zadd, zout};
    int nb_red = ceil_div(t.nred, 256), nb_black = ceil_div(t.n - t.nred, 256);
    KtScope ks(s->capturing ? nullptr : &s->kt[1], s->stream);
    // the folded casts: r64 read and r written in place of the r read; zadd read
    // and zout written
    const double es = sizeof(T), nb = t.nb;
    ks.bytes(kernel_bytes(s, 1) + (r64 ? 16.0 * nb : 0.0) + (zout ? nb * (2 * es + 16.0) : 0.0));
    if (nb_red) ilus_red_fwd<T><<<nb_red, 256, 0, s->stream>>>(a);
    if (nb_black) ilus_black<T><<<nb_black, 256, 0, s->stream>>>(a);
    if (t.nw) ilus_well<T><<<t.nw, 256, 0, s->stream>>>(a);
    if (nb_red) ilus_red_bwd<T><<<nb_red, 256, 0, s->stream>>>(a);
    DP_LAUNCH_CHECK();
}
template void ilu_solve<double>(dp_sim*, const d2*, d2*, const d2*, double, const d2*, d2*);
template void ilu_solve<float>(dp_sim*, const f2*, f2*, const d2*, double, const f2*, d2*);

}  // namespace dp
