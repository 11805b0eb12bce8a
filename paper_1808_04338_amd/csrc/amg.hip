// Classical algebraic multigrid on the pressure system: setup (strength of
// connection, PMIS splitting, distance-two interpolation in matrix-product form
// with truncation, Galerkin coarse operators) and the V(1,1) cycle with
// l1-Jacobi smoothing.  The coarsest operator is inverted densely by a blocked
// Gauss-Jordan whose rank-32 updates run on FP64 MFMA.
//
// Setup runs in FP64; the apply copies (SELL-64 operators, l1 diagonals, dense
// coarse inverse) are kept in the preconditioner precision.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "kernels.h"
#include "primitives.h"

namespace dp {

constexpr int C_BASE = 1 << 20;  // PMIS state >= C_BASE: C point chosen in iteration state-C_BASE
constexpr int ST_U = 0;
constexpr int ST_F = -1;

// ---------------------------------------------------------------------------
// Level-0 pressure matrix: entry (0,0) of each block of the decoupled matrix,
// with the matrix-node pressures eliminated exactly.  A matrix node couples
// only to its own fracture node, so the Schur complement changes only the
// fracture diagonal: a_ff - a_fm (1/a_mm) a_mf.
// ---------------------------------------------------------------------------
// The same values are also written by slot for the fracture rows (st: [8n],
// faces 0..5, diagonal, well column; zero where absent), in the preconditioner
// precision, for the V-cycle's stencil form of level 0.
template <class T>
__global__ void extract_ap_kernel(BMat<double> A, const int* __restrict__ rowptr,
                                  const int* __restrict__ src, const int* __restrict__ fperf, int n,
                                  int nr, double* val, T* st) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    if (r < n) {
#pragma unroll
        for (int k = 0; k < 8; ++k) st[(int64_t)k * n + r] = T(0);  // overwritten below where present
    }
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        int code = src[e];
        double v;
        if (r < n) {
            int q = r;
            if (code < 6) {
                v = A.f0[(int64_t)code * n + q].x;
            } else if (code == 7) {
                v = A.d0[n + q].x - A.f0[(int64_t)6 * n + q].x * (1.0 / A.d0[q].x) * A.m0[q].x;
            } else {
                v = A.fw0[fperf[q]].x;
            }
        } else {
            v = code < 0 ? A.d0[n + r].x : A.wf0[code].x;
        }
        val[e] = v;
        if (r < n) st[(int64_t)(code < 6 ? code : code - 1) * n + r] = (T)v;
    }
}

void amg_extract_level0(dp_sim* s) {
    Topo& t = s->topo;
    int nr = t.n + t.nw;
    if (s->fp32)
        extract_ap_kernel<float><<<ceil_div(nr, 256), 256, 0, s->stream>>>(s->A, s->Ap0.rowptr, s->ap_src, t.fperf,
                                                                          t.n, nr, s->Ap0.val, (float*)s->st0);
    else
        extract_ap_kernel<double><<<ceil_div(nr, 256), 256, 0, s->stream>>>(s->A, s->Ap0.rowptr, s->ap_src, t.fperf,
                                                                           t.n, nr, s->Ap0.val, (double*)s->st0);
    DP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Strength: j strongly influences i if -a_ij sgn(a_ii) >= theta max_k(-a_ik sgn(a_ii))
// and that maximum is > 0.  Also |S^T_i| (integer atomics) and the diagonal.
// ---------------------------------------------------------------------------
// Row kernels below give each row RL consecutive lanes (a subgroup); the
// subgroup reductions use xor shuffles of width RL.
constexpr int RL = 8;

__device__ inline double rl_sum(double v) {
#pragma unroll
    for (int o = RL / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, RL);
    return v;
}
__device__ inline double rl_max(double v) {
#pragma unroll
    for (int o = RL / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, RL));
    return v;
}
__device__ inline int rl_or(int v) {
#pragma unroll
    for (int o = RL / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o, RL);
    return v;
}
__device__ inline int rl_isum(int v) {
#pragma unroll
    for (int o = RL / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, RL);
    return v;
}
inline int rl_grid(int n) { return ceil_div((int64_t)n * RL, 256); }

__global__ void strength_kernel(Csr A, double theta, unsigned char* smask, int* nst, double* diag) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int i = g / RL, l = g % RL;
    if (i >= A.n) return;  // whole subgroup
    int b = A.rowptr[i], e1 = A.rowptr[i + 1];
    double d = 0.0;
    for (int e = b + l; e < e1; e += RL)
        if (A.col[e] == i) d = A.val[e];
    d = rl_sum(d);  // one lane holds the diagonal
    double sg = d < 0.0 ? -1.0 : 1.0;
    double mx = -INFINITY;
    for (int e = b + l; e < e1; e += RL)
        if (A.col[e] != i) mx = fmax(mx, -A.val[e] * sg);
    mx = rl_max(mx);
    for (int e = b + l; e < e1; e += RL) {
        int j = A.col[e];
        bool st = (j != i) && (mx > 0.0) && (-A.val[e] * sg >= theta * mx);
        smask[e] = st ? 1 : 0;
        if (st) atomicAdd(&nst[j], 1);
    }
    if (l == 0) diag[i] = d;
}

// lowbias32 integer hash (C. Wellons)
__device__ inline uint32_t lowbias32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

constexpr int PMIS_BATCH = 4;  // PMIS iterations between termination checks

__global__ void pmis_init(int n, const int* __restrict__ nst, int* state, double* wgt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    state[i] = nst[i] == 0 ? ST_F : ST_U;
    wgt[i] = (double)nst[i] + (double)lowbias32((uint32_t)i) * (1.0 / 4294967296.0);
}

// For every strong edge with both ends undecided, the end with the smaller
// (weight, index) is beaten in this iteration.
// RL lanes per row: every undecided neighbour pair through a strong edge marks
// the loser (the lower weight, ties to the lower index) as beaten this iteration
// (all writers store the same value).
__global__ void pmis_beat(Csr A, const unsigned char* __restrict__ smask, const int* __restrict__ state,
                          const double* __restrict__ wgt, int iter, int* beaten) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int i = g / RL, l = g % RL;
    if (i >= A.n || state[i] != ST_U) return;  // whole subgroup
    double wi = wgt[i];
    for (int e = A.rowptr[i] + l; e < A.rowptr[i + 1]; e += RL) {
        if (!smask[e]) continue;
        int j = A.col[e];
        if (state[j] != ST_U) continue;
        double wj = wgt[j];
        bool j_wins = (wj > wi) || (wj == wi && j > i);
        if (j_wins) beaten[i] = iter;
        else beaten[j] = iter;
    }
}

__global__ void pmis_select(int n, int* state, const int* __restrict__ beaten, int iter) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || state[i] != ST_U) return;
    if (beaten[i] != iter) state[i] = C_BASE + iter;
}

// Undecided points that depend strongly on a C point of this iteration become F
// (RL lanes per row; a C state of this iteration does not change in this pass).
__global__ void pmis_fpass(Csr A, const unsigned char* __restrict__ smask, int* state, int iter,
                           int* undecided) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int i = g / RL, l = g % RL;
    bool und = false;
    if (i < A.n && state[i] == ST_U) {  // whole subgroup
        int f = 0;
        for (int e = A.rowptr[i] + l; e < A.rowptr[i + 1]; e += RL)
            if (smask[e] && state[A.col[e]] == C_BASE + iter) f = 1;
        f = rl_or(f);
        if (l == 0) {
            if (f) state[i] = ST_F;
            else und = true;
        }
    }
    // a flag, not a count: the host only asks whether any point is undecided
    // (every writer stores 1; no atomic serialises the wavefronts)
    uint64_t m = __ballot(und);
    if (threadIdx.x % WAVE == 0 && m) *undecided = 1;
}

__global__ void pmis_final(int n, const int* __restrict__ state, int* cf, int64_t* cflag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool c = state[i] >= C_BASE;
    cf[i] = c ? 1 : -1;
    cflag[i] = c ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Interpolation (distance two, matrix-product form):
//   abar_kj = a_kj if j strong C of k and a_kj a_kk < 0;  beta_k = sum_j abar_kj
//   d_i = a_ii + sum_{weak n} a_in + sum_{k strong F, beta_k = 0} a_ik
//   s_ij = a_ij [j strong C] + sum_{k strong F, beta_k != 0} a_ik (abar_kj / beta_k)
//   w_ij = -s_ij / d_i, truncated to the largest entries (row sum kept)
// ---------------------------------------------------------------------------
__global__ void interp_beta(Csr A, const unsigned char* __restrict__ smask, const int* __restrict__ cf,
                            const double* __restrict__ diag, double* beta, int* g) {
    int gi = blockIdx.x * blockDim.x + threadIdx.x;
    int k = gi / RL, l = gi % RL;
    if (k >= A.n) return;  // whole subgroup
    double bsum = 0.0;
    int cnt = 0;
    if (cf[k] < 0) {
        double dk = diag[k];
        for (int e = A.rowptr[k] + l; e < A.rowptr[k + 1]; e += RL) {
            int j = A.col[e];
            double v = A.val[e];
            if (smask[e] && cf[j] > 0 && v * dk < 0.0) {
                bsum += v;
                ++cnt;
            }
        }
    }
    bsum = rl_sum(bsum);
    cnt = rl_isum(cnt);
    if (l == 0) {
        beta[k] = bsum;
        g[k] = cnt;
    }
}

// Row of every stored entry (thread per row).
__global__ void entry_rows(Csr A, int* erow) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int i = g / RL, l = g % RL;
    if (i >= A.n) return;
    for (int e = A.rowptr[i] + l; e < A.rowptr[i + 1]; e += RL) erow[e] = i;
}

// d_i of every F row: diagonal + weak entries + strong F entries whose row
// cannot distribute (beta_k = 0); weak entries first, then those, column order.
__global__ void interp_d(Csr A, const unsigned char* __restrict__ smask, const int* __restrict__ cf,
                         const double* __restrict__ diag, const double* __restrict__ beta, double* dd) {
    int gi = blockIdx.x * blockDim.x + threadIdx.x;
    int i = gi / RL, l = gi % RL;
    if (i >= A.n) return;  // whole subgroup
    double s = 0.0;
    if (cf[i] < 0) {
        for (int e = A.rowptr[i] + l; e < A.rowptr[i + 1]; e += RL) {
            int j = A.col[e];
            if (j == i) continue;
            if (!smask[e] || (cf[j] < 0 && beta[j] == 0.0)) s += A.val[e];
        }
    }
    s = rl_sum(s);
    if (l == 0) dd[i] = diag[i] + s;
}

// Number of products each stored entry (i, k) of an F row contributes to row i
// of W: 1 for a strong C neighbour, g_k for a strong F neighbour with beta_k != 0.
__global__ void interp_count_e(Csr A, const int* __restrict__ erow, const unsigned char* __restrict__ smask,
                               const int* __restrict__ cf, const double* __restrict__ beta,
                               const int* __restrict__ g, int64_t* cnt) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.nnz) return;
    int i = erow[e];
    int j = A.col[e];
    int64_t c = 0;
    if (cf[i] < 0 && j != i && smask[e]) {
        if (cf[j] > 0) c = 1;
        else if (beta[j] != 0.0) c = g[j];
    }
    cnt[e] = c;
}

__global__ void interp_expand_e(Csr A, const int* __restrict__ erow, const unsigned char* __restrict__ smask,
                                const int* __restrict__ cf, const int64_t* __restrict__ cidx,
                                const double* __restrict__ diag, const double* __restrict__ beta,
                                const int64_t* __restrict__ off, int cbits, uint64_t* keys, double* vals) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.nnz) return;
    int i = erow[e];
    int j = A.col[e];
    if (cf[i] > 0 || j == i || !smask[e]) return;
    int64_t o = off[e];
    uint64_t rk = (uint64_t)i << cbits;
    double a = A.val[e];
    if (cf[j] > 0) {
        keys[o] = rk | (uint64_t)cidx[j];
        vals[o] = a;
    } else if (beta[j] != 0.0) {
        double bk = beta[j], dk = diag[j];
        for (int f = A.rowptr[j]; f < A.rowptr[j + 1]; ++f) {
            int jj = A.col[f];
            double v = A.val[f];
            if (smask[f] && cf[jj] > 0 && v * dk < 0.0) {
                keys[o] = rk | (uint64_t)cidx[jj];
                vals[o] = a * (v / bk);
                ++o;
            }
        }
    }
}

// Distance-two pieces of every F row k with beta_k != 0: its strong C
// neighbours j with a_kj a_kk < 0, as (coarse index, a_kj / beta_k), in row
// order at goff[k] (RL lanes per row; a ballot prefix count keeps the order).
__global__ void interp_pieces(Csr A, const unsigned char* __restrict__ smask, const int* __restrict__ cf,
                              const int64_t* __restrict__ cidx, const double* __restrict__ diag,
                              const double* __restrict__ beta, const int64_t* __restrict__ goff, int* pcol,
                              double* pval) {
    int gi = blockIdx.x * blockDim.x + threadIdx.x;
    int k = gi / RL, l = gi % RL;
    if (k >= A.n || cf[k] > 0 || beta[k] == 0.0) return;  // whole subgroup
    const double bk = beta[k], dk = diag[k];
    const int sub0 = (int)(threadIdx.x % WAVE) - l;
    int64_t o = goff[k];
    for (int fb = A.rowptr[k]; fb < A.rowptr[k + 1]; fb += RL) {
        int f = fb + l;
        bool take = false;
        int jj = 0;
        double v = 0.0;
        if (f < A.rowptr[k + 1]) {
            jj = A.col[f];
            v = A.val[f];
            take = smask[f] && cf[jj] > 0 && v * dk < 0.0;
        }
        uint64_t mine = (__ballot(take) >> sub0) & ((1ull << RL) - 1);
        if (take) {
            int64_t q = o + __popcll(mine & ((1ull << l) - 1));
            pcol[q] = (int)cidx[jj];
            pval[q] = v / bk;
        }
        o += __popcll(mine);
    }
}

// The same interpolation terms as column/value pairs (the segmented path):
// terms of F row i are contiguous because A's entries are grouped by row.  A
// strong F neighbour k contributes a_ik times each of its pieces.
__global__ void interp_expand_c(Csr A, const int* __restrict__ erow, const unsigned char* __restrict__ smask,
                                const int* __restrict__ cf, const int64_t* __restrict__ cidx,
                                const double* __restrict__ beta, const int64_t* __restrict__ goff,
                                const int* __restrict__ pcol, const double* __restrict__ pval,
                                const int64_t* __restrict__ off, int* cols, double* vals) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.nnz) return;
    int i = erow[e];
    int j = A.col[e];
    if (cf[i] > 0 || j == i || !smask[e]) return;
    int64_t o = off[e];
    double a = A.val[e];
    if (cf[j] > 0) {
        cols[o] = (int)cidx[j];
        vals[o] = a;
    } else if (beta[j] != 0.0) {
        for (int64_t t = goff[j]; t < goff[j + 1]; ++t, ++o) {
            cols[o] = pcol[t];
            vals[o] = a * pval[t];
        }
    }
}

// a[0..n) widened to int64 with a[n] = 0 (for an exclusive scan that leaves the total there)
__global__ void int_to_i64(const int* __restrict__ a, int n, int64_t* b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) b[i] = i < n ? (int64_t)a[i] : 0;
}

// Row offsets of terms generated per matrix entry: row r starts where its first
// entry's terms start (eoff: exclusive scan over the nnz entries, total m).
__global__ void seg_off_from_entries(const int* __restrict__ rowptr, const int64_t* __restrict__ eoff, int n,
                                     int64_t nnz, int64_t m, int64_t* seg) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) seg[i] = rowptr[i] < nnz ? eoff[rowptr[i]] : m;
    if (i == n) seg[n] = m;
}

constexpr int TRUNC_MAX = 8;

// Selection of the kept entries of one F row: the 'trunc' largest |w|
// (ties: lower column), in that order.
struct Sel {
    int n;
    int col[TRUNC_MAX];
    double w[TRUNC_MAX];
};

__device__ inline bool better(double aw, int ac, double bw, int bc) {
    double fa = fabs(aw), fb = fabs(bw);
    return fa > fb || (fa == fb && ac < bc);
}

// The trunc best entries of W's row i (best first), the row sum and the count
// of non-zero entries.  Each entry is inserted where the sequential insertion
// would put it: pos = the number of kept entries that stay ahead of it (the
// kept list is sorted, so "better" holds from pos on).  Every array index is a
// compile-time constant, so the selection stays in registers.
__device__ inline void select_row(const Csr& W, int i, double d, int trunc, Sel& sel, double& total,
                                  int& nnzw) {
    sel.n = 0;
    total = 0.0;
    nnzw = 0;
    for (int e = W.rowptr[i]; e < W.rowptr[i + 1]; ++e) {
        double w = -W.val[e] / d;
        if (w == 0.0) continue;
        ++nnzw;
        total += w;
        int c = W.col[e];
        int pos = 0;
#pragma unroll
        for (int t = 0; t < TRUNC_MAX; ++t)
            if (t < sel.n && !better(w, c, sel.w[t], sel.col[t])) ++pos;
        if (pos < trunc) {
#pragma unroll
            for (int t = TRUNC_MAX - 1; t > 0; --t) {
                if (t > pos && t <= sel.n && t < trunc) {
                    sel.w[t] = sel.w[t - 1];
                    sel.col[t] = sel.col[t - 1];
                }
            }
#pragma unroll
            for (int t = 0; t < TRUNC_MAX; ++t) {
                if (t == pos) {
                    sel.w[t] = w;
                    sel.col[t] = c;
                }
            }
            if (sel.n < trunc) ++sel.n;
        }
    }
}

__global__ void pcount_kernel(Csr W, const int* __restrict__ cf, const double* __restrict__ dd, int trunc,
                              int64_t* cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W.n) return;
    if (cf[i] > 0) {
        cnt[i] = 1;
        return;
    }
    double d = dd[i];
    if (d == 0.0) {
        cnt[i] = 0;
        return;
    }
    int nz = 0;
    for (int e = W.rowptr[i]; e < W.rowptr[i + 1]; ++e)
        if (-W.val[e] / d != 0.0) ++nz;
    cnt[i] = nz < trunc ? nz : trunc;
}

__global__ void pfill_kernel(Csr W, const int* __restrict__ cf, const int64_t* __restrict__ cidx,
                             const double* __restrict__ dd, int trunc, const int64_t* __restrict__ off,
                             int* pcol, double* pval) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W.n) return;
    int64_t o = off[i];
    if (cf[i] > 0) {
        pcol[o] = (int)cidx[i];
        pval[o] = 1.0;
        return;
    }
    double d = dd[i];
    if (d == 0.0) return;
    Sel sel;
    double total;
    int nnzw;
    select_row(W, i, d, trunc, sel, total, nnzw);
    double scale = 1.0;
    if (nnzw > trunc) {
        double kept = 0.0;
#pragma unroll
        for (int t = 0; t < TRUNC_MAX; ++t)
            if (t < sel.n) kept += sel.w[t];
        scale = kept != 0.0 ? total / kept : 1.0;
    }
    // kept entries in column order (columns are distinct; an exchange network
    // with compile-time indices)
#pragma unroll
    for (int p = 0; p < TRUNC_MAX - 1; ++p) {
#pragma unroll
        for (int b = 0; b < TRUNC_MAX - 1 - p; ++b) {
            if (b + 1 < sel.n && sel.col[b + 1] < sel.col[b]) {
                int tc = sel.col[b];
                sel.col[b] = sel.col[b + 1];
                sel.col[b + 1] = tc;
                double tw = sel.w[b];
                sel.w[b] = sel.w[b + 1];
                sel.w[b + 1] = tw;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < TRUNC_MAX; ++t) {
        if (t < sel.n) {
            pcol[o + t] = sel.col[t];
            pval[o + t] = nnzw > trunc ? sel.w[t] * scale : sel.w[t];
        }
    }
}

// ---------------------------------------------------------------------------
// Galerkin product by expansion + stable sort + ordered sums (fallback path)
// ---------------------------------------------------------------------------
// Transpose R = P^T by counting: entries per column, offsets, a scatter with a
// cursor per column, then every R row sorted by its column (the fine row) in
// the segmented tiles.  Keys are unique within a row, so the result does not
// depend on the order the scatter wrote it in.
__global__ void transpose_count(Csr P, unsigned long long* cnt) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < P.nnz) atomicAdd(&cnt[P.col[e]], 1ull);
}

__global__ void transpose_scatter(Csr P, const int64_t* __restrict__ roff, int* cur, int* rcol, double* rval) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    for (int e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) {
        int c = P.col[e];
        int64_t pos = roff[c] + atomicAdd(&cur[c], 1);
        rcol[pos] = i;
        rval[pos] = P.val[e];
    }
}

// Fallback for rows beyond the segmented tiles: insertion sort, one thread per row.
__global__ void transpose_sort_rows(int nr, const int64_t* __restrict__ roff, int* rcol, double* rval) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    int64_t b = roff[r], e1 = roff[r + 1];
    for (int64_t a = b + 1; a < e1; ++a) {
        int c = rcol[a];
        double v = rval[a];
        int64_t q = a;
        while (q > b && rcol[q - 1] > c) {
            rcol[q] = rcol[q - 1];
            rval[q] = rval[q - 1];
            --q;
        }
        rcol[q] = c;
        rval[q] = v;
    }
}

// Products of stored entry (i, k): |P_i| |P_k|.
__global__ void rap_count_e(Csr A, const int* __restrict__ erow, Csr P, int64_t* cnt) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.nnz) return;
    int i = erow[e], k = A.col[e];
    cnt[e] = (int64_t)(P.rowptr[i + 1] - P.rowptr[i]) * (P.rowptr[k + 1] - P.rowptr[k]);
}

// A_c(I,J) = sum_{i,k} P_iI a_ik P_kJ: entry (i, k) emits P_iI a_ik P_kJ.
__global__ void rap_expand_e(Csr A, const int* __restrict__ erow, Csr P, const int64_t* __restrict__ off,
                             int cbits, uint64_t* keys, double* vals) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.nnz) return;
    int i = erow[e], k = A.col[e];
    double a = A.val[e];
    int64_t o = off[e];
    int qb = P.rowptr[k], qe = P.rowptr[k + 1];
    for (int u = P.rowptr[i]; u < P.rowptr[i + 1]; ++u) {
        uint64_t rk = (uint64_t)P.col[u] << cbits;
        double pa = P.val[u] * a;
        for (int v = qb; v < qe; ++v) {
            keys[o] = rk | (uint64_t)P.col[v];
            vals[o] = pa * P.val[v];
            ++o;
        }
    }
}

// ---------------------------------------------------------------------------
// SELL-64 conversion and the l1-Jacobi diagonal
// ---------------------------------------------------------------------------
// Slice widths (w[nslices] = 0, so that the exclusive scan leaves the total
// there) and the longest row (atomic max into *maxw).
__global__ void sell_width(Csr A, int nslices, int64_t* w, int* maxw) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nslices) return;
    if (s == nslices) {
        w[s] = 0;
        return;
    }
    int mx = 0;
    for (int r = s * 64; r < s * 64 + 64 && r < A.n; ++r) mx = max(mx, A.rowptr[r + 1] - A.rowptr[r]);
    w[s] = (int64_t)mx * 64;
    atomicMax(maxw, mx);
}

__global__ void sell_ptr(const int64_t* __restrict__ off, int nslices, int64_t total, int* sptr) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nslices) return;
    sptr[s] = s < nslices ? (int)off[s] : (int)total;
}

template <class T>
__global__ void sell_fill(Csr A, const int* __restrict__ sptr, int pad_self, int* col, T* val) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    int s = r / 64, lane = r % 64;
    if (s >= (A.n + 63) / 64) return;
    int base = sptr[s];
    int w = (sptr[s + 1] - base) / 64;
    int b = 0, len = 0;
    if (r < A.n) {
        b = A.rowptr[r];
        len = A.rowptr[r + 1] - b;
    }
    for (int k = 0; k < w; ++k) {
        int e = base + k * 64 + lane;
        if (k < len) {
            col[e] = A.col[b + k];
            val[e] = (T)A.val[b + k];
        } else {
            col[e] = (pad_self && r < A.n) ? r : 0;
            val[e] = (T)0;
        }
    }
}

template <class T>
__global__ void l1_kernel(Csr A, T* dinv) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int i = g / RL, l = g % RL;
    if (i >= A.n) return;
    double d = 0.0, s = 0.0;
    for (int e = A.rowptr[i] + l; e < A.rowptr[i + 1]; e += RL) {
        if (A.col[e] == i) d = A.val[e];
        else s += fabs(A.val[e]);
    }
    d = rl_sum(d);
    s = rl_sum(s);
    double sg = d < 0.0 ? -1.0 : 1.0;
    if (l == 0) dinv[i] = (T)(1.0 / (d + sg * s));
}

__global__ void i64_to_i32(const int64_t* __restrict__ a, int n, int64_t total, int* b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    b[i] = i < n ? (int)a[i] : (int)total;
}

// ---------------------------------------------------------------------------
// Dense coarse inverse: blocked Gauss-Jordan, 32-wide panels.  The diagonal
// panel block is inverted with partial pivoting inside the block; the rank-32
// updates of the rest of the matrix use V_MFMA_F64_16X16X4_F64.
// ---------------------------------------------------------------------------
constexpr int GJ_B = 32;
typedef double d4v __attribute__((ext_vector_type(4)));

__global__ void dense_fill(Csr A, int np, double* M) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)np * np) return;
    int r = (int)(idx / np), c = (int)(idx % np);
    double v = (r == c && r >= A.n) ? 1.0 : 0.0;
    if (r < A.n && c < A.n) {
        for (int e = A.rowptr[r]; e < A.rowptr[r + 1]; ++e)
            if (A.col[e] == c) v = A.val[e];
    }
    M[idx] = v;
}

// Invert the 32x32 block M_kk into P (row-major 32x32) by Gauss-Jordan with
// partial pivoting, in one wavefront: lane j holds column j of [M_kk | I] (64
// columns, 64 lanes) in registers.  The pivot search runs in every lane on its
// own column and lane C's answer is broadcast with readlane; the row swap, the
// scaling and the elimination are register operations on every column, with
// the factors a[r][C] broadcast from lane C.  Each pivot step is a template
// instance so that every register index is a compile-time constant.
__device__ __forceinline__ double lane_bcast(double v, int l) {
    long long b = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <int C>
__device__ __forceinline__ void gj_step(double (&a)[GJ_B], int* bad) {
    double best = fabs(a[C]);
    int p = C;
#pragma unroll
    for (int r = C + 1; r < GJ_B; ++r) {
        double v = fabs(a[r]);
        if (v > best) {
            best = v;
            p = r;
        }
    }
    p = __builtin_amdgcn_readlane(p, C);
    if (lane_bcast(best, C) == 0.0 && threadIdx.x == 0) *bad = 1;
    // p is the same on every lane: the swap is skipped as a whole when the
    // diagonal entry is already the pivot (written as selects so that the array
    // stays in registers)
    if (p != C) {
#pragma unroll
        for (int r = C + 1; r < GJ_B; ++r) {
            const bool sw = r == p;
            const double ac = a[C], ar = a[r];
            a[C] = sw ? ar : ac;
            a[r] = sw ? ac : ar;
        }
    }
    double inv = 1.0 / lane_bcast(a[C], C);
    a[C] *= inv;
#pragma unroll
    for (int r = 0; r < GJ_B; ++r) {
        if (r != C) {
            double f = lane_bcast(a[r], C);
            a[r] = fma(-f, a[C], a[r]);
        }
    }
}

template <int C>
__device__ __forceinline__ void gj_steps(double (&a)[GJ_B], int* bad) {
    if constexpr (C < GJ_B) {
        gj_step<C>(a, bad);
        gj_steps<C + 1>(a, bad);
    }
}

__global__ void __launch_bounds__(64) gj_diag(const double* __restrict__ M, int np, int kb, double* P,
                                              int* bad) {
    int j = threadIdx.x;
    int k0 = kb * GJ_B;
    double a[GJ_B];
#pragma unroll
    for (int r = 0; r < GJ_B; ++r)
        a[r] = j < GJ_B ? M[(int64_t)(k0 + r) * np + k0 + j] : (r == j - GJ_B ? 1.0 : 0.0);
    gj_steps<0>(a, bad);
    if (j >= GJ_B) {
#pragma unroll
        for (int r = 0; r < GJ_B; ++r) P[r * GJ_B + (j - GJ_B)] = a[r];
    }
}

// Output element i of lane l of a 16x16 FP64 MFMA tile (A row r supplied by
// lane r + 16k): row (l/16) + 4i, column l%16 (checked on the device).
__device__ inline void tile_rc(int i, int qr, int qc, int& r, int& c) {
    int lane = threadIdx.x % WAVE;
    r = qr * 16 + (lane / 16) + 4 * i;
    c = qc * 16 + lane % 16;
}

// 32x32 tile product acc = X (32x32, leading dim ldx) * Y (32x32, ldy) with
// MFMA: wave q of 4 computes the 16x16 quadrant (q/2, q%2).
__device__ inline d4v mfma_tile(const double* X, int64_t ldx, const double* Y, int64_t ldy, int qr,
                                int qc) {
    int lane = threadIdx.x % WAVE;
    d4v acc = {0.0, 0.0, 0.0, 0.0};
    int ar = qr * 16 + lane % 16;
    int bc = qc * 16 + lane % 16;
    int kk = lane / 16;
#pragma unroll
    for (int t = 0; t < GJ_B / 4; ++t) {
        double av = X[(int64_t)ar * ldx + 4 * t + kk];
        double bv = Y[(int64_t)(4 * t + kk) * ldy + bc];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    return acc;
}




// Row panel k: M_kj <- P M_kj (j != k).  Also copies the old column panel
// M_ik into Cbuf (np x 32).
__global__ void __launch_bounds__(256) gj_row(double* M, int np, int kb, const double* __restrict__ P,
                                              double* Cbuf) {
    int nbk = np / GJ_B;
    int tile = blockIdx.x;
    int wv = threadIdx.x / WAVE;
    int qr = wv / 2, qc = wv % 2;
    if (tile < nbk) {
        int jb = tile;
        if (jb == kb) return;
        double* Y = M + (int64_t)kb * GJ_B * np + jb * GJ_B;
        d4v acc = mfma_tile(P, GJ_B, Y, np, qr, qc);
        __syncthreads();  // every wave has read its operands of Y before any write
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int r, c;
            tile_rc(i, qr, qc, r, c);
            Y[(int64_t)r * np + c] = acc[i];
        }
    } else {
        int ib = tile - nbk;
        for (int e = threadIdx.x; e < GJ_B * GJ_B; e += 256) {
            int r = e / GJ_B, c = e % GJ_B;
            Cbuf[(int64_t)(ib * GJ_B + r) * GJ_B + c] = M[(int64_t)(ib * GJ_B + r) * np + kb * GJ_B + c];
        }
    }
}

// All tiles (i, j) with i != k: M_ij -= C_i M_kj (j != k), M_ik = -C_i P.
// Tile (k, k) becomes P.  Look-ahead (Pn given): block 0 takes tile
// (k+1, k+1), the next diagonal block, and once it is updated inverts it into
// Pn exactly as gj_diag would, while the other blocks update the rest.
__global__ void __launch_bounds__(256) gj_update(double* M, int np, int kb, const double* __restrict__ P,
                                                 const double* __restrict__ Cbuf, double* Pn, int* bad) {
    __shared__ double tl[GJ_B][GJ_B + 1];
    int nbk = np / GJ_B;
    const int la = Pn ? (kb + 1) * nbk + (kb + 1) : -1;
    int t = blockIdx.x;
    if (la >= 0) t = t == 0 ? la : (t <= la ? t - 1 : t);
    int ib = t / nbk, jb = t % nbk;
    int wv = threadIdx.x / WAVE;
    int qr = wv / 2, qc = wv % 2;
    double* T = M + (int64_t)ib * GJ_B * np + jb * GJ_B;
    if (ib == kb) {
        if (jb == kb)
            for (int e = threadIdx.x; e < GJ_B * GJ_B; e += 256)
                T[(int64_t)(e / GJ_B) * np + e % GJ_B] = P[e];
        return;
    }
    const double* X = Cbuf + (int64_t)ib * GJ_B * GJ_B;
    if (jb == kb) {
        d4v acc = mfma_tile(X, GJ_B, P, GJ_B, qr, qc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int r, c;
            tile_rc(i, qr, qc, r, c);
            T[(int64_t)r * np + c] = -acc[i];
        }
    } else {
        const double* Y = M + (int64_t)kb * GJ_B * np + jb * GJ_B;
        d4v acc = mfma_tile(X, GJ_B, Y, np, qr, qc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int r, c;
            tile_rc(i, qr, qc, r, c);
            const double v = T[(int64_t)r * np + c] - acc[i];
            T[(int64_t)r * np + c] = v;
            if (t == la) tl[r][c] = v;
        }
        if (t == la) {
            __syncthreads();
            if (wv == 0) {
                const int j = threadIdx.x;
                double a[GJ_B];
#pragma unroll
                for (int r = 0; r < GJ_B; ++r) a[r] = j < GJ_B ? tl[r][j] : (r == j - GJ_B ? 1.0 : 0.0);
                gj_steps<0>(a, bad);
                if (j >= GJ_B) {
#pragma unroll
                    for (int r = 0; r < GJ_B; ++r) Pn[r * GJ_B + (j - GJ_B)] = a[r];
                }
            }
        }
    }
}

// In-place inverse of the np x np row-major matrix M (np a multiple of 32).
// P: 2 x 32x32 scratch (the pivot blocks of even and odd panels), C: np x 32
// scratch, bad: set to 1 on a zero pivot.  Only the first diagonal block has a
// launch of its own; each later one is inverted inside the previous panel's
// update.
void gj_invert(hipStream_t st, double* M, int np, double* P, double* C, int* bad) {
    int nbk = np / GJ_B;
    if (nbk == 0) return;
    gj_diag<<<1, 64, 0, st>>>(M, np, 0, P, bad);
    for (int kb = 0; kb < nbk; ++kb) {
        double* Pk = P + (kb & 1) * GJ_B * GJ_B;
        double* Pn = kb + 1 < nbk ? P + ((kb + 1) & 1) * GJ_B * GJ_B : nullptr;
        gj_row<<<2 * nbk, 256, 0, st>>>(M, np, kb, Pk, C);
        gj_update<<<nbk * nbk, 256, 0, st>>>(M, np, kb, Pk, C, Pn, bad);
    }
    DP_LAUNCH_CHECK();
}

template <class T>
__global__ void copy_inv(const double* __restrict__ M, int np, int n, T* out) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    int r = (int)(idx / n), c = (int)(idx % n);
    out[idx] = (T)M[(int64_t)r * np + c];
}

// ---------------------------------------------------------------------------
// Setup driver
// ---------------------------------------------------------------------------
template <class T>
__global__ void cast_vals(const double* __restrict__ a, int64_t n, T* b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)a[i];
}

// Row blocks of a CSR operator for the blocked apply: block k starts at the
// first row whose entry offset reaches k * chunk, so with chunk = CSRS_CAP -
// (longest row) its entries end before (k + 1) * chunk + (longest row), and the
// last block ends at nnz <= nb * chunk: every block holds at most CSRS_CAP
// entries.  desc[k] = (first row, its entry offset); desc[nb] = (n, nnz).  Each
// k in [1, nb) has exactly one row r with rowptr[r-1] < k * chunk <= rowptr[r].
constexpr int CSRS_NT = 512, CSRS_K = 4, CSRS_CAP = CSRS_NT * CSRS_K;

__global__ void csrs_desc(const int* __restrict__ rowptr, int n, int64_t chunk, int nb, int2* desc) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    if (r == 0) desc[0] = make_int2(0, rowptr[0]);
    if (r == n) desc[nb] = make_int2(n, rowptr[n]);
    if (r == 0) return;
    const int64_t lo = rowptr[r - 1], hi = rowptr[r];
    for (int64_t k = lo / chunk + 1; k * chunk <= hi && k < nb; ++k) desc[k] = make_int2(r, (int)hi);
}

// The slice widths of SELL-64 (their scan in w) and the longest row of A, read
// back into two pinned slots with the caller's one synchronisation.
struct OpShape {
    int nsl = 0;
    int64_t* w = nullptr;
    int64_t total = 0, maxw = 0;
};

static void op_measure(dp_sim* s, const Csr& A, OpShape& m, Arena& Sc, int64_t* hslots) {
    hipStream_t st = s->stream;
    m.nsl = (A.n + 63) / 64;
    m.w = Sc.get<int64_t>(m.nsl + 2, "sell widths");
    int64_t* tmp = Sc.get<int64_t>(scan_tmp_size(m.nsl + 2), "sell scan");
    int* dmax = Sc.get<int>(1, "sell width");
    if (m.nsl == 0) return;
    DP_HIP(hipMemsetAsync(dmax, 0, sizeof(int), st));
    sell_width<<<ceil_div(m.nsl + 1, 256), 256, 0, st>>>(A, m.nsl, m.w, dmax);
    DP_LAUNCH_CHECK();
    scan_inplace(st, m.w, m.nsl + 1, tmp);
    DP_HIP(hipMemcpyAsync(&hslots[0], m.w + m.nsl, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DP_HIP(hipMemcpyAsync(&hslots[1], dmax, sizeof(int), hipMemcpyDeviceToHost, st));
}

// Choose and build the apply form of a CSR operator.  SELL-64 when it pads by
// at most 30% and no row is longer than 48; otherwise row blocks of at most
// CSRS_CAP entries when no row is longer than half of that, with 4 lanes per
// row in the sums (8 from a mean of 32 entries per row); otherwise CSR with G
// lanes per row (G the power of two at or above the mean row length, 4..64).
static void op_build(dp_sim* s, const Csr& A, Op& op, bool pad_self, const OpShape& m, Arena& H,
                     const char* what) {
    hipStream_t st = s->stream;
    op.n = A.n;
    op.nnz = A.nnz;
    const int nsl = m.nsl;
    int64_t* w = m.w;
    const int64_t total = m.total, maxw = m.maxw;
    bool sell = total <= (int64_t)(1.3 * (double)A.nnz) + 64 && maxw <= 48;
    size_t es = s->fp32 ? sizeof(float) : sizeof(double);
    if (sell) {
        op.kind = 0;
        Sell& S = op.s;
        S.n = A.n;
        S.nslices = nsl;
        S.nel = total;
        S.sptr = H.get<int>(nsl + 1, what);
        sell_ptr<<<ceil_div(nsl + 1, 256), 256, 0, st>>>(w, nsl, total, S.sptr);
        DP_LAUNCH_CHECK();
        S.col = H.get<int>(total, what);
        S.val = H.take(es * (total > 0 ? total : 1), what);
        if (nsl) {
            if (s->fp32) sell_fill<float><<<nsl, 64, 0, st>>>(A, S.sptr, pad_self, S.col, (float*)S.val);
            else sell_fill<double><<<nsl, 64, 0, st>>>(A, S.sptr, pad_self, S.col, (double*)S.val);
            DP_LAUNCH_CHECK();
        }
    } else {
        double mean = A.n > 0 ? (double)A.nnz / A.n : 1.0;
        if (maxw <= CSRS_CAP / 2) {
            op.kind = 2;
            const int64_t chunk = CSRS_CAP - maxw;
            op.nb = (int)std::max<int64_t>(1, (A.nnz + chunk - 1) / chunk);
            op.L = mean < 4 ? 1 : (mean < 32 ? 4 : 8);
            op.desc = H.get<int2>(op.nb + 1, what);
            csrs_desc<<<ceil_div(A.n + 1, 256), 256, 0, st>>>(A.rowptr, A.n, chunk, op.nb, op.desc);
            DP_LAUNCH_CHECK();
        } else {
            op.kind = 1;
            // two entries per lane and pass, at least 4 lanes per row (measured best
            // over 1-4 entries and 1-4 lanes on the V-cycle of the 4.49M-DOF model)
            const int U = 2;
            int G = 4;
            while (G < 64 && G * U < mean) G <<= 1;
            op.G = G;
            op.U = U;
        }
        op.rowptr = A.rowptr;
        op.col = A.col;
        if (s->fp32) {
            op.val = H.get<float>(A.nnz, what);
            if (A.nnz)
                cast_vals<float><<<ceil_div(A.nnz, 256), 256, 0, st>>>(A.val, A.nnz, (float*)op.val);
            DP_LAUNCH_CHECK();
        } else {
            op.val = A.val;
        }
    }
}

// The apply forms of a level's A, P and R, with one host synchronisation for
// the three shapes.
static void build_level_ops(dp_sim* s, const Csr& A, const Csr& P, const Csr& R, AmgLevel& L, Arena& H,
                            Arena& Sc) {
    const size_t mark = Sc.top;
    int64_t* h = pinned_slots() + 1;  // slots 1..6: (total, longest row) of A, P, R
    const Csr* src[3] = {&A, &P, &R};
    OpShape m[3];
    bool any = false;
    for (int k = 0; k < 3; ++k) {
        op_measure(s, *src[k], m[k], Sc, h + 2 * k);
        any = any || m[k].nsl > 0;
    }
    if (any) DP_HIP(hipStreamSynchronize(s->stream));
    for (int k = 0; k < 3; ++k) {
        if (m[k].nsl == 0) continue;
        m[k].total = h[2 * k];
        m[k].maxw = *reinterpret_cast<const int*>(&h[2 * k + 1]);
    }
    op_build(s, A, L.Aop, true, m[0], H, "A apply");
    op_build(s, P, L.Pop, false, m[1], H, "P apply");
    op_build(s, R, L.Rop, false, m[2], H, "R apply");
    Sc.top = mark;
}

static void level_apply_data(dp_sim* s, AmgLevel& L, Arena& H, Arena& Sc) {
    size_t es = s->fp32 ? sizeof(float) : sizeof(double);
    L.dinv = H.take(es * (L.n > 0 ? L.n : 1), "amg dinv");
    L.x = H.take(es * (L.n > 0 ? L.n : 1), "amg x");
    L.b = H.take(es * (L.n > 0 ? L.n : 1), "amg b");
    L.r = H.take(es * (L.n > 0 ? L.n : 1), "amg r");
    L.t = H.take(es * (L.n > 0 ? L.n : 1), "amg t");
    if (L.n == 0) return;
    if (s->fp32) l1_kernel<float><<<rl_grid(L.n), 256, 0, s->stream>>>(L.A, (float*)L.dinv);
    else l1_kernel<double><<<rl_grid(L.n), 256, 0, s->stream>>>(L.A, (double*)L.dinv);
    DP_LAUNCH_CHECK();
}

static void coarse_inverse(dp_sim* s, const Csr& A, Arena& H, Arena& Sc) {
    hipStream_t st = s->stream;
    int n = A.n;
    s->coarse_n = n;
    if (n == 0) return;
    int np = ((n + GJ_B - 1) / GJ_B) * GJ_B;
    size_t mark = Sc.top;
    double* M = Sc.get<double>((int64_t)np * np, "coarse dense");
    double* P = Sc.get<double>(2 * GJ_B * GJ_B, "coarse pivot blocks");
    double* C = Sc.get<double>((int64_t)np * GJ_B, "coarse column panel");
    int* bad = Sc.get<int>(1, "coarse flag");
    DP_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    dense_fill<<<ceil_div((int64_t)np * np, 256), 256, 0, st>>>(A, np, M);
    DP_LAUNCH_CHECK();
    gj_invert(st, M, np, P, C, bad);
    if (s->fp32) {
        s->coarse_inv = H.get<float>((int64_t)n * n, "coarse inverse");
        copy_inv<float><<<ceil_div((int64_t)n * n, 256), 256, 0, st>>>(M, np, n, (float*)s->coarse_inv);
    } else {
        s->coarse_inv = H.get<double>((int64_t)n * n, "coarse inverse");
        copy_inv<double><<<ceil_div((int64_t)n * n, 256), 256, 0, st>>>(M, np, n, (double*)s->coarse_inv);
    }
    DP_LAUNCH_CHECK();
    int* hbad = reinterpret_cast<int*>(pinned_slots() + 1);
    DP_HIP(hipMemcpyAsync(hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    DP_HIP(hipStreamSynchronize(st));
    if (*hbad) fail(DP_E_NUMERIC, "zero pivot in the coarsest-level dense inverse");
    Sc.top = mark;
}

void amg_setup(dp_sim* s) {
    hipStream_t st = s->stream;
    Arena& H = s->hier;
    Arena& Sc = s->scr;
    H.top = 0;
    Sc.top = 0;
    s->levels.clear();
    s->coarse_inv = nullptr;
    s->coarse_n = 0;
    const dp_sim_desc& d = s->desc;
    ++s->amg_setups;
    Csr A = s->Ap0;
    for (;;) {
        AmgLevel L;
        L.n = A.n;
        L.A = A;
        level_apply_data(s, L, H, Sc);
        // error-path test hook: the first level's launches are queued
        if (s->levels.empty() && d.fail_setup > 0 && s->amg_setups == d.fail_setup)
            fail(DP_E_NOMEM, "AMG setup " + std::to_string(s->amg_setups) + " failed (fail_setup test hook)");
        bool last = (A.n <= d.amg_coarse_max) || ((int)s->levels.size() + 1 >= d.amg_max_levels);
        int n = A.n;
        int nc = 0;
        int64_t* cidx = nullptr;
        unsigned char* smask = nullptr;
        double* diag = nullptr;
        size_t smark = Sc.top;
        if (!last) {
            // strength + PMIS
            smask = Sc.get<unsigned char>(A.nnz, "strength mask");
            int* nst = Sc.get<int>(n, "nst");
            diag = Sc.get<double>(n, "diag");
            int* state = Sc.get<int>(n, "pmis state");
            double* wgt = Sc.get<double>(n, "pmis weight");
            int* beaten = Sc.get<int>(n, "pmis beaten");
            int* und = Sc.get<int>(PMIS_BATCH, "pmis undecided flags");
            cidx = Sc.get<int64_t>(n + 1, "coarse index");
            int64_t* stmp = Sc.get<int64_t>(scan_tmp_size(n + 1), "scan tmp");
            L.cf = H.get<int>(n, "cf");
            DP_HIP(hipMemsetAsync(nst, 0, sizeof(int) * n, st));
            DP_HIP(hipMemsetAsync(beaten, 0xff, sizeof(int) * n, st));
            strength_kernel<<<rl_grid(n), 256, 0, st>>>(A, d.amg_theta, smask, nst, diag);
            pmis_init<<<ceil_div(n, 256), 256, 0, st>>>(n, nst, state, wgt);
            DP_LAUNCH_CHECK();
            // iterations in batches: once no point is undecided an iteration
            // changes nothing, so only the last count of a batch is checked
            for (int iter = 0;;) {
                if (iter > 10000) fail(DP_E_NUMERIC, "PMIS did not terminate");
                DP_HIP(hipMemsetAsync(und, 0, sizeof(int) * PMIS_BATCH, st));
                for (int b = 0; b < PMIS_BATCH; ++b, ++iter) {
                    pmis_beat<<<rl_grid(n), 256, 0, st>>>(A, smask, state, wgt, iter, beaten);
                    pmis_select<<<ceil_div(n, 256), 256, 0, st>>>(n, state, beaten, iter);
                    pmis_fpass<<<rl_grid(n), 256, 0, st>>>(A, smask, state, iter, und + b);
                }
                DP_LAUNCH_CHECK();
                int* hup = reinterpret_cast<int*>(pinned_slots() + 1);
                DP_HIP(hipMemcpyAsync(hup, und + PMIS_BATCH - 1, sizeof(int), hipMemcpyDeviceToHost, st));
                DP_HIP(hipStreamSynchronize(st));
                if (*hup == 0) break;
            }
            pmis_final<<<ceil_div(n, 256), 256, 0, st>>>(n, state, L.cf, cidx);
            DP_LAUNCH_CHECK();
            int64_t tot = 0;
            exclusive_scan(st, cidx, n, stmp, &tot);
            nc = (int)tot;
            if (nc == 0 || nc >= n) last = true;
        }
        if (last) {
            Sc.top = smark;
            L.cf = nullptr;
            coarse_inverse(s, A, H, Sc);
            s->levels.push_back(L);
            break;
        }
        // interpolation
        {
            double* beta = Sc.get<double>(n, "beta");
            int* g = Sc.get<int>(n, "g");
            double* dd = Sc.get<double>(n, "d");
            int64_t* stmp = Sc.get<int64_t>(scan_tmp_size(n + 1), "scan tmp");
            int* erow = Sc.get<int>(A.nnz, "entry rows");
            int64_t* ecnt = Sc.get<int64_t>(A.nnz + 1, "interp entry count");
            int64_t* etmp = Sc.get<int64_t>(scan_tmp_size(A.nnz + 1), "scan tmp");
            entry_rows<<<rl_grid(n), 256, 0, st>>>(A, erow);
            interp_beta<<<rl_grid(n), 256, 0, st>>>(A, smask, L.cf, diag, beta, g);
            interp_d<<<rl_grid(n), 256, 0, st>>>(A, smask, L.cf, diag, beta, dd);
            interp_count_e<<<ceil_div(A.nnz, 256), 256, 0, st>>>(A, erow, smask, L.cf, beta, g, ecnt);
            DP_LAUNCH_CHECK();
            int64_t m = 0;
            exclusive_scan(st, ecnt, A.nnz, etmp, &m);
            Csr W;
            W.ncols = nc;
            // segmented path: terms are already grouped by F row
            bool done = false;
            {
                size_t wmark = Sc.top;
                int* wc = Sc.get<int>(m, "interp terms");
                double* wv = Sc.get<double>(m, "interp terms");
                int64_t* woff = Sc.get<int64_t>(n + 1, "interp rows");
                // pieces of every F row: offsets from g (a device-only scan; at most nnz)
                int64_t* goff = Sc.get<int64_t>(n + 1, "interp piece offsets");
                int* pcol = Sc.get<int>(A.nnz, "interp pieces");
                double* pval = Sc.get<double>(A.nnz, "interp pieces");
                int_to_i64<<<ceil_div(n + 1, 256), 256, 0, st>>>(g, n, goff);
                DP_LAUNCH_CHECK();
                scan_inplace(st, goff, n + 1, stmp);
                interp_pieces<<<rl_grid(n), 256, 0, st>>>(A, smask, L.cf, cidx, diag, beta, goff, pcol, pval);
                interp_expand_c<<<ceil_div(A.nnz, 256), 256, 0, st>>>(A, erow, smask, L.cf, cidx, beta, goff, pcol,
                                                                      pval, ecnt, wc, wv);
                seg_off_from_entries<<<ceil_div(n + 1, 256), 256, 0, st>>>(A.rowptr, ecnt, n, A.nnz, m, woff);
                DP_LAUNCH_CHECK();
                done = seg_sort_reduce(st, woff, n, nc, wc, wv, m, Sc, Sc, W, "interp W", &s->seg_fallbacks);
                if (!done) Sc.top = wmark;
            }
            if (!done) {
                int cbits = bits_for(nc);
                int rbits = bits_for(n);
                uint64_t* k0 = Sc.get<uint64_t>(m, "interp keys");
                double* v0 = Sc.get<double>(m, "interp vals");
                uint64_t* k1 = Sc.get<uint64_t>(m, "interp keys");
                double* v1 = Sc.get<double>(m, "interp vals");
                int64_t* rtmp = Sc.get<int64_t>(sort_tmp_size(m), "sort tmp");
                interp_expand_e<<<ceil_div(A.nnz, 256), 256, 0, st>>>(A, erow, smask, L.cf, cidx, diag, beta,
                                                                      ecnt, cbits, k0, v0);
                DP_LAUNCH_CHECK();
                int which = radix_sort(st, k0, v0, k1, v1, m, rbits + cbits, rtmp);
                uint64_t* ks = which ? k1 : k0;
                double* vs = which ? v1 : v0;
                // the idle half of the sort's double buffer holds the run flags and sums
                int64_t* flag = (int64_t*)(which ? k0 : k1);
                double* sums = which ? v0 : v1;
                int* rowkey = Sc.get<int>(m, "rbk rows");
                reduce_to_csr(st, ks, vs, m, cbits, n, flag, sums, rowkey, rtmp, Sc, W, "interp W");
                s->seg_fallbacks += 1;
            }
            // truncation into P
            int64_t* pc = Sc.get<int64_t>(n + 1, "P count");
            pcount_kernel<<<ceil_div(n, 256), 256, 0, st>>>(W, L.cf, dd, d.amg_trunc, pc);
            DP_LAUNCH_CHECK();
            int64_t pn = 0;
            exclusive_scan(st, pc, n, stmp, &pn);
            L.P.n = n;
            L.P.ncols = nc;
            L.P.nnz = pn;
            L.P.rowptr = H.get<int>(n + 1, "P rowptr");
            L.P.col = H.get<int>(pn, "P col");
            L.P.val = H.get<double>(pn, "P val");
            i64_to_i32<<<ceil_div(n + 1, 256), 256, 0, st>>>(pc, n, pn, L.P.rowptr);
            pfill_kernel<<<ceil_div(n, 256), 256, 0, st>>>(W, L.cf, cidx, dd, d.amg_trunc, pc, L.P.col,
                                                           L.P.val);
            DP_LAUNCH_CHECK();
        }
        Sc.top = smark;
        // R = P^T (counting transpose, rows sorted in the segmented tiles)
        Csr R;
        {
            int64_t m = L.P.nnz;
            int64_t* roff = Sc.get<int64_t>(nc + 1, "PT offsets");
            int64_t* stmp = Sc.get<int64_t>(scan_tmp_size(nc + 1), "scan tmp");
            int* cur = Sc.get<int>(nc, "PT cursors");
            int* tcol = Sc.get<int>(m, "PT terms");
            double* tval = Sc.get<double>(m, "PT terms");
            DP_HIP(hipMemsetAsync(roff, 0, sizeof(int64_t) * (nc + 1), st));
            DP_HIP(hipMemsetAsync(cur, 0, sizeof(int) * (nc > 0 ? nc : 1), st));
            if (m > 0) {
                transpose_count<<<ceil_div(m, 256), 256, 0, st>>>(L.P, (unsigned long long*)roff);
                DP_LAUNCH_CHECK();
            }
            scan_inplace(st, roff, nc + 1, stmp);
            if (m > 0) {
                transpose_scatter<<<ceil_div(n, 256), 256, 0, st>>>(L.P, roff, cur, tcol, tval);
                DP_LAUNCH_CHECK();
            }
            R.ncols = n;
            if (!seg_sort_reduce(st, roff, nc, n, tcol, tval, m, Sc, H, R, "R", &s->seg_fallbacks)) {
                // rows beyond the tiles: scatter again (the tiles rewrite the rows they
                // finished in place), sort in place and take the arrays as R
                DP_HIP(hipMemsetAsync(cur, 0, sizeof(int) * (nc > 0 ? nc : 1), st));
                if (m > 0) transpose_scatter<<<ceil_div(n, 256), 256, 0, st>>>(L.P, roff, cur, tcol, tval);
                transpose_sort_rows<<<ceil_div(nc, 256), 256, 0, st>>>(nc, roff, tcol, tval);
                DP_LAUNCH_CHECK();
                R.n = nc;
                R.nnz = m;
                R.rowptr = H.get<int>(nc + 1, "R");
                R.col = H.get<int>(m, "R");
                R.val = H.get<double>(m, "R");
                i64_to_i32<<<ceil_div(nc + 1, 256), 256, 0, st>>>(roff, nc, m, R.rowptr);
                DP_LAUNCH_CHECK();
                DP_HIP(hipMemcpyAsync(R.col, tcol, sizeof(int) * m, hipMemcpyDeviceToDevice, st));
                DP_HIP(hipMemcpyAsync(R.val, tval, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
            }
        }
        Sc.top = smark;
        // Galerkin A_c = R (A P), both products row by row
        Csr Ac;
        Ac.ncols = nc;
        bool rap_done = false;
        {
            Csr AP;
            if (seg_product(st, A, L.P, Sc, Sc, AP, "A P", &s->kt[2], &s->seg_fallbacks))
                rap_done = seg_product(st, R, AP, Sc, H, Ac, "coarse A", &s->kt[2], &s->seg_fallbacks);
            Sc.top = smark;
        }
        if (!rap_done) {
            s->seg_fallbacks += 1;
            int* erow = Sc.get<int>(A.nnz, "entry rows");
            int64_t* cnt = Sc.get<int64_t>(A.nnz + 1, "rap count");
            int64_t* stmp = Sc.get<int64_t>(scan_tmp_size(A.nnz + 1), "scan tmp");
            entry_rows<<<rl_grid(n), 256, 0, st>>>(A, erow);
            rap_count_e<<<ceil_div(A.nnz, 256), 256, 0, st>>>(A, erow, L.P, cnt);
            DP_LAUNCH_CHECK();
            int64_t m = 0;
            exclusive_scan(st, cnt, A.nnz, stmp, &m);
            int cb = bits_for(nc);
            uint64_t* k0 = Sc.get<uint64_t>(m, "rap keys");
            double* v0 = Sc.get<double>(m, "rap vals");
            uint64_t* k1 = Sc.get<uint64_t>(m, "rap keys");
            double* v1 = Sc.get<double>(m, "rap vals");
            int64_t* rtmp = Sc.get<int64_t>(sort_tmp_size(m) + scan_tmp_size(m + 1), "sort tmp");
            rap_expand_e<<<ceil_div(A.nnz, 256), 256, 0, st>>>(A, erow, L.P, cnt, cb, k0, v0);
            DP_LAUNCH_CHECK();
            int which = radix_sort(st, k0, v0, k1, v1, m, 2 * cb, rtmp);
            int64_t* flag = (int64_t*)(which ? k0 : k1);
            double* sums = which ? v0 : v1;
            int* rowkey = Sc.get<int>(m, "rbk rows");
            reduce_to_csr(st, which ? k1 : k0, which ? v1 : v0, m, cb, nc, flag, sums, rowkey, rtmp, H,
                          Ac, "coarse A");
        }
        Sc.top = smark;
        L.nc = nc;
        L.R = R;
        build_level_ops(s, A, L.P, R, L, H, Sc);
        s->levels.push_back(L);
        A = Ac;
    }
    // the coarsest level's operator is only used through its dense inverse
}

// ---------------------------------------------------------------------------
// V(1,1) cycle
// ---------------------------------------------------------------------------
// Y: y = A x.  PRE: y = dinv b (one smoothing step from zero), y2 = b - A y.
// PROL: y += A x.  POST: y = x + dinv (b - A x).  YD (restriction into a level
// that is smoothed next): y = A x and y2 = dinv y, so that level starts with
// x = dinv b already formed.  RES: y = b - A x.
enum { SV_Y = 0, SV_PRE = 1, SV_PROL = 2, SV_POST = 3, SV_YD = 4, SV_RES = 5 };

template <class T, int MODE>
__global__ void __launch_bounds__(256) sell_kernel(const int* __restrict__ sptr, const int* __restrict__ col,
                                                   const T* __restrict__ val, int n,
                                                   const T* __restrict__ dinv, const T* __restrict__ b,
                                                   const T* __restrict__ x, T* y, T* y2) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int s = r >> 6, lane = r & 63;
    int base = sptr[s];
    int w = (sptr[s + 1] - base) >> 6;
    T acc = 0;
    for (int k = 0; k < w; ++k) {
        int e = base + (k << 6) + lane;
        int c = col[e];
        T v = val[e];
        if (MODE == SV_PRE) acc += v * (dinv[c] * b[c]);
        else acc += v * x[c];
    }
    if (MODE == SV_Y) {
        y[r] = acc;
    } else if (MODE == SV_PRE) {  // y = dinv b (smoothed x from zero), y2 = b - A y
        y[r] = dinv[r] * b[r];
        y2[r] = b[r] - acc;
    } else if (MODE == SV_PROL) {  // y += P x
        y[r] += acc;
    } else if (MODE == SV_YD) {
        y[r] = acc;
        y2[r] = dinv[r] * acc;
    } else if (MODE == SV_RES) {
        y[r] = b[r] - acc;
    } else {  // y = x + dinv (b - A x)
        y[r] = x[r] + dinv[r] * (b[r] - acc);
    }
}

template <class T>
__global__ void __launch_bounds__(256) dense_gemv(const T* __restrict__ M, int n, const T* __restrict__ b,
                                                  T* y) {
    int row = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int lane = threadIdx.x % WAVE;
    if (row >= n) return;
    // four loads in flight per lane, summed in the same order as one at a time
    const T* m = M + (int64_t)row * n;
    T acc = 0;
    int c = lane;
    for (; c + 3 * WAVE < n; c += 4 * WAVE) {
        const T m0 = m[c], m1 = m[c + WAVE], m2 = m[c + 2 * WAVE], m3 = m[c + 3 * WAVE];
        const T b0 = b[c], b1 = b[c + WAVE], b2 = b[c + 2 * WAVE], b3 = b[c + 3 * WAVE];
        acc += m0 * b0;
        acc += m1 * b1;
        acc += m2 * b2;
        acc += m3 * b3;
    }
    for (; c < n; c += WAVE) acc += m[c] * b[c];
    acc = wave_sum(acc);
    if (lane == 0) y[row] = acc;
}

// CSR operator with G lanes per row; each lane takes U entries per pass, their
// column and value loads issued together ahead of the dependent gathers, so a
// wavefront keeps several loads in flight per lane.  The G partial sums are
// combined by a fixed butterfly inside the group.
template <class T, int MODE, int G, int U>
__global__ void __launch_bounds__(256) csrv_kernel(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                   const T* __restrict__ val, int n,
                                                   const T* __restrict__ dinv, const T* __restrict__ b,
                                                   const T* __restrict__ x, T* y, T* y2) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    int r = gid / G, l = gid % G;
    if (r >= n) return;
    const int beg = rowptr[r], end = rowptr[r + 1];
    T acc = 0;
    for (int e0 = beg + l; e0 < end; e0 += G * U) {
        int c[U];
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int e = e0 + u * G;
            c[u] = e < end ? col[e] : -1;
            v[u] = e < end ? val[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (c[u] >= 0) {
                T xv = MODE == SV_PRE ? dinv[c[u]] * b[c[u]] : x[c[u]];
                acc += v[u] * xv;
            }
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (l != 0) return;
    if (MODE == SV_Y) {
        y[r] = acc;
    } else if (MODE == SV_PRE) {
        y[r] = dinv[r] * b[r];
        y2[r] = b[r] - acc;
    } else if (MODE == SV_PROL) {
        y[r] += acc;
    } else if (MODE == SV_YD) {
        y[r] = acc;
        y2[r] = dinv[r] * acc;
    } else if (MODE == SV_RES) {
        y[r] = b[r] - acc;
    } else {
        y[r] = x[r] + dinv[r] * (b[r] - acc);
    }
}

// The CSR operator in row blocks (desc from csrs_desc): every product of the
// block's entries is formed with coalesced loads into LDS, CSRS_K per thread
// issued together, then each row is summed by L lanes (strided partial sums in
// entry order, combined by a fixed butterfly).
template <class T, int MODE, int L>
__global__ void __launch_bounds__(CSRS_NT) csrs_kernel(const int2* __restrict__ desc,
                                                       const int* __restrict__ rowptr, const int* __restrict__ col,
                                                       const T* __restrict__ val, const T* __restrict__ dinv,
                                                       const T* __restrict__ b, const T* __restrict__ x, T* y,
                                                       T* y2) {
    __shared__ T prod[CSRS_CAP];
    const int tid = threadIdx.x;
    const int2 d0 = desc[blockIdx.x], d1 = desc[blockIdx.x + 1];
    const int r0 = d0.x, r1 = d1.x, e0 = d0.y, e1 = d1.y;
    int c[CSRS_K];
    T v[CSRS_K];
#pragma unroll
    for (int u = 0; u < CSRS_K; ++u) {
        const int e = e0 + tid + u * CSRS_NT;
        c[u] = e < e1 ? col[e] : -1;
        v[u] = e < e1 ? val[e] : T(0);
    }
    // the offsets of this thread's first row, fetched while the products load
    const int ra = r0 + tid / L;
    int pa = 0, pz = 0;
    if (ra < r1) {
        pa = rowptr[ra];
        pz = rowptr[ra + 1];
    }
#pragma unroll
    for (int u = 0; u < CSRS_K; ++u) {
        if (c[u] >= 0) prod[tid + u * CSRS_NT] = v[u] * (MODE == SV_PRE ? dinv[c[u]] * b[c[u]] : x[c[u]]);
    }
    __syncthreads();
    // all L lanes of a row take the same trip through this loop
    for (int q = tid; q < (r1 - r0) * L; q += CSRS_NT) {
        const int r = r0 + q / L, l = q % L;
        int a = pa, z = pz;
        if (q != tid) {
            a = rowptr[r];
            z = rowptr[r + 1];
        }
        T acc = 0;
        for (int i = a - e0 + l; i < z - e0; i += L) acc += prod[i];
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
        if (l != 0) continue;
        if (MODE == SV_Y) {
            y[r] = acc;
        } else if (MODE == SV_PRE) {
            y[r] = dinv[r] * b[r];
            y2[r] = b[r] - acc;
        } else if (MODE == SV_PROL) {
            y[r] += acc;
        } else if (MODE == SV_YD) {
            y[r] = acc;
            y2[r] = dinv[r] * acc;
        } else if (MODE == SV_RES) {
            y[r] = b[r] - acc;
        } else {
            y[r] = x[r] + dinv[r] * (b[r] - acc);
        }
    }
}

template <class T, int MODE, int U>
static void csrv_launch(dp_sim* s, const Op& op, const T* v, const T* dinv, const T* b, const T* x, T* y,
                        T* y2) {
    int grid = ceil_div((int64_t)op.n * op.G, 256);
    switch (op.G) {
        case 4: csrv_kernel<T, MODE, 4, U><<<grid, 256, 0, s->stream>>>(op.rowptr, op.col, v, op.n, dinv, b, x, y, y2); break;
        case 8: csrv_kernel<T, MODE, 8, U><<<grid, 256, 0, s->stream>>>(op.rowptr, op.col, v, op.n, dinv, b, x, y, y2); break;
        case 16: csrv_kernel<T, MODE, 16, U><<<grid, 256, 0, s->stream>>>(op.rowptr, op.col, v, op.n, dinv, b, x, y, y2); break;
        case 32: csrv_kernel<T, MODE, 32, U><<<grid, 256, 0, s->stream>>>(op.rowptr, op.col, v, op.n, dinv, b, x, y, y2); break;
        default: csrv_kernel<T, MODE, 64, U><<<grid, 256, 0, s->stream>>>(op.rowptr, op.col, v, op.n, dinv, b, x, y, y2); break;
    }
}

template <class T, int MODE>
static void op_launch(dp_sim* s, const Op& op, const T* dinv, const T* b, const T* x, T* y, T* y2) {
    if (op.n == 0) return;
    if (op.kind == 0) {
        const Sell& S = op.s;
        sell_kernel<T, MODE><<<ceil_div(S.n, 256), 256, 0, s->stream>>>(S.sptr, S.col, (const T*)S.val, S.n,
                                                                        dinv, b, x, y, y2);
    } else if (op.kind == 2) {
        const T* v = (const T*)op.val;
        switch (op.L) {
            case 1: csrs_kernel<T, MODE, 1><<<op.nb, CSRS_NT, 0, s->stream>>>(op.desc, op.rowptr, op.col, v, dinv, b, x, y, y2); break;
            case 4: csrs_kernel<T, MODE, 4><<<op.nb, CSRS_NT, 0, s->stream>>>(op.desc, op.rowptr, op.col, v, dinv, b, x, y, y2); break;
            case 8: csrs_kernel<T, MODE, 8><<<op.nb, CSRS_NT, 0, s->stream>>>(op.desc, op.rowptr, op.col, v, dinv, b, x, y, y2); break;
            default: throw Error(DP_E_INVALID, "blocked CSR operator built with another lane count");
        }
    } else {
        const T* v = (const T*)op.val;
        if (op.U != 2) throw Error(DP_E_INVALID, "CSR operator built for another unroll");
        csrv_launch<T, MODE, 2>(s, op, v, dinv, b, x, y, y2);
    }
    DP_LAUNCH_CHECK();
}

// Level 0 (the reduced pressure system) in stencil form: fracture row q takes
// its six face neighbours (fcol; an absent face points at the row itself with
// a zero value), its diagonal and, when perforated, its well, with values by
// slot (st0, written with the CSR values at setup); well rows come from the
// FP64 CSR, one workgroup each.  Same modes as the CSR kernels (PRE, POST).
template <class T>
struct St0Args {
    const T* v;
    const int* fcol;
    const int* fperf;
    const int* perf_well;
    const int* rowptr;
    const int* col;
    const double* val;  // the FP64 CSR of level 0 (well rows), cast as the apply copies are
    const T* dinv;
    const T* b;
    const T* x;
    T* y;
    T* y2;
    int n;
};

template <class T, int MODE>
__device__ inline T st0_x(const St0Args<T>& a, int c) {
    return MODE == SV_PRE ? a.dinv[c] * a.b[c] : a.x[c];
}

template <class T, int MODE>
__device__ inline void st0_store(const St0Args<T>& a, int r, T acc) {
    if (MODE == SV_PRE) {
        a.y[r] = a.dinv[r] * a.b[r];
        a.y2[r] = a.b[r] - acc;
    } else {
        a.y[r] = a.x[r] + a.dinv[r] * (a.b[r] - acc);
    }
}

template <class T, int MODE>
__global__ void __launch_bounds__(256) st0_kernel(St0Args<T> a, int bf) {
    __shared__ T sh[256 / WAVE];
    const int b = blockIdx.x;
    const int n = a.n;
    if (b < bf) {
        const int q = xcd_block(b, bf) * blockDim.x + threadIdx.x;
        if (q >= n) return;
        T acc = 0;
#pragma unroll
        for (int sl = 0; sl < 6; ++sl)
            acc += a.v[(int64_t)sl * n + q] * st0_x<T, MODE>(a, a.fcol[(int64_t)sl * n + q] - n);
        acc += a.v[(int64_t)6 * n + q] * st0_x<T, MODE>(a, q);
        const int p = a.fperf[q];
        if (p >= 0) acc += a.v[(int64_t)7 * n + q] * st0_x<T, MODE>(a, n + a.perf_well[p]);
        st0_store<T, MODE>(a, q, acc);
    } else {
        const int r = n + (b - bf);
        T acc = 0;
        for (int e = a.rowptr[r] + (int)threadIdx.x; e < a.rowptr[r + 1]; e += blockDim.x)
            acc += (T)a.val[e] * st0_x<T, MODE>(a, a.col[e]);
        acc = wave_sum(acc);
        if (threadIdx.x % WAVE == 0) sh[threadIdx.x / WAVE] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            T t = 0;
            for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) t += sh[i];
            st0_store<T, MODE>(a, r, t);
        }
    }
}

template <class T, int MODE>
static void st0_launch(dp_sim* s, const AmgLevel& lv, const T* dinv, const T* b, const T* x, T* y, T* y2) {
    const Topo& t = s->topo;
    if (lv.n != t.n + t.nw) throw Error(DP_E_INVALID, "level 0 is not the reduced pressure system");
    St0Args<T> a{(const T*)s->st0, t.fcol, t.fperf, t.perf_well, lv.A.rowptr, lv.A.col, lv.A.val,
                 dinv, b, x, y, y2, t.n};
    const int bf = ceil_div(t.n, 256);
    if (bf + t.nw > 0) st0_kernel<T, MODE><<<bf + t.nw, 256, 0, s->stream>>>(a, bf);
    DP_LAUNCH_CHECK();
}

template <class T>
T* amg_vcycle(dp_sim* s) {
    int L = (int)s->levels.size();
    for (int l = 0; l < L - 1; ++l) {
        AmgLevel& lv = s->levels[l];
        AmgLevel& nx = s->levels[l + 1];
        // level 0 forms x = dinv b itself; the restriction into a smoothed
        // level forms it there (one gather per entry in the residual instead of two)
        if (l == 0) st0_launch<T, SV_PRE>(s, lv, (T*)lv.dinv, (T*)lv.b, nullptr, (T*)lv.x, (T*)lv.r);
        else op_launch<T, SV_RES>(s, lv.Aop, nullptr, (T*)lv.b, (T*)lv.x, (T*)lv.r, nullptr);
        if (l + 1 < L - 1) op_launch<T, SV_YD>(s, lv.Rop, (T*)nx.dinv, nullptr, (T*)lv.r, (T*)nx.b, (T*)nx.x);
        else op_launch<T, SV_Y>(s, lv.Rop, nullptr, nullptr, (T*)lv.r, (T*)nx.b, nullptr);
    }
    AmgLevel& co = s->levels[L - 1];
    if (co.n > 0) {
        dense_gemv<T><<<ceil_div(co.n, 256 / WAVE), 256, 0, s->stream>>>((const T*)s->coarse_inv, co.n,
                                                                        (T*)co.b, (T*)co.x);
        DP_LAUNCH_CHECK();
    }
    T* xs = (T*)co.x;
    for (int l = L - 2; l >= 0; --l) {
        AmgLevel& lv = s->levels[l];
        op_launch<T, SV_PROL>(s, lv.Pop, nullptr, nullptr, xs, (T*)lv.x, nullptr);
        if (l == 0) st0_launch<T, SV_POST>(s, lv, (T*)lv.dinv, (T*)lv.b, (T*)lv.x, (T*)lv.t, nullptr);
        else op_launch<T, SV_POST>(s, lv.Aop, (T*)lv.dinv, (T*)lv.b, (T*)lv.x, (T*)lv.t, nullptr);
        xs = (T*)lv.t;
    }
    return xs;
}
template double* amg_vcycle<double>(dp_sim*);
template float* amg_vcycle<float>(dp_sim*);

}  // namespace dp

// ---------------------------------------------------------------------------
// Test hooks: one preconditioner stage, dense inverse self-test
// ---------------------------------------------------------------------------
namespace dp {

__global__ void set_flag_kernel(int* p, int v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

// One dense inverse with its device scratch taken from 'ar': the matrix padded
// to a multiple of the panel width (identity in the padding), the two pivot
// blocks, one column panel and the pivot flag.  a and ainv are host arrays
// (row-major n x n); synchronises st.
static dp_status dense_inverse_in(Arena& ar, const double* a, int n, double* ainv, hipStream_t st) {
    int np = ((n + GJ_B - 1) / GJ_B) * GJ_B;
    double* M = ar.get<double>((int64_t)np * np, "dense matrix");
    double* P = ar.get<double>(2 * GJ_B * GJ_B, "pivot blocks");
    double* C = ar.get<double>((int64_t)np * GJ_B, "column panel");
    int* bad = ar.get<int>(1, "flag");
    std::vector<double> h((size_t)np * np, 0.0);
    for (int r = 0; r < np; ++r)
        for (int c = 0; c < np; ++c)
            h[(size_t)r * np + c] = (r < n && c < n) ? a[(size_t)r * n + c] : (r == c ? 1.0 : 0.0);
    DP_HIP(hipMemcpyAsync(M, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st));
    set_flag_kernel<<<1, 64, 0, st>>>(bad, 0);
    DP_LAUNCH_CHECK();
    gj_invert(st, M, np, P, C, bad);
    int hb = 0;
    DP_HIP(hipMemcpyAsync(h.data(), M, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    DP_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    DP_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) ainv[(size_t)r * n + c] = h[(size_t)r * np + c];
    return hb ? DP_E_NUMERIC : DP_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the scratch of dense_inverse_in for n up to
// DENSE_NOALLOC_MAX lives in a static device array of this module.  Host code
// never passes the array's name (a host-side stand-in, not a device address):
// its address on each device is looked up once with hipGetSymbolAddress, with
// that device current, and kept per device.  One lock serialises the calls of
// this process, which all share the array.
// ---------------------------------------------------------------------------
constexpr int DENSE_NOALLOC_MAX = 1024;
constexpr size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t DENSE_NOALLOC_BYTES =
    round256(sizeof(double) * (size_t)DENSE_NOALLOC_MAX * DENSE_NOALLOC_MAX) +
    round256(sizeof(double) * 2 * GJ_B * GJ_B) + round256(sizeof(double) * (size_t)DENSE_NOALLOC_MAX * GJ_B) +
    round256(sizeof(int));

static __device__ __align__(256) unsigned char scratch[DENSE_NOALLOC_BYTES];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;  // per device ordinal; null until looked up

// Device address of 'scratch' on the current device (caller holds g_scratch_mu).
static void* scratch_on_current_device() {
    int dev = 0;
    DP_HIP(hipGetDevice(&dev));
    if (dev < 0) fail(DP_E_DEVICE, "no current device");
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            fail(DP_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace dp

extern "C" dp_status dp_selftest_dense_inverse(const double* a, int32_t n, double* ainv, void* d_ws,
                                               size_t bytes, void* stream) {
    using namespace dp;
    if (!a || !ainv || !d_ws || n <= 0 || n > 4096) return DP_E_INVALID;
    try {
        Arena ar;
        ar.base = (char*)d_ws;
        ar.cap = bytes;
        return dense_inverse_in(ar, a, n, ainv, (hipStream_t)stream);
    } catch (const Error& e) {
        return e.code;
    }
}

extern "C" dp_status dp_selftest_dense_inverse_noalloc(const double* a, int32_t n, double* ainv,
                                                       void* stream) {
    using namespace dp;
    if (!a || !ainv || n <= 0 || n > DENSE_NOALLOC_MAX) return DP_E_INVALID;
    try {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        Arena ar;
        ar.base = (char*)scratch_on_current_device();
        ar.cap = DENSE_NOALLOC_BYTES;
        return dense_inverse_in(ar, a, n, ainv, (hipStream_t)stream);
    } catch (const Error& e) {
        return e.code;
    }
}
