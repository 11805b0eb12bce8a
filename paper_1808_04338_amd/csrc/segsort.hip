// Row-wise sparse sums into CSR, for AMG setup products whose terms are known
// per output row: the interpolation rows (terms staged in a buffer) and the
// products C = X Y (terms generated on the fly from X and Y).
//
// Row r's terms are ordered by column with ties kept in term order, equal
// columns are summed sequentially in term order and zero sums are dropped.
// Rows are processed in LDS:
//   * one wavefront per group of G consecutive rows whose terms (at most SW_MAX
//     together) are sorted at once on the key (row, col, term index) -- rows
//     stay inside their own index ranges, so groups need no merge;
//   * a row that does not fit its group is handled alone by the wavefront when
//     it has at most SW_MAX terms, else listed for 256-thread workgroups that
//     take up to SM_MAX terms (25 KB of LDS), then up to SB_MAX (101 KB);
//   * a longer row makes the call return false (the caller then takes the
//     global radix-sort path).
// Sorting is a bitonic network on 64-bit keys; sums, compaction ranks (ballot
// prefix counts) and row lengths are deterministic.
#include <type_traits>

#include "primitives.h"

namespace dp {

constexpr int SW_MAX = 256;
constexpr int SM_MAX = 1024;  // 25 KB of LDS per workgroup
constexpr int SB_MAX = 4096;  // 101 KB of LDS per workgroup
constexpr int SEG_TARGET = 128;  // terms per wavefront group
constexpr int SEG_GMAX = 64;     // rows per group

// MAXE is a power of two: the bitonic network runs over pow2ceil(terms) <= MAXE keys
template <int MAXE>
struct SegTile {
    static_assert((MAXE & (MAXE - 1)) == 0, "tile size must be a power of two");
    uint64_t key[MAXE];
    double v[MAXE];       // term values in term order; run sums at run heads
    int rank[MAXE + 1];   // product mode, before the sort: Y row start of every X entry
    int eo[MAXE + 1];     // product mode: term offset of every X entry of the tile
    unsigned char erow[MAXE];  // product mode: tile-local row of every X entry
    int64_t rowoff[SEG_GMAX + 1];  // term offsets of the tile's rows
    int xoff[SEG_GMAX + 1];        // product mode: X entry offsets of the tile's rows
};

__device__ inline int pow2ceil(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// last index i in [0, n) with a[i] <= x (a ascending, a[0] <= x)
template <class A>
__device__ inline int upper_idx(const A* a, int n, long long x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((long long)a[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Term sources.  Buffer: terms of row r at [off[r], off[r+1]) of (col, val),
// results written back in place.  Product: row r of X Y, terms (Y.col[f],
// X.val[e] * Y.val[f]) for e in X_r, f in Y_{X.col[e]}; results written at the
// row's term offset into separate arrays.
struct BufSrc {
    const int64_t* off;
    int* col;
    double* val;
};
struct ProdSrc {
    const int64_t* off;
    Csr X, Y;
    int* ocol;
    double* oval;
};

template <int NT, int MAXE, class Src>
__device__ void tile_run(SegTile<MAXE>& T, const Src& S, int ra, int rb, int64_t* cnt) {
    constexpr int IB = MAXE > 2048 ? 12 : (MAXE > 512 ? 11 : 9);  // bits of the term index (t < MAXE)
    constexpr uint64_t IMASK = (1ull << IB) - 1;
    constexpr uint64_t CMASK = (1ull << (40 - IB)) - 1;
    constexpr bool PROD = std::is_same<Src, ProdSrc>::value;
    const int tid = threadIdx.x;
    const int nr = rb - ra;
    for (int i = tid; i <= nr; i += NT) {
        T.rowoff[i] = S.off[ra + i];
        if constexpr (PROD) T.xoff[i] = S.X.rowptr[ra + i];
    }
    __syncthreads();
    const int64_t base = T.rowoff[0];
    const int total = (int)(T.rowoff[nr] - base);
    const int P2 = max(2 * NT, pow2ceil(total));
    if constexpr (PROD) {
        // every X entry of the tile, all threads: its Y row start and term count
        // (one round of dependent loads) and its tile-local row, kept in LDS
        const int e0 = T.xoff[0], ne = T.xoff[nr] - e0;
        for (int j = tid; j < ne; j += NT) {
            int k = S.X.col[e0 + j];
            int a = S.Y.rowptr[k];
            T.eo[j] = S.Y.rowptr[k + 1] - a;
            T.rank[j] = a;
            T.erow[j] = (unsigned char)upper_idx(T.xoff, nr, e0 + j);
        }
        __syncthreads();
        // exclusive scan of the term counts into term offsets (wave 0, 64 at a time)
        if (tid < WAVE) {
            int run = 0;
            for (int c0 = 0; c0 < ne; c0 += WAVE) {
                int j = c0 + tid;
                int len = j < ne ? T.eo[j] : 0;
                int x = len;
#pragma unroll
                for (int o = 1; o < WAVE; o <<= 1) {
                    int y = __shfl_up(x, o, WAVE);
                    if (tid >= o) x += y;
                }
                if (j < ne) T.eo[j] = run + x - len;
                run += __shfl(x, WAVE - 1, WAVE);
            }
            if (tid == 0) T.eo[ne] = run;
        }
        __syncthreads();
        for (int t = tid; t < P2; t += NT) {
            if (t < total) {
                // entries with no terms have equal offsets: upper_idx gives the last one
                int j = upper_idx(T.eo, ne, t);
                int f = T.rank[j] + (t - T.eo[j]);
                T.key[t] = ((uint64_t)T.erow[j] << 40) | ((uint64_t)(uint32_t)S.Y.col[f] << IB) | (uint64_t)t;
                T.v[t] = S.X.val[e0 + j] * S.Y.val[f];
            } else {
                T.key[t] = ~0ull;
            }
        }
        __syncthreads();  // the sums below overwrite rank
    } else {
        for (int t = tid; t < P2; t += NT) {
            if (t < total) {
                int rl = upper_idx(T.rowoff, nr, base + t);
                T.key[t] = ((uint64_t)rl << 40) | ((uint64_t)(uint32_t)S.col[base + t] << IB) | (uint64_t)t;
                T.v[t] = S.val[base + t];
            } else {
                T.key[t] = ~0ull;
            }
        }
    }
    __syncthreads();
    // bitonic network, ascending
    for (int k = 2; k <= P2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = tid; p < (P2 >> 1); p += NT) {
                int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                int l = i + j;
                bool up = (i & k) == 0;
                uint64_t a = T.key[i], b = T.key[l];
                if ((a > b) == up) {
                    T.key[i] = b;
                    T.key[l] = a;
                }
            }
            __syncthreads();
        }
    }
    // run sums at the heads, in term order within each run; a head's sum goes to
    // its own term's slot (every run reads only its own terms)
    for (int t = tid; t < total; t += NT) {
        uint64_t rc = T.key[t] >> IB;
        bool head = t == 0 || (T.key[t - 1] >> IB) != rc;
        double s = 0.0;
        if (head) {
            for (int u = t; u < total && (T.key[u] >> IB) == rc; ++u) s += T.v[T.key[u] & IMASK];
        }
        T.rank[t] = (head && s != 0.0) ? 1 : 0;
        if (head) T.v[T.key[t] & IMASK] = s;
    }
    __syncthreads();
    // exclusive ranks of the kept heads (wave 0, 64 at a time)
    if (tid < WAVE) {
        int run = 0;
        uint64_t lt = tid == 0 ? 0ull : (~0ull >> (64 - tid));
        for (int c0 = 0; c0 < total; c0 += WAVE) {
            int t = c0 + tid;
            bool keep = t < total && T.rank[t] != 0;
            uint64_t m = __ballot(keep);
            if (t < total) T.rank[t] = run + __popcll(m & lt);
            run += __popcll(m);
        }
        if (tid == 0) T.rank[total] = run;
    }
    __syncthreads();
    for (int i = tid; i < nr; i += NT) {
        int s0 = (int)(T.rowoff[i] - base), s1 = (int)(T.rowoff[i + 1] - base);
        cnt[ra + i] = T.rank[s1] - T.rank[s0];
    }
    for (int t = tid; t < total; t += NT) {
        uint64_t kt = T.key[t];
        uint64_t rc = kt >> IB;
        bool head = t == 0 || (T.key[t - 1] >> IB) != rc;
        if (!head) continue;
        double s = T.v[kt & IMASK];
        if (s == 0.0) continue;
        int rl = (int)(kt >> 40);
        int s0 = (int)(T.rowoff[rl] - base);
        int64_t o = T.rowoff[rl] + (T.rank[t] - T.rank[s0]);
        if constexpr (PROD) {
            S.ocol[o] = (int)(rc & CMASK);
            S.oval[o] = s;
        } else {
            S.col[o] = (int)(rc & CMASK);
            S.val[o] = s;
        }
    }
    __syncthreads();
}

// Does rows [ra, rb) fit one tile of MAXE terms (and, for products, X entries)?
template <int MAXE, class Src>
__device__ inline bool fits(const Src& S, int ra, int rb) {
    if (S.off[rb] - S.off[ra] > MAXE) return false;
    if constexpr (std::is_same<Src, ProdSrc>::value) {
        if (S.X.rowptr[rb] - S.X.rowptr[ra] > MAXE) return false;
    }
    return true;
}

template <class Src>
__global__ void __launch_bounds__(WAVE) seg_wave(Src S, int nrows, int G, int64_t* cnt, int* longlist,
                                                 int* nlong) {
    __shared__ SegTile<SW_MAX> T;
    int r0 = blockIdx.x * G;
    int r1 = min(r0 + G, nrows);
    if (fits<SW_MAX>(S, r0, r1)) {
        tile_run<WAVE, SW_MAX>(T, S, r0, r1, cnt);
        return;
    }
    for (int r = r0; r < r1; ++r) {
        if (fits<SW_MAX>(S, r, r + 1)) {
            tile_run<WAVE, SW_MAX>(T, S, r, r + 1, cnt);
        } else if (threadIdx.x == 0) {
            longlist[atomicAdd(nlong, 1)] = r;
        }
    }
}

// Persistent workgroups over a list of long rows (count in *nlist): rows of at
// most MAXE terms are done here, longer ones go to the next list, or raise the
// overflow flag when there is none.
template <int MAXE, class Src>
__global__ void __launch_bounds__(256) seg_block(Src S, const int* __restrict__ list, const int* nlist,
                                                 int64_t* cnt, int* next, int* nnext, int* overflow) {
    extern __shared__ char smem[];
    SegTile<MAXE>& T = *reinterpret_cast<SegTile<MAXE>*>(smem);
    const int nl = *nlist;
    for (int q = blockIdx.x; q < nl; q += gridDim.x) {
        int r = list[q];
        if (fits<MAXE>(S, r, r + 1)) {
            tile_run<256, MAXE>(T, S, r, r + 1, cnt);
        } else if (threadIdx.x == 0) {
            if (next) next[atomicAdd(nnext, 1)] = r;
            else *overflow = 1;
        }
    }
}

// CSR copy: group g's rows [r0, r1) occupy [rowptr[r0], rowptr[r1]) of the
// output; entry o of row r comes from off[r] + (o - rowptr[r]).
__global__ void __launch_bounds__(WAVE) seg_copy(const int64_t* __restrict__ off, const int* __restrict__ rowptr,
                                                 int nrows, int G, const int* __restrict__ col,
                                                 const double* __restrict__ val, int* ocol, double* oval) {
    int r0 = blockIdx.x * G;
    int r1 = min(r0 + G, nrows);
    int o0 = rowptr[r0], o1 = rowptr[r1];
    for (int o = o0 + (int)threadIdx.x; o < o1; o += WAVE) {
        int r = r0 + upper_idx(rowptr + r0, r1 - r0, o);
        int64_t src = off[r] + (o - rowptr[r]);
        ocol[o] = col[src];
        oval[o] = val[src];
    }
}

__global__ void seg_rowptr(const int64_t* __restrict__ c, int n, int64_t total, int* rowptr) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rowptr[i] = (int)c[i];
    if (i == n) rowptr[n] = (int)total;
}

__global__ void seg_set_last(int64_t* off, int n, int64_t m) { off[n] = m; }

// terms of row r of X Y
// Terms of every product row, PCL lanes per row (row lengths reach 50 on the
// coarse levels).
constexpr int PCL = 8;
__global__ void prod_count(Csr X, Csr Y, int64_t* cnt) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int r = g / PCL, l = g % PCL;
    if (r >= X.n) return;  // whole subgroup
    long long c = 0;
    for (int e = X.rowptr[r] + l; e < X.rowptr[r + 1]; e += PCL) {
        int k = X.col[e];
        c += Y.rowptr[k + 1] - Y.rowptr[k];
    }
#pragma unroll
    for (int o = PCL / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, PCL);
    if (l == 0) cnt[r] = c;
}

// Shared driver: runs the tiles, then scans the row lengths and copies the
// compacted rows (found at off[r] of rcol/rval) into the CSR from 'out'.
template <class Src>
static bool seg_run(hipStream_t st, const Src& S, const int64_t* off, int nrows, int ncols, int64_t m,
                    const int* rcol, const double* rval, Arena& sc, Arena& out, Csr& csr, const char* what,
                    KernelTimer* kt = nullptr, double xbytes = 0.0) {
    if (ncols >= (1 << 28) || nrows >= (1 << 24)) return false;  // key packing
    int64_t* cnt = sc.get<int64_t>(nrows + 1, "segment counts");
    int64_t* tmp = sc.get<int64_t>(scan_tmp_size(nrows + 1), "scan tmp");
    int* longlist = sc.get<int>(nrows, "long rows");
    int* list2 = sc.get<int>(nrows, "long rows");
    int* flags = sc.get<int>(4, "segment flags");  // [0] long rows, [1] longer rows, [2] overflow
    DP_HIP(hipMemsetAsync(flags, 0, 4 * sizeof(int), st));
    double avg = nrows > 0 ? (double)m / nrows : 0.0;
    int G = avg > 0 ? (int)(SEG_TARGET / avg) : SEG_GMAX;
    G = std::max(1, std::min(SEG_GMAX, G));
    int ngroups = ceil_div(nrows, G);
    int64_t total = 0;
    int hf[4] = {0, 0, 0, 0};
    if (nrows > 0) {
        size_t shm_m = sizeof(SegTile<SM_MAX>), shm_b = sizeof(SegTile<SB_MAX>);
        DP_HIP(hipFuncSetAttribute((const void*)seg_block<SB_MAX, Src>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm_b));
        int kidx;
        {
            // timed as one group: wavefront tiles, then the two workgroup tiers
            KtScope ks(kt, st);
            kidx = ks.idx;
            seg_wave<Src><<<ngroups, WAVE, 0, st>>>(S, nrows, G, cnt, longlist, flags);
            seg_block<SM_MAX, Src><<<1024, 256, shm_m, st>>>(S, longlist, flags, cnt, list2, flags + 1, flags + 2);
            seg_block<SB_MAX, Src><<<256, 256, shm_b, st>>>(S, list2, flags + 1, cnt, nullptr, nullptr, flags + 2);
            DP_LAUNCH_CHECK();
        }
        // the flags arrive with the scan's synchronisation
        DP_HIP(hipMemcpyAsync(hf, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
        exclusive_scan(st, cnt, nrows, tmp, &total);
        if (hf[2]) return false;
        // algorithmic bytes: the sources (xbytes), term offsets and row lengths,
        // the results (column and value)
        if (kt && kidx >= 0) kt->bytes += xbytes + 16.0 * (nrows + 1) + 12.0 * total;
    }
    csr.n = nrows;
    csr.ncols = ncols;
    csr.nnz = total;
    csr.rowptr = out.get<int>(nrows + 1, what);
    csr.col = out.get<int>(total, what);
    csr.val = out.get<double>(total, what);
    seg_rowptr<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(cnt, nrows, total, csr.rowptr);
    DP_LAUNCH_CHECK();
    if (total > 0) {
        seg_copy<<<ngroups, WAVE, 0, st>>>(off, csr.rowptr, nrows, G, rcol, rval, csr.col, csr.val);
        DP_LAUNCH_CHECK();
    }
    return true;
}

bool seg_sort_reduce(hipStream_t st, const int64_t* off, int nrows, int ncols, int* col, double* val,
                     int64_t m, Arena& sc, Arena& out, Csr& csr, const char* what) {
    size_t mark = sc.top;
    BufSrc S{off, col, val};
    bool ok = seg_run(st, S, off, nrows, ncols, m, col, val, sc, out, csr, what);
    if (!ok || &out != &sc) sc.top = mark;
    return ok;
}

bool seg_product(hipStream_t st, const Csr& X, const Csr& Y, Arena& sc, Arena& out, Csr& C, const char* what,
                 KernelTimer* kt) {
    size_t mark = sc.top;
    int nrows = X.n;
    int64_t* off = sc.get<int64_t>(nrows + 1, "product rows");
    int64_t* tmp = sc.get<int64_t>(scan_tmp_size(nrows + 1), "scan tmp");
    int64_t m = 0;
    if (nrows > 0) {
        prod_count<<<ceil_div((int64_t)nrows * PCL, 256), 256, 0, st>>>(X, Y, off);
        DP_LAUNCH_CHECK();
        exclusive_scan(st, off, nrows, tmp, &m);
    }
    seg_set_last<<<1, 1, 0, st>>>(off, nrows, m);
    DP_LAUNCH_CHECK();
    int* ocol = sc.get<int>(m, "product terms");
    double* oval = sc.get<double>(m, "product terms");
    ProdSrc S{off, X, Y, ocol, oval};
    // X read once (row offsets, columns, values), Y's row offsets once per X
    // entry and one Y entry (column, value) per term
    double xbytes = 4.0 * (nrows + 1) + 12.0 * X.nnz + 8.0 * X.nnz + 12.0 * m;
    bool ok = seg_run(st, S, off, nrows, Y.ncols, m, ocol, oval, sc, out, C, what, kt, xbytes);
    if (!ok || &out != &sc) sc.top = mark;
    return ok;
}

}  // namespace dp
