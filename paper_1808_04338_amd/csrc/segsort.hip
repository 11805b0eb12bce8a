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
//     it has at most SW_MAX terms, else listed for workgroup tiles that
//     take up to SM_MAX terms (25 KB of LDS), then up to SB_MAX (101 KB);
//   * a longer row is listed once more, and the listed rows' terms are sorted
//     together by the stable global radix sort on (list index, column): the
//     same order, sums and compaction as a tile, written back in place (the
//     call returns false, and the caller takes the global path for the whole
//     product, only when the scratch region cannot hold those terms).
// Sorting is a bitonic network on 64-bit keys; sums, compaction ranks (ballot
// prefix counts) and row lengths are deterministic.
#include <initializer_list>
#include <type_traits>

#include "primitives.h"

namespace dp {

constexpr int SW_MAX = 256;
constexpr int SM_MAX = 1024;  // 25 KB of LDS per workgroup
constexpr int SB_MAX = 4096;  // 101 KB of LDS per workgroup
constexpr int SM_NT = 256;    // threads of a workgroup tile of SM_MAX terms
constexpr int SB_NT = 1024;   // threads of a workgroup tile of SB_MAX terms
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
    int nh;                        // run heads listed (in eo)
    int wsum[16];                  // workgroup tiles: kept heads per wavefront's part
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

// Bitonic stages in registers over a wavefront's KPL * WAVE consecutive keys
// starting at element base: element e = base + KPL * lane + i sits in register
// i of its lane.  Stages j = jstart, jstart / 2, ..., 1 of merge step k: those
// with a distance below KPL compare registers of one lane, the others exchange
// the same register with lane ^ (j / KPL).  Element e keeps the minimum of its
// pair when (e is the lower of the pair) == (the pair sorts ascending,
// e & k == 0), exactly the compare-exchange of the LDS network.
template <int KPL>
__device__ inline void reg_stages(uint64_t (&v)[KPL], int base, int k, int jstart) {
    const int lane = threadIdx.x % WAVE;
    const int e0 = base + KPL * lane;
#pragma unroll
    for (int j = jstart; j > 0; j >>= 1) {
        if (j < KPL) {
#pragma unroll
            for (int i = 0; i < KPL; ++i) {
                if ((i & j) == 0) {
                    const int l = i | j;
                    const bool up = ((e0 + i) & k) == 0;
                    const uint64_t a = v[i], b = v[l];
                    const uint64_t mn = a < b ? a : b, mx = a < b ? b : a;
                    v[i] = up ? mn : mx;
                    v[l] = up ? mx : mn;
                }
            }
        } else {
            const int lj = j / KPL;
            const bool lower = (lane & lj) == 0;
#pragma unroll
            for (int i = 0; i < KPL; ++i) {
                const uint64_t o = __shfl_xor(v[i], lj, WAVE);
                const bool up = ((e0 + i) & k) == 0;
                const uint64_t mn = v[i] < o ? v[i] : o, mx = v[i] < o ? o : v[i];
                v[i] = (lower == up) ? mn : mx;
            }
        }
    }
}

// The whole bitonic network over the KPL * WAVE keys of one wavefront.
template <int KPL>
__device__ inline void wave_bitonic(uint64_t* key) {
    const int lane = threadIdx.x % WAVE;
    constexpr int N = KPL * WAVE;
    uint64_t v[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) v[i] = key[KPL * lane + i];
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) reg_stages<KPL>(v, 0, k, k >> 1);
#pragma unroll
    for (int i = 0; i < KPL; ++i) key[KPL * lane + i] = v[i];
}

// The bitonic network over P2 = NW KPL WAVE keys of a workgroup of NW
// wavefronts: every wavefront sorts its part in registers (the merge steps up
// to the part's size), and each larger merge step k takes its stages of
// distance at least a part in LDS, the rest in registers.  Every stage compares
// the same pairs in the same direction as the plain LDS network.
template <int KPL, int NW>
__device__ __forceinline__ void block_bitonic(uint64_t* key) {
    constexpr int C = KPL * WAVE, P2 = NW * C, NT = NW * WAVE;
    const int tid = threadIdx.x, lane = tid % WAVE;
    const int base = (tid / WAVE) * C;
    uint64_t v[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) v[i] = key[base + KPL * lane + i];
#pragma unroll
    for (int k = 2; k <= C; k <<= 1) reg_stages<KPL>(v, base, k, k >> 1);
#pragma unroll
    for (int i = 0; i < KPL; ++i) key[base + KPL * lane + i] = v[i];
#pragma unroll
    for (int k = 2 * C; k <= P2; k <<= 1) {
        __syncthreads();
        for (int j = k >> 1; j >= C; j >>= 1) {
            for (int p = tid; p < (P2 >> 1); p += NT) {
                const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                const int l = i + j;
                const bool up = (i & k) == 0;
                const uint64_t a = key[i], b = key[l];
                if ((a > b) == up) {
                    key[i] = b;
                    key[l] = a;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < KPL; ++i) v[i] = key[base + KPL * lane + i];
        reg_stages<KPL>(v, base, k, C >> 1);
#pragma unroll
        for (int i = 0; i < KPL; ++i) key[base + KPL * lane + i] = v[i];
    }
    __syncthreads();
}

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
    // bitonic network, ascending: in registers for a one-wavefront tile, in LDS
    // for a workgroup tile (the keys are unique, so both give the same order)
    if constexpr (NT == WAVE && MAXE <= 4 * WAVE) {
        if (P2 <= 2 * WAVE) wave_bitonic<2>(T.key);
        else wave_bitonic<4>(T.key);
        __syncthreads();
    } else if constexpr (NT > WAVE && MAXE >= 2 * NT) {
        // P2 = 2, 4, 8 or 16 times NT here (P2 >= 2 NT); KPL = P2 / NT keys per lane
        constexpr int NW = NT / WAVE;
        if (P2 == 2 * NT) block_bitonic<2, NW>(T.key);
        else if constexpr (MAXE >= 4 * NT) {
            if (P2 == 4 * NT) block_bitonic<4, NW>(T.key);
            else if constexpr (MAXE >= 8 * NT) {
                if (P2 == 8 * NT) block_bitonic<8, NW>(T.key);
                else if constexpr (MAXE >= 16 * NT) block_bitonic<16, NW>(T.key);
            }
        }
    } else {
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
    }
    // run sums at the heads, in term order within each run; a head's sum goes to
    // its own term's slot (every run reads only its own terms).  rank[t] is then
    // 1 at a kept head (a non-zero sum), 0 elsewhere.
    // The heads are listed first (in any order, each run is summed alone) and
    // each thread sums one run, so that a wavefront waits for one run instead of
    // one per position it visits.
    if (tid == 0) T.nh = 0;
    __syncthreads();
    for (int t = tid; t < total; t += NT) {
        const uint64_t rc = T.key[t] >> IB;
        T.rank[t] = 0;
        if (t == 0 || (T.key[t - 1] >> IB) != rc) T.eo[atomicAdd(&T.nh, 1)] = t;
    }
    __syncthreads();
    const int nh = T.nh;
    for (int h = tid; h < nh; h += NT) {
        const int t = T.eo[h];
        const uint64_t rc = T.key[t] >> IB;
        double s = 0.0;
        for (int u = t; u < total && (T.key[u] >> IB) == rc; ++u) s += T.v[T.key[u] & IMASK];
        T.rank[t] = s != 0.0 ? 1 : 0;
        T.v[T.key[t] & IMASK] = s;
    }
    __syncthreads();
    // exclusive ranks of the kept heads, 64 at a time: one wavefront over the
    // tile, or in a workgroup tile each wavefront over its part, then the
    // parts' offsets added
    if constexpr (NT > WAVE) {
        constexpr int NW = NT / WAVE;
        static_assert(NW <= 16, "at most 16 wavefronts per workgroup tile");
        const int w = tid / WAVE, lane = tid % WAVE;
        const int q = ((total + NT - 1) / NT) * WAVE;
        const int c_begin = w * q, c_end = min(total, c_begin + q);
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        int run = 0;
        for (int c0 = c_begin; c0 < c_end; c0 += WAVE) {
            const int t = c0 + lane;
            const bool keep = t < c_end && T.rank[t] != 0;
            const uint64_t m = __ballot(keep);
            if (t < c_end) T.rank[t] = run + __popcll(m & lt);
            run += __popcll(m);
        }
        if (lane == 0) T.wsum[w] = run;
        __syncthreads();
        int off = 0;
        for (int i = 0; i < w; ++i) off += T.wsum[i];
        if (off)
            for (int t = c_begin + lane; t < c_end; t += WAVE) T.rank[t] += off;
        if (tid == 0) {
            int kept = 0;
            for (int i = 0; i < NW; ++i) kept += T.wsum[i];
            T.rank[total] = kept;
        }
    } else if (tid < WAVE) {
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
    for (int h = tid; h < nh; h += NT) {
        const int t = T.eo[h];
        uint64_t kt = T.key[t];
        uint64_t rc = kt >> IB;
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
template <int MAXE, int NT, class Src>
__global__ void __launch_bounds__(NT) seg_block(Src S, const int* __restrict__ list, const int* nlist,
                                                 int64_t* cnt, int* next, int* nnext, int* overflow) {
    extern __shared__ char smem[];
    SegTile<MAXE>& T = *reinterpret_cast<SegTile<MAXE>*>(smem);
    const int nl = *nlist;
    for (int q = blockIdx.x; q < nl; q += gridDim.x) {
        int r = list[q];
        if (fits<MAXE>(S, r, r + 1)) {
            tile_run<NT, MAXE>(T, S, r, r + 1, cnt);
        } else if (threadIdx.x == 0) {
            cnt[r] = 0;  // set by the tier (or the global sort) that takes the row
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
    // the group's row offsets (G <= SEG_GMAX) in LDS for the per-entry row search
    __shared__ int rp[SEG_GMAX + 1];
    __shared__ int64_t ro[SEG_GMAX];
    int r0 = blockIdx.x * G;
    int r1 = min(r0 + G, nrows);
    for (int i = threadIdx.x; i <= r1 - r0; i += WAVE) {
        rp[i] = rowptr[r0 + i];
        if (i < r1 - r0) ro[i] = off[r0 + i];
    }
    __syncthreads();
    int o0 = rp[0], o1 = rp[r1 - r0];
    for (int o = o0 + (int)threadIdx.x; o < o1; o += WAVE) {
        int rl = upper_idx(rp, r1 - r0, o);
        int64_t src = ro[rl] + (o - rp[rl]);
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

// ---------------------------------------------------------------------------
// Rows beyond the largest tile (list of n3 rows).  Their terms are written in
// term order keyed (list index << cbits | column), sorted by the stable radix
// sort, summed per run in sorted (= term) order and compacted at the row's
// term offset exactly as a tile would.
// ---------------------------------------------------------------------------
template <class Src>
__global__ void long_len(Src S, const int* __restrict__ list, int n3, int64_t* len) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) len[i] = S.off[list[i] + 1] - S.off[list[i]];
}

// one workgroup per listed row: X entries in order, each one's Y row spread
// over the threads
__global__ void __launch_bounds__(256) long_expand(ProdSrc S, const int* __restrict__ list,
                                                   const int64_t* __restrict__ loff, int cbits, uint64_t* key,
                                                   double* val) {
    const int i = blockIdx.x;
    const int r = list[i];
    int64_t o = loff[i];
    for (int e = S.X.rowptr[r]; e < S.X.rowptr[r + 1]; ++e) {
        const int k = S.X.col[e];
        const int a = S.Y.rowptr[k], b = S.Y.rowptr[k + 1];
        const double xv = S.X.val[e];
        for (int f = a + (int)threadIdx.x; f < b; f += blockDim.x) {
            key[o + (f - a)] = ((uint64_t)i << cbits) | (uint64_t)(uint32_t)S.Y.col[f];
            val[o + (f - a)] = xv * S.Y.val[f];
        }
        o += b - a;
    }
}
__global__ void __launch_bounds__(256) long_expand(BufSrc S, const int* __restrict__ list,
                                                   const int64_t* __restrict__ loff, int cbits, uint64_t* key,
                                                   double* val) {
    const int i = blockIdx.x;
    const int r = list[i];
    const int64_t b0 = S.off[r], n = S.off[r + 1] - b0, o = loff[i];
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        key[o + t] = ((uint64_t)i << cbits) | (uint64_t)(uint32_t)S.col[b0 + t];
        val[o + t] = S.val[b0 + t];
    }
}

// run heads: the sum of the run in order, and whether it is kept (non-zero)
__global__ void long_sum(const uint64_t* __restrict__ key, const double* __restrict__ val, int64_t T,
                         int64_t* keep, double* sum) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const uint64_t k = key[t];
    const bool head = t == 0 || key[t - 1] != k;
    double s = 0.0;
    if (head)
        for (int64_t u = t; u < T && key[u] == k; ++u) s += val[u];
    keep[t] = (head && s != 0.0) ? 1 : 0;
    sum[t] = s;
}

// kept heads to the row's term offset (pos: exclusive ranks of keep; loff has
// n3 + 1 entries); row lengths of the listed rows into cnt
__global__ void long_counts(const int* __restrict__ list, int n3, const int64_t* __restrict__ loff,
                            const int64_t* __restrict__ pos, int64_t T, int64_t kept, int64_t* cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    int64_t a = loff[i], b = loff[i + 1];
    int64_t pa = a < T ? pos[a] : kept, pb = b < T ? pos[b] : kept;
    cnt[list[i]] = pb - pa;
}
template <class Src>
__global__ void long_write(Src S, const int* __restrict__ list, const int64_t* __restrict__ loff,
                           const uint64_t* __restrict__ key, const double* __restrict__ sum,
                           const int64_t* __restrict__ keep, const int64_t* __restrict__ pos, int64_t T,
                           int cbits) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T || !keep[t]) return;
    const uint64_t k = key[t];
    const int i = (int)(k >> cbits);
    const int r = list[i];
    const int64_t o = S.off[r] + (pos[t] - pos[loff[i]]);
    const int c = (int)(k & ((1ull << cbits) - 1));
    if constexpr (std::is_same<Src, ProdSrc>::value) {
        S.ocol[o] = c;
        S.oval[o] = sum[t];
    } else {
        S.col[o] = c;
        S.val[o] = sum[t];
    }
}

// row lengths back from their exclusive scan (total: the sum)
__global__ void unscan(const int64_t* __restrict__ ex, int n, int64_t total, int64_t* len) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) len[r] = (r + 1 < n ? ex[r + 1] : total) - ex[r];
}

static size_t arena_need(std::initializer_list<size_t> bytes) {
    size_t t = 0;
    for (size_t b : bytes) t += ((b + 255) & ~size_t(255)) + 256;
    return t;
}

// The listed rows (n3 > 0) of a product whose other rows the tiles finished:
// cnt holds the exclusive scan of the row lengths (total: its sum; the listed
// rows counted as empty).  On success cnt points at the scan of
// the corrected lengths and total is their sum.  Returns false, with the
// scratch released, when the sort's buffers do not fit.
template <class Src>
static bool long_rows(hipStream_t st, const Src& S, const int* list, int n3, int nrows, int ncols,
                      int64_t*& cnt, int64_t& total, Arena& sc) {
    const size_t mark = sc.top;
    if (sc.top + arena_need({8 * (size_t)(n3 + 1), 8 * (size_t)scan_tmp_size(n3 + 1)}) > sc.cap) return false;
    int64_t* loff = sc.get<int64_t>(n3 + 1, "long rows");
    int64_t* ltmp = sc.get<int64_t>(scan_tmp_size(n3 + 1), "scan tmp");
    long_len<Src><<<ceil_div(n3, 256), 256, 0, st>>>(S, list, n3, loff);
    DP_LAUNCH_CHECK();
    int64_t T = 0;
    exclusive_scan(st, loff, n3, ltmp, &T);
    seg_set_last<<<1, 1, 0, st>>>(loff, n3, T);
    DP_LAUNCH_CHECK();
    const int cbits = bits_for(ncols);
    const int nbits = bits_for(n3) + cbits;
    const size_t need = arena_need({8 * (size_t)(nrows + 1), 8 * (size_t)T, 8 * (size_t)T, 8 * (size_t)T,
                                    8 * (size_t)T, 8 * (size_t)sort_tmp_size(T), 8 * (size_t)(T + 1),
                                    8 * (size_t)(T + 1), 8 * (size_t)scan_tmp_size(T + 1),
                                    8 * (size_t)scan_tmp_size(nrows + 1)});
    if (nbits > 64 || sc.top + need > sc.cap) {
        sc.top = mark;
        return false;
    }
    int64_t* len = sc.get<int64_t>(nrows + 1, "segment counts");
    uint64_t* k0 = sc.get<uint64_t>(T, "long row keys");
    double* v0 = sc.get<double>(T, "long row values");
    uint64_t* k1 = sc.get<uint64_t>(T, "long row keys");
    double* v1 = sc.get<double>(T, "long row values");
    int64_t* rtmp = sc.get<int64_t>(sort_tmp_size(T), "sort tmp");
    int64_t* keep = sc.get<int64_t>(T + 1, "long row flags");
    int64_t* pos = sc.get<int64_t>(T + 1, "long row ranks");
    int64_t* ktmp = sc.get<int64_t>(scan_tmp_size(T + 1), "scan tmp");
    int64_t* ntmp = sc.get<int64_t>(scan_tmp_size(nrows + 1), "scan tmp");
    unscan<<<ceil_div(nrows, 256), 256, 0, st>>>(cnt, nrows, total, len);
    long_expand<<<n3, 256, 0, st>>>(S, list, loff, cbits, k0, v0);
    DP_LAUNCH_CHECK();
    const int which = radix_sort(st, k0, v0, k1, v1, T, nbits, rtmp);
    const uint64_t* ks = which ? k1 : k0;
    const double* vs = which ? v1 : v0;
    double* sums = which ? v0 : v1;  // the idle half of the double buffer
    long_sum<<<ceil_div(T, 256), 256, 0, st>>>(ks, vs, T, keep, sums);
    DP_LAUNCH_CHECK();
    DP_HIP(hipMemcpyAsync(pos, keep, sizeof(int64_t) * T, hipMemcpyDeviceToDevice, st));
    int64_t kept = 0;
    exclusive_scan(st, pos, T, ktmp, &kept);
    long_counts<<<ceil_div(n3, 256), 256, 0, st>>>(list, n3, loff, pos, T, kept, len);
    long_write<Src><<<ceil_div(T, 256), 256, 0, st>>>(S, list, loff, ks, sums, keep, pos, T, cbits);
    DP_LAUNCH_CHECK();
    exclusive_scan(st, len, nrows, ntmp, &total);
    cnt = len;
    return true;
}

// Shared driver: runs the tiles, then scans the row lengths and copies the
// compacted rows (found at off[r] of rcol/rval) into the CSR from 'out'.
template <class Src>
static bool seg_run(hipStream_t st, const Src& S, const int64_t* off, int nrows, int ncols, int64_t m,
                    const int* rcol, const double* rval, Arena& sc, Arena& out, Csr& csr, const char* what,
                    KernelTimer* kt = nullptr, double xbytes = 0.0, int64_t* long_products = nullptr) {
    if (ncols >= (1 << 28) || nrows >= (1 << 24)) return false;  // key packing
    int64_t* cnt = sc.get<int64_t>(nrows + 1, "segment counts");
    int64_t* tmp = sc.get<int64_t>(scan_tmp_size(nrows + 1), "scan tmp");
    int* longlist = sc.get<int>(nrows, "long rows");
    int* list2 = sc.get<int>(nrows, "long rows");
    int* flags = sc.get<int>(4, "segment flags");  // [0] long rows, [1] longer rows, [2] beyond the tiles
    DP_HIP(hipMemsetAsync(flags, 0, 4 * sizeof(int), st));
    double avg = nrows > 0 ? (double)m / nrows : 0.0;
    int G = avg > 0 ? (int)(SEG_TARGET / avg) : SEG_GMAX;
    G = std::max(1, std::min(SEG_GMAX, G));
    int ngroups = ceil_div(nrows, G);
    int64_t total = 0;
    int hf[4] = {0, 0, 0, 0};
    if (nrows > 0) {
        size_t shm_m = sizeof(SegTile<SM_MAX>), shm_b = sizeof(SegTile<SB_MAX>);
        DP_HIP(hipFuncSetAttribute((const void*)seg_block<SB_MAX, SB_NT, Src>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm_b));
        int kidx;
        {
            // timed as one group: wavefront tiles, then the two workgroup tiers
            KtScope ks(kt, st);
            kidx = ks.idx;
            seg_wave<Src><<<ngroups, WAVE, 0, st>>>(S, nrows, G, cnt, longlist, flags);
            seg_block<SM_MAX, SM_NT, Src><<<1024, SM_NT, shm_m, st>>>(S, longlist, flags, cnt, list2, flags + 1,
                                                                    flags + 2);
            // rows beyond SB_MAX go back to the first list (consumed by then)
            seg_block<SB_MAX, SB_NT, Src><<<256, SB_NT, shm_b, st>>>(S, list2, flags + 1, cnt, longlist, flags + 2,
                                                                    flags + 3);
            DP_LAUNCH_CHECK();
        }
        // the flags arrive with the scan's synchronisation
        int* hfp = reinterpret_cast<int*>(pinned_slots() + 1);
        DP_HIP(hipMemcpyAsync(hfp, flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
        exclusive_scan(st, cnt, nrows, tmp, &total);
        for (int i = 0; i < 4; ++i) hf[i] = hfp[i];
        if (hf[2]) {
            if (!long_rows(st, S, longlist, hf[2], nrows, ncols, cnt, total, sc)) return false;
            if (long_products) *long_products += 1;
        }
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
                     int64_t m, Arena& sc, Arena& out, Csr& csr, const char* what, int64_t* long_products) {
    size_t mark = sc.top;
    BufSrc S{off, col, val};
    bool ok = seg_run(st, S, off, nrows, ncols, m, col, val, sc, out, csr, what, nullptr, 0.0, long_products);
    if (!ok || &out != &sc) sc.top = mark;
    return ok;
}

bool seg_product(hipStream_t st, const Csr& X, const Csr& Y, Arena& sc, Arena& out, Csr& C, const char* what,
                 KernelTimer* kt, int64_t* long_products) {
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
    bool ok = seg_run(st, S, off, nrows, Y.ncols, m, ocol, oval, sc, out, C, what, kt, xbytes, long_products);
    if (!ok || &out != &sc) sc.top = mark;
    return ok;
}

}  // namespace dp
