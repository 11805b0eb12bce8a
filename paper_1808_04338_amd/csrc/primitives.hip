// Device primitives used by the AMG setup: exclusive scan of int64 counts and a
// stable LSD radix sort of (64-bit key, double) pairs, plus reduce-by-key into
// CSR.  All are deterministic.
#include <mutex>
#include <vector>
#include "primitives.h"

namespace dp {

// ---------------------------------------------------------------------------
// Exclusive scan (in place) of int64 values.  Blocks of 1024 elements
// (256 threads x 4); block totals are scanned recursively.
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256;
constexpr int SCAN_IT = 4;
constexpr int SCAN_TILE = SCAN_T * SCAN_IT;

__device__ inline int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t* total) {
    // inclusive wave scan
    int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int64_t y = __shfl_up(x, o, WAVE);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) sh[wv] = x;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int i = 0; i < SCAN_T / WAVE; ++i) {
        if (i < wv) off += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__global__ void scan_tiles(int64_t* data, int64_t n, int64_t* block_sums) {
    __shared__ int64_t sh[SCAN_T / WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
    int64_t v[SCAN_IT];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_IT; ++i) {
        v[i] = base + i < n ? data[base + i] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t off = block_excl_scan(s, sh, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_IT; ++i) {
        if (base + i < n) data[base + i] = off;
        off += v[i];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ void scan_add(int64_t* data, int64_t n, const int64_t* block_offs) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
    int64_t add = block_offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_IT; ++i)
        if (base + i < n) data[base + i] += add;
}

// Returns the total; data holds the exclusive prefix sums.  tmp needs
// scan_tmp_size(n) int64 entries.
int64_t scan_tmp_size(int64_t n) {
    int64_t tot = 0;
    while (n > 1) {
        n = (n + SCAN_TILE - 1) / SCAN_TILE;
        tot += n + 1;
    }
    return tot + 2;
}

// Returns the device address that holds the sum of all n values: the tile sum
// written by the single tile of the deepest level.
static int64_t* scan_rec(hipStream_t st, int64_t* data, int64_t n, int64_t* tmp) {
    int nblk = ceil_div(n, SCAN_TILE);
    int64_t* sums = tmp;
    scan_tiles<<<nblk, SCAN_T, 0, st>>>(data, n, sums);
    DP_LAUNCH_CHECK();
    if (nblk == 1) return sums;
    int64_t* total = scan_rec(st, sums, nblk, tmp + nblk + 1);
    scan_add<<<nblk, SCAN_T, 0, st>>>(data, n, sums);
    DP_LAUNCH_CHECK();
    return total;
}

void scan_inplace(hipStream_t st, int64_t* data, int64_t n, int64_t* tmp) {
    if (n > 0) scan_rec(st, data, n, tmp);
}

// Small pinned host buffer of the calling thread, for results read back after
// a synchronisation (a DMA into pinned memory instead of a staged pageable
// copy).  A thread takes a buffer from a shared free list (or allocates one)
// on first use and returns it to the list when it exits, so the pinned memory
// held is bounded by the largest number of threads that ran setups at once.
namespace {
std::mutex g_pin_mu;
std::vector<int64_t*> g_pin_free;
struct PinHolder {
    int64_t* p = nullptr;
    ~PinHolder() {
        if (p) {
            std::lock_guard<std::mutex> g(g_pin_mu);
            g_pin_free.push_back(p);
        }
    }
};
}  // namespace

int64_t* pinned_slots() {
    thread_local PinHolder h;
    if (!h.p) {
        {
            std::lock_guard<std::mutex> g(g_pin_mu);
            if (!g_pin_free.empty()) {
                h.p = g_pin_free.back();
                g_pin_free.pop_back();
            }
        }
        if (!h.p) DP_HIP(hipHostMalloc((void**)&h.p, sizeof(int64_t) * PINNED_SLOTS, hipHostMallocDefault));
    }
    return h.p;
}

int64_t exclusive_scan(hipStream_t st, int64_t* data, int64_t n, int64_t* tmp, int64_t* host_total) {
    if (n <= 0) return 0;
    const int64_t* total = scan_rec(st, data, n, tmp + 1);
    int64_t* h = pinned_slots();
    DP_HIP(hipMemcpyAsync(h, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DP_HIP(hipStreamSynchronize(st));
    if (host_total) *host_total = h[0];
    return h[0];
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs, 8-bit digits.
// Upsweep: per-tile digit histogram, digit-major, so that the global exclusive
// scan gives every (digit, tile) its output offset in stable order.
// Downsweep: per tile, elements are ranked round by round (256 per round, in
// index order); within a round the rank among equal digits comes from wave
// ballots and per-wave counts.
// ---------------------------------------------------------------------------
constexpr int RS_T = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_T * RS_ROUNDS;
constexpr int RS_RADIX = 256;

__global__ void rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift, int64_t* hist,
                        int ntiles) {
    __shared__ int cnt[RS_RADIX];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t i = base + r * RS_T + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xFF], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void rs_scatter(const uint64_t* __restrict__ kin, const double* __restrict__ vin,
                           uint64_t* kout, double* vout, int64_t n, int shift,
                           const int64_t* __restrict__ offs, int ntiles) {
    __shared__ int64_t goff[RS_RADIX];
    __shared__ int run[RS_RADIX];
    __shared__ int wcnt[RS_T / WAVE][RS_RADIX];
    goff[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
    run[threadIdx.x] = 0;
    int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        for (int i = threadIdx.x; i < (RS_T / WAVE) * RS_RADIX; i += RS_T) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        int64_t i = base + r * RS_T + threadIdx.x;
        bool valid = i < n;
        uint64_t k = valid ? kin[i] : 0;
        double v = valid ? vin[i] : 0.0;
        int d = (int)((k >> shift) & 0xFF);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot(valid && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        int rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[wv][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int before = 0;
            for (int ww = 0; ww < wv; ++ww) before += wcnt[ww][d];
            int64_t dst = goff[d] + run[d] + before + rank;
            kout[dst] = k;
            vout[dst] = v;
        }
        __syncthreads();
        {
            int dd = threadIdx.x;
            int tot = 0;
            for (int ww = 0; ww < RS_T / WAVE; ++ww) tot += wcnt[ww][dd];
            run[dd] += tot;
        }
        __syncthreads();
    }
}

int64_t sort_tmp_size(int64_t n) {
    int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    int64_t h = ntiles * RS_RADIX;
    return h + scan_tmp_size(h) + 4;
}

// Sorts (k0, v0) by the low 'bits' bits of the key.  Returns 0 if the result is
// in (k0, v0), 1 if in (k1, v1).
int radix_sort(hipStream_t st, uint64_t* k0, double* v0, uint64_t* k1, double* v1, int64_t n,
               int bits, int64_t* tmp) {
    if (n <= 1) return 0;
    int ntiles = ceil_div(n, RS_TILE);
    int64_t* hist = tmp;
    int64_t* stmp = tmp + (int64_t)ntiles * RS_RADIX;
    int cur = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        uint64_t* ki = cur ? k1 : k0;
        double* vi = cur ? v1 : v0;
        uint64_t* ko = cur ? k0 : k1;
        double* vo = cur ? v0 : v1;
        rs_hist<<<ntiles, RS_T, 0, st>>>(ki, n, shift, hist, ntiles);
        DP_LAUNCH_CHECK();
        scan_rec(st, hist, (int64_t)ntiles * RS_RADIX, stmp);
        rs_scatter<<<ntiles, RS_T, 0, st>>>(ki, vi, ko, vo, n, shift, hist, ntiles);
        DP_LAUNCH_CHECK();
        cur ^= 1;
    }
    return cur;
}

// ---------------------------------------------------------------------------
// Reduce sorted (key, value) runs into CSR: equal keys are summed in order,
// exact-zero sums are dropped.  key = row << cbits | col.
// ---------------------------------------------------------------------------
__global__ void rbk_heads(const uint64_t* __restrict__ k, int64_t n, int64_t* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = (i == 0 || k[i] != k[i - 1]) ? 1 : 0;
}

// Segmented sums of the sorted runs, computed by every element in parallel.
// Pass 1 (per wave of 64 consecutive elements): inclusive segmented scan with a
// fixed shuffle tree; each wave records the partial sum running off its end
// (carry) and whether it holds a run start.  Pass 2: the last element of each
// run adds, for a run that began in an earlier wave, the carries of the waves
// back to the one holding its start.  The representative of a run is its last
// element: flag = 1 there if the sum is nonzero.  Deterministic.
__global__ void rbk_scan1(const uint64_t* __restrict__ k, const double* __restrict__ v, int64_t n,
                          double* part, double* carry, int* wave_head) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int lane = threadIdx.x % WAVE;
    bool valid = i < n;
    uint64_t key = valid ? k[i] : 0;
    bool head = valid && (i == 0 || key != k[i - 1]);
    double val = valid ? v[i] : 0.0;
    int flag = head ? 1 : 0;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        double pv = __shfl_up(val, d, WAVE);
        int pf = __shfl_up(flag, d, WAVE);
        if (lane >= d && !flag) {
            val = pv + val;
            flag = pf;
        }
    }
    if (valid) part[i] = val;
    uint64_t anyhead = __ballot(head);
    int64_t w = i / WAVE;
    if (lane == WAVE - 1 && (w * WAVE < n)) {
        carry[w] = val;
        wave_head[w] = anyhead != 0ull;
    }
}

__global__ void rbk_scan2(const uint64_t* __restrict__ k, const double* __restrict__ part,
                          const double* __restrict__ carry, const int* __restrict__ wave_head, int64_t n,
                          int64_t* flag, double* sums) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t key = k[i];
    bool last = (i == n - 1) || k[i + 1] != key;
    int64_t keep = 0;
    if (last) {
        double s = part[i];
        // start of this run inside the wave?  (some element of the wave at or
        // before i is the start of this run)
        int64_t w = i / WAVE;
        int64_t wstart = w * WAVE;
        bool started_here = false;
        // the run started in this wave iff the wave's first element is not part
        // of it or is its start
        if (wstart == 0 || k[wstart] != key || k[wstart - 1] != key) started_here = true;
        if (!started_here) {
            for (int64_t ww = w - 1; ww >= 0; --ww) {
                s += carry[ww];
                if (wave_head[ww]) break;
            }
        }
        sums[i] = s;
        keep = (s != 0.0) ? 1 : 0;
    }
    flag[i] = keep;
}

__global__ void rbk_write(const uint64_t* __restrict__ k, const double* __restrict__ sums,
                          const int64_t* __restrict__ pos, int64_t n, int cbits, int* col,
                          double* val, int* rowkey) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool keep = (i + 1 < n) ? (pos[i + 1] != pos[i]) : false;
    // the last element: decided by the caller passing the total; handled in rbk_write_last
    if (!keep) return;
    int64_t o = pos[i];
    uint64_t kk = k[i];
    col[o] = (int)(kk & ((1ull << cbits) - 1));
    rowkey[o] = (int)(kk >> cbits);
    val[o] = sums[i];
}

__global__ void rbk_write_last(const uint64_t* __restrict__ k, const double* __restrict__ sums,
                               const int64_t* __restrict__ pos, int64_t n, int64_t total, int cbits,
                               int* col, double* val, int* rowkey) {
    int64_t i = n - 1;
    if (pos[i] != total) {
        int64_t o = pos[i];
        uint64_t kk = k[i];
        col[o] = (int)(kk & ((1ull << cbits) - 1));
        rowkey[o] = (int)(kk >> cbits);
        val[o] = sums[i];
    }
}

// rowptr from the sorted row of every output entry
__global__ void rows_to_ptr(const int* __restrict__ rowkey, int64_t nnz, int nrows, int* rowptr) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e > nnz) return;
    int r = e < nnz ? rowkey[e] : nrows;
    int rp = e == 0 ? -1 : rowkey[e - 1];
    for (int rr = rp + 1; rr <= r; ++rr) rowptr[rr] = (int)e;
}

__global__ void fill_ptr_empty(int* rowptr, int nrows) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= nrows) rowptr[i] = 0;
}

int64_t reduce_to_csr(hipStream_t st, const uint64_t* k, const double* v, int64_t n, int cbits,
                      int nrows, int64_t* flag, double* sums, int* rowkey, int64_t* tmp, Arena& out,
                      Csr& csr, const char* what) {
    int64_t total = 0;
    if (n > 0) {
        // per-wave carries and flags in the scan scratch (free until the scan)
        int64_t nwv = (n + WAVE - 1) / WAVE;
        double* carry = (double*)(tmp);
        int* whead = (int*)(tmp + nwv);
        rbk_scan1<<<ceil_div(n, 256), 256, 0, st>>>(k, v, n, sums, carry, whead);
        DP_LAUNCH_CHECK();
        // pass 2 writes sums only at run ends, reading part (= sums) at i: in place
        rbk_scan2<<<ceil_div(n, 256), 256, 0, st>>>(k, sums, carry, whead, n, flag, sums);
        DP_LAUNCH_CHECK();
        exclusive_scan(st, flag, n, tmp, &total);
    }
    csr.nnz = total;
    csr.n = nrows;
    csr.rowptr = out.get<int>(nrows + 1, what);
    csr.col = out.get<int>(total, what);
    csr.val = out.get<double>(total, what);
    if (total > 0) {
        rbk_write<<<ceil_div(n, 256), 256, 0, st>>>(k, sums, flag, n, cbits, csr.col, csr.val, rowkey);
        DP_LAUNCH_CHECK();
        rbk_write_last<<<1, 1, 0, st>>>(k, sums, flag, n, total, cbits, csr.col, csr.val, rowkey);
        DP_LAUNCH_CHECK();
        rows_to_ptr<<<ceil_div(total + 1, 256), 256, 0, st>>>(rowkey, total, nrows, csr.rowptr);
        DP_LAUNCH_CHECK();
    } else {
        fill_ptr_empty<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(csr.rowptr, nrows);
        DP_LAUNCH_CHECK();
    }
    return total;
}

}  // namespace dp
