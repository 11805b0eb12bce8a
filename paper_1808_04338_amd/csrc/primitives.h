// Deterministic device primitives: int64 exclusive scan, stable radix sort of
// (uint64 key, double) pairs, reduce-by-key into CSR.
#pragma once

#include "sim.h"

namespace dp {

int64_t scan_tmp_size(int64_t n);
// In-place exclusive scan; returns the total (synchronises the stream).
int64_t exclusive_scan(hipStream_t st, int64_t* data, int64_t n, int64_t* tmp, int64_t* host_total);

int64_t sort_tmp_size(int64_t n);
// Sort by the low 'bits' bits; returns 0 if the result is in (k0,v0), 1 if in (k1,v1).
int radix_sort(hipStream_t st, uint64_t* k0, double* v0, uint64_t* k1, double* v1, int64_t n,
               int bits, int64_t* tmp);

// Sorted keys (row << cbits | col) and values -> CSR with nrows rows; equal keys
// summed (fixed tree order), zero sums dropped.  flag/sums/rowkey: scratch of n
// entries; tmp: scan scratch of at least max(scan_tmp_size(n), 2 ceil(n/64))
// entries.  The CSR arrays come from 'out'.
int64_t reduce_to_csr(hipStream_t st, const uint64_t* k, const double* v, int64_t n, int cbits,
                      int nrows, int64_t* flag, double* sums, int* rowkey, int64_t* tmp, Arena& out,
                      Csr& csr, const char* what);

inline int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

}  // namespace dp
