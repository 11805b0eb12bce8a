// Deterministic device primitives: int64 exclusive scan, stable radix sort of
// (uint64 key, double) pairs, reduce-by-key into CSR.
#pragma once

#include "sim.h"

namespace dp {

// The calling thread's pinned host buffer of PINNED_SLOTS int64 (slot 0: scan
// totals; slots 1..7 free for other small read-backs before a synchronisation).
constexpr int PINNED_SLOTS = 8;
int64_t* pinned_slots();

int64_t scan_tmp_size(int64_t n);
// In-place exclusive scan; returns the total (synchronises the stream).
int64_t exclusive_scan(hipStream_t st, int64_t* data, int64_t n, int64_t* tmp, int64_t* host_total);

// In-place exclusive scan without a host synchronisation (tmp: scan_tmp_size(n)).
void scan_inplace(hipStream_t st, int64_t* data, int64_t n, int64_t* tmp);

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

// Segmented sort-and-reduce into CSR: row r's terms (col[e], val[e]) for e in
// [off[r], off[r+1]) (off: nrows + 1 entries, m = off[nrows]) are ordered by
// column, ties in term order; equal columns are summed in term order and zero
// sums dropped.  col/val are overwritten.  The CSR arrays come from 'out',
// temporaries from 'sc' (released unless out is sc).  Rows with more terms
// than one workgroup sorts in LDS (4096) are sorted together by the global
// radix sort, to the same result; *long_products (if given) counts the calls
// that had such rows.  Returns false, with nothing allocated from 'out', only
// when the scratch cannot hold those rows' terms; the caller then takes the
// global sort path for the whole call.
bool seg_sort_reduce(hipStream_t st, const int64_t* off, int nrows, int ncols, int* col, double* val,
                     int64_t m, Arena& sc, Arena& out, Csr& csr, const char* what,
                     int64_t* long_products = nullptr);

// C = X Y row by row (terms of row r: X_re Y_ef for the entries e of X's row r
// and f of Y's row e, summed per column in that order, zero sums dropped).  C
// comes from 'out', temporaries from 'sc'.  Rows longer than the LDS tiles
// and the return value as for seg_sort_reduce.
// kt (may be null): live timer of the product's tile kernels.
bool seg_product(hipStream_t st, const Csr& X, const Csr& Y, Arena& sc, Arena& out, Csr& C, const char* what,
                 KernelTimer* kt = nullptr, int64_t* long_products = nullptr);

inline int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

}  // namespace dp
