// Shared definitions of the dpsim HIP library: error handling, the workspace
// arena, 2-vectors and 2x2 block helpers, wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "dpsim.h"

namespace dp {

// ---------------------------------------------------------------------------
// Errors: internal code throws dp::Error; the C ABI converts it to dp_status.
// ---------------------------------------------------------------------------
struct Error : public std::runtime_error {
    dp_status code;
    Error(dp_status c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

[[noreturn]] inline void fail(dp_status c, const std::string& msg) { throw Error(c, msg); }

#define DP_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            ::dp::fail(DP_E_DEVICE, std::string(#call " failed: ") + hipGetErrorString(e_) + \
                                        " (" __FILE__ ":" + std::to_string(__LINE__) + ")"); \
    } while (0)

#define DP_LAUNCH_CHECK() DP_HIP(hipGetLastError())

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Workspace arena: a bump allocator over caller-provided device memory.
// ---------------------------------------------------------------------------
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t top = 0;
    bool counting = false;  // footprint mode: only accumulate sizes

    void* take(size_t bytes, const char* what) {
        size_t off = (top + 255) & ~size_t(255);
        size_t end = off + ((bytes + 255) & ~size_t(255));
        if (!counting && end > cap)
            fail(DP_E_NOMEM, std::string("workspace too small for ") + what + ": need at least " +
                                 std::to_string(end) + " bytes, have " + std::to_string(cap));
        top = end;
        return counting ? nullptr : base + off;
    }
    template <class T>
    T* get(int64_t count, const char* what) {
        return (T*)take(sizeof(T) * (size_t)(count > 0 ? count : 1), what);
    }
};

// ---------------------------------------------------------------------------
// 2-vectors and 2x2 blocks.  A block is stored as two row 2-vectors:
// row0 = (a00, a01), row1 = (a10, a11).
// ---------------------------------------------------------------------------
template <class T>
struct V2 {
    T x, y;
};
template <>
struct __align__(16) V2<double> {
    double x, y;
};
template <>
struct __align__(8) V2<float> {
    float x, y;
};
using d2 = V2<double>;
using f2 = V2<float>;

template <class T>
struct Blk {
    T a00, a01, a10, a11;
};

template <class T>
__host__ __device__ inline V2<T> mk2(T x, T y) {
    V2<T> r;
    r.x = x;
    r.y = y;
    return r;
}

template <class T>
__host__ __device__ inline Blk<T> mkb(V2<T> r0, V2<T> r1) {
    return Blk<T>{r0.x, r0.y, r1.x, r1.y};
}

template <class T>
__host__ __device__ inline V2<T> bmv(const Blk<T>& a, V2<T> v) {
    return mk2<T>(a.a00 * v.x + a.a01 * v.y, a.a10 * v.x + a.a11 * v.y);
}

template <class T>
__host__ __device__ inline Blk<T> bmm(const Blk<T>& a, const Blk<T>& b) {
    return Blk<T>{a.a00 * b.a00 + a.a01 * b.a10, a.a00 * b.a01 + a.a01 * b.a11,
                  a.a10 * b.a00 + a.a11 * b.a10, a.a10 * b.a01 + a.a11 * b.a11};
}

template <class T>
__host__ __device__ inline Blk<T> bsub(const Blk<T>& a, const Blk<T>& b) {
    return Blk<T>{a.a00 - b.a00, a.a01 - b.a01, a.a10 - b.a10, a.a11 - b.a11};
}

template <class T>
__host__ __device__ inline Blk<T> badd(const Blk<T>& a, const Blk<T>& b) {
    return Blk<T>{a.a00 + b.a00, a.a01 + b.a01, a.a10 + b.a10, a.a11 + b.a11};
}

// Inverse of a 2x2 block by the adjugate formula.
template <class T>
__host__ __device__ inline Blk<T> binv(const Blk<T>& a) {
    T det = a.a00 * a.a11 - a.a01 * a.a10;
    T r = T(1) / det;
    return Blk<T>{a.a11 * r, -a.a01 * r, -a.a10 * r, a.a00 * r};
}

template <class T>
__host__ __device__ inline V2<T> vsub(V2<T> a, V2<T> b) {
    return mk2<T>(a.x - b.x, a.y - b.y);
}
template <class T>
__host__ __device__ inline V2<T> vadd(V2<T> a, V2<T> b) {
    return mk2<T>(a.x + b.x, a.y + b.y);
}

// Load/store a block from a pair of row planes.
template <class T>
__device__ inline Blk<T> ldb(const V2<T>* r0, const V2<T>* r1, int64_t i) {
    return mkb(r0[i], r1[i]);
}
template <class T>
__device__ inline void stb(V2<T>* r0, V2<T>* r1, int64_t i, const Blk<T>& b) {
    r0[i] = mk2(b.a00, b.a01);
    r1[i] = mk2(b.a10, b.a11);
}

// ---------------------------------------------------------------------------
// Wavefront (64 lanes) reductions in a fixed butterfly order: deterministic.
// ---------------------------------------------------------------------------
constexpr int WAVE = 64;

// Workgroups go to the eight XCDs round-robin (workgroup b runs on XCD b mod
// 8), and each XCD has its own L2.  xcd_block renumbers the blocks of a grid of
// nblk so that every XCD sweeps one contiguous stretch of the logical blocks:
// rows that gather from nearby rows (a grid layer up or down, a few dozen
// workgroups away) then find them in their own L2.  A bijection on [0, nblk).
__device__ inline int xcd_block(int b, int nblk) {
    constexpr int NXCD = 8;
    int q = nblk / NXCD, r = nblk % NXCD;
    int x = b % NXCD, k = b / NXCD;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

}  // namespace dp
