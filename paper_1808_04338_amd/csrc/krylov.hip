// Vector kernels of the GMRES iteration: classical Gram-Schmidt passes fused
// with their dot products, norms, the solution update, and precision casts.
//
// Reductions are deterministic: every block writes its partial sums in a fixed
// order, and a one-block kernel adds them in block order (the kernel boundary
// orders the partials; no fences or counters across the chip).
#include "kernels.h"

namespace dp {

constexpr int KMAX = 32;  // restart <= 30: at most 31 basis vectors
constexpr int RBLK = 256;
constexpr int MAX_RED_BLOCKS = 2048;

struct Coef {
    double c[KMAX];
};

__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    __syncthreads();
    if (threadIdx.x % WAVE == 0) sh[threadIdx.x / WAVE] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < RBLK / WAVE; ++i) s += sh[i];
    return s;
}

// OP 0: out_k = V_k . w                           (k < nv)
// OP 1: u = w - sum_k h_k V_k; out_k = V_k . u (k < nv), out_nv = u . u;
//       u is written to wout (one read of every V_k)
// OP 3: out_0 = w . w
// OP 4: V_nv = (V_nv - sum_k h_k V_k) * sc, written in place; out_k = V_k . w
//       for k <= nv, the last with the new V_nv (one read of every V_k)
// NV bounds nv at compile time so that the per-thread accumulators of a short
// basis stay few (occupancy); every thread handles (x, y) pairs (16-byte loads).
// len is even and V, w are 16-byte aligned with an even leading dimension.
template <int OP>
__host__ __device__ constexpr int red_results(int nv) {
    return OP == 3 ? 1 : (OP == 0 ? nv : nv + 1);
}

template <int OP, int NV>
__global__ void __launch_bounds__(RBLK) red_kernel(double* V, int64_t ld, int nv,
                                                   const double* __restrict__ h, double sc, double* w,
                                                   double* wout, int64_t len, double* part) {
    constexpr int NR = NV + 1;
    __shared__ double sh[NR][RBLK / WAVE];
    double acc[NV];
    double extra = 0.0;  // result nv of OP 1 and OP 4, result 0 of OP 3
    double hh[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) hh[k] = (OP == 1 || OP == 4) && k < nv ? h[k] : 0.0;
    const int64_t half = len >> 1;
    const int64_t ld2 = ld >> 1;
    double2* V2 = reinterpret_cast<double2*>(V);
    const double2* w2 = reinterpret_cast<const double2*>(w);
    double2* o2 = reinterpret_cast<double2*>(wout);
    const int64_t stride = (int64_t)gridDim.x * RBLK;
    for (int64_t i = (int64_t)blockIdx.x * RBLK + threadIdx.x; i < half; i += stride) {
        double2 wi = w2[i];
        if (OP == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (k < nv) {
                    double2 v = V2[k * ld2 + i];
                    acc[k] += v.x * wi.x + v.y * wi.y;
                }
        } else if (OP == 1) {
            double2 v[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] = k < nv ? V2[k * ld2 + i] : make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (k < nv) {
                    wi.x -= hh[k] * v[k].x;
                    wi.y -= hh[k] * v[k].y;
                }
            o2[i] = wi;
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (k < nv) acc[k] += v[k].x * wi.x + v[k].y * wi.y;
            extra += wi.x * wi.x + wi.y * wi.y;
        } else if (OP == 4) {
            double2 v[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] = k < nv ? V2[k * ld2 + i] : make_double2(0.0, 0.0);
            double2 p = V2[nv * ld2 + i];
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (k < nv) {
                    p.x -= hh[k] * v[k].x;
                    p.y -= hh[k] * v[k].y;
                }
            p.x *= sc;
            p.y *= sc;
            V2[nv * ld2 + i] = p;
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (k < nv) acc[k] += v[k].x * wi.x + v[k].y * wi.y;
            extra += p.x * wi.x + p.y * wi.y;
        } else {
            extra += wi.x * wi.x + wi.y * wi.y;
        }
    }
    // result k: dot k for k < nv (OP 3: none), then the extra one
    const int nd = OP == 3 ? 0 : nv;
    const int nres = red_results<OP>(nv);
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        if (k < nres) {
            double v = wave_sum(k < nd ? acc[k < NV ? k : NV - 1] : extra);
            if (lane == 0) sh[k][wv] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nres) {
        double b = 0.0;
#pragma unroll
        for (int q = 0; q < RBLK / WAVE; ++q) b += sh[threadIdx.x][q];
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = b;
    }
}

// out[k] = sum over the nblk block partials of result k (stored result-major,
// part[k nblk + b], so a workgroup reads its result's partials contiguously):
// one workgroup per result; thread t adds blocks t, t + RBLK, ... in order,
// then a fixed wavefront butterfly and the wavefronts' sums in order.
__global__ void __launch_bounds__(RBLK) red_final(const double* __restrict__ part, int nblk, double* out) {
    __shared__ double sh[RBLK / WAVE];
    const int k = blockIdx.x;
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RBLK) acc += part[(int64_t)k * nblk + b];
    double v = wave_sum(acc);
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < RBLK / WAVE; ++q) t += sh[q];
        out[k] = t;
    }
}

static int red_grid(int64_t len) {
    int64_t g = (len / 2 + RBLK * 4 - 1) / (RBLK * 4);
    if (g < 1) g = 1;
    if (g > MAX_RED_BLOCKS) g = MAX_RED_BLOCKS;
    return (int)g;
}

template <int OP, int NV>
static void red_go(dp_sim* s, int g, double* V, int64_t ld, int nv, const double* h, double sc, double* w,
                   double* wout, int64_t len, double* out) {
    // one round of workgroups: about as many as the chip holds at once for this
    // register bound (the larger bounds keep fewer wavefronts per SIMD)
    constexpr int g_res = NV >= 32 ? 512 : (NV >= 16 ? 1024 : MAX_RED_BLOCKS);
    if (g > g_res) g = g_res;
    red_kernel<OP, NV><<<g, RBLK, 0, s->stream>>>(V, ld, nv, h, sc, w, wout, len, s->red_part);
    if (red_results<OP>(nv) > 0) red_final<<<red_results<OP>(nv), RBLK, 0, s->stream>>>(s->red_part, g, out);
}

template <int OP>
static void red_launch(dp_sim* s, double* V, int64_t ld, int nv, const double* h, double sc, double* w,
                       double* wout, int64_t len, double* out) {
    if (nv < 0 || red_results<OP>(nv) > KMAX || (OP == 4 && nv + 1 > KMAX)) fail(DP_E_INVALID, "too many Krylov vectors");
    if ((len & 1) || (ld & 1)) fail(DP_E_INVALID, "Krylov vectors must have even length");
    int g = red_grid(len);
    if (g > s->red_blocks) fail(DP_E_INVALID, "reduction buffer too small");
    if constexpr (OP == 3) {
        red_go<OP, 1>(s, g, V, ld, nv, h, sc, w, wout, len, out);
    } else if (nv <= 2) {
        red_go<OP, 2>(s, g, V, ld, nv, h, sc, w, wout, len, out);
    } else if (nv <= 4) {
        red_go<OP, 4>(s, g, V, ld, nv, h, sc, w, wout, len, out);
    } else if (nv <= 8) {
        red_go<OP, 8>(s, g, V, ld, nv, h, sc, w, wout, len, out);
    } else if (nv <= 16) {
        red_go<OP, 16>(s, g, V, ld, nv, h, sc, w, wout, len, out);
    } else {
        red_go<OP, KMAX>(s, g, V, ld, nv, h, sc, w, wout, len, out);
    }
    DP_LAUNCH_CHECK();
}

void dot_multi(dp_sim* s, const double* V, int64_t ld, int k, const double* w, int64_t len, double* out) {
    red_launch<0>(s, const_cast<double*>(V), ld, k, nullptr, 1.0, const_cast<double*>(w), nullptr, len, out);
}
void gs_update_dot_norm(dp_sim* s, const double* V, int64_t ld, int k, const double* h, const double* w,
                        double* u, int64_t len, double* out) {
    red_launch<1>(s, const_cast<double*>(V), ld, k, h, 1.0, const_cast<double*>(w), u, len, out);
}
void gs_finish_dot(dp_sim* s, double* V, int64_t ld, int k, const double* a, double sc, const double* w,
                   int64_t len, double* out) {
    red_launch<4>(s, V, ld, k, a, sc, const_cast<double*>(w), nullptr, len, out);
}
void norm2(dp_sim* s, const double* x, int64_t len, double* out) {
    red_launch<3>(s, nullptr, 0, 1, nullptr, 1.0, const_cast<double*>(x), nullptr, len, out);
}

// x += sum_k y_k Z_k
__global__ void combine_kernel(const double* __restrict__ Z, int64_t ld, int k, Coef y, double* x,
                               int64_t len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    double acc = x[i];
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        if (j < k) acc += y.c[j] * Z[j * ld + i];
    x[i] = acc;
}

void combine(dp_sim* s, const double* Z, int64_t ld, int k, const double* y, double* x, int64_t len) {
    Coef c{};
    for (int j = 0; j < k && j < KMAX; ++j) c.c[j] = y[j];
    combine_kernel<<<ceil_div(len, 256), 256, 0, s->stream>>>(Z, ld, k, c, x, len);
    DP_LAUNCH_CHECK();
}

__global__ void scale_kernel(const double* __restrict__ x, double a, double* y, int64_t len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) y[i] = a * x[i];
}
__global__ void axpy_kernel(double a, const double* __restrict__ x, double* y, int64_t len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) y[i] += a * x[i];
}
__global__ void zero_kernel(double* x, int64_t len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) x[i] = 0.0;
}
// Elementwise casts take two elements per thread (16-byte FP64 and 8-byte FP32
// accesses; the arrays start 256-byte aligned); an odd last element alone.
__global__ void f32_kernel(const double* __restrict__ x, double a, float* y, int64_t len) {
    int64_t e = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (e + 1 < len) {
        double2 v = *reinterpret_cast<const double2*>(x + e);
        *reinterpret_cast<float2*>(y + e) = make_float2((float)(a * v.x), (float)(a * v.y));
    } else if (e < len) {
        y[e] = (float)(a * x[e]);
    }
}
__global__ void f64_kernel(const float* __restrict__ x, double* y, int64_t len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) y[i] = (double)x[i];
}
__global__ void add_f64_kernel(const float* __restrict__ a, const float* __restrict__ b, double* y,
                               int64_t len) {
    int64_t e = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (e + 1 < len) {
        float2 u = *reinterpret_cast<const float2*>(a + e);
        float2 v = *reinterpret_cast<const float2*>(b + e);
        *reinterpret_cast<double2*>(y + e) = make_double2((double)(u.x + v.x), (double)(u.y + v.y));
    } else if (e < len) {
        y[e] = (double)(a[e] + b[e]);
    }
}
template <class T>
__global__ void add3_kernel(const T* __restrict__ a, const T* __restrict__ b, T* y, int64_t len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) y[i] = a[i] + b[i];
}

// plain streaming copy (the reference kernel for the HBM traffic counters)
__global__ void copy_f64_kernel(const double2* __restrict__ x, double2* __restrict__ y, int64_t half) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < half) y[i] = x[i];
}
void copy_f64(dp_sim* s, const double* x, double* y, int64_t len) {
    if (len & 1) fail(DP_E_INVALID, "copy length must be even");
    copy_f64_kernel<<<ceil_div(len / 2, 256), 256, 0, s->stream>>>((const double2*)x, (double2*)y, len / 2);
    DP_LAUNCH_CHECK();
}

template <class T>
__global__ void fill_zero_kernel(T* x, int64_t len) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) x[i] = T(0);
}
template <class T>
void vec_fill_zero(dp_sim* s, T* x, int64_t len) {
    fill_zero_kernel<T><<<ceil_div(len, 256), 256, 0, s->stream>>>(x, len);
    DP_LAUNCH_CHECK();
}
template void vec_fill_zero<float>(dp_sim*, float*, int64_t);
template void vec_fill_zero<double>(dp_sim*, double*, int64_t);

void vec_copy(dp_sim* s, const double* x, double* y, int64_t len) {
    DP_HIP(hipMemcpyAsync(y, x, sizeof(double) * len, hipMemcpyDeviceToDevice, s->stream));
}
void vec_zero(dp_sim* s, double* x, int64_t len) {
    zero_kernel<<<ceil_div(len, 256), 256, 0, s->stream>>>(x, len);
    DP_LAUNCH_CHECK();
}
void vec_scale_to(dp_sim* s, const double* x, double alpha, double* y, int64_t len) {
    scale_kernel<<<ceil_div(len, 256), 256, 0, s->stream>>>(x, alpha, y, len);
    DP_LAUNCH_CHECK();
}
void vec_axpy(dp_sim* s, double alpha, const double* x, double* y, int64_t len) {
    axpy_kernel<<<ceil_div(len, 256), 256, 0, s->stream>>>(alpha, x, y, len);
    DP_LAUNCH_CHECK();
}
void to_f32(dp_sim* s, const double* x, float* y, int64_t len, double a) {
    f32_kernel<<<ceil_div((len + 1) / 2, 256), 256, 0, s->stream>>>(x, a, y, len);
    DP_LAUNCH_CHECK();
}
void to_f64(dp_sim* s, const float* x, double* y, int64_t len) {
    f64_kernel<<<ceil_div(len, 256), 256, 0, s->stream>>>(x, y, len);
    DP_LAUNCH_CHECK();
}
void add_to_f64(dp_sim* s, const float* a, const float* b, double* y, int64_t len) {
    add_f64_kernel<<<ceil_div((len + 1) / 2, 256), 256, 0, s->stream>>>(a, b, y, len);
    DP_LAUNCH_CHECK();
}
template <class T>
void vec_add3(dp_sim* s, const T* a, const T* b, T* y, int64_t len) {
    add3_kernel<T><<<ceil_div(len, 256), 256, 0, s->stream>>>(a, b, y, len);
    DP_LAUNCH_CHECK();
}
template void vec_add3<double>(dp_sim*, const double*, const double*, double*, int64_t);
template void vec_add3<float>(dp_sim*, const float*, const float*, float*, int64_t);

}  // namespace dp
