// Vector kernels of the L-BFGS solve (float64 state on the device).
//
//   k_multidot  several dot products (and one max |.|) in one pass, block
//               partials; k_multidot_final sums them in a fixed order
//   k_lincomb   out = sum_q c_q v_q (search direction from the compact
//               representation of the L-BFGS matrix)
//   k_trial     x_t = x + alpha p, also as float32 for the evaluation
//   k_accept    s = x_t - x, y = g_t - g, then x = x_t, g = g_t
#include <hip/hip_runtime.h>

#include <algorithm>

#include "octmc_internal.h"

namespace octmc {
namespace {

constexpr int kB = 256;
constexpr int kMaxBlocks = 512;

// sum (or max for the last row when `maxrow`) of a double over the 64 lanes
// of a wave, in a fixed butterfly order
__device__ __forceinline__ double wave_reduce(double v, bool maxrow)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off);
        v = maxrow ? fmax(v, o) : v + o;
    }
    return v;
}

__global__ __launch_bounds__(kB) void k_multidot(const DotSpec spec, size_t n, double* __restrict__ blk)
{
    const int nd = spec.ndots;
    double acc[kMaxDots];
#pragma unroll
    for (int q = 0; q < kMaxDots; ++q) acc[q] = 0.0;
    double gmax = 0.0;
    for (size_t t = (size_t)blockIdx.x * kB + threadIdx.x; t < n; t += (size_t)gridDim.x * kB) {
#pragma unroll
        for (int q = 0; q < kMaxDots; ++q)
            if (q < nd) acc[q] += spec.v[spec.a[q]][t] * spec.v[spec.b[q]][t];
        if (spec.gmax_vec >= 0) gmax = fmax(gmax, fabs(spec.v[spec.gmax_vec][t]));
    }
    // rows reduced within each wave (butterfly), then the waves in order
    __shared__ double sh[kB / 64][kMaxDots + 1];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < kMaxDots; ++q) {
        if (q < nd) {  // uniform
            const double v = wave_reduce(acc[q], false);
            if (lane == 0) sh[wv][q] = v;
        }
    }
    {
        const double v = wave_reduce(gmax, true);
        if (lane == 0) sh[wv][nd] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q <= nd; q += kB) {
        double s = sh[0][q];
        for (int w = 1; w < kB / 64; ++w) s = (q == nd) ? fmax(s, sh[w][q]) : s + sh[w][q];
        blk[(size_t)blockIdx.x * (kMaxDots + 1) + q] = s;
    }
}

// Products that all share one of two key vectors (every product an L-BFGS
// iteration needs has the gradient or the newest gradient difference as a
// factor): each distinct vector is read once per element instead of once per
// product it appears in.  Partial row v (< nv) is x_v . x_key0, row
// kMaxDotVecs + v is x_v . x_key1, row 2 kMaxDotVecs the max |x_key0|.  Each
// product is formed and accumulated exactly as k_multidot forms it.
struct KeyedDots {
    const double* v[kMaxDotVecs];
    int nv, key0, key1;  // key1 < 0: one key
    int gmax;            // reduce max |x_key0| too
};
constexpr int kKeyedRows = 2 * kMaxDotVecs + 1;
static_assert(kKeyedRows <= kMaxDots + 1, "keyed rows must fit the partial buffer");

__global__ __launch_bounds__(kB) void k_multidot_keyed(const KeyedDots spec, size_t n, double* __restrict__ blk)
{
    const int nv = spec.nv;
    const bool two = spec.key1 >= 0;
    double acc0[kMaxDotVecs], acc1[kMaxDotVecs];
#pragma unroll
    for (int v = 0; v < kMaxDotVecs; ++v) acc0[v] = acc1[v] = 0.0;
    double gmax = 0.0;
    for (size_t t = (size_t)blockIdx.x * kB + threadIdx.x; t < n; t += (size_t)gridDim.x * kB) {
        double x[kMaxDotVecs];
#pragma unroll
        for (int v = 0; v < kMaxDotVecs; ++v) x[v] = v < nv ? spec.v[v][t] : 0.0;
        double k0 = 0.0, k1 = 0.0;
#pragma unroll
        for (int v = 0; v < kMaxDotVecs; ++v) {
            k0 = v == spec.key0 ? x[v] : k0;
            k1 = v == spec.key1 ? x[v] : k1;
        }
#pragma unroll
        for (int v = 0; v < kMaxDotVecs; ++v) {
            if (v < nv) {  // uniform
                acc0[v] += x[v] * k0;
                if (two) acc1[v] += x[v] * k1;
            }
        }
        if (spec.gmax) gmax = fmax(gmax, fabs(k0));
    }
    __shared__ double sh[kB / 64][kKeyedRows];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < kMaxDotVecs; ++v) {
        if (v < nv) {  // uniform
            const double r0 = wave_reduce(acc0[v], false);
            if (lane == 0) sh[wv][v] = r0;
            if (two) {
                const double r1 = wave_reduce(acc1[v], false);
                if (lane == 0) sh[wv][kMaxDotVecs + v] = r1;
            }
        }
    }
    {
        const double r = wave_reduce(gmax, true);
        if (lane == 0) sh[wv][2 * kMaxDotVecs] = r;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kKeyedRows; q += kB) {
        const bool used = q == 2 * kMaxDotVecs || (q < kMaxDotVecs ? q < nv : (two && q - kMaxDotVecs < nv));
        if (!used) continue;
        const bool mx = q == 2 * kMaxDotVecs;
        double s2 = sh[0][q];
        for (int w = 1; w < kB / 64; ++w) s2 = mx ? fmax(s2, sh[w][q]) : s2 + sh[w][q];
        blk[(size_t)blockIdx.x * (kMaxDots + 1) + q] = s2;
    }
}

// fixed-order final sum: output q sums partial row map.row[q]; the outputs
// are dealt round robin to the waves; a lane sums a contiguous run of
// blocks in order, the wave then reduces its lanes in a fixed butterfly order
struct RowMap {
    unsigned char row[kMaxDots + 1];
};
constexpr int kFinalThreads = 1024;

__global__ __launch_bounds__(kFinalThreads) void k_multidot_final(int nrow, int gmax_row, int nblk, const RowMap map,
                                                                  const double* __restrict__ blk,
                                                                  double* __restrict__ out)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int per = (nblk + 63) / 64;
    for (int q = wv; q < nrow; q += kFinalThreads / 64) {
        const bool mx = q == gmax_row;
        const int r = map.row[q];
        double s = 0.0;
        for (int e = 0; e < per; ++e) {
            const int b = lane * per + e;
            if (b < nblk) {
                const double v = blk[(size_t)b * (kMaxDots + 1) + r];
                s = mx ? fmax(s, v) : s + v;
            }
        }
        s = wave_reduce(s, mx);
        if (lane == 0) out[q] = s;
    }
}

__global__ void k_lincomb(const CombSpec spec, size_t n, double* __restrict__ out)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < spec.nv; ++q) s += spec.c[q] * spec.v[q][t];
        out[t] = s;
    }
}

__global__ void k_trial(const double* __restrict__ x, const double* __restrict__ p, double alpha, size_t n,
                        double* __restrict__ xt, float* __restrict__ xt32)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double v = x[t] + alpha * p[t];
        xt[t] = v;
        xt32[t] = (float)v;
    }
}

__global__ void k_accept(double* __restrict__ x, double* __restrict__ g, const double* __restrict__ xt,
                         const double* __restrict__ gt, double* __restrict__ s_out, double* __restrict__ y_out,
                         size_t n)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double xn = xt[t], gn = gt[t];
        s_out[t] = xn - x[t];
        y_out[t] = gn - g[t];
        x[t] = xn;
        g[t] = gn;
    }
}

__global__ void k_to_f64(const float* __restrict__ in, double* __restrict__ out, size_t n)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        out[t] = (double)in[t];
}

__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, size_t n)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        out[t] = (float)in[t];
}

__global__ void k_fill_u32(unsigned* p, unsigned v, size_t n)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        p[t] = v;
}

inline int grid_for(size_t n, int cap = 4096)
{
    size_t g = (n + 255) / 256;
    if (g > (size_t)cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

}  // namespace

hipError_t launch_multidot(const DotSpec& spec, size_t n, double* blk, double* out, hipStream_t s)
{
    const int nd = spec.ndots;
    if (nd > kMaxDots) return hipErrorInvalidValue;
    const int nb = grid_for(n, kMaxBlocks);
    // the keyed form when every product has the max vector or one other
    // vector as a factor
    KeyedDots kd{};
    RowMap map{};
    int nv = 0;
    for (int q = 0; q < nd; ++q) nv = std::max(nv, std::max((int)spec.a[q], (int)spec.b[q]) + 1);
    bool keyed = spec.gmax_vec >= 0 && nv <= kMaxDotVecs;
    kd.nv = std::max(nv, spec.gmax_vec + 1);
    kd.key0 = spec.gmax_vec;
    kd.key1 = -1;
    kd.gmax = 1;
    for (int q = 0; q < nd && keyed; ++q) {
        const int a = spec.a[q], b = spec.b[q];
        int which, other;
        if (b == kd.key0) which = 0, other = a;
        else if (a == kd.key0) which = 0, other = b;
        else {
            if (kd.key1 < 0) kd.key1 = b;
            if (b == kd.key1) which = 1, other = a;
            else if (a == kd.key1) which = 1, other = b;
            else {
                keyed = false;
                break;
            }
        }
        map.row[q] = (unsigned char)(which * kMaxDotVecs + other);
    }
    if (keyed) {
        for (int v = 0; v < kd.nv; ++v) kd.v[v] = spec.v[v];
        map.row[nd] = (unsigned char)(2 * kMaxDotVecs);
        hipLaunchKernelGGL(k_multidot_keyed, dim3(nb), dim3(kB), 0, s, kd, n, blk);
    } else {
        for (int q = 0; q <= nd; ++q) map.row[q] = (unsigned char)q;
        hipLaunchKernelGGL(k_multidot, dim3(nb), dim3(kB), 0, s, spec, n, blk);
    }
    hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(kFinalThreads), 0, s, nd + 1, nd, nb, map, blk, out);
    return hipGetLastError();
}
hipError_t launch_lincomb(const CombSpec& spec, size_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(256), 0, s, spec, n, out);
    return hipGetLastError();
}
hipError_t launch_trial(const double* x, const double* p, double alpha, size_t n, double* xt, float* xt32,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_trial, dim3(grid_for(n)), dim3(256), 0, s, x, p, alpha, n, xt, xt32);
    return hipGetLastError();
}
hipError_t launch_accept(double* x, double* g, const double* xt, const double* gt, double* s_out, double* y_out,
                         size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_accept, dim3(grid_for(n)), dim3(256), 0, s, x, g, xt, gt, s_out, y_out, n);
    return hipGetLastError();
}
hipError_t launch_to_f64(const float* in, double* out, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f64, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t launch_to_f32(const double* in, float* out, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace octmc
