// Ingest and pyramid kernels (run once per pair) and the level transition.
//
//   k_to_storage  float32 -> storage type (round to nearest even)
//   k_pyr3/2/1    factor-2 pyramid (Sec. 2.1): coarse sample I is the mean of
//                 fine samples 2I and min(2I + 1, n - 1) along every axis
//   k_enface_mean depth mean of an OCTA volume (stand-in for the projection of
//                 Sec. 2.3)
//   k_copy_bscans nearest-valid replacement of invalid OCTA B-scans (Sec. 2.5)
//   k_upsample    level transition: twice the bilinear interpolation of the
//                 coarse field at ((i - 1/2) / 2, (j - 1/2) / 2)
#include <hip/hip_runtime.h>

#include "octmc_internal.h"

namespace octmc {
namespace {

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__global__ void k_to_storage(const float* __restrict__ in, void* __restrict__ out, size_t n, int dt)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const float v = in[q];
        if (dt == OCTMC_F32) {
            static_cast<float*>(out)[q] = v;
        } else if (dt == OCTMC_BF16) {
            static_cast<unsigned short*>(out)[q] = f32_to_bf16_rne(v);
        } else {
            static_cast<unsigned short*>(out)[q] = __builtin_bit_cast(unsigned short, (_Float16)v);
        }
    }
}

// The same into A-scan columns of dp >= d samples: samples d .. dp - 1 of a
// column repeat sample d - 1 (one thread per stored sample).
__global__ void k_to_storage_pad(const float* __restrict__ in, void* __restrict__ out, int na, int d, int dp, int dt)
{
    const size_t n = (size_t)na * dp;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const size_t a = q / dp;
        const int k = (int)(q - a * dp);
        const float v = in[a * d + (k < d ? k : d - 1)];
        if (dt == OCTMC_BF16) static_cast<unsigned short*>(out)[q] = f32_to_bf16_rne(v);
        else static_cast<unsigned short*>(out)[q] = __builtin_bit_cast(unsigned short, (_Float16)v);
    }
}

// one thread per coarse sample; depth fastest for coalescing
__global__ void k_pyr3(const float* __restrict__ in, int w, int h, int d, float* __restrict__ out)
{
    const int w2 = (w + 1) / 2, h2 = (h + 1) / 2, d2 = (d + 1) / 2;
    const size_t total = (size_t)w2 * h2 * d2;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
        const int K = (int)(q % d2);
        const size_t c = q / d2;
        const int I = (int)(c % w2), J = (int)(c / w2);
        const int y0 = 2 * J, y1 = min(2 * J + 1, h - 1);
        const int x0 = 2 * I, x1 = min(2 * I + 1, w - 1);
        const int z0 = 2 * K, z1 = min(2 * K + 1, d - 1);
        const float* r00 = in + ((size_t)y0 * w + x0) * d;
        const float* r01 = in + ((size_t)y0 * w + x1) * d;
        const float* r10 = in + ((size_t)y1 * w + x0) * d;
        const float* r11 = in + ((size_t)y1 * w + x1) * d;
        const float s = ((r00[z0] + r00[z1]) + (r01[z0] + r01[z1])) + ((r10[z0] + r10[z1]) + (r11[z0] + r11[z1]));
        out[q] = 0.125f * s;
    }
}

__global__ void k_pyr2(const float* __restrict__ in, int w, int h, float* __restrict__ out)
{
    const int w2 = (w + 1) / 2, h2 = (h + 1) / 2;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < w2 * h2; q += gridDim.x * blockDim.x) {
        const int I = q % w2, J = q / w2;
        const int y1 = min(2 * J + 1, h - 1), x1 = min(2 * I + 1, w - 1);
        out[q] = 0.25f * ((in[(size_t)2 * J * w + 2 * I] + in[(size_t)2 * J * w + x1]) +
                          (in[(size_t)y1 * w + 2 * I] + in[(size_t)y1 * w + x1]));
    }
}

__global__ void k_pyr1(const float* __restrict__ in, int n, float* __restrict__ out)
{
    const int n2 = (n + 1) / 2;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n2; q += gridDim.x * blockDim.x)
        out[q] = 0.5f * (in[2 * q] + in[min(2 * q + 1, n - 1)]);
}

// one wavefront per A-scan
__global__ void k_enface_mean(const float* __restrict__ vol, int na, int d, float* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int a = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (a >= na) return;
    const float* col = vol + (size_t)a * d;
    double s = 0.0;
    for (int k = lane; k < d; k += 64) s += col[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[a] = (float)(s / d);
}

__global__ void k_count_nonfinite(const float* __restrict__ v, size_t n, unsigned* counter)
{
    unsigned bad = 0;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        bad += !isfinite(v[q]);
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(counter, bad);
}

// src[b] = the B-scan whose data B-scan b takes (b itself when valid)
__global__ void k_copy_bscans(float* __restrict__ vol, int w, int h, int d, const int* __restrict__ src, int V)
{
    const size_t total = (size_t)w * h * d;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(q % d);
        const size_t a = q / d;
        const int i = (int)(a % w), j = (int)(a / w);
        const int b = (V == 0) ? j : i;
        const int sb = src[b];
        if (sb == b) continue;
        const size_t from = (V == 0) ? ((size_t)sb * w + i) : ((size_t)j * w + sb);
        vol[q] = vol[from * d + k];
    }
}

__global__ void k_upsample(const double* __restrict__ C, int wc, int hc, double* __restrict__ Fo, int wf, int hf,
                           int nvol)
{
    const int total = nvol * wf * hf;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        const int V = q / (wf * hf);
        const int r = q % (wf * hf);
        const int i = r % wf, j = r / wf;
        double x = (i - 0.5) * 0.5, y = (j - 0.5) * 0.5;
        x = fmin(fmax(x, 0.0), (double)(wc - 1));
        y = fmin(fmax(y, 0.0), (double)(hc - 1));
        const int x0 = (int)floor(x), y0 = (int)floor(y);
        const int x1 = min(x0 + 1, wc - 1), y1 = min(y0 + 1, hc - 1);
        const double fx = x - x0, fy = y - y0;
        const double* CV = C + (size_t)V * wc * hc * 3;
        for (int c = 0; c < 3; ++c) {
            const double v00 = CV[((size_t)y0 * wc + x0) * 3 + c], v10 = CV[((size_t)y0 * wc + x1) * 3 + c];
            const double v01 = CV[((size_t)y1 * wc + x0) * 3 + c], v11 = CV[((size_t)y1 * wc + x1) * 3 + c];
            const double v = (1 - fy) * ((1 - fx) * v00 + fx * v10) + fy * ((1 - fx) * v01 + fx * v11);
            Fo[(size_t)q * 3 + c] = 2.0 * v;
        }
    }
}

inline int grid_for(size_t n, int block = 256, int cap = 65536)
{
    size_t g = (n + block - 1) / block;
    if (g > (size_t)cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

// Input validity of an OCTA volume (Sec. 2.2).  Step 1: mean decorrelation
// of every B-scan (one block per B-scan, float64, fixed-order sum): rows j
// of the X-fast scan (V = 0), columns i of the Y-fast scan (V = 1).
constexpr int kVB = 256;

__device__ __forceinline__ double block_sum_d(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kVB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kVB) void k_bscan_mean(const float* __restrict__ vol, int w, int h, int d, int V,
                                                    double* __restrict__ m)
{
    __shared__ double sh[kVB];
    const int b = blockIdx.x;
    const int na = V == 0 ? w : h;
    double s = 0.0;
    if (V == 0) {  // one contiguous run of w * d samples
        const float* p = vol + (size_t)b * w * d;
        const size_t n = (size_t)w * d;
        for (size_t q = threadIdx.x; q < n; q += kVB) s += (double)p[q];
    } else {  // h A-scans of d samples, w * d apart
        for (int o = 0; o < h; ++o) {
            const float* p = vol + ((size_t)o * w + b) * d;
            for (int k = threadIdx.x; k < d; k += kVB) s += (double)p[k];
        }
    }
    s = block_sum_d(s, sh);
    if (threadIdx.x == 0) m[b] = s / ((double)na * (double)d);
}

// Step 2 (one block): mean mu and population standard deviation sigma of the
// B-scan means; B-scan b is flagged if m_b > mu + 3 sigma, and valid (1) if
// none of b - 2 .. b + 2 is flagged.
__global__ __launch_bounds__(kVB) void k_validity(const double* __restrict__ m, int nb, float* __restrict__ v)
{
    __shared__ double sh[kVB];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kVB) s += m[b];
    const double mu = block_sum_d(s, sh) / nb;
    double q = 0.0;
    for (int b = threadIdx.x; b < nb; b += kVB) q += (m[b] - mu) * (m[b] - mu);
    const double thr = mu + 3.0 * sqrt(block_sum_d(q, sh) / nb);
    for (int b = threadIdx.x; b < nb; b += kVB) {
        bool bad = false;
        for (int o = b - 2; o <= b + 2; ++o)
            if (o >= 0 && o < nb && m[o] > thr) bad = true;
        v[b] = bad ? 0.f : 1.f;
    }
}

}  // namespace

hipError_t launch_validity(const float* vol, int w, int h, int d, int V, double* means, float* valid,
                           hipStream_t s)
{
    const int nb = V == 0 ? h : w;
    hipLaunchKernelGGL(k_bscan_mean, dim3(nb), dim3(kVB), 0, s, vol, w, h, d, V, means);
    hipLaunchKernelGGL(k_validity, dim3(1), dim3(kVB), 0, s, means, nb, valid);
    return hipGetLastError();
}

hipError_t launch_to_storage(const float* in, void* out, size_t n, octmc_dtype dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_storage, dim3(grid_for(n)), dim3(256), 0, s, in, out, n, (int)dt);
    return hipGetLastError();
}
hipError_t launch_to_storage_pitched(const float* in, void* out, int na, int d, int dp, octmc_dtype dt,
                                     hipStream_t s)
{
    if (dp == d) return launch_to_storage(in, out, (size_t)na * d, dt, s);
    if (dp < d || dt == OCTMC_F32) return hipErrorInvalidValue;  // only 16-bit storage is padded
    const size_t n = (size_t)na * dp;
    hipLaunchKernelGGL(k_to_storage_pad, dim3(grid_for(n)), dim3(256), 0, s, in, out, na, d, dp, (int)dt);
    return hipGetLastError();
}
hipError_t launch_pyr3(const float* in, int w, int h, int d, float* out, hipStream_t s)
{
    const size_t n = (size_t)((w + 1) / 2) * ((h + 1) / 2) * ((d + 1) / 2);
    hipLaunchKernelGGL(k_pyr3, dim3(grid_for(n)), dim3(256), 0, s, in, w, h, d, out);
    return hipGetLastError();
}
hipError_t launch_pyr2(const float* in, int w, int h, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_pyr2, dim3(grid_for((size_t)w * h / 4 + 1)), dim3(256), 0, s, in, w, h, out);
    return hipGetLastError();
}
hipError_t launch_pyr1(const float* in, int n, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_pyr1, dim3(grid_for((size_t)n)), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}
hipError_t launch_enface_mean(const float* vol, int na, int d, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_enface_mean, dim3((na + 3) / 4), dim3(256), 0, s, vol, na, d, out);
    return hipGetLastError();
}
hipError_t launch_count_nonfinite(const float* v, size_t n, unsigned* counter, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(n)), dim3(256), 0, s, v, n, counter);
    return hipGetLastError();
}
hipError_t launch_copy_bscans(float* vol, int w, int h, int d, const int* src, int V, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_bscans, dim3(grid_for((size_t)w * h * d)), dim3(256), 0, s, vol, w, h, d, src, V);
    return hipGetLastError();
}
hipError_t launch_upsample(const double* coarse, int wc, int hc, double* fine, int wf, int hf, hipStream_t s,
                           int nvol)
{
    hipLaunchKernelGGL(k_upsample, dim3(grid_for((size_t)nvol * wf * hf)), dim3(256), 0, s, coarse, wc, hc, fine, wf,
                       hf, nvol);
    return hipGetLastError();
}

}  // namespace octmc
