// Output kernels (Sec. 2.1 "merging", Sec. 2.5): sampling density, merge
// weights and the weighted average of the two resampled scans.
//
//   k_density       every output A-scan splats its (clamped) sample position
//                   bilinearly into a per-scan h x w grid; fixed-point 64-bit
//                   integer atomics keep the sums independent of order
//   k_merge_weights density read back at the sample position -> weight
//                   exp(-kappa max(0, rho - 1)), clipped below tau, normalised;
//                   the OCTA weights are further multiplied by the resampled
//                   validity (Eq. 5); where both vanish, OCT keeps the scan with
//                   the lower density and OCTA is 0
//   k_merge_volume  resample both scans with their fields (Eq. 2 interpolator,
//                   value only) and write the weighted sum
#include <hip/hip_runtime.h>

#include "octmc_internal.h"

namespace octmc {
namespace {

constexpr double kFix = 4294967296.0;  // 2^32

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ void bilin(float x, float y, int w, int h, int& x0, int& y0, int& x1, int& y1, float& fx,
                                      float& fy)
{
    x = fminf(fmaxf(x, 0.f), (float)(w - 1));
    y = fminf(fmaxf(y, 0.f), (float)(h - 1));
    x0 = (int)floorf(x);
    y0 = (int)floorf(y);
    x1 = min(x0 + 1, w - 1);
    y1 = min(y0 + 1, h - 1);
    fx = x - x0;
    fy = y - y0;
}

__global__ void k_density(const float* __restrict__ disp, int w, int h, unsigned long long* __restrict__ grid,
                          int nvol)
{
    const int na = w * h;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nvol * na; q += gridDim.x * blockDim.x) {
        const int V = q / na, a = q % na;
        const int i = a % w, j = a / w;
        int x0, y0, x1, y1;
        float fx, fy;
        bilin(i + disp[(size_t)q * 3], j + disp[(size_t)q * 3 + 1], w, h, x0, y0, x1, y1, fx, fy);
        unsigned long long* G = grid + (size_t)V * na;
        atomicAdd(G + (size_t)y0 * w + x0, (unsigned long long)llrint((1.0 - fx) * (1.0 - fy) * kFix));
        atomicAdd(G + (size_t)y0 * w + x1, (unsigned long long)llrint((double)fx * (1.0 - fy) * kFix));
        atomicAdd(G + (size_t)y1 * w + x0, (unsigned long long)llrint((1.0 - fx) * (double)fy * kFix));
        atomicAdd(G + (size_t)y1 * w + x1, (unsigned long long)llrint((double)fx * (double)fy * kFix));
    }
}

__device__ __forceinline__ void cr_w(float t, float w[4])
{
    const float t2 = t * t, t3 = t2 * t;
    w[0] = 0.5f * (-t3 + 2.f * t2 - t);
    w[1] = 0.5f * (3.f * t3 - 5.f * t2 + 2.f);
    w[2] = 0.5f * (-3.f * t3 + 4.f * t2 + t);
    w[3] = 0.5f * (t3 - t2);
}

__device__ __forceinline__ float valid_at(const float* v, int n, int idx, float dv)
{
    const float f = floorf(dv);
    const int nx = idx + (int)f;
    float w[4];
    cr_w(dv - f, w);
    float s = 0.f;
    for (int a = 0; a < 4; ++a) s = fmaf(w[a], v[clampi(nx - 1 + a, 0, n - 1)], s);
    return fminf(fmaxf(s, 0.f), 1.f);
}

__global__ void k_merge_weights(const float* __restrict__ disp, int w, int h,
                                const unsigned long long* __restrict__ grid, const float* __restrict__ vx,
                                const float* __restrict__ vy, double kappa, double tau, float4* __restrict__ wts)
{
    const int na = w * h;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < na; a += gridDim.x * blockDim.x) {
        const int i = a % w, j = a / w;
        double rho[2];
        for (int V = 0; V < 2; ++V) {
            const float* dv = disp + ((size_t)V * na + a) * 3;
            int x0, y0, x1, y1;
            float fx, fy;
            bilin(i + dv[0], j + dv[1], w, h, x0, y0, x1, y1, fx, fy);
            const unsigned long long* G = grid + (size_t)V * na;
            rho[V] = ((1.0 - fx) * (1.0 - fy) * (double)G[(size_t)y0 * w + x0] +
                      (double)fx * (1.0 - fy) * (double)G[(size_t)y0 * w + x1] +
                      (1.0 - fx) * (double)fy * (double)G[(size_t)y1 * w + x0] +
                      (double)fx * (double)fy * (double)G[(size_t)y1 * w + x1]) / kFix;
        }
        double wx = exp(-kappa * fmax(0.0, rho[0] - 1.0)), wy = exp(-kappa * fmax(0.0, rho[1] - 1.0));
        if (wx < tau) wx = 0.0;
        if (wy < tau) wy = 0.0;
        double ax, ay;
        if (wx + wy > 0) {
            ax = wx / (wx + wy);
            ay = wy / (wx + wy);
        } else if (rho[0] <= rho[1]) {
            ax = 1.0;
            ay = 0.0;
        } else {
            ax = 0.0;
            ay = 1.0;
        }
        double ox = 0.0, oy = 0.0;
        if (vx && vy) {
            ox = wx * valid_at(vx, h, j, disp[(size_t)a * 3 + 1]);
            oy = wy * valid_at(vy, w, i, disp[((size_t)na + a) * 3]);
            const double s = ox + oy;
            if (s > 0) {
                ox /= s;
                oy /= s;
            }
        }
        wts[a] = make_float4((float)ax, (float)ay, (float)ox, (float)oy);
    }
}

template <typename T>
__device__ __forceinline__ float ld(const void* p, size_t q);
template <>
__device__ __forceinline__ float ld<float>(const void* p, size_t q) { return static_cast<const float*>(p)[q]; }
struct bf16_t {};
struct f16_t {};
template <>
__device__ __forceinline__ float ld<bf16_t>(const void* p, size_t q)
{
    return __builtin_bit_cast(float, (uint32_t) static_cast<const unsigned short*>(p)[q] << 16);
}
template <>
__device__ __forceinline__ float ld<f16_t>(const void* p, size_t q)
{
    return (float)__builtin_bit_cast(_Float16, static_cast<const unsigned short*>(p)[q]);
}

// 32-bit buffer loads of one sample (wave-uniform column offset in soff)
template <typename T>
__device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float ldb<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float ldb<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0) << 16);
}
template <>
__device__ __forceinline__ float ldb<f16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
template <typename T> struct bytes_of { static constexpr uint32_t v = 2; };
template <> struct bytes_of<float> { static constexpr uint32_t v = 4; };

// value of the next lane (DPP whole-wave shift; lane 63 reads 0 by bound control)
__device__ __forceinline__ float next_lane(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

// Depth steps of 61 output samples on 64 lanes: lane l holds source sample
// base + 61 n + l (clamped to the A-scan), and output lane l < 61 reads the
// blended values of lanes l .. l + 3.
constexpr int kMergeStep = 61;

// one wavefront per output A-scan, lanes along depth; which = 0 uses the OCT
// weights (wts.x, wts.y), which = 1 the OCTA weights (wts.z, wts.w).  The 16
// lateral columns of each scan are read with 32-bit buffer offsets (their
// offsets and weights wave-uniform), each source sample once per step.
template <typename T>
__global__ __launch_bounds__(256) void k_merge_volume(const void* __restrict__ sx, const void* __restrict__ sy,
                                                      const float* __restrict__ disp, const float4* __restrict__ wts,
                                                      int which, int w, int h, int d, int dp, uint32_t vol_bytes,
                                                      float* __restrict__ out)
{
    // sx, sy: [h][w] columns of dp samples (the first d are the A-scan); out: [h][w][d]
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int na = w * h;
    const int a = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);
    if (a >= na) return;
    const int i = a % w, j = a / w;
    const float4 wt = wts[a];
    const float wgt[2] = {which ? wt.z : wt.x, which ? wt.w : wt.y};
    const void* vol[2] = {sx, sy};
    __amdgpu_buffer_rsrc_t rs[2];
    uint32_t off[2][16];
    float wl[2][16], wz[2][4];
    int base[2];
#pragma unroll
    for (int V = 0; V < 2; ++V) {
        rs[V] = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(vol[V]), (short)0, (int)vol_bytes, 0x00020000);
        const float* dv = disp + ((size_t)V * na + a) * 3;
        const float fxf = floorf(dv[0]), fyf = floorf(dv[1]), fzf = floorf(dv[2]);
        const int nx = i + (int)fxf, ny = j + (int)fyf, nz = (int)fzf;
        float wx[4], wy[4];
        cr_w(dv[0] - fxf, wx);
        cr_w(dv[1] - fyf, wy);
        cr_w(dv[2] - fzf, wz[V]);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                off[V][b * 4 + c] = (uint32_t)__builtin_amdgcn_readfirstlane(
                    (int)((uint32_t)(clampi(ny - 1 + b, 0, h - 1) * w + clampi(nx - 1 + c, 0, w - 1)) * (uint32_t)dp *
                          bytes_of<T>::v));
                wl[V][b * 4 + c] = wx[c] * wy[b];
            }
        base[V] = nz - 1;
    }
    const int nsteps = (d + kMergeStep - 1) / kMergeStep;
    for (int n = 0; n < nsteps; ++n) {
        float res = 0.f;
#pragma unroll
        for (int V = 0; V < 2; ++V) {
            const uint32_t voff = (uint32_t)clampi(base[V] + kMergeStep * n + lane, 0, d - 1) * bytes_of<T>::v;
            float c = 0.f;
#pragma unroll
            for (int q = 0; q < 16; ++q) c = fmaf(wl[V][q], ldb<T>(rs[V], voff, off[V][q]), c);
            const float c1 = next_lane(c), c2 = next_lane(c1), c3 = next_lane(c2);
            float iv = 0.f;
            iv = fmaf(wz[V][0], c, iv);
            iv = fmaf(wz[V][1], c1, iv);
            iv = fmaf(wz[V][2], c2, iv);
            iv = fmaf(wz[V][3], c3, iv);
            res = fmaf(wgt[V], iv, res);
        }
        const int k = kMergeStep * n + lane;
        if (lane < kMergeStep && k < d) out[(size_t)a * d + k] = res;
    }
}

// n-volume merge weights: OCT weights wo[V][a] normalised over the volumes
// (the lowest-density volume where all vanish; the first on a tie) and OCTA
// weights wa[V][a] = OCT weight before normalisation times the resampled
// validity along the volume's slow axis, normalised (0 where all vanish)
__global__ void k_merge_weights_multi(const float* __restrict__ disp, int w, int h,
                                      const unsigned long long* __restrict__ grid, const MultiVols mv, double kappa,
                                      double tau, float* __restrict__ wo, float* __restrict__ wa)
{
    const int na = w * h;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < na; a += gridDim.x * blockDim.x) {
        const int i = a % w, j = a / w;
        double rho[kMaxVol], wt[kMaxVol], ow[kMaxVol];
        double sw = 0.0, so = 0.0;
        int lowest = 0;
        for (int V = 0; V < mv.n; ++V) {
            const float* dv = disp + ((size_t)V * na + a) * 3;
            int x0, y0, x1, y1;
            float fx, fy;
            bilin(i + dv[0], j + dv[1], w, h, x0, y0, x1, y1, fx, fy);
            const unsigned long long* G = grid + (size_t)V * na;
            rho[V] = ((1.0 - fx) * (1.0 - fy) * (double)G[(size_t)y0 * w + x0] +
                      (double)fx * (1.0 - fy) * (double)G[(size_t)y0 * w + x1] +
                      (1.0 - fx) * (double)fy * (double)G[(size_t)y1 * w + x0] +
                      (double)fx * (double)fy * (double)G[(size_t)y1 * w + x1]) / kFix;
            wt[V] = exp(-kappa * fmax(0.0, rho[V] - 1.0));
            if (wt[V] < tau) wt[V] = 0.0;
            sw += wt[V];
            if (rho[V] < rho[lowest]) lowest = V;
            ow[V] = 0.0;
            if (mv.valid[V])
                ow[V] = wt[V] * (mv.orient[V] == 0 ? valid_at(mv.valid[V], h, j, dv[1])
                                                    : valid_at(mv.valid[V], w, i, dv[0]));
            so += ow[V];
        }
        for (int V = 0; V < mv.n; ++V) {
            const double o = sw > 0 ? wt[V] / sw : (V == lowest ? 1.0 : 0.0);
            wo[(size_t)V * na + a] = (float)o;
            wa[(size_t)V * na + a] = (float)(so > 0 ? ow[V] / so : 0.0);
        }
    }
}

// one thread per output sample: the weighted sum over the volumes of the
// Eq. 2 interpolator's value at each volume's sample position
template <typename T>
__global__ __launch_bounds__(256) void k_merge_volume_multi(const MultiVols mv, const float* __restrict__ disp,
                                                            const float* __restrict__ wts, int w, int h, int d,
                                                            int dp, float* __restrict__ out)
{
    const int na = w * h;
    const size_t total = (size_t)na * d;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (size_t)gridDim.x * blockDim.x) {
        const int a = (int)(q / d), k = (int)(q - (size_t)a * d);
        const int i = a % w, j = a / w;
        float res = 0.f;
        for (int V = 0; V < mv.n; ++V) {
            const float wgt = wts[(size_t)V * na + a];
            if (wgt == 0.f) continue;
            const float* dv = disp + ((size_t)V * na + a) * 3;
            const float fxf = floorf(dv[0]), fyf = floorf(dv[1]), fzf = floorf(dv[2]);
            const int nx = i + (int)fxf, ny = j + (int)fyf, nz = k + (int)fzf;
            float wx[4], wy[4], wz[4];
            cr_w(dv[0] - fxf, wx);
            cr_w(dv[1] - fyf, wy);
            cr_w(dv[2] - fzf, wz);
            float v = 0.f;
            for (int b = 0; b < 4; ++b) {
                const size_t row = (size_t)clampi(ny - 1 + b, 0, h - 1) * w;
                for (int c = 0; c < 4; ++c) {
                    const size_t col = (row + clampi(nx - 1 + c, 0, w - 1)) * dp;  // volumes [h][w][dp]
                    float z = 0.f;
                    for (int e = 0; e < 4; ++e) z = fmaf(wz[e], ld<T>(mv.vol[V], col + clampi(nz - 1 + e, 0, d - 1)), z);
                    v = fmaf(wx[c] * wy[b], z, v);
                }
            }
            res = fmaf(wgt, v, res);
        }
        out[q] = res;
    }
}

inline int grid_for(size_t n, int cap = 65536)
{
    size_t g = (n + 255) / 256;
    if (g > (size_t)cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

}  // namespace

hipError_t launch_density(const float* disp, int w, int h, unsigned long long* grid, hipStream_t s, int nvol)
{
    hipLaunchKernelGGL(k_density, dim3(grid_for((size_t)nvol * w * h)), dim3(256), 0, s, disp, w, h, grid, nvol);
    return hipGetLastError();
}
hipError_t launch_merge_weights_multi(const float* disp, int w, int h, const unsigned long long* grid,
                                      const MultiVols& mv, double kappa, double tau, float* wo, float* wa,
                                      hipStream_t s)
{
    hipLaunchKernelGGL(k_merge_weights_multi, dim3(grid_for((size_t)w * h)), dim3(256), 0, s, disp, w, h, grid, mv,
                       kappa, tau, wo, wa);
    return hipGetLastError();
}
hipError_t launch_merge_volume_multi(const MultiVols& mv, octmc_dtype dt, const float* disp, const float* wts, int w,
                                     int h, int d, int dp, float* out, hipStream_t s)
{
    const size_t n = (size_t)w * h * d;
    switch (dt) {
    case OCTMC_F32:
        hipLaunchKernelGGL(k_merge_volume_multi<float>, dim3(grid_for(n)), dim3(256), 0, s, mv, disp, wts, w, h, d,
                           dp, out);
        break;
    case OCTMC_BF16:
        hipLaunchKernelGGL(k_merge_volume_multi<bf16_t>, dim3(grid_for(n)), dim3(256), 0, s, mv, disp, wts, w, h, d,
                           dp, out);
        break;
    case OCTMC_F16:
        hipLaunchKernelGGL(k_merge_volume_multi<f16_t>, dim3(grid_for(n)), dim3(256), 0, s, mv, disp, wts, w, h, d,
                           dp, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
hipError_t launch_merge_weights(const float* disp, int w, int h, const unsigned long long* grid, const float* vx,
                                const float* vy, double kappa, double tau, float4* wts, hipStream_t s)
{
    hipLaunchKernelGGL(k_merge_weights, dim3(grid_for((size_t)w * h)), dim3(256), 0, s, disp, w, h, grid, vx, vy,
                       kappa, tau, wts);
    return hipGetLastError();
}
hipError_t launch_merge_volume(const void* vx_, const void* vy_, octmc_dtype dt, const float* disp,
                               const float4* wts, int which, int w, int h, int d, int dp, float* out, hipStream_t s)
{
    const int blocks = (w * h + 3) / 4;
    const size_t bytes = (size_t)w * h * dp * (dt == OCTMC_F32 ? 4 : 2);
    if (bytes >= (1ull << 31)) return hipErrorInvalidValue;  // 32-bit buffer offsets
    const uint32_t vb = (uint32_t)bytes;
    switch (dt) {
    case OCTMC_F32:
        hipLaunchKernelGGL(k_merge_volume<float>, dim3(blocks), dim3(256), 0, s, vx_, vy_, disp, wts, which, w, h, d, dp,
                           vb, out);
        break;
    case OCTMC_BF16:
        hipLaunchKernelGGL(k_merge_volume<bf16_t>, dim3(blocks), dim3(256), 0, s, vx_, vy_, disp, wts, which, w, h,
                           d, dp, vb, out);
        break;
    case OCTMC_F16:
        hipLaunchKernelGGL(k_merge_volume<f16_t>, dim3(blocks), dim3(256), 0, s, vx_, vy_, disp, wts, which, w, h,
                           d, dp, vb, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace octmc
