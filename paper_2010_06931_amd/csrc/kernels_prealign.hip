// Stage 1, rough axial prealignment (Fig. 1, Sec. 2.1 "optimization"):
// kernels that expand the per-B-scan axial offsets and tilts into a
// displacement field, reduce a field gradient back onto them, and resample
// volumes axially (the prealigned volumes).
//
// theta holds, for the X-fast scan, h B-scans (rows j; fast axis x, w
// A-scans each) and then, for the Y-fast scan, w B-scans (columns i; fast
// axis y, h A-scans each), as (z_b, t_b) pairs; the field is
//   dz(f, b) = z_b + t_b (f - (n_f - 1) / 2),  dx = dy = 0,
// with f the index along the fast axis and n_f the B-scan length.
#include "octmc_internal.h"

namespace octmc {
namespace {

// [2][h][w][3] float32 field (dx = dy = 0) and, if dz != nullptr, the axial
// component alone as [2][h][w].
__global__ void k_tilt_expand(const double* __restrict__ th, int w, int h, float* __restrict__ disp,
                              float* __restrict__ dz, const int* __restrict__ skip)
{
    if (skip && *skip) return;
    const size_t na = (size_t)w * h;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 2 * na) return;
    const int V = q >= na ? 1 : 0;
    const size_t a = q - (size_t)V * na;
    const int i = (int)(a % w), j = (int)(a / w);
    const int f = V == 0 ? i : j, b = V == 0 ? j : i;
    const int nf = V == 0 ? w : h;
    const double* t = th + (V == 0 ? 0 : 2 * (size_t)h) + 2 * (size_t)b;
    const float v = (float)(t[0] + t[1] * ((double)f - 0.5 * (nf - 1)));
    if (disp) {
        disp[q * 3 + 0] = 0.0f;
        disp[q * 3 + 1] = 0.0f;
        disp[q * 3 + 2] = v;
    }
    if (dz) dz[q] = v;
}

// Adjoint of the expansion: one wave per B-scan sums the axial gradient and
// its first moment about the B-scan centre in float64, in a fixed order.
__global__ __launch_bounds__(256) void k_tilt_reduce(const float* __restrict__ grad, int w, int h,
                                                     double* __restrict__ gth, const int* __restrict__ skip)
{
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63;
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid >= h + w) return;  // uniform per wave
    const int V = wid < h ? 0 : 1;
    const int b = V == 0 ? wid : wid - h;
    const int nf = V == 0 ? w : h;
    const double c = 0.5 * (nf - 1);
    const size_t base = (size_t)V * w * h;
    double s0 = 0.0, s1 = 0.0;
    for (int f = lane; f < nf; f += 64) {
        const size_t a = V == 0 ? (size_t)b * w + f : (size_t)f * w + b;
        const double g = grad[(base + a) * 3 + 2];
        s0 += g;
        s1 += g * ((double)f - c);
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        s0 += __shfl_xor(s0, m);
        s1 += __shfl_xor(s1, m);
    }
    if (lane == 0) {
        double* o = gth + (V == 0 ? 0 : 2 * (size_t)h) + 2 * (size_t)b;
        o[0] = s0;
        o[1] = s1;
    }
}

// Sum over a 256-thread workgroup in a fixed tree order (every thread gets it).
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// The tilt term of one evaluation: T = sum_V kappa_V (sum_b t_b)^2 with
// kappa_V = gamma_t d n_f (n_f^2 - 1) / (24 n_b), its gradient 2 kappa_V
// sum_b t_b on every tilt of scan V, then F + T and g . p.
__global__ __launch_bounds__(256) void k_tilt_finish(const double* __restrict__ th, double* __restrict__ g, int w,
                                                     int h, int d, double gamma, const double* __restrict__ tin,
                                                     const double* __restrict__ p, double* __restrict__ tout,
                                                     double* __restrict__ T_out, const int* __restrict__ skip)
{
    if (skip && *skip) return;
    __shared__ double sh[256];
    double sum[2], kap[2];
    for (int V = 0; V < 2; ++V) {
        const int nb = V == 0 ? h : w, nf = V == 0 ? w : h;
        const double* t = th + (V == 0 ? 0 : 2 * (size_t)h);
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) v += t[2 * b + 1];
        sum[V] = block_sum(v, sh);
        kap[V] = gamma * d * (double)nf * ((double)nf * nf - 1.0) / (24.0 * nb);
    }
    const double T = kap[0] * sum[0] * sum[0] + kap[1] * sum[1] * sum[1];
    const int n = 2 * (w + h);
    double gp = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        double gk = g[k];
        if (k & 1) gk += 2.0 * (k < 2 * h ? kap[0] * sum[0] : kap[1] * sum[1]);
        g[k] = gk;
        if (p) gp += gk * p[k];
    }
    gp = block_sum(gp, sh);
    if (threadIdx.x < OCTMC_NTERMS) {
        const int q = threadIdx.x;
        tout[q] = q == OCTMC_TERM_F ? tin[q] + T : (q == OCTMC_TERM_GP ? gp : tin[q]);
    }
    if (threadIdx.x == 0 && T_out) *T_out = T;
}

// out(i, j, k) = I(vol, i, j, k + dz(i, j)): the cubic Hermite interpolator
// with central-difference tangents (Catmull-Rom) along depth, tap indices
// clamped to the A-scan.  One block per A-scan (its shift and taps are
// uniform), threads along depth.
__global__ __launch_bounds__(256) void k_resample_z(const float* __restrict__ vol, const float* __restrict__ dz, int d,
                                                   float* __restrict__ out)
{
    const size_t a = blockIdx.x;
    // integer and fractional parts of the shift taken apart so that the
    // fraction is exact (k + dz rounded in float32 would not be); beyond
    // +-(d + 2) every tap is clamped anyway
    const float z = fminf(fmaxf(dz[a], -(float)(d + 2)), (float)(d + 2));
    const float fz = floorf(z);
    const float t = z - fz;
    const float t2 = t * t, t3 = t2 * t;
    const float h00 = 2.0f * t3 - 3.0f * t2 + 1.0f, h10 = t3 - 2.0f * t2 + t;
    const float h01 = -2.0f * t3 + 3.0f * t2, h11 = t3 - t2;
    const float wt[4] = {-0.5f * h10, h00 - 0.5f * h11, h01 + 0.5f * h10, 0.5f * h11};
    const float* __restrict__ col = vol + a * d;
    float* __restrict__ o = out + a * d;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        const int n = k + (int)fz;
        float v = 0.0f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int idx = n - 1 + e;
            idx = idx < 0 ? 0 : (idx >= d ? d - 1 : idx);
            v += wt[e] * col[idx];
        }
        o[k] = v;
    }
}

}  // namespace

hipError_t launch_tilt_expand(const double* theta, int w, int h, float* disp, float* dz, hipStream_t s,
                              const int* skip)
{
    const size_t n = 2 * (size_t)w * h;
    hipLaunchKernelGGL(k_tilt_expand, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, w, h, disp, dz,
                       skip);
    return hipGetLastError();
}

hipError_t launch_tilt_reduce(const float* grad, int w, int h, double* gtheta, hipStream_t s, const int* skip)
{
    hipLaunchKernelGGL(k_tilt_reduce, dim3((unsigned)((w + h + 3) / 4)), dim3(256), 0, s, grad, w, h, gtheta,
                       skip);
    return hipGetLastError();
}

hipError_t launch_tilt_finish(const double* theta, double* gtheta, int w, int h, int d, double gamma_t,
                              const double* terms_in, const double* p, double* terms_out, double* T_out,
                              hipStream_t s, const int* skip)
{
    hipLaunchKernelGGL(k_tilt_finish, dim3(1), dim3(256), 0, s, theta, gtheta, w, h, d, gamma_t, terms_in, p,
                       terms_out, T_out, skip);
    return hipGetLastError();
}

hipError_t launch_resample_z(const float* vol, const float* dz, size_t na, int d, float* out, hipStream_t s)
{
    if (na == 0 || d <= 0) return hipSuccess;
    if (na > 0x7fffffffu) return hipErrorInvalidValue;  // one block per A-scan
    hipLaunchKernelGGL(k_resample_z, dim3((unsigned)na), dim3(256), 0, s, vol, dz, d, out);
    return hipGetLastError();
}

}  // namespace octmc
