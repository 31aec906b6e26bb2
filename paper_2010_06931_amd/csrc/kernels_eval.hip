// Hot-path kernels: one evaluation of the registration objective and its
// gradient (Eqs. 1-10 of Ploner et al., without the stage-1 tilt term).
//
//   k_sum     sum of the displacements of both scans (mean term M)
//   k_struct  per output A-scan: resample both structural volumes with
//             their displacement (Eq. 2), residual, pseudo-Huber loss (Eq. 4)
//             and the depth sums of the loss and of its gradient with respect
//             to the A-scan's displacement; one depth sample per lane (float32
//             storage, and 16-bit volumes of odd depth in the caller's layout)
//   k_struct2 the same with two 16-bit samples per lane (every level a pair
//             stores: an odd depth is stored with one padding sample)
//   k_struct_multi, k_struct_multi1  the structural partials of every volume
//             pair of n = 3 or 4 volumes, each volume resampled once
//   k_combine per output A-scan: en face residual (Eq. 7), resampled
//             validity (Eq. 5), weight delta (Eq. 8), combination with eta
//             (Eq. 9), scan-order regulariser, mean term, gradient; float64
//             block partials
//   k_finalize the float64 global sums in a fixed order (one block per job;
//             a kernel boundary, not a device-scope fence per block, makes
//             the partials visible)
#include <hip/hip_runtime.h>

#include "octmc_internal.h"

namespace octmc {

namespace {

__device__ __forceinline__ float uni(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Cubic Hermite spline with central-difference tangents (Catmull-Rom), the
// C1 "Hermitian" interpolator of Eq. 2: weights of the samples at n-1 .. n+2
// for the fraction t in [0, 1), and their derivatives.
__device__ __forceinline__ void cr_taps(float t, float w[4], float dw[4])
{
    const float t2 = t * t, t3 = t2 * t;
    w[0] = 0.5f * (-t3 + 2.f * t2 - t);
    w[1] = 0.5f * (3.f * t3 - 5.f * t2 + 2.f);
    w[2] = 0.5f * (-3.f * t3 + 4.f * t2 + t);
    w[3] = 0.5f * (t3 - t2);
    dw[0] = 0.5f * (-3.f * t2 + 4.f * t - 1.f);
    dw[1] = 0.5f * (9.f * t2 - 10.f * t);
    dw[2] = 0.5f * (-9.f * t2 + 8.f * t + 1.f);
    dw[3] = 0.5f * (3.f * t2 - 2.f * t);
}

// Split an integer grid coordinate plus a displacement into the integer base
// and the fraction without rounding: dv = floor(dv) + frac exactly.
__device__ __forceinline__ void split(int idx, float dv, int& n, float& t)
{
    const float f = floorf(dv);
    t = dv - f;
    n = idx + (int)f;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <typename T>
__device__ __forceinline__ float ldv(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float ldv<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
struct bf16_t {};
struct f16_t {};
template <>
__device__ __forceinline__ float ldv<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}
template <>
__device__ __forceinline__ float ldv<f16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    return (float)__builtin_bit_cast(_Float16, b);
}
template <typename T> struct esize { static constexpr uint32_t v = 2; };
template <> struct esize<float> { static constexpr uint32_t v = 4; };

constexpr uint32_t kRsrcWord3 = 0x00020000u;

// Stage 1 (rough axial prealignment) evaluates at dx = dy = 0, where the
// lateral weights are (0, 1, 0, 0) in x and y: the blend of the 16 columns
// is exactly the centre column (index 5; every other product is an exact 0),
// so the axial kernels load that column alone and skip the lateral adjoint.
constexpr int kCentre = 5;

// Per-scan stencil of one output A-scan: 16 lateral columns with their
// (wave-uniform) byte offsets and blend weights, and the depth taps.  The
// lateral derivative taps are recomputed after the depth loop (from tx, ty,
// or from make_stencils' per-lane taps), so they do not occupy registers
// during it.
struct Stencil {
    float w[16];
    uint32_t off[16];
    float wz[4], dwz[4];
    float tx, ty;
    int base;  // source sample of the first depth tap of output sample 0
};

// One scan's stencil, every tap and product computed on wave-uniform values
// (the two-samples-per-lane kernel's form: with the per-lane form below its
// register allocation changed and the BF16 kernel ran 21 % slower).
template <typename T>
__device__ __forceinline__ void make_stencil(Stencil& s, int i, int j, float dx, float dy, float dz, int w,
                                             int h, int d)
{
    int nx, ny, nz;
    float tx, ty, tz;
    split(i, uni(dx), nx, tx);
    split(j, uni(dy), ny, ty);
    split(0, uni(dz), nz, tz);
    nx = uni(nx);
    ny = uni(ny);
    nz = uni(nz);
    float wx[4], dwx[4], wy[4], dwy[4];
    cr_taps(uni(tx), wx, dwx);
    cr_taps(uni(ty), wy, dwy);
    cr_taps(uni(tz), s.wz, s.dwz);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        s.wz[c] = uni(s.wz[c]);
        s.dwz[c] = uni(s.dwz[c]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int row = clampi(ny - 1 + b, 0, h - 1);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int col = clampi(nx - 1 + a, 0, w - 1);
            s.off[b * 4 + a] = (uint32_t)uni((int)((uint32_t)(row * w + col) * (uint32_t)d * esize<T>::v));
            s.w[b * 4 + a] = uni(wx[a] * wy[b]);
        }
    }
    s.tx = uni(tx);
    s.ty = uni(ty);
    s.base = uni(nz - 1);
}

// The stencil of the axial kernels (every displacement has dx = dy = 0, so
// the lateral weights are (0, 1, 0, 0) along x and y and the blend is the
// centre column): the depth taps, the centre column's offset and the base;
// the other offsets and weights are left unset (the axial kernels read
// neither).
template <typename T>
__device__ __forceinline__ void make_stencil_axial(Stencil& s, int i, int j, float dz, int w, int d)
{
    int nz;
    float tz;
    split(0, uni(dz), nz, tz);
    cr_taps(uni(tz), s.wz, s.dwz);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        s.wz[c] = uni(s.wz[c]);
        s.dwz[c] = uni(s.dwz[c]);
    }
    s.off[kCentre] = (uint32_t)((uint32_t)(j * w + i) * (uint32_t)d * esize<T>::v);
    s.tx = s.ty = 0.f;
    s.base = uni(nz) - 1;
}

// Both scans' stencils of one output A-scan.  The taps are computed one per
// lane, lane 12 V + 4 p + c holding tap c of scan V's coordinate p (0: x,
// 1: y, 2: z), and the lateral weights w_ab = wx_a wy_b one per lane (lane
// 32 + 16 V + 4 b + a); each is then read out as a wave-uniform value.  That
// takes a few dozen instructions per wave instead of computing every tap and
// product on uniform operands one after another.  tw and tdw keep each
// lane's tap and tap derivative for the lateral gradient after the depth
// loop (tap_x/tap_y read them).
template <typename T>
__device__ __forceinline__ void make_stencils(Stencil& SX, Stencil& SY, float& tw, float& tdw, int i, int j,
                                              const float* dX, const float* dY, int w, int h, int d, int lane)
{
    float t[6];
    int n[6];
    split(i, uni(dX[0]), n[0], t[0]);
    split(j, uni(dX[1]), n[1], t[1]);
    split(0, uni(dX[2]), n[2], t[2]);
    split(i, uni(dY[0]), n[3], t[3]);
    split(j, uni(dY[1]), n[4], t[4]);
    split(0, uni(dY[2]), n[5], t[5]);
#pragma unroll
    for (int k = 0; k < 6; ++k) n[k] = uni(n[k]);
    const int p = lane >> 2, c = lane & 3;
    float tl = t[0];
#pragma unroll
    for (int k = 1; k < 6; ++k) tl = p == k ? t[k] : tl;
    float wv[4], dv[4];
    cr_taps(tl, wv, dv);
    float wl = wv[0], dl = dv[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        wl = c == k ? wv[k] : wl;
        dl = c == k ? dv[k] : dl;
    }
    tw = wl;
    tdw = dl;
    // lanes 32 + 16 V + 4 b + a: wx_a wy_b of scan V
    const int V = (lane >> 4) & 1, b = (lane >> 2) & 3, a = lane & 3;
    const float prod = __shfl(wl, 12 * V + a) * __shfl(wl, 12 * V + 4 + b);
    const int pb = __builtin_bit_cast(int, prod), wb = __builtin_bit_cast(int, wl), db = __builtin_bit_cast(int, dl);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        SX.w[q] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(pb, 32 + q));
        SY.w[q] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(pb, 48 + q));
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        SX.wz[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(wb, 8 + k));
        SX.dwz[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(db, 8 + k));
        SY.wz[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(wb, 20 + k));
        SY.dwz[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(db, 20 + k));
    }
    Stencil* S[2] = {&SX, &SY};
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const int nx = n[3 * v], ny = n[3 * v + 1];
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            const int row = clampi(ny - 1 + bb, 0, h - 1);
#pragma unroll
            for (int aa = 0; aa < 4; ++aa) {
                const int col = clampi(nx - 1 + aa, 0, w - 1);
                S[v]->off[bb * 4 + aa] = (uint32_t)uni((int)((uint32_t)(row * w + col) * (uint32_t)d * esize<T>::v));
            }
        }
        S[v]->base = n[3 * v + 2] - 1;
    }
}

// The lateral taps and their derivatives of scan V (x: p = 0, y: p = 1),
// read back from make_stencils' per-lane values.
__device__ __forceinline__ void lateral_taps(float tw, float tdw, int V, int p, float w[4], float dw[4])
{
    const int wb = __builtin_bit_cast(int, tw), db = __builtin_bit_cast(int, tdw);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(wb, 12 * V + 4 * p + k));
        dw[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(db, 12 * V + 4 * p + k));
    }
}

// Depth is processed in steps of 61 output samples on 64 lanes: lane l holds
// source sample base + 61 n + l, output lane l (< 61) reads source lanes
// l .. l+3, and the adjoint of output lane l goes to the same source lanes.
// Every step is therefore self-contained (a source sample shared by two
// steps receives each step's part of the adjoint separately).
constexpr int kOutPerStep = 61;

template <typename T>
__device__ __forceinline__ void load_cols(float (&v)[16], __amdgpu_buffer_rsrc_t r, const Stencil& s, int step,
                                          int lane, int d)
{
    const int m = clampi(s.base + step * kOutPerStep + lane, 0, d - 1);
    const uint32_t voff = (uint32_t)m * esize<T>::v;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = ldv<T>(r, voff, s.off[q]);
}


__device__ __forceinline__ float blend(const float (&v)[16], const Stencil& s)
{
    float c = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) c = fmaf(s.w[q], v[q], c);
    return c;
}

// Whole-wave lane shifts (DPP): shl1 gives lane l the value of lane l + 1,
// shr1 that of lane l - 1; a lane whose source lies outside the wave reads 0
// (bound control), so the shift can fold into the instruction that uses it.
__device__ __forceinline__ float shl1(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float shr1(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}

// Sum over the wave in float32, left in lane 63: within each row of 16 lanes
// (DPP row shifts; the last lane of a row ends with the row's sum), then two
// row broadcasts (rows 1 and 3 add the last lane of the row before them, then
// rows 2 and 3 add lane 31): (r3 + r2) + (r1 + r0).  Six DPP additions, no
// lane reads.
template <int S>
__device__ __forceinline__ float row_shr_add(float v)
{
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 | S, 0xF,
                                                                     0xF, true));
}
__device__ __forceinline__ float wave_sum_last(float x)
{
    float v = row_shr_add<1>(x);
    v = row_shr_add<2>(v);
    v = row_shr_add<4>(v);
    v = row_shr_add<8>(v);
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false));
    return v;
}
// the same sum, wave-uniform (lane 63's)
__device__ __forceinline__ float wave_sum(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wave_sum_last(x)), 63));
}

// Logical block of a physical one: workgroups are dispatched to the 8 XCDs
// round robin, so give every XCD a contiguous range of tiles (neighbouring
// A-scans then share that XCD's L2).  The grid is a multiple of 8.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    return (b & 7) * (nb >> 3) + (b >> 3);
}

template <typename T, bool AXIAL>
__global__ __launch_bounds__(256) void k_struct(const StructJobs jobs)
{
    if (jobs.skip && *jobs.skip) return;
    const int wv = uni((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    int jid = -1;
    for (int q = 0; q < jobs.n; ++q)
        if (lb >= jobs.j[q].blk_begin) jid = q;
    if (jid < 0) return;  // whole block
    const StructJob& J = jobs.j[jid];
    const int w = J.w, h = J.h, d = J.d;
    const int dp = J.dp;  // storage pitch: d, or d + 1 (a padding sample) for an odd depth in 16-bit storage
    // 2 x 2 tile of output A-scans per workgroup, one per wave.  The tile
    // rows form 8 bands (one per XCD when the job fills the grid); a band is
    // swept column by column, so the rows a tile reads are still in that
    // XCD's L2 when the neighbouring column of tiles reads them again.
    const int tpr = (w + 1) >> 1;
    const int trows = (h + 1) >> 1;
    const int rpb = (trows + 7) >> 3;
    const int t = lb - J.blk_begin;
    const int band = t / (rpb * tpr), tb = t - band * (rpb * tpr);
    const int trow = band * rpb + tb % rpb;
    if (t >= 8 * rpb * tpr || trow >= trows) return;  // whole block
    const int i = 2 * (tb / rpb) + (wv & 1);
    const int j = 2 * trow + (wv >> 1);
    // With float32 storage the waves of a tile step through depth together
    // (one barrier per step), so the columns they share are still in the L1
    // cache when the others read them (measured: no gain for 16-bit
    // storage).  A wave outside the scan only takes part in the barriers.
    const bool active = i < w && j < h;  // wave-uniform
    const int a = uni(active ? j * w + i : 0);
    const float* dX = J.disp + (size_t)a * 3;
    const float* dY = J.disp + ((size_t)J.na + a) * 3;
    Stencil SX, SY;
    float tw = 0.f, tdw = 0.f;
    if constexpr (AXIAL) {
        make_stencil_axial<T>(SX, i, j, dX[2], w, dp);
        make_stencil_axial<T>(SY, i, j, dY[2], w, dp);
    } else {
        make_stencils<T>(SX, SY, tw, tdw, i, j, dX, dY, w, h, dp, lane);
    }
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(J.sx), (short)0, (int)J.vol_bytes, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t ry =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(J.sy), (short)0, (int)J.vol_bytes, kRsrcWord3);
    const float eps = J.eps_h;
    const float inv_eps = 1.0f / J.eps_h;

    float sx[16], sy[16];
    float PX[16], PY[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) PX[q] = PY[q] = 0.f;
    float lam = 0.f, gzx = 0.f, gzy = 0.f;
    const int nsteps = (d + kOutPerStep - 1) / kOutPerStep;
    for (int n = 0; n < nsteps; ++n) {
        if (active) {
            float vx, vy;
            if constexpr (AXIAL) {
                const int m = clampi(SX.base + n * kOutPerStep + lane, 0, d - 1);
                const int my = clampi(SY.base + n * kOutPerStep + lane, 0, d - 1);
                vx = ldv<T>(rx, (uint32_t)m * esize<T>::v, SX.off[kCentre]);
                vy = ldv<T>(ry, (uint32_t)my * esize<T>::v, SY.off[kCentre]);
            } else {
                load_cols<T>(sx, rx, SX, n, lane, d);
                load_cols<T>(sy, ry, SY, n, lane, d);
                vx = blend(sx, SX);
                vy = blend(sy, SY);
            }
            // blended columns, then the depth interpolation of Eq. 2 and its
            // depth derivative: output lane l reads source lanes l .. l + 3
            float ix = 0.f, izx = 0.f, iy = 0.f, izy = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ix = fmaf(SX.wz[c], vx, ix);
                izx = fmaf(SX.dwz[c], vx, izx);
                iy = fmaf(SY.wz[c], vy, iy);
                izy = fmaf(SY.dwz[c], vy, izy);
                if (c < 3) {
                    vx = shl1(vx);
                    vy = shl1(vy);
                }
            }
            // residual (Eq. 2) and pseudo-Huber loss (Eq. 4) in the form
            // eps u^2 / (sqrt(1 + u^2) + 1), u = r / eps, and its derivative u / sqrt(1 + u^2)
            const float r = ix - iy;
            const float u = r * inv_eps;
            const float q = u * u;
            const float rs = __builtin_amdgcn_rsqf(1.f + q);
            const float sq = (1.f + q) * rs;
            const bool valid = lane < kOutPerStep && (n * kOutPerStep + lane) < d;
            const float L = valid ? eps * q * __builtin_amdgcn_rcpf(sq + 1.f) : 0.f;
            const float G = valid ? u * rs : 0.f;
            lam += L;
            gzx += valid ? G * izx : 0.f;
            gzy += valid ? G * izy : 0.f;
            if constexpr (!AXIAL) {
                // adjoint of the depth interpolation: source lane l collects the
                // derivatives of output lanes l - 3 .. l (invalid lanes carry 0)
                float hx = 0.f, hy = 0.f, g = G;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    hx = fmaf(SX.wz[c], g, hx);
                    hy = fmaf(SY.wz[c], g, hy);
                    if (c < 3) g = shr1(g);
                }
#pragma unroll
                for (int q2 = 0; q2 < 16; ++q2) {
                    PX[q2] = fmaf(sx[q2], hx, PX[q2]);
                    PY[q2] = fmaf(sy[q2], hy, PY[q2]);
                }
            }
        }
        if constexpr (esize<T>::v == 4) __builtin_amdgcn_s_barrier();
    }
    if (!active) return;
    // Gamma_x = sum_b wy_b sum_a dwx_a P_ab, Gamma_y = sum_b dwy_b sum_a wx_a P_ab
    // (left at 0 by the axial kernel: stage 1 uses only the z components)
    float wx[4], dwx[4], wy[4], dwy[4];
    float gxx = 0.f, gyx = 0.f, gxy = 0.f, gyy = 0.f;
    if constexpr (!AXIAL) {
        lateral_taps(tw, tdw, 0, 0, wx, dwx);
        lateral_taps(tw, tdw, 0, 1, wy, dwy);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float rv = 0.f, rd = 0.f;
#pragma unroll
            for (int a2 = 0; a2 < 4; ++a2) {
                rv = fmaf(wx[a2], PX[b * 4 + a2], rv);
                rd = fmaf(dwx[a2], PX[b * 4 + a2], rd);
            }
            gxx = fmaf(wy[b], rd, gxx);
            gyx = fmaf(dwy[b], rv, gyx);
        }
        lateral_taps(tw, tdw, 1, 0, wx, dwx);
        lateral_taps(tw, tdw, 1, 1, wy, dwy);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float rv = 0.f, rd = 0.f;
#pragma unroll
            for (int a2 = 0; a2 < 4; ++a2) {
                rv = fmaf(wx[a2], PY[b * 4 + a2], rv);
                rd = fmaf(dwx[a2], PY[b * 4 + a2], rd);
            }
            gxy = fmaf(wy[b], rd, gxy);
            gyy = fmaf(dwy[b], rv, gyy);
        }
    }
    lam = wave_sum(lam);
    gxx = wave_sum(gxx);
    gyx = wave_sum(gyx);
    gzx = wave_sum(gzx);
    gxy = wave_sum(gxy);
    gyy = wave_sum(gyy);
    gzy = wave_sum(gzy);
    if (lane == 0) {
        float4* o = reinterpret_cast<float4*>(J.part + (size_t)a * 8);
        o[0] = make_float4(lam, gxx, gyx, gzx);
        o[1] = make_float4(gxy, gyy, gzy, 0.f);
    }
}

// Two depth samples per lane (16-bit storage).  A step covers outputs o = 122 n + p - sx,
// p = 2 l + e in [sx, 121 + sx] (lane l, e in {0, 1}), sx = parity of the
// X-fast scan's first depth tap.  Pair position p of scan V holds the
// sample base_V + o of output o's first tap, so the depth interpolation of
// output p reads positions p .. p + 3 (this lane and the next one or two, by
// DPP).  Each scan loads even-aligned pairs (q0, q1) = samples (E + 2l,
// E + 2l + 1) with one 32-bit load per column; a
// scan whose positions start one sample after an even boundary (r = 1) uses
// c0 = q1 and c1 = the next lane's q0 (so the taps of every output, up to
// position 125, lie inside the 128 loaded samples).  Samples outside the A-scan take the
// edge value (clamp), applied to the blended columns and, for the adjoint, to
// the weights of q0 and q1.  Every step is self-contained as in k_struct.
constexpr int kOutPerStep2 = 122;

// A pair of 16-bit samples is one 32-bit load.  (Float32 storage keeps one
// sample per lane: 64-bit loads measured slower per byte than 32-bit ones on
// this path, so pairs would not pay.)
template <typename T>
__device__ __forceinline__ void ld2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float& a, float& b);
template <>
__device__ __forceinline__ void ld2<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float& a, float& b)
{
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    a = __builtin_bit_cast(float, v << 16);
    b = __builtin_bit_cast(float, v & 0xFFFF0000u);
}
template <>
__device__ __forceinline__ void ld2<f16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float& a, float& b)
{
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    a = (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xFFFFu));
    b = (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16));
}

template <typename T>
__device__ __forceinline__ void load_pairs(float (&q0)[16], float (&q1)[16], __amdgpu_buffer_rsrc_t rs,
                                           const Stencil& S, int m, int dp)
{
    const int mc = clampi(m, 0, dp - 2);
    const uint32_t voff = (uint32_t)mc * esize<T>::v;
#pragma unroll
    for (int q = 0; q < 16; ++q) ld2<T>(rs, voff, S.off[q], q0[q], q1[q]);
}

template <typename T, bool AXIAL>
__global__ __launch_bounds__(256) void k_struct2(const StructJobs jobs)
{
    if (jobs.skip && *jobs.skip) return;
    const int wv = uni((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    int jid = -1;
    for (int q = 0; q < jobs.n; ++q)
        if (lb >= jobs.j[q].blk_begin) jid = q;
    if (jid < 0) return;  // whole block
    const StructJob& J = jobs.j[jid];
    const int w = J.w, h = J.h, d = J.d;
    const int dp = J.dp;  // storage pitch: d, or d + 1 (a padding sample) for an odd depth in 16-bit storage
    // 2 x 2 tiles in 8 bands of tile rows, swept column by column (as k_struct)
    const int tpr = (w + 1) >> 1;
    const int trows = (h + 1) >> 1;
    const int rpb = (trows + 7) >> 3;
    const int t = lb - J.blk_begin;
    const int band = t / (rpb * tpr), tb = t - band * (rpb * tpr);
    const int trow = band * rpb + tb % rpb;
    if (t >= 8 * rpb * tpr || trow >= trows) return;  // whole block
    const int i = 2 * (tb / rpb) + (wv & 1);
    const int j = 2 * trow + (wv >> 1);
    const bool active = i < w && j < h;  // wave-uniform
    const int a = uni(active ? j * w + i : 0);
    const float* dX = J.disp + (size_t)a * 3;
    const float* dY = J.disp + ((size_t)J.na + a) * 3;
    Stencil SX, SY;
    if constexpr (AXIAL) {
        make_stencil_axial<T>(SX, i, j, dX[2], w, dp);
        make_stencil_axial<T>(SY, i, j, dY[2], w, dp);
    } else {
        make_stencil<T>(SX, i, j, dX[0], dX[1], dX[2], w, h, dp);
        make_stencil<T>(SY, i, j, dY[0], dY[1], dY[2], w, h, dp);
    }
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(J.sx), (short)0, (int)J.vol_bytes, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t ry =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(J.sy), (short)0, (int)J.vol_bytes, kRsrcWord3);
    const float eps = J.eps_h;
    const float inv_eps = 1.0f / J.eps_h;
    // position 0 of step 0 holds sample base_V - sx of scan V
    const int sx = SX.base & 1;
    const int rY = uni((SY.base - sx) & 1);
    const int EX = SX.base - sx, EY = SY.base - sx - rY;  // even

    float x0[16], x1[16], y0[16], y1[16];
    float PX[16], PY[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) PX[q] = PY[q] = 0.f;
    float lam = 0.f, gzx = 0.f, gzy = 0.f;
    const int nsteps = (d + kOutPerStep2 - 1) / kOutPerStep2;
    for (int n = 0; n < nsteps; ++n) {
        if (active) {
            const int mX = EX + kOutPerStep2 * n + 2 * lane;
            const int mY = EY + kOutPerStep2 * n + 2 * lane;
            float bx0, bx1, by0, by1;
            if constexpr (AXIAL) {
                ld2<T>(rx, (uint32_t)clampi(mX, 0, dp - 2) * esize<T>::v, SX.off[kCentre], bx0, bx1);
                ld2<T>(ry, (uint32_t)clampi(mY, 0, dp - 2) * esize<T>::v, SY.off[kCentre], by0, by1);
            } else {
                load_pairs<T>(x0, x1, rx, SX, mX, dp);
                load_pairs<T>(y0, y1, ry, SY, mY, dp);
                bx0 = blend(x0, SX);
                bx1 = blend(x1, SX);
                by0 = blend(y0, SY);
                by1 = blend(y1, SY);
            }
            // clamp: a pair below the A-scan holds sample 0 twice, one above it sample d - 1 twice
            // (with an odd depth the last stored pair is sample d - 1 and its padding copy)
            const bool loX = mX < 0, hiX = mX > dp - 2, loY = mY < 0, hiY = mY > dp - 2;
            const float cx0 = hiX ? bx1 : bx0, cx1 = loX ? bx0 : bx1;
            const float ty0 = hiY ? by1 : by0, ty1 = loY ? by0 : by1;
            // Y positions start one sample after the pair boundary when rY = 1
            const float ty0n = shl1(ty0);
            const float cy0 = rY ? ty1 : ty0, cy1 = rY ? ty0n : ty1;
            // depth interpolation (Eq. 2) of outputs at positions 2l and 2l + 1
            const float cx0n = shl1(cx0), cx1n = shl1(cx1), cx0nn = shl1(cx0n);
            const float cy0n = shl1(cy0), cy1n = shl1(cy1), cy0nn = shl1(cy0n);
            const float ix0 = SX.wz[0] * cx0 + SX.wz[1] * cx1 + SX.wz[2] * cx0n + SX.wz[3] * cx1n;
            const float ix1 = SX.wz[0] * cx1 + SX.wz[1] * cx0n + SX.wz[2] * cx1n + SX.wz[3] * cx0nn;
            const float zx0 = SX.dwz[0] * cx0 + SX.dwz[1] * cx1 + SX.dwz[2] * cx0n + SX.dwz[3] * cx1n;
            const float zx1 = SX.dwz[0] * cx1 + SX.dwz[1] * cx0n + SX.dwz[2] * cx1n + SX.dwz[3] * cx0nn;
            const float iy0 = SY.wz[0] * cy0 + SY.wz[1] * cy1 + SY.wz[2] * cy0n + SY.wz[3] * cy1n;
            const float iy1 = SY.wz[0] * cy1 + SY.wz[1] * cy0n + SY.wz[2] * cy1n + SY.wz[3] * cy0nn;
            const float zy0 = SY.dwz[0] * cy0 + SY.dwz[1] * cy1 + SY.dwz[2] * cy0n + SY.dwz[3] * cy1n;
            const float zy1 = SY.dwz[0] * cy1 + SY.dwz[1] * cy0n + SY.dwz[2] * cy1n + SY.dwz[3] * cy0nn;
            // residual and pseudo-Huber loss (Eq. 4), eps u^2 / (sqrt(1 + u^2) + 1), and u / sqrt(1 + u^2)
            const int p0 = 2 * lane;
            const int o0 = kOutPerStep2 * n + p0 - sx;
            const bool v0 = p0 >= sx && p0 <= 121 + sx && o0 < d;
            const bool v1 = p0 + 1 <= 121 + sx && o0 + 1 < d;
            float L0, G0, L1, G1;
            {
                const float u = (ix0 - iy0) * inv_eps, q = u * u;
                const float rs = __builtin_amdgcn_rsqf(1.f + q), sq = (1.f + q) * rs;
                L0 = v0 ? eps * q * __builtin_amdgcn_rcpf(sq + 1.f) : 0.f;
                G0 = v0 ? u * rs : 0.f;
            }
            {
                const float u = (ix1 - iy1) * inv_eps, q = u * u;
                const float rs = __builtin_amdgcn_rsqf(1.f + q), sq = (1.f + q) * rs;
                L1 = v1 ? eps * q * __builtin_amdgcn_rcpf(sq + 1.f) : 0.f;
                G1 = v1 ? u * rs : 0.f;
            }
            lam += L0 + L1;
            gzx += G0 * zx0 + G1 * zx1;
            gzy += G0 * zy0 + G1 * zy1;
            if constexpr (!AXIAL) {
                // adjoint of the depth interpolation: position q collects the
                // derivatives of the outputs at q, q - 1, q - 2, q - 3
                const float G0p = shr1(G0), G1p = shr1(G1), G1pp = shr1(G1p);
                const float hx0 = SX.wz[0] * G0 + SX.wz[1] * G1p + SX.wz[2] * G0p + SX.wz[3] * G1pp;
                const float hx1 = SX.wz[0] * G1 + SX.wz[1] * G0 + SX.wz[2] * G1p + SX.wz[3] * G0p;
                const float hy0 = SY.wz[0] * G0 + SY.wz[1] * G1p + SY.wz[2] * G0p + SY.wz[3] * G1pp;
                const float hy1 = SY.wz[0] * G1 + SY.wz[1] * G0 + SY.wz[2] * G1p + SY.wz[3] * G0p;
                // back to the loaded samples q0, q1: alignment shift, then clamp
                const float hy1p = shr1(hy1);
                const float uy0 = rY ? hy1p : hy0, uy1 = rY ? hy0 : hy1;
                const float wx0 = loX ? hx0 + hx1 : (hiX ? 0.f : hx0);
                const float wx1 = hiX ? hx0 + hx1 : (loX ? 0.f : hx1);
                const float wy0 = loY ? uy0 + uy1 : (hiY ? 0.f : uy0);
                const float wy1 = hiY ? uy0 + uy1 : (loY ? 0.f : uy1);
#pragma unroll
                for (int q2 = 0; q2 < 16; ++q2) {
                    PX[q2] = fmaf(x0[q2], wx0, fmaf(x1[q2], wx1, PX[q2]));
                    PY[q2] = fmaf(y0[q2], wy0, fmaf(y1[q2], wy1, PY[q2]));
                }
            }
        }
    }
    if (!active) return;
    float wx[4], dwx[4], wy[4], dwy[4];
    float gxx = 0.f, gyx = 0.f, gxy = 0.f, gyy = 0.f;
    if constexpr (!AXIAL) {
        cr_taps(SX.tx, wx, dwx);
        cr_taps(SX.ty, wy, dwy);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float rv = 0.f, rd = 0.f;
#pragma unroll
            for (int a2 = 0; a2 < 4; ++a2) {
                rv = fmaf(wx[a2], PX[b * 4 + a2], rv);
                rd = fmaf(dwx[a2], PX[b * 4 + a2], rd);
            }
            gxx = fmaf(wy[b], rd, gxx);
            gyx = fmaf(dwy[b], rv, gyx);
        }
        cr_taps(SY.tx, wx, dwx);
        cr_taps(SY.ty, wy, dwy);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float rv = 0.f, rd = 0.f;
#pragma unroll
            for (int a2 = 0; a2 < 4; ++a2) {
                rv = fmaf(wx[a2], PY[b * 4 + a2], rv);
                rd = fmaf(dwx[a2], PY[b * 4 + a2], rd);
            }
            gxy = fmaf(wy[b], rd, gxy);
            gyy = fmaf(dwy[b], rv, gyy);
        }
    }
    lam = wave_sum(lam);
    gxx = wave_sum(gxx);
    gyx = wave_sum(gyx);
    gzx = wave_sum(gzx);
    gxy = wave_sum(gxy);
    gyy = wave_sum(gyy);
    gzy = wave_sum(gzy);
    if (lane == 0) {
        float4* o = reinterpret_cast<float4*>(J.part + (size_t)a * 8);
        o[0] = make_float4(lam, gxx, gyx, gzx);
        o[1] = make_float4(gxy, gyy, gzy, 0.f);
    }
}

// ---------------------------------------------------------------------------
// deterministic block reduction helpers

template <int N>
__device__ __forceinline__ void block_reduce_store(double (&v)[N], double* blk_row)
{
    __shared__ double sh[N][kRedBlock];
#pragma unroll
    for (int q = 0; q < N; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < N; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < N) blk_row[threadIdx.x] = sh[threadIdx.x][0];
}

// Fixed-order sum of the rows of block partials (strided per thread, then a
// fixed tree); every thread of the block receives the result, and every block
// that sums the same rows gets the same bits.
template <int N>
__device__ __forceinline__ void sum_rows(const double* blk, int nblk, double (&out)[N])
{
    __shared__ double sh[N][kRedBlock];
    double acc[N];
#pragma unroll
    for (int q = 0; q < N; ++q) acc[q] = 0.0;
    for (int r = threadIdx.x; r < nblk; r += kRedBlock) {
#pragma unroll
        for (int q = 0; q < N; ++q) acc[q] += blk[(size_t)r * N + q];
    }
#pragma unroll
    for (int q = 0; q < N; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < N; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < N; ++q) out[q] = sh[q][0];
}

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kRedBlock) void k_sum(const SumJobs jobs)
{
    if (jobs.skip && *jobs.skip) return;
    int jid = 0;
    for (int q = 1; q < jobs.n; ++q)
        if ((int)blockIdx.x >= jobs.j[q].blk_begin) jid = q;
    const SumJob& J = jobs.j[jid];
    const int b = blockIdx.x - J.blk_begin;
    double v[4] = {0, 0, 0, 0};
    const int total = 2 * J.na;
    for (int q = b * kRedBlock + threadIdx.x; q < total; q += J.nblk * kRedBlock) {
        const float* dq = q < J.na ? J.disp[0] + (size_t)q * 3 : J.disp[1] + (size_t)(q - J.na) * 3;
        v[0] += (double)dq[0];
        v[1] += (double)dq[1];
        v[2] += (double)dq[2];
    }
    block_reduce_store<4>(v, J.blk + (size_t)b * 4);
}

// pseudo-Huber in float64 (regulariser and en face terms)
__device__ __forceinline__ void huber_d(double x, double eps, double& L, double& dL)
{
    const double u = x / eps;
    const double s = sqrt(1.0 + u * u);
    L = eps * u * u / (s + 1.0);
    dL = u / s;
}

// 2-D / 1-D Catmull-Rom samples (value and derivatives) in float32
__device__ __forceinline__ void sample2(const float* img, int w, int h, int i, int j, float dx, float dy,
                                        float out[3])
{
    int nx, ny;
    float tx, ty;
    split(i, dx, nx, tx);
    split(j, dy, ny, ty);
    float wx[4], dwx[4], wy[4], dwy[4];
    cr_taps(tx, wx, dwx);
    cr_taps(ty, wy, dwy);
    float v = 0.f, gx = 0.f, gy = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float* row = img + (size_t)clampi(ny - 1 + b, 0, h - 1) * w;
        float rv = 0.f, rd = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const float s = row[clampi(nx - 1 + a, 0, w - 1)];
            rv = fmaf(wx[a], s, rv);
            rd = fmaf(dwx[a], s, rd);
        }
        v = fmaf(wy[b], rv, v);
        gx = fmaf(wy[b], rd, gx);
        gy = fmaf(dwy[b], rv, gy);
    }
    out[0] = v;
    out[1] = gx;
    out[2] = gy;
}

__device__ __forceinline__ void sample1(const float* vec, int n, int i, float dv, float out[2])
{
    int nx;
    float t;
    split(i, dv, nx, t);
    float w[4], dw[4];
    cr_taps(t, w, dw);
    float v = 0.f, g = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const float s = vec[clampi(nx - 1 + a, 0, n - 1)];
        v = fmaf(w[a], s, v);
        g = fmaf(dw[a], s, g);
    }
    out[0] = v;
    out[1] = g;
}

// Neighbours of output A-scan (i, j) in scan V's acquisition order (X-fast:
// along rows, then to the next row; Y-fast: along columns).  Returns the
// A-scan index or -1, and the link weight (1 inside a B-scan, wfb across the
// flyback between B-scans).
__device__ __forceinline__ int prev_ascan(int V, int i, int j, int w, int h, double wfb, double& om)
{
    if (V == 0) {
        if (i > 0) { om = 1.0; return j * w + i - 1; }
        if (j > 0) { om = wfb; return (j - 1) * w + (w - 1); }
    } else {
        if (j > 0) { om = 1.0; return (j - 1) * w + i; }
        if (i > 0) { om = wfb; return (h - 1) * w + (i - 1); }
    }
    om = 0.0;
    return -1;
}
__device__ __forceinline__ int next_ascan(int V, int i, int j, int w, int h, double wfb, double& om)
{
    if (V == 0) {
        if (i < w - 1) { om = 1.0; return j * w + i + 1; }
        if (j < h - 1) { om = wfb; return (j + 1) * w; }
    } else {
        if (j < h - 1) { om = 1.0; return (j + 1) * w + i; }
        if (i < w - 1) { om = wfb; return i + 1; }
    }
    om = 0.0;
    return -1;
}

__global__ __launch_bounds__(kRedBlock) void k_combine(const CombineJobs jobs)
{
    if (jobs.skip && *jobs.skip) return;
    int jid = 0;
    for (int q = 1; q < jobs.n; ++q)
        if ((int)blockIdx.x >= jobs.j[q].blk_begin) jid = q;
    const CombineJob& J = jobs.j[jid];
    const int b = blockIdx.x - J.blk_begin;
    const int a = b * kRedBlock + threadIdx.x;
    // sum of all displacements (mean term), from the partials of k_sum
    double sumd[4] = {0, 0, 0, 0};
    if (J.mode == 1) sum_rows<4>(J.sum_blk, J.nsum, sumd);  // block-uniform
    // partial sums: data, str, ang, reg, (unused), str05, ang05, g.p
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (a < J.na) {
        const int w = J.w, h = J.h, na = J.na;
        const double dd = (double)J.d;
        const int i = a % w, j = a / w;
        const float4 p0 = reinterpret_cast<const float4*>(J.part)[(size_t)a * 2];
        const float4 p1 = reinterpret_cast<const float4*>(J.part)[(size_t)a * 2 + 1];
        const double lam = p0.x;
        const float* dX = J.disp[0] + (size_t)a * 3;
        const float* dY = J.disp[1] + (size_t)a * 3;
        float jx[3], jy[3];
        sample2(J.ax, w, h, i, j, dX[0], dX[1], jx);
        sample2(J.ay, w, h, i, j, dY[0], dY[1], jy);
        double LA, GA;
        huber_d((double)jx[0] - (double)jy[0], J.eps_h, LA, GA);
        // validity (Eq. 5) varies along each scan's slow axis: y for an X-fast
        // scan (index j, component dy), x for a Y-fast scan
        const int oX = J.orient & 1, oY = (J.orient >> 1) & 1;
        float rx[2], ry[2];
        if (oX == 0) sample1(J.vx, h, j, dX[1], rx);
        else sample1(J.vx, w, i, dX[0], rx);
        if (oY == 1) sample1(J.vy, w, i, dY[0], ry);
        else sample1(J.vy, h, j, dY[1], ry);
        const double tvx = rx[0] <= 0.f ? 0.0 : (rx[0] >= 1.f ? 1.0 : (double)rx[0]);
        const double dtvx = (rx[0] > 0.f && rx[0] < 1.f) ? (double)rx[1] : 0.0;
        const double tvy = ry[0] <= 0.f ? 0.0 : (ry[0] >= 1.f ? 1.0 : (double)ry[0]);
        const double dtvy = (ry[0] > 0.f && ry[0] < 1.f) ? (double)ry[1] : 0.0;
        v[5] = (1.0 - 0.5 * tvx * tvy) * lam;
        v[6] = 0.5 * tvx * tvy * dd * LA;
        if (J.mode == 1) {
            const double eta = *J.eta;
            const double delta = J.delta0 * tvx * tvy;  // Eq. 8
            const double ws = eta * (1.0 - delta);       // structural weight (Eqs. 6, 9)
            const double wa = dd / eta * delta;          // angiographic weight (Eqs. 7, 9)
            v[1] = (1.0 - delta) * lam;
            v[2] = delta * dd * LA;
            v[0] = eta * v[1] + v[2] / eta;
            const double dpd = -eta * lam + dd / eta * LA;  // d(data)/d(delta)
            double g[6];
            g[0] = ws * p0.y + wa * GA * jx[1];
            g[1] = ws * p0.z + wa * GA * jx[2];
            g[2] = ws * p0.w;
            g[3] = -(ws * p1.x + wa * GA * jy[1]);
            g[4] = -(ws * p1.y + wa * GA * jy[2]);
            g[5] = -(ws * p1.z);
            g[oX == 0 ? 1 : 0] += dpd * J.delta0 * tvy * dtvx;
            g[oY == 1 ? 3 : 4] += dpd * J.delta0 * tvx * dtvy;
            // scan-order regulariser (gather form: this A-scan's two links)
            double reg = 0.0;
            for (int V = 0; V < 2; ++V) {
                const float* DV = J.disp[V];
                const float* da = DV + (size_t)a * 3;
                const int oV = V == 0 ? oX : oY;  // acquisition order of the slot's scan
                double omp, omn;
                const int pa = prev_ascan(oV, i, j, w, h, J.wfb, omp);
                const int nb = next_ascan(oV, i, j, w, h, J.wfb, omn);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double Lr, dLr;
                    if (pa >= 0) {
                        huber_d((double)da[c] - (double)DV[(size_t)pa * 3 + c], J.eps_r, Lr, dLr);
                        g[V * 3 + c] += J.alpha * dd * omp * dLr;
                    }
                    if (nb >= 0) {
                        huber_d((double)DV[(size_t)nb * 3 + c] - (double)da[c], J.eps_r, Lr, dLr);
                        g[V * 3 + c] -= J.alpha * dd * omn * dLr;
                        reg += dd * omn * Lr;
                    }
                }
            }
            v[3] = reg;
            // mean-displacement term: dM/dd_c = gamma d sum_c / N_A
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double gm = J.gamma * dd * sumd[c] / (double)na;
                g[c] += gm;
                g[3 + c] += gm;
            }
            if (J.grad) {
                float* gX = J.grad + (size_t)a * 3;
                float* gY = J.grad + ((size_t)na + a) * 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    gX[c] = (float)g[c];
                    gY[c] = (float)g[3 + c];
                }
            }
            if (J.grad64) {
                double* gX = J.grad64 + (size_t)a * 3;
                double* gY = J.grad64 + ((size_t)na + a) * 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    gX[c] = g[c];
                    gY[c] = g[3 + c];
                }
            }
            if (J.p) {  // directional derivative g . p (line search)
                const double* pX = J.p + (size_t)a * 3;
                const double* pY = J.p + ((size_t)na + a) * 3;
                double gp = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) gp += g[c] * pX[c] + g[3 + c] * pY[c];
                v[7] = gp;
            }
        }
    }
    block_reduce_store<8>(v, J.blk + (size_t)b * 8);
}

// Final sums of one evaluation per job (one block each), after k_combine:
// the objective terms (mode 1) or the level's eta (mode 0, Eq. 10).
__global__ __launch_bounds__(kRedBlock) void k_finalize(const CombineJobs jobs)
{
    if (jobs.skip && *jobs.skip) return;
    const CombineJob& J = jobs.j[blockIdx.x];
    double s[8];
    sum_rows<8>(J.blk, J.nblk, s);
    if (J.mode == 0) {
        // eta = 1 where a term vanishes (identical inputs)
        if (threadIdx.x == 0) *J.eta = (s[5] > 1e-300 && s[6] > 1e-300) ? sqrt(s[6] / s[5]) : 1.0;
        return;
    }
    double sumd[4];
    sum_rows<4>(J.sum_blk, J.nsum, sumd);
    if (threadIdx.x == 0) {
        const double eta = *J.eta;
        double m = 0.0;
        for (int c = 0; c < 3; ++c) m += sumd[c] * sumd[c];
        m *= J.gamma * (double)J.d / (2.0 * (double)J.na);
        double* t = J.terms;
        t[OCTMC_TERM_DATA] = s[0];
        t[OCTMC_TERM_STR] = s[1];
        t[OCTMC_TERM_ANG] = s[2];
        t[OCTMC_TERM_REG] = s[3];
        t[OCTMC_TERM_MEAN] = m;
        t[OCTMC_TERM_STR05] = s[5];
        t[OCTMC_TERM_ANG05] = s[6];
        t[OCTMC_TERM_ETA] = eta;
        t[OCTMC_TERM_GP] = s[7];
        t[OCTMC_TERM_F] = s[0] + J.alpha * s[3] + m;
    }
}

// ---------------------------------------------------------------------------
// k_struct_multi: the structural data term of n = 3 or 4 volumes at one
// level (16-bit storage, even depth).  Each output A-scan resamples every
// volume once: the lateral blend of its value and of its x and y derivatives
// (separable: 4 taps along x per source row, then 4 along y), the depth
// interpolation (Eq. 2) of all three, and the depth derivative of the value.
// Every volume pair P < Q then forms the residual I_P - I_Q, the
// pseudo-Huber loss (Eq. 4) and the loss derivative times both volumes'
// derivatives, and writes the eight partial sums per A-scan that k_struct2
// writes for one pair (loss; x, y, z of P; x, y, z of Q; 0).  The pair
// kernels instead resample every volume once per pair it belongs to.
// Lanes hold two samples each, on the output grid of the first volume, as
// in k_struct2.

struct StencilS {
    uint32_t roff[4], coff[4];  // byte offsets of the 4 source rows and the 4 source columns
    float wx[4], dwx[4], wy[4], dwy[4];
    float wz[4], dwz[4];
    int base;  // source sample of the first depth tap of output sample 0
};

template <typename T>
__device__ __forceinline__ void make_stencil_s(StencilS& s, int i, int j, float dx, float dy, float dz, int w, int h,
                                               int d)
{
    int nx, ny, nz;
    float tx, ty, tz;
    split(i, uni(dx), nx, tx);
    split(j, uni(dy), ny, ty);
    split(0, uni(dz), nz, tz);
    nx = uni(nx);
    ny = uni(ny);
    nz = uni(nz);
    cr_taps(uni(tx), s.wx, s.dwx);
    cr_taps(uni(ty), s.wy, s.dwy);
    cr_taps(uni(tz), s.wz, s.dwz);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        s.wz[c] = uni(s.wz[c]);
        s.dwz[c] = uni(s.dwz[c]);
        s.roff[c] = (uint32_t)uni((int)((uint32_t)clampi(ny - 1 + c, 0, h - 1) * (uint32_t)w * (uint32_t)d *
                                        esize<T>::v));
        s.coff[c] = (uint32_t)uni((int)((uint32_t)clampi(nx - 1 + c, 0, w - 1) * (uint32_t)d * esize<T>::v));
    }
    s.base = uni(nz - 1);
}

// value, x derivative and y derivative blends of the 16 columns at one depth
__device__ __forceinline__ void blend3(const float (&c)[16], const StencilS& S, float& v, float& vx, float& vy)
{
    float r[4], dr[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        r[b] = S.wx[0] * c[b * 4];
        dr[b] = S.dwx[0] * c[b * 4];
#pragma unroll
        for (int a = 1; a < 4; ++a) {
            r[b] = fmaf(S.wx[a], c[b * 4 + a], r[b]);
            dr[b] = fmaf(S.dwx[a], c[b * 4 + a], dr[b]);
        }
    }
    v = S.wy[0] * r[0];
    vx = S.wy[0] * dr[0];
    vy = S.dwy[0] * r[0];
#pragma unroll
    for (int b = 1; b < 4; ++b) {
        v = fmaf(S.wy[b], r[b], v);
        vx = fmaf(S.wy[b], dr[b], vx);
        vy = fmaf(S.dwy[b], r[b], vy);
    }
}

// Blended values t0, t1 of the loaded pair (samples m, m + 1) to positions 2l
// and 2l + 1 of the output grid: clamp (a pair below the A-scan holds sample
// 0 twice, one above it sample d - 1 twice), then the shift by one sample
// when the volume's positions start one sample after a pair boundary (r = 1).
__device__ __forceinline__ void grid2(float t0, float t1, bool lo, bool hi, int r, float& c0, float& c1)
{
    const float u0 = hi ? t1 : t0, u1 = lo ? t0 : t1;
    const float u0n = shl1(u0);
    c0 = r ? u1 : u0;
    c1 = r ? u0n : u1;
}

// the resampled value and its x, y, z derivatives at positions 2l, 2l + 1
struct Resampled {
    float i[2], x[2], y[2], z[2];
};

template <typename T>
__device__ __forceinline__ void resample_step(Resampled& o, __amdgpu_buffer_rsrc_t rs, const StencilS& S, int E, int r,
                                              int n, int lane, int dp)
{
    const int m = E + kOutPerStep2 * n + 2 * lane;
    const uint32_t voff = (uint32_t)clampi(m, 0, dp - 2) * esize<T>::v;
    float q0[16], q1[16];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) ld2<T>(rs, voff, S.roff[b] + S.coff[a], q0[b * 4 + a], q1[b * 4 + a]);
    const bool lo = m < 0, hi = m > dp - 2;
    float v0, vx0, vy0, v1, vx1, vy1;
    blend3(q0, S, v0, vx0, vy0);
    blend3(q1, S, v1, vx1, vy1);
    float c0, c1;
    grid2(v0, v1, lo, hi, r, c0, c1);
    {
        const float c0n = shl1(c0), c1n = shl1(c1), c0nn = shl1(c0n);
        o.i[0] = S.wz[0] * c0 + S.wz[1] * c1 + S.wz[2] * c0n + S.wz[3] * c1n;
        o.i[1] = S.wz[0] * c1 + S.wz[1] * c0n + S.wz[2] * c1n + S.wz[3] * c0nn;
        o.z[0] = S.dwz[0] * c0 + S.dwz[1] * c1 + S.dwz[2] * c0n + S.dwz[3] * c1n;
        o.z[1] = S.dwz[0] * c1 + S.dwz[1] * c0n + S.dwz[2] * c1n + S.dwz[3] * c0nn;
    }
    grid2(vx0, vx1, lo, hi, r, c0, c1);
    {
        const float c0n = shl1(c0), c1n = shl1(c1), c0nn = shl1(c0n);
        o.x[0] = S.wz[0] * c0 + S.wz[1] * c1 + S.wz[2] * c0n + S.wz[3] * c1n;
        o.x[1] = S.wz[0] * c1 + S.wz[1] * c0n + S.wz[2] * c1n + S.wz[3] * c0nn;
    }
    grid2(vy0, vy1, lo, hi, r, c0, c1);
    {
        const float c0n = shl1(c0), c1n = shl1(c1), c0nn = shl1(c0n);
        o.y[0] = S.wz[0] * c0 + S.wz[1] * c1 + S.wz[2] * c0n + S.wz[3] * c1n;
        o.y[1] = S.wz[0] * c1 + S.wz[1] * c0n + S.wz[2] * c1n + S.wz[3] * c0nn;
    }
}

template <int N>
struct StructMultiJob {
    const void* vol[N];            // storage-type volumes of this level, [h][w][dp]
    const float* disp;             // [N][h][w][3]
    float* part[N * (N - 1) / 2];  // per pair (P, Q), P < Q in lexicographic order: [na][8]
    int w, h, d, na;
    int dp;                        // storage pitch (d, or d + 1 for an odd depth in 16-bit storage)
    uint32_t vol_bytes;
    float eps_h;
    const int* skip;  // device flag: when nonzero the launch does nothing (may be null)
};

template <typename T, int N>
__global__ __launch_bounds__(256) void k_struct_multi(const StructMultiJob<N> J)
{
    if (J.skip && *J.skip) return;
    constexpr int NP = N * (N - 1) / 2;
    const int wv = uni((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int w = J.w, h = J.h, d = J.d, dp = J.dp;
    // 2 x 2 tiles in 8 bands of tile rows, swept column by column (as k_struct2)
    const int tpr = (w + 1) >> 1;
    const int trows = (h + 1) >> 1;
    const int rpb = (trows + 7) >> 3;
    const int band = lb / (rpb * tpr), tb = lb - band * (rpb * tpr);
    const int trow = band * rpb + tb % rpb;
    if (lb >= 8 * rpb * tpr || trow >= trows) return;  // whole block
    const int i = 2 * (tb / rpb) + (wv & 1);
    const int j = 2 * trow + (wv >> 1);
    if (i >= w || j >= h) return;  // whole wave
    const int a = uni(j * w + i);
    StencilS S[N];
    __amdgpu_buffer_rsrc_t rs[N];
#pragma unroll
    for (int V = 0; V < N; ++V) {
        const float* dv = J.disp + ((size_t)V * J.na + a) * 3;
        make_stencil_s<T>(S[V], i, j, dv[0], dv[1], dv[2], w, h, dp);
        rs[V] = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(J.vol[V]), (short)0, (int)J.vol_bytes, kRsrcWord3);
    }
    // output grid: position 0 of step 0 holds sample base_0 - s0 of volume 0
    const int s0 = S[0].base & 1;
    int r[N], E[N];
#pragma unroll
    for (int V = 0; V < N; ++V) {
        r[V] = uni((S[V].base - s0) & 1);
        E[V] = S[V].base - s0 - r[V];  // even
    }
    const float eps = J.eps_h;
    const float inv_eps = 1.0f / J.eps_h;
    float acc[NP][7];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[q][c] = 0.f;
    const int nsteps = (d + kOutPerStep2 - 1) / kOutPerStep2;
    for (int n = 0; n < nsteps; ++n) {
        Resampled R[N];
#pragma unroll
        for (int V = 0; V < N; ++V) resample_step<T>(R[V], rs[V], S[V], E[V], r[V], n, lane, dp);
        const int p0 = 2 * lane;
        const int o0 = kOutPerStep2 * n + p0 - s0;
        const bool ok[2] = {p0 >= s0 && p0 <= 121 + s0 && o0 < d, p0 + 1 <= 121 + s0 && o0 + 1 < d};
        int q = 0;
#pragma unroll
        for (int P = 0; P < N; ++P)
#pragma unroll
            for (int Q = P + 1; Q < N; ++Q, ++q) {
                float L[2], G[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float u = (R[P].i[e] - R[Q].i[e]) * inv_eps, uu = u * u;
                    const float rsq = __builtin_amdgcn_rsqf(1.f + uu), sq = (1.f + uu) * rsq;
                    L[e] = ok[e] ? eps * uu * __builtin_amdgcn_rcpf(sq + 1.f) : 0.f;
                    G[e] = ok[e] ? u * rsq : 0.f;
                }
                acc[q][0] += L[0] + L[1];
                acc[q][1] += G[0] * R[P].x[0] + G[1] * R[P].x[1];
                acc[q][2] += G[0] * R[P].y[0] + G[1] * R[P].y[1];
                acc[q][3] += G[0] * R[P].z[0] + G[1] * R[P].z[1];
                acc[q][4] += G[0] * R[Q].x[0] + G[1] * R[Q].x[1];
                acc[q][5] += G[0] * R[Q].y[0] + G[1] * R[Q].y[1];
                acc[q][6] += G[0] * R[Q].z[0] + G[1] * R[Q].z[1];
            }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        float v[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = wave_sum_last(acc[q][c]);
        if (lane == 63) {
            float4* o = reinterpret_cast<float4*>(J.part[q] + (size_t)a * 8);
            o[0] = make_float4(v[0], v[1], v[2], v[3]);
            o[1] = make_float4(v[4], v[5], v[6], 0.f);
        }
    }
}

// The same pass for float32 storage (any depth): one sample per lane, lane l
// holding source sample base_V + 61 n + l of volume V, as in k_struct; the
// depth interpolation of output lane l (< 61) reads source lanes l .. l + 3,
// and taps outside the A-scan take the edge sample (clamped load index).
// Three waves per SIMD (at most 168 registers): for n = 4 that spills a few
// values (six scratch accesses per step) and measured 4 % faster than two.
template <int N>
__global__ __launch_bounds__(256, 3) void k_struct_multi1(const StructMultiJob<N> J)
{
    if (J.skip && *J.skip) return;
    constexpr int NP = N * (N - 1) / 2;
    const int wv = uni((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int w = J.w, h = J.h, d = J.d;
    const int tpr = (w + 1) >> 1;
    const int trows = (h + 1) >> 1;
    const int rpb = (trows + 7) >> 3;
    const int band = lb / (rpb * tpr), tb = lb - band * (rpb * tpr);
    const int trow = band * rpb + tb % rpb;
    if (lb >= 8 * rpb * tpr || trow >= trows) return;  // whole block
    const int i = 2 * (tb / rpb) + (wv & 1);
    const int j = 2 * trow + (wv >> 1);
    if (i >= w || j >= h) return;  // whole wave
    const int a = uni(j * w + i);
    StencilS S[N];
    __amdgpu_buffer_rsrc_t rs[N];
#pragma unroll
    for (int V = 0; V < N; ++V) {
        const float* dv = J.disp + ((size_t)V * J.na + a) * 3;
        make_stencil_s<float>(S[V], i, j, dv[0], dv[1], dv[2], w, h, d);
        rs[V] = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(J.vol[V]), (short)0, (int)J.vol_bytes, kRsrcWord3);
    }
    const float eps = J.eps_h;
    const float inv_eps = 1.0f / J.eps_h;
    float acc[NP][7];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[q][c] = 0.f;
    const int nsteps = (d + kOutPerStep - 1) / kOutPerStep;
    for (int n = 0; n < nsteps; ++n) {
        float I[N], X[N], Y[N], Z[N];
#pragma unroll
        for (int V = 0; V < N; ++V) {
            const uint32_t voff = (uint32_t)clampi(S[V].base + kOutPerStep * n + lane, 0, d - 1) * 4u;
            float c[16];
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int a2 = 0; a2 < 4; ++a2) c[b * 4 + a2] = ldv<float>(rs[V], voff, S[V].roff[b] + S[V].coff[a2]);
            float v, vx, vy;
            blend3(c, S[V], v, vx, vy);
            float iv = 0.f, iz = 0.f, ix = 0.f, iy = 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                iv = fmaf(S[V].wz[e], v, iv);
                iz = fmaf(S[V].dwz[e], v, iz);
                ix = fmaf(S[V].wz[e], vx, ix);
                iy = fmaf(S[V].wz[e], vy, iy);
                if (e < 3) {
                    v = shl1(v);
                    vx = shl1(vx);
                    vy = shl1(vy);
                }
            }
            I[V] = iv;
            X[V] = ix;
            Y[V] = iy;
            Z[V] = iz;
            // one volume's loads in flight at a time: hoisting all of them
            // would take 64 more registers (one wave per SIMD)
            __builtin_amdgcn_sched_barrier(0);
        }
        const bool ok = lane < kOutPerStep && n * kOutPerStep + lane < d;
        int q = 0;
#pragma unroll
        for (int P = 0; P < N; ++P)
#pragma unroll
            for (int Q = P + 1; Q < N; ++Q, ++q) {
                const float u = (I[P] - I[Q]) * inv_eps, uu = u * u;
                const float rsq = __builtin_amdgcn_rsqf(1.f + uu), sq = (1.f + uu) * rsq;
                const float L = ok ? eps * uu * __builtin_amdgcn_rcpf(sq + 1.f) : 0.f;
                const float G = ok ? u * rsq : 0.f;
                acc[q][0] += L;
                acc[q][1] = fmaf(G, X[P], acc[q][1]);
                acc[q][2] = fmaf(G, Y[P], acc[q][2]);
                acc[q][3] = fmaf(G, Z[P], acc[q][3]);
                acc[q][4] = fmaf(G, X[Q], acc[q][4]);
                acc[q][5] = fmaf(G, Y[Q], acc[q][5]);
                acc[q][6] = fmaf(G, Z[Q], acc[q][6]);
            }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        float v[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = wave_sum_last(acc[q][c]);
        if (lane == 63) {
            float4* o = reinterpret_cast<float4*>(J.part[q] + (size_t)a * 8);
            o[0] = make_float4(v[0], v[1], v[2], v[3]);
            o[1] = make_float4(v[4], v[5], v[6], 0.f);
        }
    }
}

}  // namespace

hipError_t launch_sum(const SumJobs& jobs, int total_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum, dim3(total_blocks), dim3(kRedBlock), 0, s, jobs);
    return hipGetLastError();
}

template <typename T, bool AXIAL>
static hipError_t launch_struct_subsets(const StructJobs& jobs, hipStream_t s)
{
    // 16-bit storage: two samples per lane for the jobs whose storage pitch
    // is even (every level of a pair: an odd depth is stored with one padding
    // sample); an odd pitch (volumes in the caller's layout with an odd depth)
    // keeps one sample per lane, since its sample pairs would not all be
    // 32-bit aligned.  The kernel is chosen per job, so a job's result does not
    // depend on the other jobs of its launch; each subset has its own grid (a
    // multiple of the 8 XCDs).
    StructJobs even{}, odd{};
    even.skip = odd.skip = jobs.skip;
    int be = 0, bo = 0;
    for (int q = 0; q < jobs.n; ++q) {
        StructJob J = jobs.j[q];
        const int nb = struct_blocks(J.w, J.h);
        if (J.dp % 2 == 0) {
            J.blk_begin = be;
            be += nb;
            even.j[even.n++] = J;
        } else {
            J.blk_begin = bo;
            bo += nb;
            odd.j[odd.n++] = J;
        }
    }
    if (even.n) hipLaunchKernelGGL((k_struct2<T, AXIAL>), dim3((be + 7) / 8 * 8), dim3(256), 0, s, even);
    if (odd.n) hipLaunchKernelGGL((k_struct<T, AXIAL>), dim3((bo + 7) / 8 * 8), dim3(256), 0, s, odd);
    return hipGetLastError();
}

template <bool AXIAL>
static hipError_t launch_struct_t(const StructJobs& jobs, int total_blocks, octmc_dtype dt, hipStream_t s)
{
    switch (dt) {
    case OCTMC_F32:
        hipLaunchKernelGGL((k_struct<float, AXIAL>), dim3(total_blocks), dim3(256), 0, s, jobs);
        return hipGetLastError();
    case OCTMC_BF16:
        return launch_struct_subsets<bf16_t, AXIAL>(jobs, s);
    case OCTMC_F16:
        return launch_struct_subsets<f16_t, AXIAL>(jobs, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_struct(const StructJobs& jobs, int total_blocks, octmc_dtype dt, hipStream_t s, bool axial)
{
    return axial ? launch_struct_t<true>(jobs, total_blocks, dt, s) : launch_struct_t<false>(jobs, total_blocks, dt, s);
}

hipError_t launch_combine(const CombineJobs& jobs, int total_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_combine, dim3(total_blocks), dim3(kRedBlock), 0, s, jobs);
    hipLaunchKernelGGL(k_finalize, dim3(jobs.n), dim3(kRedBlock), 0, s, jobs);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_struct_multi_n(const void* const* vol, const float* disp, float* const* part, int w, int h,
                                        int d, int dp, uint32_t vol_bytes, float eps_h, octmc_dtype dt,
                                        hipStream_t s, const int* skip)
{
    StructMultiJob<N> J{};
    J.skip = skip;
    for (int V = 0; V < N; ++V) J.vol[V] = vol[V];
    for (int q = 0; q < N * (N - 1) / 2; ++q) J.part[q] = part[q];
    J.disp = disp;
    J.w = w;
    J.h = h;
    J.d = d;
    J.dp = dp;
    J.na = w * h;
    J.vol_bytes = vol_bytes;
    J.eps_h = eps_h;
    const int blocks = (struct_blocks(w, h) + 7) / 8 * 8;  // a multiple of the 8 XCDs
    if (dt == OCTMC_F32)
        hipLaunchKernelGGL((k_struct_multi1<N>), dim3(blocks), dim3(256), 0, s, J);
    else if (dt == OCTMC_BF16)
        hipLaunchKernelGGL((k_struct_multi<bf16_t, N>), dim3(blocks), dim3(256), 0, s, J);
    else
        hipLaunchKernelGGL((k_struct_multi<f16_t, N>), dim3(blocks), dim3(256), 0, s, J);
    return hipGetLastError();
}

bool struct_multi_supported(int n, int dp, octmc_dtype dt)
{
    // 16-bit storage holds two samples per lane, which needs an even pitch
    // (every level the n-volume path stores: odd depths are padded)
    return (n == 3 || n == 4) && (dt == OCTMC_F32 || ((dt == OCTMC_BF16 || dt == OCTMC_F16) && dp % 2 == 0));
}

hipError_t launch_struct_multi(const void* const* vol, int n, const float* disp, float* const* part, int w, int h,
                               int d, int dp, uint32_t vol_bytes, float eps_h, octmc_dtype dt, hipStream_t s,
                               const int* skip)
{
    if (!struct_multi_supported(n, dp, dt) || (dt == OCTMC_F32 && dp != d)) return hipErrorInvalidValue;
    if (n == 3) return launch_struct_multi_n<3>(vol, disp, part, w, h, d, dp, vol_bytes, eps_h, dt, s, skip);
    return launch_struct_multi_n<4>(vol, disp, part, w, h, d, dp, vol_bytes, eps_h, dt, s, skip);
}

}  // namespace octmc
