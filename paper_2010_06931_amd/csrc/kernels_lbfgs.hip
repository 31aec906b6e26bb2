// Vector kernels of the L-BFGS solve (float64 state on the device).
//
//   k_multidot  several dot products (and one max |.|) in one pass, block
//               partials; k_multidot_final sums them in a fixed order
//   k_lincomb   out = sum_q c_q v_q (search direction from the compact
//               representation of the L-BFGS matrix)
//   k_trial     x_t = x + alpha p, also as float32 for the evaluation
//   k_accept    s = x_t - x, y = g_t - g, then x = x_t, g = g_t
//
// and the controllers of the iteration with its decisions on the device
// (k_lb_*): single-thread kernels that take the host solver's decisions in the
// same float64 operations (FMA contraction off), and predicated forms of the
// vector kernels above.
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

// The pending accept of the device solver (LB): when st->do_accept is set,
// the step found by the previous iteration's line search is committed here,
// element by element, before the products use the new values: s_c = x_t - x,
// y_c = g_t - g into vec[1], vec[2], then x = x_t, g = g_t (the arithmetic of
// k_accept).
struct LbAccept {
    double* x;
    const double* xt;
    const double* gt;
};

// LB: the device solver's form: the vectors' addresses come from its table
// st->vec (vector 0 the gradient, 1 and 2 the candidate pair), the launch does
// nothing when st->skip_iter is set, and the pending accept is done first.
template <bool LB>
__global__ __launch_bounds__(kB) void k_multidot_keyed(const KeyedDots spec, const LbState* __restrict__ st,
                                                       const LbAccept acc, size_t n, double* __restrict__ blk)
{
    bool accept = false;
    if constexpr (LB) {
        if (st->skip_iter) return;
        accept = st->do_accept != 0;  // uniform
    }
    const int nv = spec.nv;
    const bool two = spec.key1 >= 0;
    double* vp[kMaxDotVecs];
#pragma unroll
    for (int v = 0; v < kMaxDotVecs; ++v)
        vp[v] = LB ? (v < nv ? st->vec[v] : nullptr) : const_cast<double*>(spec.v[v]);
    double acc0[kMaxDotVecs], acc1[kMaxDotVecs];
#pragma unroll
    for (int v = 0; v < kMaxDotVecs; ++v) acc0[v] = acc1[v] = 0.0;
    double gmax = 0.0;
    for (size_t t = (size_t)blockIdx.x * kB + threadIdx.x; t < n; t += (size_t)gridDim.x * kB) {
        double x[kMaxDotVecs];
#pragma unroll
        for (int v = 0; v < kMaxDotVecs; ++v) x[v] = v < nv && !(accept && (v == 1 || v == 2)) ? vp[v][t] : 0.0;
        if (LB && accept) {
            const double xn = acc.xt[t], gn = acc.gt[t];
            const double sv = xn - acc.x[t], yv = gn - x[0];
            vp[1][t] = sv;
            vp[2][t] = yv;
            acc.x[t] = xn;
            vp[0][t] = gn;
            x[0] = gn;
            x[1] = sv;
            x[2] = yv;
        }
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

// rows q of the final sums, dealt to the block's waves (nthreads / 64)
__device__ __forceinline__ void final_rows(int nrow, int gmax_row, int nblk, const RowMap& map,
                                           const double* __restrict__ blk, double* out, int nthreads)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int per = (nblk + 63) / 64;
    for (int q = wv; q < nrow; q += nthreads / 64) {
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

__global__ __launch_bounds__(kFinalThreads) void k_multidot_final(int nrow, int gmax_row, int nblk, const RowMap map,
                                                                  const double* __restrict__ blk,
                                                                  double* __restrict__ out)
{
    final_rows(nrow, gmax_row, nblk, map, blk, out, kFinalThreads);
}

__global__ void k_lincomb(const CombSpec spec, size_t n, double* __restrict__ out)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < spec.nv; ++q) s = fma(spec.c[q], spec.v[q][t], s);
        out[t] = s;
    }
}

__global__ void k_trial(const double* __restrict__ x, const double* __restrict__ p, double alpha, size_t n,
                        double* __restrict__ xt, float* __restrict__ xt32)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double v = fma(alpha, p[t], x[t]);
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

namespace {

// The keyed form of a set of products when every product has the max vector
// or one other vector as a factor; false otherwise.  map.row[q] is the partial
// row of output q.
bool keyed_plan(const DotSpec& spec, KeyedDots& kd, RowMap& map)
{
    const int nd = spec.ndots;
    int nv = 0;
    for (int q = 0; q < nd; ++q) nv = std::max(nv, std::max((int)spec.a[q], (int)spec.b[q]) + 1);
    if (spec.gmax_vec < 0 || nv > kMaxDotVecs) return false;
    kd = KeyedDots{};
    map = RowMap{};
    kd.nv = std::max(nv, spec.gmax_vec + 1);
    kd.key0 = spec.gmax_vec;
    kd.key1 = -1;
    kd.gmax = 1;
    for (int q = 0; q < nd; ++q) {
        const int a = spec.a[q], b = spec.b[q];
        int which, other;
        if (b == kd.key0) which = 0, other = a;
        else if (a == kd.key0) which = 0, other = b;
        else {
            if (kd.key1 < 0) kd.key1 = b;
            if (b == kd.key1) which = 1, other = a;
            else if (a == kd.key1) which = 1, other = b;
            else return false;
        }
        map.row[q] = (unsigned char)(which * kMaxDotVecs + other);
    }
    map.row[nd] = (unsigned char)(2 * kMaxDotVecs);
    for (int v = 0; v < kd.nv; ++v) kd.v[v] = spec.v[v];
    return true;
}

}  // namespace

hipError_t launch_multidot(const DotSpec& spec, size_t n, double* blk, double* out, hipStream_t s)
{
    const int nd = spec.ndots;
    if (nd > kMaxDots) return hipErrorInvalidValue;
    const int nb = grid_for(n, kMaxBlocks);
    KeyedDots kd;
    RowMap map;
    if (keyed_plan(spec, kd, map)) {
        hipLaunchKernelGGL(k_multidot_keyed<false>, dim3(nb), dim3(kB), 0, s, kd, nullptr, LbAccept{}, n, blk);
    } else {
        map = RowMap{};
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


// ===========================================================================
// The iteration with its decisions on the device.  The controllers follow
// LevelRun::run step for step (the same tests, the same float64 expressions
// in the same order, FMA contraction off), so that the two forms give the
// same iterates bit for bit.  Each controller launch reads the whole state
// (and its inputs) into LDS with all its lanes in one round of loads, takes
// the decisions on one lane, and writes the state back with all lanes: its
// cost is then about two memory round trips rather than one per dependent
// field.

namespace {

constexpr int M = kLbMaxM;
static_assert(sizeof(LbState) % 8 == 0 && alignof(LbState) == 8, "the state moves as 64-bit words");
constexpr int kLbWords = (int)(sizeof(LbState) / 8);

__device__ __forceinline__ void state_in(LbState& S, const LbState* st, int nthreads)
{
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(st);
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(&S);
    for (int w = threadIdx.x; w < kLbWords; w += nthreads) dst[w] = src[w];
}
__device__ __forceinline__ void state_out(LbState* st, const LbState& S, int nthreads)
{
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(&S);
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(st);
    for (int w = threadIdx.x; w < kLbWords; w += nthreads) dst[w] = src[w];
}

__device__ __forceinline__ void lb_stop(LbState* st, int status)
{
    st->h.status = status;
    st->skip_iter = 1;
    st->skip_trial = 1;
}

__global__ __launch_bounds__(64) void k_lb_init(LbState* __restrict__ st, const LbInit in,
                                                const double* __restrict__ terms)
{
    if (threadIdx.x != 0) return;
    const double f = terms[OCTMC_TERM_F];
    st->h.status = in.iters_max > 0 ? 0 : 3;
    st->h.stall = 0;
    st->h.it = 0;
    st->h.evals = 1;
    st->h.ls_done = 0;
    st->h.ls_ok = 0;
    st->h.f = f;
    st->h.f_start = f;
    st->skip_iter = st->h.status != 0;
    st->skip_trial = 1;
    st->do_accept = 0;
    st->resume = 0;
    st->m = in.m;
    st->count = 0;
    st->has_cand = 0;
    st->iters_max = in.iters_max;
    st->ls_max_evals = in.ls_max_evals;
    st->ls_phase = 0;
    st->ls_i = 0;
    st->ls_start = 0;
    st->ncomb = 0;
    st->c1 = in.c1;
    st->c2 = in.c2;
    for (int v = 0; v < 3 + 2 * M; ++v) st->vec[v] = in.vec[v];
    for (int k = 0; k < M; ++k)
        for (int l = 0; l < M; ++l) st->SY[k][l] = st->YY[k][l] = 0.0;
}

// After the iteration's dot products: the candidate pair enters the history
// when it passes the curvature test, the gradient test, then the search
// direction from the compact form and the start of the line search.  The dot
// products are by position: 0 g.g; 1+k S_k.g; 1+m+k Y_k.g; 1+2m+k S_k.y_c;
// 1+3m+k y_c.Y_k; 1+4m s_c.g; 2+4m y_c.g; 3+4m s_c.y_c; 4+4m y_c.y_c; 5+4m
// max |g|.  Every array is indexed by unrolled constants only.
__device__ __forceinline__ void c1_decide(LbState* st, const double* dots)
{
#pragma clang fp contract(off)
    if (st->skip_iter) return;  // a pending accept is left to the level's last accept
    st->do_accept = 0;          // the dot-product pass has committed the pending accept
    if (st->h.it >= st->iters_max) {
        lb_stop(st, 3);
        return;
    }
    const int m = st->m;
    int c = st->count;
    const double gg = dots[0], gmax = dots[5 + 4 * m];
    // the history's products are updated in place (st is the launch's LDS copy)
    double(&SY)[M][M] = st->SY;
    double(&YY)[M][M] = st->YY;
    double a_s[M], b_y[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        a_s[k] = k < c ? dots[1 + k] : 0.0;
        b_y[k] = k < c ? dots[1 + m + k] : 0.0;
    }
    if (st->has_cand) {
        const double sy = dots[3 + 4 * m], yy = dots[4 + 4 * m];
        if (sy > 1e-12 * yy && yy > 0) {
            double syc[M], ycy[M];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                syc[k] = k < c ? dots[1 + 2 * m + k] : 0.0;
                ycy[k] = k < c ? dots[1 + 3 * m + k] : 0.0;
            }
            double** vec = st->vec;
            if (c == m) {  // the oldest pair leaves; its buffers take the next candidate
                double* os = vec[3];
                double* oy = vec[3 + m];
                for (int k = 0; k + 1 < m; ++k) {
                    vec[3 + k] = vec[4 + k];
                    vec[3 + m + k] = vec[4 + m + k];
                }
                vec[2 + m] = vec[1];
                vec[2 + 2 * m] = vec[2];
                vec[1] = os;
                vec[2] = oy;
#pragma unroll
                for (int k = 0; k + 1 < M; ++k) {
#pragma unroll
                    for (int l = 0; l + 1 < M; ++l) {
                        SY[k][l] = SY[k + 1][l + 1];
                        YY[k][l] = YY[k + 1][l + 1];
                    }
                    a_s[k] = a_s[k + 1];
                    b_y[k] = b_y[k + 1];
                    syc[k] = syc[k + 1];
                    ycy[k] = ycy[k + 1];
                }
                c = m - 1;
            } else {
                double* t = vec[3 + c];
                vec[3 + c] = vec[1];
                vec[1] = t;
                t = vec[3 + m + c];
                vec[3 + m + c] = vec[2];
                vec[2] = t;
            }
            const double csg = dots[1 + 4 * m], cyg = dots[2 + 4 * m];
#pragma unroll
            for (int p = 0; p < M; ++p) {
                if (p == c) {
#pragma unroll
                    for (int k = 0; k < p; ++k) {
                        SY[k][p] = syc[k];
                        YY[k][p] = ycy[k];
                        YY[p][k] = ycy[k];
                    }
                    SY[p][p] = sy;
                    YY[p][p] = yy;
                    a_s[p] = csg;
                    b_y[p] = cyg;
                }
            }
            c += 1;
        }
        st->has_cand = 0;
    }
    const double f = st->h.f;
    const double af = fabs(f);
    if (gmax <= 1e-10 * (1.0 < af ? af : 1.0)) {
        st->count = c;
        lb_stop(st, 1);
        return;
    }
    double c_g, gp;
    double cs[M], cy[M];
#pragma unroll
    for (int k = 0; k < M; ++k) cs[k] = cy[k] = 0.0;
    if (c > 0) {
        // H g = gamma g + S u + gamma Y v with v = -R^-1 a and
        // u = R^-T ((D + gamma Y'Y) R^-1 a - gamma b), R = upper(S'Y)
        double gamma = 0.0;
#pragma unroll
        for (int p = 0; p < M; ++p)
            if (p == c - 1) gamma = SY[p][p] / YY[p][p];
        double t1[M], u[M];
#pragma unroll
        for (int k = M - 1; k >= 0; --k) {  // R t1 = a
            t1[k] = 0.0;
            if (k < c) {
                double v = a_s[k];
#pragma unroll
                for (int l = k + 1; l < M; ++l)
                    if (l < c) v -= SY[k][l] * t1[l];
                t1[k] = v / SY[k][k];
            }
        }
#pragma unroll
        for (int k = 0; k < M; ++k) {  // R' u = (D + gamma Y'Y) t1 - gamma b
            u[k] = 0.0;
            if (k < c) {
                double v = SY[k][k] * t1[k];
#pragma unroll
                for (int l = 0; l < M; ++l)
                    if (l < c) v += gamma * YY[k][l] * t1[l];
                v = v - gamma * b_y[k];
#pragma unroll
                for (int l = 0; l < k; ++l) v -= SY[l][k] * u[l];
                u[k] = v / SY[k][k];
            }
        }
        c_g = -gamma;
        double hg = gamma * gg;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            if (k < c) {
                cs[k] = -u[k];
                cy[k] = gamma * t1[k];
                hg += u[k] * a_s[k] - gamma * t1[k] * b_y[k];
            }
        }
        gp = -hg;
    }
    if (c == 0 || !(gp < 0)) {  // steepest descent (no memory, or not a descent direction: the memory is dropped)
        c = 0;
        c_g = -1.0 / gmax;
        gp = -gg / gmax;
    }
    st->count = c;
    st->ncomb = c;
    st->c_g = c_g;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        st->c_s[k] = cs[k];
        st->c_y[k] = cy[k];
    }
    st->gp = gp;
    st->ls_phase = 0;
    st->ls_i = 1;
    st->ls_start = st->h.evals;
    st->a_try = 1.0;
    st->a_prev = 0.0;
    st->f_prev = f;
    st->g_prev = gp;
    st->f0 = f;
    st->g0 = gp;
    st->h.ls_done = 0;
    st->h.ls_ok = 0;
    st->skip_trial = 0;
}

// The final sums of the iteration's dot products (as k_multidot_final forms
// them), then c1_decide.
__global__ __launch_bounds__(kFinalThreads) void k_lb_c1(LbState* __restrict__ st, int nd, int nblk,
                                                         const RowMap map, const double* __restrict__ blk)
{
    __shared__ LbState S;
    __shared__ double dots[kMaxDots + 1];
    state_in(S, st, kFinalThreads);
    final_rows(nd + 1, nd, nblk, map, blk, dots, kFinalThreads);
    __syncthreads();
    if (threadIdx.x == 0) c1_decide(&S, dots);
    __syncthreads();
    state_out(st, S, kFinalThreads);
}

// The search direction and the first trial point x + p (a_try = 1 after
// c1_decide), each term in the order of k_lincomb and k_trial.
__global__ void k_lb_lincomb(const LbState* __restrict__ st, const double* __restrict__ x, size_t n,
                             double* __restrict__ out, double* __restrict__ xt, float* __restrict__ xt32)
{
    if (st->skip_iter) return;
    const int nc = st->ncomb, m = st->m;
    const double* g = st->vec[0];
    const double cg = st->c_g, alpha = st->a_try;
    const double* sp[M];
    const double* yp[M];
    double cs[M], cy[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        sp[k] = k < nc ? st->vec[3 + k] : nullptr;
        yp[k] = k < nc ? st->vec[3 + m + k] : nullptr;
        cs[k] = st->c_s[k];
        cy[k] = st->c_y[k];
    }
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        double s = fma(cg, g[t], 0.0);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            if (k < nc) {  // uniform
                s = fma(cs[k], sp[k][t], s);
                s = fma(cy[k], yp[k][t], s);
            }
        }
        out[t] = s;
        const double v = fma(alpha, s, x[t]);
        xt[t] = v;
        xt32[t] = (float)v;
    }
}

__global__ void k_lb_trial(const LbState* __restrict__ st, const double* __restrict__ x, const double* __restrict__ p,
                           size_t n, double* __restrict__ xt, float* __restrict__ xt32)
{
    if (st->skip_trial) return;
    const double alpha = st->a_try;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double v = fma(alpha, p[t], x[t]);
        xt[t] = v;
        xt32[t] = (float)v;
    }
}

// After a trial evaluation: one step of the strong Wolfe line search
// (bracketing, then zoom with the safeguarded cubic step).
__device__ __forceinline__ void c2_decide(LbState* st, double fa, double ga, int last)
{
#pragma clang fp contract(off)
    if (st->skip_trial) return;
    const double a = st->a_try, f0 = st->f0, g0 = st->g0, c1 = st->c1, c2 = st->c2;
    st->h.evals += 1;
    bool ok = false;
    if (st->ls_phase == 0) {
        if (fa > f0 + c1 * a * g0 || (st->ls_i > 1 && fa >= st->f_prev)) {
            st->lo = st->a_prev;
            st->flo = st->f_prev;
            st->glo = st->g_prev;
            st->hi = a;
            st->fhi = fa;
            st->ghi = ga;
            st->ls_phase = 1;
        } else if (fabs(ga) <= -c2 * g0) {
            ok = true;
        } else if (ga >= 0) {
            st->hi = st->a_prev;
            st->fhi = st->f_prev;
            st->ghi = st->g_prev;
            st->lo = a;
            st->flo = fa;
            st->glo = ga;
            st->ls_phase = 1;
        } else {
            st->a_prev = a;
            st->f_prev = fa;
            st->g_prev = ga;
            st->a_try = 2.0 * a;
            st->ls_i += 1;
        }
    } else {
        if (fa > f0 + c1 * a * g0 || fa >= st->flo) {
            st->hi = a;
            st->fhi = fa;
            st->ghi = ga;
        } else if (fabs(ga) <= -c2 * g0) {
            ok = true;
        } else {
            if (ga * (st->hi - st->lo) >= 0) {
                st->hi = st->lo;
                st->fhi = st->flo;
                st->ghi = st->glo;
            }
            st->lo = a;
            st->flo = fa;
            st->glo = ga;
        }
    }
    if (ok) {
        st->h.ls_done = 1;
        st->h.ls_ok = 1;
        st->do_accept = 1;
        st->has_cand = 1;
        st->h.f = fa;
        st->h.it += 1;
        st->skip_trial = 1;
        if (st->h.it >= st->iters_max) lb_stop(st, 3);
        return;
    }
    if (st->h.evals - st->ls_start >= st->ls_max_evals) {
        st->h.ls_done = 1;
        lb_stop(st, 2);
        return;
    }
    if (st->ls_phase == 1) st->a_try = cubic_min(st->lo, st->flo, st->glo, st->hi, st->fhi, st->ghi);
    if (last && !st->resume) {
        st->h.stall = 1;
        st->skip_iter = 1;
        st->skip_trial = 1;
    }
}

__global__ __launch_bounds__(64) void k_lb_c2(LbState* __restrict__ st, const double* __restrict__ terms, int last)
{
    __shared__ LbState S;
    __shared__ double fg[2];
    state_in(S, st, 64);
    if (threadIdx.x == 0) fg[0] = terms[OCTMC_TERM_F];
    if (threadIdx.x == 1) fg[1] = terms[OCTMC_TERM_GP];
    __syncthreads();
    const bool run = !S.skip_trial;  // uniform
    if (threadIdx.x == 0) c2_decide(&S, fg[0], fg[1], last);
    __syncthreads();
    if (run) state_out(st, S, 64);
}

__global__ void k_lb_accept(const LbState* __restrict__ st, double* __restrict__ x, double* __restrict__ g,
                            const double* __restrict__ xt, const double* __restrict__ gt, size_t n)
{
    if (!st->do_accept) return;
    double* s_out = st->vec[1];
    double* y_out = st->vec[2];
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double xn = xt[t], gn = gt[t];
        s_out[t] = xn - x[t];
        y_out[t] = gn - g[t];
        x[t] = xn;
        g[t] = gn;
    }
}

__global__ __launch_bounds__(64) void k_lb_resume(LbState* __restrict__ st, int resume)
{
    if (threadIdx.x != 0) return;
    if (resume) {
        st->h.stall = 0;
        st->resume = 1;
        st->skip_iter = 0;
        st->skip_trial = 0;
    } else {
        st->resume = 0;
        st->skip_iter = st->h.status != 0;
        st->skip_trial = 1;
    }
}

}  // namespace

hipError_t launch_lb_init(LbState* st, const LbInit& in, const double* terms, hipStream_t s)
{
    if (in.m < 1 || in.m > kLbMaxM) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lb_init, dim3(1), dim3(64), 0, s, st, in, terms);
    return hipGetLastError();
}
hipError_t launch_lb_head(LbState* st, int m, size_t n, double* blk, double* x, const double* gt, double* p,
                          double* xt, float* xt32, hipStream_t s)
{
    if (m < 1 || m > kLbMaxM) return hipErrorInvalidValue;
    // vectors 0 g, 1 s_c, 2 y_c, 3 + k S_k, 3 + m + k Y_k; the products in the
    // order c1_decide reads them
    DotSpec ds{};
    int nd = 0;
    auto dot = [&](int a, int b) {
        ds.a[nd] = (unsigned char)a;
        ds.b[nd] = (unsigned char)b;
        ++nd;
    };
    dot(0, 0);
    for (int k = 0; k < m; ++k) dot(3 + k, 0);
    for (int k = 0; k < m; ++k) dot(3 + m + k, 0);
    for (int k = 0; k < m; ++k) dot(3 + k, 2);
    for (int k = 0; k < m; ++k) dot(2, 3 + m + k);
    dot(1, 0);
    dot(2, 0);
    dot(1, 2);
    dot(2, 2);
    ds.ndots = nd;
    ds.gmax_vec = 0;
    for (int v = 0; v < 3 + 2 * m; ++v) ds.v[v] = nullptr;  // from the table
    KeyedDots kd;
    RowMap map;
    if (nd > kMaxDots || !keyed_plan(ds, kd, map) || kd.nv != 3 + 2 * m || kd.key1 != 2) return hipErrorInvalidValue;
    const int nb = grid_for(n, kMaxBlocks);
    hipLaunchKernelGGL(k_multidot_keyed<true>, dim3(nb), dim3(kB), 0, s, kd, st, LbAccept{x, xt, gt}, n, blk);
    hipLaunchKernelGGL(k_lb_c1, dim3(1), dim3(kFinalThreads), 0, s, st, nd, nb, map, blk);
    hipLaunchKernelGGL(k_lb_lincomb, dim3(grid_for(n)), dim3(256), 0, s, st, x, n, p, xt, xt32);
    return hipGetLastError();
}
hipError_t launch_lb_trial(const LbState* st, const double* x, const double* p, size_t n, double* xt, float* xt32,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_lb_trial, dim3(grid_for(n)), dim3(256), 0, s, st, x, p, n, xt, xt32);
    return hipGetLastError();
}
hipError_t launch_lb_c2(LbState* st, const double* terms, int last, hipStream_t s)
{
    hipLaunchKernelGGL(k_lb_c2, dim3(1), dim3(64), 0, s, st, terms, last);
    return hipGetLastError();
}
hipError_t launch_lb_accept(const LbState* st, double* x, double* g, const double* xt, const double* gt, size_t n,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_lb_accept, dim3(grid_for(n)), dim3(256), 0, s, st, x, g, xt, gt, n);
    return hipGetLastError();
}
hipError_t launch_lb_resume(LbState* st, int resume, hipStream_t s)
{
    hipLaunchKernelGGL(k_lb_resume, dim3(1), dim3(64), 0, s, st, resume);
    return hipGetLastError();
}

}  // namespace octmc
