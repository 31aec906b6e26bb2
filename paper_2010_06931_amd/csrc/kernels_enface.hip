// Segmentation-free en face OCTA projection (Sec. 2.3) for gfx950.
//
// Volumes are [h][w][d] float32 in the common frame (depth contiguous).  The
// fast scan axis is x for the X-fast scan (V = 0) and y for the Y-fast scan
// (V = 1); B-scans are rows j (V = 0) or columns i (V = 1).  Steps:
//   k_median3      3-D median of radius 1 (clamped borders)
//   k_rank15       width-15 rank filter keeping the 3rd smallest value, along
//                  one lateral axis (run for the fast, then the slow axis)
//   k_radix_hist   three radix passes (11, 11, 10 bits; the first counted by
//   k_radix_select the slow-axis rank filter) that select the two order
//                  statistics on each side of the 5th and 95th percentile
//                  of the filtered volume over the valid B-scans
//   k_noise_sum    mean and standard deviation of the OCT noise samples
//   k_mask_mean    both masks and the masked depth mean per A-scan
//   k_bscan_median per-B-scan median
//   k_enface_finish median subtraction and nearest-valid substitution
// Every selection (median, rank filter, order statistic) is made with min,
// max and median-of-three instructions on the float values themselves, so
// it is exact; the thresholds are formed in FP64 with the arithmetic order
// written out and no contraction.
#include <algorithm>
#include <cmath>

#include "octmc_internal.h"

namespace octmc {
namespace {

constexpr int kMedTile = 62;   // depth outputs per wave (64 lanes, one halo lane each side)
constexpr int kMedSeg = 30;    // x positions per wave, a multiple of 3
constexpr int kHistBins = 2048;
constexpr int kHistBlocks = 2048;
constexpr int kNoiseBlocks = 2048;
constexpr int kMaxBscan = 8192;  // A-scans per B-scan (LDS sort of the B-scan median)

__device__ __forceinline__ float shl1(float v)  // lane l gets lane l + 1 (lane 63 gets 0)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float shr1(float v)  // lane l gets lane l - 1 (lane 0 gets 0)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float min3f(float a, float b, float c) { return __builtin_fminf(__builtin_fminf(a, b), c); }
__device__ __forceinline__ float max3f(float a, float b, float c) { return __builtin_fmaxf(__builtin_fmaxf(a, b), c); }
__device__ __forceinline__ float med3f(float a, float b, float c) { return __builtin_amdgcn_fmed3f(a, b, c); }
__device__ __forceinline__ void sort3(float& a, float& b, float& c)
{
    const float lo = min3f(a, b, c), mi = med3f(a, b, c), hi = max3f(a, b, c);
    a = lo;
    b = mi;
    c = hi;
}
__device__ __forceinline__ void ce(float& a, float& b)
{
    const float lo = __builtin_fminf(a, b), hi = __builtin_fmaxf(a, b);
    a = lo;
    b = hi;
}

// ---------------------------------------------------------------------------
// 3-D median of radius 1.
//
// A wave owns one row j, 64 consecutive depths (62 outputs) and kMedSeg
// consecutive x positions, which it walks in order.  For each x it sorts the
// nine samples of the (j, k) plane at that x: the three rows j-1..j+1 are
// loaded and sorted per lane, the neighbours k-1 and k+1 come from the
// adjacent lanes, the three rank rows are sorted across k, and three more
// 3-sorts complete the order of this rows-and-columns-sorted 3 x 3 grid.
// With the three sorted planes A, B, C of x-1, x, x+1, sorting each rank m
// across the planes leaves a 3 x 9 grid sorted both ways; the element at
// (a, m) has at least (a+1)(m+1) samples at or below it and (3-a)(9-m) at
// or above it, which rules out 7 samples below and 7 above the median.  The
// median of the 27 is then the 7th smallest of the 13 remaining ones: the
// minima of ranks 5..8, the medians of ranks 2..6 and the maxima of ranks
// 0..3, three sorted lists.  The first and last are merged (Batcher), and
// the 7th smallest of that list X and the medians Y is min over r + s = 7
// of max(X_r, Y_s).
struct Plane {
    float v[9];
};

__device__ __forceinline__ Plane sorted_plane(const float* __restrict__ in, size_t rm, size_t r0, size_t rp, int x,
                                              int w, int d, int k)
{
    x = x < 0 ? 0 : (x >= w ? w - 1 : x);
    float a = in[(rm + x) * d + k], b = in[(r0 + x) * d + k], c = in[(rp + x) * d + k];
    sort3(a, b, c);
    Plane p;
    p.v[0] = shr1(a);
    p.v[1] = a;
    p.v[2] = shl1(a);
    p.v[3] = shr1(b);
    p.v[4] = b;
    p.v[5] = shl1(b);
    p.v[6] = shr1(c);
    p.v[7] = c;
    p.v[8] = shl1(c);
    sort3(p.v[0], p.v[1], p.v[2]);
    sort3(p.v[3], p.v[4], p.v[5]);
    sort3(p.v[6], p.v[7], p.v[8]);
    sort3(p.v[2], p.v[4], p.v[6]);
    sort3(p.v[1], p.v[2], p.v[3]);
    sort3(p.v[5], p.v[6], p.v[7]);
    return p;
}

__device__ __forceinline__ float median27(const Plane& A, const Plane& B, const Plane& C)
{
    float x[8], y[5];
#pragma unroll
    for (int m = 0; m < 4; ++m) x[m] = min3f(A.v[m + 5], B.v[m + 5], C.v[m + 5]);
#pragma unroll
    for (int m = 0; m < 4; ++m) x[m + 4] = max3f(A.v[m], B.v[m], C.v[m]);
#pragma unroll
    for (int m = 0; m < 5; ++m) y[m] = med3f(A.v[m + 2], B.v[m + 2], C.v[m + 2]);
    // odd-even merge of the sorted halves x[0..3], x[4..7]
    ce(x[0], x[4]);
    ce(x[2], x[6]);
    ce(x[2], x[4]);
    ce(x[1], x[5]);
    ce(x[3], x[7]);
    ce(x[3], x[5]);
    ce(x[1], x[2]);
    ce(x[3], x[4]);
    ce(x[5], x[6]);
    const float t = min3f(__builtin_fmaxf(x[1], y[4]), __builtin_fmaxf(x[2], y[3]), __builtin_fmaxf(x[3], y[2]));
    return __builtin_fminf(min3f(t, __builtin_fmaxf(x[4], y[1]), __builtin_fmaxf(x[5], y[0])), x[6]);
}

__global__ __launch_bounds__(256) void k_median3(const float* __restrict__ in, float* __restrict__ out, int w, int h,
                                                 int d)
{
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.z * 4 + (threadIdx.x >> 6);
    if (j >= h) return;  // uniform per wave; no barrier in this kernel
    const int kk = blockIdx.x * kMedTile - 1 + lane;
    const int k = kk < 0 ? 0 : (kk >= d ? d - 1 : kk);
    const bool store = lane >= 1 && lane <= kMedTile && kk < d;
    const int x0 = blockIdx.y * kMedSeg, x1 = min(x0 + kMedSeg, w);
    const size_t rm = (size_t)max(j - 1, 0) * w, r0 = (size_t)j * w, rp = (size_t)min(j + 1, h - 1) * w;
    Plane A = sorted_plane(in, rm, r0, rp, x0 - 1, w, d, k);
    Plane B = sorted_plane(in, rm, r0, rp, x0, w, d, k);
    for (int x = x0; x < x1; x += 3) {  // the three planes rotate roles
        Plane C = sorted_plane(in, rm, r0, rp, x + 1, w, d, k);
        float r = median27(A, B, C);
        if (store) out[(r0 + x) * d + kk] = r;
        if (x + 1 >= x1) break;
        A = sorted_plane(in, rm, r0, rp, x + 2, w, d, k);
        r = median27(B, C, A);
        if (store) out[(r0 + x + 1) * d + kk] = r;
        if (x + 2 >= x1) break;
        B = sorted_plane(in, rm, r0, rp, x + 3, w, d, k);
        r = median27(C, A, B);
        if (store) out[(r0 + x + 2) * d + kk] = r;
        // A and B now hold the planes of x + 2 and x + 3, as the next step needs
    }
}

// ---------------------------------------------------------------------------
// Order statistics by radix selection on the order-preserving integer image
// of the float values.  State lives in device memory so that the passes run
// back to back on the stream.
struct SelState {
    unsigned n;            // number of samples in the valid B-scans
    unsigned any_valid;    // 0: no B-scan valid, every sample counts
    unsigned prefix[4];    // selected high bits of each target
    unsigned rank[4];      // rank of each target among the samples with that prefix
    unsigned uprefix[4];   // the distinct prefixes, one histogram each in the next pass
    unsigned slot[4];      // index of each target's prefix in uprefix
    unsigned nu;           // number of distinct prefixes
    unsigned pad;
    double value[4];       // the four order statistics
    double p5, p95, thr_r; // percentiles and the threshold on the filtered volume
    double mu, thr_s;      // OCT noise mean and threshold
};

__device__ __forceinline__ unsigned ord_key(float v)
{
    const unsigned u = __builtin_bit_cast(unsigned, v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_key(unsigned k)
{
    return __builtin_bit_cast(float, (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// ---------------------------------------------------------------------------
// Rank filter: the 3rd smallest of the 15 samples p-7 .. p+7 along one
// lateral axis, clamped at the ends.
//
// A wave owns 64 consecutive depths of one line and a segment of kRankSeg
// positions, which it walks in chunks of 15 aligned so that chunk c spans
// p0-7+15c .. p0+7+15c.  The window of output p = p0+15c+t is the tail of
// chunk c from offset t joined with the head of chunk c+1 up to offset t-1:
// the three smallest of each part are kept sorted (suffix triples of chunk
// c, a running prefix triple of chunk c+1), and the 3rd smallest of the
// union of two sorted triples a, b is min(a3, b3, max(a1, b2), max(a2, b1)).
// Inserting v into a sorted triple gives (min(a1, v), med3(a1, a2, v),
// med3(a2, a3, v)).  Every sample is loaded once per segment.
//
// With kHist (the slow-axis pass, whose positions are the B-scans) the
// kernel also counts bits 31..21 of every output of a valid B-scan: the
// first radix pass of the percentile selection.  Along the walk a lane's
// outputs change bin rarely, so each lane adds runs of equal bins.
constexpr int kRankSeg = 120;  // a multiple of 15

struct Tri {
    float a, b, c;
};
__device__ __forceinline__ Tri insert(Tri t, float v)
{
    return Tri{__builtin_fminf(t.a, v), med3f(t.a, t.b, v), med3f(t.b, t.c, v)};
}
__device__ __forceinline__ float third_of_union(Tri s, Tri p)
{
    return min3f(__builtin_fminf(s.c, p.c), __builtin_fmaxf(s.a, p.b), __builtin_fmaxf(s.b, p.a));
}

template <bool kHist>
__global__ __launch_bounds__(256) void k_rank15(const float* __restrict__ in, float* __restrict__ out, int w, int h,
                                                int d, int axis, const float* __restrict__ valid,
                                                const SelState* __restrict__ st, unsigned* __restrict__ hist)
{
    __shared__ unsigned lh[kHist ? kHistBins : 1];
    if (kHist) {
        for (int t = threadIdx.x; t < kHistBins; t += blockDim.x) lh[t] = 0u;
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int ktiles = (d + 63) >> 6;
    const int n = axis == 0 ? w : h;
    const int nseg = (n + kRankSeg - 1) / kRankSeg;
    const int nlines = axis == 0 ? h : w;
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid < nlines * ktiles * nseg) {  // uniform per wave
        const int seg = wid % nseg, rest = wid / nseg;
        const int kt = rest % ktiles, o = rest / ktiles;
        const int k = kt * 64 + lane;
        const int kc = k < d ? k : d - 1;
        const bool store = k < d;
        const int p0 = seg * kRankSeg, p1 = min(p0 + kRankSeg, n);
        const size_t stride = axis == 0 ? (size_t)d : (size_t)w * d;
        const size_t base = (axis == 0 ? (size_t)o * w * d : (size_t)o * d) + kc;
        const float* __restrict__ p = in + base;
        float* __restrict__ q = out + base;
        const unsigned anyv = kHist ? st->any_valid : 0u;
        int cur = -1;       // bin of the current run of this lane's outputs
        unsigned run = 0u;  // and its length
        auto ld = [&](int pos) {
            pos = pos < 0 ? 0 : (pos >= n ? n - 1 : pos);
            return p[(size_t)pos * stride];
        };
        constexpr float inf = __builtin_inff();
        float u[15];
        Tri s[15];
#pragma unroll
        for (int t = 0; t < 15; ++t) u[t] = ld(p0 - 7 + t);
        s[14] = Tri{u[14], inf, inf};
#pragma unroll
        for (int t = 13; t >= 0; --t) s[t] = insert(s[t + 1], u[t]);
        for (int c0 = p0; c0 < p1; c0 += 15) {
#pragma unroll
            for (int t = 0; t < 15; ++t) u[t] = ld(c0 + 8 + t);
            Tri pre{inf, inf, inf};
#pragma unroll
            for (int t = 0; t < 15; ++t) {
                if (c0 + t < p1) {  // uniform
                    const float r = third_of_union(s[t], pre);
                    if (store) q[(size_t)(c0 + t) * stride] = r;
                    if (kHist) {
                        const bool ok = store && (!anyv || valid[c0 + t] > 0.5f);
                        const int bin = ok ? (int)(ord_key(r) >> 21) : -1;
                        if (bin != cur) {
                            if (cur >= 0) atomicAdd(&lh[cur], run);
                            cur = bin;
                            run = 0u;
                        }
                        ++run;
                    }
                }
                pre = insert(pre, u[t]);
            }
            s[14] = Tri{u[14], inf, inf};
#pragma unroll
            for (int t = 13; t >= 0; --t) s[t] = insert(s[t + 1], u[t]);
        }
        if (kHist && cur >= 0) atomicAdd(&lh[cur], run);
    }
    if (kHist) {
        __syncthreads();
        for (int t = threadIdx.x; t < kHistBins; t += blockDim.x)
            if (lh[t]) atomicAdd(&hist[t], lh[t]);
    }
}

// Nearest valid B-scan of each B-scan (the lower index on a tie; itself when
// none is valid), whether any is valid, and cleared histogram counters.
__global__ __launch_bounds__(256) void k_enface_init(const float* __restrict__ valid, int nb, int* __restrict__ from,
                                                     SelState* st, unsigned* __restrict__ hist)
{
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        if (valid[b] > 0.5f) any = 1;  // benign race: every writer stores 1
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        int src = b;
        if (any && !(valid[b] > 0.5f)) {
            src = -1;
            for (int dist = 1; dist < nb && src < 0; ++dist) {
                if (b - dist >= 0 && valid[b - dist] > 0.5f) src = b - dist;
                else if (b + dist < nb && valid[b + dist] > 0.5f) src = b + dist;
            }
        }
        from[b] = src;
    }
    for (int t = threadIdx.x; t < 4 * kHistBins; t += blockDim.x) hist[t] = 0u;
    if (threadIdx.x == 0) {
        st->any_valid = any;
        st->n = 0;
    }
}

// Radix passes 1 and 2 over the filtered volume: pass 1 counts bits 20..10
// of the samples whose bits 31..21 equal one of the distinct target
// prefixes, pass 2 bits 9..0 of those whose bits 31..10 do; one histogram of
// kHistBins counters per distinct prefix.  Few samples match, so each adds
// its own count.  A wave walks A-scans with eight loads in flight per lane.
// Pass 0 is counted by the slow-axis rank filter.
__global__ __launch_bounds__(256) void k_radix_hist(const float* __restrict__ vol, int w, int h, int d, int V,
                                                    const float* __restrict__ valid, const SelState* __restrict__ st,
                                                    int pass, unsigned* __restrict__ hist)
{
    __shared__ unsigned lh[4 * kHistBins];
    const int nu = (int)st->nu;
    for (int t = threadIdx.x; t < nu * kHistBins; t += blockDim.x) lh[t] = 0u;
    __syncthreads();
    const unsigned any = st->any_valid;
    unsigned pre[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) pre[t] = t < nu ? st->uprefix[t] : 0xFFFFFFFFu;
    const int shift = pass == 1 ? 21 : 10;
    const unsigned dmask = pass == 1 ? 2047u : 1023u;
    const int dshift = pass == 1 ? 10 : 0;
    const int lane = threadIdx.x & 63;
    const unsigned nwaves = gridDim.x * (blockDim.x >> 6);
    const unsigned na = (unsigned)w * (unsigned)h;
    for (unsigned a = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); a < na; a += nwaves) {
        const unsigned j = a / (unsigned)w, i = a - j * (unsigned)w;
        const unsigned b = V == 0 ? j : i;
        if (any && !(valid[b] > 0.5f)) continue;  // uniform per wave
        const float* __restrict__ col = vol + (size_t)a * d;
        for (int k0 = 0; k0 < d; k0 += 512) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int kk = k0 + e * 64 + lane;
                v[e] = kk < d ? col[kk] : 0.0f;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (k0 + e * 64 + lane < d) {
                    const unsigned key = ord_key(v[e]);
                    const unsigned hi = key >> shift;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (hi == pre[t]) atomicAdd(&lh[t * kHistBins + ((key >> dshift) & dmask)], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nu * kHistBins; t += blockDim.x)
        if (lh[t]) atomicAdd(&hist[t], lh[t]);
}

// One block: for each target, the bin whose counts cross its rank (a block
// scan of the histogram); after the last pass the order statistics, the
// percentiles and the threshold.  Clears the histograms it read.
__global__ __launch_bounds__(256) void k_radix_select(unsigned* __restrict__ hist, SelState* st, int pass)
{
#pragma clang fp contract(off)
    __shared__ unsigned scan[256];
    __shared__ unsigned target[4];
    const int nbins = pass == 2 ? 1024 : kHistBins;
    const int per = nbins / 256;
    const int nslot = pass == 0 ? 1 : (int)st->nu;
    const int tid = threadIdx.x;
    for (int u = 0; u < nslot; ++u) {
        const unsigned* hh = hist + (size_t)u * kHistBins;
        unsigned c[8];
        unsigned local = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            c[e] = e < per ? hh[tid * per + e] : 0u;
            local += c[e];
        }
        scan[tid] = local;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {  // inclusive scan
            const unsigned v = tid >= off ? scan[tid - off] : 0u;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        const unsigned excl = scan[tid] - local;
        if (pass == 0 && tid == 0) {
            const unsigned n = scan[255];
            st->n = n;
            const double q[2] = {0.05, 0.95};
            for (int e = 0; e < 2; ++e) {
                const double pos = q[e] * (double)(n - 1);
                unsigned lo = (unsigned)floor(pos);
                if (lo >= n - 1) lo = n - 1;
                target[2 * e] = lo;
                target[2 * e + 1] = lo + 1 < n ? lo + 1 : n - 1;
            }
        } else if (pass > 0 && tid < 4) {
            target[tid] = st->rank[tid];
        }
        __syncthreads();
        for (int t = 0; t < 4; ++t) {
            if (pass > 0 && (int)st->slot[t] != u) continue;
            const unsigned r = target[t];
            if (r >= excl && r < excl + local) {
                unsigned cum = excl;
                int e = 0;
                for (; e < per - 1; ++e) {
                    if (r < cum + c[e]) break;
                    cum += c[e];
                }
                const unsigned bin = (unsigned)(tid * per + e);
                if (pass == 0) st->prefix[t] = bin;
                else if (pass == 1) st->prefix[t] = (st->prefix[t] << 11) | bin;
                else st->value[t] = (double)from_key((st->prefix[t] << 10) | bin);
                st->rank[t] = r - cum;
            }
        }
        __syncthreads();
    }
    for (int t = tid; t < nslot * kHistBins; t += blockDim.x) hist[t] = 0u;
    __syncthreads();
    if (tid != 0) return;
    if (pass < 2) {
        unsigned nu = 0;
        for (int t = 0; t < 4; ++t) {
            unsigned u = 0;
            while (u < nu && st->uprefix[u] != st->prefix[t]) ++u;
            if (u == nu) st->uprefix[nu++] = st->prefix[t];
            st->slot[t] = u;
        }
        st->nu = nu;
        return;
    }
    const unsigned n = st->n;
    const double q[2] = {0.05, 0.95};
    double p[2];
    for (int e = 0; e < 2; ++e) {
        const double pos = q[e] * (double)(n - 1);
        unsigned lo = (unsigned)floor(pos);
        if (lo >= n - 1) lo = n - 1;
        const double frac = pos - (double)lo;
        const double x0 = st->value[2 * e], x1 = st->value[2 * e + 1];
        if (lo + 1 < n) {
            const double dx = x1 - x0;
            const double step = frac * dx;
            p[e] = x0 + step;
        } else {
            p[e] = x0;
        }
    }
    st->p5 = p[0];
    st->p95 = p[1];
    const double span = p[1] - p[0];
    const double off = 0.1 * span;
    st->thr_r = p[0] + off;
}

// A fixed normalisation mapping in place of the percentiles.
__global__ void k_set_fixed(SelState* st, double p5, double p95)
{
#pragma clang fp contract(off)
    st->p5 = p5;
    st->p95 = p95;
    const double span = p95 - p5;
    const double off = 0.1 * span;
    st->thr_r = p5 + off;
}

// OCT noise statistics over the first nz samples of every A-scan: pass 0
// sums the samples, pass 1 the squared deviations from their mean.  One wave
// per A-scan; partial sums per block, combined in a fixed order by
// k_noise_final.
__device__ __forceinline__ double block_sum(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(256) void k_noise_sum(const float* __restrict__ oct, size_t na, int d, int nz,
                                                   const SelState* __restrict__ st, int pass,
                                                   double* __restrict__ partial)
{
    __shared__ double red[256];
    const double mu = pass ? st->mu : 0.0;
    const int lane = threadIdx.x & 63;
    const size_t nwaves = (size_t)gridDim.x * (blockDim.x >> 6);
    double acc = 0.0;
#pragma unroll 4
    for (size_t a = (size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); a < na; a += nwaves) {
        for (int k = lane; k < nz; k += 64) {
            const double x = oct[a * d + k];
            if (pass == 0) {
                acc += x;
            } else {
                const double t = x - mu;
                acc += t * t;
            }
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_noise_final(const double* __restrict__ partial, int nblk, double cnt,
                                                     int pass, SelState* st)
{
    __shared__ double red[256];
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partial[b];
    const double s = block_sum(v, red);
    if (threadIdx.x != 0) return;
    if (pass == 0) st->mu = s / cnt;
    else st->thr_s = st->mu + 2.0 * sqrt(s / cnt);
}

// Both masks and the masked depth mean; one wave per A-scan.  kVec: four
// depths per lane with 16-byte loads (d a multiple of 4, aligned volumes).
template <bool kVec>
__global__ __launch_bounds__(256) void k_mask_mean(const float* __restrict__ filt, const float* __restrict__ oct,
                                                   const float* __restrict__ octa, size_t na, int d,
                                                   const SelState* __restrict__ st, double* __restrict__ E,
                                                   int* __restrict__ cnt)
{
    const int lane = threadIdx.x & 63;
    const double thr_r = st->thr_r, thr_s = st->thr_s;
    const size_t nwaves = (size_t)gridDim.x * (blockDim.x >> 6);
    for (size_t a = (size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); a < na; a += nwaves) {
        const size_t o = a * d;
        double acc = 0.0;
        int c = 0;
        if (kVec) {
            const float4* __restrict__ r4 = reinterpret_cast<const float4*>(filt + o);
            const float4* __restrict__ s4 = reinterpret_cast<const float4*>(oct + o);
            const float4* __restrict__ a4 = reinterpret_cast<const float4*>(octa + o);
            const int d4 = d >> 2;
#pragma unroll 4
            for (int k = lane; k < d4; k += 64) {
                const float4 r = r4[k], s = s4[k], v = a4[k];
                if ((double)r.x < thr_r && (double)s.x > thr_s) { acc += (double)v.x; ++c; }
                if ((double)r.y < thr_r && (double)s.y > thr_s) { acc += (double)v.y; ++c; }
                if ((double)r.z < thr_r && (double)s.z > thr_s) { acc += (double)v.z; ++c; }
                if ((double)r.w < thr_r && (double)s.w > thr_s) { acc += (double)v.w; ++c; }
            }
        } else {
            for (int k = lane; k < d; k += 64) {
                const double r = filt[o + k], s = oct[o + k];
                if (r < thr_r && s > thr_s) {
                    acc += (double)octa[o + k];
                    ++c;
                }
            }
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            acc += __shfl_xor(acc, m);
            c += __shfl_xor(c, m);
        }
        if (lane == 0) {
            E[a] = c ? acc / c : 0.0;
            if (cnt) cnt[a] = c;
        }
    }
}

// Median of each B-scan's en face values (the mean of the two middle ones
// for an even count): bitonic sort in LDS, one block per B-scan.
__global__ __launch_bounds__(512) void k_bscan_median(const double* __restrict__ E, int w, int h, int V,
                                                      double* __restrict__ med)
{
    __shared__ double s[kMaxBscan];
    const int b = blockIdx.x;
    const int na = V == 0 ? w : h;
    int P = 1;
    while (P < na) P <<= 1;
    for (int t = threadIdx.x; t < P; t += blockDim.x)
        s[t] = t < na ? (V == 0 ? E[(size_t)b * w + t] : E[(size_t)t * w + b]) : __builtin_inf();
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int t = threadIdx.x; t < P; t += blockDim.x) {
                const int u = t ^ jj;
                if (u > t) {
                    const double x = s[t], y = s[u];
                    const bool up = (t & k) == 0;
                    if ((x > y) == up) {
                        s[t] = y;
                        s[u] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) med[b] = (na & 1) ? s[na / 2] : 0.5 * (s[na / 2 - 1] + s[na / 2]);
}

__global__ void k_enface_finish(const double* __restrict__ E, const double* __restrict__ med,
                                const int* __restrict__ from, int w, int h, int V, float* __restrict__ out)
{
    const size_t a = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= (size_t)w * h) return;
    const int i = (int)(a % w), j = (int)(a / w);
    const int b = V == 0 ? j : i;
    const int src = from[b];
    const size_t sa = V == 0 ? (size_t)src * w + i : (size_t)j * w + src;
    out[a] = (float)(E[sa] - med[src]);
}

__global__ void k_fill_ones(float* __restrict__ p, size_t n)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 1.0f;
}

inline size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t enface_scratch_bytes(int w, int h, int d)
{
    const size_t na = (size_t)w * h, nv = na * d, nb = (size_t)(w > h ? w : h);
    return 2 * al(nv * 4) + al(na * 8) + al(na * 4) + al(nb * 8) + al(nb * 4) + al(nb * 4) +
           al(4 * kHistBins * 4) + al(sizeof(SelState)) + al(kNoiseBlocks * 8);
}

int enface_max_bscan() { return kMaxBscan; }

hipError_t launch_enface_project(const float* oct, const float* octa, int w, int h, int d, int V,
                                 const float* valid, const double* fixed, float* out, int* count, double* stats_host,
                                 void* scratch, hipStream_t s)
{
    const size_t na = (size_t)w * h, nv = na * d, nb = (size_t)(V == 0 ? h : w), nbm = (size_t)(w > h ? w : h);
    char* p = static_cast<char*>(scratch);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += al(bytes);
        return q;
    };
    float* v0 = (float*)take(nv * 4);
    float* v1 = (float*)take(nv * 4);
    double* E = (double*)take(na * 8);
    int* cnt = (int*)take(na * 4);
    double* med = (double*)take(nbm * 8);
    int* from = (int*)take(nbm * 4);
    float* vd = (float*)take(nbm * 4);
    unsigned* hist = (unsigned*)take(4 * kHistBins * 4);
    SelState* st = (SelState*)take(sizeof(SelState));
    double* part = (double*)take(kNoiseBlocks * 8);
    if (!valid) {
        hipLaunchKernelGGL(k_fill_ones, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, vd, nb);
        valid = vd;
    }
    hipLaunchKernelGGL(k_enface_init, dim3(1), dim3(256), 0, s, valid, (int)nb, from, st, hist);
    // filtering; the slow-axis pass also counts the first radix digit
    const dim3 gm((d + kMedTile - 1) / kMedTile, (w + kMedSeg - 1) / kMedSeg, (h + 3) / 4);
    hipLaunchKernelGGL(k_median3, gm, dim3(256), 0, s, octa, v0, w, h, d);
    const int ktiles = (d + 63) / 64;
    const int fast = V == 0 ? 0 : 1, slow = 1 - fast;
    auto waves = [&](int axis) {
        const int n = axis == 0 ? w : h, lines = axis == 0 ? h : w;
        return lines * ktiles * ((n + kRankSeg - 1) / kRankSeg);
    };
    hipLaunchKernelGGL(k_rank15<false>, dim3((waves(fast) + 3) / 4), dim3(256), 0, s, v0, v1, w, h, d, fast, valid,
                       st, hist);
    if (fixed) {
        hipLaunchKernelGGL(k_rank15<false>, dim3((waves(slow) + 3) / 4), dim3(256), 0, s, v1, v0, w, h, d, slow,
                           valid, st, hist);
        hipLaunchKernelGGL(k_set_fixed, dim3(1), dim3(1), 0, s, st, fixed[0], fixed[1]);
    } else {
        hipLaunchKernelGGL(k_rank15<true>, dim3((waves(slow) + 3) / 4), dim3(256), 0, s, v1, v0, w, h, d, slow,
                           valid, st, hist);
        hipLaunchKernelGGL(k_radix_select, dim3(1), dim3(256), 0, s, hist, st, 0);
        for (int pass = 1; pass < 3; ++pass) {
            hipLaunchKernelGGL(k_radix_hist, dim3(kHistBlocks), dim3(256), 0, s, v0, w, h, d, V, valid, st, pass,
                               hist);
            hipLaunchKernelGGL(k_radix_select, dim3(1), dim3(256), 0, s, hist, st, pass);
        }
    }
    // OCT noise threshold
    const int nz = (int)floor(0.05 * d + 0.5) < 1 ? 1 : (int)floor(0.05 * d + 0.5);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_noise_sum, dim3(kNoiseBlocks), dim3(256), 0, s, oct, na, d, nz, st, pass, part);
        hipLaunchKernelGGL(k_noise_final, dim3(1), dim3(256), 0, s, part, kNoiseBlocks, (double)na * nz, pass, st);
    }
    // masks, depth mean, B-scan median, substitution
    const bool vec = (d & 3) == 0 && ((uintptr_t)oct & 15) == 0 && ((uintptr_t)octa & 15) == 0;
    const dim3 gmm((unsigned)std::min<size_t>((na + 3) / 4, 65536));
    if (vec)
        hipLaunchKernelGGL(k_mask_mean<true>, gmm, dim3(256), 0, s, v0, oct, octa, na, d, st, E, count ? count : cnt);
    else
        hipLaunchKernelGGL(k_mask_mean<false>, gmm, dim3(256), 0, s, v0, oct, octa, na, d, st, E, count ? count : cnt);
    hipLaunchKernelGGL(k_bscan_median, dim3((unsigned)nb), dim3(512), 0, s, E, w, h, V, med);
    hipLaunchKernelGGL(k_enface_finish, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, E, med, from, w, h, V,
                       out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && stats_host) e = hipMemcpyAsync(stats_host, &st->p5, 3 * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && stats_host) e = hipMemcpyAsync(stats_host + 3, &st->thr_s, 8, hipMemcpyDeviceToHost, s);
    return e;
}

}  // namespace octmc
